// bf_weights.hip -- weight generation on the device (FP64) and the MFMA
// operand layout of the weights.
//
// Phase model of Eq. 1 (Sec. 1): steering beam b to the unit direction k_b
// applies to antenna n at r_n the phase shift
//     W[c][b][n] = exp(-i 2 pi f_c (k_b . r_n) / c0).
// Sec. 3.2 recomputes coefficients whenever pointings change, overlapped
// with the previous iteration; here that is one kernel per bf_set_weights.
//
// Numerics: the phase in cycles f (k.r)/c0 reaches ~10^3 for a 500 m array
// at 416 MHz, so it is formed in FP64, reduced to [-1/2, 1/2] cycles in
// FP64 (exact subtraction of the nearest integer), and only then passed to
// sincospi.  Each weight component is rounded once, to nearest even,
// directly from FP64 to the storage format (no FP64 -> FP32 -> FP16 double
// rounding).
//
// Operand layout (what the beamform kernel stages in LDS):
//     w[c][bp][h][k],  bp < Bpad (B rounded up to 16), h = 0 (re-row) or
//     1 (im-row), k < Kpad (2N rounded up to 64);
//     re-row: k = 2n -> Re W, k = 2n+1 -> -Im W
//     im-row: k = 2n -> Im W, k = 2n+1 ->  Re W
// and zero for b >= B or n >= N, so that Re(W x) = re-row . [xr, xi] and
// Im(W x) = im-row . [xr, xi] over interleaved voltages.
#include "bf_internal.h"

namespace bf {

constexpr double kC0 = 299792458.0;  // m/s

// Round an FP64 value to nearest even in a binary format with MB stored
// mantissa bits and EB exponent bits; returns the encoded bits.  Handles
// signed zero, subnormal results, overflow to infinity and NaN.
template <int MB, int EB>
__device__ __forceinline__ uint32_t round_f64(double d) {
  constexpr int bias = (1 << (EB - 1)) - 1;
  constexpr int emin = 1 - bias;
  constexpr int emax = bias;
  constexpr uint32_t inf = ((1u << EB) - 1u) << MB;
  const uint64_t bits = (uint64_t)__double_as_longlong(d);
  const uint32_t sign = (uint32_t)(bits >> 63) << (MB + EB);
  const int ex = (int)((bits >> 52) & 0x7FF);
  const uint64_t man = bits & 0xFFFFFFFFFFFFFull;
  if (ex == 0x7FF) return sign | inf | (man ? (1u << (MB - 1)) : 0u);
  if (ex == 0) return sign;  // FP64 subnormals are far below any target's range
  int e = ex - 1023;
  const uint64_t m = man | (1ull << 52);
  const int s = (e >= emin) ? 52 - MB : 52 - MB + (emin - e);
  if (s > 53) return sign;  // below half the smallest subnormal
  uint64_t q = m >> s;
  const uint64_t rem = m & ((1ull << s) - 1);
  const uint64_t half = 1ull << (s - 1);
  if (rem > half || (rem == half && (q & 1))) ++q;
  if (e >= emin) {
    if (q == (2ull << MB)) {  // mantissa carried out
      q >>= 1;
      ++e;
    }
    if (e > emax) return sign | inf;
    return sign | ((uint32_t)(e + bias) << MB) | (uint32_t)(q & ((1u << MB) - 1));
  }
  return sign | (uint32_t)q;  // subnormal (q == 2^MB encodes the smallest normal)
}

template <int PREC> struct Store;
template <> struct Store<0> {
  using T = float;
  static __device__ T cvt(double v) { return (float)v; }  // IEEE RNE
};
template <> struct Store<1> {
  using T = uint16_t;
  static __device__ T cvt(double v) { return (uint16_t)round_f64<10, 5>(v); }
};
template <> struct Store<2> {
  using T = uint16_t;
  static __device__ T cvt(double v) { return (uint16_t)round_f64<7, 8>(v); }
};

// Writes the four operand entries of (c, b, n) from an FP64 weight.
template <int PREC>
__device__ __forceinline__ void put(void* w, int64_t c, int b, int n, int Bpad, int Kpad,
                                    double wr, double wi) {
  using T = typename Store<PREC>::T;
  T* row = reinterpret_cast<T*>(w) + (((int64_t)c * Bpad + b) * 2) * Kpad;
  row[2 * n] = Store<PREC>::cvt(wr);
  row[2 * n + 1] = Store<PREC>::cvt(-wi);
  row[Kpad + 2 * n] = Store<PREC>::cvt(wi);
  row[Kpad + 2 * n + 1] = Store<PREC>::cvt(wr);
}

// One thread per (c, b < Bpad, n < Kpad/2).  mask[n] == 0 drops antenna n
// (zero weight column: a sub-array beam).
template <int PREC>
__global__ void weights_geom_kernel(const double* __restrict__ pos, const double* __restrict__ dir,
                                    const double* __restrict__ freq,
                                    const double* __restrict__ mask, int N, int C, int B,
                                    int Bpad, int Kpad, void* w) {
  const int half = Kpad / 2;
  const int64_t total = (int64_t)C * Bpad * half;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(i % half);
    const int64_t cb = i / half;
    const int b = (int)(cb % Bpad);
    const int64_t c = cb / Bpad;
    double wr = 0.0, wi = 0.0;
    if (n < N && b < B && mask[n] != 0.0) {
      const double kr = dir[3 * b] * pos[3 * n] + dir[3 * b + 1] * pos[3 * n + 1] +
                        dir[3 * b + 2] * pos[3 * n + 2];        // metres
      const double cyc = freq[c] * kr / kC0;                    // phase in cycles
      const double frac = cyc - rint(cyc);                      // exact, |frac| <= 1/2
      double sn, cs;
      sincospi(2.0 * frac, &sn, &cs);
      wr = cs;   // exp(-i phi) = cos(phi) - i sin(phi)
      wi = -sn;
    }
    put<PREC>(w, c, b, n, Bpad, Kpad, wr, wi);
  }
}

// Raw complex weights [C][B][N][2] (device copy) -> operand layout.
template <int PREC>
__global__ void weights_raw_kernel(const double* __restrict__ wraw, int N, int C, int B, int Bpad,
                                   int Kpad, void* w) {
  const int half = Kpad / 2;
  const int64_t total = (int64_t)C * Bpad * half;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(i % half);
    const int64_t cb = i / half;
    const int b = (int)(cb % Bpad);
    const int64_t c = cb / Bpad;
    double wr = 0.0, wi = 0.0;
    if (n < N && b < B) {
      const double* src = wraw + ((c * B + b) * N + n) * 2;
      wr = src[0];
      wi = src[1];
    }
    put<PREC>(w, c, b, n, Bpad, Kpad, wr, wi);
  }
}

__global__ void queue_reset_kernel(int32_t* q) { *q = 0; }

// Copies a set table from the kernel arguments into device memory, one dword
// per thread per step.
__global__ void __launch_bounds__(kThreads) table_store_kernel(const Launch L, Launch* dst) {
  static_assert(sizeof(Launch) % 4 == 0, "the table is copied in dwords");
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&L);
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(Launch) / 4); i += kThreads) d[i] = src[i];
}

static int grid_for(int64_t total) {
  int64_t g = (total + 255) / 256;
  return (int)(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

template <typename K, typename... A>
static hipError_t launch(K kern, int grid, int block, hipStream_t s, A... a) {
  void* args[] = {reinterpret_cast<void*>(&a)...};
  return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(block), args, 0, s);
}

hipError_t launch_weights_geom(int prec, const double* pos, const double* dir, const double* freq,
                               const double* mask, int N, int C, int B, int Bpad, int Kpad,
                               void* w, hipStream_t s) {
  const int grid = grid_for((int64_t)C * Bpad * (Kpad / 2));
  if (prec == 0)
    return launch(weights_geom_kernel<0>, grid, 256, s, pos, dir, freq, mask, N, C, B, Bpad, Kpad,
                  w);
  if (prec == 1)
    return launch(weights_geom_kernel<1>, grid, 256, s, pos, dir, freq, mask, N, C, B, Bpad, Kpad,
                  w);
  return launch(weights_geom_kernel<2>, grid, 256, s, pos, dir, freq, mask, N, C, B, Bpad, Kpad,
                w);
}

hipError_t launch_weights_raw(int prec, const double* wraw, int N, int C, int B, int Bpad,
                              int Kpad, void* w, hipStream_t s) {
  const int grid = grid_for((int64_t)C * Bpad * (Kpad / 2));
  if (prec == 0) return launch(weights_raw_kernel<0>, grid, 256, s, wraw, N, C, B, Bpad, Kpad, w);
  if (prec == 1) return launch(weights_raw_kernel<1>, grid, 256, s, wraw, N, C, B, Bpad, Kpad, w);
  return launch(weights_raw_kernel<2>, grid, 256, s, wraw, N, C, B, Bpad, Kpad, w);
}

hipError_t launch_queue_reset(int32_t* q, hipStream_t s) {
  return launch(queue_reset_kernel, 1, 1, s, q);
}

hipError_t launch_table_store(const Launch& L, Launch* dst, hipStream_t s) {
  return launch(table_store_kernel, 1, kThreads, s, L, dst);
}

}  // namespace bf
