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

// Operand entries (2n, 2n+1) of the re-row and the im-row of beam b of
// channel c: [Re W, -Im W] and [Im W, Re W], each pair one store.
template <int PREC>
__device__ __forceinline__ void put(void* w, int64_t row, int n, int Kpad, double wr, double wi) {
  using T = typename Store<PREC>::T;
  T* r0 = reinterpret_cast<T*>(w) + row * 2 * Kpad;
  if constexpr (PREC == 0) {
    reinterpret_cast<float2*>(r0)[n] = float2{Store<0>::cvt(wr), Store<0>::cvt(-wi)};
    reinterpret_cast<float2*>(r0 + Kpad)[n] = float2{Store<0>::cvt(wi), Store<0>::cvt(wr)};
  } else {
    const uint32_t re = Store<PREC>::cvt(wr), nim = Store<PREC>::cvt(-wi),
                   im = Store<PREC>::cvt(wi);
    reinterpret_cast<uint32_t*>(r0)[n] = re | (nim << 16);
    reinterpret_cast<uint32_t*>(r0 + Kpad)[n] = im | (re << 16);
  }
}

// One workgroup per operand row (c, b < Bpad) at a time, its threads over
// the antennas n < Kpad/2 (padding written as zeros).  mask[n] == 0 drops
// antenna n (zero weight column: a sub-array beam).
template <int PREC>
__global__ void __launch_bounds__(64) weights_geom_kernel(
    const double* __restrict__ pos, const double* __restrict__ dir,
    const double* __restrict__ freq, const double* __restrict__ mask, int N, int C, int B,
    int Bpad, int Kpad, void* w) {
  const int half = Kpad / 2;
  const int64_t rows = (int64_t)C * Bpad;
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const int b = (int)(row % Bpad);
    const int64_t c = row / Bpad;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    if (b < B) {
      d0 = dir[3 * b];
      d1 = dir[3 * b + 1];
      d2 = dir[3 * b + 2];
    }
    for (int n = threadIdx.x; n < half; n += blockDim.x) {
      double wr = 0.0, wi = 0.0;
      if (n < N && b < B && mask[n] != 0.0) {
        const double kr = d0 * pos[3 * n] + d1 * pos[3 * n + 1] + d2 * pos[3 * n + 2];  // m
        const double cyc = freq[c] * kr / kC0;                    // phase in cycles
        const double frac = cyc - rint(cyc);                      // exact, |frac| <= 1/2
        double sn, cs;
        sincospi(2.0 * frac, &sn, &cs);
        wr = cs;   // exp(-i phi) = cos(phi) - i sin(phi)
        wi = -sn;
      }
      put<PREC>(w, row, n, Kpad, wr, wi);
    }
  }
}

// Raw complex weights [C][B][N][2] (device copy) -> operand layout.
template <int PREC>
__global__ void __launch_bounds__(64) weights_raw_kernel(const double* __restrict__ wraw, int N,
                                                         int C, int B, int Bpad, int Kpad,
                                                         void* w) {
  const int half = Kpad / 2;
  const int64_t rows = (int64_t)C * Bpad;
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const int b = (int)(row % Bpad);
    const int64_t c = row / Bpad;
    for (int n = threadIdx.x; n < half; n += blockDim.x) {
      double wr = 0.0, wi = 0.0;
      if (n < N && b < B) {
        const double* src = wraw + ((c * B + b) * N + n) * 2;
        wr = src[0];
        wi = src[1];
      }
      put<PREC>(w, row, n, Kpad, wr, wi);
    }
  }
}

__global__ void queue_reset_kernel(int32_t* q) {
  if (threadIdx.x < kXcds) q[threadIdx.x * kQueueStride] = 0;
}

// Copies a set table from the kernel arguments into device memory, one dword
// per thread per step.
__global__ void __launch_bounds__(kThreads) table_store_kernel(const Launch L, Launch* dst) {
  static_assert(sizeof(Launch) % 4 == 0, "the table is copied in dwords");
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&L);
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(Launch) / 4); i += kThreads) d[i] = src[i];
}

// One workgroup per operand row, at most 2^20 of them (each then loops).
static int grid_rows(int64_t rows) {
  return (int)(rows < (1 << 20) ? (rows > 0 ? rows : 1) : (1 << 20));
}

template <typename K, typename... A>
static hipError_t launch(K kern, int grid, int block, hipStream_t s, A... a) {
  void* args[] = {reinterpret_cast<void*>(&a)...};
  return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(block), args, 0, s);
}

hipError_t launch_weights_geom(int prec, const double* pos, const double* dir, const double* freq,
                               const double* mask, int N, int C, int B, int Bpad, int Kpad,
                               void* w, hipStream_t s) {
  const int grid = grid_rows((int64_t)C * Bpad);
  if (prec == 0)
    return launch(weights_geom_kernel<0>, grid, 64, s, pos, dir, freq, mask, N, C, B, Bpad, Kpad,
                  w);
  if (prec == 1)
    return launch(weights_geom_kernel<1>, grid, 64, s, pos, dir, freq, mask, N, C, B, Bpad, Kpad,
                  w);
  return launch(weights_geom_kernel<2>, grid, 64, s, pos, dir, freq, mask, N, C, B, Bpad, Kpad,
                w);
}

hipError_t launch_weights_raw(int prec, const double* wraw, int N, int C, int B, int Bpad,
                              int Kpad, void* w, hipStream_t s) {
  const int grid = grid_rows((int64_t)C * Bpad);
  if (prec == 0) return launch(weights_raw_kernel<0>, grid, 64, s, wraw, N, C, B, Bpad, Kpad, w);
  if (prec == 1) return launch(weights_raw_kernel<1>, grid, 64, s, wraw, N, C, B, Bpad, Kpad, w);
  return launch(weights_raw_kernel<2>, grid, 64, s, wraw, N, C, B, Bpad, Kpad, w);
}

hipError_t launch_queue_reset(int32_t* q, hipStream_t s) {
  return launch(queue_reset_kernel, 1, kXcds, s, q);
}

hipError_t launch_table_store(const Launch& L, Launch* dst, hipStream_t s) {
  return launch(table_store_kernel, 1, kThreads, s, L, dst);
}

}  // namespace bf
