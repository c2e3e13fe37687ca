// bf_pattern.hip -- beam-pattern (array-factor) map of a plan's weights over
// a grid of directions.
//
// For channel c, beam b and grid direction k_g (Sec. 3.1 simulates the
// BEST-2 beam pattern from the coefficients over a sky grid; Eq. 1 is the
// array factor of the antenna layout):
//
//     P[c][b][g] = | sum_n W[c][b][n] * exp(+i 2 pi f_c (k_g . r_n) / c0) |^2
//
// i.e. the beam the plan forms, evaluated for a unit plane wave from every
// grid direction, with the plan's own rounded weights.  The steering phase is
// formed in FP64 and reduced modulo one cycle; sin/cos of the reduced phase
// and the sums are FP32.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bf_internal.h"

namespace bf {
namespace {

constexpr double kC0 = 299792458.0;  // m/s
constexpr int kPatG = 64;            // grid directions per workgroup
constexpr int kPatB = 16;            // beams per workgroup
constexpr int kPatN = 64;            // antennas per LDS chunk

// (Re W, Im W) of antenna n from the re-row of operand row `row` (the row
// holds [Re W, -Im W] per antenna in the storage precision).
template <int PREC>
__device__ __forceinline__ float2 load_w(const void* w, int64_t row, int n, int Kpad) {
  if constexpr (PREC == 0) {
    const float2 v = reinterpret_cast<const float2*>(reinterpret_cast<const float*>(w) +
                                                     row * 2 * Kpad)[n];
    return float2{v.x, -v.y};
  } else {
    const uint32_t u = reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint16_t*>(w) +
                                                         row * 2 * Kpad)[n];
    float re, nim;
    if constexpr (PREC == 1) {
      re = (float)__builtin_bit_cast(_Float16, (uint16_t)(u & 0xFFFFu));
      nim = (float)__builtin_bit_cast(_Float16, (uint16_t)(u >> 16));
    } else {
      re = __builtin_bit_cast(float, u << 16);
      nim = __builtin_bit_cast(float, u & 0xFFFF0000u);
    }
    return float2{re, -nim};
  }
}

// Workgroup (g tile, b tile, channels z, z + gridDim.z, ...): 64 directions x
// 16 beams; thread (bq, gl) owns direction gl and beams bq, bq+4, bq+8, bq+12.
// Per chunk of 64 antennas the workgroup forms the steering tile
// S[n][g] and the weight tile in LDS, then every thread accumulates.
template <int PREC>
__global__ void __launch_bounds__(256) pattern_kernel(const void* __restrict__ w,
                                                      const double* __restrict__ pos,
                                                      const double* __restrict__ gdir,
                                                      const double* __restrict__ freq, int N,
                                                      int C, int B, int Bpad, int Kpad, int G,
                                                      float* __restrict__ out) {
  __shared__ float2 S[kPatN][kPatG];
  __shared__ float2 Wt[kPatB][kPatN];
  const int tid = threadIdx.x;
  const int gl = tid & (kPatG - 1);
  const int bq = tid / kPatG;
  const int g0 = blockIdx.x * kPatG;
  const int b0 = blockIdx.y * kPatB;
  for (int c = blockIdx.z; c < C; c += gridDim.z) {
    const double fc = freq[c];
    float2 acc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = float2{0.f, 0.f};
    for (int n0 = 0; n0 < N; n0 += kPatN) {
      __syncthreads();  // the previous chunk's tiles have been read
      for (int e = tid; e < kPatN * kPatG; e += 256) {
        const int nn = e / kPatG, gg = e % kPatG;
        const int g = g0 + gg, n = n0 + nn;
        float2 v = {0.f, 0.f};
        if (g < G && n < N) {
          const double kr = gdir[3 * g] * pos[3 * n] + gdir[3 * g + 1] * pos[3 * n + 1] +
                            gdir[3 * g + 2] * pos[3 * n + 2];
          const double cyc = fc * kr / kC0;
          const float frac = (float)(cyc - rint(cyc));  // |frac| <= 1/2
          float sn, cs;
          sincospif(2.0f * frac, &sn, &cs);
          v = float2{cs, sn};
        }
        S[nn][gg] = v;
      }
      for (int e = tid; e < kPatB * kPatN; e += 256) {
        const int bb = e / kPatN, nn = e % kPatN;
        const int b = b0 + bb, n = n0 + nn;
        Wt[bb][nn] = (b < B && n < N) ? load_w<PREC>(w, (int64_t)c * Bpad + b, n, Kpad)
                                      : float2{0.f, 0.f};
      }
      __syncthreads();
      const int nlim = min(kPatN, N - n0);
      for (int nn = 0; nn < nlim; ++nn) {
        const float2 s = S[nn][gl];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float2 wv = Wt[bq + 4 * k][nn];
          acc[k].x = __builtin_fmaf(wv.x, s.x, __builtin_fmaf(-wv.y, s.y, acc[k].x));
          acc[k].y = __builtin_fmaf(wv.x, s.y, __builtin_fmaf(wv.y, s.x, acc[k].y));
        }
      }
    }
    const int g = g0 + gl;
    if (g < G) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int b = b0 + bq + 4 * k;
        if (b < B)
          out[((int64_t)c * B + b) * G + g] =
              __builtin_fmaf(acc[k].x, acc[k].x, acc[k].y * acc[k].y);
      }
    }
  }
}

}  // namespace

// Geometry staging of the allocation-free entry point: antenna positions,
// channel frequencies and grid directions (FP64) of one call, at most
// kPatScratchDoubles values.  Each GPU the library runs on holds its own
// copy until the process ends, and every call on that GPU shares it.
static __device__ __align__(256) double scratch[kPatScratchDoubles];

// Device address of `scratch` on device `dev` (made current by the caller),
// looked up once per device.  The array's name is a host-side stand-in in
// host code; only this address may reach kernels or copies.
hipError_t pattern_scratch(int dev, double** out) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static double* addr[kMaxDev] = {};
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(ptr);
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t launch_beam_pattern(int prec, const void* w, const double* pos, const double* gdir,
                               const double* freq, int N, int C, int B, int Bpad, int Kpad, int G,
                               float* out, hipStream_t s) {
  const dim3 grid((G + kPatG - 1) / kPatG, Bpad / kPatB, C < 65535 ? C : 65535);
  const void* k = prec == 0   ? reinterpret_cast<const void*>(pattern_kernel<0>)
                  : prec == 1 ? reinterpret_cast<const void*>(pattern_kernel<1>)
                              : reinterpret_cast<const void*>(pattern_kernel<2>);
  void* args[] = {&w, &pos, &gdir, &freq, &N, &C, &B, &Bpad, &Kpad, &G, &out};
  return hipLaunchKernel(k, grid, dim3(256), args, 0, s);
}

}  // namespace bf
