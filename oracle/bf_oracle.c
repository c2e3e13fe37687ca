/*
 * bf_oracle.c -- plain FP64 CPU oracle for the coherent beamformer.
 * TEST INFRASTRUCTURE ONLY (see bf_oracle.h).  Deliberately unblocked and
 * unfused: one loop per index of the defining sums, so that each line can be
 * checked against the paper by eye.
 */
#include "bf_oracle.h"

#include <math.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Eq. 1 phase model (Sec. 1): steering beam b to k_b multiplies antenna n's
 * signal by exp(-i 2 pi f (k_b . r_n) / c0), so that a plane wave from k_b,
 * which reaches antenna n with phase exp(+i 2 pi f (k_b . r_n) / c0), adds
 * in phase over all antennas. */
int bfo_weights(int32_t N, int32_t C, int32_t B, const double* pos, const double* dir,
                const double* freq, double* w) {
  if (N < 1 || C < 1 || B < 1 || !pos || !dir || !freq || !w) return -1;
  const double two_pi = 2.0 * M_PI;
  for (int32_t c = 0; c < C; ++c)
    for (int32_t b = 0; b < B; ++b)
      for (int32_t n = 0; n < N; ++n) {
        double kr = dir[3 * b + 0] * pos[3 * n + 0] + dir[3 * b + 1] * pos[3 * n + 1] +
                    dir[3 * b + 2] * pos[3 * n + 2];           /* metres   */
        double phi = two_pi * freq[c] * kr / BFO_C0;           /* radians  */
        size_t o = (((size_t)c * B + b) * N + n) * 2;
        w[o + 0] = cos(phi);  /* exp(-i phi) = cos(phi) - i sin(phi) */
        w[o + 1] = -sin(phi);
      }
  return 0;
}

/* Sec. 2.1: per channel, every time sample's antenna vector is multiplied by
 * the B x N coefficient matrix; the power of each beam sample is taken in
 * the same pass and summed over I consecutive samples.  Exactly one of x8 /
 * x64 is non-null. */
static int beamform(int32_t N, int32_t C, int32_t B, int64_t T, int32_t I,
                    const double* w, const int8_t* x8, const double* x64, double* p) {
  if (N < 1 || C < 1 || B < 1 || T < 1 || I < 1 || T % I != 0 || !w || !p) return -1;
  if ((x8 == NULL) == (x64 == NULL)) return -1;
  const int64_t nwin = T / I;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int32_t c = 0; c < C; ++c)
    for (int32_t b = 0; b < B; ++b) {
      const double* wb = w + ((size_t)c * B + b) * (size_t)N * 2;
      double* pb = p + ((size_t)c * B + b) * (size_t)nwin;
      for (int64_t k = 0; k < nwin; ++k) pb[k] = 0.0;
      for (int64_t t = 0; t < T; ++t) {
        size_t xo = ((size_t)c * T + t) * (size_t)N * 2;
        double re = 0.0, im = 0.0;
        for (int32_t n = 0; n < N; ++n) {
          double wr = wb[2 * n], wi = wb[2 * n + 1];
          double xr = x8 ? (double)x8[xo + 2 * n] : x64[xo + 2 * n];
          double xi = x8 ? (double)x8[xo + 2 * n + 1] : x64[xo + 2 * n + 1];
          re += wr * xr - wi * xi; /* Re(W X) */
          im += wr * xi + wi * xr; /* Im(W X) */
        }
        pb[t / I] += re * re + im * im; /* |B|^2, summed over the window */
      }
    }
  return 0;
}

int bfo_beamform_i8(int32_t N, int32_t C, int32_t B, int64_t T, int32_t I,
                    const double* w, const int8_t* x, double* p) {
  if (!x) return -1;
  return beamform(N, C, B, T, I, w, x, NULL, p);
}

int bfo_beamform_f64(int32_t N, int32_t C, int32_t B, int64_t T, int32_t I,
                     const double* w, const double* x, double* p) {
  if (!x) return -1;
  return beamform(N, C, B, T, I, w, NULL, x, p);
}

int bfo_beams_f64(int32_t N, int32_t C, int32_t B, int64_t T,
                  const double* w, const double* x, double* beams) {
  if (N < 1 || C < 1 || B < 1 || T < 1 || !w || !x || !beams) return -1;
  for (int32_t c = 0; c < C; ++c)
    for (int32_t b = 0; b < B; ++b)
      for (int64_t t = 0; t < T; ++t) {
        const double* wb = w + ((size_t)c * B + b) * (size_t)N * 2;
        const double* xt = x + ((size_t)c * T + t) * (size_t)N * 2;
        double re = 0.0, im = 0.0;
        for (int32_t n = 0; n < N; ++n) {
          re += wb[2 * n] * xt[2 * n] - wb[2 * n + 1] * xt[2 * n + 1];
          im += wb[2 * n] * xt[2 * n + 1] + wb[2 * n + 1] * xt[2 * n];
        }
        size_t o = (((size_t)c * B + b) * T + t) * 2;
        beams[o] = re;
        beams[o + 1] = im;
      }
  return 0;
}

int bfo_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void bfo_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
