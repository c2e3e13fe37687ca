/*
 * bf_oracle.h -- plain FP64 CPU oracle for the coherent beamformer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * What it computes (Magro, Zarb Adami & Hickish, "GPU-Powered Coherent
 * Beamforming"):
 *   - weights: the phase model behind Eq. 1 (Sec. 1): a beam steered to the
 *     unit direction k_b applies to antenna n at position r_n the phase
 *     shift  W[c][b][n] = exp(-i * 2*pi * f_c * (k_b . r_n) / c0);
 *   - beams: per channel, the N_b x N_a coefficient matrix times the antenna
 *     vector of every time sample (Sec. 2.1), B[c][b][t] = sum_n W X;
 *   - detection: power |B|^2 inside the beamformer (Sec. 2.1);
 *   - integration: non-overlapping sums of I consecutive power samples,
 *     windows aligned at t = 0 (the paper's kernel stores every sample; the
 *     integrated form is what this library produces).
 * All arithmetic is FP64 with explicit real/imaginary parts.
 *
 * Array layouts (row-major, all host memory owned by the caller):
 *   pos  [N][3]       antenna positions, metres (x = E, y = N, z = up)
 *   dir  [B][3]       beam pointings, unit vectors toward the sky
 *   freq [C]          channel centre frequencies, Hz
 *   w    [C][B][N][2] complex weights (re, im)
 *   x    [C][T][N][2] complex voltages (re, im), int8 or double
 *   p    [C][B][T/I]  integrated power
 * Preconditions (not checked beyond returning -1): sizes >= 1, T % I == 0,
 * non-null pointers.
 */
#ifndef BF_ORACLE_H
#define BF_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define BFO_C0 299792458.0 /* m/s */

int bfo_weights(int32_t N, int32_t C, int32_t B, const double* pos, const double* dir,
                const double* freq, double* w);

int bfo_beamform_i8(int32_t N, int32_t C, int32_t B, int64_t T, int32_t I,
                    const double* w, const int8_t* x, double* p);

int bfo_beamform_f64(int32_t N, int32_t C, int32_t B, int64_t T, int32_t I,
                     const double* w, const double* x, double* p);

/* complex beams before detection: beams [C][B][T][2] */
int bfo_beams_f64(int32_t N, int32_t C, int32_t B, int64_t T,
                  const double* w, const double* x, double* beams);

int bfo_max_threads(void);
void bfo_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
