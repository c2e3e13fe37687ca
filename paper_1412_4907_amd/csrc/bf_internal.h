// bf_internal.h -- types shared by the host runtime and the gfx950 kernels
// of the beamformer library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bf_tiles.h"

namespace bf {

// One beam set (plan) inside a launch.  Lives in the kernel-argument
// segment, so every field is read through scalar loads.
struct Prob {
  const int8_t* x;    // [C][T][N][2] int8 (4-bit input: [C][T][N] bytes)
  float* p;           // [C][B][W] float; complex output: [C][B][T] pairs of FP16
  const void* w;      // [C][Bpad][2][Kpad] storage precision (operand layout)
  int64_t T;          // samples per block
  int64_t W;          // windows = T / I
  int64_t unit_begin; // first work unit of this set in the launch
  int32_t N, C, B, I;
  int32_t Bpad;       // B rounded up to 16
  int32_t Kpad;       // 2N rounded up to kChunk
  int32_t nbr;        // beam ranges (workgroup beam slices) per channel
  int32_t ntr;        // time ranges (work units) per channel per beam range
  int32_t sgw;        // 16-window store groups per wave per work unit
  int32_t G;          // MFMA row tiles per store group
  int32_t QI;         // MFMA row tiles per window (general mode)
  int32_t SG;         // store groups per channel
  int32_t accumulate; // add into P instead of overwriting
  int32_t variant;    // multi-variant launches: index into BF_TILE_LIST_MULTI
  int32_t br_fast;    // unit order (c, tr, br) instead of (c, br, tr): the beam
                      // ranges of one time range run back to back and share its
                      // voltages through L2
  float out_scale;    // complex output: factor applied to B before FP16 rounding
};

struct Launch {
  Prob prob[kMaxProbs];
  int64_t total_units;
  int32_t* queue;     // persistent mode: kXcds device counters, kQueueStride apart
                      // (zeroed before launch); else null
  int32_t nprob;
  int32_t xcd_remap;  // non-persistent mode: group consecutive units per XCD
  int32_t chan_units; // > 0: every set reads the same voltages (same block,
                      // C and T); the eight-wave kernels' queues then hand
                      // out all sets' units of one channel together,
                      // chan_units of them
};

// Host-side launcher for one (precision, mode, vec16, input format, tile)
// instantiation.  Returns hipSuccess or the launch error.
hipError_t launch_beamform(int prec, int mode, bool vec16, bool in4, Tile tile, const Launch& L,
                           int grid, size_t lds_bytes, hipStream_t stream);
// Persistent batching kernel (per-set variants).  table != null: the form
// that reads its set table from that device copy (L unused).
// occupancy != null only queries workgroups per CU.  wide: the eight-wave
// kernels (FP16/BF16, I == 1 or I % 4 == 0; variants index
// BF_TILE_LIST_WIDE) instead of the four-wave ones (BF_TILE_LIST_MULTI).
hipError_t launch_beamform_multi(int prec, int mode, bool in4, const Launch& L,
                                 const Launch* table, int grid, size_t lds_bytes,
                                 hipStream_t stream, int* occupancy, bool wide = false);

// Beam-pattern map: P[c][b][g] over G grid directions (device pos [N][3],
// gdir [G][3], freq [C]; weights in the plan's operand layout).
hipError_t launch_beam_pattern(int prec, const void* w, const double* pos, const double* gdir,
                               const double* freq, int N, int C, int B, int Bpad, int Kpad, int G,
                               float* out, hipStream_t stream);
// Capacity, in doubles, of the beam-pattern geometry staging array that the
// allocation-free entry point uses (3N + C + 3G values per call).
constexpr size_t kPatScratchDoubles = (size_t)1 << 20;
// Device address of that array on device `dev`, which must be current.
hipError_t pattern_scratch(int dev, double** out);

// mask: device [N], 0 drops an antenna (every weight of it is zero).
hipError_t launch_weights_geom(int prec, const double* pos, const double* dir,
                               const double* freq, const double* mask, int N, int C, int B,
                               int Bpad, int Kpad, void* w, hipStream_t stream);
hipError_t launch_weights_raw(int prec, const double* wraw, int N, int C, int B, int Bpad,
                              int Kpad, void* w, hipStream_t stream);
hipError_t launch_queue_reset(int32_t* q, hipStream_t stream);
// Stores a set table into device memory (one workgroup, vector stores), in
// stream order before the table kernel that reads it.
hipError_t launch_table_store(const Launch& L, Launch* dst, hipStream_t stream);

}  // namespace bf
