/*
 * bf.h -- C ABI of the MI355X (gfx950) coherent beamformer.
 *
 * The library forms, for every frequency channel c, time sample t and beam b,
 *
 *     B[c][b][t]  = sum_n W[c][b][n] * X[c][t][n]                (Sec. 2.1)
 *     W[c][b][n]  = exp(-i 2 pi f_c (k_b . r_n) / c0)             (Eq. 1, Sec. 1)
 *     P[c][b][w]  = sum_{j<I} |B[c][b][w*I + j]|^2                (Sec. 2.1)
 *
 * i.e. a per-channel complex matrix product (beams x antennas times
 * antennas x samples; Sec. 2.1 describes it as an N_b x N_a coefficient
 * matrix applied to each antenna vector), with power detection and
 * integration over I consecutive samples fused into the same kernel so that
 * complex beams never reach device memory (Sec. 2.1 argues for fusing
 * unpacking, conversion and power into the beamformer).  Throughput is
 * counted at 8 flop per complex multiply-accumulate (Sec. 2.2).
 *
 * Conventions
 *   - Antenna positions r_n in metres (x = East, y = North, z = up), beam
 *     pointings k_b unit vectors toward the sky, channel centre frequencies
 *     f_c in Hz, c0 = 299792458 m/s.  A plane wave from k_s reaches antenna n
 *     as s(t) exp(+i 2 pi f (k_s . r_n) / c0), so a beam with k_b = k_s sums
 *     it in phase (power N^2 |s|^2).
 *   - Voltages X: device memory, int8 two's complement, layout
 *     [C][T][N][2] = (re, im) interleaved, antenna fastest.  Every value in
 *     [-128, 127] is accepted and converted exactly.
 *   - Output P: device memory, float32, layout [C][B][T/I].
 *   - Non-overlapping integration windows, aligned at t = 0; T % I == 0.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the legacy
 *     default stream).  All device work is asynchronous and stream-ordered;
 *     a call that returns BF_OK has only enqueued work.  Device faults
 *     surface at the caller's next synchronisation.
 *   - Every entry point returns a status (BF_OK or a negative BF_ERR_*)
 *     and never throws or aborts.  A plan or batch is not thread-safe;
 *     distinct handles are.
 *
 * Precision forms
 *   BF_FP32  weights rounded from FP64 to FP32; int8 voltages converted to
 *            FP32; products on FP32 matrix cores (MFMA), FP32 accumulation.
 *   BF_FP16  weights rounded from FP64 to FP16 (round to nearest even, one
 *            rounding); voltages converted exactly to FP16; FP16 MFMA with
 *            FP32 accumulation.
 *   BF_BF16  as BF_FP16 with BF16 weights and BF16 MFMA.
 *   In every form the weight phase f_c (k_b . r_n) / c0 (in cycles) is
 *   computed and reduced modulo 1 in FP64 on the device before sin/cos.
 */
#ifndef BF_H
#define BF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bf_plan_s* bf_plan_t;
typedef struct bf_batch_s* bf_batch_t;
typedef struct bf_table_s* bf_table_t;

typedef enum { BF_FP32 = 0, BF_FP16 = 1, BF_BF16 = 2 } bf_precision_t;

enum {
  BF_OK = 0,
  BF_ERR_INVALID_ARG = -1, /* bad size, null or misaligned pointer, bad value   */
  BF_ERR_OOM = -2,         /* device or pinned-host allocation failed             */
  BF_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed          */
  BF_ERR_STATE = -4,       /* e.g. bf_run before any weights were set             */
  BF_ERR_UNSUPPORTED = -5  /* valid request outside what the library implements   */
};

/* Plan flags. */
#define BF_ACCUMULATE 1u /* bf_run adds into P instead of overwriting it, so an
                            integration window can span several blocks        */
/* 4-bit complex voltages (Sec. 2.1: the F-engine emits 4-bit two's
 * complement components, one antenna sample per byte).  X is then device
 * uint8 [C][T][N], one byte per antenna sample: the real part in the high
 * nibble, the imaginary part in the low nibble, each a two's complement
 * value in [-8, 7]; N must be a multiple of 8 (else BF_ERR_UNSUPPORTED).
 * The result equals, bit for bit, the int8 form run on the same values
 * widened to [C][T][N][2].  Half the input bytes of the int8 form. */
#define BF_INPUT_4BIT 2u
/* Complex (electric-field) beam output instead of detected power (Sec. 1.1:
 * the S-engine emits selected beams as 16-bit complex words for coherent
 * downstream processing such as pulsar folding).  P is then device
 * [C][B][T] complex samples, each two IEEE binary16 values (re, im) in
 * 4 bytes, beam-major so each beam's series is contiguous: the value
 * written is s * B[c][b][t] per component (s = bf_plan_set_output_scale,
 * default 1), clamped to +-65504 and rounded to nearest even once from the
 * FP32 accumulation.  Requires integration 1 and excludes BF_ACCUMULATE
 * (else BF_ERR_INVALID_ARG); not accepted by the batching and table forms
 * (BF_ERR_UNSUPPORTED). */
#define BF_OUTPUT_COMPLEX 4u

/* Human-readable text for a status code (static storage, never NULL). */
const char* bf_strerror(int status);

/* Version string of the library build (static storage). */
const char* bf_version(void);

/* Name and text of the last HIP error this thread's calls into the library
 * turned into BF_ERR_HIP / BF_ERR_OOM ("no error" if none).  Thread-local
 * storage, valid until the thread's next failing call. */
const char* bf_last_hip_error(void);

/*
 * Tile cache (Sec. 2.2 tunes the K20 kernel's thread and accumulator counts
 * by sweeping them on the device; the autotuner here times the compiled tile
 * variants and writes the fastest per problem shape to a JSON file).
 *
 * bf_tune_load reads such a file (path: host NUL-terminated string) into a
 * process-wide table that replaces any table loaded before; it returns the
 * number of entries read (>= 0), or BF_ERR_INVALID_ARG if the file cannot be
 * read or is not a JSON object.  Entries are {"<key>": {"tile": [mt, nbt,
 * nbp, kres, sg_per_wave], ...}, ...}; entries without such a tile are
 * skipped.  If nothing was loaded explicitly, the first plan creation reads
 * the file named by the environment variable BF_TUNE_CACHE, if set.
 * From then on bf_plan_create[_ex] gives a plan the cached tile for its
 * shape when the table has one that can run it (else the built-in choice).
 * Thread-safe.
 */
int bf_tune_load(const char* path);

/*
 * The cache key of a plan's shape (for the autotuner that writes the file):
 * "gfx950/p<precision>/N<N>/B~<b>/I<I>/C~<c>/T~<t>" followed by "/in4" for
 * 4-bit input, "/cx" for complex output and "/batch" if batch != 0 (the
 * entry for the batching and table kernels), where b, c, t are the largest
 * powers of two not above B, C and T.  Writes the NUL-terminated key into
 * buf (len bytes) and returns its length, or BF_ERR_INVALID_ARG (null plan
 * or buffer, buffer too small).
 */
int bf_tune_key(bf_plan_t plan, int32_t batch, char* buf, int32_t len);

/*
 * Gives the plan the loaded cache's tile for its shape: the single-run entry
 * (batch == 0, as at creation) or the batching kernels' entry (batch != 0,
 * for a plan about to join a bf_batch or bf_table).  Returns 1 if a tile was
 * applied, 0 if the cache has no usable entry (the plan is unchanged), or
 * BF_ERR_INVALID_ARG (null plan).
 */
int bf_plan_apply_tuned(bf_plan_t plan, int32_t batch);

/*
 * Create a plan for N antennas, C channels, B beams, T samples per block and
 * integration I (all >= 1, T % I == 0, N <= 4096, B <= 65536, C <= 2^24).
 * bf_plan_create makes an FP32 plan with no flags.  The plan allocates its
 * device weight buffer (C * ceil(B/16)*16 * 2 * K rows, K = 64*ceil(N/32),
 * in the storage precision) on the current device and a small pinned host
 * staging area.  On success *out owns them until bf_plan_destroy.
 * Work units stage their beams' weights for all K = 2N in LDS up to
 * N = 1248 (FP16/BF16) or N = 608 (FP32); larger arrays read the weight
 * fragments from device memory instead (tile kres = -1, chosen
 * automatically; not accepted by the batching and table forms).
 * Errors: BF_ERR_INVALID_ARG (sizes, null out, unknown precision or flags),
 * BF_ERR_UNSUPPORTED (an unsupported flag combination such as 4-bit input
 * with N % 8 != 0), BF_ERR_OOM, BF_ERR_HIP.
 * *out is set to NULL on failure.
 */
int bf_plan_create(bf_plan_t* out, int32_t n_antennas, int32_t n_channels, int32_t n_beams,
                   int64_t n_samples, int32_t integration);
int bf_plan_create_ex(bf_plan_t* out, int32_t n_antennas, int32_t n_channels, int32_t n_beams,
                      int64_t n_samples, int32_t integration, bf_precision_t precision,
                      uint32_t flags);

/*
 * Generate the plan's weights on the device from geometry (Eq. 1 phase
 * model, Sec. 1; Sec. 3.2 recomputes them whenever pointings change):
 *   ant_xyz_m    host [N][3] double, metres
 *   beam_dir     host [B][3] double, unit vectors (|norm - 1| <= 1e-9)
 *   chan_freq_hz host [C]    double, Hz, finite and > 0
 * The host arrays are copied before return; the caller may free them at
 * once.  The phase is evaluated in FP64, reduced modulo one cycle, and each
 * weight component is rounded once to the storage precision.
 * Errors: BF_ERR_INVALID_ARG (null pointer, non-finite value, non-unit
 * direction, non-positive frequency), BF_ERR_HIP.
 */
int bf_set_weights(bf_plan_t plan, const double* ant_xyz_m, const double* beam_dir,
                   const double* chan_freq_hz, void* stream);

/*
 * Time-varying weights (Sec. 3.2: coefficients for the next pointing are
 * computed while the previous buffer is being beamformed; Sec. 3.1: tracking
 * beams).  Generates weights from geometry exactly as bf_set_weights, but
 * into a second plan-owned buffer, enqueued on `stream` (typically not the
 * stream the runs use), so it overlaps the runs in flight.  The next bf_run
 * or bf_batch_run of the plan (on any stream) waits on the device for this
 * generation to finish and then reads the new weights; runs enqueued before
 * that keep the previous ones.  The generation itself waits on the device
 * for the runs that last read the spare buffer.  The first call allocates
 * the spare buffer (the size of the weight buffer), kept until
 * bf_plan_destroy.  A later bf_set_weights or bf_set_weights_raw
 * supersedes a refresh not yet taken by a run.  The host arrays are copied
 * before return (the call may wait for the previous weight generation of
 * the plan to finish reading its staging area).  Plans refreshed this way
 * are not accepted by bf_table_set (BF_ERR_UNSUPPORTED).
 * Errors: as bf_set_weights, plus BF_ERR_OOM.
 */
int bf_set_weights_async(bf_plan_t plan, const double* ant_xyz_m, const double* beam_dir,
                         const double* chan_freq_hz, void* stream);

/*
 * Sub-arraying (Sec. 3.1: an antenna mask restricts beamforming to the
 * antennas a sub-array needs).  mask: host [N], nonzero = antenna used;
 * NULL = every antenna.  Copied; applies to the weights generated by later
 * bf_set_weights / bf_set_weights_async calls (a masked antenna gets zero
 * weights, so its voltages do not enter any beam).  Errors:
 * BF_ERR_INVALID_ARG (null plan).
 */
int bf_plan_set_antenna_mask(bf_plan_t plan, const uint8_t* mask);

/*
 * Beam-pattern (array-factor) map of the plan's weights (Sec. 3.1 simulates
 * the BEST-2 beam pattern from the beamforming coefficients over a sky grid;
 * Eq. 1): for every channel c, beam b and grid direction k_g,
 *     P[c][b][g] = | sum_n W[c][b][n] exp(+i 2 pi f_c (k_g . r_n) / c0) |^2,
 * the power the plan's beam b collects from a unit plane wave arriving from
 * k_g (N^2 on the beam's own direction for unit weights), computed with the
 * plan's rounded weights (so the map shows the precision form's real beam)
 * and the antenna mask they carry.  ant_xyz_m host [N][3], chan_freq_hz
 * host [C] (as for bf_set_weights), grid_dir host [n_dirs][3] unit vectors,
 * 1 <= n_dirs <= 2^24; p_dev device float [C][B][n_dirs], 4-byte aligned.
 * The steering phase is formed in FP64 and reduced modulo one cycle; sin/cos
 * and the sums are FP32.  A validation tool, not a hot path: it allocates a
 * device buffer for the geometry and returns after the map is complete.
 * Errors: BF_ERR_INVALID_ARG (null pointer, size, misaligned output,
 * non-finite value, non-unit direction, non-positive frequency),
 * BF_ERR_STATE (no weights), BF_ERR_OOM, BF_ERR_HIP.
 */
int bf_beam_pattern(bf_plan_t plan, const double* ant_xyz_m, const double* chan_freq_hz,
                    const double* grid_dir, int32_t n_dirs, float* p_dev, void* stream);

/*
 * bf_beam_pattern for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation): the
 * same map, computed by the same kernel, but the geometry is staged in a
 * fixed array the library holds on each GPU for the life of the process
 * (2^20 doubles, 8 MiB per device) instead of a buffer allocated per call.
 * It calls no allocator and does not wait: the three host arrays are copied
 * on `stream` before return (the caller may reuse them at once), and the map
 * is complete when `stream` reaches this point.  Arguments, layout and the
 * other errors as for bf_beam_pattern; BF_ERR_INVALID_ARG also when
 * 3 N + C + 3 n_dirs exceeds 2^20.  Every call on a GPU shares that GPU's
 * array: calls on one stream are ordered, calls on different streams of one
 * GPU that overlap in time race for it and must be serialised by the caller.
 */
int bf_beam_pattern_noalloc(bf_plan_t plan, const double* ant_xyz_m, const double* chan_freq_hz,
                            const double* grid_dir, int32_t n_dirs, float* p_dev, void* stream);

/*
 * Load arbitrary complex weights (host [C][B][N][2] double, re/im), each
 * component rounded once to the storage precision.  Synchronous (returns
 * after the device copy is complete).  Used for DFT/integer-weight tests
 * and for weights computed elsewhere.
 * Errors: BF_ERR_INVALID_ARG (null, non-finite), BF_ERR_OOM, BF_ERR_HIP.
 */
int bf_set_weights_raw(bf_plan_t plan, const double* weights, void* stream);

/*
 * Copy the plan's rounded weights back to host [C][B][N][2] double: the ones
 * the next run reads (after a pending bf_set_weights_async, those).
 * Synchronous.  Errors: BF_ERR_INVALID_ARG, BF_ERR_STATE (none set),
 * BF_ERR_HIP.
 */
int bf_get_weights(bf_plan_t plan, double* weights_out, void* stream);

/*
 * The hot path: one block.  x_dev: device int8 [C][T][N][2] (uint8 [C][T][N]
 * for a BF_INPUT_4BIT plan); p_dev: device float [C][B][T/I] (FP16 pairs
 * [C][B][T][2] for a BF_OUTPUT_COMPLEX plan); both 16-byte aligned and not
 * overlapping.  Enqueues
 * one kernel on `stream`; no host synchronisation, no allocation.
 * Errors: BF_ERR_INVALID_ARG (null or misaligned pointer, the two byte
 * ranges overlap), BF_ERR_STATE (weights never set), BF_ERR_HIP (launch
 * failure).
 */
int bf_run(bf_plan_t plan, const int8_t* x_dev, float* p_dev, void* stream);

/* Plan introspection (tile choice and sizes), filled by bf_plan_info. */
typedef struct {
  int32_t n_antennas, n_channels, n_beams, integration;
  int64_t n_samples;
  int32_t precision;      /* bf_precision_t                                     */
  int32_t k_padded;       /* 2N rounded up to a multiple of 64                  */
  int32_t beams_padded;   /* B rounded up to a multiple of 16                   */
  int32_t tile_mt;        /* 16-sample MFMA row tiles per wave step             */
  int32_t tile_nbt;       /* 16-beam tiles per workgroup                        */
  int32_t tile_nbp;       /* 16-beam tiles per accumulator pass                 */
  int32_t tile_kres;      /* 64-element K chunks held in registers (0: streamed,
                             -1: streamed, weights read from device memory) */
  int32_t sg_per_wave;    /* 16-window store groups per wave per work unit      */
  int64_t work_units;     /* workgroups of one bf_run                           */
  int64_t weight_bytes;   /* device bytes of the weight buffer                  */
  int64_t lds_bytes;      /* LDS per workgroup                                  */
  double flops;           /* 8 * C * B * T * N                                  */
  int32_t tile_tuned;     /* 1 if the tile came from the tile cache             */
} bf_plan_info_t;
int bf_plan_info(bf_plan_t plan, bf_plan_info_t* info);

/*
 * Override the plan's tile choice (used by the autotuner): mt row tiles of
 * 16 samples per wave step, nbt 16-beam tiles per workgroup, nbp beam tiles
 * per accumulator pass, kres K chunks of 64 held in registers (0 = streamed
 * K with the unit's weights in LDS, -1 = streamed K with the weights read
 * from device memory), sg_per_wave 16-window store groups per wave per work
 * unit.  A
 * combination the library does not compile, or that the plan's K or LDS
 * budget excludes, returns BF_ERR_UNSUPPORTED and leaves the plan unchanged;
 * sg_per_wave * (row tiles per store group) must be a multiple of mt
 * (else BF_ERR_INVALID_ARG).  The choice never changes the results.
 */
int bf_plan_set_tile(bf_plan_t plan, int32_t mt, int32_t nbt, int32_t nbp, int32_t kres,
                     int32_t sg_per_wave);

/*
 * Scale applied to the complex beams of a BF_OUTPUT_COMPLEX plan before
 * their FP16 rounding (so that |s B| stays within the FP16 range, e.g.
 * 1/sqrt(N) for noise-like inputs).  Takes effect for later bf_run calls.
 * Errors: BF_ERR_INVALID_ARG (null plan, scale not finite or <= 0),
 * BF_ERR_STATE (the plan does not output complex beams).
 */
int bf_plan_set_output_scale(bf_plan_t plan, float scale);

/*
 * List the compiled tile variants that can run this plan: writes up to
 * max_tiles rows of (mt, nbt, nbp, kres) into tiles[][4] and returns how
 * many exist (which may exceed max_tiles; tiles may be NULL when
 * max_tiles == 0), or BF_ERR_INVALID_ARG.
 */
int bf_plan_tile_candidates(bf_plan_t plan, int32_t* tiles, int32_t max_tiles);

/* Free the plan.  Its device memory is released on the device only after
 * the plan's own outstanding work -- weight generation, refreshes, and the
 * bf_run / bf_batch_run / bf_beam_pattern launches that read its weights --
 * has completed, through events the plan records; the call itself does not
 * wait for that work, nor for any other work on the device.  Launches of a bf_table that
 * read the plan are not tracked by the plan: they must have completed (or
 * the table must hold another set) before the plan is destroyed.
 * NULL is accepted (no-op). */
int bf_plan_destroy(bf_plan_t plan);

/*
 * Batching form: several independent plans (sub-arrays or beam sets of
 * uneven N, C, B, T; Sec. 1 mentions partitioning an array into independent
 * phased sub-arrays) run in one persistent launch: a grid sized to the
 * device whose workgroups take work units from device queues spanning all
 * sets (one queue counter per XCD; a workgroup drains its own XCD's queue,
 * which holds the channels c with c % 8 == XCD index, then helps the
 * others).  In an FP16/BF16 batch with I == 1 or I % 4 == 0, the sets whose
 * 2N exceeds 128 run in a second persistent launch of the eight-wave
 * streamed form, queued first on the same stream (one launch per kernel
 * form); when all of those sets read one voltage block, its queues hand out
 * their units channel by channel over the sets.  All
 * plans must share precision, input format and integration class (I == 1,
 * I == 2, or I >= 3) and have their weights set; up to 16 plans.  The batch
 * references the plans (they must outlive it) and owns the device queue
 * counters.
 * Errors: BF_ERR_INVALID_ARG, BF_ERR_UNSUPPORTED, BF_ERR_OOM, BF_ERR_HIP.
 */
int bf_batch_create(bf_batch_t* out, const bf_plan_t* plans, int32_t n_plans);

/* As bf_plan_tile_candidates, restricted to the variants the persistent
 * batching kernel carries (a set whose own tile is among them runs with it
 * inside a batch; otherwise the closest one is used).  Returns 0 for plans
 * with 2N % 16 != 0, which batch under one common variant. */
int bf_batch_tile_candidates(bf_plan_t plan, int32_t* tiles, int32_t max_tiles);

/* x_dev[i], p_dev[i]: host arrays of device pointers, one per plan, same
 * layout and alignment rules as bf_run; no output may overlap any set's
 * voltages or another set's output (else BF_ERR_INVALID_ARG).  One launch per
 * kernel form on `stream`, each after a one-thread queue reset kernel.  Each set's output is
 * bitwise identical to bf_run of that plan alone. */
int bf_batch_run(bf_batch_t batch, const int8_t* const* x_dev, float* const* p_dev, void* stream);

/* Free the batch (not its plans) after its own last bf_batch_run has
 * completed (an event recorded by that run; other device work is not waited
 * for).  NULL is accepted. */
int bf_batch_destroy(bf_batch_t batch);

/*
 * Table batch, for streaming use (a sequence of blocks whose set of active
 * plans changes between blocks; Sec. 2.2 and Sec. 3.2 describe beamforming
 * block after block while new pointings are prepared).  The same persistent
 * kernel as bf_batch_run, but its set table lives in device memory owned by
 * the table, so every bf_table_run enqueues the same two launches with the
 * same arguments: a hipGraph captured around one bf_table_run serves every
 * table stored afterwards.
 *
 * bf_table_create: for plans with n_antennas antennas, integration I, the
 * given precision and input format (flags: 0 or BF_INPUT_4BIT; 2 n_antennas
 * must be a multiple of 16) on the current device.  It fixes the launch:
 * for FP16/BF16 with I == 1 or I % 4 == 0 and 2N > 128 the eight-wave
 * streamed kernel (dynamic LDS of its widest beam range, one workgroup per
 * CU; sets that read one voltage block, as in serving, are handed out
 * channel by channel), else the four-wave kernel with the dynamic LDS of the
 * largest batching variant that keeps two workgroups per CU; grid = CUs x
 * workgroups per CU.  Owns a device table (a few KB) and the per-XCD queue
 * counters.
 * Errors: BF_ERR_INVALID_ARG, BF_ERR_UNSUPPORTED, BF_ERR_OOM, BF_ERR_HIP.
 */
int bf_table_create(bf_table_t* out, int32_t n_antennas, int32_t integration, int32_t precision,
                    uint32_t flags);

/* Stores the set table for the next bf_table_run on `stream`: plans[i] with
 * voltages x_dev[i] and output p_dev[i] (device pointers, layout and
 * alignment as bf_run), 0 <= n <= 16; n = 0 makes the next run a no-op.
 * Every plan must match the table's antennas, integration, precision, input
 * format and device and have its weights set; each set runs its own tile if the
 * batching kernel carries it and its LDS fits, else the closest that does.
 * The store is a one-workgroup kernel on `stream` (the table travels as its
 * argument), so the host arrays may be reused as soon as this returns; it is
 * ordered with bf_table_run only through `stream`.  Plans and buffers must
 * stay valid until the runs that use them have completed.  Each set's
 * output is bitwise identical to bf_run of that plan alone.
 * Errors: BF_ERR_INVALID_ARG, BF_ERR_UNSUPPORTED, BF_ERR_STATE, BF_ERR_HIP. */
int bf_table_set(bf_table_t table, const bf_plan_t* plans, const int8_t* const* x_dev,
                 float* const* p_dev, int32_t n, void* stream);

/* Enqueues the batched launch over the stored table on `stream` (queue reset
 * kernel + persistent kernel; no allocation, no memset, no host sync), so it
 * may be captured into a hipGraph.  Runs on one stream must not overlap: they
 * share the table and the queue counter. */
int bf_table_run(bf_table_t table, void* stream);

/* Free the table after its own last bf_table_set and bf_table_run have
 * completed (an event recorded by each call that was not made during a
 * graph capture; launches replayed from a captured graph are the caller's to
 * wait for).  NULL is accepted. */
int bf_table_destroy(bf_table_t table);

#ifdef __cplusplus
}
#endif
#endif /* BF_H */
