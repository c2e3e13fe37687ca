// bf_api.cpp -- host runtime of the beamformer: plans, validation, tile
// choice, weight upload, launches and the batching form.  Every entry point
// is extern "C", returns a status code and never lets an exception escape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/bf.h"
#include "bf_internal.h"

using bf::Launch;
using bf::Prob;
using bf::Tile;

struct bf_plan_s {
  int32_t N = 0, C = 0, B = 0, I = 0;
  int64_t T = 0;
  int prec = 0;
  uint32_t flags = 0;
  int32_t Bpad = 0, Kpad = 0;
  int mode = 0;
  bool vec16 = true;
  bool in4 = false;  // 4-bit complex input (one byte per antenna sample)
  bool cx = false;   // complex beam output (FP16 pairs) instead of power
  float out_scale = 1.0f;
  Tile tile{4, 1, 1};
  int32_t sgw = 1;
  int device = 0;
  int n_cu = 256;
  size_t w_bytes = 0;
  void* w_dev = nullptr;  // the weights runs read
  bool weights_set = false;
  // geometry staging for bf_set_weights: pinned host + device, reused
  // (positions, directions, frequencies, antenna mask)
  double* geo_host = nullptr;
  double* geo_dev = nullptr;
  size_t geo_count = 0;
  hipEvent_t geo_done = nullptr;  // recorded after the last weight kernel read geo_dev
  bool geo_pending = false;
  std::vector<double> mask;  // [N], 1 = antenna used
  // asynchronous refresh (bf_set_weights_async): a second buffer, filled on
  // the caller's stream while runs read w_dev; the next run waits for it and
  // swaps.  used_cur / used_alt mark the last run that read each buffer.
  void* w_alt = nullptr;
  hipEvent_t w_ready = nullptr;
  hipEvent_t used_cur = nullptr, used_alt = nullptr;
  bool refresh_pending = false;
};

struct bf_batch_s {
  std::vector<bf_plan_t> plans;
  int32_t* queue = nullptr;
  int device = 0;
};

struct bf_table_s {
  int32_t N = 0, I = 0;
  int prec = 0, mode = 0;
  bool in4 = false;
  int32_t Kpad = 0;
  size_t lds = 0;     // fixed dynamic LDS of every launch
  int grid = 1;       // fixed persistent grid: CUs x workgroups per CU
  int device = 0;
  int n_cu = 256;
  int32_t* queue = nullptr;
  Launch* table = nullptr;  // device copy of the set table
};

namespace {

constexpr int kMaxN = 4096;
constexpr int kMaxB = 65536;
constexpr int kMaxC = 1 << 24;
constexpr size_t kLdsMax = 160 * 1024 - 256;  // dynamic LDS; the rest is static

int es_of(int prec) { return prec == BF_FP32 ? 4 : 2; }

size_t lds_bytes(int prec, int Kpad, int nbt) {
  return (size_t)2 * 16 * nbt * ((size_t)Kpad * es_of(prec) + bf::kLdsPad);
}

// Dynamic LDS of a tile: the unit's weight rows, none when they are read
// from device memory.
size_t tile_lds(int prec, int Kpad, Tile t) { return t.kres < 0 ? 0 : lds_bytes(prec, Kpad, t.nbt); }

int mode_of(int32_t I) {
  return I == 1 ? bf::kModeI1 : I == 2 ? bf::kModeI2 : (I % 4 == 0 ? bf::kModeGen4 : bf::kModeGen);
}

// Geometry of the row-tile schedule for integration I (see bf_beamform.inc).
void schedule(int32_t I, int64_t T, int32_t* G, int32_t* QI, int32_t* SG) {
  int64_t W = T / I;
  if (I == 1) {
    *G = 1;
    *QI = 1;
  } else if (I == 2) {
    *G = 2;
    *QI = 1;
  } else {
    *QI = (I + 3) / 4;
    *G = 4 * *QI;
  }
  *SG = (int32_t)((W + 15) / 16);
}

int gcd(int a, int b) { return b ? gcd(b, a % b) : a; }

const Tile kVecTiles[] = {
#define BF_TILE(MT, NBT, NBP, KRES) Tile{MT, NBT, NBP, KRES},
    BF_TILE_LIST_VEC16
#undef BF_TILE
};
const Tile kMultiTiles[] = {
#define BF_TILE(MT, NBT, NBP, KRES) Tile{MT, NBT, NBP, KRES},
    BF_TILE_LIST_MULTI
#undef BF_TILE
};
const Tile kGenTiles[] = {
#define BF_TILE(MT, NBT, NBP, KRES) Tile{MT, NBT, NBP, KRES},
    BF_TILE_LIST_GENERIC
#undef BF_TILE
};
const Tile kIn4Tiles[] = {
#define BF_TILE(MT, NBT, NBP, KRES) Tile{MT, NBT, NBP, KRES},
    BF_TILE_LIST_IN4
#undef BF_TILE
};
const Tile kCxTiles[] = {
#define BF_TILE(MT, NBT, NBP, KRES) Tile{MT, NBT, NBP, KRES},
    BF_TILE_LIST_CX
#undef BF_TILE
};

bool same_tile(const Tile& a, const Tile& b) {
  return a.mt == b.mt && a.nbt == b.nbt && a.nbp == b.nbp && a.kres == b.kres;
}

// The single-set variants compiled for a plan's output, input format and
// row width.
template <class F>
void for_each_tile(const bf_plan_s* p, F f) {
  if (p->cx && p->vec16)
    for (const Tile& x : kCxTiles) f(x);
  else if (p->in4)
    for (const Tile& x : kIn4Tiles) f(x);
  else if (p->vec16)
    for (const Tile& x : kVecTiles) f(x);
  else
    for (const Tile& x : kGenTiles) f(x);
}

bool tile_exists(const bf_plan_s* p, Tile t) {
  bool found = false;
  for_each_tile(p, [&](const Tile& x) { found = found || same_tile(x, t); });
  return found;
}

// Work units per bf_run for a tile/sgw choice.
int64_t units_for(const bf_plan_s* p, Tile t, int32_t sgw) {
  int32_t G, QI, SG;
  schedule(p->I, p->T, &G, &QI, &SG);
  int64_t nbr = (p->Bpad / 16 + t.nbt - 1) / t.nbt;
  int64_t ntr = (SG + (int64_t)bf::kWaves * sgw - 1) / ((int64_t)bf::kWaves * sgw);
  return (int64_t)p->C * nbr * ntr;
}

// Whether a compiled tile can run plan p.
bool tile_ok(const bf_plan_s* p, Tile t) {
  if (!tile_exists(p, t)) return false;
  if (t.kres > 0 && p->Kpad / bf::kChunk > t.kres) return false;
  return tile_lds(p->prec, p->Kpad, t) <= kLdsMax;
}

// Default tile: the largest beam range whose weight slice fits 80 KB of LDS
// (two workgroups per CU) without exceeding the plan's beams; voltages held
// in registers when K <= 128 (MT = 8 for FP16/BF16 at K <= 64, where the
// per-pass fragment reuse matters most); streamed K otherwise.  Then
// enough store groups per wave that a launch has >= 8 workgroups per CU,
// capped at 256 row tiles per wave per unit.
void choose_tile(bf_plan_s* p) {
  const int need = p->Bpad / 16;
  const int nch = p->Kpad / bf::kChunk;
  int nbt = 8;
  while (nbt > 1 && (lds_bytes(p->prec, p->Kpad, nbt) > 80 * 1024 || nbt / 2 >= need)) nbt /= 2;
  Tile t{4, 1, 1, 0};
  if (lds_bytes(p->prec, p->Kpad, 1) > kLdsMax) {
    t = Tile{4, 2, 2, -1};  // one beam tile's weights do not fit LDS
  } else if (!p->vec16) {
    t = nbt == 8 ? Tile{4, 8, 2, 0} : Tile{4, 1, 1, 0};
  } else if (nch == 1 && nbt >= 4) {
    t = (p->prec == BF_FP32 || p->in4 || p->cx) ? Tile{4, nbt, 1, 1} : Tile{8, nbt, 1, 1};
  } else if (nch == 2 && nbt >= 4) {
    t = Tile{4, nbt, 1, 2};
  } else {
    t = nbt >= 4 ? Tile{4, nbt, 2, 0} : nbt == 2 ? Tile{4, 2, 2, 0} : Tile{4, 1, 1, 0};
  }
  // the 4-bit and complex-output variants carry fewer forms: fall back to
  // the streamed form of the same beam range
  if (!tile_ok(p, t) && nbt >= 2) t = Tile{4, nbt, 2, 0};
  if (!tile_ok(p, t) && nbt >= 2) t = Tile{4, 2, 2, 0};
  if (!tile_ok(p, t)) t = Tile{4, 1, 1, 0};
  if (!tile_ok(p, t)) t = Tile{4, 2, 2, -1};
  int32_t G, QI, SG;
  schedule(p->I, p->T, &G, &QI, &SG);
  const int32_t base = t.mt / gcd(t.mt, G);  // sgw * G must be a multiple of MT
  int32_t sgw = base;
  const int64_t want = (int64_t)p->n_cu * 8;
  for (int32_t k = 2;; ++k) {
    int32_t s = base * k;
    if ((int64_t)s * G > 256 || units_for(p, t, s) < want) break;
    if ((int64_t)(s - base) * bf::kWaves >= SG) break;
    sgw = s;
  }
  p->tile = t;
  p->sgw = sgw;
}

Prob make_prob(const bf_plan_s* p, const int8_t* x, float* out, int64_t unit_begin) {
  Prob q;
  std::memset(&q, 0, sizeof(q));
  q.x = x;
  q.p = out;
  q.w = p->w_dev;
  q.T = p->T;
  q.W = p->T / p->I;
  q.unit_begin = unit_begin;
  q.N = p->N;
  q.C = p->C;
  q.B = p->B;
  q.I = p->I;
  q.Bpad = p->Bpad;
  q.Kpad = p->Kpad;
  int32_t G, QI, SG;
  schedule(p->I, p->T, &G, &QI, &SG);
  q.G = G;
  q.QI = QI;
  q.SG = SG;
  q.sgw = p->sgw;
  q.nbr = (p->Bpad / 16 + p->tile.nbt - 1) / p->tile.nbt;
  q.ntr = (int32_t)((SG + (int64_t)bf::kWaves * p->sgw - 1) / ((int64_t)bf::kWaves * p->sgw));
  q.accumulate = (p->flags & BF_ACCUMULATE) ? 1 : 0;
  q.variant = -1;
  // several beam ranges per channel: a time range's voltage rows (its
  // share of the channel block) serve every beam range from L2 if those
  // units run together, whereas one beam range's weights are small
  q.br_fast = q.nbr > 1 ? 1 : 0;
  q.out_scale = p->out_scale;
  return q;
}

thread_local char g_last_error[256] = "no error";

int from_hip(hipError_t e) {
  if (e == hipSuccess) return BF_OK;
  (void)hipGetLastError();  // the status is returned; do not leave it pending for others
  std::snprintf(g_last_error, sizeof(g_last_error), "%s (%d): %s", hipGetErrorName(e), (int)e,
                hipGetErrorString(e));
  if (e == hipErrorOutOfMemory) return BF_ERR_OOM;
  return BF_ERR_HIP;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// The set table of a batched launch: each set's tile (its own if the
// persistent kernel carries it, else the closest carried variant whose LDS
// fits lds_cap), unit ranges and the largest LDS size any set needs.
// Byte-load sets (2N % 16 != 0) share one generic variant (*common).
int fill_sets(const bf_plan_t* plans, int n, const int8_t* const* x, float* const* out,
              size_t lds_cap, Launch* L, size_t* lds_out, Tile* common) {
  std::memset(L, 0, sizeof(*L));
  for (int i = 0; i < n; ++i) {
    const bf_plan_s* p = plans[i];
    if (!x[i] || !out[i] || !aligned16(x[i]) || !aligned16(out[i])) return BF_ERR_INVALID_ARG;
    if (!p->weights_set) return BF_ERR_STATE;
    // the batching kernels stage weights in LDS
    if (lds_bytes(p->prec, p->Kpad, 1) > lds_cap) return BF_ERR_UNSUPPORTED;
  }
  int64_t begin = 0;
  size_t lds = 0;
  const bool multi = plans[0]->vec16;
  *common = Tile{4, 1, 1, 0};
  if (!multi) {
    std::vector<Tile> cand;
    for (int i = 0; i < n; ++i) cand.push_back(plans[i]->tile);
    std::stable_sort(cand.begin(), cand.end(),
                     [](const Tile& a, const Tile& b) { return a.nbt > b.nbt; });
    for (const Tile& c : cand) {
      bool ok = true;
      for (int i = 0; i < n && ok; ++i) ok = tile_ok(plans[i], c);
      if (ok) {
        *common = c;
        break;
      }
    }
  }
  for (int i = 0; i < n; ++i) {
    bf_plan_s tmp = *plans[i];  // the same set under its launch tile
    Tile t = *common;
    int variant = -1;
    if (multi) {
      const int nm = (int)(sizeof(kMultiTiles) / sizeof(kMultiTiles[0]));
      auto fits = [&](const Tile& c) {
        return tile_ok(&tmp, c) && lds_bytes(tmp.prec, tmp.Kpad, c.nbt) <= lds_cap;
      };
      for (int v = 0; v < nm && variant < 0; ++v) {
        const Tile& c = kMultiTiles[v];
        if (c.mt == tmp.tile.mt && c.nbt == tmp.tile.nbt && c.nbp == tmp.tile.nbp &&
            c.kres == tmp.tile.kres && fits(c))
          variant = v;
      }
      for (int v = 0; v < nm && variant < 0; ++v)
        if (fits(kMultiTiles[v]) && kMultiTiles[v].kres == tmp.tile.kres &&
            kMultiTiles[v].nbt <= tmp.tile.nbt)
          variant = v;
      for (int v = 0; v < nm && variant < 0; ++v)
        if (fits(kMultiTiles[v])) variant = v;
      if (variant < 0) return BF_ERR_UNSUPPORTED;
      t = kMultiTiles[variant];
    }
    int32_t G, QI, SG;
    schedule(tmp.I, tmp.T, &G, &QI, &SG);
    const int32_t base = t.mt / gcd(t.mt, G);
    const bool same = t.mt == tmp.tile.mt && t.nbt == tmp.tile.nbt && t.nbp == tmp.tile.nbp &&
                      t.kres == tmp.tile.kres;
    tmp.tile = t;
    tmp.sgw = same ? tmp.sgw : std::max(base, tmp.sgw / base * base);
    L->prob[i] = make_prob(&tmp, x[i], out[i], begin);
    L->prob[i].variant = variant;
    begin += units_for(&tmp, t, tmp.sgw);
    lds = std::max(lds, lds_bytes(tmp.prec, tmp.Kpad, t.nbt));
  }
  if (lds > lds_cap) return BF_ERR_UNSUPPORTED;
  L->nprob = n;
  L->total_units = begin;
  L->xcd_remap = 0;
  *lds_out = lds;
  return BF_OK;
}

// Validates the geometry and enqueues its upload and the weight kernel on
// s, writing the operand-layout weights of plan p (with its antenna mask)
// into dst.
int generate_weights(bf_plan_s* p, const double* pos, const double* dir, const double* freq,
                     void* dst, hipStream_t s) {
  if (!pos || !dir || !freq) return BF_ERR_INVALID_ARG;
  for (int64_t i = 0; i < 3 * (int64_t)p->N; ++i)
    if (!std::isfinite(pos[i])) return BF_ERR_INVALID_ARG;
  for (int b = 0; b < p->B; ++b) {
    const double* d = dir + 3 * b;
    if (!std::isfinite(d[0]) || !std::isfinite(d[1]) || !std::isfinite(d[2]))
      return BF_ERR_INVALID_ARG;
    double nrm = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (std::fabs(nrm - 1.0) > 1e-9) return BF_ERR_INVALID_ARG;
  }
  for (int c = 0; c < p->C; ++c)
    if (!std::isfinite(freq[c]) || !(freq[c] > 0.0)) return BF_ERR_INVALID_ARG;
  // the previous weight kernel must have finished reading the staging area
  if (p->geo_pending) {
    hipError_t e = hipEventSynchronize(p->geo_done);
    if (e != hipSuccess) return from_hip(e);
    p->geo_pending = false;
  }
  double* h = p->geo_host;
  const int N = p->N, B = p->B, C = p->C;
  std::memcpy(h, pos, sizeof(double) * 3 * N);
  std::memcpy(h + 3 * N, dir, sizeof(double) * 3 * B);
  std::memcpy(h + 3 * N + 3 * B, freq, sizeof(double) * C);
  std::memcpy(h + 3 * N + 3 * B + C, p->mask.data(), sizeof(double) * N);
  hipError_t e = hipMemcpyAsync(p->geo_dev, h, p->geo_count * sizeof(double),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return from_hip(e);
  const double* d = p->geo_dev;
  e = bf::launch_weights_geom(p->prec, d, d + 3 * N, d + 3 * N + 3 * B, d + 3 * N + 3 * B + C, N,
                              C, B, p->Bpad, p->Kpad, dst, s);
  if (e != hipSuccess) return from_hip(e);
  e = hipEventRecord(p->geo_done, s);
  if (e != hipSuccess) return from_hip(e);
  p->geo_pending = true;
  return BF_OK;
}

// A run on stream s is about to read the plan's weights: take a finished
// asynchronous refresh (the stream waits for it) and swap buffers.
hipError_t take_refresh(bf_plan_s* p, hipStream_t s) {
  if (!p->refresh_pending) return hipSuccess;
  hipError_t e = hipStreamWaitEvent(s, p->w_ready, 0);
  if (e != hipSuccess) return e;
  std::swap(p->w_dev, p->w_alt);
  std::swap(p->used_cur, p->used_alt);
  p->refresh_pending = false;
  p->weights_set = true;
  return hipSuccess;
}

// After a launch on s that read the plan's current buffer.
hipError_t mark_used(bf_plan_s* p, hipStream_t s) {
  return p->used_cur ? hipEventRecord(p->used_cur, s) : hipSuccess;
}

}  // namespace

extern "C" {

const char* bf_strerror(int status) {
  switch (status) {
    case BF_OK: return "success";
    case BF_ERR_INVALID_ARG: return "invalid argument";
    case BF_ERR_OOM: return "out of memory";
    case BF_ERR_HIP: return "HIP runtime error";
    case BF_ERR_STATE: return "invalid state (weights not set?)";
    case BF_ERR_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

const char* bf_version(void) { return "bf 0.1 gfx950"; }

const char* bf_last_hip_error(void) { return g_last_error; }

int bf_plan_create_ex(bf_plan_t* out, int32_t N, int32_t C, int32_t B, int64_t T, int32_t I,
                      bf_precision_t precision, uint32_t flags) {
  try {
    if (!out) return BF_ERR_INVALID_ARG;
    *out = nullptr;
    if (N < 1 || N > kMaxN || C < 1 || C > kMaxC || B < 1 || B > kMaxB || T < 1 || I < 1 ||
        T % I != 0 || T > ((int64_t)1 << 40))
      return BF_ERR_INVALID_ARG;
    if (precision != BF_FP32 && precision != BF_FP16 && precision != BF_BF16)
      return BF_ERR_INVALID_ARG;
    if (flags & ~(BF_ACCUMULATE | BF_INPUT_4BIT | BF_OUTPUT_COMPLEX)) return BF_ERR_INVALID_ARG;
    // complex beams are per sample and overwrite their output
    if ((flags & BF_OUTPUT_COMPLEX) && (I != 1 || (flags & BF_ACCUMULATE)))
      return BF_ERR_INVALID_ARG;
    // 4-bit rows are read 8 bytes (8 antennas) at a time
    if ((flags & BF_INPUT_4BIT) && N % 8 != 0) return BF_ERR_UNSUPPORTED;
    bf_plan_s* p = new (std::nothrow) bf_plan_s();
    if (!p) return BF_ERR_OOM;
    p->N = N;
    p->C = C;
    p->B = B;
    p->T = T;
    p->I = I;
    p->prec = precision;
    p->flags = flags;
    p->Bpad = (B + 15) / 16 * 16;
    p->Kpad = (2 * N + bf::kChunk - 1) / bf::kChunk * bf::kChunk;
    p->mode = mode_of(I);
    p->vec16 = (2 * N) % 16 == 0;
    p->in4 = (flags & BF_INPUT_4BIT) != 0;
    p->cx = (flags & BF_OUTPUT_COMPLEX) != 0;
    if (p->cx) p->mode = bf::kModeCx;
    if (hipGetDevice(&p->device) != hipSuccess) {
      delete p;
      return BF_ERR_HIP;
    }
    (void)hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
    if (p->n_cu < 1) p->n_cu = 256;
    choose_tile(p);
    p->w_bytes = (size_t)C * p->Bpad * 2 * p->Kpad * es_of(p->prec);
    hipError_t e = hipMalloc(&p->w_dev, p->w_bytes);
    if (e != hipSuccess) {
      delete p;
      return from_hip(e);
    }
    // no clearing: both weight kernels write every element of the buffer
    // (padding included), and nothing reads it before one of them has run
    p->geo_count = (size_t)3 * N + (size_t)3 * B + (size_t)C + (size_t)N;
    p->mask.assign(N, 1.0);
    e = hipHostMalloc((void**)&p->geo_host, p->geo_count * sizeof(double), 0);
    if (e == hipSuccess) e = hipMalloc(&p->geo_dev, p->geo_count * sizeof(double));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->geo_done, hipEventDisableTiming);
    if (e != hipSuccess) {
      bf_plan_destroy(p);
      return from_hip(e);
    }
    *out = p;
    return BF_OK;
  } catch (...) {
    return BF_ERR_OOM;
  }
}

int bf_plan_create(bf_plan_t* out, int32_t N, int32_t C, int32_t B, int64_t T, int32_t I) {
  return bf_plan_create_ex(out, N, C, B, T, I, BF_FP32, 0u);
}

int bf_plan_destroy(bf_plan_t p) {
  if (!p) return BF_OK;
  try {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    if (p->w_dev) (void)hipFree(p->w_dev);
    if (p->geo_dev) (void)hipFree(p->geo_dev);
    if (p->geo_host) (void)hipHostFree(p->geo_host);
    if (p->geo_done) (void)hipEventDestroy(p->geo_done);
    if (p->w_alt) (void)hipFree(p->w_alt);
    if (p->w_ready) (void)hipEventDestroy(p->w_ready);
    if (p->used_cur) (void)hipEventDestroy(p->used_cur);
    if (p->used_alt) (void)hipEventDestroy(p->used_alt);
    (void)hipSetDevice(dev);
    delete p;
    return BF_OK;
  } catch (...) {
    return BF_ERR_HIP;
  }
}

int bf_set_weights(bf_plan_t p, const double* pos, const double* dir, const double* freq,
                   void* stream) {
  try {
    if (!p) return BF_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int st = generate_weights(p, pos, dir, freq, p->w_dev, s);
    if (st != BF_OK) return st;
    p->refresh_pending = false;  // superseded
    p->weights_set = true;
    return BF_OK;
  } catch (...) {
    return BF_ERR_HIP;
  }
}

int bf_set_weights_async(bf_plan_t p, const double* pos, const double* dir, const double* freq,
                         void* stream) {
  try {
    if (!p) return BF_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!p->w_alt) {
      void* alt = nullptr;
      hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
      hipError_t e = hipMalloc(&alt, p->w_bytes);
      for (int i = 0; i < 3 && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
      if (e != hipSuccess) {  // leave the plan as it was
        for (hipEvent_t x : ev)
          if (x) (void)hipEventDestroy(x);
        if (alt) (void)hipFree(alt);
        return from_hip(e);
      }
      p->w_alt = alt;
      p->w_ready = ev[0];
      p->used_cur = ev[1];
      p->used_alt = ev[2];
    }
    // the runs that read the spare buffer must have finished (an event never
    // recorded is complete), and a refresh not yet taken is overwritten in
    // order after itself
    hipError_t e = hipStreamWaitEvent(s, p->used_alt, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p->w_ready, 0);
    if (e != hipSuccess) return from_hip(e);
    const int st = generate_weights(p, pos, dir, freq, p->w_alt, s);
    if (st != BF_OK) return st;
    e = hipEventRecord(p->w_ready, s);
    if (e != hipSuccess) return from_hip(e);
    p->refresh_pending = true;
    return BF_OK;
  } catch (...) {
    return BF_ERR_HIP;
  }
}

int bf_beam_pattern(bf_plan_t p, const double* pos, const double* freq, const double* grid_dir,
                    int32_t n_dirs, float* p_dev, void* stream) {
  try {
    if (!p || !pos || !freq || !grid_dir || !p_dev || n_dirs < 1 || n_dirs > (1 << 24) ||
        ((uintptr_t)p_dev & 3u) != 0)
      return BF_ERR_INVALID_ARG;
    if (!p->weights_set && !p->refresh_pending) return BF_ERR_STATE;
    for (int64_t i = 0; i < 3 * (int64_t)p->N; ++i)
      if (!std::isfinite(pos[i])) return BF_ERR_INVALID_ARG;
    for (int c = 0; c < p->C; ++c)
      if (!std::isfinite(freq[c]) || !(freq[c] > 0.0)) return BF_ERR_INVALID_ARG;
    for (int g = 0; g < n_dirs; ++g) {
      const double* d = grid_dir + 3 * (int64_t)g;
      if (!std::isfinite(d[0]) || !std::isfinite(d[1]) || !std::isfinite(d[2]))
        return BF_ERR_INVALID_ARG;
      if (std::fabs(std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - 1.0) > 1e-9)
        return BF_ERR_INVALID_ARG;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = take_refresh(p, s);
    if (e != hipSuccess) return from_hip(e);
    const size_t nd = (size_t)3 * p->N + (size_t)p->C + (size_t)3 * n_dirs;
    std::vector<double> h(nd);
    std::memcpy(h.data(), pos, sizeof(double) * 3 * p->N);
    std::memcpy(h.data() + 3 * p->N, freq, sizeof(double) * p->C);
    std::memcpy(h.data() + 3 * p->N + p->C, grid_dir, sizeof(double) * 3 * (size_t)n_dirs);
    double* d = nullptr;
    e = hipMalloc(&d, nd * sizeof(double));
    if (e != hipSuccess) return from_hip(e);
    e = hipMemcpyAsync(d, h.data(), nd * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = bf::launch_beam_pattern(p->prec, p->w_dev, d, d + 3 * p->N + p->C, d + 3 * p->N,
                                  p->N, p->C, p->B, p->Bpad, p->Kpad, n_dirs, p_dev, s);
    if (e == hipSuccess) e = mark_used(p, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(d);
    if (e != hipSuccess) return from_hip(e);
    return from_hip(e2);
  } catch (...) {
    return BF_ERR_HIP;
  }
}

int bf_plan_set_antenna_mask(bf_plan_t p, const uint8_t* mask) {
  if (!p) return BF_ERR_INVALID_ARG;
  for (int n = 0; n < p->N; ++n) p->mask[n] = (!mask || mask[n]) ? 1.0 : 0.0;
  return BF_OK;
}

int bf_set_weights_raw(bf_plan_t p, const double* w, void* stream) {
  try {
    if (!p || !w) return BF_ERR_INVALID_ARG;
    const size_t n = (size_t)p->C * p->B * p->N * 2;
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(w[i])) return BF_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double* dw = nullptr;
    hipError_t e = hipMalloc(&dw, n * sizeof(double));
    if (e != hipSuccess) return from_hip(e);
    e = hipMemcpyAsync(dw, w, n * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = bf::launch_weights_raw(p->prec, dw, p->N, p->C, p->B, p->Bpad, p->Kpad, p->w_dev, s);
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(dw);
    if (e != hipSuccess) return from_hip(e);
    if (e2 != hipSuccess) return from_hip(e2);
    p->refresh_pending = false;  // superseded
    p->weights_set = true;
    return BF_OK;
  } catch (...) {
    return BF_ERR_HIP;
  }
}

int bf_get_weights(bf_plan_t p, double* out, void* stream) {
  try {
    if (!p || !out) return BF_ERR_INVALID_ARG;
    if (!p->weights_set && !p->refresh_pending) return BF_ERR_STATE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::vector<uint8_t> buf(p->w_bytes);
    // the weights the next run reads: a pending refresh once it is written
    const void* src = p->refresh_pending ? p->w_alt : p->w_dev;
    hipError_t e = p->refresh_pending ? hipStreamWaitEvent(s, p->w_ready, 0) : hipSuccess;
    if (e == hipSuccess)
      e = hipMemcpyAsync(buf.data(), src, p->w_bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return from_hip(e);
    auto val = [&](size_t idx) -> double {
      if (p->prec == BF_FP32) {
        float f;
        std::memcpy(&f, buf.data() + idx * 4, 4);
        return f;
      }
      uint16_t h;
      std::memcpy(&h, buf.data() + idx * 2, 2);
      if (p->prec == BF_BF16) {
        uint32_t u = (uint32_t)h << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return f;
      }
      // binary16 -> double
      int sgn = h >> 15, ex = (h >> 10) & 31, man = h & 1023;
      double v = ex == 0 ? std::ldexp((double)man, -24)
                         : ex == 31 ? (man ? NAN : INFINITY) : std::ldexp(1024.0 + man, ex - 25);
      return sgn ? -v : v;
    };
    for (int64_t c = 0; c < p->C; ++c)
      for (int64_t b = 0; b < p->B; ++b) {
        size_t row = ((size_t)c * p->Bpad + b) * 2 * p->Kpad;  // re-row
        for (int64_t n = 0; n < p->N; ++n) {
          double* o = out + ((c * p->B + b) * p->N + n) * 2;
          o[0] = val(row + 2 * n);
          o[1] = -val(row + 2 * n + 1);
        }
      }
    return BF_OK;
  } catch (...) {
    return BF_ERR_HIP;
  }
}

int bf_run(bf_plan_t p, const int8_t* x, float* out, void* stream) {
  try {
    if (!p || !x || !out || !aligned16(x) || !aligned16(out)) return BF_ERR_INVALID_ARG;
    if (!p->weights_set && !p->refresh_pending) return BF_ERR_STATE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = take_refresh(p, s);
    if (e != hipSuccess) return from_hip(e);
    Launch L;
    std::memset(&L, 0, sizeof(L));
    L.prob[0] = make_prob(p, x, out, 0);
    L.nprob = 1;
    L.total_units = units_for(p, p->tile, p->sgw);
    L.queue = nullptr;
    L.xcd_remap = 1;
    const int64_t grid = (L.total_units + 7) / 8 * 8;
    if (grid > 0x7FFFFFFF) return BF_ERR_UNSUPPORTED;
    e = bf::launch_beamform(p->prec, p->mode, p->vec16, p->in4, p->tile, L, (int)grid,
                            tile_lds(p->prec, p->Kpad, p->tile), s);
    if (e == hipSuccess) e = mark_used(p, s);
    return from_hip(e);
  } catch (...) {
    return BF_ERR_HIP;
  }
}

int bf_plan_info(bf_plan_t p, bf_plan_info_t* info) {
  if (!p || !info) return BF_ERR_INVALID_ARG;
  std::memset(info, 0, sizeof(*info));
  info->n_antennas = p->N;
  info->n_channels = p->C;
  info->n_beams = p->B;
  info->integration = p->I;
  info->n_samples = p->T;
  info->precision = p->prec;
  info->k_padded = p->Kpad;
  info->beams_padded = p->Bpad;
  info->tile_mt = p->tile.mt;
  info->tile_nbt = p->tile.nbt;
  info->tile_nbp = p->tile.nbp;
  info->tile_kres = p->tile.kres;
  info->sg_per_wave = p->sgw;
  info->work_units = units_for(p, p->tile, p->sgw);
  info->weight_bytes = (int64_t)p->w_bytes;
  info->lds_bytes = (int64_t)tile_lds(p->prec, p->Kpad, p->tile);
  info->flops = 8.0 * p->C * (double)p->B * (double)p->T * p->N;
  return BF_OK;
}

int bf_plan_set_tile(bf_plan_t p, int32_t mt, int32_t nbt, int32_t nbp, int32_t kres,
                     int32_t sgw) {
  if (!p || sgw < 1) return BF_ERR_INVALID_ARG;
  Tile t{mt, nbt, nbp, kres};
  if (!tile_ok(p, t)) return BF_ERR_UNSUPPORTED;
  int32_t G, QI, SG;
  schedule(p->I, p->T, &G, &QI, &SG);
  if (((int64_t)sgw * G) % mt != 0) return BF_ERR_INVALID_ARG;
  p->tile = t;
  p->sgw = sgw;
  return BF_OK;
}

int bf_plan_set_output_scale(bf_plan_t p, float scale) {
  if (!p || !std::isfinite(scale) || !(scale > 0.0f)) return BF_ERR_INVALID_ARG;
  if (!p->cx) return BF_ERR_STATE;
  p->out_scale = scale;
  return BF_OK;
}

int bf_plan_tile_candidates(bf_plan_t p, int32_t* tiles, int32_t max_tiles) {
  if (!p || max_tiles < 0 || (max_tiles > 0 && !tiles)) return BF_ERR_INVALID_ARG;
  int32_t n = 0;
  auto add = [&](const Tile& t) {
    if (!tile_ok(p, t)) return;
    if (n < max_tiles) {
      tiles[4 * n + 0] = t.mt;
      tiles[4 * n + 1] = t.nbt;
      tiles[4 * n + 2] = t.nbp;
      tiles[4 * n + 3] = t.kres;
    }
    ++n;
  };
  for_each_tile(p, add);
  return n;
}

int bf_batch_tile_candidates(bf_plan_t p, int32_t* tiles, int32_t max_tiles) {
  if (!p || max_tiles < 0 || (max_tiles > 0 && !tiles)) return BF_ERR_INVALID_ARG;
  int32_t n = 0;
  if (!p->vec16 || p->cx) return 0;
  for (const Tile& t : kMultiTiles) {
    if (!tile_ok(p, t)) continue;
    if (n < max_tiles) {
      tiles[4 * n + 0] = t.mt;
      tiles[4 * n + 1] = t.nbt;
      tiles[4 * n + 2] = t.nbp;
      tiles[4 * n + 3] = t.kres;
    }
    ++n;
  }
  return n;
}

int bf_batch_create(bf_batch_t* out, const bf_plan_t* plans, int32_t n) {
  try {
    if (!out) return BF_ERR_INVALID_ARG;
    *out = nullptr;
    if (!plans || n < 1) return BF_ERR_INVALID_ARG;
    if (n > bf::kMaxProbs) return BF_ERR_UNSUPPORTED;
    for (int i = 0; i < n; ++i) {
      if (!plans[i]) return BF_ERR_INVALID_ARG;
      if (!plans[i]->weights_set && !plans[i]->refresh_pending) return BF_ERR_STATE;
      const bf_plan_s* a = plans[0];
      const bf_plan_s* b = plans[i];
      if (b->cx || b->prec != a->prec || b->mode != a->mode || b->vec16 != a->vec16 ||
          b->in4 != a->in4 || b->device != a->device)
        return BF_ERR_UNSUPPORTED;
    }
    bf_batch_s* bt = new bf_batch_s();
    bt->plans.assign(plans, plans + n);
    bt->device = plans[0]->device;
    hipError_t e = hipMalloc((void**)&bt->queue, sizeof(int32_t));
    if (e != hipSuccess) {
      delete bt;
      return from_hip(e);
    }
    *out = bt;
    return BF_OK;
  } catch (...) {
    return BF_ERR_OOM;
  }
}

int bf_batch_run(bf_batch_t bt, const int8_t* const* x, float* const* out, void* stream) {
  try {
    if (!bt || !x || !out) return BF_ERR_INVALID_ARG;
    const int n = (int)bt->plans.size();
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (int i = 0; i < n; ++i) {
      hipError_t e = take_refresh(bt->plans[i], s);
      if (e != hipSuccess) return from_hip(e);
    }
    Launch L;
    size_t lds = 0;
    Tile common{4, 1, 1, 0};
    const int st = fill_sets(bt->plans.data(), n, x, out, kLdsMax, &L, &lds, &common);
    if (st != BF_OK) return st;
    L.queue = bt->queue;
    const bf_plan_s* p0 = bt->plans[0];
    const bool multi = p0->vec16;
    int per_cu = lds <= 80 * 1024 ? 2 : 1;
    hipError_t e = hipSuccess;
    if (multi) {
      int occ = 0;
      e = bf::launch_beamform_multi(p0->prec, p0->mode, p0->in4, L, nullptr, 0, lds, s, &occ);
      if (e != hipSuccess) return from_hip(e);
      per_cu = std::max(1, occ);
    }
    int64_t grid = std::min<int64_t>(L.total_units, (int64_t)p0->n_cu * per_cu);
    if (grid < 1) grid = 1;
    e = bf::launch_queue_reset(bt->queue, s);
    if (e == hipSuccess) {
      e = multi ? bf::launch_beamform_multi(p0->prec, p0->mode, p0->in4, L, nullptr, (int)grid,
                                            lds, s, nullptr)
                : bf::launch_beamform(p0->prec, p0->mode, p0->vec16, p0->in4, common, L,
                                      (int)grid, lds, s);
    }
    for (int i = 0; i < n && e == hipSuccess; ++i) e = mark_used(bt->plans[i], s);
    return from_hip(e);
  } catch (...) {
    return BF_ERR_HIP;
  }
}

int bf_batch_destroy(bf_batch_t bt) {
  if (!bt) return BF_OK;
  (void)hipDeviceSynchronize();
  if (bt->queue) (void)hipFree(bt->queue);
  delete bt;
  return BF_OK;
}

int bf_table_create(bf_table_t* out, int32_t n_antennas, int32_t integration, int32_t precision,
                    uint32_t flags) {
  try {
    if (!out) return BF_ERR_INVALID_ARG;
    *out = nullptr;
    if (n_antennas < 1 || n_antennas > kMaxN || integration < 1) return BF_ERR_INVALID_ARG;
    if (precision != BF_FP32 && precision != BF_FP16 && precision != BF_BF16)
      return BF_ERR_INVALID_ARG;
    if (flags & ~BF_INPUT_4BIT) return BF_ERR_INVALID_ARG;
    if ((2 * n_antennas) % 16 != 0) return BF_ERR_UNSUPPORTED;
    bf_table_s* t = new bf_table_s();
    t->N = n_antennas;
    t->I = integration;
    t->prec = precision;
    t->in4 = (flags & BF_INPUT_4BIT) != 0;
    t->mode = mode_of(integration);
    t->Kpad = 64 * ((2 * n_antennas + 63) / 64);
    // one LDS size for every launch: the largest batching variant that still
    // leaves two workgroups per CU (at least the smallest variant)
    t->lds = lds_bytes(precision, t->Kpad, 1);
    for (const Tile& c : kMultiTiles) {
      const size_t l = lds_bytes(precision, t->Kpad, c.nbt);
      if (l <= 80 * 1024) t->lds = std::max(t->lds, l);
    }
    if (t->lds > kLdsMax) {
      delete t;
      return BF_ERR_UNSUPPORTED;
    }
    hipError_t e = hipGetDevice(&t->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&t->n_cu, hipDeviceAttributeMultiprocessorCount,
                                                   t->device);
    if (e == hipSuccess) e = hipMalloc((void**)&t->queue, sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&t->table, sizeof(Launch));
    int occ = 0;
    if (e == hipSuccess) {
      Launch L;
      std::memset(&L, 0, sizeof(L));
      e = bf::launch_beamform_multi(precision, t->mode, t->in4, L, t->table, 0, t->lds, nullptr,
                                    &occ);
    }
    if (e != hipSuccess) {
      if (t->queue) (void)hipFree(t->queue);
      if (t->table) (void)hipFree(t->table);
      delete t;
      return from_hip(e);
    }
    t->grid = std::max(1, t->n_cu * std::max(1, occ));
    *out = t;
    return BF_OK;
  } catch (...) {
    return BF_ERR_OOM;
  }
}

int bf_table_set(bf_table_t t, const bf_plan_t* plans, const int8_t* const* x, float* const* out,
                 int32_t n, void* stream) {
  try {
    if (!t || n < 0 || (n > 0 && (!plans || !x || !out))) return BF_ERR_INVALID_ARG;
    if (n > bf::kMaxProbs) return BF_ERR_UNSUPPORTED;
    for (int i = 0; i < n; ++i) {
      const bf_plan_s* p = plans[i];
      if (!p) return BF_ERR_INVALID_ARG;
      // a table's runs are not tracked per plan, so plans refreshed with
      // bf_set_weights_async (two weight buffers) are not accepted
      if (p->cx || p->w_alt || p->N != t->N || p->I != t->I || p->prec != t->prec ||
          p->in4 != t->in4 || p->device != t->device)
        return BF_ERR_UNSUPPORTED;
    }
    Launch L;
    std::memset(&L, 0, sizeof(L));
    if (n > 0) {
      size_t lds = 0;
      Tile common{4, 1, 1, 0};
      const int st = fill_sets(plans, n, x, out, t->lds, &L, &lds, &common);
      if (st != BF_OK) return st;
    }
    L.queue = t->queue;
    return from_hip(bf::launch_table_store(L, t->table, reinterpret_cast<hipStream_t>(stream)));
  } catch (...) {
    return BF_ERR_HIP;
  }
}

int bf_table_run(bf_table_t t, void* stream) {
  if (!t) return BF_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Launch unused;
  std::memset(&unused, 0, sizeof(unused));
  hipError_t e = bf::launch_queue_reset(t->queue, s);
  if (e == hipSuccess)
    e = bf::launch_beamform_multi(t->prec, t->mode, t->in4, unused, t->table, t->grid, t->lds, s,
                                  nullptr);
  return from_hip(e);
}

int bf_table_destroy(bf_table_t t) {
  if (!t) return BF_OK;
  (void)hipDeviceSynchronize();
  if (t->queue) (void)hipFree(t->queue);
  if (t->table) (void)hipFree(t->table);
  delete t;
  return BF_OK;
}

}  // extern "C"

namespace bf {

template <int PREC, bool IN4>
hipError_t launch_prec_in(int mode, bool vec16, Tile t, const Launch& L, int grid, size_t lds,
                          hipStream_t s);
template <int PREC, bool IN4>
hipError_t launch_multi_in(int mode, const Launch& L, const Launch* table, int grid, size_t lds,
                           hipStream_t s, int* occupancy);
#define BF_EXTERN(P, F)                                                                     \
  extern template hipError_t launch_prec_in<P, F>(int, bool, Tile, const Launch&, int, size_t, \
                                                  hipStream_t);                              \
  extern template hipError_t launch_multi_in<P, F>(int, const Launch&, const Launch*, int,    \
                                                   size_t, hipStream_t, int*);
BF_EXTERN(0, false)
BF_EXTERN(1, false)
BF_EXTERN(2, false)
BF_EXTERN(0, true)
BF_EXTERN(1, true)
BF_EXTERN(2, true)
#undef BF_EXTERN

hipError_t launch_beamform_multi(int prec, int mode, bool in4, const Launch& L,
                                 const Launch* table, int grid, size_t lds, hipStream_t s,
                                 int* occ) {
  if (in4) {
    if (prec == 0) return launch_multi_in<0, true>(mode, L, table, grid, lds, s, occ);
    if (prec == 1) return launch_multi_in<1, true>(mode, L, table, grid, lds, s, occ);
    return launch_multi_in<2, true>(mode, L, table, grid, lds, s, occ);
  }
  if (prec == 0) return launch_multi_in<0, false>(mode, L, table, grid, lds, s, occ);
  if (prec == 1) return launch_multi_in<1, false>(mode, L, table, grid, lds, s, occ);
  return launch_multi_in<2, false>(mode, L, table, grid, lds, s, occ);
}

hipError_t launch_beamform(int prec, int mode, bool vec16, bool in4, Tile tile, const Launch& L,
                           int grid, size_t lds, hipStream_t s) {
  if (in4) {
    if (prec == 0) return launch_prec_in<0, true>(mode, vec16, tile, L, grid, lds, s);
    if (prec == 1) return launch_prec_in<1, true>(mode, vec16, tile, L, grid, lds, s);
    return launch_prec_in<2, true>(mode, vec16, tile, L, grid, lds, s);
  }
  if (prec == 0) return launch_prec_in<0, false>(mode, vec16, tile, L, grid, lds, s);
  if (prec == 1) return launch_prec_in<1, false>(mode, vec16, tile, L, grid, lds, s);
  return launch_prec_in<2, false>(mode, vec16, tile, L, grid, lds, s);
}

}  // namespace bf
