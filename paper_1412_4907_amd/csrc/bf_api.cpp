// bf_api.cpp -- host runtime of the beamformer: plans, validation, tile
// choice, weight upload, launches and the batching form.  Every entry point
// is extern "C", returns a status code and never lets an exception escape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bf.h"
#include "bf_host.h"
#include "bf_internal.h"

using bf::Launch;
using bf::Prob;
using bf::Tile;

struct bf_plan_s : bf::Shape {
  float out_scale = 1.0f;
  Tile tile{4, 1, 1, 0};
  int32_t sgw = 1;
  bool tuned = false;  // tile taken from the tile cache
  int device = 0;
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
  // swaps.  used_cur / used_alt mark the last run that read each buffer;
  // w_ready the last generation into the spare.  Together with geo_done they
  // cover every piece of device work the plan enqueues, so destroying a plan
  // waits for exactly its own work.
  void* w_alt = nullptr;
  hipEvent_t w_ready = nullptr;
  hipEvent_t used_cur = nullptr, used_alt = nullptr;
  bool refresh_pending = false;
};

struct bf_batch_s {
  std::vector<bf_plan_t> plans;
  int32_t* queue = nullptr;
  int device = 0;
  hipEvent_t last_use = nullptr;  // recorded after each bf_batch_run
};

struct bf_table_s {
  int32_t N = 0, I = 0;
  int prec = 0, mode = 0;
  bool in4 = false;
  bool wide = false;  // every set runs the eight-wave streamed form
  int32_t Kpad = 0;
  size_t lds = 0;     // fixed dynamic LDS of every launch
  int grid = 1;       // fixed persistent grid: CUs x workgroups per CU
  int device = 0;
  int n_cu = 256;
  int32_t* queue = nullptr;
  Launch* table = nullptr;  // device copy of the set table
  hipEvent_t last_use = nullptr;  // recorded after each set and (uncaptured) run
};

namespace {

using bf::choose_tile;
using bf::es_of;
using bf::kLdsMax;
using bf::lds_bytes;
using bf::same_tile;
using bf::schedule;
using bf::tile_lds;
using bf::tile_ok;
using bf::units_for;

int gcd(int a, int b) { return b ? gcd(b, a % b) : a; }

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
  const int64_t per = (int64_t)bf::waves_of(p->tile) * p->sgw;  // store groups per unit
  q.ntr = (int32_t)((SG + per - 1) / per);
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

// ---- device memory owned by handles ----
// hipFree waits for every stream of the device, so handles never use it:
// their device buffers come from a library-owned stream-ordered pool per
// device.  An allocation is made on a private stream that carries nothing
// else (so waiting for it waits for nothing but the allocation), and a
// handle's buffers are released with hipFreeAsync on a second private
// stream, after waits on the handle's own events: destroying a handle never
// waits for, or is ordered behind, other work on the device.  The pool does
// not let an allocation wait for a pending release (no internal
// dependencies): memory is reused only once its release has run.
struct DevMem {
  hipStream_t alloc = nullptr;
  hipStream_t release = nullptr;
  hipMemPool_t pool = nullptr;
};
constexpr int kMaxDevices = 64;
std::mutex g_mem_mu;
DevMem g_mem[kMaxDevices];

hipError_t dev_mem(int dev, DevMem** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mem_mu);
  DevMem& d = g_mem[dev];
  if (!d.pool) {
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    hipStream_t a = nullptr, r = nullptr;
    hipError_t e = hipMemPoolCreate(&pool, &props);
    int zero = 0;
    if (e == hipSuccess)
      e = hipMemPoolSetAttribute(pool, hipMemPoolReuseAllowInternalDependencies, &zero);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&a, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&r, hipStreamNonBlocking);
    if (e != hipSuccess) {
      if (a) (void)hipStreamDestroy(a);
      if (r) (void)hipStreamDestroy(r);
      if (pool) (void)hipMemPoolDestroy(pool);
      return e;
    }
    d.pool = pool;
    d.alloc = a;
    d.release = r;
  }
  *out = &d;
  return hipSuccess;
}

// n bytes of device memory on `dev`, usable from any stream on return.
hipError_t dev_alloc(int dev, void** ptr, size_t n) {
  *ptr = nullptr;
  DevMem* d = nullptr;
  hipError_t e = dev_mem(dev, &d);
  if (e != hipSuccess) return e;
  e = hipMallocFromPoolAsync(ptr, n, d->pool, d->alloc);
  if (e == hipSuccess) e = hipStreamSynchronize(d->alloc);
  if (e != hipSuccess && *ptr) {
    (void)hipFreeAsync(*ptr, d->alloc);
    *ptr = nullptr;
  }
  return e;
}

// Releases device buffers of `dev` once every event in `after` has
// completed (events never recorded count as complete); does not wait.
hipError_t dev_release(int dev, std::initializer_list<hipEvent_t> after,
                       std::initializer_list<void*> ptrs) {
  DevMem* d = nullptr;
  hipError_t e = dev_mem(dev, &d);
  if (e != hipSuccess) return e;
  for (hipEvent_t ev : after)
    if (ev && e == hipSuccess) e = hipStreamWaitEvent(d->release, ev, 0);
  for (void* ptr : ptrs)
    if (ptr && e == hipSuccess) e = hipFreeAsync(ptr, d->release);
  return e;
}

// Pinned host staging buffers are recycled rather than freed (hipHostFree
// may wait for the device): a released buffer is kept for a later plan.
struct Pinned {
  void* p;
  size_t n;
};
std::mutex g_pin_mu;
std::vector<Pinned> g_pinned;

hipError_t pinned_acquire(size_t n, void** out) {
  {
    std::lock_guard<std::mutex> lock(g_pin_mu);
    size_t best = g_pinned.size();
    for (size_t i = 0; i < g_pinned.size(); ++i)
      if (g_pinned[i].n >= n && (best == g_pinned.size() || g_pinned[i].n < g_pinned[best].n))
        best = i;
    if (best < g_pinned.size()) {
      *out = g_pinned[best].p;
      g_pinned.erase(g_pinned.begin() + (std::ptrdiff_t)best);
      return hipSuccess;
    }
  }
  // round up so that buffers are reusable across nearby sizes
  size_t cap = 4096;
  while (cap < n) cap *= 2;
  return hipHostMalloc(out, cap, 0);
}

void pinned_release(void* p, size_t n) {
  if (!p) return;
  size_t cap = 4096;
  while (cap < n) cap *= 2;
  std::lock_guard<std::mutex> lock(g_pin_mu);
  g_pinned.push_back(Pinned{p, cap});
}

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
              size_t lds_cap, Launch* L, size_t* lds_out, Tile* common, bool wide = false) {
  std::memset(L, 0, sizeof(*L));
  for (int i = 0; i < n; ++i) {
    const bf_plan_s* p = plans[i];
    if (!x[i] || !out[i] || !aligned16(x[i]) || !aligned16(out[i])) return BF_ERR_INVALID_ARG;
    if (!p->weights_set) return BF_ERR_STATE;
    // the batching kernels stage weights in LDS
    if (lds_bytes(p->prec, p->Kpad, 1) > lds_cap) return BF_ERR_UNSUPPORTED;
  }
  // no set's output may overlap any set's voltages or another set's output
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (bf::ranges_overlap(out[i], bf::output_bytes(*plans[i]), x[j],
                             bf::input_bytes(*plans[j])))
        return BF_ERR_INVALID_ARG;
      if (j > i && bf::ranges_overlap(out[i], bf::output_bytes(*plans[i]), out[j],
                                      bf::output_bytes(*plans[j])))
        return BF_ERR_INVALID_ARG;
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
      for (int i = 0; i < n && ok; ++i) ok = tile_ok(*plans[i], c);
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
    if (wide) {
      // the widest eight-wave beam range whose weights fit the launch's LDS
      // and that the set's beams fill beyond one narrower range
      const std::vector<Tile> kWide = bf::wide_tiles();
      for (int v = 0; v < (int)kWide.size() && variant < 0; ++v) {
        const Tile& c = kWide[v];
        const bool last = v + 1 == (int)kWide.size();
        if (tile_ok(tmp, c) && lds_bytes(tmp.prec, tmp.Kpad, c.nbt) <= lds_cap &&
            (last || tmp.Bpad / 16 > c.nbt / 2))
          variant = v;
      }
      if (variant < 0) return BF_ERR_UNSUPPORTED;
      t = kWide[variant];
    } else if (multi) {
      const std::vector<Tile> kMultiTiles = bf::multi_tiles();
      const int nm = (int)kMultiTiles.size();
      auto fits = [&](const Tile& c) {
        return tile_ok(tmp, c) && lds_bytes(tmp.prec, tmp.Kpad, c.nbt) <= lds_cap;
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
    if (wide && !same) {
      // the set's own store-group count per wave was chosen for a four-wave
      // tile; an eight-wave unit instead takes as much of the channel's time
      // range as spreads over its eight waves (at least one MT-aligned step
      // each): no wave of a unit idles on a short block, and a long block is
      // split into as few units as that allows, each staging its weights
      // once.  Measured on the 12-set batch against the set's own count
      // capped the same way: 19.05-19.10 -> 18.76-18.80 ms.
      tmp.sgw = std::max(base, SG / bf::kWideWaves / base * base);
    }
    L->prob[i] = make_prob(&tmp, x[i], out[i], begin);
    L->prob[i].variant = variant;
    begin += units_for(tmp, t, tmp.sgw);
    lds = std::max(lds, lds_bytes(tmp.prec, tmp.Kpad, t.nbt));
  }
  if (lds > lds_cap) return BF_ERR_UNSUPPORTED;
  L->nprob = n;
  L->total_units = begin;
  L->xcd_remap = 0;
  // sets that beamform one voltage block (serving: every request reads the
  // block of the ring slot): units go out channel by channel over all sets,
  // so the sets' beam ranges of one channel meet its voltages in L2
  bool shared = n > 1;
  for (int i = 1; i < n && shared; ++i)
    shared = x[i] == x[0] && plans[i]->C == plans[0]->C && plans[i]->T == plans[0]->T &&
             plans[i]->N == plans[0]->N && plans[i]->in4 == plans[0]->in4;
  int64_t per_chan = 0;
  for (int i = 0; i < n; ++i) per_chan += (int64_t)L->prob[i].ntr * L->prob[i].nbr;
  L->chan_units = shared && per_chan < ((int64_t)1 << 30) ? (int32_t)per_chan : 0;
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
hipError_t mark_used(bf_plan_s* p, hipStream_t s) { return hipEventRecord(p->used_cur, s); }

// Records ev on s, except while s is being captured into a graph (a replay
// of the graph is then tracked by the caller, not by the event).
hipError_t record_unless_capturing(hipEvent_t ev, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e != hipSuccess) return e;
  return cs == hipStreamCaptureStatusNone ? hipEventRecord(ev, s) : hipSuccess;
}

// ---- tile cache (written by the autotuner, read here) ----
std::mutex g_tune_mu;
std::vector<bf::TuneEntry> g_tune;
bool g_tune_env_tried = false;

int load_tune_file(const char* path, std::vector<bf::TuneEntry>* out) {
  std::FILE* f = std::fopen(path, "rb");
  if (!f) return BF_ERR_INVALID_ARG;
  std::string text;
  char buf[65536];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) {
    text.append(buf, n);
    if (text.size() > ((size_t)64 << 20)) {  // not a tile cache
      std::fclose(f);
      return BF_ERR_INVALID_ARG;
    }
  }
  std::fclose(f);
  const int k = bf::parse_tune_cache(text.data(), text.size(), out);
  return k < 0 ? BF_ERR_INVALID_ARG : k;
}

// Applies the cache entry for the plan's shape (single-run or batching
// kernel), if one exists and its tile can run the plan.  Returns whether a
// tile was applied.
bool apply_tuned(bf_plan_s* p, bool batch) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (!g_tune_env_tried) {
    g_tune_env_tried = true;
    const char* env = std::getenv("BF_TUNE_CACHE");
    if (env && *env && g_tune.empty()) (void)load_tune_file(env, &g_tune);
  }
  const std::string key = bf::tune_key(*p, batch);
  for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it) {
    if (it->key != key) continue;
    if (bf::check_tile(*p, it->tile, it->sgw) != BF_OK) return false;
    p->tile = it->tile;
    p->sgw = it->sgw;
    p->tuned = true;
    return true;
  }
  return false;
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

int bf_tune_load(const char* path) {
  try {
    if (!path) return BF_ERR_INVALID_ARG;
    std::vector<bf::TuneEntry> got;
    const int k = load_tune_file(path, &got);
    if (k < 0) return k;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_env_tried = true;  // an explicit load replaces the environment's
    g_tune.swap(got);
    return k;
  } catch (...) {
    return BF_ERR_OOM;
  }
}

int bf_tune_key(bf_plan_t p, int32_t batch, char* buf, int32_t len) {
  try {
    if (!p || !buf || len < 1) return BF_ERR_INVALID_ARG;
    const std::string k = bf::tune_key(*p, batch != 0);
    if ((size_t)len < k.size() + 1) return BF_ERR_INVALID_ARG;
    std::memcpy(buf, k.c_str(), k.size() + 1);
    return (int)k.size();
  } catch (...) {
    return BF_ERR_OOM;
  }
}

int bf_plan_apply_tuned(bf_plan_t p, int32_t batch) {
  try {
    if (!p) return BF_ERR_INVALID_ARG;
    return apply_tuned(p, batch != 0) ? 1 : 0;
  } catch (...) {
    return BF_ERR_OOM;
  }
}

const char* bf_last_hip_error(void) { return g_last_error; }

int bf_plan_create_ex(bf_plan_t* out, int32_t N, int32_t C, int32_t B, int64_t T, int32_t I,
                      bf_precision_t precision, uint32_t flags) {
  try {
    if (!out) return BF_ERR_INVALID_ARG;
    *out = nullptr;
    bf::Shape sh;
    const int st = bf::make_shape(N, C, B, T, I, (int)precision, flags, 256, &sh);
    if (st != BF_OK) return st;
    bf_plan_s* p = new (std::nothrow) bf_plan_s();
    if (!p) return BF_ERR_OOM;
    static_cast<bf::Shape&>(*p) = sh;
    if (hipGetDevice(&p->device) != hipSuccess) {
      delete p;
      return BF_ERR_HIP;
    }
    (void)hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
    if (p->n_cu < 1) p->n_cu = 256;
    choose_tile(*p, &p->tile, &p->sgw);
    apply_tuned(p, false);
    p->w_bytes = (size_t)C * p->Bpad * 2 * p->Kpad * es_of(p->prec);
    hipError_t e = dev_alloc(p->device, &p->w_dev, p->w_bytes);
    if (e != hipSuccess) {
      delete p;
      return from_hip(e);
    }
    // no clearing: both weight kernels write every element of the buffer
    // (padding included), and nothing reads it before one of them has run
    p->geo_count = (size_t)3 * N + (size_t)3 * B + (size_t)C + (size_t)N;
    p->mask.assign(N, 1.0);
    e = pinned_acquire(p->geo_count * sizeof(double), (void**)&p->geo_host);
    if (e == hipSuccess) e = dev_alloc(p->device, (void**)&p->geo_dev, p->geo_count * sizeof(double));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->geo_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->used_cur, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->used_alt, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->w_ready, hipEventDisableTiming);
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
    // device buffers: released on the device after the plan's own work
    // (weight generation, refreshes, the runs that read either buffer)
    (void)dev_release(p->device, {p->geo_done, p->w_ready, p->used_cur, p->used_alt},
                      {p->w_dev, p->w_alt, p->geo_dev});
    // the pinned staging area is reused by later plans once the copy that
    // read it (ordered before geo_done) is done
    if (p->geo_host) {
      if (p->geo_done) (void)hipEventSynchronize(p->geo_done);
      pinned_release(p->geo_host, p->geo_count * sizeof(double));
    }
    for (hipEvent_t ev : {p->geo_done, p->w_ready, p->used_cur, p->used_alt})
      if (ev) (void)hipEventDestroy(ev);
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
      hipError_t e = dev_alloc(p->device, &alt, p->w_bytes);
      if (e != hipSuccess) return from_hip(e);  // the plan is left as it was
      p->w_alt = alt;
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

// Arguments of the beam-pattern entry points.
static int pattern_args(const bf_plan_s* p, const double* pos, const double* freq,
                 const double* grid_dir, int32_t n_dirs, const float* p_dev) {
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
  return BF_OK;
}

int bf_beam_pattern(bf_plan_t p, const double* pos, const double* freq, const double* grid_dir,
                    int32_t n_dirs, float* p_dev, void* stream) {
  try {
    const int st = pattern_args(p, pos, freq, grid_dir, n_dirs, p_dev);
    if (st != BF_OK) return st;
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

int bf_beam_pattern_noalloc(bf_plan_t p, const double* pos, const double* freq,
                            const double* grid_dir, int32_t n_dirs, float* p_dev, void* stream) {
  try {
    const int st = pattern_args(p, pos, freq, grid_dir, n_dirs, p_dev);
    if (st != BF_OK) return st;
    const size_t nd = (size_t)3 * p->N + (size_t)p->C + (size_t)3 * n_dirs;
    if (nd > bf::kPatScratchDoubles) return BF_ERR_INVALID_ARG;
    // the staging array's address on the plan's device, looked up with that
    // device current
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return from_hip(e);
    if (cur != p->device) e = hipSetDevice(p->device);
    double* d = nullptr;
    if (e == hipSuccess) e = bf::pattern_scratch(p->device, &d);
    if (cur != p->device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return from_hip(e);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    e = take_refresh(p, s);
    // stream-ordered copies: a previous call's map on this stream has read
    // the array before it is overwritten (calls on other streams race)
    if (e == hipSuccess)
      e = hipMemcpyAsync(d, pos, sizeof(double) * 3 * p->N, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d + 3 * p->N, freq, sizeof(double) * p->C, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d + 3 * p->N + p->C, grid_dir, sizeof(double) * 3 * (size_t)n_dirs,
                         hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = bf::launch_beam_pattern(p->prec, p->w_dev, d, d + 3 * p->N + p->C, d + 3 * p->N,
                                  p->N, p->C, p->B, p->Bpad, p->Kpad, n_dirs, p_dev, s);
    if (e == hipSuccess) e = mark_used(p, s);
    return from_hip(e);
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
    if (bf::ranges_overlap(x, bf::input_bytes(*p), out, bf::output_bytes(*p)))
      return BF_ERR_INVALID_ARG;
    if (!p->weights_set && !p->refresh_pending) return BF_ERR_STATE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = take_refresh(p, s);
    if (e != hipSuccess) return from_hip(e);
    Launch L;
    std::memset(&L, 0, sizeof(L));
    L.prob[0] = make_prob(p, x, out, 0);
    L.nprob = 1;
    L.total_units = units_for(*p, p->tile, p->sgw);
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
  info->work_units = units_for(*p, p->tile, p->sgw);
  info->weight_bytes = (int64_t)p->w_bytes;
  info->lds_bytes = (int64_t)tile_lds(p->prec, p->Kpad, p->tile);
  info->flops = 8.0 * p->C * (double)p->B * (double)p->T * p->N;
  info->tile_tuned = p->tuned ? 1 : 0;
  return BF_OK;
}

int bf_plan_set_tile(bf_plan_t p, int32_t mt, int32_t nbt, int32_t nbp, int32_t kres,
                     int32_t sgw) {
  if (!p) return BF_ERR_INVALID_ARG;
  const Tile t{mt, nbt, nbp, kres};
  const int st = bf::check_tile(*p, t, sgw);
  if (st != BF_OK) return st;
  p->tile = t;
  p->sgw = sgw;
  p->tuned = false;
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
    if (!tile_ok(*p, t)) return;
    if (n < max_tiles) {
      tiles[4 * n + 0] = t.mt;
      tiles[4 * n + 1] = t.nbt;
      tiles[4 * n + 2] = t.nbp;
      tiles[4 * n + 3] = t.kres;
    }
    ++n;
  };
  for (const Tile& t : bf::compiled_tiles(*p)) add(t);
  return n;
}

int bf_batch_tile_candidates(bf_plan_t p, int32_t* tiles, int32_t max_tiles) {
  if (!p || max_tiles < 0 || (max_tiles > 0 && !tiles)) return BF_ERR_INVALID_ARG;
  int32_t n = 0;
  if (!p->vec16 || p->cx) return 0;
  for (const Tile& t : bf::multi_tiles()) {
    if (!tile_ok(*p, t)) continue;
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
    // queue counters of the two persistent launches (four- and eight-wave)
    hipError_t e = dev_alloc(bt->device, (void**)&bt->queue, 2 * bf::kQueueInts * sizeof(int32_t));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->last_use, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)dev_release(bt->device, {}, {bt->queue});
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
    // validates every set (pointers, state, no output overlapping any input
    // or another output) and fills the four-wave table of all of them
    int st = fill_sets(bt->plans.data(), n, x, out, kLdsMax, &L, &lds, &common);
    if (st != BF_OK) return st;
    L.queue = bt->queue;
    const bf_plan_s* p0 = bt->plans[0];
    const bool multi = p0->vec16;
    hipError_t e = hipSuccess;
    // Sets whose K needs more than two 64-wide chunks run the eight-wave
    // streamed form in a persistent launch of their own (FP16/BF16, I == 1
    // or I % 4 == 0); the others share the four-wave persistent launch.
    if (multi && p0->prec != BF_FP32 && (p0->mode == bf::kModeI1 || p0->mode == bf::kModeGen4)) {
      std::vector<bf_plan_t> wp, rp;
      std::vector<const int8_t*> wx, rx;
      std::vector<float*> wo, ro;
      for (int i = 0; i < n; ++i) {
        bf_plan_s* p = bt->plans[i];
        const bool wide = p->Kpad > 2 * bf::kChunk && tile_ok(*p, bf::wide_tiles().back()) &&
                          lds_bytes(p->prec, p->Kpad, bf::wide_tiles().back().nbt) <= kLdsMax;
        (wide ? wp : rp).push_back(p);
        (wide ? wx : rx).push_back(x[i]);
        (wide ? wo : ro).push_back(out[i]);
      }
      if (!wp.empty()) {
        Launch LW;
        size_t ldw = 0;
        st = fill_sets(wp.data(), (int)wp.size(), wx.data(), wo.data(), kLdsMax, &LW, &ldw, &common,
                       true);
        if (st != BF_OK) return st;
        LW.queue = bt->queue + bf::kQueueInts;  // counters of its own
        int occ = 0;
        e = bf::launch_beamform_multi(p0->prec, p0->mode, p0->in4, LW, nullptr, 0, ldw, s, &occ,
                                      true);
        if (e != hipSuccess) return from_hip(e);
        int64_t gw = std::min<int64_t>(LW.total_units, (int64_t)p0->n_cu * std::max(1, occ));
        e = bf::launch_queue_reset(LW.queue, s);
        if (e == hipSuccess)
          e = bf::launch_beamform_multi(p0->prec, p0->mode, p0->in4, LW, nullptr,
                                        (int)std::max<int64_t>(1, gw), ldw, s, nullptr, true);
        if (e != hipSuccess) return from_hip(e);
        if (!rp.empty()) {
          st = fill_sets(rp.data(), (int)rp.size(), rx.data(), ro.data(), kLdsMax, &L, &lds,
                         &common);
          if (st != BF_OK) return st;
          L.queue = bt->queue;
        } else {
          L.total_units = 0;
        }
      }
    }
    int per_cu = lds <= 80 * 1024 ? 2 : 1;
    if (multi) {
      int occ = 0;
      e = bf::launch_beamform_multi(p0->prec, p0->mode, p0->in4, L, nullptr, 0, lds, s, &occ);
      if (e != hipSuccess) return from_hip(e);
      per_cu = std::max(1, occ);
    }
    int64_t grid = std::min<int64_t>(L.total_units, (int64_t)p0->n_cu * per_cu);
    if (grid < 1) grid = 1;
    if (L.total_units > 0) {
      e = bf::launch_queue_reset(bt->queue, s);
      if (e == hipSuccess) {
        e = multi ? bf::launch_beamform_multi(p0->prec, p0->mode, p0->in4, L, nullptr, (int)grid,
                                              lds, s, nullptr)
                  : bf::launch_beamform(p0->prec, p0->mode, p0->vec16, p0->in4, common, L,
                                        (int)grid, lds, s);
      }
    }
    for (int i = 0; i < n && e == hipSuccess; ++i) e = mark_used(bt->plans[i], s);
    if (e == hipSuccess) e = hipEventRecord(bt->last_use, s);
    return from_hip(e);
  } catch (...) {
    return BF_ERR_HIP;
  }
}

int bf_batch_destroy(bf_batch_t bt) {
  if (!bt) return BF_OK;
  // the queue counters are released on the device after the batch's own
  // last launch
  (void)dev_release(bt->device, {bt->last_use}, {bt->queue});
  if (bt->last_use) (void)hipEventDestroy(bt->last_use);
  delete bt;
  return BF_OK;
}

int bf_table_create(bf_table_t* out, int32_t n_antennas, int32_t integration, int32_t precision,
                    uint32_t flags) {
  try {
    if (!out) return BF_ERR_INVALID_ARG;
    *out = nullptr;
    if (n_antennas < 1 || n_antennas > bf::kMaxN || integration < 1) return BF_ERR_INVALID_ARG;
    if (precision != BF_FP32 && precision != BF_FP16 && precision != BF_BF16)
      return BF_ERR_INVALID_ARG;
    if (flags & ~BF_INPUT_4BIT) return BF_ERR_INVALID_ARG;
    if ((2 * n_antennas) % 16 != 0) return BF_ERR_UNSUPPORTED;
    bf_table_s* t = new bf_table_s();
    t->N = n_antennas;
    t->I = integration;
    t->prec = precision;
    t->in4 = (flags & BF_INPUT_4BIT) != 0;
    t->mode = bf::mode_of(integration);
    t->Kpad = 64 * ((2 * n_antennas + 63) / 64);
    // Arrays whose K needs more than two 64-wide chunks (where the four-wave
    // kernel streams K) run every set in the eight-wave streamed form, FP16
    // and BF16 with I == 1 or I % 4 == 0; its LDS holds the widest beam
    // range that fits.  Otherwise one LDS size for every launch: the largest
    // four-wave batching variant that still leaves two workgroups per CU (at
    // least the smallest variant).
    t->wide = precision != BF_FP32 && (t->mode == bf::kModeI1 || t->mode == bf::kModeGen4) &&
              t->Kpad > 2 * bf::kChunk;
    if (t->wide) {
      t->lds = 0;
      for (const Tile& c : bf::wide_tiles()) {
        const size_t l = lds_bytes(precision, t->Kpad, c.nbt);
        if (l <= kLdsMax) t->lds = std::max(t->lds, l);
      }
      if (t->lds == 0) t->wide = false;
    }
    if (!t->wide) {
      t->lds = lds_bytes(precision, t->Kpad, 1);
      for (const Tile& c : bf::multi_tiles()) {
        const size_t l = lds_bytes(precision, t->Kpad, c.nbt);
        if (l <= 80 * 1024) t->lds = std::max(t->lds, l);
      }
    }
    if (t->lds > kLdsMax) {
      delete t;
      return BF_ERR_UNSUPPORTED;
    }
    hipError_t e = hipGetDevice(&t->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&t->n_cu, hipDeviceAttributeMultiprocessorCount,
                                                   t->device);
    if (e == hipSuccess)
      e = dev_alloc(t->device, (void**)&t->queue, bf::kQueueInts * sizeof(int32_t));
    if (e == hipSuccess) e = dev_alloc(t->device, (void**)&t->table, sizeof(Launch));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&t->last_use, hipEventDisableTiming);
    int occ = 0;
    if (e == hipSuccess) {
      Launch L;
      std::memset(&L, 0, sizeof(L));
      e = bf::launch_beamform_multi(precision, t->mode, t->in4, L, t->table, 0, t->lds, nullptr,
                                    &occ, t->wide);
    }
    if (e != hipSuccess) {
      if (t->last_use) (void)hipEventDestroy(t->last_use);
      (void)dev_release(t->device, {}, {t->queue, t->table});
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
      const int st = fill_sets(plans, n, x, out, t->lds, &L, &lds, &common, t->wide);
      if (st != BF_OK) return st;
    }
    L.queue = t->queue;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = bf::launch_table_store(L, t->table, s);
    if (e == hipSuccess) e = record_unless_capturing(t->last_use, s);
    return from_hip(e);
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
                                  nullptr, t->wide);
  if (e == hipSuccess) e = record_unless_capturing(t->last_use, s);
  return from_hip(e);
}

int bf_table_destroy(bf_table_t t) {
  if (!t) return BF_OK;
  // released on the device after the table's own last store and uncaptured
  // run (launches replayed from a captured graph are the caller's to wait
  // for)
  (void)dev_release(t->device, {t->last_use}, {t->queue, t->table});
  if (t->last_use) (void)hipEventDestroy(t->last_use);
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
                           hipStream_t s, int* occupancy, bool wide);
#define BF_EXTERN(P, F)                                                                     \
  extern template hipError_t launch_prec_in<P, F>(int, bool, Tile, const Launch&, int, size_t, \
                                                  hipStream_t);                              \
  extern template hipError_t launch_multi_in<P, F>(int, const Launch&, const Launch*, int,    \
                                                   size_t, hipStream_t, int*, bool);
BF_EXTERN(0, false)
BF_EXTERN(1, false)
BF_EXTERN(2, false)
BF_EXTERN(0, true)
BF_EXTERN(1, true)
BF_EXTERN(2, true)
#undef BF_EXTERN

hipError_t launch_beamform_multi(int prec, int mode, bool in4, const Launch& L,
                                 const Launch* table, int grid, size_t lds, hipStream_t s,
                                 int* occ, bool wide) {
  if (in4) {
    if (prec == 0) return launch_multi_in<0, true>(mode, L, table, grid, lds, s, occ, wide);
    if (prec == 1) return launch_multi_in<1, true>(mode, L, table, grid, lds, s, occ, wide);
    return launch_multi_in<2, true>(mode, L, table, grid, lds, s, occ, wide);
  }
  if (prec == 0) return launch_multi_in<0, false>(mode, L, table, grid, lds, s, occ, wide);
  if (prec == 1) return launch_multi_in<1, false>(mode, L, table, grid, lds, s, occ, wide);
  return launch_multi_in<2, false>(mode, L, table, grid, lds, s, occ, wide);
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
