// bf_host.cpp -- host-side logic with no HIP dependency (see bf_host.h).
#include "bf_host.h"

#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace bf {

namespace {

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
const Tile kWideTiles[] = {
#define BF_TILE(MT, NBT, NBP, KRES) Tile{MT, NBT, NBP, KRES},
    BF_TILE_LIST_WIDE
#undef BF_TILE
};
const Tile kCxTiles[] = {
#define BF_TILE(MT, NBT, NBP, KRES) Tile{MT, NBT, NBP, KRES},
    BF_TILE_LIST_CX
#undef BF_TILE
};

template <size_t K>
std::vector<Tile> as_vector(const Tile (&a)[K]) {
  return std::vector<Tile>(a, a + K);
}

int gcd(int a, int b) { return b ? gcd(b, a % b) : a; }

int64_t floor_pow2(int64_t v) {
  int64_t r = 1;
  while (r <= v / 2) r *= 2;
  return r;
}

}  // namespace

int make_shape(int32_t N, int32_t C, int32_t B, int64_t T, int32_t I, int prec, uint32_t flags,
               int n_cu, Shape* out) {
  if (!out) return BF_ERR_INVALID_ARG;
  if (N < 1 || N > kMaxN || C < 1 || C > kMaxC || B < 1 || B > kMaxB || T < 1 || I < 1 ||
      T > kMaxT || T % I != 0)
    return BF_ERR_INVALID_ARG;
  if (prec != BF_FP32 && prec != BF_FP16 && prec != BF_BF16) return BF_ERR_INVALID_ARG;
  if (flags & ~(uint32_t)(BF_ACCUMULATE | BF_INPUT_4BIT | BF_OUTPUT_COMPLEX))
    return BF_ERR_INVALID_ARG;
  // complex beams are per sample and overwrite their output
  if ((flags & BF_OUTPUT_COMPLEX) && (I != 1 || (flags & BF_ACCUMULATE))) return BF_ERR_INVALID_ARG;
  // 4-bit rows are read 8 bytes (8 antennas) at a time
  if ((flags & BF_INPUT_4BIT) && N % 8 != 0) return BF_ERR_UNSUPPORTED;
  Shape s;
  s.N = N;
  s.C = C;
  s.B = B;
  s.T = T;
  s.I = I;
  s.prec = prec;
  s.flags = flags;
  s.in4 = (flags & BF_INPUT_4BIT) != 0;
  s.cx = (flags & BF_OUTPUT_COMPLEX) != 0;
  s.vec16 = (2 * N) % 16 == 0;
  s.Bpad = (B + 15) / 16 * 16;
  s.Kpad = (2 * N + kChunk - 1) / kChunk * kChunk;
  s.mode = s.cx ? kModeCx : mode_of(I);
  s.n_cu = n_cu > 0 ? n_cu : 256;
  *out = s;
  return BF_OK;
}

int es_of(int prec) { return prec == BF_FP32 ? 4 : 2; }

int mode_of(int32_t I) {
  return I == 1 ? kModeI1 : I == 2 ? kModeI2 : (I % 4 == 0 ? kModeGen4 : kModeGen);
}

size_t lds_bytes(int prec, int32_t Kpad, int nbt) {
  return (size_t)2 * 16 * (size_t)nbt * ((size_t)Kpad * (size_t)es_of(prec) + kLdsPad);
}

size_t tile_lds(int prec, int32_t Kpad, Tile t) {
  return t.kres == -1 ? 0 : lds_bytes(prec, Kpad, t.nbt);
}

void schedule(int32_t I, int64_t T, int32_t* G, int32_t* QI, int32_t* SG) {
  const int64_t W = T / I;
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

bool same_tile(const Tile& a, const Tile& b) {
  return a.mt == b.mt && a.nbt == b.nbt && a.nbp == b.nbp && a.kres == b.kres;
}

// The eight-wave form's conditions: FP16/BF16 power output, 16-byte rows,
// I == 1 or I % 4 == 0 (I % MT == 0 is checked per tile), overwriting
// output, whole 16-byte window quads (T / I % 4 == 0), and byte offsets
// within one channel's voltages (rows up to the last store group's padding,
// plus the out-of-range marker 2^31 added to them) and one channel's output
// rows that fit the 32-bit buffer offsets it uses.
static bool wide_shape(const Shape& s) {
  if (s.prec == BF_FP32 || s.cx || !s.vec16 || (s.flags & BF_ACCUMULATE)) return false;
  if (s.mode != kModeI1 && s.mode != kModeGen4) return false;
  const int64_t W = s.T / s.I;
  if (W % 4 != 0) return false;
  const int64_t rowb = s.in4 ? s.N : 2 * (int64_t)s.N;
  return (s.T + 16 * (int64_t)s.I) * rowb < 0x7FFFFFFF && (int64_t)s.B * W * 4 < 0x7FFFFFFF;
}

std::vector<Tile> compiled_tiles(const Shape& s) {
  std::vector<Tile> v;
  if (s.cx && s.vec16)
    v = as_vector(kCxTiles);
  else if (s.in4)
    v = as_vector(kIn4Tiles);
  else if (s.vec16)
    v = as_vector(kVecTiles);
  else
    v = as_vector(kGenTiles);
  if (wide_shape(s))
    for (const Tile& t : kWideTiles) v.push_back(t);
  return v;
}

std::vector<Tile> multi_tiles() { return as_vector(kMultiTiles); }

std::vector<Tile> wide_tiles() { return as_vector(kWideTiles); }

bool tile_exists(const Shape& s, Tile t) {
  for (const Tile& x : compiled_tiles(s))
    if (same_tile(x, t)) return true;
  return false;
}

bool tile_ok(const Shape& s, Tile t) {
  if (!tile_exists(s, t)) return false;
  if (t.kres > 0 && s.Kpad / kChunk > t.kres) return false;
  if (t.kres == kKresWide && s.mode == kModeGen4 && s.I % t.mt != 0) return false;
  return tile_lds(s.prec, s.Kpad, t) <= kLdsMax;
}

int64_t units_for(const Shape& s, Tile t, int32_t sgw) {
  int32_t G, QI, SG;
  schedule(s.I, s.T, &G, &QI, &SG);
  const int64_t nbr = (s.Bpad / 16 + t.nbt - 1) / t.nbt;
  const int64_t per = (int64_t)waves_of(t) * sgw;
  const int64_t ntr = (SG + per - 1) / per;
  return (int64_t)s.C * nbr * ntr;
}

// Default tile: the largest beam range whose weight slice fits 80 KB of LDS
// (two workgroups per CU) without exceeding the plan's beams; voltages held
// in registers when K <= 128 (MT = 8 for FP16/BF16 at K <= 64, where the
// per-pass fragment reuse matters most); streamed K otherwise.  Then
// enough store groups per wave that a launch has >= 8 workgroups per CU,
// capped at 256 row tiles per wave per unit.
void choose_tile(const Shape& s, Tile* out, int32_t* out_sgw) {
  const int need = s.Bpad / 16;
  const int nch = s.Kpad / kChunk;
  int nbt = 8;
  while (nbt > 1 && (lds_bytes(s.prec, s.Kpad, nbt) > 80 * 1024 || nbt / 2 >= need)) nbt /= 2;
  Tile t{4, 1, 1, 0};
  if (lds_bytes(s.prec, s.Kpad, 1) > kLdsMax) {
    t = Tile{4, 2, 2, -1};  // one beam tile's weights do not fit LDS
  } else if (!s.vec16) {
    t = nbt == 8 ? Tile{4, 8, 2, 0} : Tile{4, 1, 1, 0};
  } else if (nch == 1 && nbt >= 4) {
    t = (s.prec == BF_FP32 || s.in4 || s.cx) ? Tile{4, nbt, 1, 1} : Tile{8, nbt, 1, 1};
  } else if (nch == 2 && nbt >= 4) {
    t = Tile{4, nbt, 1, 2};
  } else {
    t = nbt >= 4 ? Tile{4, nbt, 2, 0} : nbt == 2 ? Tile{4, 2, 2, 0} : Tile{4, 1, 1, 0};
  }
  // the 4-bit and complex-output variants carry fewer forms: fall back to
  // the streamed form of the same beam range
  if (!tile_ok(s, t) && nbt >= 2) t = Tile{4, nbt, 2, 0};
  if (!tile_ok(s, t) && nbt >= 2) t = Tile{4, 2, 2, 0};
  if (!tile_ok(s, t)) t = Tile{4, 1, 1, 0};
  if (!tile_ok(s, t)) t = Tile{4, 2, 2, -1};
  int32_t G, QI, SG;
  schedule(s.I, s.T, &G, &QI, &SG);
  const int32_t base = t.mt / gcd(t.mt, G);  // sgw * G must be a multiple of MT
  int32_t sgw = base;
  const int64_t want = (int64_t)s.n_cu * 8;
  for (int32_t k = 2;; ++k) {
    const int32_t v = base * k;
    if ((int64_t)v * G > 256 || units_for(s, t, v) < want) break;
    if ((int64_t)(v - base) * waves_of(t) >= SG) break;
    sgw = v;
  }
  *out = t;
  *out_sgw = sgw;
}

int check_tile(const Shape& s, Tile t, int32_t sgw) {
  if (sgw < 1) return BF_ERR_INVALID_ARG;
  if (!tile_ok(s, t)) return BF_ERR_UNSUPPORTED;
  int32_t G, QI, SG;
  schedule(s.I, s.T, &G, &QI, &SG);
  if (((int64_t)sgw * G) % t.mt != 0) return BF_ERR_INVALID_ARG;
  return BF_OK;
}

uint64_t input_bytes(const Shape& s) {
  const uint64_t row = s.in4 ? (uint64_t)s.N : 2 * (uint64_t)s.N;
  return (uint64_t)s.C * (uint64_t)s.T * row;
}

uint64_t output_bytes(const Shape& s) {
  const uint64_t per_beam = s.cx ? (uint64_t)s.T * 4 : (uint64_t)(s.T / s.I) * 4;
  return (uint64_t)s.C * (uint64_t)s.B * per_beam;
}

bool ranges_overlap(const void* a, uint64_t na, const void* b, uint64_t nb) {
  if (na == 0 || nb == 0) return false;
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  // [x, x + na) and [y, y + nb) intersect iff each starts before the other ends
  return x < y ? (y - x) < na : (x - y) < nb;
}

std::string tune_key(const Shape& s, bool batch, const char* arch) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s/p%d/N%d/B~%lld/I%d/C~%lld/T~%lld%s%s%s", arch ? arch : "",
                s.prec, s.N, (long long)floor_pow2(s.B), s.I, (long long)floor_pow2(s.C),
                (long long)floor_pow2(s.T), s.in4 ? "/in4" : "", s.cx ? "/cx" : "",
                batch ? "/batch" : "");
  return std::string(buf);
}

// ---- a minimal JSON reader for the tile cache ----
namespace {

class Reader {
 public:
  Reader(const char* p, size_t n) : p_(p), e_(p + n) {}

  // The whole text: one object whose members are cache entries.
  bool top(std::vector<TuneEntry>* out) {
    if (!lit('{')) return false;
    if (lit('}')) return end();
    for (;;) {
      std::string key;
      if (!str(&key) || !lit(':')) return false;
      TuneEntry e;
      bool good = false;
      if (peek() == '{') {
        if (!entry(&e, &good)) return false;
      } else if (!skip()) {
        return false;
      }
      if (good) {
        e.key = key;
        out->push_back(e);
      }
      if (lit(',')) continue;
      if (lit('}')) return end();
      return false;
    }
  }

 private:
  const char* p_;
  const char* e_;
  int depth_ = 0;

  void ws() {
    while (p_ < e_ && (*p_ == ' ' || *p_ == '\n' || *p_ == '\r' || *p_ == '\t')) ++p_;
  }
  char peek() {
    ws();
    return p_ < e_ ? *p_ : '\0';
  }
  bool lit(char c) {
    ws();
    if (p_ < e_ && *p_ == c) {
      ++p_;
      return true;
    }
    return false;
  }
  bool end() {
    ws();
    return p_ == e_;
  }
  bool word(const char* w) {
    const size_t n = std::strlen(w);
    if ((size_t)(e_ - p_) >= n && std::memcmp(p_, w, n) == 0) {
      p_ += n;
      return true;
    }
    return false;
  }
  bool str(std::string* out) {
    if (!lit('"')) return false;
    while (p_ < e_ && *p_ != '"') {
      char c = *p_++;
      if ((unsigned char)c < 0x20) return false;
      if (c == '\\') {
        if (p_ >= e_) return false;
        const char d = *p_++;
        switch (d) {
          case '"': case '\\': case '/': c = d; break;
          case 'b': c = '\b'; break;
          case 'f': c = '\f'; break;
          case 'n': c = '\n'; break;
          case 'r': c = '\r'; break;
          case 't': c = '\t'; break;
          case 'u':
            if (e_ - p_ < 4) return false;
            for (int i = 0; i < 4; ++i)
              if (!std::isxdigit((unsigned char)p_[i])) return false;
            p_ += 4;
            c = '?';  // keys of the cache are ASCII; anything else never matches
            break;
          default: return false;
        }
      }
      if (out) out->push_back(c);
    }
    if (p_ >= e_) return false;
    ++p_;
    return true;
  }
  bool num(double* v) {
    ws();
    const char* s = p_;
    while (p_ < e_ && (std::isdigit((unsigned char)*p_) || *p_ == '-' || *p_ == '+' ||
                       *p_ == '.' || *p_ == 'e' || *p_ == 'E'))
      ++p_;
    if (p_ == s || p_ - s > 64) return false;
    char buf[72];
    std::memcpy(buf, s, (size_t)(p_ - s));
    buf[p_ - s] = '\0';
    char* endp = nullptr;
    const double x = std::strtod(buf, &endp);
    if (endp != buf + (p_ - s) || !std::isfinite(x)) return false;
    if (v) *v = x;
    return true;
  }
  bool array(std::vector<double>* nums, bool* all_num) {
    if (!lit('[')) return false;
    if (lit(']')) return true;
    for (;;) {
      const char c = peek();
      if (c == '-' || (c >= '0' && c <= '9')) {
        double x;
        if (!num(&x)) return false;
        if (nums) nums->push_back(x);
      } else {
        if (all_num) *all_num = false;
        if (!skip()) return false;
      }
      if (lit(',')) continue;
      return lit(']');
    }
  }
  bool object_skip() {
    if (!lit('{')) return false;
    if (lit('}')) return true;
    for (;;) {
      if (!str(nullptr) || !lit(':') || !skip()) return false;
      if (lit(',')) continue;
      return lit('}');
    }
  }
  bool skip() {
    if (++depth_ > 64) return false;
    bool ok;
    const char c = peek();
    if (c == '{') ok = object_skip();
    else if (c == '[') ok = array(nullptr, nullptr);
    else if (c == '"') ok = str(nullptr);
    else if (c == 't') ok = word("true");
    else if (c == 'f') ok = word("false");
    else if (c == 'n') ok = word("null");
    else ok = num(nullptr);
    --depth_;
    return ok;
  }
  // {"tile": [mt, nbt, nbp, kres, sgw], ...}
  bool entry(TuneEntry* e, bool* good) {
    if (!lit('{')) return false;
    *good = false;
    if (lit('}')) return true;
    for (;;) {
      std::string k;
      if (!str(&k) || !lit(':')) return false;
      if (k == "tile" && peek() == '[') {
        std::vector<double> v;
        bool all_num = true;
        if (!array(&v, &all_num)) return false;
        bool ints = all_num && v.size() == 5;
        for (size_t i = 0; ints && i < v.size(); ++i)
          ints = v[i] == std::floor(v[i]) && v[i] >= -1024 && v[i] <= 1048576;
        if (ints) {
          e->tile = Tile{(int)v[0], (int)v[1], (int)v[2], (int)v[3]};
          e->sgw = (int32_t)v[4];
          *good = true;
        }
      } else if (!skip()) {
        return false;
      }
      if (lit(',')) continue;
      return lit('}');
    }
  }
};

}  // namespace

int parse_tune_cache(const char* text, size_t len, std::vector<TuneEntry>* out) {
  if (!text || !out) return -1;
  std::vector<TuneEntry> got;
  Reader r(text, len);
  if (!r.top(&got)) return -1;
  out->insert(out->end(), got.begin(), got.end());
  return (int)got.size();
}

}  // namespace bf
