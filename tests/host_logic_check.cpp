// Host-logic checks of the beamformer library, built for the CPU with
// address and undefined-behaviour sanitizers (tests/test_host_sanitized.py):
// plan validation, the work schedule and default tile of many shapes, byte
// range overlap, tile-cache keys, and the tile-cache reader on well-formed,
// truncated and corrupted text.  Prints "OK ..." and exits 0, or names the
// first failed check and exits 1.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "bf_host.h"

using bf::Shape;
using bf::Tile;

static int g_checks = 0;

#define CHECK(cond)                                                               \
  do {                                                                            \
    ++g_checks;                                                                   \
    if (!(cond)) {                                                                \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);                \
      return 1;                                                                   \
    }                                                                             \
  } while (0)

static int check_validation() {
  Shape s;
  CHECK(bf::make_shape(32, 1024, 128, 65536, 16, BF_FP32, 0, 256, &s) == BF_OK);
  CHECK(s.Bpad == 128 && s.Kpad == 64 && s.mode == bf::kModeGen4 && s.vec16);
  CHECK(bf::make_shape(0, 1, 1, 1, 1, BF_FP32, 0, 256, &s) == BF_ERR_INVALID_ARG);
  CHECK(bf::make_shape(4097, 1, 1, 1, 1, BF_FP32, 0, 256, &s) == BF_ERR_INVALID_ARG);
  CHECK(bf::make_shape(8, 1, 65537, 1, 1, BF_FP32, 0, 256, &s) == BF_ERR_INVALID_ARG);
  CHECK(bf::make_shape(8, (1 << 24) + 1, 1, 1, 1, BF_FP32, 0, 256, &s) == BF_ERR_INVALID_ARG);
  CHECK(bf::make_shape(8, 1, 1, 10, 3, BF_FP32, 0, 256, &s) == BF_ERR_INVALID_ARG);  // T % I
  CHECK(bf::make_shape(8, 1, 1, ((int64_t)1 << 40) + 16, 16, BF_FP32, 0, 256, &s) ==
        BF_ERR_INVALID_ARG);
  CHECK(bf::make_shape(8, 1, 1, 16, 1, 7, 0, 256, &s) == BF_ERR_INVALID_ARG);
  CHECK(bf::make_shape(8, 1, 1, 16, 1, BF_FP16, 8u, 256, &s) == BF_ERR_INVALID_ARG);
  CHECK(bf::make_shape(8, 1, 1, 16, 2, BF_FP16, BF_OUTPUT_COMPLEX, 256, &s) ==
        BF_ERR_INVALID_ARG);
  CHECK(bf::make_shape(8, 1, 1, 16, 1, BF_FP16, BF_OUTPUT_COMPLEX | BF_ACCUMULATE, 256, &s) ==
        BF_ERR_INVALID_ARG);
  CHECK(bf::make_shape(12, 1, 1, 16, 1, BF_FP16, BF_INPUT_4BIT, 256, &s) == BF_ERR_UNSUPPORTED);
  CHECK(bf::make_shape(16, 1, 1, 16, 1, BF_FP16, BF_INPUT_4BIT, 256, &s) == BF_OK && s.in4);
  CHECK(bf::make_shape(8, 1, 1, 16, 1, BF_FP16, 0, 256, nullptr) == BF_ERR_INVALID_ARG);
  return 0;
}

// Every shape of a sweep gets a default tile that can run it, a legal store
// group count and a positive number of work units; every candidate tile the
// list offers passes or fails check_tile consistently with tile_ok.
static int check_tiles() {
  const int Ns[] = {1, 2, 3, 5, 8, 16, 17, 24, 32, 33, 64, 128, 256, 300, 608, 616, 1248, 1256,
                    4096};
  const int Bs[] = {1, 4, 15, 16, 17, 100, 128, 512, 2048};
  const int64_t Ts[] = {16, 96, 4096, 65536};
  const int Is[] = {1, 2, 3, 4, 5, 16, 17, 64};
  const uint32_t Fs[] = {0u, BF_ACCUMULATE, BF_INPUT_4BIT, BF_OUTPUT_COMPLEX};
  int shapes = 0;
  for (int prec = 0; prec < 3; ++prec)
    for (int N : Ns)
      for (int B : Bs)
        for (int64_t T : Ts)
          for (int I : Is)
            for (uint32_t f : Fs) {
              Shape s;
              const int st = bf::make_shape(N, 3, B, T, I, prec, f, 256, &s);
              if (st != BF_OK) continue;
              ++shapes;
              Tile t{};
              int32_t sgw = 0;
              bf::choose_tile(s, &t, &sgw);
              CHECK(bf::tile_ok(s, t));
              CHECK(bf::check_tile(s, t, sgw) == BF_OK);
              CHECK(bf::units_for(s, t, sgw) > 0);
              CHECK(bf::tile_lds(s.prec, s.Kpad, t) <= bf::kLdsMax);
              int32_t G, QI, SG;
              bf::schedule(s.I, s.T, &G, &QI, &SG);
              CHECK(G >= 1 && QI >= 1 && SG >= 1 && (int64_t)sgw * G % t.mt == 0);
              CHECK((int64_t)SG * 16 * s.I >= s.T);
              for (const Tile& c : bf::compiled_tiles(s)) {
                const int r = bf::check_tile(s, c, c.mt);
                CHECK(r == (bf::tile_ok(s, c) ? BF_OK : BF_ERR_UNSUPPORTED));
              }
              CHECK(bf::check_tile(s, t, 0) == BF_ERR_INVALID_ARG);
              CHECK(bf::input_bytes(s) == (uint64_t)3 * T * (s.in4 ? N : 2 * N));
              CHECK(bf::output_bytes(s) == (uint64_t)3 * B * (s.cx ? T * 4 : T / I * 4));
            }
  CHECK(shapes > 10000);
  return 0;
}

static int check_overlap() {
  char buf[64];
  CHECK(!bf::ranges_overlap(buf, 16, buf + 16, 16));
  CHECK(!bf::ranges_overlap(buf + 16, 16, buf, 16));
  CHECK(bf::ranges_overlap(buf, 17, buf + 16, 16));
  CHECK(bf::ranges_overlap(buf + 16, 16, buf, 17));
  CHECK(bf::ranges_overlap(buf, 64, buf + 10, 1));
  CHECK(bf::ranges_overlap(buf + 10, 1, buf, 64));
  CHECK(!bf::ranges_overlap(buf, 0, buf, 64));
  CHECK(bf::ranges_overlap(buf, 1, buf, 1));
  // far-apart addresses near the top of the address space: no wrap-around
  const void* hi = reinterpret_cast<const void*>(~(uintptr_t)0 - 31);
  const void* lo = reinterpret_cast<const void*>((uintptr_t)64);
  CHECK(!bf::ranges_overlap(hi, 32, lo, 64));
  CHECK(!bf::ranges_overlap(lo, 64, hi, 32));
  CHECK(bf::ranges_overlap(hi, 32, reinterpret_cast<const void*>(~(uintptr_t)0 - 1), 2));
  return 0;
}

static int check_keys() {
  Shape s;
  CHECK(bf::make_shape(32, 1024, 128, 65536, 16, BF_FP16, 0, 256, &s) == BF_OK);
  CHECK(bf::tune_key(s, false) == "gfx950/p1/N32/B~128/I16/C~1024/T~65536");
  CHECK(bf::make_shape(256, 1000, 600, 8192, 64, BF_FP16, 0, 256, &s) == BF_OK);
  CHECK(bf::tune_key(s, true) == "gfx950/p1/N256/B~512/I64/C~512/T~8192/batch");
  CHECK(bf::make_shape(32, 1024, 128, 65536, 1, BF_BF16, BF_INPUT_4BIT | BF_OUTPUT_COMPLEX, 256,
                       &s) == BF_OK);
  CHECK(bf::tune_key(s, false) == "gfx950/p2/N32/B~128/I1/C~1024/T~65536/in4/cx");
  CHECK(bf::make_shape(5, 1, 1, 1, 1, BF_FP32, 0, 256, &s) == BF_OK);
  CHECK(bf::tune_key(s, false) == "gfx950/p0/N5/B~1/I1/C~1/T~1");
  return 0;
}

static const char* kGood =
    "{\n \"gfx950/p1/N32/B~128/I16/C~1024/T~65536\": {\n  \"candidates\": 84,\n  \"ms\": 2.03,\n"
    "  \"tile\": [\n   4,\n   8,\n   1,\n   1,\n   8\n  ]\n },\n"
    " \"k2\": {\"tile\": [4, 2, 2, 0, 2], \"note\": [1, {\"a\": null}, true, \"x\\u0041\\n\"]},\n"
    " \"bad-len\": {\"tile\": [4, 2, 2]},\n"
    " \"bad-frac\": {\"tile\": [4.5, 2, 2, 0, 2]},\n"
    " \"bad-type\": {\"tile\": [\"4\", 2, 2, 0, 2]},\n"
    " \"not-an-object\": 3,\n"
    " \"neg\": {\"tile\": [8, 1, 1, -1, 4]}\n}\n";

static int check_parser() {
  std::vector<bf::TuneEntry> v;
  CHECK(bf::parse_tune_cache(kGood, std::strlen(kGood), &v) == 3);
  CHECK(v[0].key == "gfx950/p1/N32/B~128/I16/C~1024/T~65536");
  CHECK(v[0].tile.mt == 4 && v[0].tile.nbt == 8 && v[0].tile.nbp == 1 && v[0].tile.kres == 1 &&
        v[0].sgw == 8);
  CHECK(v[1].key == "k2" && v[1].sgw == 2);
  CHECK(v[2].key == "neg" && v[2].tile.kres == -1);
  // every proper prefix is rejected (the object is never closed) or, if it
  // ends inside trailing whitespace, accepted with the same entries
  const size_t n = std::strlen(kGood);
  for (size_t k = 0; k < n; ++k) {
    std::vector<bf::TuneEntry> w;
    // exact-size heap copy, so that any read past byte k is caught
    std::vector<char> pre(kGood, kGood + k);
    const int r = bf::parse_tune_cache(pre.data(), pre.size(), &w);
    CHECK(r == -1 || (r == 3 && k >= n - 1));
    CHECK(r != -1 || w.empty());
  }
  // corrupted bytes: never a crash, never an entry with a malformed tile
  uint64_t st = 0x9E3779B97F4A7C15ull;
  for (int it = 0; it < 20000; ++it) {
    std::string t(kGood);
    const int flips = 1 + (int)(st % 4);
    for (int f = 0; f < flips; ++f) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      const size_t pos = (size_t)(st >> 33) % t.size();
      const char alphabet[] = "{}[]\":,\\-0123456789.eE tfnu\x01\xff";
      t[pos] = alphabet[(st >> 13) % (sizeof(alphabet) - 1)];
    }
    std::vector<bf::TuneEntry> w;
    std::vector<char> exact(t.begin(), t.end());
    const int r = bf::parse_tune_cache(exact.data(), exact.size(), &w);
    CHECK(r >= -1 && r <= 16);
    CHECK((int)w.size() == (r < 0 ? 0 : r));
  }
  // nesting deeper than the reader follows is rejected, not recursed into
  std::string deep = "{\"k\": {\"x\": ";
  for (int i = 0; i < 100000; ++i) deep += "[";
  std::vector<bf::TuneEntry> w;
  CHECK(bf::parse_tune_cache(deep.data(), deep.size(), &w) == -1);
  CHECK(bf::parse_tune_cache("[]", 2, &w) == -1);
  CHECK(bf::parse_tune_cache("{}", 2, &w) == 0);
  CHECK(bf::parse_tune_cache("{} x", 4, &w) == -1);
  CHECK(bf::parse_tune_cache("", 0, &w) == -1);
  CHECK(bf::parse_tune_cache(nullptr, 0, &w) == -1);
  { const char* inf = "{\"a\": {\"tile\": [1e999, 1, 1, 1, 1]}}"; CHECK(bf::parse_tune_cache(inf, std::strlen(inf), &w) == -1); }
  return 0;
}

// The repository's own cache file: every entry is read and its key is one
// the library can produce.
static int check_file(const char* path) {
  std::ifstream f(path, std::ios::binary);
  CHECK(f.good());
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  std::vector<bf::TuneEntry> v;
  const int r = bf::parse_tune_cache(text.data(), text.size(), &v);
  CHECK(r > 0);
  int keys = 0;
  for (size_t i = 0; i + 1 < text.size(); ++i)
    if (text.compare(i, 8, "\"gfx950/") == 0) ++keys;
  CHECK(r == keys);
  for (const auto& e : v) {
    CHECK(e.key.compare(0, 8, "gfx950/p") == 0);
    CHECK(e.key.find("/B~") != std::string::npos);
    CHECK(e.sgw >= 1 && e.tile.mt >= 1);
  }
  return 0;
}

int main(int argc, char** argv) {
  if (check_validation() || check_tiles() || check_overlap() || check_keys() || check_parser())
    return 1;
  if (argc > 1 && check_file(argv[1])) return 1;
  std::printf("OK %d checks\n", g_checks);
  return 0;
}
