// bf_host.h -- host-side logic of the beamformer library that needs no HIP:
// argument checks, the work schedule of a plan, the default tile choice, and
// the reader of the autotuner's tile cache.  bf_api.cpp builds on it, and a
// CPU-only test build compiles it with address and undefined-behaviour
// sanitizers.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/bf.h"
#include "bf_tiles.h"

namespace bf {

// Limits of bf_plan_create_ex.
constexpr int32_t kMaxN = 4096;
constexpr int32_t kMaxB = 65536;
constexpr int32_t kMaxC = 1 << 24;
constexpr int64_t kMaxT = (int64_t)1 << 40;
constexpr size_t kLdsMax = 160 * 1024 - 256;  // dynamic LDS; the rest is static

// The facts about a plan that the host logic needs.
struct Shape {
  int32_t N = 0, C = 0, B = 0, I = 0;
  int64_t T = 0;
  int prec = 0;          // bf_precision_t
  uint32_t flags = 0;    // BF_ACCUMULATE | BF_INPUT_4BIT | BF_OUTPUT_COMPLEX
  bool in4 = false;      // 4-bit input (one byte per antenna sample)
  bool cx = false;       // complex FP16 beam output
  bool vec16 = true;     // 2N % 16 == 0: a lane's 16 K values are one 16-byte load
  int32_t Bpad = 0;      // B rounded up to 16
  int32_t Kpad = 0;      // 2N rounded up to kChunk
  int mode = 0;          // Mode
  int n_cu = 256;        // compute units of the device
};

// Validates a plan request and fills *out.  Returns BF_OK,
// BF_ERR_INVALID_ARG (sizes, precision, unknown flags, complex output with
// I != 1 or with BF_ACCUMULATE) or BF_ERR_UNSUPPORTED (4-bit input with
// N % 8 != 0).
int make_shape(int32_t N, int32_t C, int32_t B, int64_t T, int32_t I, int prec, uint32_t flags,
               int n_cu, Shape* out);

int es_of(int prec);
int mode_of(int32_t I);
// Dynamic LDS of a beam range of nbt 16-beam tiles (weight rows for all K).
size_t lds_bytes(int prec, int32_t Kpad, int nbt);
// Dynamic LDS of a tile: none when the weights are read from device memory.
size_t tile_lds(int prec, int32_t Kpad, Tile t);
// Row-tile schedule for integration I: MFMA row tiles per store group (G),
// per window (QI) and store groups per channel (SG).
void schedule(int32_t I, int64_t T, int32_t* G, int32_t* QI, int32_t* SG);
bool same_tile(const Tile& a, const Tile& b);
// Whether the single-set kernel compiled for this shape's input, output
// and row width carries tile t.
bool tile_exists(const Shape& s, Tile t);
// Whether a compiled tile can run the shape (K and LDS budget).
bool tile_ok(const Shape& s, Tile t);
// Work units (workgroups) of one run under (t, sgw).
int64_t units_for(const Shape& s, Tile t, int32_t sgw);
// The default tile and store groups per wave.
void choose_tile(const Shape& s, Tile* t, int32_t* sgw);
// BF_OK if (t, sgw) can run the shape; BF_ERR_UNSUPPORTED (tile not
// compiled, K or LDS) or BF_ERR_INVALID_ARG (sgw).
int check_tile(const Shape& s, Tile t, int32_t sgw);
// Every single-set tile compiled for the shape's form, in list order.
std::vector<Tile> compiled_tiles(const Shape& s);
// The variants the persistent batching kernel carries.
std::vector<Tile> multi_tiles();
// Variants of the eight-wave batching kernels (BF_TILE_LIST_WIDE order).
std::vector<Tile> wide_tiles();

// Bytes of one block of voltages, and of one run's output.
uint64_t input_bytes(const Shape& s);
uint64_t output_bytes(const Shape& s);
// Whether byte ranges [a, a + na) and [b, b + nb) share a byte.
bool ranges_overlap(const void* a, uint64_t na, const void* b, uint64_t nb);

// ---- tile cache written by the autotuner ----
// Key of a shape: precision, input and output form, N, I exactly; B, C and
// T as the largest power of two not above them (their effect on the best
// tile is through the number of work units, which changes slowly); batch
// selects the batching kernel's own entry.
std::string tune_key(const Shape& s, bool batch, const char* arch = "gfx950");
struct TuneEntry {
  std::string key;
  Tile tile;
  int32_t sgw;
};
// Reads the JSON object the autotuner writes ({"key": {"tile": [mt, nbt,
// nbp, kres, sgw], ...}, ...}); entries without a well-formed five-integer
// "tile" are skipped.  Returns the number of entries appended to *out, or -1
// if the text is not a JSON object (out is then unchanged).
int parse_tune_cache(const char* text, size_t len, std::vector<TuneEntry>* out);

}  // namespace bf
