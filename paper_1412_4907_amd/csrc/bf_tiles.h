// bf_tiles.h -- constants, integration classes and the compiled tile
// variants of the beamform kernel.  Plain C++ with no HIP dependency: the
// kernels (through bf_internal.h) and the host logic (bf_host.h) share it.
#pragma once

#include <stdint.h>

namespace bf {

constexpr int kMaxProbs = 16;   // beam sets per launch (kernel-argument table)
constexpr int kWaves = 4;       // waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kWideWaves = 8;   // waves per workgroup of the eight-wave form
constexpr int kWideThreads = 64 * kWideWaves;
constexpr int kKresWide = -2;   // Tile::kres of the eight-wave streamed form
constexpr int kXcds = 8;        // accelerator dies (XCDs), each with its own L2
constexpr int kQueueStride = 16;  // int32 slots between the per-XCD queue counters
constexpr int kQueueInts = kXcds * kQueueStride;  // one persistent launch's counters
constexpr int kChunk = 64;      // real K elements (32 antennas) per chunk
constexpr int kLdsPad = 16;     // bytes added to each LDS weight row

// Integration classes; each is a separate kernel instantiation:
// I == 1, I == 2, I >= 3 with I % 4 != 0 (padded windows), I % 4 == 0;
// and complex beam output (no detection, I == 1 row mapping).
enum Mode : int { kModeI1 = 0, kModeI2 = 1, kModeGen = 2, kModeGen4 = 3, kModeCx = 4 };

// Tile variant of the beamform kernel.
struct Tile {
  int mt;    // 16-row MFMA tiles per wave step
  int nbt;   // 16-beam tiles per workgroup beam range
  int nbp;   // 16-beam tiles per accumulator pass
  int kres;  // K chunks held in registers per wave step (0: streamed)
};

// Waves that share one work unit's staged weights.
constexpr int waves_of(Tile t) { return t.kres == kKresWide ? kWideWaves : kWaves; }

// Compiled tile variants: (MT, NBT, NBP, KRES).  KRES > 0 variants serve
// plans with Kpad / 64 <= KRES; KRES == 0 streams K with the unit's weights
// in LDS; KRES == -1 streams K with the weights read from device memory (any
// K: arrays whose weight rows do not fit LDS); KRES == -2 is the eight-wave
// streamed form below.  The generic (byte-load)
// list serves plans whose 2N is not a multiple of 16.
#define BF_TILE_LIST_VEC16                                                        \
  BF_TILE(8, 8, 1, 1) BF_TILE(4, 8, 2, 1) BF_TILE(4, 8, 1, 1) BF_TILE(8, 4, 1, 1)  \
  BF_TILE(4, 4, 1, 1) BF_TILE(4, 8, 1, 2) BF_TILE(4, 4, 1, 2) BF_TILE(4, 8, 2, 0)  \
  BF_TILE(4, 4, 2, 0) BF_TILE(4, 2, 2, 0) BF_TILE(4, 2, 1, 0) BF_TILE(4, 1, 1, 0)  \
  BF_TILE(4, 2, 2, -1) BF_TILE(8, 1, 1, -1)
#define BF_TILE_LIST_GENERIC BF_TILE(4, 8, 2, 0) BF_TILE(4, 1, 1, 0) BF_TILE(4, 2, 2, -1)
// Variants compiled for 4-bit input.
#define BF_TILE_LIST_IN4                                                          \
  BF_TILE(4, 8, 1, 1) BF_TILE(4, 8, 2, 1) BF_TILE(4, 4, 1, 1) BF_TILE(4, 8, 1, 2)  \
  BF_TILE(4, 8, 2, 0) BF_TILE(4, 4, 2, 0) BF_TILE(4, 2, 2, 0) BF_TILE(4, 1, 1, 0)  \
  BF_TILE(4, 2, 2, -1)
// Variants compiled for complex beam output (16-byte rows; byte-load plans
// use the generic list).
#define BF_TILE_LIST_CX                                                           \
  BF_TILE(4, 8, 1, 1) BF_TILE(4, 4, 1, 1) BF_TILE(4, 8, 1, 2) BF_TILE(4, 8, 2, 0)  \
  BF_TILE(4, 2, 2, 0) BF_TILE(4, 1, 1, 0) BF_TILE(4, 2, 2, -1)
// Eight-wave streamed form (FP16/BF16, power output with I == 1 or
// I % MT == 0, every beam tile of the range in one pass: NBP == NBT): the
// unit's weights for all K are staged in LDS once and shared by eight waves,
// two per SIMD.
#define BF_TILE_LIST_WIDE BF_TILE(4, 4, 4, -2) BF_TILE(4, 2, 2, -2)
// Variants compiled into the persistent batching kernel (16-byte loads).
// (MT = 8 variants are left out: their register use would halve the
// kernel's occupancy for every set.)
#define BF_TILE_LIST_MULTI                                                        \
  BF_TILE(4, 8, 1, 1) BF_TILE(4, 8, 1, 2) BF_TILE(4, 4, 2, 0) BF_TILE(4, 2, 2, 0)  \
  BF_TILE(4, 1, 1, 0)

}  // namespace bf
