// Device tables of the wave-propagation library (patch rows, tile lists,
// workspace carve-up): plain structs shared by the host runtime, the HIP
// kernels and host-only code that builds the tables.  Not part of the public
// ABI.
#pragma once

#include <stdint.h>

namespace ws {

constexpr int kThreads = 256;  // threads per workgroup of every tile kernel
constexpr int kGroups = 8;     // tile groups of the persistent launch, one per XCD
constexpr int kLine = 32;      // retirement counters sit 128 bytes (32 uints) apart
constexpr int kMaxRowsPerThread = 64;  // DIRECT tiles
constexpr int kMaxMarchRows = 64;      // MARCH segments

// Tile kernels.  DIRECT: one thread per column, every cell computed from its
// 13-point footprint.  MARCH: lane segments sweep up their columns carrying
// the y-direction terms in registers and exchanging x-direction terms with
// neighbouring lanes; a segment of w lanes updates w-4 columns.  PACKED: the
// MARCH sweep with the wavefront's lanes shared by column blocks of several
// narrow patches side by side (each with its own two halo lanes per side).
enum TileVariant { kDirect = 0, kMarch = 1, kPacked = 2 };
constexpr int kMarchWidth = 64;  // MARCH segments are one wavefront wide
constexpr int kSumTile = 64;     // conservation sums: tiles of 64 x 64 cells

// One wavefront of a PACKED tile: up to kMaxPieces column blocks (patch,
// first column c0, w columns) on lanes lane0 .. lane0 + w + 3 (two halo lanes
// each side), all over the rows [r0, r1), which every piece's patch has.
// Each piece carries its addressing, so a wavefront reads nothing per lane
// before its data: org, the pool byte offset of the piece's column c0 - 2 in
// row -2 of plane p; the row and plane strides ldb, plb (bytes); lim, the
// last column offset from c0 - 2 that lies in the padded patch (mx + 3 - c0,
// at most 127).  n = 0: the wavefront has no work (patch[0] still names a
// patch of the tile, for the tile's coefficients).
constexpr int kMaxPieces = 4;
struct PackWave {
  int32_t r0, r1, n, pad_;
  int32_t patch[kMaxPieces];
  uint32_t org[kMaxPieces], ldb[kMaxPieces], plb[kMaxPieces];
  int16_t c0[kMaxPieces], w[kMaxPieces], lane0[kMaxPieces], lim[kMaxPieces];
};
static_assert(sizeof(PackWave) == 112, "PackWave is 28 words");

// One row of the device patch table.
struct PatchRow {
  int64_t q_off;   // element offset of the patch's storage (row j = -2 of plane p)
  int32_t mx, my;  // interior cells
  int32_t ld;      // row stride (elements)
  int32_t col0;    // storage column of interior i = 0 (ghost i=-2 sits at col0-2)
  int64_t plane;   // plane stride (elements): ld * (my + 4)
  int32_t inst;    // instance (material, dt)
  int32_t bc;      // WS_BC_*
  int32_t variant;  // TileVariant
  int32_t tw, th;  // DIRECT: tile of tw x th cells; MARCH: segments of tw lanes, th rows
  int32_t ntx, nty;  // tiles in x and y
  double dx, dy;
  int64_t mask_off;  // byte offset of the patch's (mx+1)*(my+1) mask bytes
  int32_t tile_begin, n_tiles;  // the patch's tiles in the tile list (PACKED: one tile holding it)
  int32_t sum_begin, sum_n;     // the patch's tiles in the conservation-sum list
};

// A tile: patch and tile position; a PACKED tile has patch = -1 - g and its
// four wavefronts are PackWave 4g .. 4g+3.
struct TileEntry {
  int32_t patch;
  uint16_t tx, ty;
};

struct InstRow {
  double c, Z;
};

// Workspace carve-up (byte offsets inside the caller's workspace buffer).
struct WsLayout {
  int64_t patches, inst, tiles, packs, stiles, dt, cfl_tile, inst_acc, cfl_last, cfl_max,
      cfl_patch_last, level_last, retire, partials, patch_sums, sums, total;
  int64_t max_tiles, max_pack_waves, n_sum_tiles;
};

}  // namespace ws
