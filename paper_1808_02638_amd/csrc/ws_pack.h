// Host-side construction of the PACKED tiles and of the conservation-sum
// tiles of a level: plain C++ over the device tables' structs (no HIP), so
// the same code serves the library and host-only checks of its invariants.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "ws_tables.h"

namespace ws {

// PACKED tiles cut a patch into column blocks of at most kPieceCols columns
// and row segments of at least kMinPackedRows rows; a block that fills the
// room left in a wavefront has at least kMinPieceCols columns.
constexpr int kPieceCols = kMarchWidth - 4;
constexpr int kMinPackedRows = 4;
constexpr int kMinPieceCols = 8;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// PACKED tiles an mx x my patch can add: each of its column blocks (a first
// one in the room another patch left, then at most ceil(mx / kPieceCols)
// more) starts at most one lane column, whose tiles are ceil(my / th) with
// th >= 4 kMinPackedRows.  Four wavefronts per tile.
inline int64_t packed_tile_bound(int mx, int my) {
  return (ceil_div(mx, kPieceCols) + 1) * ceil_div(my, 4 * kMinPackedRows);
}
inline int64_t packed_wave_bound(int mx, int my) { return 4 * packed_tile_bound(mx, my); }

inline int64_t sum_tiles_of(int mx, int my) {
  return ceil_div(mx, kSumTile) * ceil_div(my, kSumTile);
}

// Conservation-sum tiles: kSumTile x kSumTile cells, each patch's row by row,
// patches in index order (fixed by the patch sizes alone).
inline void sum_tiles(std::vector<PatchRow> &rows, std::vector<TileEntry> &stiles) {
  stiles.clear();
  for (int k = 0; k < (int)rows.size(); ++k) {
    PatchRow &r = rows[k];
    const int sx = (int)ceil_div(r.mx, kSumTile), sy = (int)ceil_div(r.my, kSumTile);
    r.sum_begin = (int32_t)stiles.size();
    for (int ty = 0; ty < sy; ++ty)
      for (int tx = 0; tx < sx; ++tx) stiles.push_back(TileEntry{k, (uint16_t)tx, (uint16_t)ty});
    r.sum_n = (int32_t)stiles.size() - r.sum_begin;
  }
}

// Append the PACKED tiles of the patches whose variant is kPacked (visited
// in `order`) to `tiles`, their wavefronts to `packs` (cleared first); the
// pieces' byte offsets are for elements of elem_bytes and must stay below
// 2^32 (the caller's pools are under 2^31 bytes).
//
// Patches that share an instance, cell sizes, height and tile height form a
// group: one wavefront's coefficients serve them all and they have the same
// rows.  A group's patches are laid side by side into lane columns, next-fit:
// a patch's columns go into the room left in the current lane column (a
// block of its width plus four halo lanes), the rest into fresh lane columns
// of up to kPieceCols columns, so only the halo lanes and a column's last
// few lanes stay idle; a lane column holds at most kMaxPieces blocks.  Each
// lane column is then tiled like a MARCH patch: ceil(H / th) tiles, each
// with four wavefronts marching stacked row segments of equal height (at
// most th / 4 rows; empty past the last row only when H < 4), so the rows
// two segments share are read by one workgroup.  A
// patch's tile_begin names one tile holding it (n_tiles = 1): its Courant
// number is that tile's, since every patch of the tile has the same
// instance and cell sizes.
inline void pack_level(std::vector<PatchRow> &rows, const std::vector<int> &order, int elem_bytes,
                       std::vector<TileEntry> &tiles, std::vector<PackWave> &packs) {
  packs.clear();
  const int n = (int)rows.size();
  std::vector<int> group_of(n, -1);
  std::vector<int> leaders;  // first patch of each group
  for (int k : order) {
    const PatchRow &r = rows[k];
    if (r.variant != kPacked) continue;
    for (int g = 0; g < (int)leaders.size(); ++g) {
      const PatchRow &q = rows[leaders[g]];
      if (q.inst == r.inst && q.dx == r.dx && q.dy == r.dy && q.my == r.my && q.th == r.th) {
        group_of[k] = g;
        break;
      }
    }
    if (group_of[k] < 0) {
      group_of[k] = (int)leaders.size();
      leaders.push_back(k);
    }
  }
  std::vector<PackWave> cols;  // the current group's lane columns (rows unset)
  for (int g = 0; g < (int)leaders.size(); ++g) {
    cols.clear();
    int used = kMarchWidth;  // lanes taken in the current lane column (none open yet)
    for (int k : order) {
      if (group_of[k] != g) continue;
      const PatchRow &r = rows[k];
      for (int c0 = 0; c0 < r.mx;) {
        const int room = kMarchWidth - used - 4;
        if (room < std::min(kMinPieceCols, r.mx - c0) || cols.back().n == kMaxPieces) {
          cols.push_back(PackWave{});
          used = 0;
          continue;
        }
        const int w = std::min(r.mx - c0, room);
        PackWave &pw = cols.back();
        pw.patch[pw.n] = k;
        pw.org[pw.n] = (uint32_t)((r.q_off + r.col0 + c0 - 2) * elem_bytes);
        pw.ldb[pw.n] = (uint32_t)(r.ld * elem_bytes);
        pw.plb[pw.n] = (uint32_t)(r.plane * elem_bytes);
        pw.c0[pw.n] = (int16_t)c0;
        pw.w[pw.n] = (int16_t)w;
        pw.lane0[pw.n] = (int16_t)used;
        pw.lim[pw.n] = (int16_t)std::min(r.mx + 3 - c0, 127);
        ++pw.n;
        used += w + 4;
        c0 += w;
      }
    }
    // ceil(H / th) tiles per lane column, their rows spread evenly over the
    // four wavefronts (at most th / 4 each)
    const int H = rows[leaders[g]].my, th = rows[leaders[g]].th;
    const int seg = (int)ceil_div(H, 4 * ceil_div(H, th));
    for (const PackWave &col : cols)
      for (int y0 = 0; y0 < H; y0 += 4 * seg) {
        const int tix = (int)tiles.size();
        tiles.push_back(TileEntry{-1 - (int32_t)(packs.size() / 4), 0, 0});
        for (int q = 0; q < 4; ++q) {
          PackWave pw = col;
          pw.r0 = y0 + q * seg;
          pw.r1 = std::min(pw.r0 + seg, H);
          if (pw.r0 >= H) pw.n = 0, pw.r0 = pw.r1 = 0;
          packs.push_back(pw);
        }
        for (int m = 0; m < col.n; ++m) {
          PatchRow &r = rows[col.patch[m]];
          r.tile_begin = tix;
          r.n_tiles = 1;
        }
      }
  }
  for (PatchRow &r : rows)
    if (r.variant == kPacked) r.ntx = r.nty = 1;
}

}  // namespace ws
