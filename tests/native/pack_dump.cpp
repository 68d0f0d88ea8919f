// Host-only driver of the library's tile-list builders (ws_pack.h): reads a
// level's patches from stdin, builds the conservation-sum tiles and the
// PACKED tiles exactly as the library does, and prints the tables as text
// for the replay in test_pack_tiles.py.
//
// stdin: n, then per patch "mx my inst dx dy variant th".  The patches get
// a pool layout of FP64 elements (wide ones with their interior aligned away
// from column 2, as the library does for alignment).
// stdout: lines "P k tile_begin n_tiles sum_begin sum_n q_off col0 ld plane",
// "T patch tx ty", "S patch tx ty", "W r0 r1 n patch[4] c0[4] w[4] lane0[4]
// org[4] ldb[4] plb[4] lim[4]", then "BOUND max_pack_waves".
#include <cstdio>
#include <numeric>
#include <vector>

#include "../../paper_1808_02638_amd/csrc/ws_pack.h"

int main() {
  using namespace ws;
  int n = 0;
  if (std::scanf("%d", &n) != 1 || n < 1) return 2;
  std::vector<PatchRow> rows(n);
  int64_t bound = 0;
  for (int k = 0; k < n; ++k) {
    PatchRow &r = rows[k];
    if (std::scanf("%d %d %d %lf %lf %d %d", &r.mx, &r.my, &r.inst, &r.dx, &r.dy, &r.variant,
                   &r.th) != 7)
      return 2;
    r.tw = kMarchWidth;
    bound += packed_wave_bound(r.mx, r.my);
  }
  int64_t cur = 0;
  for (PatchRow &r : rows) {
    r.col0 = r.mx >= 128 ? 16 : 2;
    r.ld = (int32_t)((r.col0 + r.mx + 2 + 15) / 16 * 16);
    r.plane = (int64_t)r.ld * (r.my + 4);
    r.q_off = (cur + 31) / 32 * 32;
    cur = r.q_off + 3 * r.plane;
  }
  // the library's patch order: largest first, stable
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (int64_t)rows[a].mx * rows[a].my > (int64_t)rows[b].mx * rows[b].my;
  });
  std::vector<TileEntry> stiles, tiles;
  std::vector<PackWave> packs;
  sum_tiles(rows, stiles);
  pack_level(rows, order, 8, tiles, packs);
  for (int k = 0; k < n; ++k)
    std::printf("P %d %d %d %d %d %lld %d %d %lld\n", k, rows[k].tile_begin, rows[k].n_tiles,
                rows[k].sum_begin, rows[k].sum_n, (long long)rows[k].q_off, rows[k].col0,
                rows[k].ld, (long long)rows[k].plane);
  for (const TileEntry &t : tiles) std::printf("T %d %d %d\n", t.patch, t.tx, t.ty);
  for (const TileEntry &t : stiles) std::printf("S %d %d %d\n", t.patch, t.tx, t.ty);
  for (const PackWave &w : packs) {
    std::printf("W %d %d %d", w.r0, w.r1, w.n);
    for (int m = 0; m < kMaxPieces; ++m) std::printf(" %d", w.patch[m]);
    for (int m = 0; m < kMaxPieces; ++m) std::printf(" %d", w.c0[m]);
    for (int m = 0; m < kMaxPieces; ++m) std::printf(" %d", w.w[m]);
    for (int m = 0; m < kMaxPieces; ++m) std::printf(" %d", w.lane0[m]);
    for (int m = 0; m < kMaxPieces; ++m) std::printf(" %u", w.org[m]);
    for (int m = 0; m < kMaxPieces; ++m) std::printf(" %u", w.ldb[m]);
    for (int m = 0; m < kMaxPieces; ++m) std::printf(" %u", w.plb[m]);
    for (int m = 0; m < kMaxPieces; ++m) std::printf(" %d", w.lim[m]);
    std::printf("\n");
  }
  std::printf("BOUND %lld\n", (long long)bound);
  return 0;
}
