// Host runtime of the wave-propagation library: the C ABI declared in
// include/wavestep.h.  It owns host metadata only; device memory and the
// stream belong to the caller.
//
// Level batching (after the paper's kernel merging, Sec. 3.1.3, and its
// largest-first patch order): every patch is cut into tiles, the tiles of all
// patches go into one device tile list ordered by patch size (largest patch
// first), and one persistent launch works the list, split into one contiguous
// run per XCD.  The per-patch baseline launches the same kernel once per patch.  The paper's
// per-patch maximum-speed array (Sec. 3.2.2) is kept, and the level-wide
// maximum is also reduced on the device, so dt can be updated there too.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/wavestep.h"
#include "ws_internal.h"
#include "ws_pack.h"

using namespace ws;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(WS_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }
bool same_rel(double a, double b) { return std::fabs(a - b) <= 1e-12 * std::fabs(b); }

constexpr int kTileWidths[] = {8, 16, 32, 64, 128, 256};

struct PoolLayout {
  std::vector<int64_t> off;  // element offsets
  std::vector<int32_t> ld, col0;
  std::vector<int64_t> plane;
  int64_t elems = 0;
};

// Device layout of the q pools: per patch three planes of (my+4) rows of ld
// elements.  Wide patches align interior column 0 to 128 bytes; every patch
// starts on a 256-byte boundary.
PoolLayout pool_layout(const ws_patch_desc *p, int n, int dtype) {
  PoolLayout L;
  const int64_t es = dtype == WS_F32 ? 4 : 8;
  const int64_t al = 128 / es;
  int64_t cur = 0;
  for (int k = 0; k < n; ++k) {
    int32_t col0, ld;
    if (p[k].mx >= 8 * al) {
      col0 = (int32_t)al;
      ld = (int32_t)round_up(col0 + p[k].mx + 2, al);
    } else {
      col0 = 2;
      ld = (int32_t)round_up(p[k].mx + 4, 4);
    }
    const int64_t plane = (int64_t)ld * (p[k].my + 4);
    cur = round_up(cur, 256 / es);
    L.off.push_back(cur);
    L.ld.push_back(ld);
    L.col0.push_back(col0);
    L.plane.push_back(plane);
    cur += 3 * plane;
  }
  L.elems = round_up(cur, 256 / es);
  return L;
}

// Columns a tile updates: DIRECT tw, MARCH tw - 4 (two halo lanes per side).
int tile_cols(int variant, int tw) { return variant == kMarch ? tw - 4 : tw; }

int64_t tiles_of(int mx, int my, int variant, int tw, int th) {
  const int cols = tile_cols(variant, tw);
  return (int64_t)((mx + cols - 1) / cols) * ((my + th - 1) / th);
}

// Upper bound of the tile count over every valid tiling (sizes the workspace).
int64_t max_tiles_of(const ws_patch_desc *p, int n) {
  int64_t t = 0;
  for (int k = 0; k < n; ++k) {
    int64_t m = 0;
    for (int tw : kTileWidths) {
      m = std::max(m, tiles_of(p[k].mx, p[k].my, kDirect, tw, kThreads / tw));
      if (tw == kMarchWidth)
        m = std::max(m, tiles_of(p[k].mx, p[k].my, kMarch, tw, kThreads / tw));
    }
    t += m;
  }
  return t;
}

// Workspace of a level.  Tiles: a patch takes at most max_tiles_of's count,
// or with frozen ghosts packed_tile_bound's; PACKED wavefronts stay within
// packed_wave_bound per patch.
WsLayout ws_layout_of(const ws_patch_desc *p, int n, int n_inst) {
  WsLayout L{};
  int64_t cur = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = cur;
    cur = round_up(cur + std::max<int64_t>(bytes, 8), 256);
    return o;
  };
  L.max_tiles = max_tiles_of(p, n);
  L.max_pack_waves = 0;
  L.n_sum_tiles = 0;
  for (int k = 0; k < n; ++k) {
    if (p[k].bc == WS_BC_NONE) {
      L.max_tiles += packed_tile_bound(p[k].mx, p[k].my);
      L.max_pack_waves += packed_wave_bound(p[k].mx, p[k].my);
    }
    L.n_sum_tiles += sum_tiles_of(p[k].mx, p[k].my);
  }
  L.patches = take((int64_t)n * sizeof(PatchRow));
  L.inst = take((int64_t)n_inst * sizeof(InstRow));
  L.tiles = take(L.max_tiles * (int64_t)sizeof(TileEntry));
  L.packs = take(L.max_pack_waves * (int64_t)sizeof(PackWave));
  L.stiles = take(L.n_sum_tiles * (int64_t)sizeof(TileEntry));
  L.dt = take(8LL * n_inst);
  L.cfl_tile = take(8 * L.max_tiles);
  L.inst_acc = take(8LL * kGroups * n_inst);
  L.cfl_last = take(8LL * n_inst);
  L.cfl_max = take(8LL * n_inst);
  L.cfl_patch_last = take(8LL * n);
  L.level_last = take(8);
  L.retire = take(4LL * kLine * (kGroups + 1));
  L.partials = take(24 * L.n_sum_tiles);
  L.patch_sums = take(24LL * n);
  L.sums = take(24LL * n_inst);
  L.total = cur;
  return L;
}

bool valid_tile(int variant, int tw, int th) {
  if (variant == kPacked)  // four wavefronts of th / 4 rows
    return tw == kMarchWidth && th % 4 == 0 && th / 4 >= kMinPackedRows &&
           th / 4 <= kMaxMarchRows;
  if (variant != kDirect && variant != kMarch) return false;
  bool ok_w = false;
  for (int w : kTileWidths) ok_w |= (w == tw);
  if (!ok_w) return false;
  if (variant == kMarch && tw != kMarchWidth) return false;
  const int nty = kThreads / tw;
  const int rmax = variant == kMarch ? kMaxMarchRows : kMaxRowsPerThread;
  return th >= nty && th % nty == 0 && th / nty <= rmax;
}

// Default tiling.  Patches at least 24 cells wide (not periodic): MARCH tiles
// of four 60-column segments.  A large patch gets the segment height that
// makes its tile count just fit one round of resident workgroups (assumed 4
// per CU); a small one spreads its rows over the four segments (up to 16
// rows each, so that many patches fill the GPU together); up to 64 rows per
// segment.  Narrower patches: DIRECT tiles whose width in {8..64} wastes the
// fewest columns (larger on ties), up to 8 rows per thread.
void default_tile(int mx, int my, int bc, int n_cu, int *variant, int *tw, int *th) {
  if (mx >= 24 && bc != WS_BC_PERIODIC) {
    *variant = kMarch;
    *tw = kMarchWidth;
    const int ntx = (mx + kMarchWidth - 5) / (kMarchWidth - 4);
    const int tile_rows = std::max(1, 4 * std::max(n_cu, 1) / ntx);  // rows of tiles
    const int seg = (my + 4 * tile_rows - 1) / (4 * tile_rows);      // rows per segment
    *th = 4 * std::max(std::min(seg, kMaxMarchRows), std::min(16, (my + 3) / 4));
    return;
  }
  *variant = kDirect;
  int best = 64;
  {
    int64_t best_waste = -1;
    for (int w : {64, 32, 16, 8}) {
      const int64_t waste = (int64_t)((mx + w - 1) / w) * w - mx;
      if (best_waste < 0 || waste < best_waste) {
        best_waste = waste;
        best = w;
      }
    }
  }
  const int nty = kThreads / best;
  int r = (my + nty - 1) / nty;
  r = std::max(1, std::min(r, 8));
  *tw = best;
  *th = nty * r;
}

// MARCH tiles address a patch with 32-bit byte offsets (all three planes).
bool march_fits(int64_t plane, int dtype) {
  return 3 * plane * (dtype == WS_F32 ? 4 : 8) < (int64_t{1} << 31);
}

int check_desc(const ws_patch_desc *p, int n, int n_inst) {
  if (n < 1 || !p) return fail(WS_EINVAL, "need at least one patch");
  if (n_inst < 1) return fail(WS_EINVAL, "need at least one instance");
  for (int k = 0; k < n; ++k) {
    const ws_patch_desc &d = p[k];
    if (d.mx < 1 || d.my < 1) return fail(WS_EINVAL, "patch %d: mx, my must be >= 1", k);
    if (d.mx > 65535 * 8 || d.my > 1000000)
      return fail(WS_EINVAL, "patch %d: too large", k);
    if (!(d.dx > 0.0) || !(d.dy > 0.0) || !std::isfinite(d.dx) || !std::isfinite(d.dy))
      return fail(WS_EINVAL, "patch %d: dx, dy must be finite and > 0", k);
    if (d.instance < 0 || d.instance >= n_inst)
      return fail(WS_EINVAL, "patch %d: instance %d out of range", k, d.instance);
    if (d.bc != WS_BC_NONE && d.bc != WS_BC_EXTRAP && d.bc != WS_BC_PERIODIC)
      return fail(WS_EINVAL, "patch %d: unknown bc %d", k, d.bc);
    if (d.bc == WS_BC_PERIODIC && (d.mx < 2 || d.my < 2))
      return fail(WS_EINVAL, "patch %d: periodic needs mx, my >= 2", k);
  }
  return WS_OK;
}

}  // namespace

struct ws_ctx {
  int dtype = WS_F64, limiter = WS_LIM_MC;
  int n_patches = 0, n_inst = 0;
  hipStream_t stream = nullptr;
  void *pool[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t pool_bytes = 0;
  char *ws = nullptr;
  WsLayout L{};
  PoolLayout P;
  std::vector<ws_patch_desc> desc;
  std::vector<PatchRow> rows;
  std::vector<TileEntry> tiles;
  std::vector<PackWave> packs;  // wavefronts of the PACKED tiles
  std::vector<TileEntry> stiles;  // conservation-sum tiles (fixed by the patch sizes)
  std::vector<int> order;  // patches largest first
  int n_cu = 0, wg_per_cu = 0, grid = 0, occupancy = 0;
  int vars = 1;          // tile variants present (bit 0 DIRECT, bit 1 MARCH, bit 2 PACKED)
  int wg_override = 0;   // workgroups per CU set by the caller (0: occupancy)
  int max_padded_cells = 0;
  int max_ring = 0;  // interior cells next to a side, largest patch
  int max_mx = 0, max_my = 0;
  int64_t mask_total = 0;  // bytes of the branch masks of all patches
  double *host_buf = nullptr;
  int64_t host_buf_bytes = 0;
  char *stage = nullptr;  // pinned staging for downloads into pageable host memory
  int64_t stage_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_steps = 0, graph_start_pool = 0;
  std::vector<InstRow> inst_host;  // (c, Z) per instance, as on the device
  void *medium = nullptr;          // per-cell (c, Z) planes, laid out like a q pool
  // tiled level: per-patch ghost-ring offsets and the ghost source table
  const int64_t *link_ring0 = nullptr;
  const int64_t *link_src = nullptr;
  int link_max_ring = 0;
  int fine_in_couplings = 0;  // couplings whose fine level this is (its ghosts come from them)
  // limiter code of the kernel launchers (the medium selects its own kernel)
  int lim_code() const { return limiter | (medium ? kMediumFlag : 0); }

  CflSlots slots() {
    CflSlots c;
    c.dt = reinterpret_cast<double *>(ws + L.dt);
    c.cfl_tile = reinterpret_cast<double *>(ws + L.cfl_tile);
    c.inst_acc = reinterpret_cast<unsigned long long *>(ws + L.inst_acc);
    c.cfl_last = reinterpret_cast<double *>(ws + L.cfl_last);
    c.cfl_max = reinterpret_cast<double *>(ws + L.cfl_max);
    c.level_last = reinterpret_cast<double *>(ws + L.level_last);
    c.n_inst = n_inst;
    return c;
  }
  const PatchRow *d_patches() const { return reinterpret_cast<const PatchRow *>(ws + L.patches); }
  const TileEntry *d_tiles() const { return reinterpret_cast<const TileEntry *>(ws + L.tiles); }

  StepArgs step_args(int src, double dt_override, double cfl_desired) {
    StepArgs a{};
    a.patches = d_patches();
    a.tiles = d_tiles();
    a.n_tiles = (int32_t)tiles.size();
    a.tile_base = 0;
    a.persistent = 1;
    a.packs = reinterpret_cast<const PackWave *>(ws + L.packs);
    a.qin = pool[src];
    a.qout = pool[1 - src];
    a.pool_bytes = (int32_t)std::min<int64_t>(pool_bytes, INT32_MAX);
    a.inst = reinterpret_cast<const InstRow *>(ws + L.inst);
    a.slots = slots();
    a.dt = a.slots.dt;
    a.dt_override = dt_override;
    a.cfl_desired = cfl_desired;
    a.retire = reinterpret_cast<unsigned int *>(ws + L.retire);
    a.masks = nullptr;
    a.medium = medium;
    return a;
  }

  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    graph_steps = 0;
  }

  int pack_tiles() {
    pack_level(rows, order, dtype == WS_F32 ? 4 : 8, tiles, packs);
    if ((int64_t)packs.size() > L.max_pack_waves)
      return fail(WS_EINVAL, "PACKED wavefront list overflow");
    return WS_OK;
  }

  // Tile list: patches largest first, each patch's tiles row by row; then the
  // PACKED tiles.
  int build_tiles() {
    tiles.clear();
    for (int k : order) {
      PatchRow &r = rows[k];
      if (r.variant == kPacked) continue;
      const int cols = tile_cols(r.variant, r.tw);
      r.ntx = (r.mx + cols - 1) / cols;
      r.nty = (r.my + r.th - 1) / r.th;
      r.tile_begin = (int32_t)tiles.size();
      for (int ty = 0; ty < r.nty; ++ty)
        for (int tx = 0; tx < r.ntx; ++tx) tiles.push_back(TileEntry{k, (uint16_t)tx, (uint16_t)ty});
      r.n_tiles = (int32_t)tiles.size() - r.tile_begin;
    }
    if (int rc = pack_tiles()) return rc;
    if ((int64_t)tiles.size() > L.max_tiles) return fail(WS_EINVAL, "tile list overflow");
    vars = 0;
    for (const PatchRow &r : rows) vars |= r.variant == kPacked ? 4 : r.variant == kMarch ? 2 : 1;
    if (step_occupancy(dtype, lim_code(), vars, &occupancy) != 0 || occupancy < 1) occupancy = 1;
    wg_per_cu = wg_override > 0 ? wg_override : occupancy;
    HIPCHK(hipMemcpyAsync(ws + L.patches, rows.data(), rows.size() * sizeof(PatchRow),
                          hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(ws + L.tiles, tiles.data(), tiles.size() * sizeof(TileEntry),
                          hipMemcpyHostToDevice, stream));
    if (!packs.empty())
      HIPCHK(hipMemcpyAsync(ws + L.packs, packs.data(), packs.size() * sizeof(PackWave),
                            hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(ws + L.stiles, stiles.data(), stiles.size() * sizeof(TileEntry),
                          hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
    grid = (int)std::min<int64_t>((int64_t)n_cu * wg_per_cu, (int64_t)tiles.size());
    return WS_OK;
  }
};

extern "C" {

const char *ws_last_error(void) { return g_err.c_str(); }

int ws_layout(const ws_patch_desc *patches, int32_t n_patches, int32_t n_instances, int32_t dtype,
              int64_t *pool_bytes, int64_t *ws_bytes) {
  if (dtype != WS_F64 && dtype != WS_F32) return fail(WS_EINVAL, "unknown dtype %d", dtype);
  if (int rc = check_desc(patches, n_patches, n_instances)) return rc;
  const PoolLayout P = pool_layout(patches, n_patches, dtype);
  const WsLayout L = ws_layout_of(patches, n_patches, n_instances);
  if (pool_bytes) *pool_bytes = P.elems * (dtype == WS_F32 ? 4 : 8);
  if (ws_bytes) *ws_bytes = L.total;
  return WS_OK;
}

}  // extern "C"

// Arguments every level set-up checks: dtype, limiter, the patch list and
// the materials.
static int check_level(const ws_patch_desc *patches, int32_t n_patches, const ws_material *mats,
                       int32_t n_instances, int32_t dtype, int32_t limiter) {
  if (dtype != WS_F64 && dtype != WS_F32) return fail(WS_EINVAL, "unknown dtype %d", dtype);
  {
    const int lim = limiter & ~WS_TRANSVERSE_CORR;
    if (lim != WS_LIM_MC && lim != WS_LIM_NONE && lim != WS_LIM_VANLEER)
      return fail(WS_EINVAL, "unknown limiter %d", limiter);
  }
  if (int rc = check_desc(patches, n_patches, n_instances)) return rc;
  if (!mats) return fail(WS_EINVAL, "materials are NULL");
  for (int k = 0; k < n_instances; ++k)
    if (!(mats[k].rho > 0.0) || !(mats[k].K > 0.0) || !std::isfinite(mats[k].rho) ||
        !std::isfinite(mats[k].K))
      return fail(WS_EINVAL, "instance %d: rho and K must be finite and > 0", k);
  return WS_OK;
}

// Host metadata of a level over the given pools and workspace: pool layout,
// patch rows with the default tiling, the instance table and the patch order
// (largest first).  Touches no device memory.
static int setup_level(ws_ctx *c, const ws_patch_desc *patches, int32_t n_patches,
                       const ws_material *mats, int32_t n_instances, int32_t dtype,
                       int32_t limiter, void *pool_a, void *pool_b, int64_t pool_bytes, char *ws,
                       hipStream_t stream) {
  c->dtype = dtype;
  c->limiter = limiter;
  c->n_patches = n_patches;
  c->n_inst = n_instances;
  c->stream = stream;
  c->pool[0] = pool_a;
  c->pool[1] = pool_b;
  c->pool_bytes = pool_bytes;
  c->ws = ws;
  c->L = ws_layout_of(patches, n_patches, n_instances);
  c->P = pool_layout(patches, n_patches, dtype);
  c->desc.assign(patches, patches + n_patches);

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(WS_EHIP, "hipGetDevice failed");
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(WS_EHIP, "cannot query the CU count");

  std::vector<InstRow> inst(n_instances);
  for (int k = 0; k < n_instances; ++k) {
    inst[k].c = std::sqrt(mats[k].K / mats[k].rho);
    inst[k].Z = mats[k].rho * inst[k].c;
  }
  c->inst_host = inst;
  c->rows.resize(n_patches);
  int64_t mask_off = 0;
  for (int k = 0; k < n_patches; ++k) {
    PatchRow &r = c->rows[k];
    const ws_patch_desc &d = patches[k];
    r.q_off = c->P.off[k];
    r.mx = d.mx;
    r.my = d.my;
    r.ld = c->P.ld[k];
    r.col0 = c->P.col0[k];
    r.plane = c->P.plane[k];
    r.inst = d.instance;
    r.bc = d.bc;
    default_tile(d.mx, d.my, d.bc, c->n_cu, &r.variant, &r.tw, &r.th);
    if (r.variant == kMarch && !march_fits(r.plane, dtype)) {
      default_tile(d.mx, d.my, WS_BC_PERIODIC, c->n_cu, &r.variant, &r.tw, &r.th);  // DIRECT
    }
    r.dx = d.dx;
    r.dy = d.dy;
    r.mask_off = mask_off;
    mask_off += (int64_t)(d.mx + 1) * (d.my + 1);
    c->max_padded_cells = std::max(c->max_padded_cells, (d.mx + 4) * (d.my + 4));
    c->max_ring = std::max(c->max_ring, 2 * (d.mx + d.my));
    c->max_mx = std::max(c->max_mx, d.mx);
    c->max_my = std::max(c->max_my, d.my);
  }
  c->mask_total = mask_off;
  sum_tiles(c->rows, c->stiles);
  c->order.resize(n_patches);
  std::iota(c->order.begin(), c->order.end(), 0);
  std::stable_sort(c->order.begin(), c->order.end(), [&](int a, int b) {
    return (int64_t)patches[a].mx * patches[a].my > (int64_t)patches[b].mx * patches[b].my;
  });

  return WS_OK;
}

extern "C" {

int ws_init_patches(ws_ctx **out, const ws_patch_desc *patches, int32_t n_patches,
                    const ws_material *mats, int32_t n_instances, int32_t mbc, int32_t dtype,
                    int32_t limiter, void *q_pool_a, void *q_pool_b, int64_t pool_bytes,
                    void *workspace, int64_t ws_bytes, void *hip_stream) {
  if (!out) return fail(WS_EINVAL, "out is NULL");
  *out = nullptr;
  if (mbc != 2) return fail(WS_EINVAL, "mbc must be 2 (got %d)", mbc);
  if (int rc = check_level(patches, n_patches, mats, n_instances, dtype, limiter)) return rc;
  if (!q_pool_a || !q_pool_b || !workspace) return fail(WS_EINVAL, "pool or workspace is NULL");
  if (q_pool_a == q_pool_b) return fail(WS_EINVAL, "the two pools must differ");
  int64_t need_pool = 0, need_ws = 0;
  ws_layout(patches, n_patches, n_instances, dtype, &need_pool, &need_ws);
  if (pool_bytes < need_pool)
    return fail(WS_ENOMEM, "pool too small: %lld < %lld bytes", (long long)pool_bytes,
                (long long)need_pool);
  if (ws_bytes < need_ws)
    return fail(WS_ENOMEM, "workspace too small: %lld < %lld bytes", (long long)ws_bytes,
                (long long)need_ws);

  ws_ctx *c = new ws_ctx();
  auto bail = [&](int rc) {
    delete c;
    return rc;
  };
  if (int rc = setup_level(c, patches, n_patches, mats, n_instances, dtype, limiter, q_pool_a,
                           q_pool_b, pool_bytes, reinterpret_cast<char *>(workspace),
                           reinterpret_cast<hipStream_t>(hip_stream)))
    return bail(rc);
  const std::vector<InstRow> &inst = c->inst_host;
  c->host_buf_bytes = std::max<int64_t>(4096, 8LL * 3 * std::max(n_instances, n_patches));
  if (hipHostMalloc(reinterpret_cast<void **>(&c->host_buf), c->host_buf_bytes) != hipSuccess)
    return bail(fail(WS_EHIP, "hipHostMalloc of %lld bytes failed", (long long)c->host_buf_bytes));
  // clear the bookkeeping slots, then fill the tables
  if (hipMemsetAsync(c->ws + c->L.dt, 0, c->L.partials - c->L.dt, c->stream) != hipSuccess)
    return bail(fail(WS_EHIP, "clearing the workspace failed"));
  if (hipMemcpyAsync(c->ws + c->L.inst, inst.data(), inst.size() * sizeof(InstRow),
                     hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return bail(fail(WS_EHIP, "uploading the instance table failed"));
  if (int rc = c->build_tiles()) return bail(rc);
  *out = c;
  return WS_OK;
}

int ws_set_tiling(ws_ctx *c, const int32_t *variant, const int32_t *tile_w,
                  const int32_t *tile_h, int32_t wg_per_cu) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if ((tile_w == nullptr) != (tile_h == nullptr) || (variant != nullptr && tile_w == nullptr))
    return fail(WS_EINVAL, "give variant, tile_w and tile_h together, or none");
  if (wg_per_cu < 0 || wg_per_cu > 1024) return fail(WS_EINVAL, "wg_per_cu out of range");
  if (tile_w)
    for (int k = 0; k < c->n_patches; ++k) {
      const int v = variant ? variant[k] : kDirect;
      if (!valid_tile(v, tile_w[k], tile_h[k]))
        return fail(WS_EINVAL, "patch %d: invalid tile variant %d, %dx%d", k, v, tile_w[k],
                    tile_h[k]);
      if (v == kMarch && c->rows[k].bc == WS_BC_PERIODIC)
        return fail(WS_EINVAL, "patch %d: periodic patches take DIRECT tiles only", k);
      if (v == kMarch && !march_fits(c->rows[k].plane, c->dtype))
        return fail(WS_EINVAL, "patch %d: too large for MARCH tiles (32-bit offsets)", k);
      if (v == kPacked && c->rows[k].bc != WS_BC_NONE)
        return fail(WS_EINVAL, "patch %d: PACKED tiles take patches with frozen ghosts only", k);
      if (v == kPacked && c->medium)
        return fail(WS_EINVAL, "patch %d: a heterogeneous medium takes DIRECT or MARCH tiles", k);
      if (v == kPacked && c->P.elems * (c->dtype == WS_F32 ? 4 : 8) >= (int64_t{1} << 31))
        return fail(WS_EINVAL, "PACKED tiles need pools under 2 GiB (32-bit offsets)");
    }
  HIPCHK(hipStreamSynchronize(c->stream));
  if (tile_w)
    for (int k = 0; k < c->n_patches; ++k) {
      c->rows[k].variant = variant ? variant[k] : kDirect;
      c->rows[k].tw = tile_w[k];
      c->rows[k].th = tile_h[k];
    }
  c->wg_override = wg_per_cu;  // 0: the kernel's occupancy
  c->drop_graph();
  return c->build_tiles();
}

int ws_attach_medium(ws_ctx *c, void *medium, int64_t bytes) {
  if (!c || !medium) return fail(WS_EINVAL, "NULL argument");
  if (bytes < c->pool_bytes)
    return fail(WS_ENOMEM, "medium buffer too small (%lld < %lld bytes)", (long long)bytes,
                (long long)c->pool_bytes);
  if (c->limiter & WS_TRANSVERSE_CORR)
    return fail(WS_EINVAL, "a heterogeneous medium needs the default transverse variant");
  // the medium kernel addresses a patch's three planes with 32-bit offsets
  const int64_t es = c->dtype == WS_F32 ? 4 : 8;
  for (int k = 0; k < c->n_patches; ++k)
    if (3 * c->rows[k].plane * es >= ((int64_t)1 << 32))
      return fail(WS_EINVAL, "patch %d: its three planes span 4 GiB or more (too large for a "
                  "heterogeneous medium)", k);
  HIPCHK(hipStreamSynchronize(c->stream));
  c->medium = medium;
  // DIRECT tiles (the default DIRECT shape of each patch)
  for (int k = 0; k < c->n_patches; ++k) {
    PatchRow &r = c->rows[k];
    default_tile(r.mx, r.my, WS_BC_PERIODIC, c->n_cu, &r.variant, &r.tw, &r.th);
  }
  c->drop_graph();
  return c->build_tiles();
}

int ws_upload_medium(ws_ctx *c, int32_t patch, const double *rho, const double *K) {
  if (!c || !rho || !K) return fail(WS_EINVAL, "NULL argument");
  if (!c->medium) return fail(WS_ESTATE, "no medium attached");
  if (patch < 0 || patch >= c->n_patches) return fail(WS_EINVAL, "patch %d out of range", patch);
  const PatchRow &r = c->rows[patch];
  const size_t w = (size_t)r.mx + 4, h = (size_t)r.my + 4, n = w * h;
  const bool f32 = c->dtype == WS_F32;
  const size_t es = f32 ? 4 : 8;
  std::vector<char> host(3 * n * es);
  for (size_t x = 0; x < n; ++x) {
    if (!(rho[x] > 0.0) || !(K[x] > 0.0) || !std::isfinite(rho[x]) || !std::isfinite(K[x]))
      return fail(WS_EINVAL, "patch %d: rho and K must be finite and > 0 (cell %zu)", patch, x);
    const double cs = std::sqrt(K[x] / rho[x]), Z = rho[x] * cs;
    if (f32) {
      const float Zf = (float)Z;
      reinterpret_cast<float *>(host.data())[x] = (float)cs;
      reinterpret_cast<float *>(host.data())[n + x] = Zf;
      reinterpret_cast<float *>(host.data())[2 * n + x] = 1.0f / (Zf * Zf + 1.0f);
    } else {
      reinterpret_cast<double *>(host.data())[x] = cs;
      reinterpret_cast<double *>(host.data())[n + x] = Z;
      reinterpret_cast<double *>(host.data())[2 * n + x] = 1.0 / (Z * Z + 1.0);
    }
  }
  const int64_t first = r.q_off + r.col0 - 2;  // padded (i=-2, j=-2) of plane 0
  HIPCHK(hipMemcpy2DAsync(reinterpret_cast<char *>(c->medium) + first * es, r.ld * es,
                          host.data(), w * es, w * es, 3 * h, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return WS_OK;
}

int ws_link_layout(ws_ctx *c, int64_t *bytes) {
  if (!c || !bytes) return fail(WS_EINVAL, "NULL argument");
  int64_t ghosts = 0;
  for (const PatchRow &r : c->rows) ghosts += ring_size(r.mx, r.my);
  *bytes = round_up(8 * (int64_t)std::max(c->n_patches, 1), 256) + round_up(16 * ghosts, 256);
  return WS_OK;
}

int ws_link_level(ws_ctx *c, const int32_t *origins, int32_t domain_mx, int32_t domain_my,
                  int32_t periodic, void *buffer, int64_t bytes) {
  if (!c || !origins || !buffer) return fail(WS_EINVAL, "NULL argument");
  if (domain_mx < 1 || domain_my < 1 || c->n_patches < 1) return fail(WS_EINVAL, "empty domain");
  if (c->fine_in_couplings > 0)
    return fail(WS_EINVAL, "the level is the fine level of a coupling (its ghosts come from the "
                "coarse level)");
  if (periodic & ~3) return fail(WS_EINVAL, "periodic takes bits 0 (x) and 1 (y) only");
  int64_t need = 0;
  ws_link_layout(c, &need);
  if (bytes < need)
    return fail(WS_ENOMEM, "link buffer too small (%lld < %lld bytes)", (long long)bytes,
                (long long)need);
  const PatchRow &r0 = c->rows[0];
  for (int k = 0; k < c->n_patches; ++k) {
    const PatchRow &r = c->rows[k];
    if (r.bc != WS_BC_NONE)
      return fail(WS_EINVAL, "patch %d: a tiled level's ghosts come from the exchange (bc must "
                  "be WS_BC_NONE)", k);
    if (r.inst != r0.inst) return fail(WS_EINVAL, "patch %d: another instance than patch 0", k);
    if (!same_rel(r.dx, r0.dx) || !same_rel(r.dy, r0.dy))
      return fail(WS_EINVAL, "patch %d: another cell size than patch 0", k);
  }
  // the patch holding each domain cell; the patches must tile the domain
  const int64_t DX = domain_mx, DY = domain_my;
  std::vector<int32_t> own((size_t)(DX * DY), -1);
  for (int k = 0; k < c->n_patches; ++k) {
    const int64_t x0 = origins[2 * k], y0 = origins[2 * k + 1];
    const int mx = c->rows[k].mx, my = c->rows[k].my;
    if (x0 < 0 || y0 < 0 || x0 + mx > DX || y0 + my > DY)
      return fail(WS_EINVAL, "patch %d does not lie in the domain", k);
    for (int j = 0; j < my; ++j)
      for (int i = 0; i < mx; ++i) {
        int32_t &o = own[(size_t)((y0 + j) * DX + x0 + i)];
        if (o >= 0) return fail(WS_EINVAL, "patches %d and %d overlap", o, k);
        o = k;
      }
  }
  for (int64_t x = 0; x < DX * DY; ++x)
    if (own[(size_t)x] < 0) return fail(WS_EINVAL, "the patches do not cover the domain");
  // each ghost: mapped into the domain by the physical condition of its
  // direction (wrap or clamp), then the interior cell of the holding patch
  std::vector<int64_t> ring0(c->n_patches);
  std::vector<int64_t> src;
  for (int k = 0; k < c->n_patches; ++k) {
    const int mx = c->rows[k].mx, my = c->rows[k].my, n = ring_size(mx, my);
    ring0[k] = (int64_t)src.size() / 2;
    for (int g = 0; g < n; ++g) {
      int i, j;
      ring_cell(g, mx, my, i, j);
      int64_t gx = origins[2 * k] + i, gy = origins[2 * k + 1] + j;
      gx = (periodic & 1) ? ((gx % DX) + DX) % DX : std::min<int64_t>(std::max<int64_t>(gx, 0), DX - 1);
      gy = (periodic & 2) ? ((gy % DY) + DY) % DY : std::min<int64_t>(std::max<int64_t>(gy, 0), DY - 1);
      const int32_t o = own[(size_t)(gy * DX + gx)];
      const PatchRow &sr = c->rows[o];
      const int64_t si = gx - origins[2 * o], sj = gy - origins[2 * o + 1];
      src.push_back(sr.q_off + (sj + 2) * (int64_t)sr.ld + sr.col0 + si);
      src.push_back(sr.plane);
    }
  }
  char *b = static_cast<char *>(buffer);
  const int64_t off_src = round_up(8 * (int64_t)std::max(c->n_patches, 1), 256);
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpyAsync(b, ring0.data(), 8 * ring0.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(b + off_src, src.data(), 8 * src.size(), hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->link_ring0 = reinterpret_cast<const int64_t *>(b);
  c->link_src = reinterpret_cast<const int64_t *>(b + off_src);
  c->link_max_ring = 0;
  for (const PatchRow &r : c->rows) c->link_max_ring = std::max(c->link_max_ring, ring_size(r.mx, r.my));
  c->drop_graph();
  return WS_OK;
}

int ws_get_tiling(ws_ctx *c, int32_t *variant, int32_t *tile_w, int32_t *tile_h,
                  int32_t *wg_per_cu, int32_t *grid) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  for (int k = 0; k < c->n_patches; ++k) {
    if (variant) variant[k] = c->rows[k].variant;
    if (tile_w) tile_w[k] = c->rows[k].tw;
    if (tile_h) tile_h[k] = c->rows[k].th;
  }
  if (wg_per_cu) *wg_per_cu = c->wg_per_cu;
  if (grid) *grid = c->grid;
  return WS_OK;
}

static int copy_patch(ws_ctx *c, int32_t patch, const void *src, void *dst, bool up) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (patch < 0 || patch >= c->n_patches) return fail(WS_EINVAL, "patch %d out of range", patch);
  if (!(up ? src : dst)) return fail(WS_EINVAL, "buffer is NULL");
  const PatchRow &r = c->rows[patch];
  const size_t es = c->dtype == WS_F32 ? 4 : 8;
  const size_t w = (size_t)(r.mx + 4) * es;
  const size_t h = 3 * (size_t)(r.my + 4);
  const int64_t first = r.q_off + r.col0 - 2;  // padded (i=-2, j=-2) of plane p
  if (up) {
    for (int b = 0; b < 2; ++b)
      HIPCHK(hipMemcpy2DAsync(reinterpret_cast<char *>(c->pool[b]) + first * es, r.ld * es, src, w,
                              w, h, hipMemcpyDefault, c->stream));
  } else {
    const char *from = reinterpret_cast<const char *>(c->pool[c->cur]) + first * es;
    hipPointerAttribute_t attr{};
    const bool device = hipPointerGetAttributes(&attr, dst) == hipSuccess &&
                        attr.type == hipMemoryTypeDevice;
    (void)hipGetLastError();  // the query fails for pageable memory; that is not an error
    if (device) {
      HIPCHK(hipMemcpy2DAsync(dst, w, from, r.ld * es, w, h, hipMemcpyDeviceToDevice, c->stream));
    } else {
      // into host memory through the context's pinned buffer, a block of rows
      // at a time: each block is complete in pinned memory (the stream is
      // synchronised) before the host copies it on
      constexpr int64_t kStage = int64_t{8} << 20;
      if (!c->stage) {
        if (hipHostMalloc(reinterpret_cast<void **>(&c->stage), kStage) != hipSuccess)
          return fail(WS_EHIP, "hipHostMalloc of %lld bytes failed", (long long)kStage);
        c->stage_bytes = kStage;
      }
      const size_t rows = std::max<size_t>(1, (size_t)c->stage_bytes / w);
      for (size_t r0 = 0; r0 < h; r0 += rows) {
        const size_t n = std::min(rows, h - r0);
        HIPCHK(hipMemcpy2DAsync(c->stage, w, from + r0 * r.ld * es, r.ld * es, w, n,
                                hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        std::memcpy(static_cast<char *>(dst) + r0 * w, c->stage, n * w);
      }
      return WS_OK;
    }
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return WS_OK;
}

int ws_upload_patch(ws_ctx *c, int32_t patch, const void *src) {
  return copy_patch(c, patch, src, nullptr, true);
}

int ws_download_patch(ws_ctx *c, int32_t patch, void *dst) {
  return copy_patch(c, patch, nullptr, dst, false);
}

int ws_fill_ghosts(ws_ctx *c) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (c->link_src)
    HIPCHK(launch_link_ghosts(c->dtype, c->d_patches(), c->n_patches, c->link_max_ring,
                              c->link_ring0, c->link_src, c->pool[c->cur], c->stream));
  else
    HIPCHK(launch_fill_ghosts(c->dtype, c->d_patches(), c->n_patches, c->max_padded_cells,
                              c->pool[c->cur], c->stream));
  return WS_OK;
}

// After a step that wrote pool `dst`: a tiled level's ghosts from the
// neighbouring patches (the step itself writes the physical ghosts of
// periodic and extrapolating patches).
static int link_after_step(ws_ctx *c, int dst) {
  if (c->link_src)
    HIPCHK(launch_link_ghosts(c->dtype, c->d_patches(), c->n_patches, c->link_max_ring,
                              c->link_ring0, c->link_src, c->pool[dst], c->stream));
  return WS_OK;
}

static int read_level_cfl(ws_ctx *c, double *cfl_out) {
  if (!cfl_out) return WS_OK;
  HIPCHK(hipMemcpyAsync(c->host_buf, c->ws + c->L.level_last, 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *cfl_out = c->host_buf[0];
  return WS_OK;
}

int ws_step_level(ws_ctx *c, double dt, double *cfl_out) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(WS_EINVAL, "dt must be finite and > 0");
  // one persistent launch; its last workgroup also files the Courant numbers
  StepArgs a = c->step_args(c->cur, dt, 0.0);
  HIPCHK(launch_step(c->dtype, c->lim_code(), c->vars, a, c->grid, c->stream));
  if (int rc = link_after_step(c, 1 - c->cur)) return rc;
  c->cur = 1 - c->cur;
  return read_level_cfl(c, cfl_out);
}

int ws_step_level_per_patch(ws_ctx *c, double dt, double *cfl_out) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (c->vars & 4) return fail(WS_EINVAL, "per-patch launches need a tiling without PACKED tiles");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(WS_EINVAL, "dt must be finite and > 0");
  HIPCHK(launch_set_dt(c->slots(), dt, c->stream));
  StepArgs a = c->step_args(c->cur, 0.0, 0.0);
  a.persistent = 0;
  for (int k : c->order) {  // largest patch first
    a.tile_base = c->rows[k].tile_begin;
    HIPCHK(launch_step(c->dtype, c->lim_code(), c->vars, a, c->rows[k].n_tiles, c->stream));
  }
  HIPCHK(launch_finish_step(c->slots(), 0.0, c->stream));
  if (int rc = link_after_step(c, 1 - c->cur)) return rc;
  c->cur = 1 - c->cur;
  return read_level_cfl(c, cfl_out);
}

int ws_set_dt(ws_ctx *c, const double *dt_per_instance) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (!dt_per_instance) return fail(WS_EINVAL, "dt is NULL");
  for (int k = 0; k < c->n_inst; ++k)
    if (!(dt_per_instance[k] > 0.0) || !std::isfinite(dt_per_instance[k]))
      return fail(WS_EINVAL, "dt[%d] must be finite and > 0", k);
  HIPCHK(hipStreamSynchronize(c->stream));
  std::memcpy(c->host_buf, dt_per_instance, 8 * (size_t)c->n_inst);
  HIPCHK(hipMemcpyAsync(c->ws + c->L.dt, c->host_buf, 8 * (size_t)c->n_inst,
                        hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemsetAsync(c->ws + c->L.cfl_max, 0, 8 * (size_t)c->n_inst, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return WS_OK;
}

static int enqueue_auto(ws_ctx *c, int src, double cfl_desired) {
  StepArgs a = c->step_args(src, 0.0, cfl_desired);
  HIPCHK(launch_step(c->dtype, c->lim_code(), c->vars, a, c->grid, c->stream));
  return link_after_step(c, 1 - src);
}

int ws_step_auto(ws_ctx *c, double cfl_desired) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (!(cfl_desired > 0.0) || !std::isfinite(cfl_desired))
    return fail(WS_EINVAL, "cfl_desired must be finite and > 0");
  if (int rc = enqueue_auto(c, c->cur, cfl_desired)) return rc;
  c->cur = 1 - c->cur;
  return WS_OK;
}

int ws_capture_steps(ws_ctx *c, int32_t n_steps, double cfl_desired) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (n_steps < 1) return fail(WS_EINVAL, "n_steps must be >= 1");
  if (!(cfl_desired > 0.0) || !std::isfinite(cfl_desired))
    return fail(WS_EINVAL, "cfl_desired must be finite and > 0");
  c->drop_graph();
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int rc = WS_OK;
  for (int s = 0; s < n_steps && rc == WS_OK; ++s) rc = enqueue_auto(c, (c->cur + s) & 1, cfl_desired);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (rc != WS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(WS_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  c->graph = g;
  HIPCHK(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  c->graph_steps = n_steps;
  c->graph_start_pool = c->cur;
  return WS_OK;
}

int ws_graph_launch(ws_ctx *c) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (!c->gexec) return fail(WS_ESTATE, "no captured graph");
  if (c->cur != c->graph_start_pool)
    return fail(WS_ESTATE, "the state is in the other pool than at capture time; capture again");
  HIPCHK(hipGraphLaunch(c->gexec, c->stream));
  c->cur = (c->cur + c->graph_steps) & 1;
  return WS_OK;
}

int ws_read_dt_cfl(ws_ctx *c, double *dt, double *cfl_last, double *cfl_max) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  const size_t n = 8 * (size_t)c->n_inst;
  double *h = c->host_buf;
  HIPCHK(hipMemcpyAsync(h, c->ws + c->L.dt, n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(h + c->n_inst, c->ws + c->L.cfl_last, n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(h + 2 * c->n_inst, c->ws + c->L.cfl_max, n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (dt) std::memcpy(dt, h, n);
  if (cfl_last) std::memcpy(cfl_last, h + c->n_inst, n);
  if (cfl_max) std::memcpy(cfl_max, h + 2 * c->n_inst, n);
  return WS_OK;
}

int ws_read_patch_cfl(ws_ctx *c, double *cfl) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (!cfl) return fail(WS_EINVAL, "cfl is NULL");
  double *dpatch = reinterpret_cast<double *>(c->ws + c->L.cfl_patch_last);
  HIPCHK(launch_patch_cfl(c->d_patches(), c->n_patches, c->slots().cfl_tile, dpatch, c->stream));
  const size_t n = 8 * (size_t)c->n_patches;
  HIPCHK(hipMemcpyAsync(c->host_buf, dpatch, n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::memcpy(cfl, c->host_buf, n);
  return WS_OK;
}

int ws_conservation_sums(ws_ctx *c, double *sums) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (!sums) return fail(WS_EINVAL, "sums is NULL");
  double *partials = reinterpret_cast<double *>(c->ws + c->L.partials);
  double *dsums = reinterpret_cast<double *>(c->ws + c->L.sums);
  double *psums = reinterpret_cast<double *>(c->ws + c->L.patch_sums);
  HIPCHK(launch_sums(c->dtype, c->d_patches(), c->n_patches,
                     reinterpret_cast<const TileEntry *>(c->ws + c->L.stiles),
                     (int)c->stiles.size(), c->pool[c->cur], partials, psums, c->n_inst, dsums,
                     c->stream));
  const size_t n = 24 * (size_t)c->n_inst;
  HIPCHK(hipMemcpyAsync(c->host_buf, dsums, n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::memcpy(sums, c->host_buf, n);
  return WS_OK;
}

int ws_time_step_kernel(ws_ctx *c, int32_t n_launches, int32_t per_patch, double *ms_per_step) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (n_launches < 1 || n_launches > 100000 || !ms_per_step)
    return fail(WS_EINVAL, "need 1 <= n_launches <= 100000 and an output");
  if (per_patch && (c->vars & 4))
    return fail(WS_EINVAL, "per-patch launches need a tiling without PACKED tiles");
  // one event pair per level step: the mean bracketed duration, without the
  // gaps between back-to-back launches
  std::vector<hipEvent_t> ev(2 * (size_t)n_launches, nullptr);
  hipError_t e = hipSuccess;
  size_t made = 0;
  for (; made < ev.size() && e == hipSuccess; ++made) e = hipEventCreate(&ev[made]);
  if (e != hipSuccess) --made;
  for (int s = 0; s < n_launches && e == hipSuccess; ++s) {
    e = hipEventRecord(ev[2 * s], c->stream);
    StepArgs a = c->step_args(c->cur, 0.0, 0.0);
    if (e == hipSuccess && per_patch) {
      a.persistent = 0;
      for (int k : c->order) {
        a.tile_base = c->rows[k].tile_begin;
        e = launch_step(c->dtype, c->lim_code(), c->vars, a, c->rows[k].n_tiles, c->stream);
        if (e != hipSuccess) break;
      }
      // per-patch launches leave their Courant numbers in the accumulators
      if (e == hipSuccess) e = launch_finish_step(c->slots(), 0.0, c->stream);
    } else if (e == hipSuccess) {
      e = launch_step(c->dtype, c->lim_code(), c->vars, a, c->grid, c->stream);
    }
    // the state moved to the other pool only if every launch of the step went in
    if (e == hipSuccess) c->cur = 1 - c->cur;
    if (e == hipSuccess) e = hipEventRecord(ev[2 * s + 1], c->stream);
  }
  if (e == hipSuccess) e = hipEventSynchronize(ev[2 * (size_t)n_launches - 1]);
  double total = 0.0;
  for (int s = 0; s < n_launches && e == hipSuccess; ++s) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ev[2 * s], ev[2 * s + 1]);
    total += ms;
  }
  int rc = WS_OK;
  if (e != hipSuccess) rc = fail(WS_EHIP, "timing loop: %s", hipGetErrorString(e));
  else *ms_per_step = total / n_launches;
  for (size_t k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
  return rc;
}

int ws_mask_bytes(ws_ctx *c, int64_t *bytes) {
  if (!c || !bytes) return fail(WS_EINVAL, "NULL argument");
  *bytes = c->mask_total;
  return WS_OK;
}

int ws_patch_layout(ws_ctx *c, int32_t patch, int64_t *offset, int64_t *ld, int64_t *plane) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (patch < 0 || patch >= c->n_patches) return fail(WS_EINVAL, "patch %d out of range", patch);
  const PatchRow &r = c->rows[patch];
  if (offset) *offset = r.q_off + r.col0 - 2;
  if (ld) *ld = r.ld;
  if (plane) *plane = r.plane;
  return WS_OK;
}

int ws_step_record_masks(ws_ctx *c, double dt, void *masks_dev, double *cfl_out) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (!masks_dev) return fail(WS_EINVAL, "masks buffer is NULL");
  if (c->limiter != WS_LIM_MC || c->medium)
    return fail(WS_EINVAL,
                "branches exist for the MC limiter of the default variant in a homogeneous medium");
  if (c->link_src)
    return fail(WS_EINVAL, "branch recording (for the adjoint) does not take a tiled level");
  if (c->vars & 4) return fail(WS_EINVAL, "branch recording needs a tiling without PACKED tiles");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(WS_EINVAL, "dt must be finite and > 0");
  StepArgs a = c->step_args(c->cur, dt, 0.0);
  a.masks = reinterpret_cast<uint8_t *>(masks_dev);
  HIPCHK(launch_step(c->dtype, c->lim_code(), c->vars, a, c->grid, c->stream));
  c->cur = 1 - c->cur;
  return read_level_cfl(c, cfl_out);
}

static int check_adjoint_ctx(ws_ctx *c) {
  if (!c) return fail(WS_EINVAL, "ctx is NULL");
  if (c->dtype != WS_F64) return fail(WS_EINVAL, "the adjoint needs an FP64 context");
  return WS_OK;
}

int ws_adjoint_step(ws_ctx *c, double dt, const void *masks_dev, const void *lam_in,
                    void *lam_out) {
  if (int rc = check_adjoint_ctx(c)) return rc;
  if (c->limiter != WS_LIM_MC || c->medium)
    return fail(WS_EINVAL,
                "the adjoint needs the MC limiter of the default variant in a homogeneous medium");
  if (c->link_src) return fail(WS_EINVAL, "the adjoint does not take a tiled level");
  if (!masks_dev || !lam_in || !lam_out) return fail(WS_EINVAL, "NULL buffer");
  if (lam_in == lam_out) return fail(WS_EINVAL, "lam_in and lam_out must be distinct buffers");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(WS_EINVAL, "dt must be finite and > 0");
  for (int k = 0; k < c->n_patches; ++k)
    if (c->rows[k].bc == WS_BC_PERIODIC)
      return fail(WS_EINVAL, "patch %d: the adjoint does not take periodic patches", k);
  for (int k = 0; k < c->n_patches; ++k)
    if (!march_fits(c->rows[k].plane, WS_F64))
      return fail(WS_EINVAL, "patch %d: too large for the adjoint (32-bit offsets)", k);
  HIPCHK(launch_adjoint(c->d_patches(), c->n_patches, c->max_mx, c->max_my, c->n_cu,
                        reinterpret_cast<const InstRow *>(c->ws + c->L.inst), dt,
                        reinterpret_cast<const uint8_t *>(masks_dev),
                        reinterpret_cast<const double *>(lam_in),
                        reinterpret_cast<double *>(lam_out), c->stream));
  return WS_OK;
}

static int check_cells(ws_ctx *c, int32_t patch, int32_t comp, int32_t n, const void *ij,
                       const void *vals) {
  if (int rc = check_adjoint_ctx(c)) return rc;
  if (patch < 0 || patch >= c->n_patches) return fail(WS_EINVAL, "patch %d out of range", patch);
  if (comp < 0 || comp > 2) return fail(WS_EINVAL, "component %d out of range", comp);
  if (n < 0) return fail(WS_EINVAL, "n must be >= 0");
  if (n > 0 && (!ij || !vals)) return fail(WS_EINVAL, "NULL buffer");
  return WS_OK;
}

int ws_gather(ws_ctx *c, const void *buf, int32_t patch, int32_t comp, int32_t n,
              const int32_t *ij, double *out) {
  if (int rc = check_cells(c, patch, comp, n, ij, out)) return rc;
  const void *src = buf ? buf : c->pool[c->cur];
  HIPCHK(launch_gather(c->d_patches(), patch, comp, n, ij, reinterpret_cast<const double *>(src),
                       out, c->stream));
  return WS_OK;
}

int ws_add_at(ws_ctx *c, void *buf, int32_t patch, int32_t comp, int32_t n, const int32_t *ij,
              const double *val) {
  if (int rc = check_cells(c, patch, comp, n, ij, val)) return rc;
  void *dst = buf ? buf : c->pool[c->cur];
  HIPCHK(launch_add_at(c->d_patches(), patch, comp, n, ij, val, reinterpret_cast<double *>(dst),
                       c->stream));
  return WS_OK;
}

int ws_current_pool(ws_ctx *c, int32_t *which) {
  if (!c || !which) return fail(WS_EINVAL, "NULL argument");
  *which = c->cur;
  return WS_OK;
}

// --------------------------------------------------------------------------
// Level step without allocation: the workspace lives in a file-scope device
// array of the library instead of caller memory.
// --------------------------------------------------------------------------
}  // extern "C"

namespace {
constexpr int64_t kScratchBytes = int64_t{8} << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch[kMaxDevices] = {};
}  // namespace

// Patch table, tile list and Courant-number slots of ws_step_level_noalloc.
// In host code the name is only a stand-in for the symbol: the device
// address of each GPU's copy comes from hipGetSymbolAddress.
static __device__ __align__(256) char scratch[kScratchBytes];

// The current device's copy of `scratch`, looked up once per device.
static int scratch_on_device(char **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(WS_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(WS_EHIP, "hipGetSymbolAddress returned NULL");
    g_scratch[dev] = static_cast<char *>(p);
  }
  *out = g_scratch[dev];
  return WS_OK;
}

extern "C" {

int64_t ws_noalloc_scratch_bytes(void) { return kScratchBytes; }

int ws_step_level_noalloc(const ws_patch_desc *patches, int32_t n_patches,
                          const ws_material *mats, int32_t n_instances, int32_t dtype,
                          int32_t limiter, const void *q_in, void *q_out, int64_t pool_bytes,
                          double dt, double *cfl_out, void *hip_stream) {
  if (int rc = check_level(patches, n_patches, mats, n_instances, dtype, limiter)) return rc;
  if (!q_in || !q_out) return fail(WS_EINVAL, "q_in or q_out is NULL");
  if (q_in == q_out) return fail(WS_EINVAL, "q_in and q_out must differ");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(WS_EINVAL, "dt must be finite and > 0");
  int64_t need_pool = 0, need_ws = 0;
  ws_layout(patches, n_patches, n_instances, dtype, &need_pool, &need_ws);
  if (pool_bytes < need_pool)
    return fail(WS_ENOMEM, "pool too small: %lld < %lld bytes", (long long)pool_bytes,
                (long long)need_pool);
  if (need_ws > kScratchBytes)
    return fail(WS_ENOMEM, "the level needs %lld bytes of workspace; the no-allocation step "
                "holds %lld (use ws_init_patches with a workspace)", (long long)need_ws,
                (long long)kScratchBytes);
  char *ws = nullptr;
  if (int rc = scratch_on_device(&ws)) return rc;
  ws_ctx c;  // host metadata only; no pinned buffer, no graph
  if (int rc = setup_level(&c, patches, n_patches, mats, n_instances, dtype, limiter,
                           const_cast<void *>(q_in), q_out, pool_bytes, ws,
                           reinterpret_cast<hipStream_t>(hip_stream)))
    return rc;
  // the scratch keeps the previous call's contents: clear the slots that
  // must start at zero (accumulators, retirement counters), then the tables
  HIPCHK(hipMemsetAsync(ws + c.L.dt, 0, c.L.partials - c.L.dt, c.stream));
  HIPCHK(hipMemcpyAsync(ws + c.L.inst, c.inst_host.data(), c.inst_host.size() * sizeof(InstRow),
                        hipMemcpyHostToDevice, c.stream));
  if (int rc = c.build_tiles()) return rc;  // uploads the tables, synchronises
  StepArgs a = c.step_args(0, dt, 0.0);
  HIPCHK(launch_step(c.dtype, c.lim_code(), c.vars, a, c.grid, c.stream));
  double cfl = 0.0;
  HIPCHK(hipMemcpyAsync(&cfl, ws + c.L.level_last, 8, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  if (cfl_out) *cfl_out = cfl;
  return WS_OK;
}

int ws_destroy(ws_ctx *c) {
  if (!c) return WS_OK;
  (void)hipStreamSynchronize(c->stream);
  c->drop_graph();
  if (c->host_buf) (void)hipHostFree(c->host_buf);
  if (c->stage) (void)hipHostFree(c->stage);
  delete c;
  return WS_OK;
}

}  // extern "C"

// --------------------------------------------------------------------------
// Coarse-fine coupling: one composite coarse step of two levels
// --------------------------------------------------------------------------

struct ws_cf {
  ws_ctx *coarse = nullptr, *fine = nullptr;
  ws_cf *inner = nullptr;  // coupling of the fine level with the next finer one
  int r = 1;
  char *ws = nullptr;
  int64_t off_place = 0, off_acc = 0, off_pc = 0, off_copy = 0, off_fix = 0;
  int n_fine = 0, n_fix = 0;
  int max_ring = 0;
  int max_step_blocks = 0, max_finish_blocks = 0;  // blocks per fine patch of the two launches
  int strip = 64;        // edges (threads) per block of the fine-step launch
  int64_t n_fedges = 0;  // fine boundary edges of all patches

  CfArgs args() const {
    CfArgs a{};
    a.cpatch = coarse->d_patches();
    a.fpatch = fine->d_patches();
    a.cinst = reinterpret_cast<const InstRow *>(coarse->ws + coarse->L.inst);
    a.finst = reinterpret_cast<const InstRow *>(fine->ws + fine->L.inst);
    a.place = reinterpret_cast<const CfPlace *>(ws + off_place);
    a.n_fine = n_fine;
    a.r = r;
    a.acc = reinterpret_cast<double *>(ws + off_acc);
    a.pc = reinterpret_cast<double *>(ws + off_pc);
    a.copy = reinterpret_cast<const CfCopy *>(ws + off_copy);
    a.fix = reinterpret_cast<const CfFix *>(ws + off_fix);
    a.n_fix = n_fix;
    a.strip = strip;
    a.n_fedges = n_fedges;
    return a;
  }
};

namespace {

struct CfSizes {
  int64_t place, acc, pc, copy, fix, total;
  int64_t n_fedges, n_cedges, max_copies;
};

// The copy list's bound: a sibling whose interior meets a fine patch's ghost
// ring covers a coarse cell of the ring of coarse cells (width 2) around the
// patch, and siblings do not overlap, so there are at most 4 (ncx + ncy) + 16
// of them (and at most n_fine - 1).  The fix list has at most one cell per
// coarse interface edge.
CfSizes cf_sizes(const ws_ctx *fine, int r) {
  CfSizes z{};
  for (const ws_patch_desc &d : fine->desc) {
    const int64_t ncx = d.mx / r, ncy = d.my / r;
    z.n_fedges += 2 * ((int64_t)d.mx + d.my);
    z.n_cedges += 2 * (ncx + ncy);
    z.max_copies += std::min<int64_t>(fine->n_patches - 1, 4 * (ncx + ncy) + 16);
  }
  z.place = 0;
  z.acc = round_up((int64_t)fine->n_patches * (int64_t)sizeof(CfPlace), 256);
  z.pc = z.acc + round_up(24 * (int64_t)std::max(r, 1) * std::max<int64_t>(z.n_fedges, 1), 256);
  z.copy = z.pc + round_up(24 * std::max<int64_t>(z.n_cedges, 1), 256);
  z.fix = z.copy + round_up((int64_t)sizeof(CfCopy) * std::max<int64_t>(z.max_copies, 1), 256);
  z.total = z.fix + round_up((int64_t)sizeof(CfFix) * std::max<int64_t>(z.n_cedges, 1), 256);
  return z;
}

}  // namespace

extern "C" {

int ws_cf_layout(ws_ctx *fine, int32_t ratio, int64_t *bytes) {
  if (!fine || !bytes) return fail(WS_EINVAL, "NULL argument");
  if (ratio < 1) return fail(WS_EINVAL, "refinement ratio must be >= 1");
  *bytes = cf_sizes(fine, ratio).total;
  return WS_OK;
}

int ws_cf_init(ws_cf **out, ws_ctx *coarse, ws_ctx *fine, int32_t ratio,
               const ws_fine_place *places, void *workspace, int64_t ws_bytes) {
  if (!out) return fail(WS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!coarse || !fine || !places || !workspace) return fail(WS_EINVAL, "NULL argument");
  if (coarse == fine) return fail(WS_EINVAL, "the two levels must be different contexts");
  if (ratio < 1) return fail(WS_EINVAL, "refinement ratio must be >= 1");
  if (coarse->dtype != fine->dtype) return fail(WS_EINVAL, "the levels' dtypes differ");
  if (coarse->limiter != fine->limiter) return fail(WS_EINVAL, "the levels' limiters differ");
  if (coarse->limiter & WS_TRANSVERSE_CORR)
    return fail(WS_EINVAL, "the coarse-fine coupling needs the default transverse variant");
  if (coarse->stream != fine->stream) return fail(WS_EINVAL, "the levels must share one stream");
  if (coarse->medium || fine->medium)
    return fail(WS_EINVAL, "the coarse-fine coupling needs homogeneous media");
  if (fine->link_src)
    return fail(WS_EINVAL, "the fine level's ghosts come from the coarse level (it is tiled)");
  const CfSizes z = cf_sizes(fine, ratio);
  if (ws_bytes < z.total)
    return fail(WS_ENOMEM, "coupling workspace too small (%lld < %lld bytes)", (long long)ws_bytes,
                (long long)z.total);
  std::vector<CfPlace> pl(fine->n_patches);
  int64_t fe = 0, ce = 0;
  for (int k = 0; k < fine->n_patches; ++k) {
    const ws_patch_desc &d = fine->desc[k];
    const ws_fine_place &p = places[k];
    if (p.coarse_patch < 0 || p.coarse_patch >= coarse->n_patches)
      return fail(WS_EINVAL, "fine patch %d: coarse patch %d out of range", k, p.coarse_patch);
    const ws_patch_desc &cd = coarse->desc[p.coarse_patch];
    if (d.bc != WS_BC_NONE)
      return fail(WS_EINVAL, "fine patch %d: its ghosts come from the coarse level (bc must be "
                  "WS_BC_NONE)", k);
    if (d.mx % ratio || d.my % ratio)
      return fail(WS_EINVAL, "fine patch %d: %d x %d cells is not a whole number of coarse cells",
                  k, d.mx, d.my);
    if (!same_rel(d.dx * ratio, cd.dx) || !same_rel(d.dy * ratio, cd.dy))
      return fail(WS_EINVAL, "fine patch %d: cell size times the ratio differs from the coarse", k);
    const InstRow &fi = fine->inst_host[d.instance], &ci = coarse->inst_host[cd.instance];
    if (fi.c != ci.c || fi.Z != ci.Z)
      return fail(WS_EINVAL, "fine patch %d: material differs from its coarse patch's", k);
    const int ncx = d.mx / ratio, ncy = d.my / ratio;
    if (p.ci0 < 2 || p.cj0 < 2 || p.ci0 + ncx > cd.mx - 2 || p.cj0 + ncy > cd.my - 2)
      return fail(WS_EINVAL, "fine patch %d must lie at least 2 coarse cells inside its coarse "
                  "patch", k);
    for (int o = 0; o < k; ++o) {
      const ws_fine_place &q = places[o];
      if (q.coarse_patch != p.coarse_patch) continue;
      const int oncx = fine->desc[o].mx / ratio, oncy = fine->desc[o].my / ratio;
      const int gx = std::max(q.ci0 - (p.ci0 + ncx), p.ci0 - (q.ci0 + oncx));
      const int gy = std::max(q.cj0 - (p.cj0 + ncy), p.cj0 - (q.cj0 + oncy));
      if (std::max(gx, gy) < 0)
        return fail(WS_EINVAL, "fine patches %d and %d overlap", o, k);
    }
    pl[k] = CfPlace{p.coarse_patch, p.ci0, p.cj0, ncx, ncy, (int32_t)fe, (int32_t)ce, 0, 0, 0};
    fe += 2 * ((int64_t)d.mx + d.my);
    ce += 2 * ((int64_t)ncx + ncy);
  }
  if (fe > INT32_MAX || ce > INT32_MAX) return fail(WS_EINVAL, "too many boundary edges");
  // sibling copy rectangles: the part of each sibling's interior inside the
  // patch's ghost ring, in the patch's fine coordinates
  std::vector<CfCopy> copies;
  for (int k = 0; k < fine->n_patches; ++k) {
    pl[k].copy0 = (int32_t)copies.size();
    const int mx = fine->desc[k].mx, my = fine->desc[k].my;
    for (int o = 0; o < fine->n_patches; ++o) {
      if (o == k || pl[o].coarse != pl[k].coarse) continue;
      const int di = ratio * (pl[k].ci0 - pl[o].ci0), dj = ratio * (pl[k].cj0 - pl[o].cj0);
      // sibling o's interior in k's coordinates: [-di, -di + mx_o) x [-dj, -dj + my_o)
      const int i0 = std::max(-2, -di), i1 = std::min(mx + 2, -di + fine->desc[o].mx);
      const int j0 = std::max(-2, -dj), j1 = std::min(my + 2, -dj + fine->desc[o].my);
      if (i0 < i1 && j0 < j1) copies.push_back(CfCopy{o, i0, i1, j0, j1, di, dj, 0});
    }
    pl[k].ncopy = (int32_t)copies.size() - pl[k].copy0;
  }
  if ((int64_t)copies.size() > z.max_copies)
    return fail(WS_EINVAL, "internal: %zu sibling copies exceed the bound %lld", copies.size(),
                (long long)z.max_copies);
  // the fix list: every coarse cell outside the fine patches that borders one,
  // with its (patch, interface edge) pairs in patch order
  std::vector<CfFix> fixes;
  {
    std::map<std::tuple<int, int, int>, int> at;  // (coarse patch, oi, oj) -> fix index
    std::map<int, std::vector<char>> cover;       // coarse patch -> covered cells
    for (int k = 0; k < fine->n_patches; ++k) {
      const ws_patch_desc &cd = coarse->desc[pl[k].coarse];
      std::vector<char> &cv = cover[pl[k].coarse];
      if (cv.empty()) cv.assign((size_t)cd.mx * cd.my, 0);
      for (int J = 0; J < pl[k].ncy; ++J)
        for (int I = 0; I < pl[k].ncx; ++I)
          cv[(size_t)(pl[k].cj0 + J) * cd.mx + pl[k].ci0 + I] = 1;
    }
    for (int k = 0; k < fine->n_patches; ++k) {
      const int mxc = coarse->desc[pl[k].coarse].mx;
      const std::vector<char> &cv = cover[pl[k].coarse];
      for (int e = 0; e < 2 * (pl[k].ncx + pl[k].ncy); ++e) {
        int oi, oj;
        cf_out_cell_host(pl[k], e, oi, oj);
        if (cv[(size_t)oj * mxc + oi]) continue;  // covered by a sibling: updating sets it
        auto key = std::make_tuple(pl[k].coarse, oi, oj);
        auto it = at.find(key);
        if (it == at.end()) {
          it = at.emplace(key, (int)fixes.size()).first;
          CfFix f{};
          f.coarse = pl[k].coarse, f.oi = oi, f.oj = oj, f.n = 0;
          fixes.push_back(f);
        }
        CfFix &f = fixes[it->second];
        if (f.n >= 4) return fail(WS_EINVAL, "internal: a coarse cell borders over 4 patches");
        f.patch[f.n] = k, f.edge[f.n] = e, ++f.n;
      }
    }
  }
  ws_cf *cf = new ws_cf;
  cf->coarse = coarse;
  cf->fine = fine;
  cf->r = ratio;
  cf->ws = static_cast<char *>(workspace);
  cf->off_place = z.place;
  cf->off_acc = z.acc;
  cf->off_pc = z.pc;
  cf->off_copy = z.copy;
  cf->off_fix = z.fix;
  cf->n_fine = fine->n_patches;
  cf->n_fix = (int)fixes.size();
  int max_side = 1;
  for (const ws_patch_desc &d : fine->desc) max_side = std::max(max_side, std::max(d.mx, d.my));
  cf->strip = cf_strip_host(max_side);
  cf->n_fedges = z.n_fedges;
  for (int k = 0; k < fine->n_patches; ++k) {
    const ws_patch_desc &d = fine->desc[k];
    cf->max_ring = std::max(cf->max_ring, 4 * (d.mx + 4) + 4 * d.my);
    cf->max_step_blocks = std::max(
        cf->max_step_blocks, cf_step_blocks_host(d.mx, d.my, pl[k].ncx, pl[k].ncy, true, cf->strip));
    cf->max_finish_blocks =
        std::max(cf->max_finish_blocks, cf_finish_blocks_host(pl[k].ncx, pl[k].ncy));
  }
  if (hipMemcpyAsync(cf->ws + cf->off_place, pl.data(), pl.size() * sizeof(CfPlace),
                     hipMemcpyHostToDevice, coarse->stream) != hipSuccess ||
      (!copies.empty() &&
       hipMemcpyAsync(cf->ws + cf->off_copy, copies.data(), copies.size() * sizeof(CfCopy),
                      hipMemcpyHostToDevice, coarse->stream) != hipSuccess) ||
      (!fixes.empty() &&
       hipMemcpyAsync(cf->ws + cf->off_fix, fixes.data(), fixes.size() * sizeof(CfFix),
                      hipMemcpyHostToDevice, coarse->stream) != hipSuccess) ||
      hipStreamSynchronize(coarse->stream) != hipSuccess) {
    delete cf;
    return fail(WS_EHIP, "cannot upload the placement table");
  }
  ++fine->fine_in_couplings;
  *out = cf;
  return WS_OK;
}

int ws_cf_fill_fine_ghosts(ws_cf *cf, double alpha) {
  if (!cf) return fail(WS_EINVAL, "coupling is NULL");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(WS_EINVAL, "alpha must lie in [0, 1]");
  ws_ctx *c = cf->coarse, *f = cf->fine;
  CfArgs a = cf->args();
  a.c_old = c->pool[1 - c->cur];
  a.c_new = c->pool[c->cur];
  a.f_cur = f->pool[f->cur];
  HIPCHK(launch_cf_ghosts(c->dtype, a, alpha, cf->max_ring, c->stream));
  return WS_OK;
}

int ws_cf_step(ws_cf *cf, double dt) {
  if (!cf) return fail(WS_EINVAL, "coupling is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(WS_EINVAL, "dt must be finite and > 0");
  ws_ctx *c = cf->coarse, *f = cf->fine;
  const int r = cf->r;
  const double dtf = dt / r;
  CfArgs a = cf->args();
  // the coarse step; Q_c^n stays in the pool it read
  {
    StepArgs s = c->step_args(c->cur, dt, 0.0);
    HIPCHK(launch_step(c->dtype, c->lim_code(), c->vars, s, c->grid, c->stream));
    c->cur = 1 - c->cur;
  }
  a.c_old = c->pool[1 - c->cur];
  a.c_new = c->pool[c->cur];
  // r fine steps, each after its ghost ring and boundary terms (the first
  // launch also takes the coarse interface terms from Q_c^n)
  for (int k = 0; k < r; ++k) {
    a.f_cur = f->pool[f->cur];
    HIPCHK(launch_cf_fine_step(c->dtype, c->limiter, a, k, dtf, dt, cf->max_step_blocks,
                               c->stream));
    if (cf->inner) {
      // the fine level's own composite step (its step, its finer levels,
      // their updating and fix)
      if (int rc = ws_cf_step(cf->inner, dtf)) return rc;
    } else {
      StepArgs s = f->step_args(f->cur, dtf, 0.0);
      HIPCHK(launch_step(f->dtype, f->lim_code(), f->vars, s, f->grid, f->stream));
      f->cur = 1 - f->cur;
    }
  }
  // updating and the conservation fix, then the coarse physical ghosts
  a.f_cur = f->pool[f->cur];
  HIPCHK(launch_cf_finish(c->dtype, a, dt, cf->max_finish_blocks, c->stream));
  return ws_fill_ghosts(c);
}

int ws_cf_nest(ws_cf *outer, ws_cf *inner) {
  if (!outer) return fail(WS_EINVAL, "coupling is NULL");
  if (!inner) {
    outer->inner = nullptr;
    return WS_OK;
  }
  if (inner->coarse != outer->fine)
    return fail(WS_EINVAL, "the inner coupling's coarse level must be the outer one's fine level");
  for (ws_cf *c = inner; c; c = c->inner)
    if (c == outer) return fail(WS_EINVAL, "nesting would form a cycle");
  outer->inner = inner;
  return WS_OK;
}

int ws_cf_destroy(ws_cf *cf) {
  if (!cf) return WS_OK;
  (void)hipStreamSynchronize(cf->coarse->stream);
  --cf->fine->fine_in_couplings;
  delete cf;
  return WS_OK;
}

}  // extern "C"
