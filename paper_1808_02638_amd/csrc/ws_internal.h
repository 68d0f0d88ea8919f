// Internal layout shared by the host runtime and the HIP kernels of the
// wave-propagation library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ws_tables.h"

namespace ws {

// Per-step Courant-number bookkeeping inside the workspace.
struct CflSlots {
  double *dt;                    // [n_inst]
  double *cfl_tile;              // [n_tiles] Courant number of each tile of the step
  unsigned long long *inst_acc;  // [kGroups][n_inst] per-XCD-group maxima (FP64 bits)
  double *cfl_last;              // [n_inst]  Courant number of the last step
  double *cfl_max;               // [n_inst]  largest since ws_set_dt
  double *level_last;            // [1]
  int n_inst;
};

struct StepArgs {
  const PatchRow *patches;
  const TileEntry *tiles;
  const PackWave *packs;  // wavefronts of PACKED tiles
  int32_t n_tiles;
  int32_t tile_base;   // direct mode: first tile of this launch
  int32_t persistent;  // 1: persistent launch over all tiles; 0: tile = base + blockIdx
  const void *qin;
  void *qout;
  int32_t pool_bytes;  // bytes of each pool (PACKED tiles: below 2^31)
  const InstRow *inst;
  double *dt;          // per instance
  double dt_override;  // > 0: every instance steps with this dt (stored into dt)
  double cfl_desired;  // > 0: after the step, dt <- dt * cfl_desired / cfl
  CflSlots slots;
  unsigned int *retire;  // (kGroups + 1) counters, kLine apart
  uint8_t *masks;        // nullptr unless the branches are recorded
  const void *medium;    // nullptr, or per-cell (c, Z) planes laid out like a q pool
};

// Bit OR-ed into the limiter code of the kernel launchers when the level has a
// heterogeneous medium (DIRECT tiles only).
constexpr int kMediumFlag = 0x10000;

// Kernel launchers (defined in ws_kernels.hip).
// vars: bit 0 -> DIRECT tiles present, bit 1 -> MARCH tiles present, bit 2 ->
// PACKED tiles present.
hipError_t launch_step(int dtype, int limiter, int vars, const StepArgs &a, int grid,
                       hipStream_t s);
// The ghost ring of an mx x my patch in one numbering, shared by the kernels
// that walk it and the host tables indexed by it: rows -2, -1 across the
// padded width, rows my, my+1, then columns -2, -1, mx, mx+1 of the interior
// rows.
__host__ __device__ inline int ring_size(int mx, int my) { return 4 * (mx + 4) + 4 * my; }
__host__ __device__ inline void ring_cell(int g, int mx, int my, int &i, int &j) {
  const int wx = mx + 4;
  if (g < 2 * wx) {
    j = g / wx - 2, i = g % wx - 2;
  } else if (g < 4 * wx) {
    j = my + (g - 2 * wx) / wx, i = (g - 2 * wx) % wx - 2;
  } else {
    const int h = g - 4 * wx, c = h % 4;
    j = h / 4, i = c < 2 ? c - 2 : mx + c - 2;
  }
}

// Ghosts of a level whose patches tile a domain: ghost g of patch p takes
// components m = 0, 1, 2 from pool elements src[2 e] + m src[2 e + 1],
// e = ring0[p] + g (the source cell's offset and its patch's plane stride).
hipError_t launch_link_ghosts(int dtype, const PatchRow *patches, int n_patches, int max_ring,
                              const int64_t *ring0, const int64_t *src, void *q, hipStream_t s);

hipError_t launch_fill_ghosts(int dtype, const PatchRow *patches, int n_patches,
                              int max_padded_cells, void *q, hipStream_t s);
// dt[k] = value for every instance.
hipError_t launch_set_dt(const CflSlots &c, double value, hipStream_t s);
// Move the step's accumulated Courant numbers to the *_last slots, update the
// running maxima, clear the accumulators and, if cfl_desired > 0, rescale
// each instance's dt by cfl_desired / cfl.
hipError_t launch_finish_step(const CflSlots &c, double cfl_desired, hipStream_t s);
// cfl_patch[k] = max of cfl_tile over patch k's tiles.
hipError_t launch_patch_cfl(const PatchRow *patches, int n_patches, const double *cfl_tile,
                            double *cfl_patch, hipStream_t s);
// Conservation sums over the fixed sum tiles (kSumTile x kSumTile cells of a
// patch each, independent of the step's tiling).
hipError_t launch_sums(int dtype, const PatchRow *patches, int n_patches, const TileEntry *stiles,
                       int n_stiles, const void *q, double *partials, double *patch_sums,
                       int n_inst, double *sums, hipStream_t s);
int step_occupancy(int dtype, int limiter, int vars, int *wg_per_cu);

// Adjoint and receiver helpers (defined in ws_adjoint.hip), FP64 buffers in
// the pools' layout.
// lam_out <- E^T U^T lam_in (one launch: the gather-form update transpose
// with the extrapolation ghosts folded into the boundary cells).
hipError_t launch_adjoint(const PatchRow *patches, int n_patches, int max_mx, int max_my,
                          int n_cu, const InstRow *inst, double dt, const uint8_t *masks,
                          const double *lam_in, double *lam_out, hipStream_t s);
hipError_t launch_gather(const PatchRow *patches, int patch, int comp, int n, const int32_t *ij,
                         const double *buf, double *out, hipStream_t s);
hipError_t launch_add_at(const PatchRow *patches, int patch, int comp, int n, const int32_t *ij,
                         const double *val, double *buf, hipStream_t s);

// Coarse-fine coupling of two levels (defined in ws_amr.hip).  One row per
// fine patch: where it sits in its coarse patch and where its edges' slots
// start.  Fine boundary edges are numbered left (my), right (my), bottom
// (mx), top (mx); the coarse interface edges the same way over ncy, ncx.
struct CfPlace {
  int32_t coarse;    // coarse patch index
  int32_t ci0, cj0;  // coarse cell under fine interior cell (0, 0)
  int32_t ncx, ncy;  // coarse cells covered
  int32_t fedge0;    // first fine boundary edge (accumulator slots)
  int32_t cedge0;    // first coarse interface edge
  int32_t copy0;     // first of this patch's sibling copy rectangles
  int32_t ncopy;     // how many
  int32_t pad_;
};

// Ghost cells (i, j) of a fine patch with i0 <= i < i1, j0 <= j < j1 lie in
// the interior of sibling fine patch `src`, at (i + di, j + dj) there.
struct CfCopy {
  int32_t src;
  int32_t i0, i1, j0, j1;
  int32_t di, dj;
  int32_t pad_;
};

// A coarse cell outside every fine patch that borders n (1..4) of them: the
// fix of each (fine patch, interface edge) pair, applied in this order.
struct CfFix {
  int32_t coarse, oi, oj, n;
  int32_t patch[4];
  int32_t edge[4];
};

struct CfArgs {
  const PatchRow *cpatch, *fpatch;  // device patch tables of the coarse and fine level
  const InstRow *cinst, *finst;
  const CfPlace *place;             // [n_fine]
  int32_t n_fine, r;
  const void *c_old;  // coarse state at t_n
  void *c_new;        // coarse state after the coarse step (updated in place)
  void *f_cur;        // fine current state
  double *acc;        // [r][fine edges][3] fine terms of each fine step
  double *pc;         // [coarse interface edges][3] coarse terms
  const CfCopy *copy; // sibling copy rectangles, CfPlace::copy0 .. + ncopy per fine patch
  const CfFix *fix;   // [n_fix] the coarse cells that take the fix
  int32_t n_fix;
  int32_t strip;      // boundary edges per block of the fine-step kernel (its threads)
  int64_t n_fedges;   // fine boundary edges of all patches (acc holds r slots of them)
};

hipError_t launch_cf_ghosts(int dtype, const CfArgs &a, double alpha, int max_items,
                            hipStream_t s);
// Before fine step `step` (ghost ring, fine terms; coarse terms when step is 0).
hipError_t launch_cf_fine_step(int dtype, int limiter, const CfArgs &a, int step, double dt_fine,
                               double dt, int max_blocks, hipStream_t s);
// Updating and the conservation fix (grid rows 0 .. n_fine-1 average the fine
// patches down, row n_fine applies the fix list).
hipError_t launch_cf_finish(int dtype, const CfArgs &a, double dt, int max_blocks, hipStream_t s);
// Blocks per fine patch of the two launches.
int cf_step_blocks_host(int mx, int my, int ncx, int ncy, bool coarse, int strip);
// Edges per block of the fine-step kernel for fine patches of at most
// max_side cells per side: a multiple of 64, at most 256.
int cf_strip_host(int max_side);
int cf_finish_blocks_host(int ncx, int ncy);
// The coarse cell outside interface edge e of a fine patch (edges numbered
// left, right over ncy, then bottom, top over ncx).
void cf_out_cell_host(const CfPlace &pl, int e, int &oi, int &oj);

}  // namespace ws
