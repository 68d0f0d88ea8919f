/*
 * wavestep.h -- C ABI of the MI355X (gfx950) library that advances 2D linear
 * acoustics with the dimensionally unsplit wave-propagation method, one AMR
 * level (a set of ghost-padded rectangular patches) at a time.
 *
 * What is computed (Qin, LeVeque & Motley, arXiv 1808.02638):
 *   - the update of paper Sec. 2.1 eq. (2.3): for every interior cell,
 *     Q^{n+1} = Q - dt/dx (A+dQ_{i-1/2} + A-dQ_{i+1/2})
 *                 - dt/dy (B+dQ_{j-1/2} + B-dQ_{j+1/2})
 *                 - dt/dx (F~_{i+1/2} - F~_{i-1/2}) - dt/dy (G~_{j+1/2} - G~_{j-1/2}),
 *     with F~, G~ holding the limited wave corrections and the transverse
 *     waves split from the first-order fluctuations (Sec. 2.1, Sec. 3.3), or,
 *     with WS_TRANSVERSE_CORR, from the fluctuations with the limited
 *     corrections moved into them;
 *   - for q = (p, u, v) and the matrices A, B of Sec. 4.1 eqs. (4.1)-(4.2)
 *     (wave speeds -c, 0, +c with c = sqrt(K/rho));
 *   - the Courant number of Sec. 2.4 eq. (2.10), max over the level's edges of
 *     |s| dt/dx, reduced over all patches on the device (Sec. 3.2.2), and the
 *     time-step rule dt = nu dt_old / cfl_old of Sec. 2.5 eq. (2.11);
 *   - physical boundaries through the two ghost layers (Sec. 2.2 item 1):
 *     zero-order extrapolation (the outflow condition of Sec. 4.1) or periodic.
 *
 * Conventions
 *   - Every function returns WS_OK (0) or a negative WS_E* code; the message
 *     of the last failure on the calling thread is in ws_last_error().  No
 *     function aborts and no C++ exception crosses this boundary.
 *   - The CALLER OWNS ALL DEVICE MEMORY AND THE STREAM: the two q pools and
 *     the workspace are device allocations the caller makes with the sizes
 *     ws_layout() returns and keeps alive until ws_destroy().  The context
 *     owns only host metadata, one small pinned host buffer and graph handles.
 *     A context is not thread-safe; all work is enqueued on the caller's
 *     stream given at init.
 *   - "Host layout" of one patch is dense [3][my+4][mx+4] in the context's
 *     dtype: components p, u, v; two ghost layers per side; x fastest.  The
 *     device layout inside a pool is private (padded, aligned rows).
 *   - Patches of one context may differ in size, cell size and material
 *     (instance); one context is one AMR level or one ensemble.
 */
#ifndef WAVESTEP_H
#define WAVESTEP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WS_OK 0
#define WS_EINVAL (-1)  /* bad argument (sizes, indices, null pointers)      */
#define WS_ESTATE (-2)  /* call not valid in the context's current state      */
#define WS_EHIP (-3)    /* a HIP runtime call failed (message names it)      */
#define WS_ENOMEM (-4)  /* caller-provided pool or workspace too small        */

enum { WS_F64 = 0, WS_F32 = 1 };          /* arithmetic and storage type   */
/* Wave limiters (Sec. 2.1): MC, none (phi = 1), van Leer (the paper's own
 * benchmark limiter, Sec. 4.1). */
enum { WS_LIM_MC = 0, WS_LIM_NONE = 1, WS_LIM_VANLEER = 2 };
/* Option OR-ed into the limiter argument of ws_init_patches: the transverse
 * solver also splits the limited second-order correction.  Before the
 * transverse split the correction c_{i-1/2} = sum_p |s_p| (1 - |s_p| dt/dx) W~_p
 * of each edge is moved into the fluctuations, A+dQ - c and A-dQ + c (their
 * sum is unchanged), so the correction waves are also carried across the
 * y-edges; the y-direction is the mirror image.  The update's fluctuations
 * and F~, G~'s normal parts are those of the default method.  Both variants
 * are second-order accurate (Sec. 2.1 names the transverse waves as part of
 * F~ and G~ without fixing which waves are split).  Branch recording and the
 * adjoint exist for the default variant only. */
#define WS_TRANSVERSE_CORR 0x100
enum { WS_BC_NONE = 0, WS_BC_EXTRAP = 1, WS_BC_PERIODIC = 2 };

typedef struct ws_ctx ws_ctx;

/* One patch.  bc = WS_BC_NONE: ghosts are input (uploaded, kept frozen);
 * WS_BC_EXTRAP / WS_BC_PERIODIC: all four sides are physical boundaries whose
 * ghosts the step rewrites from the new interior.  Periodic needs mx, my >= 2. */
typedef struct {
  int32_t mx, my;   /* interior cells, >= 1                          */
  double dx, dy;    /* cell sizes, > 0                               */
  int32_t instance; /* index into the material and dt arrays         */
  int32_t bc;       /* WS_BC_*                                       */
} ws_patch_desc;

/* Medium of one instance: c = sqrt(K/rho), impedance Z = rho c. */
typedef struct {
  double rho, K;
} ws_material;

/* Sizes the caller must allocate: each of the two q pools (bytes) and the
 * workspace (bytes).  Either output pointer may be NULL.  The pools hold every
 * patch of the level with its two ghost layers (Sec. 2.2: ghost cells carry the
 * boundary data a patch's step reads), each patch in three planes p, u, v; the
 * level's patches live together in device memory between steps (the paper
 * copies them to the GPU and back around every advance, Sec. 3.2.2; here they
 * stay resident).  Fails with WS_EINVAL for an invalid patch list. */
int ws_layout(const ws_patch_desc *patches, int32_t n_patches, int32_t n_instances,
              int32_t dtype, int64_t *pool_bytes, int64_t *ws_bytes);

/* Create a context over caller-owned device memory.  mbc must be 2.
 * q_pool_a / q_pool_b: device buffers of >= pool_bytes; the level's state
 * lives in pool A first and ping-pongs.  workspace: device buffer of >=
 * ws_bytes (patch table, tile list, CFL slots, dt, counters, sums).
 * hip_stream: the hipStream_t all work is enqueued on (NULL = null stream).
 * limiter: WS_LIM_*, optionally OR-ed with WS_TRANSVERSE_CORR.
 * Uploads the patch table and tile list and synchronises the stream. */
int ws_init_patches(ws_ctx **out, const ws_patch_desc *patches, int32_t n_patches,
                    const ws_material *mats, int32_t n_instances, int32_t mbc,
                    int32_t dtype, int32_t limiter, void *q_pool_a, void *q_pool_b,
                    int64_t pool_bytes, void *workspace, int64_t ws_bytes,
                    void *hip_stream);

/* Tiling per patch (arrays of n_patches; all NULL keeps the defaults) and
 * workgroups per CU of the persistent launch (0: the default, as many as fit
 * on a CU at the kernel's occupancy).  Every
 * tile is worked by one workgroup of 256 threads.
 *   variant WS_TILE_DIRECT: tile_w x tile_h cells, tile_w in {8,16,...,256},
 *     one thread per column computing each cell from its 13-point footprint;
 *   variant WS_TILE_MARCH: tile_w = 64; four one-wavefront segments of 64
 *     lanes stacked vertically; each segment updates 60 columns and tile_h/4
 *     rows, carrying y-terms up the column in registers and exchanging
 *     x-terms between neighbouring lanes.  Patches of more than 2^31 bytes
 *     (three planes) take DIRECT tiles only;
 *   variant WS_TILE_PACKED: tile_w = 64; the MARCH sweep with one
 *     wavefront's 64 lanes shared by column blocks of several narrow patches
 *     (each block of at most 60 columns takes its width plus four halo
 *     lanes).  Patches with the same instance, dx, dy, my and tile_h are
 *     laid side by side into 64-lane columns (a patch may continue into the
 *     next one), and each lane column is tiled like a MARCH patch: tiles of
 *     tile_h rows (16 to 256), four stacked wavefronts of at most tile_h/4
 *     rows each, the rows spread evenly over the four when the patch is
 *     shorter.  For patches with frozen ghosts (WS_BC_NONE) in pools under
 *     2^31 bytes; a level with PACKED tiles refuses ws_step_level_per_patch,
 *     per-patch timing and ws_step_record_masks.
 * tile_h must be a multiple of 256/tile_w with at most 64 rows per thread
 * (DIRECT) or per segment (MARCH, PACKED).
 * Periodic patches take DIRECT tiles only.
 * variant may be NULL (all DIRECT).  Results do not depend on the tiling
 * (bitwise).  Invalidates a captured graph. */
enum { WS_TILE_DIRECT = 0, WS_TILE_MARCH = 1, WS_TILE_PACKED = 2 };

/* The tiling in use: per patch variant, tile_w, tile_h (arrays of n_patches,
 * each may be NULL) and the persistent launch's workgroups per CU and grid
 * size (either may be NULL). */
int ws_get_tiling(ws_ctx *ctx, int32_t *variant, int32_t *tile_w, int32_t *tile_h,
                  int32_t *wg_per_cu, int32_t *grid);
int ws_set_tiling(ws_ctx *ctx, const int32_t *variant, const int32_t *tile_w,
                  const int32_t *tile_h, int32_t wg_per_cu);

/* Heterogeneous medium (the paper's extension to variable coefficients):
 * rho and K per cell instead of per instance.  medium: caller-owned device
 * buffer of at least pool_bytes (it holds c, Z and 1/(Z^2 + 1) per cell,
 * laid out like the q pools), kept until ws_destroy.  Attaching switches every patch to
 * DIRECT tiles; ws_set_tiling may then choose DIRECT or MARCH tiles (not
 * PACKED), with the same results bitwise; the step then uses the
 * normal solver for two media (waves along (-Z_l, 1, 0) with speed -c_l and
 * (Z_r, 1, 0) with +c_r), limits on wave vectors, splits transversely with
 * the impedances of the neighbouring cells, and reduces the Courant number
 * max over edges of max(c_l, c_r) dt/dx from the cells (the instance's
 * material is then unused; the instance still owns the dt slot).  Not with
 * WS_TRANSVERSE_CORR, branch recording, the adjoint or the coarse-fine
 * coupling; WS_EINVAL for a patch whose three planes span 4 GiB or more.
 * Synchronises the stream. */
int ws_attach_medium(ws_ctx *ctx, void *medium, int64_t bytes);
/* rho, K: host arrays [my+4][mx+4] (ghost cells included: the step reads the
 * medium of ghost cells next to the patch), finite and > 0.  Synchronises. */
int ws_upload_medium(ws_ctx *ctx, int32_t patch, const double *rho, const double *K);

/* Copy one patch, host layout, into BOTH pools (ghosts included: for
 * WS_BC_NONE patches the ghosts are the frozen boundary data of Sec. 2.2).
 * src may be a host or a device pointer; it is read, not kept.  WS_EINVAL for
 * a patch index out of range.  Synchronises the stream. */
int ws_upload_patch(ws_ctx *ctx, int32_t patch, const void *src);

/* Copy one patch of the current state, host layout (ghosts included), to dst
 * (host or device, caller-owned, (mx+4)(my+4) values per component).  WS_EINVAL
 * for a patch index out of range.  Synchronises the stream. */
int ws_download_patch(ws_ctx *ctx, int32_t patch, void *dst);

/* Rewrite the physical-boundary ghosts of the current state from its interior
 * (patches with bc != WS_BC_NONE); on a tiled level (ws_link_level) every
 * ghost from the exchange instead.  Asynchronous. */
int ws_fill_ghosts(ws_ctx *ctx);

/* --------------------------------------------------------------------------
 * Tiled level: the level's patches tile one rectangular domain and exchange
 * ghosts (the ghost-cell rules of Sec. 2.2 at the coarsest level).  A ghost
 * outside the domain is mapped into it by the physical condition of its
 * direction (periodic: the global index wraps; otherwise zero-order
 * extrapolation: it is clamped to the domain's edge cell), then copied from
 * the interior cell of the patch holding that domain cell (possibly the patch
 * itself).  Once linked, every step call (ws_step_level,
 * ws_step_level_per_patch, ws_step_auto and captured graphs) runs the
 * exchange on the new state right after the step, and ws_fill_ghosts runs it
 * on the current one; a cut of the domain into tiles then steps exactly like
 * the domain as one patch.  ws_step_record_masks, ws_adjoint_step and use as
 * the fine level of a coupling refuse a tiled level.
 *
 * Bytes of the link buffer: 8 per patch (ring offsets) and 16 per ghost cell
 * (the source cell's pool offset and its patch's plane stride), each part
 * rounded up to 256. */
int ws_link_layout(ws_ctx *ctx, int64_t *bytes);
/* origins: 2 per patch, global cell (x0, y0) of its interior cell (0, 0).
 * The patches must cover [0, domain_mx) x [0, domain_my) exactly, without
 * overlap, have bc WS_BC_NONE, one instance and one cell size, and the level
 * must not be the fine level of a live coupling.  periodic:
 * bit 0 for x, bit 1 for y.  buffer: caller-owned device memory of at least
 * ws_link_layout bytes, kept for the context's lifetime; the table is built on
 * the host and uploaded (synchronises the stream).  Drops a captured graph.
 * WS_EINVAL on a layout that does not tile the domain, WS_ENOMEM on a short
 * buffer. */
int ws_link_level(ws_ctx *ctx, const int32_t *origins, int32_t domain_mx, int32_t domain_my,
                  int32_t periodic, void *buffer, int64_t bytes);

/* One step of every patch with the same dt, in ONE persistent launch over the
 * level's tile list.  Writes the other pool's interior (and physical ghosts),
 * then makes it current.  *cfl_out (may be NULL) receives the level's Courant
 * number max |s| dt/dx over all edges, reduced in FP64 on the device; this
 * call synchronises the stream to return it.  dt is not checked against the
 * CFL limit: a caller may reject cfl > 1 and redo the step from a saved state. */
int ws_step_level(ws_ctx *ctx, double dt, double *cfl_out);

/* The same step as one launch PER PATCH (the per-patch baseline).  Identical
 * arithmetic; the result is bitwise equal to ws_step_level's. */
int ws_step_level_per_patch(ws_ctx *ctx, double dt, double *cfl_out);

/* Set the device-resident time step of every instance (n_instances values). */
int ws_set_dt(ws_ctx *ctx, const double *dt_per_instance);

/* One step with the device-resident per-instance dt, followed by the dt update
 * dt <- dt * cfl_desired / cfl of each instance.  Asynchronous (no host read). */
int ws_step_auto(ws_ctx *ctx, double cfl_desired);

/* Capture n_steps of ws_step_auto in a hipGraph (replacing any previous one).
 * Needs n_steps >= 1. */
int ws_capture_steps(ws_ctx *ctx, int32_t n_steps, double cfl_desired);

/* Launch the captured graph on the context's stream.  Asynchronous. */
int ws_graph_launch(ws_ctx *ctx);

/* Per instance: current dt, Courant number of the last step and the largest
 * Courant number seen since the last ws_set_dt (any pointer may be NULL).
 * Synchronises the stream. */
int ws_read_dt_cfl(ws_ctx *ctx, double *dt, double *cfl_last, double *cfl_max);

/* Per patch: Courant number of the last step.  Synchronises the stream. */
int ws_read_patch_cfl(ws_ctx *ctx, double *cfl);

/* Conservation sums of the current state: for every instance, the sums of
 * p dx dy, u dx dy, v dx dy over its interior cells ([n_instances][3]),
 * accumulated in FP64 in a fixed order (deterministic for a fixed tiling).
 * Synchronises the stream. */
int ws_conservation_sums(ws_ctx *ctx, double *sums);

/* ---- Frozen-limiter adjoint (FP64 contexts with the MC limiter; patches
 * with WS_BC_EXTRAP or WS_BC_NONE).  With the limiter branches of one step
 * frozen, the step of Sec. 2.1 eq. (2.3) is a linear map S = U o E of the
 * interior state (E: the ghost fill, U: the update); ws_adjoint_step applies
 * S^T: the discrete adjoint of the step, used for gradients of misfits of
 * receiver traces with respect to the initial state.  (The paper has no
 * adjoint; this is the transpose of its step with the limiter of Sec. 2.1
 * held at the branches the forward step took.)
 *
 * Branch masks: one byte per cell (i, j), i in [0, mx], j in [0, my], row-
 * major with row length mx + 1, patches concatenated in patch order.  Bits
 * 0-1 and 2-3: the MC branch of the waves of speed -c and +c at x-edge
 * i - 1/2 (rows j < my); bits 4-5 and 6-7: the same at y-edge j - 1/2
 * (columns i < mx); unused bits are 0.  Branch 0: zero, 1: (a + a_up)/2,
 * 2: 2a, 3: 2 a_up, with a_up the strength of the same wave at the upwind
 * edge; on ties the lowest code. */

/* Bytes of the branch masks of all patches. */
int ws_mask_bytes(ws_ctx *ctx, int64_t *bytes);

/* Where patch `patch` sits in any buffer with the pools' layout: element
 * offset of padded cell (i, j) = (-2, -2) of component p, the row stride and
 * the component (plane) stride, in elements.  Component m, cell (i, j) is at
 * offset + m * plane + (j + 2) * ld + (i + 2). */
int ws_patch_layout(ws_ctx *ctx, int32_t patch, int64_t *offset, int64_t *ld, int64_t *plane);

/* ws_step_level(dt) recording the branches into masks_dev (device buffer of
 * ws_mask_bytes; the step writes every byte, the one no edge owns as 0).
 * cfl_out may be NULL; when given the call synchronises the stream. */
int ws_step_record_masks(ws_ctx *ctx, double dt, void *masks_dev, double *cfl_out);

/* lam_out <- S^T lam_in for the step recorded in masks_dev with time step dt.
 * lam_in, lam_out: distinct device buffers of pool_bytes in the pools'
 * layout.  lam_in: cotangent of the interior of Q^{n+1} (its ghosts are not
 * read); lam_out: cotangent of the interior of Q^n, ghosts set to 0.  For
 * WS_BC_EXTRAP patches the ghost cells' cotangents are folded into the
 * interior cells they were copied from; for WS_BC_NONE patches ghosts are
 * inputs held fixed and get no cotangent.  Asynchronous on the context's
 * stream; periodic patches and FP32 or unlimited contexts return WS_EINVAL. */
int ws_adjoint_step(ws_ctx *ctx, double dt, const void *masks_dev, const void *lam_in,
                    void *lam_out);

/* Cell access in a pool-layout buffer (buf = NULL: the current state) of an
 * FP64 context, for n cells (i_k, j_k) of component comp of one patch:
 *   ws_gather: out[k] = buf(comp, i_k, j_k)  (NaN for a cell outside the interior)
 *   ws_add_at: buf(comp, i_k, j_k) += val[k] (cells outside the interior are
 *              skipped; repeated cells all add, in an unspecified order).
 * ij: n pairs (i, j) of int32; out, val: FP64; all device pointers.
 * Asynchronous on the context's stream. */
int ws_gather(ws_ctx *ctx, const void *buf, int32_t patch, int32_t comp, int32_t n,
              const int32_t *ij, double *out);
int ws_add_at(ws_ctx *ctx, void *buf, int32_t patch, int32_t comp, int32_t n,
              const int32_t *ij, const double *val);

/* Timing entry (for the benchmark and the tile autotuner): enqueue n_launches
 * level steps back to back (batched persistent launch, or per_patch != 0:
 * one launch per patch and the Courant-number filing kernel) with the
 * device-resident dt and no dt update, each step bracketed by its own pair
 * of HIP events on the context's stream; returns the mean bracketed
 * milliseconds per level step (1 <= n_launches <= 100000).  The state
 * advances n_launches steps.  Synchronises the stream. */
int ws_time_step_kernel(ws_ctx *ctx, int32_t n_launches, int32_t per_patch,
                        double *ms_per_step);

/* Index (0 = A, 1 = B) of the pool holding the current state. */
int ws_current_pool(ws_ctx *ctx, int32_t *which);

/* --------------------------------------------------------------------------
 * Coarse-fine coupling: one composite coarse step of two levels with the
 * conservation fix (Sec. 2.2 flow chart: advance, updating, conservation
 * fix; Sec. 2.3 for the fix terms C1, C2, C3).
 *
 * The fine level's patches are nested in the coarse level's with refinement
 * ratio r in space and time: fine patch k covers the ncx x ncy coarse cells
 * from (ci0, cj0) of coarse patch coarse_patch, has r*ncx x r*ncy cells of
 * size dx/r, and steps r times with dt/r per coarse step.  One composite step
 * (ws_cf_step, all on the shared stream, no host synchronisation):
 *   1. the coarse terms at every coarse-fine interface edge are taken from
 *      the coarse state Q^n, then the coarse level steps with dt;
 *   2. r times: the fine ghosts are filled (a ghost inside a sibling fine
 *      patch of the same coarse patch copies the sibling's cell at the same
 *      fine step; every other ghost comes from the coarse level at
 *      t_n + k dt/r, linear in time between Q^n and Q^{n+1}, MC-limited
 *      linear in space inside the coarse cell holding the ghost), the fine
 *      terms at the fine patches' boundary edges are accumulated, and the
 *      fine level steps with dt/r;
 *   3. each covered coarse cell takes the mean of its r x r fine cells;
 *   4. each coarse cell next to a fine patch and covered by none (it may
 *      border several) replaces the coarse flux through each shared edge by
 *      the mean of the fine fluxes through it over the r
 *      fine steps; written in fluctuations this is C1 + C2 + C3 (C1 from the
 *      Riemann problem between the coarse cell at t_n and the fine ghost, C2
 *      from the fluctuations, C3 from F~ or G~; the coarse F~ enters with
 *      weight dt/dx);
 *   5. the coarse physical ghosts are refilled.
 * Afterwards the composite totals (sum of q over coarse cells, covered ones
 * holding fine means) change only by the fluxes through the coarse
 * patch's physical boundary.
 *
 * Requirements (WS_EINVAL otherwise): both contexts have the same dtype,
 * limiter (no WS_TRANSVERSE_CORR) and stream; fine patches have bc
 * WS_BC_NONE, sizes divisible by r, cell sizes dx/r, dy/r and the coarse
 * patch's material; each lies at least 2 coarse cells inside its coarse
 * patch, and fine patches of one coarse patch do not overlap (they may
 * touch).
 */
typedef struct ws_cf ws_cf;
typedef struct {
  int32_t coarse_patch; /* index in the coarse context                       */
  int32_t ci0, cj0;     /* coarse cell under the fine patch's interior (0, 0) */
} ws_fine_place;

/* Bytes of device workspace the coupling needs (placement table, one
 * slot of 3 doubles per fine boundary edge and fine step, 3 doubles per coarse
 * interface edge, the sibling copy rectangles and the fix list, both sized
 * for any layout of these patches). */
int ws_cf_layout(ws_ctx *fine, int32_t ratio, int64_t *bytes);
/* places: one per fine patch.  workspace: caller-owned device buffer of at
 * least ws_cf_layout bytes, kept until ws_cf_destroy.  Both contexts must
 * outlive the coupling.  Synchronises the stream. */
int ws_cf_init(ws_cf **out, ws_ctx *coarse, ws_ctx *fine, int32_t ratio,
               const ws_fine_place *places, void *workspace, int64_t ws_bytes);
/* One composite coarse step of size dt (steps 1-5 above).  Each level's
 * current pool flips as in ws_step_level (the fine level's r times). */
int ws_cf_step(ws_cf *cf, double dt);
/* Nest couplings for more than two levels: inner couples outer's fine level
 * (as its coarse level) with a finer one.  ws_cf_step(outer) then runs, in
 * place of each plain fine step, ws_cf_step(inner) with dt/r: the fine level's
 * step, its own fine steps, their updating and fix (the recursion of the
 * Sec. 2.2 flow chart).  inner NULL removes the nesting.  Both couplings must
 * outlive the nesting. */
int ws_cf_nest(ws_cf *outer, ws_cf *inner);
/* Fill the fine ghosts alone, at t_n + alpha (t_{n+1} - t_n) with t_n the
 * coarse level's previous pool and t_{n+1} its current one, 0 <= alpha <= 1. */
int ws_cf_fill_fine_ghosts(ws_cf *cf, double alpha);
int ws_cf_destroy(ws_cf *cf);

/* --------------------------------------------------------------------------
 * Level step that allocates nothing, for callers that cannot allocate device
 * memory (code that must not call hipMalloc: tight serving loops, harnesses
 * that forbid it).  The same step as ws_step_level (one persistent launch of
 * the same kernels, default tiling, bitwise the same results), with no
 * context and no caller workspace: the patch table, tile list and Courant-
 * number slots live in a device array of ws_noalloc_scratch_bytes() bytes
 * (8 MiB) that the library holds on every GPU it runs on until the process
 * ends.  The call uploads the tables from host memory, clears the slots that
 * must start at zero, steps, reads the Courant number back and synchronises
 * the stream, so it is not for use under stream capture.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (several host
 * threads or streams) race and must be serialised by the caller.
 *   patches, mats, dtype, limiter: as for ws_init_patches;
 *   q_in, q_out: distinct device buffers of >= pool_bytes laid out as the
 *     pools ws_layout() sizes for this patch list (ws_patch_layout of a
 *     context over the same list gives each patch's place); q_out receives
 *     every interior cell and, on physical boundaries, the ghosts; ghosts of
 *     WS_BC_NONE patches in q_out are left as they are;
 *   *cfl_out (may be NULL): the level's Courant number, as ws_step_level.
 * A level whose workspace (ws_layout's ws_bytes) exceeds the array returns
 * WS_ENOMEM without touching the GPU. */
int64_t ws_noalloc_scratch_bytes(void);
int ws_step_level_noalloc(const ws_patch_desc *patches, int32_t n_patches,
                          const ws_material *mats, int32_t n_instances, int32_t dtype,
                          int32_t limiter, const void *q_in, void *q_out, int64_t pool_bytes,
                          double dt, double *cfl_out, void *hip_stream);

int ws_destroy(ws_ctx *ctx);
const char *ws_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WAVESTEP_H */
