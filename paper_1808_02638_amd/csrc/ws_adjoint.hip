// HIP kernels (gfx950) of the frozen-limiter adjoint of the level step, and
// cell gather / scatter-add helpers for receivers.
//
// With the MC branches of a step held at the ones the forward step took, the
// update of Sec. 2.1 eq. (2.3) is linear in the ghost-padded state, and the
// step S = U o E (E: ghost fill, U: update) has the transpose S^T = E^T U^T.
// U^T is evaluated in GATHER form: the cotangent of a padded cell is
// assembled from the output cotangents lam' of the cells whose update reads
// it (the transposed 13-point footprint), walking the closed forms of the
// forward kernels backwards:
//   lam_F(e)   = dtdx (lam'(e) - lam'(e-1))               (p, u) at x-edge e
//   lam_G(f)   = dtdy (lam'(f) - lam'(f-1))               (p, v) at y-edge f
//   lam_xs(i,j) = -dtdx c/2 lam'_p + gx (lam_Gp(j) - lam_Gp(j+1))
//                                  - gxz (lam_Gv(j) + lam_Gv(j+1))
//   lam_xd(i,j) = -dtdx c/(2Z) lam'_u
//   lam_l1(e)  = -fx lam_Fp + fxz lam_Fu,  lam_l2(e) = fx lam_Fp + fxz lam_Fu
//   lam_a1(e)  = w(e) lam_l1(e) + w_up(e-1) lam_l1(e-1) + lam_xs(e-1) - lam_xd(e-1)
//   lam_a2(e)  = w(e) lam_l2(e) + w_up(e+1) lam_l2(e+1) + lam_xs(e) + lam_xd(e)
//   lam_dp(e)  = lam_a2 - lam_a1,  lam_du(e) = Z (lam_a1 + lam_a2)
//   lam_pad(c) = lam'(c) + lam_d(c) - lam_d(c+1)   in each direction,
// with (w, w_up) the weights of the frozen branch (0: 0,0; 1: 1/2,1/2; 2: 2,0;
// 3: 0,2) and every lam' outside the interior taken as 0; the y-direction is
// the mirror image.  E^T adds the cotangents of the extrapolation ghosts to the
// interior cells they copy (clamped indices, corners included).
//
// One launch does both, marching like the forward MARCH tiles: a wavefront
// holds 64 neighbouring columns (60 updated, two halo lanes per side), walks
// up a range of rows with the y-direction terms carried in registers and the
// x-direction terms exchanged between neighbouring lanes, and folds the ghost
// columns (lanes next to the boundary, by lane shifts) and ghost rows (carried
// down to the first row, held up from the last) into the boundary cells
// before storing.  Per padded cell it reads lam' and one branch byte once and
// writes the cotangent once.

#include <hip/hip_runtime.h>

#include "ws_device.h"
#include "ws_internal.h"
#include "../../include/wavestep.h"

namespace ws {
namespace {

// Weights of a frozen MC branch on (own strength, upwind strength).
__device__ inline double w_own(unsigned code) {
  return code == 1u ? 0.5 : (code == 2u ? 2.0 : 0.0);
}
__device__ inline double w_up(unsigned code) {
  return code == 1u ? 0.5 : (code == 3u ? 2.0 : 0.0);
}

// One row of lam' (p, u, v) and the branch byte at one column.
struct AdjSet {
  double p, u, v;
  unsigned m;
};

// Row sets of an adjoint segment (its row loop is unrolled by this count).
constexpr int kAdjSets = 8;

// Wavefronts per CU the launch aims for when it picks the segment height.
#ifndef WS_ADJ_WAVES_PER_CU
#define WS_ADJ_WAVES_PER_CU 8
#endif

// One wavefront of the adjoint: lane l holds column c = c0 - 2 + l of one
// patch.  lam' is read through 32-bit byte offsets from the patch's padded
// origin, at clamped (interior) cells, and taken as 0 outside the interior;
// branch bytes likewise (code 0 outside [0, mx] x [0, my]).
struct AdjLanes {
  const char *lb;     // lam_in at padded cell (-2, -2) of component p
  char *ob;           // lam_out, the same place
  const uint8_t *mk;  // the patch's branch bytes
  unsigned ld, plb;   // row stride (elements), plane stride (bytes)
  int mld, mx, my, c, cl, cm;
  bool colin, colm;

  __device__ void fetch(AdjSet &S, int r) const {
    const int rr = min(max(r, 0), my - 1);
    const unsigned o = ((unsigned)(rr + 2) * ld + (unsigned)(cl + 2)) * 8u;
    S.p = *reinterpret_cast<const double *>(lb + o);
    S.u = *reinterpret_cast<const double *>(lb + plb + o);
    S.v = *reinterpret_cast<const double *>(lb + 2 * plb + o);
    const int rm = min(max(r, 0), my);
    S.m = mk[(int64_t)rm * mld + cm];
  }
  __device__ bool in(int r) const { return colin && r >= 0 && r < my; }
  __device__ unsigned code(const AdjSet &S, int r) const {
    return (colm && r >= 0 && r <= my) ? S.m : 0u;
  }
  __device__ void put(int r, double p, double u, double v) const {
    const unsigned o = ((unsigned)(r + 2) * ld + (unsigned)(c + 2)) * 8u;
    *reinterpret_cast<double *>(ob + o) = p;
    *reinterpret_cast<double *>(ob + plb + o) = u;
    *reinterpret_cast<double *>(ob + 2 * plb + o) = v;
  }
};

// Quantities of one y-edge f of the lane's column from lam' of rows f-1, f:
// lam_G and the frozen-branch terms of its two waves (own and upwind parts).
struct YEdge {
  double gp, gv, n1, t1, n2, t2;
};
__device__ inline YEdge y_edge(const Coef<double> &k, double p_lo, double v_lo, double p_hi,
                               double v_hi, unsigned code) {
  YEdge e;
  e.gp = k.dtdy * (p_hi - p_lo);
  e.gv = k.dtdy * (v_hi - v_lo);
  const double m1 = -k.fy * e.gp + k.fyz * e.gv, m2 = k.fy * e.gp + k.fyz * e.gv;
  const unsigned c1 = (code >> 4) & 3u, c2 = (code >> 6) & 3u;
  e.n1 = w_own(c1) * m1;
  e.t1 = w_up(c1) * m1;
  e.n2 = w_own(c2) * m2;
  e.t2 = w_up(c2) * m2;
  return e;
}

// lam_F (p, u) at x-edge c of a row and the cell's lam_ys, lam_yd.
struct XRow {
  double fp, fu, ys, yd;
};
__device__ inline XRow x_row(const Coef<double> &k, double p, double u, double v) {
  XRow x;
  x.fp = k.dtdx * (p - shr(p));
  x.fu = k.dtdx * (u - shr(u));
  x.ys = -k.dtdy * k.h * p + k.gy * (x.fp - shl(x.fp)) - k.gyz * (x.fu + shl(x.fu));
  x.yd = -k.dtdy * k.hz * v;
  return x;
}

// The segment's rows [r0, r1) (ghost rows included where the segment meets
// the patch's first or last row), marched upward; fold: extrapolation ghosts
// are folded into the boundary cells.
__device__ __attribute__((always_inline)) inline void adjoint_march(const AdjLanes &M,
                                                                   const Coef<double> &k,
                                                                   int l, int r0, int r1,
                                                                   bool fold, bool xedge) {
  AdjSet R0, R1, R2, R3, R4, R5, R6, R7, Sa, Sb;
  M.fetch(Sa, r0 - 2);
  M.fetch(Sb, r0 - 1);
  M.fetch(R0, r0);
  M.fetch(R1, r0 + 1);
  M.fetch(R2, r0 + 2);
  M.fetch(R3, r0 + 3);
  M.fetch(R4, r0 + 4);
  M.fetch(R5, r0 + 5);
  M.fetch(R6, r0 + 6);
  M.fetch(R7, r0 + 7);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  auto P = [&](const AdjSet &S, int r) { return M.in(r) ? S.p : 0.0; };
  auto U = [&](const AdjSet &S, int r) { return M.in(r) ? S.u : 0.0; };
  auto V = [&](const AdjSet &S, int r) { return M.in(r) ? S.v : 0.0; };
  // edge r0-1 (its t1), row r0-1 (its ys, yd), edges r0 and r0+1, row r0
  const YEdge em = y_edge(k, P(Sa, r0 - 2), V(Sa, r0 - 2), P(Sb, r0 - 1), V(Sb, r0 - 1),
                          M.code(Sb, r0 - 1));
  const XRow xm = x_row(k, P(Sb, r0 - 1), U(Sb, r0 - 1), V(Sb, r0 - 1));
  const YEdge e0 = y_edge(k, P(Sb, r0 - 1), V(Sb, r0 - 1), P(R0, r0), V(R0, r0), M.code(R0, r0));
  XRow x0 = x_row(k, P(R0, r0), U(R0, r0), V(R0, r0));
  YEdge e1 = y_edge(k, P(R0, r0), V(R0, r0), P(R1, r0 + 1), V(R1, r0 + 1), M.code(R1, r0 + 1));
  double gp0 = e0.gp, gv0 = e0.gv, t1_0 = e0.t1;
  // lam_b1, lam_b2 at edge r0 (DY = b2 - b1, SY = b1 + b2)
  double DY0, SY0;
  {
    const double b1 = e0.n1 + em.t1 + xm.ys - xm.yd, b2 = e0.n2 + e1.t2 + x0.ys + x0.yd;
    DY0 = b2 - b1;
    SY0 = b1 + b2;
  }
  // ghost rows folded into the first row, and the last row held for its ghosts
  double lo_p = 0.0, lo_u = 0.0, lo_v = 0.0, hi_p = 0.0, hi_u = 0.0, hi_v = 0.0;
  const bool st_val = l >= 2 && l <= 61 && M.c >= 0 && M.c < M.mx;
  const bool st_zero = (M.c == -2 || M.c == -1) || ((M.c == M.mx || M.c == M.mx + 1) && l >= 2);

  auto row = [&](AdjSet &A, const AdjSet &B, const AdjSet &C, int r, bool refill) {
    __builtin_amdgcn_sched_barrier(0);
    const double p0 = P(A, r), u0 = U(A, r), v0 = V(A, r);
    const unsigned m0 = M.code(A, r);
    const double p1 = P(B, r + 1), u1 = U(B, r + 1), v1 = V(B, r + 1);
    // edge r+2 and row r+1
    const YEdge e2 = y_edge(k, p1, v1, P(C, r + 2), V(C, r + 2), M.code(C, r + 2));
    const XRow x1 = x_row(k, p1, u1, v1);
    // the y-terms of edge r+1
    const double b1 = e1.n1 + t1_0 + x0.ys - x0.yd, b2 = e1.n2 + e2.t2 + x1.ys + x1.yd;
    const double DY1 = b2 - b1, SY1 = b1 + b2;
    // the x-terms of row r
    const double l1 = -k.fx * x0.fp + k.fxz * x0.fu, l2 = k.fx * x0.fp + k.fxz * x0.fu;
    const unsigned c1 = m0 & 3u, c2 = (m0 >> 2) & 3u;
    const double o1 = w_own(c1) * l1, u1w = w_up(c1) * l1;
    const double o2 = w_own(c2) * l2, u2w = w_up(c2) * l2;
    const double xs = -k.dtdx * k.h * p0 + k.gx * (gp0 - e1.gp) - k.gxz * (gv0 + e1.gv);
    const double xd = -k.dtdx * k.hz * u0;
    const double a1 = ((o1 + shr(u1w)) + shr(xs)) - shr(xd);
    const double a2 = ((o2 + shl(u2w)) + xs) + xd;
    const double DX = a2 - a1, SX = a1 + a2;
    double op = p0 + (DX - shl(DX)) + (DY0 - DY1);
    double ou = u0 + k.Z * (SX - shl(SX));
    double ov = v0 + k.Z * (SY0 - SY1);
    if (fold && xedge) {
      // ghost columns into the boundary columns of the row
      const double lp1 = shr(op), lu1 = shr(ou), lv1 = shr(ov);
      const double lp2 = shr(lp1), lu2 = shr(lu1), lv2 = shr(lv1);
      const double rp1 = shl(op), ru1 = shl(ou), rv1 = shl(ov);
      const double rp2 = shl(rp1), ru2 = shl(ru1), rv2 = shl(rv1);
      if (M.c == 0) { op += lp1 + lp2; ou += lu1 + lu2; ov += lv1 + lv2; }
      if (M.c == M.mx - 1) { op += rp1 + rp2; ou += ru1 + ru2; ov += rv1 + rv2; }
    }
    if (r < 0) {
      lo_p += op, lo_u += ou, lo_v += ov;
      if (st_val || st_zero) M.put(r, 0.0, 0.0, 0.0);
    } else if (r < M.my) {
      if (fold && r == 0) op += lo_p, ou += lo_u, ov += lo_v;
      if (st_zero) M.put(r, 0.0, 0.0, 0.0);
      if (fold && r == M.my - 1) {
        hi_p = op, hi_u = ou, hi_v = ov;
      } else if (st_val) {
        M.put(r, op, ou, ov);
      }
    } else {
      hi_p += op, hi_u += ou, hi_v += ov;
      if (st_val || st_zero) M.put(r, 0.0, 0.0, 0.0);
      if (fold && r == M.my + 1 && st_val) M.put(M.my - 1, hi_p, hi_u, hi_v);
    }
    // slide up one row
    gp0 = e1.gp, gv0 = e1.gv, t1_0 = e1.t1;
    e1 = e2;
    x0 = x1;
    DY0 = DY1, SY0 = SY1;
    __builtin_amdgcn_sched_barrier(0);
    if (refill) M.fetch(A, r + kAdjSets);
  };
  int r = r0;
  for (; r + kAdjSets <= r1; r += kAdjSets) {
    row(R0, R1, R2, r, true);
    row(R1, R2, R3, r + 1, true);
    row(R2, R3, R4, r + 2, true);
    row(R3, R4, R5, r + 3, true);
    row(R4, R5, R6, r + 4, true);
    row(R5, R6, R7, r + 5, true);
    row(R6, R7, R0, r + 6, true);
    row(R7, R0, R1, r + 7, true);
  }
  if (r < r1) { row(R0, R1, R2, r, r + kAdjSets <= r1 + 1); ++r; }
  if (r < r1) { row(R1, R2, R3, r, r + kAdjSets <= r1 + 1); ++r; }
  if (r < r1) { row(R2, R3, R4, r, r + kAdjSets <= r1 + 1); ++r; }
  if (r < r1) { row(R3, R4, R5, r, r + kAdjSets <= r1 + 1); ++r; }
  if (r < r1) { row(R4, R5, R6, r, r + kAdjSets <= r1 + 1); ++r; }
  if (r < r1) { row(R5, R6, R7, r, r + kAdjSets <= r1 + 1); ++r; }
  if (r < r1) { row(R6, R7, R0, r, r + kAdjSets <= r1 + 1); ++r; }
}

// One wavefront per workgroup: segment (tx, ty) of patch blockIdx.y, 60
// columns by `rows` rows.  Every padded cell of lam_out is written: the
// interior with its (folded) cotangent, the ghosts with 0.
__global__ __launch_bounds__(64) void adjoint_kernel(const PatchRow *patches,
                                                     const InstRow *inst, double dt,
                                                     const uint8_t *masks, const double *lam_in,
                                                     double *lam_out, int rows) {
  const PatchRow pr = uniform_row(patches[blockIdx.y]);
  const int ntx = (pr.mx + 59) / 60, nty = (pr.my + rows - 1) / rows;
  const int b = (int)blockIdx.x;
  if (b >= ntx * nty) return;
  const int tx = b % ntx, ty = b / ntx;
  const InstRow in = uniform_row(inst[pr.inst]);
  const Coef<double> k = make_coef<double>(in.c, in.Z, dt, pr.dx, pr.dy);
  const int l = (int)threadIdx.x;
  AdjLanes M;
  const int64_t org = pr.q_off + pr.col0 - 2;  // padded cell (-2, -2)
  M.lb = reinterpret_cast<const char *>(lam_in + org);
  M.ob = reinterpret_cast<char *>(lam_out + org);
  M.mk = masks + pr.mask_off;
  M.ld = (unsigned)pr.ld;
  M.plb = (unsigned)pr.plane * 8u;
  M.mld = pr.mx + 1;
  M.mx = pr.mx;
  M.my = pr.my;
  M.c = tx * 60 - 2 + l;
  M.cl = min(max(M.c, 0), pr.mx - 1);
  M.cm = min(max(M.c, 0), pr.mx);
  M.colin = M.c >= 0 && M.c < pr.mx;
  M.colm = M.c >= 0 && M.c <= pr.mx;
  const int r0 = ty * rows, r1 = min(r0 + rows, pr.my);
  const bool fold = pr.bc == WS_BC_EXTRAP;
  const bool xedge = tx == 0 || tx == ntx - 1;
  adjoint_march(M, k, l, r0 == 0 ? -2 : r0, r1 == pr.my ? pr.my + 2 : r1, fold, xedge);
}

__global__ void gather_kernel(const PatchRow *patches, int patch, int comp, int n,
                              const int32_t *ij, const double *buf, double *out) {
  const PatchRow pr = patches[patch];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int i = ij[2 * k], j = ij[2 * k + 1];
    double v = __builtin_nan("");
    if (i >= 0 && i < pr.mx && j >= 0 && j < pr.my)
      v = buf[pr.q_off + comp * pr.plane + (int64_t)(j + 2) * pr.ld + pr.col0 + i];
    out[k] = v;
  }
}

__global__ void add_at_kernel(const PatchRow *patches, int patch, int comp, int n,
                              const int32_t *ij, const double *val, double *buf) {
  const PatchRow pr = patches[patch];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int i = ij[2 * k], j = ij[2 * k + 1];
    if (i >= 0 && i < pr.mx && j >= 0 && j < pr.my)
      atomicAdd(&buf[pr.q_off + comp * pr.plane + (int64_t)(j + 2) * pr.ld + pr.col0 + i], val[k]);
  }
}

}  // namespace

hipError_t launch_adjoint(const PatchRow *patches, int n_patches, int max_mx, int max_my,
                          int n_cu, const InstRow *inst, double dt, const uint8_t *masks,
                          const double *lam_in, double *lam_out, hipStream_t s) {
  if (n_patches <= 0) return hipSuccess;
  // rows per segment: the tallest of 32, 16, 8, 4, 2 that still gives
  // WS_ADJ_WAVES_PER_CU wavefronts per CU (a small level is worked by many
  // short segments)
  const int ntx = (max_mx + 59) / 60;
  int rows = 32;
  while (rows > 2 && (int64_t)ntx * ((max_my + rows - 1) / rows) * n_patches <
                         WS_ADJ_WAVES_PER_CU * (int64_t)max(n_cu, 1))
    rows /= 2;
  const int nty = (max_my + rows - 1) / rows;
  hipLaunchKernelGGL(adjoint_kernel, dim3((unsigned)(ntx * nty), (unsigned)n_patches), dim3(64),
                     0, s, patches, inst, dt, masks, lam_in, lam_out, rows);
  return hipGetLastError();
}

hipError_t launch_gather(const PatchRow *patches, int patch, int comp, int n, const int32_t *ij,
                         const double *buf, double *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int g = min(1024, (n + 255) / 256);
  hipLaunchKernelGGL(gather_kernel, dim3(g), dim3(256), 0, s, patches, patch, comp, n, ij, buf,
                     out);
  return hipGetLastError();
}

hipError_t launch_add_at(const PatchRow *patches, int patch, int comp, int n, const int32_t *ij,
                         const double *val, double *buf, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int g = min(1024, (n + 255) / 256);
  hipLaunchKernelGGL(add_at_kernel, dim3(g), dim3(256), 0, s, patches, patch, comp, n, ij, val,
                     buf);
  return hipGetLastError();
}

}  // namespace ws
