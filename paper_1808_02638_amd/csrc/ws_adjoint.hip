// HIP kernels (gfx950) of the frozen-limiter adjoint of the level step, and
// cell gather / scatter-add helpers for receivers.
//
// With the MC branches of a step held at the ones the forward step took, the
// update of Sec. 2.1 eq. (2.3) is linear in the ghost-padded state, and the
// step S = U o E (E: ghost fill, U: update) has the transpose S^T = E^T U^T.
// The first kernel evaluates U^T in GATHER form: the cotangent of a padded
// cell is assembled from the output cotangents lam' of the cells whose update
// reads it (the transposed 13-point footprint), walking the closed forms of
// the forward kernels backwards:
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

#include <hip/hip_runtime.h>

#include <climits>

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

// One patch's view for the adjoint: lam' with zero extension outside the
// interior, and the recorded branches with code 0 outside their range.  Reads
// are clamped to the interior (and the mask array) before the zero selection,
// so no address outside the patch is formed.
struct AdjPatch {
  const double *lam;  // interior (0, 0) of component p
  int64_t ld, plane;
  int mx, my;
  const uint8_t *mk;  // (mx+1) x (my+1) bytes
  Coef<double> k;

  __device__ double L(int m, int i, int j) const {
    const int ic = min(max(i, 0), mx - 1), jc = min(max(j, 0), my - 1);
    const double v = lam[m * plane + (int64_t)jc * ld + ic];
    return (i == ic && j == jc) ? v : 0.0;
  }
  __device__ unsigned byte(int i, int j) const {
    const int ic = min(max(i, 0), mx), jc = min(max(j, 0), my);
    const unsigned v = mk[(int64_t)jc * (mx + 1) + ic];
    return (i == ic && j == jc) ? v : 0u;
  }

  // U^T: cotangent of padded cell (i, j), any i in [-2, mx+2), j in [-2, my+2).
  // Offsets below are relative to (i, j); x-edge e lies between cells e-1 and
  // e, y-edge f between rows f-1 and f.
  __device__ void pad(int i, int j, double &p, double &u, double &v) const {
    // ---- lam' on the transposed 13-point footprint
    double P[5][5], U[5][5], V[5][5];  // [dy+2][dx+2], only the footprint is read
#pragma unroll
    for (int dy = -2; dy <= 2; ++dy)
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx) {
        const int ad = (dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy);
        if (ad > 2) continue;
        P[dy + 2][dx + 2] = L(0, i + dx, j + dy);
        // u enters through x-edges only (rows -1..1), v through y-edges only
        U[dy + 2][dx + 2] = (dy >= -1 && dy <= 1) ? L(1, i + dx, j + dy) : 0.0;
        V[dy + 2][dx + 2] = (dx >= -1 && dx <= 1) ? L(2, i + dx, j + dy) : 0.0;
      }
#define LP(dx, dy) P[(dy) + 2][(dx) + 2]
#define LU(dx, dy) U[(dy) + 2][(dx) + 2]
#define LV(dx, dy) V[(dy) + 2][(dx) + 2]
    // cotangents of F~ (p, u) at x-edge e of row r, of G~ (p, v) at y-edge f of column c
#define FP(e, r) (k.dtdx * (LP(e, r) - LP((e) - 1, r)))
#define FU(e, r) (k.dtdx * (LU(e, r) - LU((e) - 1, r)))
#define GP(c, f) (k.dtdy * (LP(c, f) - LP(c, (f) - 1)))
#define GV(c, f) (k.dtdy * (LV(c, f) - LV(c, (f) - 1)))
    // cotangents of the cells' fluctuation sums and differences
    double xs[3], xd[3], ys[3], yd[3];  // [offset + 1]
#pragma unroll
    for (int o = -1; o <= 1; ++o) {
      xs[o + 1] = -k.dtdx * k.h * LP(o, 0) + k.gx * (GP(o, 0) - GP(o, 1)) -
                  k.gxz * (GV(o, 0) + GV(o, 1));
      xd[o + 1] = -k.dtdx * k.hz * LU(o, 0);
      ys[o + 1] = -k.dtdy * k.h * LP(0, o) + k.gy * (FP(0, o) - FP(1, o)) -
                  k.gyz * (FU(0, o) + FU(1, o));
      yd[o + 1] = -k.dtdy * k.hz * LV(0, o);
    }
    // cotangents of the limited strengths times the frozen weights, at x-edges
    // -1..2 of row 0 and y-edges -1..2 of column 0
    double o1[4], u1[4], o2[4], u2[4], n1[4], t1[4], n2[4], t2[4];  // [edge + 1]
#pragma unroll
    for (int e = -1; e <= 2; ++e) {
      const double fp = FP(e, 0), fu = FU(e, 0);
      const double l1 = -k.fx * fp + k.fxz * fu, l2 = k.fx * fp + k.fxz * fu;
      const unsigned bx = byte(i + e, j);
      o1[e + 1] = w_own(bx & 3u) * l1;
      u1[e + 1] = w_up(bx & 3u) * l1;
      o2[e + 1] = w_own((bx >> 2) & 3u) * l2;
      u2[e + 1] = w_up((bx >> 2) & 3u) * l2;
      const double gp = GP(0, e), gv = GV(0, e);
      const double m1 = -k.fy * gp + k.fyz * gv, m2 = k.fy * gp + k.fyz * gv;
      const unsigned by = byte(i, j + e);
      n1[e + 1] = w_own((by >> 4) & 3u) * m1;
      t1[e + 1] = w_up((by >> 4) & 3u) * m1;
      n2[e + 1] = w_own((by >> 6) & 3u) * m2;
      t2[e + 1] = w_up((by >> 6) & 3u) * m2;
    }
#undef FP
#undef FU
#undef GP
#undef GV
    // strengths at the cell's edges: wave -c takes its upwind neighbour on the
    // right (above), wave +c on the left (below)
    const double a1L = o1[1] + u1[0] + xs[0] - xd[0], a2L = o2[1] + u2[2] + xs[1] + xd[1];
    const double a1R = o1[2] + u1[1] + xs[1] - xd[1], a2R = o2[2] + u2[3] + xs[2] + xd[2];
    const double b1B = n1[1] + t1[0] + ys[0] - yd[0], b2B = n2[1] + t2[2] + ys[1] + yd[1];
    const double b1T = n1[2] + t1[1] + ys[1] - yd[1], b2T = n2[2] + t2[3] + ys[2] + yd[2];
    p = LP(0, 0) + ((a2L - a1L) - (a2R - a1R)) + ((b2B - b1B) - (b2T - b1T));
    u = LU(0, 0) + k.Z * ((a1L + a2L) - (a1R + a2R));
    v = LV(0, 0) + k.Z * ((b1B + b2B) - (b1T + b2T));
#undef LP
#undef LU
#undef LV
  }
};

__device__ inline AdjPatch make_adj(const PatchRow &pr, const InstRow &in, double dt,
                                    const uint8_t *masks, const double *lam_in) {
  AdjPatch A;
  A.lam = lam_in + pr.q_off + 2 * (int64_t)pr.ld + pr.col0;
  A.ld = pr.ld;
  A.plane = pr.plane;
  A.mx = pr.mx;
  A.my = pr.my;
  A.mk = masks + pr.mask_off;
  A.k = make_coef<double>(in.c, in.Z, dt, pr.dx, pr.dy);
  return A;
}

// U^T: one thread per padded cell of each patch (blockIdx.y); every padded
// cell of lam_out is written.
__global__ __launch_bounds__(kThreads) void adjoint_update_kernel(
    const PatchRow *patches, const InstRow *inst, double dt, const uint8_t *masks,
    const double *lam_in, double *lam_out) {
  const PatchRow pr = uniform_row(patches[blockIdx.y]);
  const AdjPatch A = make_adj(pr, uniform_row(inst[pr.inst]), dt, masks, lam_in);
  double *out = lam_out + pr.q_off + 2 * (int64_t)pr.ld + pr.col0;
  const int wx = pr.mx + 4;
  const int64_t n = (int64_t)wx * (pr.my + 4);
  for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * kThreads) {
    const int i = (int)(idx % wx) - 2, j = (int)(idx / wx) - 2;
    double p, u, v;
    A.pad(i, j, p, u, v);
    const int64_t o = (int64_t)j * pr.ld + i;
    out[o] = p;
    out[pr.plane + o] = u;
    out[2 * pr.plane + o] = v;
  }
}

// E^T: the ghost cotangents of extrapolation patches are added to the
// interior cell they were copied from (each ghost has one: clamp its
// indices), and every ghost is set to 0.  One thread per (interior cell next
// to a side, component), so each ghost value is read and cleared by exactly
// one thread; all reads come before the writes.
__global__ __launch_bounds__(kThreads) void adjoint_fold_kernel(const PatchRow *patches,
                                                              double *lam) {
  const PatchRow pr = uniform_row(patches[blockIdx.y]);
  const bool fold = pr.bc == WS_BC_EXTRAP;
  // the boundary ring of the interior: rows 0 and my-1, then columns 0 and
  // mx-1 of the rows between
  const int top = pr.my > 1 ? pr.mx : 0;
  const int mid = max(pr.my - 2, 0) * (pr.mx > 1 ? 2 : 1);
  const int ring = pr.mx + top + mid;
  for (int idx = blockIdx.x * kThreads + threadIdx.x; idx < 3 * ring;
       idx += gridDim.x * kThreads) {
    const int m = idx / ring, c = idx % ring;
    int i, j;
    if (c < pr.mx) {
      i = c, j = 0;
    } else if (c < pr.mx + top) {
      i = c - pr.mx, j = pr.my - 1;
    } else {
      const int r = c - pr.mx - top, per = pr.mx > 1 ? 2 : 1;
      j = 1 + r / per;
      i = (r % per) ? pr.mx - 1 : 0;
    }
    double *q = lam + pr.q_off + 2 * (int64_t)pr.ld + pr.col0 + m * pr.plane;
    // ghost images of (i, j): up to two ghost columns on each side of its
    // row and two ghost rows on each side of its column, and their crossings
    constexpr int kNone = INT_MIN;
    const int xs[5] = {i, i == 0 ? -1 : kNone, i == 0 ? -2 : kNone, i == pr.mx - 1 ? pr.mx : kNone,
                       i == pr.mx - 1 ? pr.mx + 1 : kNone};
    const int ys[5] = {j, j == 0 ? -1 : kNone, j == 0 ? -2 : kNone, j == pr.my - 1 ? pr.my : kNone,
                       j == pr.my - 1 ? pr.my + 1 : kNone};
    double s = q[(int64_t)j * pr.ld + i];
    if (fold) {
#pragma unroll
      for (int b = 0; b < 5; ++b)
#pragma unroll
        for (int a = 0; a < 5; ++a)
          if ((a | b) != 0 && xs[a] != kNone && ys[b] != kNone)
            s += q[(int64_t)ys[b] * pr.ld + xs[a]];
    }
#pragma unroll
    for (int b = 0; b < 5; ++b)
#pragma unroll
      for (int a = 0; a < 5; ++a)
        if ((a | b) != 0 && xs[a] != kNone && ys[b] != kNone)
          q[(int64_t)ys[b] * pr.ld + xs[a]] = 0.0;
    q[(int64_t)j * pr.ld + i] = s;
  }
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

hipError_t launch_adjoint(const PatchRow *patches, int n_patches, int max_padded_cells,
                          int max_ring, const InstRow *inst, double dt, const uint8_t *masks,
                          const double *lam_in, double *lam_out, hipStream_t s) {
  if (n_patches <= 0) return hipSuccess;
  const int gx = max(1, min(4096, (max_padded_cells + kThreads - 1) / kThreads));
  hipLaunchKernelGGL(adjoint_update_kernel, dim3(gx, n_patches), dim3(kThreads), 0, s, patches,
                     inst, dt, masks, lam_in, lam_out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int gr = max(1, min(256, (3 * max_ring + kThreads - 1) / kThreads));
  hipLaunchKernelGGL(adjoint_fold_kernel, dim3(gr, n_patches), dim3(kThreads), 0, s, patches,
                     lam_out);
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
