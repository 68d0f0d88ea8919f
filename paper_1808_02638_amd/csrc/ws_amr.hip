// HIP kernels (gfx950) coupling a coarse level and the fine level nested in
// it: the pieces of one composite coarse step that are not the level step
// itself (paper Sec. 2.2 flow chart; Sec. 2.3 updating and conservation fix).
//
//   cf_fine_step (before fine step k, after the coarse step):
//     - the fine ghosts: a ghost inside a sibling fine patch (fine patches of
//       one coarse patch may touch) copies the sibling's cell at the same
//       fine step; every other one comes from the coarse level at
//       t_n + k dt/r, linear in time between Q_c^n and Q_c^{n+1} and
//       MC-limited linear in space inside the coarse cell that holds it;
//     - the fine terms at the patch's boundary edges, one slot per fine step
//       (the last fine step sums them into the first slot): f(ghost) -
//       f(Q_O^n) (the Riemann fluctuation sum between
//       the coarse cell O outside the edge and the fine ghost next to it, C1)
//       plus A-dQ^ + F~^ (left side) or -A+dQ^ + F~^ (right side), y alike;
//     - for k = 0, the coarse terms at every coarse-fine interface edge from
//       Q_c^n (still in the coarse pool the step read), P_c = A-dQ + F~ (fine
//       patch on the edge's right) or -A+dQ + F~ (fine patch on its left);
//   cf_finish (after the fine steps):
//     - updating: each covered coarse cell takes the mean of its r x r fine
//       cells;
//     - the fix: each coarse cell O next to a fine patch (and covered by
//       none) replaces the coarse flux through their shared edge by the mean
//       of the fine fluxes, O -= dt/dx ((1/r^2) sum acc - P_c) when the patch
//       is on O's right, O += dt/dx ((1/r^2) sum acc - P_c) when it is on O's
//       left (y alike); a cell bordering several patches takes each fix, all
//       in one thread (a gathered list built at set-up), so no two threads
//       update one cell.
// A composite step is thus the coarse step, r pairs (cf_fine_step, fine
// step), cf_finish and the coarse ghost ring: few launches, as every small
// launch carries a fixed cost of a few microseconds.
// Edge terms use the closed forms of the level step (A-dQ = (c/2 a1,
// -c/(2Z) a1, 0), A+dQ = (c/2 a2, c/(2Z) a2, 0) with the unscaled strengths
// a1 = Z du - dp, a2 = Z du + dp; F~ and G~ as the step forms them).

#include <hip/hip_runtime.h>

#include "ws_device.h"
#include "ws_internal.h"
#include "../../include/wavestep.h"

namespace ws {
namespace {

// Padded planes of one patch, indexed by interior coordinates (i, j).
template <typename T>
struct View {
  const T *p, *u, *v;
  int64_t ld;
  __device__ T P(int i, int j) const { return p[(int64_t)j * ld + i]; }
  __device__ T U(int i, int j) const { return u[(int64_t)j * ld + i]; }
  __device__ T V(int i, int j) const { return v[(int64_t)j * ld + i]; }
};

template <typename T>
__device__ inline View<T> view(const void *pool, const PatchRow &pr) {
  const T *q = reinterpret_cast<const T *>(pool) + pr.q_off + 2 * (int64_t)pr.ld + pr.col0;
  return View<T>{q, q + pr.plane, q + 2 * pr.plane, pr.ld};
}

template <typename T>
__device__ inline T *cell_ptr(void *pool, const PatchRow &pr, int m, int i, int j) {
  return reinterpret_cast<T *>(pool) + pr.q_off + m * pr.plane + (int64_t)(j + 2) * pr.ld +
         pr.col0 + i;
}

// Terms at x-edge (e - 1/2, j): A-dQ, A+dQ, F~ (3 components each).
template <typename T, int LIM, class Q>
__device__ inline void xedge_terms(const Q &q, const Coef<T> &k, int e, int j, T am[3],
                                   T ap[3], T F[3]) {
  const T Z = k.Z;
  const T a1 = s1(Z, q.P(e, j) - q.P(e - 1, j), q.U(e, j) - q.U(e - 1, j));
  const T a2 = s2(Z, q.P(e, j) - q.P(e - 1, j), q.U(e, j) - q.U(e - 1, j));
  const T a1r = s1(Z, q.P(e + 1, j) - q.P(e, j), q.U(e + 1, j) - q.U(e, j));
  const T a2l = s2(Z, q.P(e - 1, j) - q.P(e - 2, j), q.U(e - 1, j) - q.U(e - 2, j));
  // y-fluctuation sums of the cells left (e-1) and right (e) of the edge
  const T ysl = s2(Z, q.P(e - 1, j) - q.P(e - 1, j - 1), q.V(e - 1, j) - q.V(e - 1, j - 1)) +
                s1(Z, q.P(e - 1, j + 1) - q.P(e - 1, j), q.V(e - 1, j + 1) - q.V(e - 1, j));
  const T ysr = s2(Z, q.P(e, j) - q.P(e, j - 1), q.V(e, j) - q.V(e, j - 1)) +
                s1(Z, q.P(e, j + 1) - q.P(e, j), q.V(e, j + 1) - q.V(e, j));
  T Fp, Fu;
  ftilde<T, LIM>(k, a1, a2, a1r, a2l, ysl, ysr, Fp, Fu);
  am[0] = k.h * a1, am[1] = -(k.hz * a1), am[2] = T(0);
  ap[0] = k.h * a2, ap[1] = k.hz * a2, ap[2] = T(0);
  F[0] = Fp, F[1] = Fu, F[2] = T(0);
}

// Terms at y-edge (i, f - 1/2): B-dQ, B+dQ, G~.
template <typename T, int LIM, class Q>
__device__ inline void yedge_terms(const Q &q, const Coef<T> &k, int i, int f, T bm[3],
                                   T bp[3], T G[3]) {
  const T Z = k.Z;
  const T b1 = s1(Z, q.P(i, f) - q.P(i, f - 1), q.V(i, f) - q.V(i, f - 1));
  const T b2 = s2(Z, q.P(i, f) - q.P(i, f - 1), q.V(i, f) - q.V(i, f - 1));
  const T b1u = s1(Z, q.P(i, f + 1) - q.P(i, f), q.V(i, f + 1) - q.V(i, f));
  const T b2d = s2(Z, q.P(i, f - 1) - q.P(i, f - 2), q.V(i, f - 1) - q.V(i, f - 2));
  const T xsl = s2(Z, q.P(i, f - 1) - q.P(i - 1, f - 1), q.U(i, f - 1) - q.U(i - 1, f - 1)) +
                s1(Z, q.P(i + 1, f - 1) - q.P(i, f - 1), q.U(i + 1, f - 1) - q.U(i, f - 1));
  const T xsh = s2(Z, q.P(i, f) - q.P(i - 1, f), q.U(i, f) - q.U(i - 1, f)) +
                s1(Z, q.P(i + 1, f) - q.P(i, f), q.U(i + 1, f) - q.U(i, f));
  T Gp, Gv;
  gtilde<T, LIM>(k, b1, b2, b1u, b2d, xsl, xsh, Gp, Gv);
  bm[0] = k.h * b1, bm[1] = T(0), bm[2] = -(k.hz * b1);
  bp[0] = k.h * b2, bp[1] = T(0), bp[2] = k.hz * b2;
  G[0] = Gp, G[1] = T(0), G[2] = Gv;
}

// Side of a fine patch an edge index falls on: edges are numbered left
// (my of them), right (my), bottom (mx), top (mx).
__host__ __device__ inline void side_of(int e, int mx, int my, int &side, int &idx) {
  if (e < my) { side = 0; idx = e; }
  else if (e < 2 * my) { side = 1; idx = e - my; }
  else if (e < 2 * my + mx) { side = 2; idx = e - 2 * my; }
  else { side = 3; idx = e - 2 * my - mx; }
}

// Coarse terms of interface edge e of one fine patch (numbered left, right
// over ncy, bottom, top over ncx) from the coarse state before the coarse
// step.
template <typename T, int LIM>
__device__ inline void coarse_edge(const CfArgs &a, const CfPlace &pl, const View<T> &q,
                                   const Coef<T> &k, int e) {
  int side, idx;
  side_of(e, pl.ncx, pl.ncy, side, idx);
  T m[3], pp[3], F[3];
  if (side < 2)
    xedge_terms<T, LIM>(q, k, side == 0 ? pl.ci0 : pl.ci0 + pl.ncx, pl.cj0 + idx, m, pp, F);
  else
    yedge_terms<T, LIM>(q, k, pl.ci0 + idx, side == 2 ? pl.cj0 : pl.cj0 + pl.ncy, m, pp, F);
  const bool low = side == 0 || side == 2;  // the fine patch is on the edge's right (upper) side
  double *o = a.pc + 3 * ((int64_t)pl.cedge0 + e);
  for (int c = 0; c < 3; ++c) o[c] = (low ? (double)m[c] : -(double)pp[c]) + (double)F[c];
}

// MC-limited slope from the one-sided differences.
template <typename T>
__device__ inline T mc_slope(T l, T r) {
  if (!(l * r > T(0))) return T(0);
  const T s = l > T(0) ? T(1) : T(-1);
  return s * fmin(fmin(T(2) * fabs(l), T(2) * fabs(r)), T(0.5) * fabs(l + r));
}

// Fine ghost values from the coarse level at t_n + alpha dt: linear in time
// between the two coarse states, then MC-limited linear in space inside the
// coarse cell holding the ghost.  Every caller evaluates a ghost with this
// one expression, so a ghost computed twice has the same bits.
template <typename T>
struct GhostSrc {
  View<T> qo, qn;
  T al, bl;
  int ci0, cj0, r;
  __device__ T q(int m, int ci, int cj) const {
    const T vo = m == 0 ? qo.P(ci, cj) : m == 1 ? qo.U(ci, cj) : qo.V(ci, cj);
    const T vn = m == 0 ? qn.P(ci, cj) : m == 1 ? qn.U(ci, cj) : qn.V(ci, cj);
    return bl * vo + al * vn;
  }
  // The coarse cell holding fine cell (i, j) and the fine cell's offsets from
  // its centre.
  __device__ void locate(int i, int j, int &ci, int &cj, T &xi, T &eta) const {
    const double X = ci0 + (i + 0.5) / r, Y = cj0 + (j + 0.5) / r;
    ci = (int)floor(X), cj = (int)floor(Y);
    xi = (T)(X - (ci + 0.5)), eta = (T)(Y - (cj + 0.5));
  }
  // The coarse cell's value at the fine time and its limited slopes, all
  // three components (the 30 coarse loads issued together).
  __device__ void slopes(int ci, int cj, T q0[3], T sx[3], T sy[3]) const {
    T c[3][5];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      c[m][0] = q(m, ci, cj);
      c[m][1] = q(m, ci - 1, cj);
      c[m][2] = q(m, ci + 1, cj);
      c[m][3] = q(m, ci, cj - 1);
      c[m][4] = q(m, ci, cj + 1);
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      q0[m] = c[m][0];
      sx[m] = mc_slope(q0[m] - c[m][1], c[m][2] - q0[m]);
      sy[m] = mc_slope(q0[m] - c[m][3], c[m][4] - q0[m]);
    }
  }
  // All three components of fine cell (i, j).
  __device__ void value3(int i, int j, T out[3]) const {
    int ci, cj;
    T xi, eta, q0[3], sx[3], sy[3];
    locate(i, j, ci, cj, xi, eta);
    slopes(ci, cj, q0, sx, sy);
#pragma unroll
    for (int m = 0; m < 3; ++m) out[m] = q0[m] + xi * sx[m] + eta * sy[m];
  }
};

template <typename T>
__device__ inline GhostSrc<T> ghost_src(const CfArgs &a, const CfPlace &pl, const PatchRow &cp,
                                        double alpha) {
  return GhostSrc<T>{view<T>(a.c_old, cp), view<T>(a.c_new, cp), (T)alpha, (T)(1.0 - alpha),
                     pl.ci0, pl.cj0, a.r};
}

// A fine ghost from the sibling that holds it, if one does (its current
// state: all fine patches are at the same fine step), else from the coarse
// level.  Siblings' interiors are read while ghosts are written: disjoint.
template <typename T>
struct FineGhost {
  GhostSrc<T> G;
  const CfCopy *cp;
  int n;
  const PatchRow *fpatch;
  const void *f_cur;
  // The ghost's value from a sibling holding it; false if none does.
  __device__ bool sibling3(int i, int j, T out[3]) const {
    for (int c = 0; c < n; ++c) {
      const CfCopy k = cp[c];
      if (i >= k.i0 && i < k.i1 && j >= k.j0 && j < k.j1) {
        const View<T> s = view<T>(f_cur, fpatch[k.src]);
        out[0] = s.P(i + k.di, j + k.dj), out[1] = s.U(i + k.di, j + k.dj),
        out[2] = s.V(i + k.di, j + k.dj);
        return true;
      }
    }
    return false;
  }
  __device__ void value3(int i, int j, T out[3]) const {
    if (!sibling3(i, j, out)) G.value3(i, j, out);
  }
};

// Floor division by a positive divisor.
__device__ inline int fdiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Coarse cells a block of the fine-step kernel stages for its ghosts: the
// coarse cells under a range of at most 4 fine indices one way and S + 4 the
// other, with one coarse cell of stencil on every side.
__host__ __device__ inline int cf_box_cells(int S, int r) {
  return ((3 + r - 1) / r + 3) * ((S + 3 + r - 1) / r + 3);
}

// Every ghost cell (outside the mx x my interior) of the fine rectangle
// [ia, ib) x [ja, jb), each handed to sink(i, j, v): a sibling's value where
// one holds it, else the coarse level's.  The block's coarse neighbourhood
// is staged in LDS first: every coarse cell of the box around the region's
// coarse cells is read once, at the fine time (GhostSrc::q's expression), by
// the whole block.  Then one thread per coarse cell evaluates the fine ghosts
// inside it (2r of them along a side for r >= 2), taking the limited slopes
// from LDS with GhostSrc::slopes' expressions, so every ghost has the same
// bits as FineGhost::value3 gives it.  box: at least 3 cf_box_cells(S, r)
// elements for the block's S threads.  Every thread of the block must call
// it.
template <typename T, class Sink>
__device__ inline void ghost_region_staged(const FineGhost<T> &F, int mx, int my, int ia, int ib,
                                           int ja, int jb, T *box, Sink &&sink) {
  const GhostSrc<T> &G = F.G;
  const int r = G.r;
  const int CIa = fdiv(2 * ia + 1, 2 * r), CIb = fdiv(2 * (ib - 1) + 1, 2 * r);
  const int CJa = fdiv(2 * ja + 1, 2 * r), CJb = fdiv(2 * (jb - 1) + 1, 2 * r);
  const int nI = CIb - CIa + 1, nJ = CJb - CJa + 1;
  // the box: coarse cells (CIa - 1 .. CIb + 1) x (CJa - 1 .. CJb + 1), relative
  const int bw = nI + 2, bh = nJ + 2;
  for (int k = (int)threadIdx.x; k < bw * bh; k += (int)blockDim.x) {
    const int ci = G.ci0 + CIa - 1 + k % bw, cj = G.cj0 + CJa - 1 + k / bw;
#pragma unroll
    for (int m = 0; m < 3; ++m) box[m * bw * bh + k] = G.q(m, ci, cj);
  }
  __syncthreads();
  auto at = [&](int m, int ci, int cj) {  // absolute coarse indices
    return box[m * bw * bh + (cj - G.cj0 - CJa + 1) * bw + (ci - G.ci0 - CIa + 1)];
  };
  for (int k = (int)threadIdx.x; k < nI * nJ; k += (int)blockDim.x) {
    const int I = CIa + k % nI, J = CJa + k / nI;
    const int i0 = max(ia, I * r), i1 = min(ib, I * r + r);
    const int j0 = max(ja, J * r), j1 = min(jb, J * r + r);
    T q0[3], sx[3], sy[3];
    bool have = false;
    for (int j = j0; j < j1; ++j)
      for (int i = i0; i < i1; ++i) {
        if (i >= 0 && i < mx && j >= 0 && j < my) continue;
        T v[3];
        if (!F.sibling3(i, j, v)) {
          int ci, cj;
          T xi, eta;
          G.locate(i, j, ci, cj, xi, eta);
          if (!have) {
#pragma unroll
            for (int m = 0; m < 3; ++m) {
              q0[m] = at(m, ci, cj);
              sx[m] = mc_slope(q0[m] - at(m, ci - 1, cj), at(m, ci + 1, cj) - q0[m]);
              sy[m] = mc_slope(q0[m] - at(m, ci, cj - 1), at(m, ci, cj + 1) - q0[m]);
            }
            have = true;
          }
#pragma unroll
          for (int m = 0; m < 3; ++m) v[m] = q0[m] + xi * sx[m] + eta * sy[m];
        }
        sink(i, j, v);
      }
  }
}

template <typename T>
__device__ inline FineGhost<T> fine_ghost(const CfArgs &a, const CfPlace &pl, const PatchRow &cp,
                                          double alpha) {
  return FineGhost<T>{ghost_src<T>(a, pl, cp, alpha), a.copy + pl.copy0, pl.ncopy, a.fpatch,
                      a.f_cur};
}

// The whole ghost ring of each fine patch (used alone by ws_cf_fill_fine_ghosts).
template <typename T>
__global__ __launch_bounds__(kThreads) void cf_ghosts_kernel(CfArgs a, double alpha) {
  const CfPlace pl = a.place[blockIdx.y];
  const PatchRow fp = a.fpatch[blockIdx.y];
  const PatchRow cp = a.cpatch[pl.coarse];
  const FineGhost<T> G = fine_ghost<T>(a, pl, cp, alpha);
  const int mx = fp.mx, my = fp.my;
  const int ring = 4 * (mx + 4) + 4 * my;
  for (int g = blockIdx.x * kThreads + threadIdx.x; g < ring; g += gridDim.x * kThreads) {
    int i, j;
    if (g < 2 * (mx + 4)) {  // rows -2, -1
      j = g / (mx + 4) - 2, i = g % (mx + 4) - 2;
    } else if (g < 4 * (mx + 4)) {  // rows my, my+1
      const int h = g - 2 * (mx + 4);
      j = my + h / (mx + 4), i = h % (mx + 4) - 2;
    } else {  // columns -2, -1, mx, mx+1 of the interior rows
      const int h = g - 4 * (mx + 4);
      j = h / 4;
      const int c = h % 4;
      i = c < 2 ? c - 2 : mx + c - 2;
    }
    T v[3];
    G.value3(i, j, v);
    for (int m = 0; m < 3; ++m) *cell_ptr<T>(a.f_cur, fp, m, i, j) = v[m];
  }
}

// A strip of a fine patch staged in LDS for the edges of one side: for a
// left or right side the columns e-2 .. e+1 of rows j0-1 .. j0+n (the cells
// of a column of edges are strided in memory); for a bottom or top side the
// rows f-2 .. f+1 of columns i0-1 .. i0+n, n the block's edges (at most the
// strip length S, so the pitch of a component is S + 2 rows or columns of
// 4).  Ghost cells are evaluated from the coarse level (or a sibling),
// interior cells read from the fine state.
constexpr int kStrip = kThreads;  // most edges per block of the fine-step kernel
template <typename T>
struct StripX {
  const T *s;  // [3][S + 2][4]: row-major in (row, column)
  int e, j0, pitch;
  __device__ T at(int m, int i, int j) const {
    return s[(m * pitch + (j - j0 + 1)) * 4 + (i - e + 2)];
  }
  __device__ T P(int i, int j) const { return at(0, i, j); }
  __device__ T U(int i, int j) const { return at(1, i, j); }
  __device__ T V(int i, int j) const { return at(2, i, j); }
};
template <typename T>
struct StripY {
  const T *s;  // [3][S + 2][4]: column-major in (column, row)
  int i0, f, pitch;
  __device__ T at(int m, int i, int j) const {
    return s[(m * pitch + (i - i0 + 1)) * 4 + (j - f + 2)];
  }
  __device__ T P(int i, int j) const { return at(0, i, j); }
  __device__ T U(int i, int j) const { return at(1, i, j); }
  __device__ T V(int i, int j) const { return at(2, i, j); }
};

// Fine terms of one boundary edge (ghost (gi, gj); cP, cN the pressure and
// normal velocity of the coarse cell O outside it at t_n) written to the
// edge's slot of this fine step; on the last of the r fine steps the
// earlier steps' terms are added in step order and the total goes to the
// first step's slot, where the fix reads it.
template <typename T, int LIM, class Q>
__device__ inline void fine_edge(const Q &q, T cP, T cN, const Coef<T> &k, bool xdir, bool low,
                                 int e_or_i, int j_or_f, int gi, int gj, double *o, int step,
                                 int r, int64_t slot) {
  T m[3], pp[3], F[3];
  if (xdir)
    xedge_terms<T, LIM>(q, k, e_or_i, j_or_f, m, pp, F);
  else
    yedge_terms<T, LIM>(q, k, e_or_i, j_or_f, m, pp, F);
  // C1: f(ghost) - f(Q_O^n), the fluctuation sum of the Riemann problem
  // between the coarse cell and the fine ghost
  const T dp = q.P(gi, gj) - cP;
  T c1[3];
  if (xdir) {
    const T du = q.U(gi, gj) - cN;
    const T w1 = s1(k.Z, dp, du), w2 = s2(k.Z, dp, du);
    c1[0] = k.h * (w1 + w2), c1[1] = k.hz * (w2 - w1), c1[2] = T(0);
  } else {
    const T dv = q.V(gi, gj) - cN;
    const T w1 = s1(k.Z, dp, dv), w2 = s2(k.Z, dp, dv);
    c1[0] = k.h * (w1 + w2), c1[1] = T(0), c1[2] = k.hz * (w2 - w1);
  }
  // the ghost is the edge's left (lower) state on the left (bottom) side
  double v[3];
  for (int c = 0; c < 3; ++c)
    v[c] = (double)c1[c] + (low ? (double)m[c] : -(double)pp[c]) + (double)F[c];
  if (step == r - 1 && r > 1) {
    double *o0 = o - step * slot;  // the first fine step's slot of this edge
    for (int c = 0; c < 3; ++c) {
      double t = o0[c];
      for (int st = 1; st < r - 1; ++st) t = t + o0[st * slot + c];
      o0[c] = t + v[c];
    }
  } else {
    for (int c = 0; c < 3; ++c) o[c] = v[c];
  }
}

// Blocks per fine patch of the fine-step kernel (blocks of S threads, S
// boundary edges each): ceil(my/S) for each of the left and right sides,
// ceil(mx/S) for each of the bottom and top sides, and (first fine step
// only) ceil(2 (ncx + ncy)/S) for the coarse interface edges.
__host__ __device__ inline int cf_step_blocks(int mx, int my, int ncx, int ncy, bool coarse,
                                              int S) {
  return 2 * ((my + S - 1) / S) + 2 * ((mx + S - 1) / S) +
         (coarse ? (2 * (ncx + ncy) + S - 1) / S : 0);
}

// Before fine step k: the fine ghost ring at t_n + k dt/r (each block writes
// the ghosts of its side's range), the fine terms at every boundary edge, and
// for k = 0 the coarse interface terms from the coarse state at t_n.
template <typename T, int LIM>
__global__ __launch_bounds__(kThreads) void cf_fine_step_kernel(CfArgs a, int step,
                                                                double dt_fine, double dt) {
  extern __shared__ char smem[];
  T *strip = reinterpret_cast<T *>(smem);  // [3][S + 2][4]
  const int S = a.strip, pitch = S + 2;
  T *box = strip + 3 * pitch * 4;  // [3][cf_box_cells(S, r)]: the staged coarse cells
  const CfPlace pl = a.place[blockIdx.y];
  const PatchRow fp = a.fpatch[blockIdx.y];
  const int mx = fp.mx, my = fp.my, r = a.r;
  const int nxb = (my + S - 1) / S, nyb = (mx + S - 1) / S;
  int b = blockIdx.x;
  if (b >= cf_step_blocks(mx, my, pl.ncx, pl.ncy, step == 0, S)) return;
  const PatchRow cp = a.cpatch[pl.coarse];
  const View<T> co = view<T>(a.c_old, cp);
  const int t = threadIdx.x;
  if (b >= 2 * nxb + 2 * nyb) {
    // coarse interface edges, from the coarse state before its step
    const InstRow ic = a.cinst[cp.inst];
    const Coef<T> kc = make_coef<T>(ic.c, ic.Z, dt, cp.dx, cp.dy);
    const int e = (b - 2 * nxb - 2 * nyb) * S + t;
    if (e < 2 * (pl.ncx + pl.ncy)) coarse_edge<T, LIM>(a, pl, co, kc, e);
    return;
  }
  // this fine step's slots of the patch's boundary edges
  double *acc = a.acc + 3 * ((int64_t)step * a.n_fedges + pl.fedge0);
  const InstRow in = a.finst[fp.inst];
  const Coef<T> k = make_coef<T>(in.c, in.Z, dt_fine, fp.dx, fp.dy);
  const View<T> q = view<T>(a.f_cur, fp);
  const FineGhost<T> G = fine_ghost<T>(a, pl, cp, (double)step / r);
  if (b < 2 * nxb) {
    // left (e = 0) or right (e = mx) side, rows j0 .. j1-1: the strip holds
    // columns e-2 .. e+1 of rows j0-1 .. j1; the block owns the side's two
    // ghost columns of its rows
    const bool left = b < nxb;
    const int j0 = (left ? b : b - nxb) * S, j1 = min(j0 + S, my);
    const int e = left ? 0 : mx;
    // the coarse cell outside this thread's edge at t_n, loaded ahead
    const int j = j0 + t;
    const int oi = left ? pl.ci0 - 1 : pl.ci0 + pl.ncx, oj = pl.cj0 + min(j, my - 1) / r;
    const T cP = co.P(oi, oj), cN = co.U(oi, oj);
    const int rows = j1 - j0 + 2;
    for (int x = t; x < rows * 4; x += S) {
      const int jj = j0 - 1 + x / 4, i = e - 2 + x % 4;
      if (i >= 0 && i < mx && jj >= 0 && jj < my)
        for (int m = 0; m < 3; ++m)
          strip[(m * pitch + (jj - j0 + 1)) * 4 + (i - e + 2)] =
              m == 0 ? q.P(i, jj) : m == 1 ? q.U(i, jj) : q.V(i, jj);
    }
    ghost_region_staged<T>(G, mx, my, e - 2, e + 2, j0 - 1, j1 + 1, box,
                           [&](int i, int jj, const T v[3]) {
      for (int m = 0; m < 3; ++m) strip[(m * pitch + (jj - j0 + 1)) * 4 + (i - e + 2)] = v[m];
      if ((left ? i < 0 : i >= mx) && jj >= j0 && jj < j1)
        for (int m = 0; m < 3; ++m) *cell_ptr<T>(a.f_cur, fp, m, i, jj) = v[m];
    });
    __syncthreads();
    if (j < j1) {
      const StripX<T> Sx{strip, e, j0, pitch};
      fine_edge<T, LIM>(Sx, cP, cN, k, true, left, e, j, left ? -1 : mx, j,
                        acc + 3 * (left ? j : my + j), step, r, 3 * a.n_fedges);
    }
  } else {
    // bottom (f = 0) or top (f = my) side, columns i0 .. i1-1: the strip holds
    // rows f-2 .. f+1 of columns i0-1 .. i1; the block owns the side's two
    // ghost rows over its columns, and the corner columns for the first and
    // last block of the side
    b -= 2 * nxb;
    const bool bottom = b < nyb;
    const int c = bottom ? b : b - nyb;
    const int i0 = c * S, i1 = min(i0 + S, mx);
    const int f = bottom ? 0 : my;
    const int i = i0 + t;
    const int oi = pl.ci0 + min(i, mx - 1) / r, oj = bottom ? pl.cj0 - 1 : pl.cj0 + pl.ncy;
    const T cP = co.P(oi, oj), cN = co.V(oi, oj);
    const int lo = c == 0 ? -2 : i0, hi = i1 == mx ? mx + 2 : i1;
    const int cols = i1 - i0 + 2;
    for (int x = t; x < cols * 4; x += S) {
      const int j = f - 2 + x / cols, ii = i0 - 1 + x % cols;  // consecutive columns
      if (ii >= 0 && ii < mx && j >= 0 && j < my)
        for (int m = 0; m < 3; ++m)
          strip[(m * pitch + (ii - i0 + 1)) * 4 + (j - f + 2)] =
              m == 0 ? q.P(ii, j) : m == 1 ? q.U(ii, j) : q.V(ii, j);
    }
    ghost_region_staged<T>(G, mx, my, min(lo, i0 - 1), max(hi, i1 + 1), f - 2, f + 2, box,
                           [&](int ii, int j, const T v[3]) {
      if (ii >= i0 - 1 && ii <= i1)
        for (int m = 0; m < 3; ++m) strip[(m * pitch + (ii - i0 + 1)) * 4 + (j - f + 2)] = v[m];
      if ((bottom ? j < 0 : j >= my) && ii >= lo && ii < hi)
        for (int m = 0; m < 3; ++m) *cell_ptr<T>(a.f_cur, fp, m, ii, j) = v[m];
    });
    __syncthreads();
    if (i < i1) {
      const StripY<T> Sy{strip, i0, f, pitch};
      fine_edge<T, LIM>(Sy, cP, cN, k, false, bottom, i, f, i, bottom ? -1 : my,
                        acc + 3 * (2 * my + (bottom ? i : mx + i)), step, r, 3 * a.n_fedges);
    }
  }
}

// After the fine steps: updating (each covered coarse cell takes the mean of
// its r x r fine cells; blocks p * nav .. p * nav + nav - 1 for fine patch p)
// and the conservation fix (the blocks after those, one thread per cell of
// the fix list).  The two write disjoint coarse cells (fix cells are covered
// by no fine patch).
__host__ __device__ inline int cf_finish_blocks(int ncx, int ncy) {
  return (ncx * ncy + kThreads - 1) / kThreads;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void cf_finish_kernel(CfArgs a, double dt, int nav) {
  const int r = a.r;
  if ((int)blockIdx.x >= nav * a.n_fine) {
    const double w = 1.0 / (double)(r * r);
    const int x = ((int)blockIdx.x - nav * a.n_fine) * kThreads + (int)threadIdx.x;
    if (x < a.n_fix) {
      const CfFix fx = a.fix[x];
      const PatchRow cp = a.cpatch[fx.coarse];
      double v[3];
      for (int m = 0; m < 3; ++m) v[m] = (double)*cell_ptr<T>(a.c_new, cp, m, fx.oi, fx.oj);
      for (int c = 0; c < fx.n; ++c) {
        const CfPlace pl = a.place[fx.patch[c]];
        const int e = fx.edge[c], mxf = pl.ncx * r, myf = pl.ncy * r;
        int side, idx;
        side_of(e, pl.ncx, pl.ncy, side, idx);
        // the r fine edges on this coarse edge, in the fine edge numbering;
        // the patch on the cell's right (top) takes -, on its left (bottom) +
        const int f0 = side == 0 ? idx * r
                       : side == 1 ? myf + idx * r
                       : side == 2 ? 2 * myf + idx * r
                                   : 2 * myf + mxf + idx * r;
        const double h = side == 0   ? -dt / cp.dx
                         : side == 1 ? dt / cp.dx
                         : side == 2 ? -dt / cp.dy
                                     : dt / cp.dy;
        const double *acc = a.acc + 3 * ((int64_t)pl.fedge0 + f0);
        const double *pc = a.pc + 3 * ((int64_t)pl.cedge0 + e);
        // each fine edge's first slot holds its terms summed over the r fine steps
        for (int m = 0; m < 3; ++m) {
          double s = 0.0;
          for (int bb = 0; bb < r; ++bb) s += acc[3 * bb + m];
          v[m] = v[m] + h * (w * s - pc[m]);
        }
      }
      for (int m = 0; m < 3; ++m) *cell_ptr<T>(a.c_new, cp, m, fx.oi, fx.oj) = (T)v[m];
    }
    return;
  }
  const int patch = (int)blockIdx.x / nav, b = (int)blockIdx.x % nav;
  const CfPlace pl = a.place[patch];
  if (b >= cf_finish_blocks(pl.ncx, pl.ncy)) return;
  const PatchRow cp = a.cpatch[pl.coarse];
  const PatchRow fp = a.fpatch[patch];
  const View<T> f = view<T>(a.f_cur, fp);
  const int cidx = b * kThreads + threadIdx.x;
  if (cidx >= pl.ncx * pl.ncy) return;
  const int I = cidx % pl.ncx, J = cidx / pl.ncx;
  // row by row, cell by cell, component by component
  double s[3] = {0.0, 0.0, 0.0};
  if (r <= 4) {
    // every load of the r x r block issued before the first addition
    T v[4][3][4];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) {
        const int i = I * r + min(aa, r - 1), j = J * r + min(bb, r - 1);
        v[bb][0][aa] = f.P(i, j), v[bb][1][aa] = f.U(i, j), v[bb][2][aa] = f.V(i, j);
      }
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int aa = 0; aa < 4; ++aa)
        if (bb < r && aa < r)
#pragma unroll
          for (int m = 0; m < 3; ++m) s[m] += (double)v[bb][m][aa];
    for (int m = 0; m < 3; ++m)
      *cell_ptr<T>(a.c_new, cp, m, pl.ci0 + I, pl.cj0 + J) = (T)(s[m] / (double)(r * r));
    return;
  }
  for (int bb = 0; bb < r; ++bb) {
    const int j = J * r + bb;
    for (int a0 = 0; a0 < r; a0 += 4) {
      T v[3][4];
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) {
        const int i = I * r + min(a0 + aa, r - 1);
        v[0][aa] = f.P(i, j), v[1][aa] = f.U(i, j), v[2][aa] = f.V(i, j);
      }
      for (int aa = 0; aa < 4 && a0 + aa < r; ++aa)
        for (int m = 0; m < 3; ++m) s[m] += (double)v[m][aa];
    }
  }
  for (int m = 0; m < 3; ++m)
    *cell_ptr<T>(a.c_new, cp, m, pl.ci0 + I, pl.cj0 + J) = (T)(s[m] / (double)(r * r));
}

inline dim3 cf_grid(int max_items, int n) {
  return dim3((unsigned)max(1, min(64, (max_items + kThreads - 1) / kThreads)), (unsigned)n);
}

template <typename T>
hipError_t fine_step_t(int limiter, const CfArgs &a, int step, double dt_fine, double dt,
                       int max_blocks, hipStream_t s) {
  const dim3 g((unsigned)max(1, max_blocks), (unsigned)a.n_fine);
  const dim3 block((unsigned)a.strip);  // one thread per edge of the block
  const size_t lds = 3 * ((size_t)(a.strip + 2) * 4 + cf_box_cells(a.strip, a.r)) * sizeof(T);
  switch (limiter) {
    case WS_LIM_NONE:
      hipLaunchKernelGGL((cf_fine_step_kernel<T, WS_LIM_NONE>), g, block, lds, s, a, step,
                         dt_fine, dt);
      break;
    case WS_LIM_VANLEER:
      hipLaunchKernelGGL((cf_fine_step_kernel<T, WS_LIM_VANLEER>), g, block, lds, s, a,
                         step, dt_fine, dt);
      break;
    default:
      hipLaunchKernelGGL((cf_fine_step_kernel<T, WS_LIM_MC>), g, block, lds, s, a, step,
                         dt_fine, dt);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cf_ghosts(int dtype, const CfArgs &a, double alpha, int max_items,
                            hipStream_t s) {
  const dim3 g = cf_grid(max_items, a.n_fine);
  if (dtype == WS_F32)
    hipLaunchKernelGGL(cf_ghosts_kernel<float>, g, dim3(kThreads), 0, s, a, alpha);
  else
    hipLaunchKernelGGL(cf_ghosts_kernel<double>, g, dim3(kThreads), 0, s, a, alpha);
  return hipGetLastError();
}

hipError_t launch_cf_fine_step(int dtype, int limiter, const CfArgs &a, int step, double dt_fine,
                               double dt, int max_blocks, hipStream_t s) {
  return dtype == WS_F32 ? fine_step_t<float>(limiter, a, step, dt_fine, dt, max_blocks, s)
                         : fine_step_t<double>(limiter, a, step, dt_fine, dt, max_blocks, s);
}

int cf_step_blocks_host(int mx, int my, int ncx, int ncy, bool coarse, int strip) {
  return cf_step_blocks(mx, my, ncx, ncy, coarse, strip);
}

int cf_strip_host(int max_side) {
  return max(64, min(kStrip, (max_side + 63) / 64 * 64));
}

int cf_finish_blocks_host(int ncx, int ncy) { return cf_finish_blocks(ncx, ncy); }

void cf_out_cell_host(const CfPlace &pl, int e, int &oi, int &oj) {
  int side, idx;
  side_of(e, pl.ncx, pl.ncy, side, idx);
  if (side == 0) oi = pl.ci0 - 1, oj = pl.cj0 + idx;
  else if (side == 1) oi = pl.ci0 + pl.ncx, oj = pl.cj0 + idx;
  else if (side == 2) oi = pl.ci0 + idx, oj = pl.cj0 - 1;
  else oi = pl.ci0 + idx, oj = pl.cj0 + pl.ncy;
}

hipError_t launch_cf_finish(int dtype, const CfArgs &a, double dt, int max_blocks,
                            hipStream_t s) {
  const int nav = max(1, max_blocks);
  const int64_t blocks = (int64_t)nav * a.n_fine + (a.n_fix + kThreads - 1) / kThreads;
  if (blocks < 1) return hipSuccess;
  const dim3 g((unsigned)blocks);
  if (dtype == WS_F32)
    hipLaunchKernelGGL(cf_finish_kernel<float>, g, dim3(kThreads), 0, s, a, dt, nav);
  else
    hipLaunchKernelGGL(cf_finish_kernel<double>, g, dim3(kThreads), 0, s, a, dt, nav);
  return hipGetLastError();
}

}  // namespace ws
