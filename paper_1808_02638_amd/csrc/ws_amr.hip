// HIP kernels (gfx950) coupling a coarse level and the fine level nested in
// it: the pieces of one composite coarse step that are not the level step
// itself (paper Sec. 2.2 flow chart; Sec. 2.3 updating and conservation fix).
//
//   cf_coarse_terms: before the coarse step, the coarse terms at every
//     coarse-fine interface edge from Q_c^n, P_c = A-dQ + F~ (fine patch on
//     the edge's right) or -A+dQ + F~ (fine patch on its left), y alike;
//   cf_ghosts: the fine ghosts at t_n + alpha dt from the coarse level, linear
//     in time between Q_c^n and Q_c^{n+1} and MC-limited linear in space
//     inside the coarse cell that holds the ghost;
//   cf_fine_terms: before fine step k, the fine terms at the patch's boundary
//     edges, accumulated over the r fine steps: f(ghost) - f(Q_O^n) (the
//     Riemann fluctuation sum between the coarse cell O outside the edge and
//     the fine ghost next to it, C1) plus A-dQ^ + F~^ (left side) or
//     -A+dQ^ + F~^ (right side), y alike;
//   cf_average: each covered coarse cell takes the mean of its r x r fine
//     cells (updating);
//   cf_fix: each coarse cell O next to a fine patch replaces the coarse flux
//     through their shared edge by the mean of the fine fluxes:
//     O -= dt/dx ((1/r^2) sum acc - P_c) when the patch is on O's right,
//     O += dt/dx ((1/r^2) sum acc - P_c) when it is on O's left (y alike).
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
__device__ inline void side_of(int e, int mx, int my, int &side, int &idx) {
  if (e < my) { side = 0; idx = e; }
  else if (e < 2 * my) { side = 1; idx = e - my; }
  else if (e < 2 * my + mx) { side = 2; idx = e - 2 * my; }
  else { side = 3; idx = e - 2 * my - mx; }
}

template <typename T, int LIM>
__global__ __launch_bounds__(kThreads) void cf_coarse_terms_kernel(CfArgs a, const void *qc,
                                                                   double dt) {
  const CfPlace pl = a.place[blockIdx.y];
  const PatchRow cp = a.cpatch[pl.coarse];
  const InstRow in = a.cinst[cp.inst];
  const Coef<T> k = make_coef<T>(in.c, in.Z, dt, cp.dx, cp.dy);
  const View<T> q = view<T>(qc, cp);
  const int n = 2 * (pl.ncx + pl.ncy);
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < n; e += gridDim.x * kThreads) {
    int side, idx;
    side_of(e, pl.ncx, pl.ncy, side, idx);
    T m[3], pp[3], F[3];
    double out[3];
    if (side < 2) {
      const int edge = side == 0 ? pl.ci0 : pl.ci0 + pl.ncx;
      xedge_terms<T, LIM>(q, k, edge, pl.cj0 + idx, m, pp, F);
      for (int c = 0; c < 3; ++c)
        out[c] = side == 0 ? (double)m[c] + (double)F[c] : -(double)pp[c] + (double)F[c];
    } else {
      const int edge = side == 2 ? pl.cj0 : pl.cj0 + pl.ncy;
      yedge_terms<T, LIM>(q, k, pl.ci0 + idx, edge, m, pp, F);
      for (int c = 0; c < 3; ++c)
        out[c] = side == 2 ? (double)m[c] + (double)F[c] : -(double)pp[c] + (double)F[c];
    }
    double *o = a.pc + 3 * ((int64_t)pl.cedge0 + e);
    o[0] = out[0], o[1] = out[1], o[2] = out[2];
  }
}

// MC-limited slope from the one-sided differences.
template <typename T>
__device__ inline T mc_slope(T l, T r) {
  if (!(l * r > T(0))) return T(0);
  const T s = l > T(0) ? T(1) : T(-1);
  return s * fmin(fmin(T(2) * fabs(l), T(2) * fabs(r)), T(0.5) * fabs(l + r));
}

template <typename T>
__global__ __launch_bounds__(kThreads) void cf_ghosts_kernel(CfArgs a, double alpha) {
  const CfPlace pl = a.place[blockIdx.y];
  const PatchRow fp = a.fpatch[blockIdx.y];
  const PatchRow cp = a.cpatch[pl.coarse];
  const View<T> qo = view<T>(a.c_old, cp), qn = view<T>(a.c_new, cp);
  const int mx = fp.mx, my = fp.my, r = a.r;
  const int ring = 4 * (mx + 4) + 4 * my;
  const T al = (T)alpha, bl = (T)(1.0 - alpha);
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
    // fine centre in coarse index units, its coarse cell and offset
    const double X = pl.ci0 + (i + 0.5) / r, Y = pl.cj0 + (j + 0.5) / r;
    const int ci = (int)floor(X), cj = (int)floor(Y);
    const T xi = (T)(X - (ci + 0.5)), eta = (T)(Y - (cj + 0.5));
    for (int m = 0; m < 3; ++m) {
      auto at = [&](int di, int dj) {
        const View<T> &o = qo;
        const T vo = m == 0 ? o.P(ci + di, cj + dj) : m == 1 ? o.U(ci + di, cj + dj) : o.V(ci + di, cj + dj);
        const T vn = m == 0 ? qn.P(ci + di, cj + dj) : m == 1 ? qn.U(ci + di, cj + dj) : qn.V(ci + di, cj + dj);
        return bl * vo + al * vn;
      };
      const T q0 = at(0, 0);
      const T sx = mc_slope(q0 - at(-1, 0), at(1, 0) - q0);
      const T sy = mc_slope(q0 - at(0, -1), at(0, 1) - q0);
      *cell_ptr<T>(a.f_cur, fp, m, i, j) = q0 + xi * sx + eta * sy;
    }
  }
}

// Columns e-2 .. e+1 of rows j0-1 .. j0+kStrip of one patch, staged in LDS
// for the edges of a left or right side (a column of edges: their cells are
// strided in memory, so the block reads the strip row by row instead).
constexpr int kStrip = kThreads;  // edges per block
template <typename T>
struct Strip {
  const T *s;  // [3][kStrip + 2][4]
  int e, j0;
  __device__ T at(int m, int i, int j) const {
    return s[(m * (kStrip + 2) + (j - j0 + 1)) * 4 + (i - e + 2)];
  }
  __device__ T P(int i, int j) const { return at(0, i, j); }
  __device__ T U(int i, int j) const { return at(1, i, j); }
  __device__ T V(int i, int j) const { return at(2, i, j); }
};

// Blocks of one fine patch: ceil(my/kStrip) for each of the left and right
// sides, then ceil(mx/kStrip) for each of the bottom and top sides.
__device__ inline int cf_side_blocks(int mx, int my) {
  return 2 * ((my + kStrip - 1) / kStrip) + 2 * ((mx + kStrip - 1) / kStrip);
}

// Fine terms of one boundary edge (ghost (gi, gj), coarse cell (oi, oj)
// outside it) added to its accumulator slot.
template <typename T, int LIM, class Q>
__device__ inline void fine_edge(const CfArgs &a, const Q &q, const View<T> &co,
                                 const Coef<T> &k, bool xdir, bool low, int e_or_i, int j_or_f,
                                 int gi, int gj, int oi, int oj, int step, double *o) {
  T m[3], pp[3], F[3];
  if (xdir)
    xedge_terms<T, LIM>(q, k, e_or_i, j_or_f, m, pp, F);
  else
    yedge_terms<T, LIM>(q, k, e_or_i, j_or_f, m, pp, F);
  // C1: f(ghost) - f(Q_O^n), the fluctuation sum of the Riemann problem
  // between the coarse cell and the fine ghost
  const T dp = q.P(gi, gj) - co.P(oi, oj);
  T c1[3];
  if (xdir) {
    const T du = q.U(gi, gj) - co.U(oi, oj);
    const T w1 = s1(k.Z, dp, du), w2 = s2(k.Z, dp, du);
    c1[0] = k.h * (w1 + w2), c1[1] = k.hz * (w2 - w1), c1[2] = T(0);
  } else {
    const T dv = q.V(gi, gj) - co.V(oi, oj);
    const T w1 = s1(k.Z, dp, dv), w2 = s2(k.Z, dp, dv);
    c1[0] = k.h * (w1 + w2), c1[1] = T(0), c1[2] = k.hz * (w2 - w1);
  }
  // the ghost is the edge's left (lower) state on the left (bottom) side
  for (int c = 0; c < 3; ++c) {
    const double v = (double)c1[c] + (low ? (double)m[c] : -(double)pp[c]) + (double)F[c];
    o[c] = step == 0 ? v : o[c] + v;
  }
}

template <typename T, int LIM>
__global__ __launch_bounds__(kThreads) void cf_fine_terms_kernel(CfArgs a, int step,
                                                                 double dt_fine) {
  __shared__ T strip[3 * (kStrip + 2) * 4];
  const CfPlace pl = a.place[blockIdx.y];
  const PatchRow fp = a.fpatch[blockIdx.y];
  const int mx = fp.mx, my = fp.my, r = a.r;
  int b = blockIdx.x;
  const int nxb = (my + kStrip - 1) / kStrip, nyb = (mx + kStrip - 1) / kStrip;
  if (b >= 2 * nxb + 2 * nyb) return;
  const PatchRow cp = a.cpatch[pl.coarse];
  const InstRow in = a.finst[fp.inst];
  const Coef<T> k = make_coef<T>(in.c, in.Z, dt_fine, fp.dx, fp.dy);
  const View<T> co = view<T>(a.c_old, cp);
  const int t = threadIdx.x;
  if (b < 2 * nxb) {
    // left (e = 0) or right (e = mx) side, rows j0 .. j1-1
    const bool left = b < nxb;
    const int j0 = (left ? b : b - nxb) * kStrip, j1 = min(j0 + kStrip, my);
    const int e = left ? 0 : mx;
    const View<T> q = view<T>(a.f_cur, fp);
    const int rows = j1 - j0 + 2;  // j0-1 .. j1
    for (int x = t; x < 3 * rows * 4; x += kThreads) {
      const int m = x / (rows * 4), rem = x % (rows * 4);
      const int j = j0 - 1 + rem / 4, i = e - 2 + rem % 4;
      const T v = m == 0 ? q.P(i, j) : m == 1 ? q.U(i, j) : q.V(i, j);
      strip[(m * (kStrip + 2) + (j - j0 + 1)) * 4 + (i - e + 2)] = v;
    }
    __syncthreads();
    const int j = j0 + t;
    if (j < j1) {
      const Strip<T> S{strip, e, j0};
      const int oi = left ? pl.ci0 - 1 : pl.ci0 + pl.ncx, oj = pl.cj0 + j / r;
      const int edge = left ? j : my + j;
      fine_edge<T, LIM>(a, S, co, k, true, left, e, j, left ? -1 : mx, j, oi, oj, step,
                        a.acc + 3 * ((int64_t)pl.fedge0 + edge));
    }
  } else {
    // bottom (f = 0) or top (f = my) side, columns i0 .. i1-1: rows of
    // cells, read directly (consecutive threads, consecutive columns)
    b -= 2 * nxb;
    const bool bottom = b < nyb;
    const int i = (bottom ? b : b - nyb) * kStrip + t;
    if (i < mx) {
      const View<T> q = view<T>(a.f_cur, fp);
      const int f = bottom ? 0 : my;
      const int oi = pl.ci0 + i / r, oj = bottom ? pl.cj0 - 1 : pl.cj0 + pl.ncy;
      const int edge = 2 * my + (bottom ? i : mx + i);
      fine_edge<T, LIM>(a, q, co, k, false, bottom, i, f, i, bottom ? -1 : my, oi, oj, step,
                        a.acc + 3 * ((int64_t)pl.fedge0 + edge));
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void cf_average_kernel(CfArgs a) {
  const CfPlace pl = a.place[blockIdx.y];
  const PatchRow fp = a.fpatch[blockIdx.y];
  const PatchRow cp = a.cpatch[pl.coarse];
  const int r = a.r, n = pl.ncx * pl.ncy;
  const View<T> f = view<T>(a.f_cur, fp);
  for (int c = blockIdx.x * kThreads + threadIdx.x; c < n; c += gridDim.x * kThreads) {
    const int I = c % pl.ncx, J = c / pl.ncx;
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < r; ++b)
      for (int aa = 0; aa < r; ++aa) {
        const int i = I * r + aa, j = J * r + b;
        s[0] += (double)f.P(i, j);
        s[1] += (double)f.U(i, j);
        s[2] += (double)f.V(i, j);
      }
    for (int m = 0; m < 3; ++m)
      *cell_ptr<T>(a.c_new, cp, m, pl.ci0 + I, pl.cj0 + J) = (T)(s[m] / (double)(r * r));
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void cf_fix_kernel(CfArgs a, double dt) {
  const CfPlace pl = a.place[blockIdx.y];
  const PatchRow cp = a.cpatch[pl.coarse];
  const int r = a.r, n = 2 * (pl.ncx + pl.ncy);
  const int mxf = pl.ncx * r, myf = pl.ncy * r;
  const double w = 1.0 / (double)(r * r);
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < n; e += gridDim.x * kThreads) {
    int side, idx;
    side_of(e, pl.ncx, pl.ncy, side, idx);
    // the r fine edges on this coarse edge, in the fine edge numbering
    int f0, oi, oj;
    double h;
    if (side == 0) f0 = idx * r, oi = pl.ci0 - 1, oj = pl.cj0 + idx, h = -dt / cp.dx;
    else if (side == 1) f0 = myf + idx * r, oi = pl.ci0 + pl.ncx, oj = pl.cj0 + idx, h = dt / cp.dx;
    else if (side == 2) f0 = 2 * myf + idx * r, oi = pl.ci0 + idx, oj = pl.cj0 - 1, h = -dt / cp.dy;
    else f0 = 2 * myf + mxf + idx * r, oi = pl.ci0 + idx, oj = pl.cj0 + pl.ncy, h = dt / cp.dy;
    const double *acc = a.acc + 3 * ((int64_t)pl.fedge0 + f0);
    const double *pc = a.pc + 3 * ((int64_t)pl.cedge0 + e);
    for (int m = 0; m < 3; ++m) {
      double s = 0.0;
      for (int b = 0; b < r; ++b) s += acc[3 * b + m];
      T *o = cell_ptr<T>(a.c_new, cp, m, oi, oj);
      *o = (T)((double)*o + h * (w * s - pc[m]));
    }
  }
}

inline dim3 cf_grid(int max_items, int n) {
  return dim3((unsigned)max(1, min(64, (max_items + kThreads - 1) / kThreads)), (unsigned)n);
}

template <typename T>
hipError_t coarse_terms_t(int limiter, const CfArgs &a, const void *qc, double dt, int max_items,
                          hipStream_t s) {
  const dim3 g = cf_grid(max_items, a.n_fine);
  switch (limiter) {
    case WS_LIM_NONE:
      hipLaunchKernelGGL((cf_coarse_terms_kernel<T, WS_LIM_NONE>), g, dim3(kThreads), 0, s, a, qc, dt);
      break;
    case WS_LIM_VANLEER:
      hipLaunchKernelGGL((cf_coarse_terms_kernel<T, WS_LIM_VANLEER>), g, dim3(kThreads), 0, s, a, qc, dt);
      break;
    default:
      hipLaunchKernelGGL((cf_coarse_terms_kernel<T, WS_LIM_MC>), g, dim3(kThreads), 0, s, a, qc, dt);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t fine_terms_t(int limiter, const CfArgs &a, int step, double dt_fine, int max_items,
                        hipStream_t s) {
  const dim3 g((unsigned)max(1, max_items), (unsigned)a.n_fine);
  switch (limiter) {
    case WS_LIM_NONE:
      hipLaunchKernelGGL((cf_fine_terms_kernel<T, WS_LIM_NONE>), g, dim3(kThreads), 0, s, a, step, dt_fine);
      break;
    case WS_LIM_VANLEER:
      hipLaunchKernelGGL((cf_fine_terms_kernel<T, WS_LIM_VANLEER>), g, dim3(kThreads), 0, s, a, step, dt_fine);
      break;
    default:
      hipLaunchKernelGGL((cf_fine_terms_kernel<T, WS_LIM_MC>), g, dim3(kThreads), 0, s, a, step, dt_fine);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cf_coarse_terms(int dtype, int limiter, const CfArgs &a, const void *qc,
                                  double dt, int max_items, hipStream_t s) {
  return dtype == WS_F32 ? coarse_terms_t<float>(limiter, a, qc, dt, max_items, s)
                         : coarse_terms_t<double>(limiter, a, qc, dt, max_items, s);
}

hipError_t launch_cf_ghosts(int dtype, const CfArgs &a, double alpha, int max_items,
                            hipStream_t s) {
  const dim3 g = cf_grid(max_items, a.n_fine);
  if (dtype == WS_F32)
    hipLaunchKernelGGL(cf_ghosts_kernel<float>, g, dim3(kThreads), 0, s, a, alpha);
  else
    hipLaunchKernelGGL(cf_ghosts_kernel<double>, g, dim3(kThreads), 0, s, a, alpha);
  return hipGetLastError();
}

hipError_t launch_cf_fine_terms(int dtype, int limiter, const CfArgs &a, int step, double dt_fine,
                                int max_items, hipStream_t s) {
  return dtype == WS_F32 ? fine_terms_t<float>(limiter, a, step, dt_fine, max_items, s)
                         : fine_terms_t<double>(limiter, a, step, dt_fine, max_items, s);
}

hipError_t launch_cf_average_fix(int dtype, const CfArgs &a, double dt, int max_cover,
                                 int max_cedges, hipStream_t s) {
  const dim3 ga = cf_grid(max_cover, a.n_fine), gf = cf_grid(max_cedges, a.n_fine);
  if (dtype == WS_F32) {
    hipLaunchKernelGGL(cf_average_kernel<float>, ga, dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(cf_fix_kernel<float>, gf, dim3(kThreads), 0, s, a, dt);
  } else {
    hipLaunchKernelGGL(cf_average_kernel<double>, ga, dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(cf_fix_kernel<double>, gf, dim3(kThreads), 0, s, a, dt);
  }
  return hipGetLastError();
}

}  // namespace ws
