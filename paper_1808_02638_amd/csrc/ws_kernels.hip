// HIP kernels (gfx950) of the unsplit wave-propagation step for 2D linear
// acoustics, one AMR level per launch.
//
// Method (Qin, LeVeque & Motley, arXiv 1808.02638): update of Sec. 2.1
// eq. (2.3) with the acoustics matrices of Sec. 4.1 eq. (4.2), MC-limited
// wave corrections and transverse waves split from the first-order
// fluctuations (Sec. 2.1, Sec. 3.3); Courant number of Sec. 2.4 eq. (2.10)
// reduced over the level on the device (Sec. 3.2.2); time step of Sec. 2.5
// eq. (2.11).
//
// Closed forms used here (derived from the eigen-structure of A and B, with
// c = sqrt(K/rho), Z = rho c).  At an x-edge with jumps dp, du the two moving
// waves have UNSCALED strengths a1 = Z du - dp (speed -c) and a2 = Z du + dp
// (speed +c); the true strengths are a/(2Z) along r1 = (-Z,1,0), r2 = (Z,1,0).
// Then, for a cell with left edge L and right edge R:
//   X  = A+dQ_L + A-dQ_R        = (c/2 xs, c/(2Z) xd, 0),  xs = a2_L + a1_R, xd = a2_L - a1_R
//   Fc = normal correction at an edge = c(1-nu_x)/4 (a2~ - a1~, (a1~ + a2~)/Z, 0)
// with a~ the MC-limited strengths (the limiter is positively homogeneous, so
// it acts on the unscaled strengths directly).  The transverse split of X by B
// only involves X_p, and gives at the cell's bottom edge
//   G~_B = Gc_B - dt/(2dx) (B-X_j + B+X_{j-1})
//        = Gc_B - (dtdx c^2/8) (xs_{j-1} - xs_j, 0, (xs_j + xs_{j-1})/Z).
// The y-direction is the mirror image with (p, v) and B.  The update is
//   p' = p - dtdx (X_p + F~_R,p - F~_L,p) - dtdy (Y_p + G~_T,p - G~_B,p)
//   u' = u - dtdx (X_u + F~_R,u - F~_L,u)
//   v' = v - dtdy (Y_v + G~_T,v - G~_B,v).
// The speed-0 wave contributes nothing (no fluctuation, zero correction
// weight), so only the two moving waves are formed.
//
// Every quantity is computed by one expression whatever the tile or thread
// that computes it, and the library is built without FP contraction, so the
// result of a cell does not depend on the tiling or on batched vs per-patch
// launches (bitwise).

#include <hip/hip_runtime.h>

#include "ws_internal.h"
#include "../../include/wavestep.h"

namespace ws {
namespace {

// --------------------------------------------------------------------------
// Per-tile coefficients (computed in FP64, rounded once to T)
// --------------------------------------------------------------------------
template <typename T>
struct Coef {
  T Z;
  T h, hz;                // c/2, c/(2Z): fluctuation factors
  T fx, fxz, fy, fyz;     // c(1-nu)/4 and /Z: correction factors
  T gx, gxz, gy, gyz;     // dtdx c^2/8 and /Z: transverse factors
  T dtdx, dtdy;
};

template <typename T>
__device__ inline Coef<T> make_coef(double c, double Z, double dt, double dx, double dy) {
  const double dtdx = dt / dx, dtdy = dt / dy;
  const double fx = 0.25 * c * (1.0 - c * dtdx), fy = 0.25 * c * (1.0 - c * dtdy);
  const double gx = 0.125 * dtdx * c * c, gy = 0.125 * dtdy * c * c;
  Coef<T> k;
  k.Z = (T)Z;
  k.h = (T)(0.5 * c);
  k.hz = (T)(0.5 * c / Z);
  k.fx = (T)fx;
  k.fxz = (T)(fx / Z);
  k.fy = (T)fy;
  k.fyz = (T)(fy / Z);
  k.gx = (T)gx;
  k.gxz = (T)(gx / Z);
  k.gy = (T)gy;
  k.gyz = (T)(gy / Z);
  k.dtdx = (T)dtdx;
  k.dtdy = (T)dtdy;
  return k;
}

// --------------------------------------------------------------------------
// Limiter on unscaled strengths: psi(a, a_up) = phi(a_up/a) a.
// MC: minmod(2a, 2a_up, (a + a_up)/2), written branch-free.
// --------------------------------------------------------------------------
template <typename T, int LIM>
__device__ inline T limited(T a, T b) {
  if constexpr (LIM == WS_LIM_NONE) {
    return a;
  } else {
    const T ta = a + a, tb = b + b, m = (a + b) * T(0.5);
    const T lo = fmin(fmin(ta, tb), m);
    const T hi = fmax(fmax(ta, tb), m);
    return fmax(lo, T(0)) + fmin(hi, T(0));
  }
}

// MC branch taken: 0 -> 0, 1 -> (a+b)/2, 2 -> 2a, 3 -> 2b; ties -> lowest.
template <typename T>
__device__ inline unsigned mc_branch(T a, T b) {
  const bool same = (a > T(0) && b > T(0)) || (a < T(0) && b < T(0));
  if (!same) return 0u;
  const T m1 = fabs(a + b) * T(0.5), m2 = fabs(a) * T(2), m3 = fabs(b) * T(2);
  if (m1 <= m2 && m1 <= m3) return 1u;
  return (m2 <= m3) ? 2u : 3u;
}

// Strengths at an edge from the jumps of (p, normal velocity).
template <typename T>
__device__ inline T s1(T Z, T dp, T dn) { return fma(Z, dn, -dp); }
template <typename T>
__device__ inline T s2(T Z, T dp, T dn) { return fma(Z, dn, dp); }

// Padded planes of one patch, indexed by interior coordinates (i, j).
template <typename T>
struct Planes {
  const T *p, *u, *v;
  int64_t ld;
  __device__ T P(int i, int j) const { return p[(int64_t)j * ld + i]; }
  __device__ T U(int i, int j) const { return u[(int64_t)j * ld + i]; }
  __device__ T V(int i, int j) const { return v[(int64_t)j * ld + i]; }
};

struct CellMasks {
  unsigned own;    // bits of the cell's left x-edge (0-3) and bottom y-edge (4-7)
  unsigned right;  // bits 0-3 of the right x-edge (stored at cell i+1)
  unsigned top;    // bits 4-7 of the top y-edge (stored at cell j+1)
};

// The whole update of one interior cell from its 13-point footprint.
template <typename T, int LIM, bool MASKS>
__device__ inline void cell_update(const Planes<T> &q, int i, int j, const Coef<T> &k, T &pn,
                                   T &un, T &vn, CellMasks *mk) {
  const T Z = k.Z;
  // ---- x-edges of row j: LL = i-3/2, L = i-1/2, R = i+1/2, RR = i+3/2
  const T pm2 = q.P(i - 2, j), pm1 = q.P(i - 1, j), p0 = q.P(i, j), pp1 = q.P(i + 1, j),
          pp2 = q.P(i + 2, j);
  const T um2 = q.U(i - 2, j), um1 = q.U(i - 1, j), u0 = q.U(i, j), up1 = q.U(i + 1, j),
          up2 = q.U(i + 2, j);
  const T a2LL = s2(Z, pm1 - pm2, um1 - um2);
  const T a1L = s1(Z, p0 - pm1, u0 - um1), a2L = s2(Z, p0 - pm1, u0 - um1);
  const T a1R = s1(Z, pp1 - p0, up1 - u0), a2R = s2(Z, pp1 - p0, up1 - u0);
  const T a1RR = s1(Z, pp2 - pp1, up2 - up1);
  // ---- y-edges of column i: BB = j-3/2, B = j-1/2, T = j+1/2, TT = j+3/2
  const T qm2 = q.P(i, j - 2), qm1 = q.P(i, j - 1), qp1 = q.P(i, j + 1), qp2 = q.P(i, j + 2);
  const T vm2 = q.V(i, j - 2), vm1 = q.V(i, j - 1), v0 = q.V(i, j), vp1 = q.V(i, j + 1),
          vp2 = q.V(i, j + 2);
  const T b2BB = s2(Z, qm1 - qm2, vm1 - vm2);
  const T b1B = s1(Z, p0 - qm1, v0 - vm1), b2B = s2(Z, p0 - qm1, v0 - vm1);
  const T b1T = s1(Z, qp1 - p0, vp1 - v0), b2T = s2(Z, qp1 - p0, vp1 - v0);
  const T b1TT = s1(Z, qp2 - qp1, vp2 - vp1);

  // ---- normal corrections (limited waves)
  const T l1L = limited<T, LIM>(a1L, a1R), l2L = limited<T, LIM>(a2L, a2LL);
  const T l1R = limited<T, LIM>(a1R, a1RR), l2R = limited<T, LIM>(a2R, a2L);
  const T l1B = limited<T, LIM>(b1B, b1T), l2B = limited<T, LIM>(b2B, b2BB);
  const T l1T = limited<T, LIM>(b1T, b1TT), l2T = limited<T, LIM>(b2T, b2B);
  const T FcLp = k.fx * (l2L - l1L), FcLu = k.fxz * (l1L + l2L);
  const T FcRp = k.fx * (l2R - l1R), FcRu = k.fxz * (l1R + l2R);
  const T GcBp = k.fy * (l2B - l1B), GcBv = k.fyz * (l1B + l2B);
  const T GcTp = k.fy * (l2T - l1T), GcTv = k.fyz * (l1T + l2T);

  // ---- first-order fluctuations entering the cell
  const T xs0 = a2L + a1R, xd0 = a2L - a1R;
  const T ys0 = b2B + b1T, yd0 = b2B - b1T;
  // xs of the rows below and above (for the transverse split into G~)
  const T pdm = q.P(i - 1, j - 1), pdp = q.P(i + 1, j - 1);
  const T udm = q.U(i - 1, j - 1), udp = q.U(i + 1, j - 1);
  const T xsm = s2(Z, qm1 - pdm, q.U(i, j - 1) - udm) + s1(Z, pdp - qm1, udp - q.U(i, j - 1));
  const T pum = q.P(i - 1, j + 1), pup = q.P(i + 1, j + 1);
  const T uum = q.U(i - 1, j + 1), uup = q.U(i + 1, j + 1);
  const T xsp = s2(Z, qp1 - pum, q.U(i, j + 1) - uum) + s1(Z, pup - qp1, uup - q.U(i, j + 1));
  // ys of the columns left and right (for the transverse split into F~)
  const T vlm = q.V(i - 1, j - 1), vl0 = q.V(i - 1, j), vlp = q.V(i - 1, j + 1);
  const T ysl = s2(Z, pm1 - pdm, vl0 - vlm) + s1(Z, pum - pm1, vlp - vl0);
  const T vrm = q.V(i + 1, j - 1), vr0 = q.V(i + 1, j), vrp = q.V(i + 1, j + 1);
  const T ysr = s2(Z, pp1 - pdp, vr0 - vrm) + s1(Z, pup - pp1, vrp - vr0);

  // ---- corrections plus transverse waves
  const T FLp = FcLp - k.gy * (ysl - ys0), FLu = FcLu - k.gyz * (ys0 + ysl);
  const T FRp = FcRp - k.gy * (ys0 - ysr), FRu = FcRu - k.gyz * (ysr + ys0);
  const T GBp = GcBp - k.gx * (xsm - xs0), GBv = GcBv - k.gxz * (xs0 + xsm);
  const T GTp = GcTp - k.gx * (xs0 - xsp), GTv = GcTv - k.gxz * (xsp + xs0);

  // ---- flux-differencing update, eq. (2.3)
  pn = p0 - k.dtdx * (k.h * xs0 + (FRp - FLp)) - k.dtdy * (k.h * ys0 + (GTp - GBp));
  un = u0 - k.dtdx * (k.hz * xd0 + (FRu - FLu));
  vn = v0 - k.dtdy * (k.hz * yd0 + (GTv - GBv));

  if constexpr (MASKS) {
    mk->own = mc_branch(a1L, a1R) | (mc_branch(a2L, a2LL) << 2) | (mc_branch(b1B, b1T) << 4) |
              (mc_branch(b2B, b2BB) << 6);
    mk->right = mc_branch(a1R, a1RR) | (mc_branch(a2R, a2L) << 2);
    mk->top = (mc_branch(b1T, b1TT) << 4) | (mc_branch(b2T, b2B) << 6);
  }
}

// Store a new cell value and, on physical boundaries, its ghost images.
template <typename T>
__device__ inline void store_cell(T *op, T *ou, T *ov, int64_t ld, int i, int j, int mx, int my,
                                  int bc, T pn, T un, T vn) {
  int xi[5], yj[5];
  int nx = 0, ny = 0;
  xi[nx++] = i;
  yj[ny++] = j;
  if (bc == WS_BC_EXTRAP) {
    if (i == 0) { xi[nx++] = -1; xi[nx++] = -2; }
    if (i == mx - 1) { xi[nx++] = mx; xi[nx++] = mx + 1; }
    if (j == 0) { yj[ny++] = -1; yj[ny++] = -2; }
    if (j == my - 1) { yj[ny++] = my; yj[ny++] = my + 1; }
  } else if (bc == WS_BC_PERIODIC) {
    if (i < 2) xi[nx++] = mx + i;
    if (i >= mx - 2) xi[nx++] = i - mx;
    if (j < 2) yj[ny++] = my + j;
    if (j >= my - 2) yj[ny++] = j - my;
  }
  for (int b = 0; b < ny; ++b)
    for (int a = 0; a < nx; ++a) {
      const int64_t o = (int64_t)yj[b] * ld + xi[a];
      op[o] = pn;
      ou[o] = un;
      ov[o] = vn;
    }
}

__device__ inline unsigned long long dbits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// One tile of one patch.  Every thread of the workgroup reaches the barrier
// at the end (the persistent loop relies on it).
template <typename T, int LIM, bool MASKS>
__device__ inline void do_tile(const StepArgs &a, int t, double *s_red) {
  const TileEntry te = a.tiles[t];
  const PatchRow pr = a.patches[te.patch];
  const InstRow in = a.inst[pr.inst];
  const double dt = a.dt[pr.inst];
  const Coef<T> k = make_coef<T>(in.c, in.Z, dt, pr.dx, pr.dy);
  const int tw = pr.tw;
  const int rows_per_thread = pr.th / (kThreads / tw);
  const int lx = threadIdx.x % tw, ly = threadIdx.x / tw;
  const int i = te.tx * tw + lx;
  const int j0 = te.ty * pr.th + ly * rows_per_thread;
  const int j1 = min(j0 + rows_per_thread, pr.my);
  const int64_t org = pr.q_off + 2 * (int64_t)pr.ld + pr.col0;
  const T *qi = reinterpret_cast<const T *>(a.qin) + org;
  T *qo = reinterpret_cast<T *>(a.qout) + org;
  const Planes<T> q{qi, qi + pr.plane, qi + 2 * pr.plane, pr.ld};
  double cfl = 0.0;
  if (i < pr.mx && j0 < j1) {
    for (int j = j0; j < j1; ++j) {
      T pn, un, vn;
      CellMasks mk;
      cell_update<T, LIM, MASKS>(q, i, j, k, pn, un, vn, &mk);
      store_cell<T>(qo, qo + pr.plane, qo + 2 * pr.plane, pr.ld, i, j, pr.mx, pr.my, pr.bc, pn,
                    un, vn);
      if constexpr (MASKS) {
        uint8_t *m = a.masks + pr.mask_off;
        const int64_t mld = pr.mx + 1;
        m[(int64_t)j * mld + i] = (uint8_t)mk.own;
        if (i == pr.mx - 1) m[(int64_t)j * mld + i + 1] = (uint8_t)mk.right;
        if (j == pr.my - 1) m[(int64_t)(j + 1) * mld + i] = (uint8_t)mk.top;
      }
    }
    // Courant number of the edges this thread owns: speeds are +-c everywhere
    // in a homogeneous instance, so each edge gives c dt/dx or c dt/dy.
    cfl = fmax(in.c * (dt / pr.dx), in.c * (dt / pr.dy));
  }
  // ---- max reduction: wavefront shuffle, then LDS across the 4 wavefronts
  cfl = wave_max(cfl);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) s_red[wave] = cfl;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = s_red[0];
    for (int w = 1; w < kThreads / 64; ++w) m = fmax(m, s_red[w]);
    if (m > 0.0) {
      const unsigned long long b = dbits(m);
      atomicMax(a.cfl_level, b);
      atomicMax(&a.cfl_acc[pr.inst], b);
      atomicMax(&a.cfl_patch[te.patch], b);
    }
  }
  __syncthreads();
}

template <typename T, int LIM, bool MASKS>
__global__ __launch_bounds__(kThreads) void step_kernel(StepArgs a) {
  __shared__ int s_tile;
  __shared__ double s_red[kThreads / 64];
  if (!a.persistent) {
    const int t = a.tile_base + (int)blockIdx.x;
    if (t < a.n_tiles) do_tile<T, LIM, MASKS>(a, t, s_red);
    return;
  }
  for (;;) {
    if (threadIdx.x == 0) s_tile = (int)atomicAdd(&a.counters[0], 1u);
    __syncthreads();
    const int t = s_tile;
    if (t >= a.n_tiles) break;
    do_tile<T, LIM, MASKS>(a, t, s_red);  // ends with a barrier
  }
  // The last workgroup to retire rewinds the tile counter for the next launch:
  // every other workgroup has finished its final fetch before it retires.
  if (threadIdx.x == 0) {
    const unsigned done = atomicAdd(&a.counters[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&a.counters[0], 0u);
      atomicExch(&a.counters[1], 0u);
    }
  }
}

// --------------------------------------------------------------------------
// Ghost fill of the current state (physical boundaries only)
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void fill_ghosts_kernel(const PatchRow *patches, T *q) {
  const PatchRow pr = patches[blockIdx.y];
  if (pr.bc == WS_BC_NONE) return;
  const int wx = pr.mx + 4, wy = pr.my + 4;
  const int64_t org = pr.q_off + 2 * (int64_t)pr.ld + pr.col0;
  T *base = q + org;
  for (int idx = blockIdx.x * kThreads + threadIdx.x; idx < wx * wy;
       idx += gridDim.x * kThreads) {
    const int i = idx % wx - 2, j = idx / wx - 2;
    if (i >= 0 && i < pr.mx && j >= 0 && j < pr.my) continue;
    int si, sj;
    if (pr.bc == WS_BC_PERIODIC) {
      si = (i + pr.mx) % pr.mx;
      sj = (j + pr.my) % pr.my;
    } else {
      si = min(max(i, 0), pr.mx - 1);
      sj = min(max(j, 0), pr.my - 1);
    }
    const int64_t d = (int64_t)j * pr.ld + i, s = (int64_t)sj * pr.ld + si;
    for (int m = 0; m < 3; ++m) base[m * pr.plane + d] = base[m * pr.plane + s];
  }
}

// --------------------------------------------------------------------------
// dt and Courant-number bookkeeping
// --------------------------------------------------------------------------
__global__ void set_dt_kernel(double *dt, int n, double value) {
  for (int k = threadIdx.x; k < n; k += blockDim.x) dt[k] = value;
}

__global__ void finish_step_kernel(CflSlots c, double cfl_desired) {
  for (int k = threadIdx.x; k < c.n_inst; k += blockDim.x) {
    const double cfl = __longlong_as_double((long long)c.cfl_acc[k]);
    c.cfl_last[k] = cfl;
    c.cfl_max[k] = fmax(c.cfl_max[k], cfl);
    if (cfl_desired > 0.0 && cfl > 0.0) c.dt[k] = c.dt[k] * cfl_desired / cfl;
    c.cfl_acc[k] = 0ull;
  }
  for (int k = threadIdx.x; k < c.n_patches; k += blockDim.x) {
    c.cfl_patch_last[k] = __longlong_as_double((long long)c.cfl_patch_acc[k]);
    c.cfl_patch_acc[k] = 0ull;
  }
  if (threadIdx.x == 0) {
    c.level_last[0] = __longlong_as_double((long long)c.level_acc[0]);
    c.level_acc[0] = 0ull;
  }
}

// --------------------------------------------------------------------------
// Conservation sums: FP64 per-tile partials in a fixed order, then a fixed-
// order pass over the tile list per instance.
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void tile_sums_kernel(const PatchRow *patches,
                                                           const TileEntry *tiles, const T *q,
                                                           double *partials) {
  __shared__ double s[3][kThreads];
  const TileEntry te = tiles[blockIdx.x];
  const PatchRow pr = patches[te.patch];
  const int tw = pr.tw;
  const int rpt = pr.th / (kThreads / tw);
  const int lx = threadIdx.x % tw, ly = threadIdx.x / tw;
  const int i = te.tx * tw + lx;
  const int j0 = te.ty * pr.th + ly * rpt;
  const int j1 = min(j0 + rpt, pr.my);
  const int64_t org = pr.q_off + 2 * (int64_t)pr.ld + pr.col0;
  double acc[3] = {0.0, 0.0, 0.0};
  if (i < pr.mx)
    for (int j = j0; j < j1; ++j)
      for (int m = 0; m < 3; ++m) acc[m] += (double)q[org + m * pr.plane + (int64_t)j * pr.ld + i];
  for (int m = 0; m < 3; ++m) s[m][threadIdx.x] = acc[m];
  __syncthreads();
  for (int w = kThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int m = 0; m < 3; ++m) s[m][threadIdx.x] += s[m][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) partials[3 * (int64_t)blockIdx.x + threadIdx.x] = s[threadIdx.x][0] * pr.dx * pr.dy;
}

__global__ void instance_sums_kernel(const PatchRow *patches, const TileEntry *tiles, int n_tiles,
                                     const double *partials, int n_inst, double *sums) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_inst; k += gridDim.x * blockDim.x) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < n_tiles; ++t)
      if (patches[tiles[t].patch].inst == k)
        for (int m = 0; m < 3; ++m) acc[m] += partials[3 * (int64_t)t + m];
    for (int m = 0; m < 3; ++m) sums[3 * k + m] = acc[m];
  }
}

template <typename T, int LIM, bool MASKS>
hipError_t launch_step_t(const StepArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((step_kernel<T, LIM, MASKS>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <typename T, int LIM>
hipError_t launch_step_m(const StepArgs &a, int grid, hipStream_t s) {
  return a.masks ? launch_step_t<T, LIM, true>(a, grid, s) : launch_step_t<T, LIM, false>(a, grid, s);
}

template <typename T>
hipError_t launch_step_l(int limiter, const StepArgs &a, int grid, hipStream_t s) {
  return limiter == WS_LIM_NONE ? launch_step_m<T, WS_LIM_NONE>(a, grid, s)
                                : launch_step_m<T, WS_LIM_MC>(a, grid, s);
}

}  // namespace

hipError_t launch_step(int dtype, int limiter, const StepArgs &a, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  return dtype == WS_F32 ? launch_step_l<float>(limiter, a, grid, s)
                         : launch_step_l<double>(limiter, a, grid, s);
}

int step_occupancy(int dtype, int limiter, int *wg_per_cu) {
  int n = 0;
  hipError_t e;
  if (dtype == WS_F32)
    e = limiter == WS_LIM_NONE
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<float, WS_LIM_NONE, false>, kThreads, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<float, WS_LIM_MC, false>, kThreads, 0);
  else
    e = limiter == WS_LIM_NONE
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<double, WS_LIM_NONE, false>, kThreads, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<double, WS_LIM_MC, false>, kThreads, 0);
  *wg_per_cu = n;
  return e == hipSuccess ? 0 : -1;
}

hipError_t launch_fill_ghosts(int dtype, const PatchRow *patches, int n_patches,
                              int max_padded_cells, void *q, hipStream_t s) {
  if (n_patches <= 0) return hipSuccess;
  const int gx = min(64, (max_padded_cells + kThreads - 1) / kThreads);
  const dim3 grid(max(gx, 1), n_patches);
  if (dtype == WS_F32)
    hipLaunchKernelGGL(fill_ghosts_kernel<float>, grid, dim3(kThreads), 0, s, patches,
                       reinterpret_cast<float *>(q));
  else
    hipLaunchKernelGGL(fill_ghosts_kernel<double>, grid, dim3(kThreads), 0, s, patches,
                       reinterpret_cast<double *>(q));
  return hipGetLastError();
}

hipError_t launch_set_dt(const CflSlots &c, double value, hipStream_t s) {
  hipLaunchKernelGGL(set_dt_kernel, dim3(1), dim3(256), 0, s, c.dt, c.n_inst, value);
  return hipGetLastError();
}

hipError_t launch_finish_step(const CflSlots &c, double cfl_desired, hipStream_t s) {
  hipLaunchKernelGGL(finish_step_kernel, dim3(1), dim3(1024), 0, s, c, cfl_desired);
  return hipGetLastError();
}

hipError_t launch_sums(int dtype, const PatchRow *patches, const TileEntry *tiles, int n_tiles,
                       const void *q, double *partials, int n_inst, double *sums, hipStream_t s) {
  if (n_tiles > 0) {
    if (dtype == WS_F32)
      hipLaunchKernelGGL(tile_sums_kernel<float>, dim3(n_tiles), dim3(kThreads), 0, s, patches,
                         tiles, reinterpret_cast<const float *>(q), partials);
    else
      hipLaunchKernelGGL(tile_sums_kernel<double>, dim3(n_tiles), dim3(kThreads), 0, s, patches,
                         tiles, reinterpret_cast<const double *>(q), partials);
  }
  hipLaunchKernelGGL(instance_sums_kernel, dim3((n_inst + 63) / 64), dim3(64), 0, s, patches,
                     tiles, n_tiles, partials, n_inst, sums);
  return hipGetLastError();
}

}  // namespace ws
