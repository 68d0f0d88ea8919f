// HIP kernels (gfx950) of the unsplit wave-propagation step for 2D linear
// acoustics, one AMR level per launch.
//
// Method (Qin, LeVeque & Motley, arXiv 1808.02638): update of Sec. 2.1
// eq. (2.3) with the acoustics matrices of Sec. 4.1 eq. (4.2), limited
// wave corrections (MC, van Leer or none) and transverse waves split from the
// first-order fluctuations, or from the fluctuations with the limited
// corrections moved into them (Sec. 2.1, Sec. 3.3); Courant number of Sec. 2.4 eq. (2.10)
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

#include <climits>

#include "ws_device.h"
#include "ws_internal.h"
#include "../../include/wavestep.h"

namespace ws {
namespace {

// MC branch taken: 0 -> 0, 1 -> (a+b)/2, 2 -> 2a, 3 -> 2b; ties -> lowest.
template <typename T>
__device__ inline unsigned mc_branch(T a, T b) {
  const bool same = (a > T(0) && b > T(0)) || (a < T(0) && b < T(0));
  if (!same) return 0u;
  const T m1 = fabs(a + b) * T(0.5), m2 = fabs(a) * T(2), m3 = fabs(b) * T(2);
  if (m1 <= m2 && m1 <= m3) return 1u;
  return (m2 <= m3) ? 2u : 3u;
}

// Transverse-correction variant: the split vectors are the fluctuations with
// the limited correction moved into them, A+dQ - 2 Fc at a cell's left edge
// and A-dQ + 2 Fc at its right edge.  Only their p parts reach the split, so
// the cell's xs becomes xs + (4/c)(Fc_R,p - Fc_L,p) = xs + (1 - nu_x)(d_R - d_L)
// with d = l2 - l1 at an edge (and the mirror image for ys); the update keeps
// the plain fluctuations.
template <typename T, int LIM>
__device__ inline T ldiff(T a1, T a2, T a1_right, T a2_left) {
  return limited<T, LIM>(a2, a2_left) - limited<T, LIM>(a1, a1_right);
}
template <typename T>
__device__ inline T moved(T xs, T t, T d_lo, T d_hi) {
  return xs + t * (d_hi - d_lo);
}

// Flux-differencing update of one cell, eq. (2.3).
template <typename T>
__device__ inline void update(const Coef<T> &k, T p0, T u0, T v0, T xs0, T xd0, T ys0, T yd0,
                              T FLp, T FLu, T FRp, T FRu, T GBp, T GBv, T GTp, T GTv, T &pn, T &un,
                              T &vn) {
  pn = p0 - k.dtdx * (k.h * xs0 + (FRp - FLp)) - k.dtdy * (k.h * ys0 + (GTp - GBp));
  un = u0 - k.dtdx * (k.hz * xd0 + (FRu - FLu));
  vn = v0 - k.dtdy * (k.hz * yd0 + (GTv - GBv));
}

// Padded planes of one patch, indexed by interior coordinates (i, j).
template <typename T>
struct Planes {
  const T *p, *u, *v;
  int64_t ld;
  __device__ T P(int i, int j) const { return p[(int64_t)j * ld + i]; }
  __device__ T U(int i, int j) const { return u[(int64_t)j * ld + i]; }
  __device__ T V(int i, int j) const { return v[(int64_t)j * ld + i]; }
};

// The same planes read through unsigned 32-bit byte offsets from a
// wave-uniform base at padded cell (-2, -2) of plane 0: each load takes the
// scalar base and one 32-bit vector offset instead of a 64-bit address of its
// own.  The three planes of a patch must span less than 4 GiB.
template <typename T>
struct Planes32 {
  const char *b;
  uint32_t ld, plb;  // row stride (elements), plane stride (bytes)
  __device__ uint32_t off(int i, int j) const {
    return ((uint32_t)(j + 2) * ld + (uint32_t)(i + 2)) * (uint32_t)sizeof(T);
  }
  __device__ T P(int i, int j) const { return *reinterpret_cast<const T *>(b + off(i, j)); }
  __device__ T U(int i, int j) const { return *reinterpret_cast<const T *>(b + plb + off(i, j)); }
  __device__ T V(int i, int j) const {
    return *reinterpret_cast<const T *>(b + 2 * plb + off(i, j));
  }
};

struct CellMasks {
  unsigned own;    // bits of the cell's left x-edge (0-3) and bottom y-edge (4-7)
  unsigned right;  // bits 0-3 of the right x-edge (stored at cell i+1)
  unsigned top;    // bits 4-7 of the top y-edge (stored at cell j+1)
};

// DIRECT path: the whole update of one interior cell from its 13-point
// footprint.
template <typename T, int LIM, bool MASKS>
__device__ __attribute__((always_inline)) inline void cell_update(const Planes<T> &q, int i, int j, const Coef<T> &k, T &pn,
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

  // ---- first-order fluctuations entering the cell (and its neighbours)
  const T xs0 = a2L + a1R, xd0 = a2L - a1R;
  const T ys0 = b2B + b1T, yd0 = b2B - b1T;
  const T pdm = q.P(i - 1, j - 1), pdp = q.P(i + 1, j - 1);
  const T udm = q.U(i - 1, j - 1), udp = q.U(i + 1, j - 1);
  const T xsm = s2(Z, qm1 - pdm, q.U(i, j - 1) - udm) + s1(Z, pdp - qm1, udp - q.U(i, j - 1));
  const T pum = q.P(i - 1, j + 1), pup = q.P(i + 1, j + 1);
  const T uum = q.U(i - 1, j + 1), uup = q.U(i + 1, j + 1);
  const T xsp = s2(Z, qp1 - pum, q.U(i, j + 1) - uum) + s1(Z, pup - qp1, uup - q.U(i, j + 1));
  const T vlm = q.V(i - 1, j - 1), vl0 = q.V(i - 1, j), vlp = q.V(i - 1, j + 1);
  const T ysl = s2(Z, pm1 - pdm, vl0 - vlm) + s1(Z, pum - pm1, vlp - vl0);
  const T vrm = q.V(i + 1, j - 1), vr0 = q.V(i + 1, j), vrp = q.V(i + 1, j + 1);
  const T ysr = s2(Z, pp1 - pdp, vr0 - vrm) + s1(Z, pup - pp1, vrp - vr0);

  // ---- F~ and G~ on the four edges, then the update
  T FLp, FLu, FRp, FRu, GBp, GBv, GTp, GTv;
  ftilde<T, LIM>(k, a1L, a2L, a1R, a2LL, ysl, ys0, FLp, FLu);
  ftilde<T, LIM>(k, a1R, a2R, a1RR, a2L, ys0, ysr, FRp, FRu);
  gtilde<T, LIM>(k, b1B, b2B, b1T, b2BB, xsm, xs0, GBp, GBv);
  gtilde<T, LIM>(k, b1T, b2T, b1TT, b2B, xs0, xsp, GTp, GTv);
  update<T>(k, p0, u0, v0, xs0, xd0, ys0, yd0, FLp, FLu, FRp, FRu, GBp, GBv, GTp, GTv, pn, un, vn);

  if constexpr (MASKS) {
    mk->own = mc_branch(a1L, a1R) | (mc_branch(a2L, a2LL) << 2) | (mc_branch(b1B, b1T) << 4) |
              (mc_branch(b2B, b2BB) << 6);
    mk->right = mc_branch(a1R, a1RR) | (mc_branch(a2R, a2L) << 2);
    mk->top = (mc_branch(b1T, b1TT) << 4) | (mc_branch(b2T, b2B) << 6);
  }
}

// DIRECT path of the transverse-correction variant: the split vectors of the
// cell and its four neighbours need the limited strengths on both x-edges of
// rows j-1 and j+1 and on both y-edges of columns i-1 and i+1, so the
// footprint grows to 21 points (rows j-1..j+1 x columns i-2..i+2 and columns
// i-1..i+1 x rows j-2..j+2).  Every quantity has the expression the MARCH
// sweeps give it.
template <typename T, int LIM>
__device__ __attribute__((always_inline)) inline void cell_update_tc(const Planes<T> &q, int i, int j, const Coef<T> &k, T &pn,
                                      T &un, T &vn) {
  const T Z = k.Z;
  // The footprint is taken in stages (split vectors of the neighbours below,
  // above, left and right, then the cell itself) with scheduling barriers
  // between them, so that not all 21 points' loads are in flight at once.
  // ---- row j-1: x-edges i-3/2 .. i+3/2, split vector of cell (i, j-1)
  T xtm;
  {
    const T pdm2 = q.P(i - 2, j - 1), pdm = q.P(i - 1, j - 1), pd0 = q.P(i, j - 1),
            pdp = q.P(i + 1, j - 1), pdp2 = q.P(i + 2, j - 1);
    const T udm2 = q.U(i - 2, j - 1), udm = q.U(i - 1, j - 1), ud0 = q.U(i, j - 1),
            udp = q.U(i + 1, j - 1), udp2 = q.U(i + 2, j - 1);
    const T a2LLd = s2(Z, pdm - pdm2, udm - udm2);
    const T a1Ld = s1(Z, pd0 - pdm, ud0 - udm), a2Ld = s2(Z, pd0 - pdm, ud0 - udm);
    const T a1Rd = s1(Z, pdp - pd0, udp - ud0), a2Rd = s2(Z, pdp - pd0, udp - ud0);
    const T a1RRd = s1(Z, pdp2 - pdp, udp2 - udp);
    xtm = moved<T>(a2Ld + a1Rd, k.tx, ldiff<T, LIM>(a1Ld, a2Ld, a1Rd, a2LLd),
                   ldiff<T, LIM>(a1Rd, a2Rd, a1RRd, a2Ld));
  }
  __builtin_amdgcn_sched_barrier(0);
  // ---- row j+1
  T xtp;
  {
    const T pum2 = q.P(i - 2, j + 1), pum = q.P(i - 1, j + 1), pu0 = q.P(i, j + 1),
            pup = q.P(i + 1, j + 1), pup2 = q.P(i + 2, j + 1);
    const T uum2 = q.U(i - 2, j + 1), uum = q.U(i - 1, j + 1), uu0 = q.U(i, j + 1),
            uup = q.U(i + 1, j + 1), uup2 = q.U(i + 2, j + 1);
    const T a2LLu = s2(Z, pum - pum2, uum - uum2);
    const T a1Lu = s1(Z, pu0 - pum, uu0 - uum), a2Lu = s2(Z, pu0 - pum, uu0 - uum);
    const T a1Ru = s1(Z, pup - pu0, uup - uu0), a2Ru = s2(Z, pup - pu0, uup - uu0);
    const T a1RRu = s1(Z, pup2 - pup, uup2 - uup);
    xtp = moved<T>(a2Lu + a1Ru, k.tx, ldiff<T, LIM>(a1Lu, a2Lu, a1Ru, a2LLu),
                   ldiff<T, LIM>(a1Ru, a2Ru, a1RRu, a2Lu));
  }
  __builtin_amdgcn_sched_barrier(0);
  // ---- column i-1: y-edges j-3/2 .. j+3/2, split vector of cell (i-1, j)
  T ytl;
  {
    const T pl2 = q.P(i - 1, j - 2), pl1 = q.P(i - 1, j - 1), pl0 = q.P(i - 1, j),
            plp = q.P(i - 1, j + 1), plp2 = q.P(i - 1, j + 2);
    const T vl2 = q.V(i - 1, j - 2), vl1 = q.V(i - 1, j - 1), vl0 = q.V(i - 1, j),
            vlp = q.V(i - 1, j + 1), vlp2 = q.V(i - 1, j + 2);
    const T b2BBl = s2(Z, pl1 - pl2, vl1 - vl2);
    const T b1Bl = s1(Z, pl0 - pl1, vl0 - vl1), b2Bl = s2(Z, pl0 - pl1, vl0 - vl1);
    const T b1Tl = s1(Z, plp - pl0, vlp - vl0), b2Tl = s2(Z, plp - pl0, vlp - vl0);
    const T b1TTl = s1(Z, plp2 - plp, vlp2 - vlp);
    ytl = moved<T>(b2Bl + b1Tl, k.ty, ldiff<T, LIM>(b1Bl, b2Bl, b1Tl, b2BBl),
                   ldiff<T, LIM>(b1Tl, b2Tl, b1TTl, b2Bl));
  }
  __builtin_amdgcn_sched_barrier(0);
  // ---- column i+1
  T ytr;
  {
    const T pr2 = q.P(i + 1, j - 2), pr1 = q.P(i + 1, j - 1), pr0 = q.P(i + 1, j),
            prp = q.P(i + 1, j + 1), prp2 = q.P(i + 1, j + 2);
    const T vr2 = q.V(i + 1, j - 2), vr1 = q.V(i + 1, j - 1), vr0 = q.V(i + 1, j),
            vrp = q.V(i + 1, j + 1), vrp2 = q.V(i + 1, j + 2);
    const T b2BBr = s2(Z, pr1 - pr2, vr1 - vr2);
    const T b1Br = s1(Z, pr0 - pr1, vr0 - vr1), b2Br = s2(Z, pr0 - pr1, vr0 - vr1);
    const T b1Tr = s1(Z, prp - pr0, vrp - vr0), b2Tr = s2(Z, prp - pr0, vrp - vr0);
    const T b1TTr = s1(Z, prp2 - prp, vrp2 - vrp);
    ytr = moved<T>(b2Br + b1Tr, k.ty, ldiff<T, LIM>(b1Br, b2Br, b1Tr, b2BBr),
                   ldiff<T, LIM>(b1Tr, b2Tr, b1TTr, b2Br));
  }
  __builtin_amdgcn_sched_barrier(0);
  // ---- the cell: row j and column i
  const T pm2 = q.P(i - 2, j), pm1 = q.P(i - 1, j), p0 = q.P(i, j), pp1 = q.P(i + 1, j),
          pp2 = q.P(i + 2, j);
  const T um2 = q.U(i - 2, j), um1 = q.U(i - 1, j), u0 = q.U(i, j), up1 = q.U(i + 1, j),
          up2 = q.U(i + 2, j);
  const T a2LL = s2(Z, pm1 - pm2, um1 - um2);
  const T a1L = s1(Z, p0 - pm1, u0 - um1), a2L = s2(Z, p0 - pm1, u0 - um1);
  const T a1R = s1(Z, pp1 - p0, up1 - u0), a2R = s2(Z, pp1 - p0, up1 - u0);
  const T a1RR = s1(Z, pp2 - pp1, up2 - up1);
  const T qm2 = q.P(i, j - 2), qm1 = q.P(i, j - 1), qp1 = q.P(i, j + 1), qp2 = q.P(i, j + 2);
  const T vm2 = q.V(i, j - 2), vm1 = q.V(i, j - 1), v0 = q.V(i, j), vp1 = q.V(i, j + 1),
          vp2 = q.V(i, j + 2);
  const T b2BB = s2(Z, qm1 - qm2, vm1 - vm2);
  const T b1B = s1(Z, p0 - qm1, v0 - vm1), b2B = s2(Z, p0 - qm1, v0 - vm1);
  const T b1T = s1(Z, qp1 - p0, vp1 - v0), b2T = s2(Z, qp1 - p0, vp1 - v0);
  const T b1TT = s1(Z, qp2 - qp1, vp2 - vp1);
  const T xs0 = a2L + a1R, xd0 = a2L - a1R;
  const T ys0 = b2B + b1T, yd0 = b2B - b1T;
  const T xt0 = moved<T>(xs0, k.tx, ldiff<T, LIM>(a1L, a2L, a1R, a2LL),
                         ldiff<T, LIM>(a1R, a2R, a1RR, a2L));
  const T yt0 = moved<T>(ys0, k.ty, ldiff<T, LIM>(b1B, b2B, b1T, b2BB),
                         ldiff<T, LIM>(b1T, b2T, b1TT, b2B));

  // ---- F~ and G~ on the four edges, then the update
  T FLp, FLu, FRp, FRu, GBp, GBv, GTp, GTv;
  ftilde<T, LIM>(k, a1L, a2L, a1R, a2LL, ytl, yt0, FLp, FLu);
  ftilde<T, LIM>(k, a1R, a2R, a1RR, a2L, yt0, ytr, FRp, FRu);
  gtilde<T, LIM>(k, b1B, b2B, b1T, b2BB, xtm, xt0, GBp, GBv);
  gtilde<T, LIM>(k, b1T, b2T, b1TT, b2B, xt0, xtp, GTp, GTv);
  update<T>(k, p0, u0, v0, xs0, xd0, ys0, yd0, FLp, FLu, FRp, FRu, GBp, GBv, GTp, GTv, pn, un, vn);
}

// --------------------------------------------------------------------------
// Heterogeneous medium: c, Z and 1/(Z^2 + 1) per cell (planes 0, 1, 2 of the
// medium pool)
// --------------------------------------------------------------------------
// Normal solve at the edge between cells l and r: strengths of the wave
// along (-Z_l, 1, 0) (speed -c_l) and of the wave along (Z_r, 1, 0) (speed
// +c_r), a1 = (Z_r dn - dp)/(Z_l + Z_r), a2 = (dp + Z_l dn)/(Z_l + Z_r); the
// fluctuations A-dQ = (c_l Z_l a1, -c_l a1), A+dQ = (c_r Z_r a2, c_r a2).
// The limiter compares wave vectors, W_up . W / W . W: for wave 1 at edge
// (l, r) the upwind wave lies at edge (r, rr) along (-Z_r, 1, 0), so the
// limited strength is psi(a1, a1' (Z_r Z_l + 1)/(Z_l^2 + 1)); mirror for
// wave 2.  The correction at the edge is
//   Fc = 1/2 c_l (1 - c_l dt/dx) a1~ (-Z_l, 1, 0) + 1/2 c_r (1 - c_r dt/dx) a2~ (Z_r, 1, 0).
// A cell's fluctuations (X_p, X_u) = (c Z xs, c xd); split by B with the
// cells below (b) and above (t), B-X = c_b X_p/(Z_b + Z) (-Z_b, 0, 1) and
// B+X = c_t X_p/(Z + Z_t) (Z_t, 0, 1): the G~ of the edge (b, t) gets
//   -dt/(2dx) (c_t Z_t X_p(b) - c_b Z_b X_p(t), c_t X_p(b) + c_b X_p(t)) / (Z_b + Z_t)
// (p and v), sharing the edge's 1/(Z_b + Z_t); F~ alike.
// 1/x for x > 0 of moderate size (a sum of two impedances): the hardware
// reciprocal refined by Newton's iteration r <- r + r (1 - x r), twice in FP64
// (each step doubles the correct bits), once in FP32.
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

template <typename T>
__device__ inline void var_strengths(T Zl, T Zr, T dp, T dn, T &a1, T &a2, T &iz) {
  iz = recip(Zl + Zr);
  a1 = (Zr * dn - dp) * iz;
  a2 = (dp + Zl * dn) * iz;
}

// Limited strengths at the edge (l, r) given the upwind strengths a1u (edge
// (r, rr)) and a2u (edge (ll, l)) and the per-cell 1/(Z^2 + 1) of l and r.
template <typename T, int LIM>
__device__ inline void var_limited(T a1, T a2, T a1u, T a2u, T Zl, T Zr, T wl, T wr, T &l1,
                                   T &l2) {
  const T zz = Zl * Zr + T(1);
  l1 = limited<T, LIM>(a1, a1u * (zz * wl));
  l2 = limited<T, LIM>(a2, a2u * (zz * wr));
}

// Normal correction (p, normal velocity) at an edge.
template <typename T>
__device__ inline void var_corr(T cl, T Zl, T cr, T Zr, T l1, T l2, T dtdx, T &Fp, T &Fn) {
  const T gl = T(0.5) * cl * (T(1) - cl * dtdx), gr = T(0.5) * cr * (T(1) - cr * dtdx);
  Fp = gr * Zr * l2 - gl * Zl * l1;
  Fn = gl * l1 + gr * l2;
}

// One direction of a cell's update in a heterogeneous medium, from the five
// cells of its row (or column) around it: the normal corrections at its two
// edges (p and normal velocity), the fluctuation sums xs, xd, and the edge
// coefficients the transverse terms need.
template <typename T>
struct VarLine {
  T Fl_p, Fl_n, Fr_p, Fr_n;  // normal corrections at the low and high edge
  T xs, xd;                  // fluctuation sums of the cell
  T izl, izr;                // 1/(Z_l + Z) and 1/(Z + Z_r) of the two edges
  T cl, zl, c0, z0, cr, zr;  // c and Z of the cell and its two neighbours
};

// The line from its four edges' strengths (edge e between cells e and e+1 of
// the five), so a caller that carries edges along a column can reuse them.
template <typename T, int LIM>
__device__ inline VarLine<T> var_line_edges(const T a1[4], const T a2[4], const T iz[4],
                                            const T C[5], const T Zc[5], T wl, T w0, T wr,
                                            T dtdx) {
  VarLine<T> L;
  T l1, l2;
  var_limited<T, LIM>(a1[1], a2[1], a1[2], a2[0], Zc[1], Zc[2], wl, w0, l1, l2);
  var_corr(C[1], Zc[1], C[2], Zc[2], l1, l2, dtdx, L.Fl_p, L.Fl_n);
  var_limited<T, LIM>(a1[2], a2[2], a1[3], a2[1], Zc[2], Zc[3], w0, wr, l1, l2);
  var_corr(C[2], Zc[2], C[3], Zc[3], l1, l2, dtdx, L.Fr_p, L.Fr_n);
  L.xs = a2[1] + a1[2];
  L.xd = a2[1] - a1[2];
  L.izl = iz[1], L.izr = iz[2];
  L.cl = C[1], L.zl = Zc[1], L.c0 = C[2], L.z0 = Zc[2], L.cr = C[3], L.zr = Zc[3];
  return L;
}

template <typename T, int LIM>
__device__ inline VarLine<T> var_line(const T P[5], const T N[5], const T C[5], const T Zc[5],
                                      T wl, T w0, T wr, T dtdx) {
  T a1[4], a2[4], iz[4];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    var_strengths(Zc[e], Zc[e + 1], P[e + 1] - P[e], N[e + 1] - N[e], a1[e], a2[e], iz[e]);
  return var_line_edges<T, LIM>(a1, a2, iz, C, Zc, wl, w0, wr, dtdx);
}

// The cell's update from its two lines and the p-parts of the neighbours'
// fluctuations: X-fluctuations of the cells below and above (Xpb, Xpt) and
// Y-fluctuations of the cells left and right (Ypl, Ypr), each c Z times the
// neighbour's own fluctuation sum.  F~ at x-edges i-1/2 and i+1/2 take the
// normal correction and the transverse waves from the y-fluctuations of the
// cells on either side; G~ alike.
template <typename T>
__device__ inline void var_combine(const VarLine<T> &X, const VarLine<T> &Y, T Xpb, T Xpt, T Ypl,
                                   T Ypr, T p0, T u0, T v0, T dtdx, T dtdy, T &pn, T &un, T &vn,
                                   T &cfl) {
  const T c0 = X.c0, Z0 = X.z0;
  const T Xp0 = c0 * Z0 * X.xs, Yp0 = c0 * Z0 * Y.xs;
  T h = T(0.5) * dtdy * X.izl;
  const T FLp = X.Fl_p - h * (X.c0 * X.z0 * Ypl - X.cl * X.zl * Yp0);
  const T FLu = X.Fl_n - h * (X.c0 * Ypl + X.cl * Yp0);
  h = T(0.5) * dtdy * X.izr;
  const T FRp = X.Fr_p - h * (X.cr * X.zr * Yp0 - X.c0 * X.z0 * Ypr);
  const T FRu = X.Fr_n - h * (X.cr * Yp0 + X.c0 * Ypr);
  h = T(0.5) * dtdx * Y.izl;
  const T GBp = Y.Fl_p - h * (Y.c0 * Y.z0 * Xpb - Y.cl * Y.zl * Xp0);
  const T GBv = Y.Fl_n - h * (Y.c0 * Xpb + Y.cl * Xp0);
  h = T(0.5) * dtdx * Y.izr;
  const T GTp = Y.Fr_p - h * (Y.cr * Y.zr * Xp0 - Y.c0 * Y.z0 * Xpt);
  const T GTv = Y.Fr_n - h * (Y.cr * Xp0 + Y.c0 * Xpt);
  pn = p0 - dtdx * (Xp0 + (FRp - FLp)) - dtdy * (Yp0 + (GTp - GBp));
  un = u0 - dtdx * (c0 * X.xd + (FRu - FLu));
  vn = v0 - dtdy * (c0 * Y.xd + (GTv - GBv));
  cfl = fmax(fmax(fmax(X.cl, X.c0), X.cr) * dtdx, fmax(fmax(Y.cl, Y.c0), Y.cr) * dtdy);
}

// DIRECT update of cell (i, j) in a heterogeneous medium (13-point footprint
// of q and of the medium), taken in stages behind scheduling barriers so that
// only a few values stay live between them; cfl receives the largest
// |s| dt/dx over its four edges.
template <typename T, int LIM>
__device__ inline void cell_update_var(const Planes32<T> &q, const Planes32<T> &md, int i, int j,
                                       const Coef<T> &k, T &pn, T &un, T &vn, T &cfl) {
  const T dtdx = k.dtdx, dtdy = k.dtdy;
  const T w0 = md.V(i, j);
  // row j: x-direction
  VarLine<T> X;
  {
    T P[5], U[5], C[5], Z[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      P[d] = q.P(i + d - 2, j), U[d] = q.U(i + d - 2, j);
      C[d] = md.P(i + d - 2, j), Z[d] = md.U(i + d - 2, j);
    }
    X = var_line<T, LIM>(P, U, C, Z, md.V(i - 1, j), w0, md.V(i + 1, j), dtdx);
  }
  __builtin_amdgcn_sched_barrier(0);
  // column i: y-direction
  VarLine<T> Y;
  {
    T P[5], V[5], C[5], Z[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      P[d] = q.P(i, j + d - 2), V[d] = q.V(i, j + d - 2);
      C[d] = md.P(i, j + d - 2), Z[d] = md.U(i, j + d - 2);
    }
    Y = var_line<T, LIM>(P, V, C, Z, md.V(i, j - 1), w0, md.V(i, j + 1), dtdy);
  }
  __builtin_amdgcn_sched_barrier(0);
  // x-fluctuation p-part of the cells below and above, y-fluctuation p-part
  // of the cells left and right
  auto xp_row = [&](int jj) {
    const T pl = q.P(i - 1, jj), p0 = q.P(i, jj), pr = q.P(i + 1, jj);
    const T ul = q.U(i - 1, jj), u0 = q.U(i, jj), ur = q.U(i + 1, jj);
    const T Zl = md.U(i - 1, jj), Z0 = md.U(i, jj), Zr = md.U(i + 1, jj), c0 = md.P(i, jj);
    T s1l, s2l, izl, s1r, s2r, izr;
    var_strengths(Zl, Z0, p0 - pl, u0 - ul, s1l, s2l, izl);
    var_strengths(Z0, Zr, pr - p0, ur - u0, s1r, s2r, izr);
    return c0 * Z0 * (s2l + s1r);
  };
  auto yp_col = [&](int ii) {
    const T pb = q.P(ii, j - 1), p0 = q.P(ii, j), pt = q.P(ii, j + 1);
    const T vb = q.V(ii, j - 1), v0 = q.V(ii, j), vt = q.V(ii, j + 1);
    const T Zb = md.U(ii, j - 1), Z0 = md.U(ii, j), Zt = md.U(ii, j + 1), c0 = md.P(ii, j);
    T s1b, s2b, izb, s1t, s2t, izt;
    var_strengths(Zb, Z0, p0 - pb, v0 - vb, s1b, s2b, izb);
    var_strengths(Z0, Zt, pt - p0, vt - v0, s1t, s2t, izt);
    return c0 * Z0 * (s2b + s1t);
  };
  const T Xpb = xp_row(j - 1), Xpt = xp_row(j + 1);
  __builtin_amdgcn_sched_barrier(0);
  const T Ypl = yp_col(i - 1), Ypr = yp_col(i + 1);
  __builtin_amdgcn_sched_barrier(0);
  var_combine(X, Y, Xpb, Xpt, Ypl, Ypr, q.P(i, j), q.U(i, j), q.V(i, j), dtdx, dtdy, pn, un, vn,
              cfl);
}

// Store a new cell value and, on physical boundaries, its ghost images.  Up
// to 5 column and 5 row positions (the cell and its images); the loops are
// fully unrolled so everything stays in registers.
template <typename T>
__device__ inline void store_cell(T *op, T *ou, T *ov, int64_t ld, int i, int j, int mx, int my,
                                  int bc, T pn, T un, T vn) {
  constexpr int kNone = INT_MIN;
  int xi[5] = {i, kNone, kNone, kNone, kNone};
  int yj[5] = {j, kNone, kNone, kNone, kNone};
  if (bc == WS_BC_EXTRAP) {
    if (i == 0) { xi[1] = -1; xi[2] = -2; }
    if (i == mx - 1) { xi[3] = mx; xi[4] = mx + 1; }
    if (j == 0) { yj[1] = -1; yj[2] = -2; }
    if (j == my - 1) { yj[3] = my; yj[4] = my + 1; }
  } else if (bc == WS_BC_PERIODIC) {
    if (i < 2) xi[1] = mx + i;
    if (i >= mx - 2) xi[2] = i - mx;
    if (j < 2) yj[1] = my + j;
    if (j >= my - 2) yj[2] = j - my;
  }
#pragma unroll
  for (int b = 0; b < 5; ++b)
#pragma unroll
    for (int a = 0; a < 5; ++a)
      if (xi[a] != kNone && yj[b] != kNone) {
        const int64_t o = (int64_t)yj[b] * ld + xi[a];
        op[o] = pn;
        ou[o] = un;
        ov[o] = vn;
      }
}

// Store, taking the ghost-image path only for cells next to a physical side.
template <typename T>
__device__ inline void store(T *qo, int64_t plane, int64_t ld, int i, int j, int mx, int my, int bc,
                             T pn, T un, T vn) {
  if (bc != WS_BC_NONE && (i < 2 || i >= mx - 2 || j < 2 || j >= my - 2)) {
    store_cell<T>(qo, qo + plane, qo + 2 * plane, ld, i, j, mx, my, bc, pn, un, vn);
  } else {
    const int64_t o = (int64_t)j * ld + i;
    qo[o] = pn;
    qo[plane + o] = un;
    qo[2 * plane + o] = vn;
  }
}

// Heterogeneous medium, one column i marched up over rows [j0, j1): the
// quantities of cell_update_var, each formed by the same expression from the
// same inputs (so every cell's result is bitwise that of cell_update_var),
// with what neighbouring rows share carried in registers: the column's
// five-row window (p, v, c, Z, 1/(Z^2 + 1)), the four y-edges along it, the
// x-line of the next row (computed one row ahead, it also gives that row's
// x-fluctuation), the x-fluctuation of the row below, and the lower y-edge of
// the neighbouring columns.  Per row: one row of loads and seven edge solves
// instead of sixteen.  Returns the largest Courant number of the cells.
template <typename T, int LIM>
__device__ inline T march_col_var(const Planes32<T> &q, const Planes32<T> &md, int i, int j0,
                                  int j1, const Coef<T> &k, T *qo, const PatchRow &pr) {
  const T dtdx = k.dtdx, dtdy = k.dtdy;
  // the column's window, rows j-2 .. j+2
  T Pc[5], Vc[5], Cc[5], Zc[5], Wc[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    Pc[d] = q.P(i, j0 + d - 2), Vc[d] = q.V(i, j0 + d - 2);
    Cc[d] = md.P(i, j0 + d - 2), Zc[d] = md.U(i, j0 + d - 2), Wc[d] = md.V(i, j0 + d - 2);
  }
  // y-edge e between window rows e and e+1
  T b1[4], b2[4], bz[4];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    var_strengths(Zc[e], Zc[e + 1], Pc[e + 1] - Pc[e], Vc[e + 1] - Vc[e], b1[e], b2[e], bz[e]);
  // x-line of row jj (centre values from the window), with p and u of the
  // centre and p of the cells left and right
  auto xline = [&](int jj, T pc, T cc, T zc, T wc, T &uc, T &pl, T &pr_) {
    T P[5], U[5], C[5], Z[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      if (d == 2) continue;
      P[d] = q.P(i + d - 2, jj), U[d] = q.U(i + d - 2, jj);
      C[d] = md.P(i + d - 2, jj), Z[d] = md.U(i + d - 2, jj);
    }
    P[2] = pc, U[2] = q.U(i, jj), C[2] = cc, Z[2] = zc;
    uc = U[2], pl = P[1], pr_ = P[3];
    return var_line<T, LIM>(P, U, C, Z, md.V(i - 1, jj), wc, md.V(i + 1, jj), dtdx);
  };
  T u0, pl0, pr0;
  VarLine<T> XL = xline(j0, Pc[2], Cc[2], Zc[2], Wc[2], u0, pl0, pr0);
  // x-fluctuation p-part of row j0-1
  T Xpb;
  {
    const int jj = j0 - 1;
    const T pl = q.P(i - 1, jj), p0 = Pc[1], pr_ = q.P(i + 1, jj);
    const T ul = q.U(i - 1, jj), uu = q.U(i, jj), ur = q.U(i + 1, jj);
    const T Zl = md.U(i - 1, jj), Z0 = Zc[1], Zr = md.U(i + 1, jj), c0 = Cc[1];
    T s1l, s2l, izl, s1r, s2r, izr;
    var_strengths(Zl, Z0, p0 - pl, uu - ul, s1l, s2l, izl);
    var_strengths(Z0, Zr, pr_ - p0, ur - uu, s1r, s2r, izr);
    Xpb = c0 * Z0 * (s2l + s1r);
  }
  // the neighbouring columns at row j: p, v, Z there and a2 of their y-edge j-1/2
  T Pl = pl0, Vl = q.V(i - 1, j0), Pr = pr0, Vr = q.V(i + 1, j0), s2bl, s2br;
  {
    T s1, iz;
    var_strengths(md.U(i - 1, j0 - 1), XL.zl, Pl - q.P(i - 1, j0 - 1), Vl - q.V(i - 1, j0 - 1),
                  s1, s2bl, iz);
    var_strengths(md.U(i + 1, j0 - 1), XL.zr, Pr - q.P(i + 1, j0 - 1), Vr - q.V(i + 1, j0 - 1),
                  s1, s2br, iz);
  }
  T cfl = T(0);
  for (int j = j0; j < j1; ++j) {
    // row j+1: its x-line and x-fluctuation, and the neighbours' p, v there
    T u1, pl1, pr1;
    const VarLine<T> XN = xline(j + 1, Pc[3], Cc[3], Zc[3], Wc[3], u1, pl1, pr1);
    const T vl1 = q.V(i - 1, j + 1), vr1 = q.V(i + 1, j + 1);
    const T Xpt = XN.c0 * XN.z0 * XN.xs;
    // y-line of row j from the carried edges
    const VarLine<T> Y = var_line_edges<T, LIM>(b1, b2, bz, Cc, Zc, Wc[1], Wc[2], Wc[3], dtdy);
    // y-fluctuation p-parts of the cells left and right: their y-edge j+1/2
    T s1tl, s2tl, izl, s1tr, s2tr, izr;
    var_strengths(XL.zl, XN.zl, pl1 - Pl, vl1 - Vl, s1tl, s2tl, izl);
    var_strengths(XL.zr, XN.zr, pr1 - Pr, vr1 - Vr, s1tr, s2tr, izr);
    const T Ypl = XL.cl * XL.zl * (s2bl + s1tl), Ypr = XL.cr * XL.zr * (s2br + s1tr);
    T pn, un, vn, cj;
    var_combine(XL, Y, Xpb, Xpt, Ypl, Ypr, Pc[2], u0, Vc[2], dtdx, dtdy, pn, un, vn, cj);
    cfl = fmax(cfl, cj);
    store<T>(qo, pr.plane, pr.ld, i, j, pr.mx, pr.my, pr.bc, pn, un, vn);
    if (j + 1 >= j1) break;
    // slide up one row
    Xpb = XL.c0 * XL.z0 * XL.xs;
    XL = XN;
    u0 = u1;
    Pl = pl1, Vl = vl1, Pr = pr1, Vr = vr1, s2bl = s2tl, s2br = s2tr;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      Pc[d] = Pc[d + 1], Vc[d] = Vc[d + 1], Cc[d] = Cc[d + 1], Zc[d] = Zc[d + 1], Wc[d] = Wc[d + 1];
    }
    Pc[4] = q.P(i, j + 3), Vc[4] = q.V(i, j + 3);
    Cc[4] = md.P(i, j + 3), Zc[4] = md.U(i, j + 3), Wc[4] = md.V(i, j + 3);
#pragma unroll
    for (int e = 0; e < 3; ++e) b1[e] = b1[e + 1], b2[e] = b2[e + 1], bz[e] = bz[e + 1];
    var_strengths(Zc[3], Zc[4], Pc[4] - Pc[3], Vc[4] - Vc[3], b1[3], b2[3], bz[3]);
  }
  return cfl;
}


// Raw buffer stores (gfx9 buffer resource, no format conversion).  An offset
// at or past the resource's size is dropped by the hardware.  The stores are
// device-scope (cache policy SC1: written through the XCD's L2), so the L2s
// hold no dirty output to write back when the launch ends; the next step's
// workgroups read it on whichever XCD they run.
constexpr int kRawBufferWord3 = 0x00020000;
constexpr unsigned kDropOffset = 0x80000000u;
constexpr int kStoreDeviceScope = 16;  // SC1
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ inline void bstore(__amdgpu_buffer_rsrc_t r, double v, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0,
                                        kStoreDeviceScope);
}
__device__ inline void bstore(__amdgpu_buffer_rsrc_t r, float v, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0,
                                        kStoreDeviceScope);
}

// s_waitcnt immediate (gfx9 encoding) waiting for vmcnt(0) only.
constexpr int kWaitVmcnt0 = 0x0F70;

// Row sets of a MARCH segment (its row loop is unrolled by this count and
// names eight sets).
constexpr int kSets = 8;

// One row of (p, u, v) of a MARCH segment's column.
template <typename T>
struct Row3 {
  T p, u, v;
};


// Lanes of one MARCH segment (one wavefront, w = 64 lanes): lane l holds
// column i = c0-2+l, the segment updates columns c0..c0+w-5 (lanes 2..w-3)
// over a range of rows.  Loads and stores use unsigned 32-bit byte offsets
// from the patch's padded origin (cell -2,-2 of plane p) off wave-uniform
// bases: ((row+2) * ld + column+2) * sizeof(T); planes u, v follow at +plb,
// +2 plb.  MARCH patches span < 2^31 bytes.
template <typename T>
struct MarchLanes {
  static constexpr int w = kMarchWidth;
  const char *base;
  __amdgpu_buffer_rsrc_t ob;  // the output patch as a raw buffer
  unsigned ld, plb;
  int l, i, ic, mx, my;
  bool out;  // lane updates an interior column of the segment
  bool ybc;  // extrapolation sides: ghost rows are written
  bool xbc;  // the segment touches a physical x side
  int gx;    // ghost-column lane: 1, 2 -> i = -1, -2 (copy column 0); 3, 4 -> i = mx, mx+1
  bool st;   // lane stores

  __device__ MarchLanes(const T *qi, T *qo, const PatchRow &pr, int l_, int i_) {
    ld = (unsigned)pr.ld;
    plb = (unsigned)pr.plane * (unsigned)sizeof(T);
    l = l_;
    i = i_;
    mx = pr.mx;
    my = pr.my;
    // lanes past the last ghost column read that column instead (never used)
    ic = min(i, mx + 1);
    base = reinterpret_cast<const char *>(qi - 2 * (int64_t)ld - 2);
    ob = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<char *>(qo - 2 * (int64_t)ld - 2), 0,
                                           (int)(3 * plb), kRawBufferWord3);
    out = l >= 2 && l <= w - 3 && i < mx;
    // periodic patches are worked by DIRECT tiles only
    ybc = pr.bc == WS_BC_EXTRAP;
    const int c0 = i - l + 2;  // first column this segment updates
    xbc = ybc && (c0 == 0 || c0 + w - 4 >= mx);
    gx = 0;
    if (xbc) {
      if (i == -1) gx = 1;
      if (i == -2) gx = 2;
      if (i == mx && l <= w - 2) gx = 3;
      if (i == mx + 1 && l <= w - 1) gx = 4;
    }
    st = out || gx != 0;
  }
  __device__ unsigned at(int r) const {
    return ((unsigned)(r + 2) * ld + (unsigned)(ic + 2)) * (unsigned)sizeof(T);
  }
  __device__ unsigned oat(int r) const {
    return ((unsigned)(r + 2) * ld + (unsigned)(i + 2)) * (unsigned)sizeof(T);
  }
  __device__ T get(unsigned boff) const { return *reinterpret_cast<const T *>(base + boff); }
  // rows past the ghost rows are clamped to them (the values are never used)
  __device__ void fetch(Row3<T> &S, int r) const {
    const unsigned o = at(min(max(r, -2), my + 1));
    S.p = get(o);
    S.u = get(o + plb);
    S.v = get(o + 2 * plb);
  }
  // Store the new values of row r.  Extrapolation boundaries: the lanes on
  // ghost columns take the new value of the nearest interior column from
  // their neighbours, and the first and last rows are repeated into the ghost
  // rows (corners through the ghost-column lanes).  Every lane issues the
  // stores (lanes that write nothing get an offset past the buffer, which the
  // hardware drops), so the compiler's wait counts before each use of a
  // prefetched row do not depend on which lanes stored; the ghost rows are a
  // wave-uniform branch taken on two rows only.
  __device__ void emit(T pn, T un, T vn, int r) const {
    if (xbc) {
      const T p1 = shl(pn), u1 = shl(un), v1 = shl(vn);
      const T p2 = shl(p1), u2 = shl(u1), v2 = shl(v1);
      const T p3 = shr(pn), u3 = shr(un), v3 = shr(vn);
      const T p4 = shr(p3), u4 = shr(u3), v4 = shr(v3);
      if (gx == 1) { pn = p1; un = u1; vn = v1; }
      if (gx == 2) { pn = p2; un = u2; vn = v2; }
      if (gx == 3) { pn = p3; un = u3; vn = v3; }
      if (gx == 4) { pn = p4; un = u4; vn = v4; }
    }
    const unsigned so = st ? oat(r) : kDropOffset;
    bstore(ob, pn, so);
    bstore(ob, un, so + plb);
    bstore(ob, vn, so + 2 * plb);
    if (ybc && (r == 0 || r == my - 1)) {
      const int g0 = r == 0 ? -2 : my;
      for (int g = g0; g <= g0 + 1; ++g) {
        const unsigned o = st ? oat(g) : kDropOffset;
        bstore(ob, pn, o);
        bstore(ob, un, o + plb);
        bstore(ob, vn, o + 2 * plb);
      }
    }
  }
};

// Lanes of one PACKED wavefront: the MARCH lanes' interface, with the patch
// chosen per lane.  Lane l belongs to the column block (piece) whose lanes it
// falls in and holds column i of that piece's patch; loads and stores use
// unsigned 32-bit byte offsets from the pool's base (the pools of a level
// with PACKED tiles span less than 2^31 bytes).  Every piece's patch has
// frozen ghosts (no ghost images are written) and holds every row the
// wavefront marches over.  A piece's two lanes on either side play the part
// of a MARCH segment's halo lanes: whatever a neighbouring piece leaves in
// them reaches no updated column.
template <typename T>
struct PackedLanes {
  static constexpr int w = kMarchWidth;
  const char *base;           // the input pool
  __amdgpu_buffer_rsrc_t ob;  // the output pool as a raw buffer
  unsigned colb;   // byte offset of the lane's read column in row -2 of plane p
  unsigned ocolb;  // the same for the lane's own column (stores)
  unsigned ldb, plb;  // row and plane strides of the lane's patch (bytes)
  int rlo, rhi;       // rows a fetch is clamped to: the march's rows and two either side
  bool out;           // lane updates a column of its piece
  // the MARCH lanes' branch-recording fields (never recorded here)
  static constexpr int l = 0, i = 0, mx = 0, my = 0;

  __device__ unsigned at(int r) const { return colb + (unsigned)(r + 2) * ldb; }
  __device__ unsigned oat(int r) const { return ocolb + (unsigned)(r + 2) * ldb; }
  __device__ T get(unsigned boff) const { return *reinterpret_cast<const T *>(base + boff); }
  __device__ void fetch(Row3<T> &S, int r) const {
    const unsigned o = at(min(max(r, rlo), rhi));
    S.p = get(o);
    S.u = get(o + plb);
    S.v = get(o + 2 * plb);
  }
  __device__ void emit(T pn, T un, T vn, int r) const {
    const unsigned so = out ? oat(r) : kDropOffset;
    bstore(ob, pn, so);
    bstore(ob, un, so + plb);
    bstore(ob, vn, so + 2 * plb);
  }
};

// Row sets of a MARCH segment: set k holds one row from its load until its
// last use (as row r+2, r+1, then r of the row being updated; mirrored for a
// downward march), and is then refilled in place with the row kSets further
// on, so kSets-2 rows are in flight and no in-flight register is copied.
// The row loops are unrolled by kSets and name eight sets; the prologues
// wait for everything they requested (vmcnt(0)), so the loops' waits are
// those of their steady state.

// The row loops, unrolled by kSets.  Upward over [r0, r1): row(A, B, C, r,
// refill) with A, B, C the sets holding rows r, r+1, r+2; the last rows
// refill only what a later row still reads (rows <= r1+1).
template <typename T, typename RowFn>
__device__ __attribute__((always_inline)) inline void sweep_up(RowFn &row, Row3<T> &R0, Row3<T> &R1, Row3<T> &R2, Row3<T> &R3,
                                Row3<T> &R4, Row3<T> &R5, Row3<T> &R6, Row3<T> &R7, int r0,
                                int r1) {
  int r = r0;
  for (; r + kSets <= r1; r += kSets) {
    row(R0, R1, R2, r, true);
    row(R1, R2, R3, r + 1, true);
    row(R2, R3, R4, r + 2, true);
    row(R3, R4, R5, r + 3, true);
    row(R4, R5, R6, r + 4, true);
    row(R5, R6, R7, r + 5, true);
    row(R6, R7, R0, r + 6, true);
    row(R7, R0, R1, r + 7, true);
  }
  if (r < r1) { row(R0, R1, R2, r, r + kSets <= r1 + 1); ++r; }
  if (r < r1) { row(R1, R2, R3, r, r + kSets <= r1 + 1); ++r; }
  if (r < r1) { row(R2, R3, R4, r, r + kSets <= r1 + 1); ++r; }
  if (r < r1) { row(R3, R4, R5, r, r + kSets <= r1 + 1); ++r; }
  if (r < r1) { row(R4, R5, R6, r, r + kSets <= r1 + 1); ++r; }
  if (r < r1) { row(R5, R6, R7, r, r + kSets <= r1 + 1); ++r; }
  if (r < r1) { row(R6, R7, R0, r, r + kSets <= r1 + 1); ++r; }
}

// Downward from row r1-1 to r0: A, B, C hold rows r, r-1, r-2; the last rows
// refill only what a later row still reads (rows >= r0-2).
template <typename T, typename RowFn>
__device__ __attribute__((always_inline)) inline void sweep_down(RowFn &row, Row3<T> &R0, Row3<T> &R1, Row3<T> &R2, Row3<T> &R3,
                                  Row3<T> &R4, Row3<T> &R5, Row3<T> &R6, Row3<T> &R7, int r0,
                                  int r1) {
  int r = r1 - 1;
  for (; r - kSets + 1 >= r0; r -= kSets) {
    row(R0, R1, R2, r, true);
    row(R1, R2, R3, r - 1, true);
    row(R2, R3, R4, r - 2, true);
    row(R3, R4, R5, r - 3, true);
    row(R4, R5, R6, r - 4, true);
    row(R5, R6, R7, r - 5, true);
    row(R6, R7, R0, r - 6, true);
    row(R7, R0, R1, r - 7, true);
  }
  if (r >= r0) { row(R0, R1, R2, r, r - kSets >= r0 - 2); --r; }
  if (r >= r0) { row(R1, R2, R3, r, r - kSets >= r0 - 2); --r; }
  if (r >= r0) { row(R2, R3, R4, r, r - kSets >= r0 - 2); --r; }
  if (r >= r0) { row(R3, R4, R5, r, r - kSets >= r0 - 2); --r; }
  if (r >= r0) { row(R4, R5, R6, r, r - kSets >= r0 - 2); --r; }
  if (r >= r0) { row(R5, R6, R7, r, r - kSets >= r0 - 2); --r; }
  if (r >= r0) { row(R6, R7, R0, r, r - kSets >= r0 - 2); --r; }
}

// Upward MARCH over rows [r0, r1).  x-neighbour terms come through lane
// shifts; y-direction terms slide up the column in registers.  Each quantity
// uses the same expression as in cell_update, so the result is bitwise equal.
template <typename T, int LIM, bool MASKS, class L>
__device__ __attribute__((always_inline)) inline void march_up(const L &M, const Coef<T> &k, int r0, int r1,
                                uint8_t *masks) {
  constexpr int w = kMarchWidth;
  const T Z = k.Z;
  const int l = M.l, i = M.i;
  Row3<T> R0, R1, R2, R3, R4, R5, R6, R7;
  // ---- prologue: rows r0-2, r0-1 and the sets (rows r0 .. r0+7)
  const unsigned om2 = M.at(r0 - 2), om1 = M.at(r0 - 1);
  const T Pm2 = M.get(om2), Pm1 = M.get(om1);
  const T Vm2 = M.get(om2 + 2 * M.plb), Vm1 = M.get(om1 + 2 * M.plb);
  const T Um1 = M.get(om1 + M.plb);
  M.fetch(R0, r0);
  M.fetch(R1, r0 + 1);
  M.fetch(R2, r0 + 2);
  M.fetch(R3, r0 + 3);
  M.fetch(R4, r0 + 4);
  M.fetch(R5, r0 + 5);
  M.fetch(R6, r0 + 6);
  M.fetch(R7, r0 + 7);
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  const T P0 = R0.p, U0 = R0.u, V0 = R0.v, P1 = R1.p, V1 = R1.v;
  const T b2mm = s2(Z, Pm1 - Pm2, Vm1 - Vm2);                                // y-edge r0-3/2
  const T b1m = s1(Z, P0 - Pm1, V0 - Vm1), b2m = s2(Z, P0 - Pm1, V0 - Vm1);  // r0-1/2
  T b1h = s1(Z, P1 - P0, V1 - V0), b2h = s2(Z, P1 - P0, V1 - V0);            // r0+1/2
  T yb2 = b2m;  // b2 of the cell's bottom edge
  // x-edges of rows r0-1 and r0
  const T pl_m = shr(Pm1), ul_m = shr(Um1);
  const T a2Lm = s2(Z, Pm1 - pl_m, Um1 - ul_m);
  const T a1Lm = s1(Z, Pm1 - pl_m, Um1 - ul_m);
  const T xsm = a2Lm + shl(a1Lm);
  const T pl_0 = shr(P0), ul_0 = shr(U0);
  T a1L = s1(Z, P0 - pl_0, U0 - ul_0), a2L = s2(Z, P0 - pl_0, U0 - ul_0);
  T a1R = shl(a1L);
  T xs0 = a2L + a1R;
  T GBp, GBv;
  gtilde<T, LIM>(k, b1m, b2m, b1h, b2mm, xsm, xs0, GBp, GBv);
  unsigned ybits = 0;
  if constexpr (MASKS) ybits = (mc_branch(b1m, b1h) << 4) | (mc_branch(b2m, b2mm) << 6);
  const int64_t mld = M.mx + 1;

  // One row r: A, B, C hold rows r, r+1, r+2; A is refilled with row r+kSets
  // at the end (the barriers keep the scheduler from moving the refill above
  // the row's last use of A, or the next row's arithmetic above this row's).
  auto row = [&](Row3<T> &A, const Row3<T> &B, const Row3<T> &C, int r, bool refill) {
    __builtin_amdgcn_sched_barrier(0);
    const T P0 = A.p, U0 = A.u, V0 = A.v;
    const T P1 = B.p, U1 = B.u, V1 = B.v;
    const T P2 = C.p, V2 = C.v;
    // y-edge r+3/2 of this column and the y-fluctuations of cell (i, r)
    const T b1hh = s1(Z, P2 - P1, V2 - V1), b2hh = s2(Z, P2 - P1, V2 - V1);
    const T ys0 = yb2 + b1h, yd0 = yb2 - b1h;
    // left x-edge of row r+1
    const T pl_1 = shr(P1), ul_1 = shr(U1);
    const T a1Ln = s1(Z, P1 - pl_1, U1 - ul_1), a2Ln = s2(Z, P1 - pl_1, U1 - ul_1);
    const T a1Rn = shl(a1Ln);
    const T xsp = a2Ln + a1Rn;
    const T xd0 = a2L - a1R;
    const T a2LL = shr(a2L);
    const T ysl = shr(ys0);
    T FLp, FLu, GTp, GTv;
    ftilde<T, LIM>(k, a1L, a2L, a1R, a2LL, ysl, ys0, FLp, FLu);
    const T FRp = shl(FLp), FRu = shl(FLu);
    gtilde<T, LIM>(k, b1h, b2h, b1hh, yb2, xs0, xsp, GTp, GTv);
    T pn, un, vn;
    update<T>(k, P0, U0, V0, xs0, xd0, ys0, yd0, FLp, FLu, FRp, FRu, GBp, GBv, GTp, GTv, pn, un, vn);
    M.emit(pn, un, vn, r);
    if constexpr (MASKS) {
      const unsigned xbits = mc_branch(a1L, a1R) | (mc_branch(a2L, a2LL) << 2);
      const unsigned tbits = (mc_branch(b1h, b1hh) << 4) | (mc_branch(b2h, yb2) << 6);
      if (M.out) {
        masks[(int64_t)r * mld + i] = (uint8_t)(xbits | ybits);
        if (r == M.my - 1) {
          masks[(int64_t)(r + 1) * mld + i] = (uint8_t)tbits;
          if (i == M.mx - 1) masks[(int64_t)(r + 1) * mld + i + 1] = 0;  // no edge owns it
        }
      } else if (i == M.mx && l >= 2 && l <= w - 2) {
        masks[(int64_t)r * mld + i] = (uint8_t)xbits;
      }
      ybits = tbits;
    }
    // slide up one row
    yb2 = b2h; b1h = b1hh; b2h = b2hh;
    GBp = GTp; GBv = GTv;
    xs0 = xsp; a1L = a1Ln; a2L = a2Ln; a1R = a1Rn;
    __builtin_amdgcn_sched_barrier(0);
    if (refill) M.fetch(A, r + kSets);
  };
  sweep_up<T>(row, R0, R1, R2, R3, R4, R5, R6, R7, r0, r1);
}

// Downward MARCH over rows [r0, r1), from row r1-1 down to r0: the mirror of
// march_up (the carried y-terms are those of the cell's top edge), with every
// quantity again computed by the same expression as in cell_update.  Vertically
// neighbouring segments march in opposite directions, so the rows two of them
// share are read by both at about the same time (both at their start, or
// both at their end) and the second read finds them in L2.
template <typename T, int LIM, class L>
__device__ __attribute__((always_inline)) inline void march_down(const L &M, const Coef<T> &k, int r0, int r1) {
  const T Z = k.Z;
  Row3<T> R0, R1, R2, R3, R4, R5, R6, R7;
  // ---- prologue: rows r1+1, r1 and the sets (rows r1-1 down to r1-8)
  const unsigned oa2 = M.at(r1 + 1), oa1 = M.at(r1);
  const T Pa2 = M.get(oa2), Pa1 = M.get(oa1);
  const T Va2 = M.get(oa2 + 2 * M.plb), Va1 = M.get(oa1 + 2 * M.plb);
  const T Ua1 = M.get(oa1 + M.plb);
  M.fetch(R0, r1 - 1);
  M.fetch(R1, r1 - 2);
  M.fetch(R2, r1 - 3);
  M.fetch(R3, r1 - 4);
  M.fetch(R4, r1 - 5);
  M.fetch(R5, r1 - 6);
  M.fetch(R6, r1 - 7);
  M.fetch(R7, r1 - 8);
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  // the top row r = r1-1 (P0) and the one below it (Pm)
  const T P0 = R0.p, U0 = R0.u, V0 = R0.v, Pm = R1.p, Vm = R1.v;
  const T b1aa = s1(Z, Pa2 - Pa1, Va2 - Va1);                                // y-edge r1+1/2
  const T b1a = s1(Z, Pa1 - P0, Va1 - V0), b2a = s2(Z, Pa1 - P0, Va1 - V0);  // r1-1/2
  T b1B = s1(Z, P0 - Pm, V0 - Vm), b2B = s2(Z, P0 - Pm, V0 - Vm);            // r1-3/2
  T b1T = b1a;  // b1 of the cell's top edge
  // x-edges of rows r1 and r1-1
  const T pl_a = shr(Pa1), ul_a = shr(Ua1);
  const T a2La = s2(Z, Pa1 - pl_a, Ua1 - ul_a);
  const T a1La = s1(Z, Pa1 - pl_a, Ua1 - ul_a);
  const T xsa = a2La + shl(a1La);
  const T pl_0 = shr(P0), ul_0 = shr(U0);
  T a1L = s1(Z, P0 - pl_0, U0 - ul_0), a2L = s2(Z, P0 - pl_0, U0 - ul_0);
  T a1R = shl(a1L);
  T xs0 = a2L + a1R;
  T GTp, GTv;  // G~ of the cell's top edge
  gtilde<T, LIM>(k, b1a, b2a, b1aa, b2B, xs0, xsa, GTp, GTv);

  // One row r: A, B, C hold rows r, r-1, r-2; A is refilled with row r-kSets.
  auto row = [&](Row3<T> &A, const Row3<T> &B, const Row3<T> &C, int r, bool refill) {
    __builtin_amdgcn_sched_barrier(0);
    const T P0 = A.p, U0 = A.u, V0 = A.v;
    const T Pm = B.p, Um = B.u, Vm = B.v;
    const T Pmm = C.p, Vmm = C.v;
    // y-edge r-3/2 of this column and the y-fluctuations of cell (i, r)
    const T b1BB = s1(Z, Pm - Pmm, Vm - Vmm), b2BB = s2(Z, Pm - Pmm, Vm - Vmm);
    const T ys0 = b2B + b1T, yd0 = b2B - b1T;
    // left x-edge of row r-1
    const T pl_m = shr(Pm), ul_m = shr(Um);
    const T a1Lm = s1(Z, Pm - pl_m, Um - ul_m), a2Lm = s2(Z, Pm - pl_m, Um - ul_m);
    const T a1Rm = shl(a1Lm);
    const T xsm = a2Lm + a1Rm;
    const T xd0 = a2L - a1R;
    const T a2LL = shr(a2L);
    const T ysl = shr(ys0);
    T FLp, FLu, GBp, GBv;
    ftilde<T, LIM>(k, a1L, a2L, a1R, a2LL, ysl, ys0, FLp, FLu);
    const T FRp = shl(FLp), FRu = shl(FLu);
    gtilde<T, LIM>(k, b1B, b2B, b1T, b2BB, xsm, xs0, GBp, GBv);
    T pn, un, vn;
    update<T>(k, P0, U0, V0, xs0, xd0, ys0, yd0, FLp, FLu, FRp, FRu, GBp, GBv, GTp, GTv, pn, un, vn);
    M.emit(pn, un, vn, r);
    // slide down one row
    b1T = b1B; b1B = b1BB; b2B = b2BB;
    GTp = GBp; GTv = GBv;
    xs0 = xsm; a1L = a1Lm; a2L = a2Lm; a1R = a1Rm;
    __builtin_amdgcn_sched_barrier(0);
    if (refill) M.fetch(A, r - kSets);
  };
  sweep_down<T>(row, R0, R1, R2, R3, R4, R5, R6, R7, r0, r1);
}

// Upward MARCH of the transverse-correction variant.  The split vector of
// cell (i, r+1) needs the limited strengths of row r+1, so they are formed one
// row ahead and carried (l1, l2) into the next row's F~; the y-edges' limited
// strengths of a cell's top edge serve its split vector and G~, and slide down
// as the bottom edge's (eB).
template <typename T, int LIM, class L>
__device__ __attribute__((always_inline)) inline void march_up_tc(const L &M, const Coef<T> &k, int r0, int r1) {
  const T Z = k.Z;
  Row3<T> R0, R1, R2, R3, R4, R5, R6, R7;
  const unsigned om2 = M.at(r0 - 2), om1 = M.at(r0 - 1);
  const T Pm2 = M.get(om2), Pm1 = M.get(om1);
  const T Vm2 = M.get(om2 + 2 * M.plb), Vm1 = M.get(om1 + 2 * M.plb);
  const T Um1 = M.get(om1 + M.plb);
  M.fetch(R0, r0);
  M.fetch(R1, r0 + 1);
  M.fetch(R2, r0 + 2);
  M.fetch(R3, r0 + 3);
  M.fetch(R4, r0 + 4);
  M.fetch(R5, r0 + 5);
  M.fetch(R6, r0 + 6);
  M.fetch(R7, r0 + 7);
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  const T P0 = R0.p, U0 = R0.u, V0 = R0.v, P1 = R1.p, V1 = R1.v;
  const T b2mm = s2(Z, Pm1 - Pm2, Vm1 - Vm2);                                // y-edge r0-3/2
  const T b1m = s1(Z, P0 - Pm1, V0 - Vm1), b2m = s2(Z, P0 - Pm1, V0 - Vm1);  // r0-1/2
  T b1h = s1(Z, P1 - P0, V1 - V0), b2h = s2(Z, P1 - P0, V1 - V0);            // r0+1/2
  T yb2 = b2m;
  const T lb1m = limited<T, LIM>(b1m, b1h), lb2m = limited<T, LIM>(b2m, b2mm);
  T eB = lb2m - lb1m;
  // row r0-1: split vector of cell (i, r0-1)
  const T pl_m = shr(Pm1), ul_m = shr(Um1);
  const T a2Lm = s2(Z, Pm1 - pl_m, Um1 - ul_m);
  const T a1Lm = s1(Z, Pm1 - pl_m, Um1 - ul_m);
  const T a1Rm = shl(a1Lm);
  const T dm = limited<T, LIM>(a2Lm, shr(a2Lm)) - limited<T, LIM>(a1Lm, a1Rm);
  const T xtm = moved<T>(a2Lm + a1Rm, k.tx, dm, shl(dm));
  // row r0
  const T pl_0 = shr(P0), ul_0 = shr(U0);
  T a1L = s1(Z, P0 - pl_0, U0 - ul_0), a2L = s2(Z, P0 - pl_0, U0 - ul_0);
  T a1R = shl(a1L);
  T xs0 = a2L + a1R;
  T l1 = limited<T, LIM>(a1L, a1R), l2 = limited<T, LIM>(a2L, shr(a2L));
  const T d0 = l2 - l1;
  T xt0 = moved<T>(xs0, k.tx, d0, shl(d0));
  T GBp, GBv;
  gtilde_l<T>(k, lb1m, lb2m, xtm, xt0, GBp, GBv);

  auto row = [&](Row3<T> &A, const Row3<T> &B, const Row3<T> &C, int r, bool refill) {
    __builtin_amdgcn_sched_barrier(0);
    const T P0 = A.p, U0 = A.u, V0 = A.v;
    const T P1 = B.p, U1 = B.u, V1 = B.v;
    const T P2 = C.p, V2 = C.v;
    const T b1hh = s1(Z, P2 - P1, V2 - V1), b2hh = s2(Z, P2 - P1, V2 - V1);
    const T ys0 = yb2 + b1h, yd0 = yb2 - b1h;
    // top edge r+1/2: limited strengths, then the split vector's ys
    const T lb1 = limited<T, LIM>(b1h, b1hh), lb2 = limited<T, LIM>(b2h, yb2);
    const T eT = lb2 - lb1;
    const T yt0 = moved<T>(ys0, k.ty, eB, eT);
    // row r+1: strengths, limited strengths and split vector
    const T pl_1 = shr(P1), ul_1 = shr(U1);
    const T a1Ln = s1(Z, P1 - pl_1, U1 - ul_1), a2Ln = s2(Z, P1 - pl_1, U1 - ul_1);
    const T a1Rn = shl(a1Ln);
    const T l1n = limited<T, LIM>(a1Ln, a1Rn), l2n = limited<T, LIM>(a2Ln, shr(a2Ln));
    const T dn = l2n - l1n;
    const T xtp = moved<T>(a2Ln + a1Rn, k.tx, dn, shl(dn));
    const T xd0 = a2L - a1R;
    const T ytl = shr(yt0);
    T FLp, FLu, GTp, GTv;
    ftilde_l<T>(k, l1, l2, ytl, yt0, FLp, FLu);
    const T FRp = shl(FLp), FRu = shl(FLu);
    gtilde_l<T>(k, lb1, lb2, xt0, xtp, GTp, GTv);
    T pn, un, vn;
    update<T>(k, P0, U0, V0, xs0, xd0, ys0, yd0, FLp, FLu, FRp, FRu, GBp, GBv, GTp, GTv, pn, un, vn);
    M.emit(pn, un, vn, r);
    yb2 = b2h; b1h = b1hh; b2h = b2hh; eB = eT;
    GBp = GTp; GBv = GTv;
    xs0 = a2Ln + a1Rn; xt0 = xtp; a2L = a2Ln; a1R = a1Rn; l1 = l1n; l2 = l2n;
    __builtin_amdgcn_sched_barrier(0);
    if (refill) M.fetch(A, r + kSets);
  };
  sweep_up<T>(row, R0, R1, R2, R3, R4, R5, R6, R7, r0, r1);
}

// Downward MARCH of the transverse-correction variant: the mirror of
// march_up_tc (limited strengths of row r-1 formed one row ahead, the top
// edge's eT carried).
template <typename T, int LIM, class L>
__device__ __attribute__((always_inline)) inline void march_down_tc(const L &M, const Coef<T> &k, int r0, int r1) {
  const T Z = k.Z;
  Row3<T> R0, R1, R2, R3, R4, R5, R6, R7;
  const unsigned oa2 = M.at(r1 + 1), oa1 = M.at(r1);
  const T Pa2 = M.get(oa2), Pa1 = M.get(oa1);
  const T Va2 = M.get(oa2 + 2 * M.plb), Va1 = M.get(oa1 + 2 * M.plb);
  const T Ua1 = M.get(oa1 + M.plb);
  M.fetch(R0, r1 - 1);
  M.fetch(R1, r1 - 2);
  M.fetch(R2, r1 - 3);
  M.fetch(R3, r1 - 4);
  M.fetch(R4, r1 - 5);
  M.fetch(R5, r1 - 6);
  M.fetch(R6, r1 - 7);
  M.fetch(R7, r1 - 8);
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  const T P0 = R0.p, U0 = R0.u, V0 = R0.v, Pm = R1.p, Vm = R1.v;
  const T b1aa = s1(Z, Pa2 - Pa1, Va2 - Va1);                                // y-edge r1+1/2
  const T b1a = s1(Z, Pa1 - P0, Va1 - V0), b2a = s2(Z, Pa1 - P0, Va1 - V0);  // r1-1/2
  T b1B = s1(Z, P0 - Pm, V0 - Vm), b2B = s2(Z, P0 - Pm, V0 - Vm);            // r1-3/2
  T b1T = b1a;
  const T lb1a = limited<T, LIM>(b1a, b1aa), lb2a = limited<T, LIM>(b2a, b2B);
  T eT = lb2a - lb1a;
  // row r1: split vector of cell (i, r1)
  const T pl_a = shr(Pa1), ul_a = shr(Ua1);
  const T a2La = s2(Z, Pa1 - pl_a, Ua1 - ul_a);
  const T a1La = s1(Z, Pa1 - pl_a, Ua1 - ul_a);
  const T a1Ra = shl(a1La);
  const T da = limited<T, LIM>(a2La, shr(a2La)) - limited<T, LIM>(a1La, a1Ra);
  const T xta = moved<T>(a2La + a1Ra, k.tx, da, shl(da));
  // row r1-1
  const T pl_0 = shr(P0), ul_0 = shr(U0);
  T a1L = s1(Z, P0 - pl_0, U0 - ul_0), a2L = s2(Z, P0 - pl_0, U0 - ul_0);
  T a1R = shl(a1L);
  T xs0 = a2L + a1R;
  T l1 = limited<T, LIM>(a1L, a1R), l2 = limited<T, LIM>(a2L, shr(a2L));
  const T d0 = l2 - l1;
  T xt0 = moved<T>(xs0, k.tx, d0, shl(d0));
  T GTp, GTv;
  gtilde_l<T>(k, lb1a, lb2a, xt0, xta, GTp, GTv);

  auto row = [&](Row3<T> &A, const Row3<T> &B, const Row3<T> &C, int r, bool refill) {
    __builtin_amdgcn_sched_barrier(0);
    const T P0 = A.p, U0 = A.u, V0 = A.v;
    const T Pm = B.p, Um = B.u, Vm = B.v;
    const T Pmm = C.p, Vmm = C.v;
    const T b1BB = s1(Z, Pm - Pmm, Vm - Vmm), b2BB = s2(Z, Pm - Pmm, Vm - Vmm);
    const T ys0 = b2B + b1T, yd0 = b2B - b1T;
    // bottom edge r-1/2: limited strengths, then the split vector's ys
    const T lb1 = limited<T, LIM>(b1B, b1T), lb2 = limited<T, LIM>(b2B, b2BB);
    const T eB = lb2 - lb1;
    const T yt0 = moved<T>(ys0, k.ty, eB, eT);
    // row r-1: strengths, limited strengths and split vector
    const T pl_m = shr(Pm), ul_m = shr(Um);
    const T a1Lm = s1(Z, Pm - pl_m, Um - ul_m), a2Lm = s2(Z, Pm - pl_m, Um - ul_m);
    const T a1Rm = shl(a1Lm);
    const T l1m = limited<T, LIM>(a1Lm, a1Rm), l2m = limited<T, LIM>(a2Lm, shr(a2Lm));
    const T dm = l2m - l1m;
    const T xtm = moved<T>(a2Lm + a1Rm, k.tx, dm, shl(dm));
    const T xd0 = a2L - a1R;
    const T ytl = shr(yt0);
    T FLp, FLu, GBp, GBv;
    ftilde_l<T>(k, l1, l2, ytl, yt0, FLp, FLu);
    const T FRp = shl(FLp), FRu = shl(FLu);
    gtilde_l<T>(k, lb1, lb2, xtm, xt0, GBp, GBv);
    T pn, un, vn;
    update<T>(k, P0, U0, V0, xs0, xd0, ys0, yd0, FLp, FLu, FRp, FRu, GBp, GBv, GTp, GTv, pn, un, vn);
    M.emit(pn, un, vn, r);
    b1T = b1B; b1B = b1BB; b2B = b2BB; eT = eB;
    GTp = GBp; GTv = GBv;
    xs0 = a2Lm + a1Rm; xt0 = xtm; a2L = a2Lm; a1R = a1Rm; l1 = l1m; l2 = l2m;
    __builtin_amdgcn_sched_barrier(0);
    if (refill) M.fetch(A, r - kSets);
  };
  sweep_down<T>(row, R0, R1, R2, R3, R4, R5, R6, R7, r0, r1);
}

__device__ inline unsigned long long dbits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// One work unit, quarter q of tile t (MARCH: segment q; DIRECT: threads
// q*64 .. q*64+63 of the tile), worked by one wavefront; returns the tile's
// Courant number.  No barrier: wavefronts take units independently.
// MARCH segment in a heterogeneous medium, marching up over rows [r0, r1):
// the quantities of cell_update_var, each formed by the same expression from
// the same inputs, so every cell's result is bitwise that of
// cell_update_var.  Each lane solves only its column's left x-edge and, once
// per row, the y-edge above its window; what a cell needs of its neighbours'
// edges and fluctuations comes through lane shifts (an x-edge's limited
// correction is the left edge of one lane and the right edge of the lane to
// its left), and along the column the five-row window of (p, u, v) and
// (c, Z, 1/(Z^2 + 1)), the four y-edges and the x-fluctuation of the row
// below are carried.  One row is loaded ahead of the window (two ahead kept
// 170 registers, two waves per SIMD, and ran slower).  D addresses
// the medium's planes as M does the state's.  Returns the largest Courant
// number of the lane's cells (0 on lanes that update none).
template <typename T>
struct VarXEdge {
  T a1, a2, iz;  // strengths of the lane's left edge and 1/(Z_left + Z)
  T Fp, Fn;      // its limited normal correction
};

template <typename T, int LIM>
__device__ __attribute__((always_inline)) inline VarXEdge<T> var_xedge(const Row3<T> &Q,
                                                                        const Row3<T> &E,
                                                                        T dtdx) {
  VarXEdge<T> X;
  const T pl = shr(Q.p), ul = shr(Q.u), cl = shr(E.p), Zl = shr(E.u), wl = shr(E.v);
  var_strengths(Zl, E.u, Q.p - pl, Q.u - ul, X.a1, X.a2, X.iz);
  T l1, l2;
  var_limited<T, LIM>(X.a1, X.a2, shl(X.a1), shr(X.a2), Zl, E.u, wl, E.v, l1, l2);
  var_corr(cl, Zl, E.p, E.u, l1, l2, dtdx, X.Fp, X.Fn);
  return X;
}

template <typename T, int LIM>
__device__ __attribute__((always_inline)) inline T march_up_var(const MarchLanes<T> &M,
                                                                const MarchLanes<T> &D,
                                                                const Coef<T> &k, int r0, int r1) {
  const T dtdx = k.dtdx, dtdy = k.dtdy;
  Row3<T> Q[5], E[5], Qa, Ea;  // window rows r-2 .. r+2; row r+3
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    M.fetch(Q[d], r0 + d - 2);
    D.fetch(E[d], r0 + d - 2);
  }
  M.fetch(Qa, r0 + 3);
  D.fetch(Ea, r0 + 3);
  // y-edge e between window rows e and e+1
  T b1[4], b2[4], bz[4];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    var_strengths(E[e].u, E[e + 1].u, Q[e + 1].p - Q[e].p, Q[e + 1].v - Q[e].v, b1[e], b2[e],
                  bz[e]);
  // x-edges of rows r0-1 and r0; the x-fluctuation p-part of row r0-1
  T Xpb;
  {
    const VarXEdge<T> B = var_xedge<T, LIM>(Q[1], E[1], dtdx);
    Xpb = E[1].p * E[1].u * (B.a2 + shl(B.a1));
  }
  VarXEdge<T> XR = var_xedge<T, LIM>(Q[2], E[2], dtdx);
  T cfl = T(0);
  for (int r = r0; r < r1; ++r) {
    // x-edges of row r+1 and its cells' x-fluctuation p-part
    const VarXEdge<T> XN = var_xedge<T, LIM>(Q[3], E[3], dtdx);
    const T Xpt = E[3].p * E[3].u * (XN.a2 + shl(XN.a1));
    // the cell's x-line: its left edge here, its right edge the next lane's left
    VarLine<T> X;
    X.Fl_p = XR.Fp, X.Fl_n = XR.Fn, X.Fr_p = shl(XR.Fp), X.Fr_n = shl(XR.Fn);
    const T a1r = shl(XR.a1);
    X.xs = XR.a2 + a1r;
    X.xd = XR.a2 - a1r;
    X.izl = XR.iz, X.izr = shl(XR.iz);
    X.cl = shr(E[2].p), X.zl = shr(E[2].u), X.c0 = E[2].p, X.z0 = E[2].u;
    X.cr = shl(E[2].p), X.zr = shl(E[2].u);
    // the y-line from the carried edges
    const T Cc[5] = {E[0].p, E[1].p, E[2].p, E[3].p, E[4].p};
    const T Zc[5] = {E[0].u, E[1].u, E[2].u, E[3].u, E[4].u};
    const VarLine<T> Y = var_line_edges<T, LIM>(b1, b2, bz, Cc, Zc, E[1].v, E[2].v, E[3].v, dtdy);
    // y-fluctuation p-parts of the cells left and right
    const T Yp = E[2].p * E[2].u * Y.xs;
    T pn, un, vn, cj;
    var_combine(X, Y, Xpb, Xpt, shr(Yp), shl(Yp), Q[2].p, Q[2].u, Q[2].v, dtdx, dtdy, pn, un, vn,
                cj);
    if (M.out) cfl = fmax(cfl, cj);
    M.emit(pn, un, vn, r);
    // slide up one row
    Xpb = X.c0 * X.z0 * X.xs;
    XR = XN;
#pragma unroll
    for (int d = 0; d < 4; ++d) Q[d] = Q[d + 1], E[d] = E[d + 1];
    Q[4] = Qa, E[4] = Ea;
    if (r + 4 <= r1 + 1) {
      M.fetch(Qa, r + 4);
      D.fetch(Ea, r + 4);
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) b1[e] = b1[e + 1], b2[e] = b2[e + 1], bz[e] = bz[e + 1];
    var_strengths(E[3].u, E[4].u, Q[4].p - Q[3].p, Q[4].v - Q[3].v, b1[3], b2[3], bz[3]);
  }
  return cfl;
}

// VARS: bit 0 -> DIRECT tiles may occur, bit 1 -> MARCH tiles, bit 2 -> PACKED
// tiles (the step without branch recording or a medium only).
// TC: the transverse-correction variant (never with MASKS).
template <typename T, int LIM, bool MASKS, int VARS, bool TC, bool VAR = false>
__device__ __attribute__((always_inline)) inline double do_unit(const StepArgs &a, int t, int q,
                                                                int &inst) {
  const TileEntry te = uniform_row(a.tiles[t]);
  if constexpr ((VARS & 4) != 0 && !MASKS && !VAR) {
    if (te.patch < 0) {
      // PACKED tile -1 - te.patch: wavefront q works its column blocks
      const PackWave pw = uniform_row(a.packs[4 * (-1 - te.patch) + q]);
      // every piece shares the first one's instance and cell sizes
      const PatchRow p0 = uniform_row(a.patches[pw.patch[0]]);
      const InstRow in = uniform_row(a.inst[p0.inst]);
      inst = p0.inst;
      const double dt = a.dt_override > 0.0 ? a.dt_override : a.dt[p0.inst];
      const Coef<T> k = make_coef<T>(in.c, in.Z, dt, p0.dx, p0.dy);
      if (pw.n > 0) {
        const int lx = (int)threadIdx.x & 63;
        // the lane's piece: the last whose first lane is at or before it
        unsigned org = pw.org[0], ldb = pw.ldb[0], plb = pw.plb[0];
        int pw_w = pw.w[0], lane0 = pw.lane0[0], lim = pw.lim[0];
#pragma unroll
        for (int n = 1; n < kMaxPieces; ++n)
          if (n < pw.n && lx >= pw.lane0[n]) {
            org = pw.org[n], ldb = pw.ldb[n], plb = pw.plb[n];
            pw_w = pw.w[n], lane0 = pw.lane0[n], lim = pw.lim[n];
          }
        const int off = lx - lane0;  // the lane holds column c0 - 2 + off of its piece
        PackedLanes<T> M;
        M.base = reinterpret_cast<const char *>(a.qin);
        M.ob = __builtin_amdgcn_make_buffer_rsrc(a.qout, 0, a.pool_bytes, kRawBufferWord3);
        M.colb = org + (unsigned)min(off, lim) * (unsigned)sizeof(T);
        M.ocolb = org + (unsigned)off * (unsigned)sizeof(T);
        M.ldb = ldb;
        M.plb = plb;
        M.rlo = pw.r0 - 2;
        M.rhi = pw.r1 + 1;
        M.out = off >= 2 && off < pw_w + 2;
        const bool up = ((t * (kThreads / kMarchWidth) + q) & 1) == 0;
        if constexpr (TC) {
          if (up)
            march_up_tc<T, LIM>(M, k, pw.r0, pw.r1);
          else
            march_down_tc<T, LIM>(M, k, pw.r0, pw.r1);
        } else {
          if (up)
            march_up<T, LIM, false>(M, k, pw.r0, pw.r1, nullptr);
          else
            march_down<T, LIM>(M, k, pw.r0, pw.r1);
        }
      }
      return fmax(in.c * (dt / p0.dx), in.c * (dt / p0.dy));
    }
  }
  const PatchRow pr = uniform_row(a.patches[te.patch]);
  const InstRow in = uniform_row(a.inst[pr.inst]);
  inst = pr.inst;
  const double dt = a.dt_override > 0.0 ? a.dt_override : a.dt[pr.inst];
  const Coef<T> k = make_coef<T>(in.c, in.Z, dt, pr.dx, pr.dy);
  const int64_t org = pr.q_off + 2 * (int64_t)pr.ld + pr.col0;
  const T *qi = reinterpret_cast<const T *>(a.qin) + org;
  T *qo = reinterpret_cast<T *>(a.qout) + org;
  uint8_t *masks = MASKS ? a.masks + pr.mask_off : nullptr;
  const int tw = pr.tw;
  if ((VARS & 2) && (!(VARS & 1) || pr.variant == kMarch)) {
    // segment q of the tile; its rows are wave-uniform
    const int lx = (int)threadIdx.x & 63;
    const int rows = pr.th / (kThreads / kMarchWidth);
    const int i = te.tx * (kMarchWidth - 4) - 2 + lx;
    const int r0 = te.ty * pr.th + q * rows;
    const int r1 = min(r0 + rows, pr.my);
    if constexpr (VAR) {
      // heterogeneous medium: the tile's Courant number is reduced from its cells
      T cfl = T(0);
      if (r0 < r1) {
        const MarchLanes<T> M(qi, qo, pr, lx, i);
        const T *mi = reinterpret_cast<const T *>(a.medium) + org;
        const MarchLanes<T> D(mi, const_cast<T *>(mi), pr, lx, i);
        cfl = march_up_var<T, LIM>(M, D, k, r0, r1);
      }
      return wave_max((double)cfl);
    }
    if (r0 < r1) {
      const MarchLanes<T> M(qi, qo, pr, lx, i);
      // segments alternate direction up the patch (the recording step marches up)
      const bool up = MASKS || ((te.ty * (kThreads / kMarchWidth) + q) & 1) == 0;
      if constexpr (TC) {
        if (up)
          march_up_tc<T, LIM>(M, k, r0, r1);
        else
          march_down_tc<T, LIM>(M, k, r0, r1);
      } else {
        if (up)
          march_up<T, LIM, MASKS>(M, k, r0, r1, masks);
        else
          march_down<T, LIM>(M, k, r0, r1);
      }
    }
  } else if (VARS & 1) {
    // the threads q*64 .. q*64+63 of the tile's 256
    const int tid = q * 64 + ((int)threadIdx.x & 63);
    const int lx = tid % tw, ly = tid / tw;
    const int rows_per_thread = pr.th / (kThreads / tw);
    const int i = te.tx * tw + lx;
    const int j0 = te.ty * pr.th + ly * rows_per_thread;
    const int j1 = min(j0 + rows_per_thread, pr.my);
    const Planes<T> q{qi, qi + pr.plane, qi + 2 * pr.plane, pr.ld};
    if constexpr (VAR) {
      // heterogeneous medium: the tile's Courant number is reduced from its cells
      const int64_t first = 2 * (int64_t)pr.ld + 2;  // padded (-2, -2) from interior (0, 0)
      const uint32_t plb = (uint32_t)(pr.plane * (int64_t)sizeof(T));
      const Planes32<T> q32{reinterpret_cast<const char *>(qi - first), (uint32_t)pr.ld, plb};
      const Planes32<T> md{reinterpret_cast<const char *>(reinterpret_cast<const T *>(a.medium) +
                                                          org - first),
                           (uint32_t)pr.ld, plb};
      T cfl = T(0);
      if (i < pr.mx && j0 < j1) cfl = march_col_var<T, LIM>(q32, md, i, j0, j1, k, qo, pr);
      return wave_max((double)cfl);
    }
    if (i < pr.mx && j0 < j1) {
      for (int j = j0; j < j1; ++j) {
        T pn, un, vn;
        CellMasks mk;
        if constexpr (TC)
          cell_update_tc<T, LIM>(q, i, j, k, pn, un, vn);
        else
          cell_update<T, LIM, MASKS>(q, i, j, k, pn, un, vn, &mk);
        store<T>(qo, pr.plane, pr.ld, i, j, pr.mx, pr.my, pr.bc, pn, un, vn);
        if constexpr (MASKS) {
          const int64_t mld = pr.mx + 1;
          masks[(int64_t)j * mld + i] = (uint8_t)mk.own;
          if (i == pr.mx - 1) masks[(int64_t)j * mld + i + 1] = (uint8_t)mk.right;
          if (j == pr.my - 1) {
            masks[(int64_t)(j + 1) * mld + i] = (uint8_t)mk.top;
            if (i == pr.mx - 1) masks[(int64_t)(j + 1) * mld + i + 1] = 0;  // no edge owns it
          }
        }
      }
    }
  }
  // Courant number of the tile (Sec. 2.4 eq. (2.10)): every edge of a
  // homogeneous instance carries the speeds -c, 0, +c, so each x-edge gives
  // c dt/dx and each y-edge c dt/dy, and every tile holds edges of both kinds.
  return fmax(in.c * (dt / pr.dx), in.c * (dt / pr.dy));
}

__device__ inline unsigned long long load_agent(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// File the step's Courant numbers: per instance the max over the XCD groups'
// accumulators (which are cleared), the level max, running maxima, and dt set
// (dt_override > 0) and rescaled by cfl_desired / cfl (cfl_desired > 0),
// Sec. 2.5 eq. (2.11).  Run by one whole workgroup after every tile of the
// step has finished.
__device__ inline void finish_step(const CflSlots &c, double dt_override, double cfl_desired) {
  __shared__ double s_lvl[kThreads / 64];
  const int tid = (int)threadIdx.x;
  double lvl = 0.0;
  for (int k = tid; k < c.n_inst; k += kThreads) {
    unsigned long long b = 0;
    for (int g = 0; g < kGroups; ++g) {
      unsigned long long *slot = &c.inst_acc[(int64_t)g * c.n_inst + k];
      b = max(b, load_agent(slot));
      __hip_atomic_store(slot, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const double cfl = __longlong_as_double((long long)b);
    c.cfl_last[k] = cfl;
    c.cfl_max[k] = fmax(c.cfl_max[k], cfl);
    double dt = dt_override > 0.0 ? dt_override : c.dt[k];
    if (cfl_desired > 0.0 && cfl > 0.0) dt = dt * cfl_desired / cfl;
    c.dt[k] = dt;
    lvl = fmax(lvl, cfl);
  }
  lvl = wave_max(lvl);
  if ((tid & 63) == 0) s_lvl[tid >> 6] = lvl;
  __syncthreads();
  if (tid == 0) {
    double m = s_lvl[0];
    for (int w = 1; w < kThreads / 64; ++w) m = fmax(m, s_lvl[w]);
    c.level_last[0] = m;
  }
}

// A workgroup's running maximum over consecutive tiles of one instance, filed
// into its XCD group's slot with one atomic max per run.  The atomic returns
// and is waited for before the workgroup retires.
struct CflRun {
  int inst = -1;
  double val = 0.0;
};

__device__ inline void flush_cfl(const StepArgs &a, int group, CflRun &run) {
  if (run.inst >= 0 && run.val > 0.0) {
    const unsigned long long old = __hip_atomic_fetch_max(
        &a.slots.inst_acc[(int64_t)group * a.slots.n_inst + run.inst], dbits(run.val),
        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("s_waitcnt vmcnt(0)" : : "v"(old) : "memory");
  }
  run.inst = -1;
  run.val = 0.0;
}

// Thread 0 after a tile: record the tile's value (for the per-patch array)
// where every XCD can read it, and fold it into the running maximum.
__device__ inline void file_tile(const StepArgs &a, int group, CflRun &run, int t, double m,
                                 int inst) {
  __hip_atomic_store(&a.slots.cfl_tile[t], m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (inst != run.inst) {
    flush_cfl(a, group, run);
    run.inst = inst;
  }
  run.val = fmax(run.val, m);
}

// Persistent launch.  Tiles are split into up to kGroups contiguous runs, one
// per XCD: workgroups are dispatched round-robin over the XCDs, so workgroup b
// takes run b % groups, and the run's neighbouring tiles (whose halos
// overlap) share that XCD's L2.  Within a run the workgroups take tiles
// round-robin (largest patches first), with no atomics; the four wavefronts
// of a workgroup work the four quarters of its tile independently.  With a
// grid of one workgroup per tile the hardware dispatcher balances the load.
// Heterogeneous medium: the four wavefronts' Courant numbers of a tile.
__device__ inline double tile_max(double m, int lane, int wave) {
  __shared__ double s_m[kThreads / 64];
  if (lane == 0) s_m[wave] = m;
  __syncthreads();
  double r = s_m[0];
  for (int w = 1; w < kThreads / 64; ++w) r = fmax(r, s_m[w]);
  __syncthreads();
  return r;
}

template <typename T, int LIM, bool MASKS, int VARS, bool TC, bool VAR = false>
__device__ __attribute__((always_inline)) inline void step_body(const StepArgs &a) {
  CflRun run;  // meaningful in lane 0 of each wavefront
  const int lane = (int)threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  if (!a.persistent) {
    const int t = a.tile_base + (int)blockIdx.x;
    if (t < a.n_tiles) {
      int inst = 0;
      double m = do_unit<T, LIM, MASKS, VARS, TC, VAR>(a, t, wave, inst);
      if constexpr (VAR) m = tile_max(m, lane, wave);
      if (lane == 0 && wave == 0) {
        file_tile(a, 0, run, t, m, inst);
        flush_cfl(a, 0, run);
      }
    }
    return;
  }
  const int G = (int)gridDim.x;
  const int groups = min(kGroups, G);
  const int x = (int)blockIdx.x % groups, y = (int)blockIdx.x / groups;
  const int in_group = G / groups + (x < G % groups ? 1 : 0);
  const int beg = (int)((int64_t)a.n_tiles * x / groups);
  const int end = (int)((int64_t)a.n_tiles * (x + 1) / groups);
  for (int t = beg + y; t < end; t += in_group) {
    int inst = 0;
    double m = do_unit<T, LIM, MASKS, VARS, TC, VAR>(a, t, wave, inst);
    if constexpr (VAR) m = tile_max(m, lane, wave);
    if (lane == 0 && wave == 0) file_tile(a, x, run, t, m, inst);
  }
  // Retire: the workgroup's values are filed (and waited for) before its
  // count; the last workgroup of each run counts the run, and the last run's
  // last workgroup files the step and rewinds the counters for the next launch.
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    flush_cfl(a, x, run);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    int last = 0;
    const unsigned d = __hip_atomic_fetch_add(&a.retire[x * kLine], 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    if ((int)d == in_group - 1) {
      const unsigned g = __hip_atomic_fetch_add(&a.retire[kGroups * kLine], 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
      last = (int)g == groups - 1;
    }
    s_last = last;
  }
  __syncthreads();
  if (s_last) {
    finish_step(a.slots, a.dt_override, a.cfl_desired);
    if (threadIdx.x <= kGroups)
      __hip_atomic_store(&a.retire[threadIdx.x * kLine], 0u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T, int LIM, bool MASKS, int VARS, bool TC>
__global__ __launch_bounds__(kThreads) void step_kernel(StepArgs a) {
  step_body<T, LIM, MASKS, VARS, TC>(a);
}

// Heterogeneous media: DIRECT tiles, MARCH tiles (VARS 2), or both (3).
template <typename T, int LIM, int VARS>
__global__ __launch_bounds__(kThreads) void step_kernel_var(StepArgs a) {
  step_body<T, LIM, false, VARS, false, true>(a);
}

// MARCH-only levels: a kernel of their own, free of the DIRECT path's registers.
template <typename T, int LIM, bool MASKS, bool TC>
__global__ __launch_bounds__(kThreads) void step_kernel_march(StepArgs a) {
  step_body<T, LIM, MASKS, 2, TC>(a);
}

// --------------------------------------------------------------------------
// Ghost fill of the current state (physical boundaries only)
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void fill_ghosts_kernel(const PatchRow *patches, T *q) {
  const PatchRow pr = patches[blockIdx.y];
  if (pr.bc == WS_BC_NONE) return;
  const int64_t org = pr.q_off + 2 * (int64_t)pr.ld + pr.col0;
  T *base = q + org;
  // the ghost ring only
  const int ring = ring_size(pr.mx, pr.my);
  for (int g = blockIdx.x * kThreads + threadIdx.x; g < ring; g += gridDim.x * kThreads) {
    int i, j;
    ring_cell(g, pr.mx, pr.my, i, j);
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

// Ghosts of the patches of a tiled level, each copied from the interior cell
// of the patch (possibly itself) that its host-built table names (Sec. 2.2:
// copied from the patch of the same level holding it, after the physical
// condition has mapped a ghost outside the domain into it).  The table holds,
// per ghost, the pool element offset of the source cell's first component and
// the source patch's plane stride, so each ghost is one table load and three
// data loads.  Writes ghosts, reads interiors: no cell is both.
template <typename T>
__global__ __launch_bounds__(kThreads) void link_ghosts_kernel(const PatchRow *patches,
                                                               const int64_t *ring0,
                                                               const int64_t *src, T *q) {
  const PatchRow pr = patches[blockIdx.y];
  const int ring = ring_size(pr.mx, pr.my);
  const int64_t *tab = src + 2 * ring0[blockIdx.y];
  T *dst = q + pr.q_off + 2 * (int64_t)pr.ld + pr.col0;
  for (int g = blockIdx.x * kThreads + threadIdx.x; g < ring; g += gridDim.x * kThreads) {
    int i, j;
    ring_cell(g, pr.mx, pr.my, i, j);
    const int64_t so = tab[2 * g], sp = tab[2 * g + 1];
    const T a = q[so], b = q[so + sp], c = q[so + 2 * sp];
    const int64_t d = (int64_t)j * pr.ld + i;
    dst[d] = a;
    dst[pr.plane + d] = b;
    dst[2 * pr.plane + d] = c;
  }
}

// --------------------------------------------------------------------------
// dt and Courant-number bookkeeping
// --------------------------------------------------------------------------
__global__ void set_dt_kernel(double *dt, int n, double value) {
  for (int k = threadIdx.x; k < n; k += blockDim.x) dt[k] = value;
}

__global__ __launch_bounds__(kThreads) void finish_step_kernel(CflSlots c, double cfl_desired) {
  finish_step(c, 0.0, cfl_desired);
}

// Per-patch Courant numbers of the last step (the per-patch maximum-speed array
// of Sec. 3.2.2), reduced from the per-tile values when they are read.
__global__ __launch_bounds__(kThreads) void patch_cfl_kernel(const PatchRow *patches,
                                                           int n_patches, const double *cfl_tile,
                                                           double *cfl_patch) {
  __shared__ double s_red[kThreads / 64];
  const int k = blockIdx.x;
  if (k >= n_patches) return;
  const PatchRow pr = patches[k];
  double m = 0.0;
  for (int t = pr.tile_begin + (int)threadIdx.x; t < pr.tile_begin + pr.n_tiles; t += kThreads)
    m = fmax(m, cfl_tile[t]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) m = fmax(m, s_red[w]);
    cfl_patch[k] = fmax(m, s_red[0]);
  }
}

// --------------------------------------------------------------------------
// Conservation sums: FP64 per-tile partials, per-patch sums of those, per-
// instance sums of those; every stage in a fixed order.
// --------------------------------------------------------------------------
// One workgroup per sum tile (kSumTile x kSumTile cells of a patch, in a
// list of their own), so the order of every addition is fixed by the patch
// sizes alone, whatever the step's tiling.
template <typename T>
__global__ __launch_bounds__(kThreads) void tile_sums_kernel(const PatchRow *patches,
                                                           const TileEntry *stiles, const T *q,
                                                           double *partials) {
  __shared__ double s[3][kThreads];
  const TileEntry te = stiles[blockIdx.x];
  const PatchRow pr = patches[te.patch];
  constexpr int rpt = kSumTile / (kThreads / kSumTile);
  const int lx = threadIdx.x % kSumTile, ly = threadIdx.x / kSumTile;
  const int i = te.tx * kSumTile + lx;
  const int j0 = te.ty * kSumTile + ly * rpt;
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

// Fixed-order FP64 reduction of 3-vectors over a workgroup: thread t adds the
// items t, t + 256, ... of its range, then a tree over the threads.
__device__ inline void block_sum3(double acc[3], double *out) {
  __shared__ double s[3][kThreads];
  for (int m = 0; m < 3; ++m) s[m][threadIdx.x] = acc[m];
  __syncthreads();
  for (int w = kThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int m = 0; m < 3; ++m) s[m][threadIdx.x] += s[m][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = s[threadIdx.x][0];
}

// One workgroup per patch: the sums of its sum tiles' partials.
__global__ __launch_bounds__(kThreads) void patch_sums_kernel(const PatchRow *patches,
                                                            const double *partials,
                                                            double *patch_sums) {
  const PatchRow pr = patches[blockIdx.x];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int t = pr.sum_begin + (int)threadIdx.x; t < pr.sum_begin + pr.sum_n; t += kThreads)
    for (int m = 0; m < 3; ++m) acc[m] += partials[3 * (int64_t)t + m];
  block_sum3(acc, patch_sums + 3 * (int64_t)blockIdx.x);
}

// One workgroup per instance: the sums over its patches, in patch order.
__global__ __launch_bounds__(kThreads) void instance_sums_kernel(const PatchRow *patches,
                                                               int n_patches,
                                                               const double *patch_sums,
                                                               double *sums) {
  const int inst = (int)blockIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int k = (int)threadIdx.x; k < n_patches; k += kThreads)
    if (patches[k].inst == inst)
      for (int m = 0; m < 3; ++m) acc[m] += patch_sums[3 * (int64_t)k + m];
  block_sum3(acc, sums + 3 * (int64_t)inst);
}

template <typename T, int LIM, bool MASKS, int VARS, bool TC>
hipError_t launch_step_t(const StepArgs &a, int grid, hipStream_t s) {
  if constexpr (VARS == 2)
    hipLaunchKernelGGL((step_kernel_march<T, LIM, MASKS, TC>), dim3(grid), dim3(kThreads), 0, s,
                       a);
  else
    hipLaunchKernelGGL((step_kernel<T, LIM, MASKS, VARS, TC>), dim3(grid), dim3(kThreads), 0, s,
                       a);
  return hipGetLastError();
}

// PACKED tiles: a kernel for levels with PACKED tiles only, one for PACKED
// with MARCH, and one with every variant.
template <typename T, int LIM, bool MASKS, bool TC>
hipError_t launch_step_v(int vars, const StepArgs &a, int grid, hipStream_t s) {
  switch (vars) {
    case 1: return launch_step_t<T, LIM, MASKS, 1, TC>(a, grid, s);
    case 2: return launch_step_t<T, LIM, MASKS, 2, TC>(a, grid, s);
    case 3: return launch_step_t<T, LIM, MASKS, 3, TC>(a, grid, s);
    default:
      if constexpr (MASKS) {
        return hipErrorInvalidValue;
      } else {
        if (vars == 4) return launch_step_t<T, LIM, false, 4, TC>(a, grid, s);
        if (vars == 6) return launch_step_t<T, LIM, false, 6, TC>(a, grid, s);
        return launch_step_t<T, LIM, false, 7, TC>(a, grid, s);
      }
  }
}

// Branch recording exists for the MC limiter of the default variant only.
template <typename T, int LIM>
hipError_t launch_step_m(bool tc, int vars, const StepArgs &a, int grid, hipStream_t s) {
  if (tc) {
    if (a.masks) return hipErrorInvalidValue;
    return launch_step_v<T, LIM, false, true>(vars, a, grid, s);
  }
  if constexpr (LIM == WS_LIM_MC) {
    if (a.masks) return launch_step_v<T, LIM, true, false>(vars, a, grid, s);
  } else {
    if (a.masks) return hipErrorInvalidValue;
  }
  return launch_step_v<T, LIM, false, false>(vars, a, grid, s);
}

template <typename T, int LIM>
hipError_t launch_step_var_l(int vars, const StepArgs &a, int grid, hipStream_t s) {
  switch (vars) {
    case 1: hipLaunchKernelGGL((step_kernel_var<T, LIM, 1>), dim3(grid), dim3(kThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL((step_kernel_var<T, LIM, 2>), dim3(grid), dim3(kThreads), 0, s, a); break;
    case 3: hipLaunchKernelGGL((step_kernel_var<T, LIM, 3>), dim3(grid), dim3(kThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_var(int lim, int vars, const StepArgs &a, int grid, hipStream_t s) {
  if (a.masks) return hipErrorInvalidValue;
  switch (lim) {
    case WS_LIM_NONE: return launch_step_var_l<T, WS_LIM_NONE>(vars, a, grid, s);
    case WS_LIM_VANLEER: return launch_step_var_l<T, WS_LIM_VANLEER>(vars, a, grid, s);
    default: return launch_step_var_l<T, WS_LIM_MC>(vars, a, grid, s);
  }
}

// limiter: WS_LIM_*, optionally with WS_TRANSVERSE_CORR or kMediumFlag.
template <typename T>
hipError_t launch_step_l(int limiter, int vars, const StepArgs &a, int grid, hipStream_t s) {
  if (limiter & kMediumFlag) {
    if (vars < 1 || vars > 3 || !a.medium || (limiter & WS_TRANSVERSE_CORR))
      return hipErrorInvalidValue;
    return launch_step_var<T>(limiter & 0xff, vars, a, grid, s);
  }
  const bool tc = (limiter & WS_TRANSVERSE_CORR) != 0;
  switch (limiter & ~WS_TRANSVERSE_CORR) {
    case WS_LIM_NONE: return launch_step_m<T, WS_LIM_NONE>(tc, vars, a, grid, s);
    case WS_LIM_VANLEER: return launch_step_m<T, WS_LIM_VANLEER>(tc, vars, a, grid, s);
    default: return launch_step_m<T, WS_LIM_MC>(tc, vars, a, grid, s);
  }
}

template <typename T, int LIM, bool TC>
int occupancy_of(int vars, int *n) {
  hipError_t e;
  switch (vars) {
    case 1:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(n, step_kernel<T, LIM, false, 1, TC>,
                                                       kThreads, 0);
      break;
    case 2:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(n, step_kernel_march<T, LIM, false, TC>,
                                                       kThreads, 0);
      break;
    case 3:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(n, step_kernel<T, LIM, false, 3, TC>,
                                                       kThreads, 0);
      break;
    case 4:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(n, step_kernel<T, LIM, false, 4, TC>,
                                                       kThreads, 0);
      break;
    case 6:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(n, step_kernel<T, LIM, false, 6, TC>,
                                                       kThreads, 0);
      break;
    default:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(n, step_kernel<T, LIM, false, 7, TC>,
                                                       kThreads, 0);
      break;
  }
  return e == hipSuccess ? 0 : -1;
}

template <typename T, int LIM>
int occupancy_t(bool tc, int vars, int *n) {
  return tc ? occupancy_of<T, LIM, true>(vars, n) : occupancy_of<T, LIM, false>(vars, n);
}

}  // namespace

hipError_t launch_step(int dtype, int limiter, int vars, const StepArgs &a, int grid,
                       hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  return dtype == WS_F32 ? launch_step_l<float>(limiter, vars, a, grid, s)
                         : launch_step_l<double>(limiter, vars, a, grid, s);
}

template <typename T, int LIM>
int occupancy_var(int vars, int *n) {
  hipError_t e;
  if (vars == 2)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(n, step_kernel_var<T, LIM, 2>, kThreads, 0);
  else if (vars == 3)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(n, step_kernel_var<T, LIM, 3>, kThreads, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(n, step_kernel_var<T, LIM, 1>, kThreads, 0);
  return e == hipSuccess ? 0 : -1;
}

template <typename T>
int occupancy_l(int limiter, int vars, int *wg_per_cu) {
  if (limiter & kMediumFlag) {
    switch (limiter & 0xff) {
      case WS_LIM_NONE: return occupancy_var<T, WS_LIM_NONE>(vars, wg_per_cu);
      case WS_LIM_VANLEER: return occupancy_var<T, WS_LIM_VANLEER>(vars, wg_per_cu);
      default: return occupancy_var<T, WS_LIM_MC>(vars, wg_per_cu);
    }
  }
  const bool tc = (limiter & WS_TRANSVERSE_CORR) != 0;
  switch (limiter & ~WS_TRANSVERSE_CORR) {
    case WS_LIM_NONE: return occupancy_t<T, WS_LIM_NONE>(tc, vars, wg_per_cu);
    case WS_LIM_VANLEER: return occupancy_t<T, WS_LIM_VANLEER>(tc, vars, wg_per_cu);
    default: return occupancy_t<T, WS_LIM_MC>(tc, vars, wg_per_cu);
  }
}

int step_occupancy(int dtype, int limiter, int vars, int *wg_per_cu) {
  return dtype == WS_F32 ? occupancy_l<float>(limiter, vars, wg_per_cu)
                         : occupancy_l<double>(limiter, vars, wg_per_cu);
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

hipError_t launch_link_ghosts(int dtype, const PatchRow *patches, int n_patches, int max_ring,
                              const int64_t *ring0, const int64_t *src, void *q, hipStream_t s) {
  if (n_patches <= 0) return hipSuccess;
  const dim3 grid((unsigned)max(1, min(64, (max_ring + kThreads - 1) / kThreads)),
                  (unsigned)n_patches);
  if (dtype == WS_F32)
    hipLaunchKernelGGL(link_ghosts_kernel<float>, grid, dim3(kThreads), 0, s, patches, ring0, src,
                       reinterpret_cast<float *>(q));
  else
    hipLaunchKernelGGL(link_ghosts_kernel<double>, grid, dim3(kThreads), 0, s, patches, ring0,
                       src, reinterpret_cast<double *>(q));
  return hipGetLastError();
}

hipError_t launch_set_dt(const CflSlots &c, double value, hipStream_t s) {
  hipLaunchKernelGGL(set_dt_kernel, dim3(1), dim3(256), 0, s, c.dt, c.n_inst, value);
  return hipGetLastError();
}

hipError_t launch_finish_step(const CflSlots &c, double cfl_desired, hipStream_t s) {
  hipLaunchKernelGGL(finish_step_kernel, dim3(1), dim3(kThreads), 0, s, c, cfl_desired);
  return hipGetLastError();
}

hipError_t launch_patch_cfl(const PatchRow *patches, int n_patches, const double *cfl_tile,
                            double *cfl_patch, hipStream_t s) {
  if (n_patches <= 0) return hipSuccess;
  hipLaunchKernelGGL(patch_cfl_kernel, dim3(n_patches), dim3(kThreads), 0, s, patches, n_patches,
                     cfl_tile, cfl_patch);
  return hipGetLastError();
}

hipError_t launch_sums(int dtype, const PatchRow *patches, int n_patches, const TileEntry *stiles,
                       int n_stiles, const void *q, double *partials, double *patch_sums,
                       int n_inst, double *sums, hipStream_t s) {
  if (n_stiles > 0) {
    if (dtype == WS_F32)
      hipLaunchKernelGGL(tile_sums_kernel<float>, dim3(n_stiles), dim3(kThreads), 0, s, patches,
                         stiles, reinterpret_cast<const float *>(q), partials);
    else
      hipLaunchKernelGGL(tile_sums_kernel<double>, dim3(n_stiles), dim3(kThreads), 0, s, patches,
                         stiles, reinterpret_cast<const double *>(q), partials);
  }
  hipLaunchKernelGGL(patch_sums_kernel, dim3(n_patches), dim3(kThreads), 0, s, patches, partials,
                     patch_sums);
  hipLaunchKernelGGL(instance_sums_kernel, dim3(n_inst), dim3(kThreads), 0, s, patches, n_patches,
                     patch_sums, sums);
  return hipGetLastError();
}

}  // namespace ws
