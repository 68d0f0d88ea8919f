// Device helpers shared by the forward and adjoint kernels of the
// wave-propagation library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/wavestep.h"

namespace ws {

// --------------------------------------------------------------------------
// Per-patch coefficients of the closed forms (computed in FP64, rounded once
// to T)
// --------------------------------------------------------------------------
template <typename T>
struct Coef {
  T Z;
  T h, hz;                // c/2, c/(2Z): fluctuation factors
  T fx, fxz, fy, fyz;     // c(1-nu)/4 and /Z: correction factors
  T gx, gxz, gy, gyz;     // dtdx c^2/8 and /Z: transverse factors
  T dtdx, dtdy;
  T tx, ty;               // 1 - nu: the correction moved into the split vectors
};

// Wave-uniform values are moved to scalar registers.
__device__ inline double uniform(double v) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
__device__ inline float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

template <typename T>
__device__ inline Coef<T> make_coef(double c, double Z, double dt, double dx, double dy) {
  const double dtdx = dt / dx, dtdy = dt / dy, iz = 1.0 / Z;
  const double fx = 0.25 * c * (1.0 - c * dtdx), fy = 0.25 * c * (1.0 - c * dtdy);
  const double gx = 0.125 * dtdx * c * c, gy = 0.125 * dtdy * c * c;
  Coef<T> k;
  k.Z = (T)Z;
  k.h = (T)(0.5 * c);
  k.hz = (T)(0.5 * c * iz);
  k.fx = (T)fx;
  k.fxz = (T)(fx * iz);
  k.fy = (T)fy;
  k.fyz = (T)(fy * iz);
  k.gx = (T)gx;
  k.gxz = (T)(gx * iz);
  k.gy = (T)gy;
  k.gyz = (T)(gy * iz);
  k.dtdx = (T)dtdx;
  k.dtdy = (T)dtdy;
  k.tx = (T)(1.0 - c * dtdx);
  k.ty = (T)(1.0 - c * dtdy);
  T *f = &k.Z;
  for (int n = 0; n < (int)(sizeof(Coef<T>) / sizeof(T)); ++n) f[n] = uniform(f[n]);
  return k;
}

// A table row read by a whole workgroup, moved to scalar registers word by
// word (the kernel stores to memory, so the compiler cannot use scalar loads
// for it and would otherwise treat its fields as per-lane values).
template <typename S>
__device__ inline S uniform_row(const S &v) {
  static_assert(sizeof(S) % 4 == 0, "row must be whole words");
  uint32_t w[sizeof(S) / 4];
  __builtin_memcpy(w, &v, sizeof(S));
#pragma unroll
  for (int n = 0; n < (int)(sizeof(S) / 4); ++n) w[n] = __builtin_amdgcn_readfirstlane(w[n]);
  S out;
  __builtin_memcpy(&out, w, sizeof(S));
  return out;
}

// Whole-wavefront lane shifts (DPP): shr gives lane l the value of lane l-1,
// shl the value of lane l+1.  Lanes without a source read 0 (never used).
__device__ inline int dpp_shr_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ inline int dpp_shl_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ inline double shr(double v) {
  return __hiloint2double(dpp_shr_i(__double2hiint(v)), dpp_shr_i(__double2loint(v)));
}
__device__ inline double shl(double v) {
  return __hiloint2double(dpp_shl_i(__double2hiint(v)), dpp_shl_i(__double2loint(v)));
}
__device__ inline float shr(float v) { return __int_as_float(dpp_shr_i(__float_as_int(v))); }
__device__ inline float shl(float v) { return __int_as_float(dpp_shl_i(__float_as_int(v))); }

// --------------------------------------------------------------------------
// Limiter on unscaled strengths: psi(a, a_up) = phi(a_up/a) a (the limiters
// are positively homogeneous).  MC: minmod(2a, 2a_up, (a + a_up)/2), written
// branch-free.
// --------------------------------------------------------------------------
template <typename T, int LIM>
__device__ inline T limited(T a, T b) {
  if constexpr (LIM == WS_LIM_NONE) {
    return a;
  } else if constexpr (LIM == WS_LIM_VANLEER) {
    // van Leer, phi(theta) = (theta + |theta|)/(1 + |theta|) with theta = b/a:
    // 0 unless a and b share a sign, then 2ab/(a + b)
    const T ab = a * b;
    return ab > T(0) ? (ab + ab) / (a + b) : T(0);
  } else {
    const T ta = a + a, tb = b + b, m = (a + b) * T(0.5);
    const T lo = fmin(fmin(ta, tb), m);
    const T hi = fmax(fmax(ta, tb), m);
    return fmax(lo, T(0)) + fmin(hi, T(0));
  }
}

// Strengths at an edge from the jumps of (p, normal velocity).
template <typename T>
__device__ inline T s1(T Z, T dp, T dn) { return fma(Z, dn, -dp); }
template <typename T>
__device__ inline T s2(T Z, T dp, T dn) { return fma(Z, dn, dp); }

// F~ at an x-edge from the limited strengths of its two waves (l1 of wave -c,
// l2 of wave +c): the normal correction plus the transverse waves A-+ split
// from the y-terms of the cells left and right.
template <typename T>
__device__ inline void ftilde_l(const Coef<T> &k, T l1, T l2, T ys_left, T ys_right, T &Fp,
                                T &Fu) {
  const T Fcp = k.fx * (l2 - l1), Fcu = k.fxz * (l1 + l2);
  Fp = Fcp - k.gy * (ys_left - ys_right);
  Fu = Fcu - k.gyz * (ys_right + ys_left);
}

// G~ at a y-edge, the mirror image: transverse waves B-+ split from the
// x-terms of the cells below (lo) and above (hi).
template <typename T>
__device__ inline void gtilde_l(const Coef<T> &k, T l1, T l2, T xs_lo, T xs_hi, T &Gp, T &Gv) {
  const T Gcp = k.fy * (l2 - l1), Gcv = k.fyz * (l1 + l2);
  Gp = Gcp - k.gx * (xs_lo - xs_hi);
  Gv = Gcv - k.gxz * (xs_hi + xs_lo);
}

// F~ from the raw strengths (wave -c takes its upwind neighbour on the right,
// wave +c on the left) and the y-fluctuations of the cells left and right.
template <typename T, int LIM>
__device__ inline void ftilde(const Coef<T> &k, T a1, T a2, T a1_right, T a2_left, T ys_left,
                              T ys_right, T &Fp, T &Fu) {
  ftilde_l<T>(k, limited<T, LIM>(a1, a1_right), limited<T, LIM>(a2, a2_left), ys_left, ys_right,
              Fp, Fu);
}

// G~ from the raw strengths and the x-fluctuations of the cells below and above.
template <typename T, int LIM>
__device__ inline void gtilde(const Coef<T> &k, T b1, T b2, T b1_up, T b2_down, T xs_lo, T xs_hi,
                              T &Gp, T &Gv) {
  gtilde_l<T>(k, limited<T, LIM>(b1, b1_up), limited<T, LIM>(b2, b2_down), xs_lo, xs_hi, Gp, Gv);
}

}  // namespace ws
