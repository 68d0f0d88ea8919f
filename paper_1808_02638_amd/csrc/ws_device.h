// Device helpers shared by the forward and adjoint kernels of the
// wave-propagation library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

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

}  // namespace ws
