// Device-side evaluation of the numeric atom-centred basis: cubic-spline radial functions in
// s = ln r times real spherical harmonics (l <= 3), with their kinetic terms and gradients.
#pragma once

#include <hip/hip_runtime.h>

#include "aims_internal.h"

namespace aims {

// Real spherical harmonics, orthonormal on the sphere, no Condon-Shortley phase, m = -l..l.
// Each is written as a homogeneous polynomial S_lm(x, y, z) of degree l so that for a unit
// vector u, Y_lm(u) = S_lm(u); the gradients below are those of S_lm.
namespace ylm {
constexpr double c00 = 0.28209479177387814;  // sqrt(1/(4 pi))
constexpr double c1 = 0.4886025119029199;    // sqrt(3/(4 pi))
constexpr double c2a = 1.0925484305920792;   // sqrt(15/pi)/2
constexpr double c20 = 0.31539156525252005;  // sqrt(5/pi)/4
constexpr double c22 = 0.5462742152960396;   // sqrt(15/pi)/4
constexpr double c33 = 0.5900435899266435;   // sqrt(35/(2 pi))/4
constexpr double c32 = 2.890611442640554;    // sqrt(105/pi)/2
constexpr double c31 = 0.4570457994644658;   // sqrt(21/(2 pi))/4
constexpr double c30 = 0.3731763325901154;   // sqrt(7/pi)/4
constexpr double c32b = 1.445305721320277;   // sqrt(105/pi)/4
}  // namespace ylm

// Values of the 2l+1 harmonics of one l on the unit vector (x, y, z).
template <typename T>
__device__ __forceinline__ void ylm_l(int l, T x, T y, T z, T* Y) {
  using namespace ylm;
  if (l == 0) {
    Y[0] = T(c00);
  } else if (l == 1) {
    Y[0] = T(c1) * y; Y[1] = T(c1) * z; Y[2] = T(c1) * x;
  } else if (l == 2) {
    Y[0] = T(c2a) * x * y;
    Y[1] = T(c2a) * y * z;
    Y[2] = T(c20) * (T(2) * z * z - x * x - y * y);
    Y[3] = T(c2a) * x * z;
    Y[4] = T(c22) * (x * x - y * y);
  } else {
    const T x2 = x * x, y2 = y * y, z2 = z * z;
    Y[0] = T(c33) * y * (T(3) * x2 - y2);
    Y[1] = T(c32) * x * y * z;
    Y[2] = T(c31) * y * (T(4) * z2 - x2 - y2);
    Y[3] = T(c30) * z * (T(2) * z2 - T(3) * x2 - T(3) * y2);
    Y[4] = T(c31) * x * (T(4) * z2 - x2 - y2);
    Y[5] = T(c32b) * z * (x2 - y2);
    Y[6] = T(c33) * x * (x2 - T(3) * y2);
  }
}

// Gradients dS_lm/d(x, y, z) of the same homogeneous polynomials, at (x, y, z).
template <typename T>
__device__ __forceinline__ void ylm_grad_l(int l, T x, T y, T z, T* gx, T* gy, T* gz) {
  using namespace ylm;
  if (l == 0) {
    gx[0] = gy[0] = gz[0] = T(0);
  } else if (l == 1) {
    gx[0] = T(0);  gy[0] = T(c1); gz[0] = T(0);
    gx[1] = T(0);  gy[1] = T(0);  gz[1] = T(c1);
    gx[2] = T(c1); gy[2] = T(0);  gz[2] = T(0);
  } else if (l == 2) {
    gx[0] = T(c2a) * y;            gy[0] = T(c2a) * x;            gz[0] = T(0);
    gx[1] = T(0);                  gy[1] = T(c2a) * z;            gz[1] = T(c2a) * y;
    gx[2] = T(-2 * c20) * x;       gy[2] = T(-2 * c20) * y;       gz[2] = T(4 * c20) * z;
    gx[3] = T(c2a) * z;            gy[3] = T(0);                  gz[3] = T(c2a) * x;
    gx[4] = T(2 * c22) * x;        gy[4] = T(-2 * c22) * y;       gz[4] = T(0);
  } else {
    const T x2 = x * x, y2 = y * y, z2 = z * z;
    // y (3x^2 - y^2)
    gx[0] = T(c33) * T(6) * x * y;  gy[0] = T(c33) * (T(3) * x2 - T(3) * y2);  gz[0] = T(0);
    // x y z
    gx[1] = T(c32) * y * z;         gy[1] = T(c32) * x * z;  gz[1] = T(c32) * x * y;
    // y (4z^2 - x^2 - y^2)
    gx[2] = T(c31) * T(-2) * x * y;
    gy[2] = T(c31) * (T(4) * z2 - x2 - T(3) * y2);
    gz[2] = T(c31) * T(8) * y * z;
    // z (2z^2 - 3x^2 - 3y^2)
    gx[3] = T(c30) * T(-6) * x * z;
    gy[3] = T(c30) * T(-6) * y * z;
    gz[3] = T(c30) * (T(6) * z2 - T(3) * x2 - T(3) * y2);
    // x (4z^2 - x^2 - y^2)
    gx[4] = T(c31) * (T(4) * z2 - T(3) * x2 - y2);
    gy[4] = T(c31) * T(-2) * x * y;
    gz[4] = T(c31) * T(8) * x * z;
    // z (x^2 - y^2)
    gx[5] = T(c32b) * T(2) * x * z; gy[5] = T(c32b) * T(-2) * y * z; gz[5] = T(c32b) * (x2 - y2);
    // x (x^2 - 3y^2)
    gx[6] = T(c33) * (T(3) * x2 - T(3) * y2); gy[6] = T(c33) * T(-6) * x * y; gz[6] = T(0);
  }
}

// Position of r on the logarithmic knot grid: interval k and offset dt = ln r - s_k (FP64,
// so that the FP32 mode loses no accuracy in the geometry).
struct RadialPos {
  int k;
  double dt;
};

__device__ __forceinline__ RadialPos radial_pos(double r, const RadialGrid& rg) {
  const double s = log(r);
  double t = floor((s - rg.s0) * rg.inv_h);
  int k = (int)fmin(fmax(t, 0.0), (double)(rg.n_log - 2));
  RadialPos rp;
  rp.k = k;
  rp.dt = s - (rg.s0 + (double)k * rg.h);
  return rp;
}

// Cubic a + b dt + c dt^2 + d dt^3 and its derivative with respect to dt.
template <typename T>
__device__ __forceinline__ T cubic(const T* c, T dt) {
  return ((c[3] * dt + c[2]) * dt + c[1]) * dt + c[0];
}
template <typename T>
__device__ __forceinline__ T cubic_d(const T* c, T dt) {
  return (T(3) * c[3] * dt + T(2) * c[2]) * dt + c[1];
}

}  // namespace aims
