// gfx950 kernels of the exchange-correlation step on the grid (spin-unpolarised LDA: Slater
// exchange + Perdew-Wang 1992 correlation).  One thread per point, batch order, with the
// caller-order density and potential reached through the point permutation; per-system sums
// by fixed-order block partials.
#include <hip/hip_runtime.h>

#include "aims_internal.h"
#include "kernels.h"
#include "xc.h"

namespace aims {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kNMin = 1e-14;          // densities at or below contribute nothing
// Perdew-Wang 1992, zeta = 0
constexpr double kA = 0.031091, kA1 = 0.21370, kB1 = 7.5957, kB2 = 3.5876, kB3 = 1.6382,
                 kB4 = 0.49294;

// eps_xc (energy per electron) and v_xc = d(n eps_xc)/dn at density n
__device__ __forceinline__ void lda_point(double n, double& eps, double& v) {
  if (!(n > kNMin)) {
    eps = 0.0;
    v = 0.0;
    return;
  }
  const double n13 = cbrt(n);
  // exchange: eps_x = -(3/4)(3/pi)^(1/3) n^(1/3), v_x = (4/3) eps_x
  const double ex = -0.75 * cbrt(3.0 / kPi) * n13;
  // correlation in rs = (3 / (4 pi n))^(1/3)
  const double rs = cbrt(3.0 / (4.0 * kPi)) / n13;
  const double srs = sqrt(rs);
  const double Q = 2.0 * kA * (kB1 * srs + kB2 * rs + kB3 * rs * srs + kB4 * rs * rs);
  const double dQ = 2.0 * kA * (0.5 * kB1 / srs + kB2 + 1.5 * kB3 * srs + 2.0 * kB4 * rs);
  const double L = log1p(1.0 / Q);
  const double ec = -2.0 * kA * (1.0 + kA1 * rs) * L;
  const double dec = -2.0 * kA * kA1 * L + 2.0 * kA * (1.0 + kA1 * rs) * dQ / (Q * Q + Q);
  eps = ex + ec;
  v = (4.0 / 3.0) * ex + ec - (rs / 3.0) * dec;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NT / 64; ++w) s += sh[w];
  return s;
}

// grid (nblk, n_sys): block b of system s takes points p0 + b*256 + k*nblk*256 of that system
__global__ void __launch_bounds__(256) lda_kernel(const double4* __restrict__ pts,
                                                  const int32_t* __restrict__ perm,
                                                  const int64_t* __restrict__ sys_pt_range,
                                                  const double* __restrict__ n_in,
                                                  double* __restrict__ v_out,
                                                  double* __restrict__ part) {
  __shared__ double sh[4];
  const int s = blockIdx.y, nblk = gridDim.x;
  const int64_t p0 = sys_pt_range[2 * s], p1 = sys_pt_range[2 * s + 1];
  double se = 0.0, sv = 0.0;
  for (int64_t i = p0 + blockIdx.x * 256 + threadIdx.x; i < p1; i += (int64_t)nblk * 256) {
    const int q = perm[i];
    const double n = n_in[q], w = pts[i].w;
    double eps, v;
    lda_point(n, eps, v);
    v_out[q] = v;
    se += w * n * eps;
    sv += w * n * v;
  }
  se = block_sum<256>(se, sh);
  sv = block_sum<256>(sv, sh);
  if (threadIdx.x == 0) {
    part[2 * ((size_t)s * nblk + blockIdx.x)] = se;
    part[2 * ((size_t)s * nblk + blockIdx.x) + 1] = sv;
  }
}

__global__ void __launch_bounds__(256) xc_sums_kernel(const double* __restrict__ part, int nblk,
                                                      double* __restrict__ sums) {
  __shared__ double sh[4];
  const int s = blockIdx.x;
  double se = 0.0, sv = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) {
    se += part[2 * ((size_t)s * nblk + b)];
    sv += part[2 * ((size_t)s * nblk + b) + 1];
  }
  se = block_sum<256>(se, sh);
  sv = block_sum<256>(sv, sh);
  if (threadIdx.x == 0) {
    sums[2 * s] = se;
    sums[2 * s + 1] = sv;
  }
}

}  // namespace

hipError_t launch_lda(const DeviceView& dv, const double* n, double* v_out, double* part,
                      double* sums_or_null, hipStream_t st) {
  hipLaunchKernelGGL(lda_kernel, dim3(kXcBlocks, dv.n_sys), dim3(256), 0, st, dv.pts, dv.perm,
                     dv.sys_pt_range, n, v_out, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !sums_or_null) return e;
  hipLaunchKernelGGL(xc_sums_kernel, dim3(dv.n_sys), dim3(256), 0, st, part, kXcBlocks,
                     sums_or_null);
  return hipGetLastError();
}

}  // namespace aims
