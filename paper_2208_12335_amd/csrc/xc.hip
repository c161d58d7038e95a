// gfx950 kernels of the exchange-correlation step on the grid (spin-unpolarised LDA: Slater
// exchange + Perdew-Wang 1992 correlation; PBE), the density gradient and the gradient term of
// the H integrand.  One thread per point, batch order, with the
// caller-order density and potential reached through the point permutation; per-system sums
// by fixed-order block partials.
#include <hip/hip_runtime.h>

#include "aims_internal.h"
#include "basis.h"
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

// ---- PBE (spin-unpolarised) by forward-mode differentiation -------------------------------
// A value with its partial derivatives with respect to n and sigma = |grad n|^2: evaluating the
// energy density once in this type gives f, df/dn and df/dsigma of the very same expression.
struct Dual2 {
  double v, dn, ds;
};
__device__ __forceinline__ Dual2 operator+(Dual2 a, Dual2 b) { return {a.v + b.v, a.dn + b.dn, a.ds + b.ds}; }
__device__ __forceinline__ Dual2 operator*(Dual2 a, Dual2 b) {
  return {a.v * b.v, a.dn * b.v + a.v * b.dn, a.ds * b.v + a.v * b.ds};
}
__device__ __forceinline__ Dual2 operator/(Dual2 a, Dual2 b) {
  const double q = a.v / b.v, ib = 1.0 / b.v;
  return {q, (a.dn - q * b.dn) * ib, (a.ds - q * b.ds) * ib};
}
__device__ __forceinline__ Dual2 operator+(double c, Dual2 a) { return {c + a.v, a.dn, a.ds}; }
__device__ __forceinline__ Dual2 operator-(double c, Dual2 a) { return {c - a.v, -a.dn, -a.ds}; }
__device__ __forceinline__ Dual2 operator*(double c, Dual2 a) { return {c * a.v, c * a.dn, c * a.ds}; }
__device__ __forceinline__ Dual2 operator/(double c, Dual2 a) {
  const double q = c / a.v;
  return {q, -q / a.v * a.dn, -q / a.v * a.ds};
}
__device__ __forceinline__ Dual2 chain(double f, double df, Dual2 a) { return {f, df * a.dn, df * a.ds}; }
__device__ __forceinline__ Dual2 d_sqrt(Dual2 a) { const double r = sqrt(a.v); return chain(r, 0.5 / r, a); }
__device__ __forceinline__ Dual2 d_cbrt(Dual2 a) { const double r = cbrt(a.v); return chain(r, r / (3.0 * a.v), a); }
__device__ __forceinline__ Dual2 d_log1p(Dual2 a) { return chain(log1p(a.v), 1.0 / (1.0 + a.v), a); }
__device__ __forceinline__ Dual2 d_expm1(Dual2 a) { const double e = expm1(a.v); return chain(e, e + 1.0, a); }

constexpr double kKappa = 0.804, kBeta = 0.06672455060314922;

// f(n, sigma) = n eps_x F_x(s) + n (eps_c + H(rs, t)) of PBE with PW92 correlation
__device__ __forceinline__ Dual2 pbe_f(Dual2 n, Dual2 sigma) {
  const double mu = kBeta * kPi * kPi / 3.0;
  const double gamma = (1.0 - 0.69314718055994530942) / (kPi * kPi);
  const Dual2 n13 = d_cbrt(n);
  const Dual2 ex = (-0.75 * cbrt(3.0 / kPi)) * n13;
  const Dual2 rs = cbrt(3.0 / (4.0 * kPi)) / n13;
  const Dual2 srs = d_sqrt(rs);
  const Dual2 Q = (2.0 * kA) * (kB1 * srs + kB2 * rs + kB3 * (rs * srs) + kB4 * (rs * rs));
  const Dual2 ec = (-2.0 * kA) * ((1.0 + kA1 * rs) * d_log1p(1.0 / Q));
  const Dual2 kF = cbrt(3.0 * kPi * kPi) * n13;
  const Dual2 n2 = n * n;
  const Dual2 s2 = sigma / (4.0 * (kF * kF * n2));
  const Dual2 Fx = (1.0 + kKappa) - kKappa / (1.0 + (mu / kKappa) * s2);
  const Dual2 t2 = sigma / (4.0 * ((4.0 / kPi) * kF * n2));
  const Dual2 A = (kBeta / gamma) / d_expm1((-1.0 / gamma) * ec);
  const Dual2 At2 = A * t2;
  const Dual2 H = gamma * d_log1p((kBeta / gamma) * (t2 * (1.0 + At2) / (1.0 + At2 + At2 * At2)));
  return n * ex * Fx + n * (ec + H);
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

// PBE per point (batch order, caller-order arrays through perm): v_out = df/dn, u_out =
// 4 df/dsigma grad n (the vector field of the raw GGA H), block partials of
// (E_xc = sum w f, sum w (n v_n + 2 sigma v_sigma))
__global__ void __launch_bounds__(256) pbe_kernel(const double4* __restrict__ pts,
                                                  const int32_t* __restrict__ perm,
                                                  const int64_t* __restrict__ sys_pt_range,
                                                  const double* __restrict__ n_in,
                                                  const double* __restrict__ grad_in,
                                                  double* __restrict__ v_out,
                                                  double* __restrict__ u_out,
                                                  double* __restrict__ part) {
  __shared__ double sh[4];
  const int s = blockIdx.y, nblk = gridDim.x;
  const int64_t p0 = sys_pt_range[2 * s], p1 = sys_pt_range[2 * s + 1];
  double se = 0.0, sv = 0.0;
  for (int64_t i = p0 + blockIdx.x * 256 + threadIdx.x; i < p1; i += (int64_t)nblk * 256) {
    const size_t q = (size_t)perm[i];
    const double n = n_in[q], w = pts[i].w;
    const double gx = grad_in[3 * q], gy = grad_in[3 * q + 1], gz = grad_in[3 * q + 2];
    double vn = 0.0, vs = 0.0, f = 0.0;
    const double sigma = gx * gx + gy * gy + gz * gz;
    if (n > kNMin) {
      const Dual2 r = pbe_f(Dual2{n, 1.0, 0.0}, Dual2{sigma, 0.0, 1.0});
      f = r.v;
      vn = r.dn;
      vs = r.ds;
    }
    v_out[q] = vn;
    u_out[3 * q] = 4.0 * vs * gx;
    u_out[3 * q + 1] = 4.0 * vs * gy;
    u_out[3 * q + 2] = 4.0 * vs * gz;
    se += w * f;
    sv += w * (n * vn + 2.0 * sigma * vs);
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

// Gradients of the 2L+1 functions of one shell at a point (u = (p - R_a)/r, ir = 1/r):
//   grad phi = (R' - L R / r) Y_lm u + (R / r) grad S_lm(u)
// handed to f(m, gx, gy, gz).
template <int L, typename F>
__device__ __forceinline__ void shell_grad(const double* __restrict__ c, double dt, double ir,
                                           double ux, double uy, double uz, F&& f) {
  const double R = cubic(c, dt), dR = cubic_d(c, dt) * ir;
  double Yl[7], Gx[7], Gy[7], Gz[7];
  ylm_l<double>(L, ux, uy, uz, Yl);
  ylm_grad_l<double>(L, ux, uy, uz, Gx, Gy, Gz);
  const double aR = dR - double(L) * R * ir, bR = R * ir;
#pragma unroll
  for (int m = 0; m < 2 * L + 1; ++m) {
    const double a = aR * Yl[m];
    f(m, a * ux + bR * Gx[m], a * uy + bR * Gy[m], a * uz + bR * Gz[m]);
  }
}

// f(column of the function within the batch, grad phi) for every function of the batch's atom k
// at point P4 (nothing beyond the cutoff)
template <typename F>
__device__ __forceinline__ void atom_grads(const BatchDesc& d, int k, double4 P4,
                                           const int32_t* __restrict__ batch_atoms,
                                           const int32_t* __restrict__ batch_acol,
                                           const double* __restrict__ atom_xyz,
                                           const int32_t* __restrict__ atom_species,
                                           const SpeciesDesc* __restrict__ species,
                                           const int32_t* __restrict__ shell_l,
                                           const double* __restrict__ spline, const RadialGrid& rg,
                                           F&& f) {
  const int atom = batch_atoms[d.atom_off + k];
  const int col0 = batch_acol[d.atom_off + k];
  const SpeciesDesc sd = species[atom_species[atom]];
  const double dx = P4.x - atom_xyz[3 * atom], dy = P4.y - atom_xyz[3 * atom + 1],
               dz = P4.z - atom_xyz[3 * atom + 2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  if (!(r < rg.rc)) return;
  const double rr = fmax(r, 1e-12), ir = 1.0 / rr;
  const double ux = dx * ir, uy = dy * ir, uz = dz * ir;
  const RadialPos rp = radial_pos(rr, rg);
  const double* c = spline + sd.spline_off + (size_t)rp.k * sd.nshell * 8;
  int col = col0;
  for (int j = 0; j < sd.nshell; ++j) {
    const int l = shell_l[sd.shell_l_off + j];
    auto g = [&](int m, double gx, double gy, double gz) { f(col + m, gx, gy, gz); };
    switch (l) {
      case 0: shell_grad<0>(c + j * 8, rp.dt, ir, ux, uy, uz, g); break;
      case 1: shell_grad<1>(c + j * 8, rp.dt, ir, ux, uy, uz, g); break;
      case 2: shell_grad<2>(c + j * 8, rp.dt, ir, ux, uy, uz, g); break;
      default: shell_grad<3>(c + j * 8, rp.dt, ir, ux, uy, uz, g); break;
    }
    col += 2 * l + 1;
  }
}

// grad n(p) = 2 sum_j X_pj grad phi_j(p) with X^T = P_b Phi^T in the function-major slab Xs
// (P symmetric).  One workgroup per batch, one thread per point, the batch's atoms in a loop:
// every point's sum stays in registers and is written once, in caller order.
__global__ void __launch_bounds__(256)
gradn_kernel(const BatchDesc* __restrict__ batches, int b0, const double4* __restrict__ pts,
             const int32_t* __restrict__ perm, const int32_t* __restrict__ batch_atoms,
             const int32_t* __restrict__ batch_acol, const double* __restrict__ atom_xyz,
             const int32_t* __restrict__ atom_species, const SpeciesDesc* __restrict__ species,
             const int32_t* __restrict__ shell_l, const double* __restrict__ spline, RadialGrid rg,
             const double* __restrict__ Xs, double* __restrict__ grad_out) {
  const BatchDesc d = batches[b0 + blockIdx.x];
  const double* X = Xs + d.slab_off;
  for (int p = threadIdx.x; p < d.n_p; p += blockDim.x) {
    const double4 P4 = pts[d.pt_off + p];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int k = 0; k < d.n_atoms; ++k)
      atom_grads(d, k, P4, batch_atoms, batch_acol, atom_xyz, atom_species, species, shell_l,
                 spline, rg, [&](int col, double ax, double ay, double az) {
                   const double xv = X[(size_t)col * d.ldp + p];
                   gx += xv * ax;
                   gy += xv * ay;
                   gz += xv * az;
                 });
    const size_t q = (size_t)perm[d.pt_off + p];
    grad_out[3 * q] = 2.0 * gx;
    grad_out[3 * q + 1] = 2.0 * gy;
    grad_out[3 * q + 2] = 2.0 * gz;
  }
}

// The gradient term of the H integrand: slab2[col][p] += w_p u_p . grad phi_col(p) on top of
// the basis evaluation's w (v phi + t phi), for the batches [b0, b0 + nbatch); u in caller
// order.  One workgroup per batch, one thread per point; each slab entry has one writer.
template <typename T>
__global__ void __launch_bounds__(256)
vector_term_kernel(const BatchDesc* __restrict__ batches, int b0, const double4* __restrict__ pts,
                   const int32_t* __restrict__ perm, const int32_t* __restrict__ batch_atoms,
                   const int32_t* __restrict__ batch_acol, const double* __restrict__ atom_xyz,
                   const int32_t* __restrict__ atom_species, const SpeciesDesc* __restrict__ species,
                   const int32_t* __restrict__ shell_l, const double* __restrict__ spline,
                   RadialGrid rg, const double* __restrict__ u, T* __restrict__ slab2) {
  const BatchDesc d = batches[b0 + blockIdx.x];
  T* S2 = slab2 + d.slab_off;
  for (int p = threadIdx.x; p < d.n_p; p += blockDim.x) {
    const double4 P4 = pts[d.pt_off + p];
    const size_t q = (size_t)perm[d.pt_off + p];
    const double wx = P4.w * u[3 * q], wy = P4.w * u[3 * q + 1], wz = P4.w * u[3 * q + 2];
    for (int k = 0; k < d.n_atoms; ++k)
      atom_grads(d, k, P4, batch_atoms, batch_acol, atom_xyz, atom_species, species, shell_l,
                 spline, rg, [&](int col, double ax, double ay, double az) {
                   T& e = S2[(size_t)col * d.ldp + p];
                   e = T((double)e + (wx * ax + wy * ay + wz * az));
                 });
  }
}

}  // namespace

template <typename T>
hipError_t launch_vector_term(const DeviceView& dv, int b0, int nbatch, const double* u, T* slab2,
                              hipStream_t st) {
  if (nbatch <= 0) return hipSuccess;
  hipLaunchKernelGGL(vector_term_kernel<T>, dim3(nbatch), dim3(256), 0, st, dv.batches, b0, dv.pts,
                     dv.perm, dv.batch_atoms, dv.batch_acol, dv.atom_xyz, dv.atom_species,
                     dv.species, dv.shell_l, dv.spline64, dv.rg, u, slab2);
  return hipGetLastError();
}
template hipError_t launch_vector_term<double>(const DeviceView&, int, int, const double*, double*,
                                               hipStream_t);
template hipError_t launch_vector_term<float>(const DeviceView&, int, int, const double*, float*,
                                              hipStream_t);

hipError_t launch_gradn(const DeviceView& dv, int b0, int nbatch, const double* X, double* grad_out,
                        hipStream_t st) {
  if (nbatch <= 0) return hipSuccess;
  hipLaunchKernelGGL(gradn_kernel, dim3(nbatch), dim3(256), 0, st, dv.batches, b0, dv.pts, dv.perm,
                     dv.batch_atoms, dv.batch_acol, dv.atom_xyz, dv.atom_species, dv.species,
                     dv.shell_l, dv.spline64, dv.rg, X, grad_out);
  return hipGetLastError();
}

hipError_t launch_pbe(const DeviceView& dv, const double* n, const double* grad, double* v_out,
                      double* u_out, double* part, double* sums_or_null, hipStream_t st) {
  hipLaunchKernelGGL(pbe_kernel, dim3(kXcBlocks, dv.n_sys), dim3(256), 0, st, dv.pts, dv.perm,
                     dv.sys_pt_range, n, grad, v_out, u_out, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !sums_or_null) return e;
  hipLaunchKernelGGL(xc_sums_kernel, dim3(dv.n_sys), dim3(256), 0, st, part, kXcBlocks,
                     sums_or_null);
  return hipGetLastError();
}

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
