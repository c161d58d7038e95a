// gfx950 kernels of the Hartree potential by atom-centred multipole expansion of the
// partitioned density:
//   multipole_kernel  rho_{a,lm}(r_k) = sum_{points on node k of atom a} w n Y_lm(u) / W_k, one
//                     wavefront per (atom, radial node), the node's points pre-sorted on the host
//   radial_kernel     one thread per (atom, lm): natural cubic spline of rho in Becke's angle,
//                     kGauss-point Gauss-Legendre per interval (nodes and weights from the host)
//                     for the two radial Poisson integrals,
//                     V_lm at the nodes and its own natural spline, and the moment q_lm
//   potential_kernel  one thread per point: v_H = sum_atoms sum_lm V_lm(r) Y_lm(u) (the V spline
//                     as per-interval cubic coefficients, one 32-byte load per term), the
//                     exterior form 4 pi q_lm / ((2l+1) r^(l+1)) beyond the atom's support (no
//                     spline, no table), (r/r_min)^l inside the innermost node
// An atom's density piece lives on its own points, which end at a finite radius (the partition
// weights vanish beyond it): rho_lm is splined from the innermost node out to the atom's edge
// node (one node outwards of its outermost occupied node) and is zero beyond, so beyond the edge
// radius V_lm is exactly the exterior form.
// Real orthonormal Y_lm without the Condon-Shortley phase, from the associated-Legendre
// recurrence in z and the powers (x + i y)^m, generated m-outer / l-inner and consumed as they
// are produced.
#include <hip/hip_runtime.h>

#include "aims_internal.h"
#include "hartree.h"
#include "kernels.h"

namespace aims {

namespace {

constexpr double kPi = 3.14159265358979323846;

// visit(l, m, Y_lm) for l <= L, every m, at the unit vector (x, y, z)
template <int L, typename F>
__device__ __forceinline__ void for_each_ylm(double x, double y, double z, F&& visit) {
  double cm = 1.0, sm = 0.0;            // Re, Im of (x + i y)^m
  double qmm = 1.0;                     // d^m P_m / dz^m = (2m - 1)!!
#pragma unroll
  for (int m = 0; m <= L; ++m) {
    if (m > 0) {
      const double c = cm * x - sm * y, s = cm * y + sm * x;
      cm = c;
      sm = s;
      qmm *= (double)(2 * m - 1);
    }
    // Q_l^m = d^m P_l / dz^m by the recurrence in l; N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
    double q2 = 0.0, q1 = qmm;          // Q_{l-2}, Q_{l-1} (start: l = m)
    double fr = 1.0;                    // (l-m)!/(l+m)! at l = m: 1/(2m)!
    for (int k = 1; k <= 2 * m; ++k) fr /= (double)k;
#pragma unroll
    for (int l = m; l <= L; ++l) {
      double q;
      if (l == m) {
        q = qmm;
      } else {
        // multiply by the (compile-time) reciprocal: an FP64 division is a long sequence
        q = ((double)(2 * l - 1) * z * q1 - (double)(l + m - 1) * q2) * (1.0 / (double)(l - m));
        q2 = q1;
        q1 = q;
        fr *= (double)(l - m) / (double)(l + m);
      }
      const double nrm = sqrt((double)(2 * l + 1) / (4.0 * kPi) * fr);
      if (m == 0) {
        visit(l, 0, nrm * q);
      } else {
        const double a = 1.4142135623730950488 * nrm * q;
        visit(l, m, a * cm);
        visit(l, -m, a * sm);
      }
    }
  }
}

template <int L>
__global__ void __launch_bounds__(256)
multipole_kernel(const HartreeShell* __restrict__ shells, int n_shells,
                 const int32_t* __restrict__ shell_pts, const double4* __restrict__ pts,
                 const int32_t* __restrict__ perm, const double* __restrict__ atom_xyz,
                 const double* __restrict__ n_in, double* __restrict__ rho) {
  constexpr int NLM = (L + 1) * (L + 1);
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (wave >= n_shells) return;                         // whole wavefront
  const HartreeShell sh = shells[wave];
  double acc[NLM];
#pragma unroll
  for (int c = 0; c < NLM; ++c) acc[c] = 0.0;
  const double ax = atom_xyz[3 * sh.atom], ay = atom_xyz[3 * sh.atom + 1], az = atom_xyz[3 * sh.atom + 2];
  for (int j = sh.p0 + lane; j < sh.p1; j += 64) {
    const int i = shell_pts[j];
    const double4 P4 = pts[i];
    const double dx = P4.x - ax, dy = P4.y - ay, dz = P4.z - az;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double ir = r > 0.0 ? 1.0 / r : 0.0;
    const double wn = P4.w * n_in[perm[i]];
    for_each_ylm<L>(dx * ir, dy * ir, r > 0.0 ? dz * ir : 1.0,
                    [&](int l, int m, double Y) { acc[l * l + l + m] += wn * Y; });
  }
#pragma unroll
  for (int c = 0; c < NLM; ++c) {
    double v = acc[c];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) rho[(size_t)sh.out * NLM + c] = v * sh.inv_w;
  }
}

// natural cubic spline value on uniform knots t_k = t0 + k h, interval i, local b in [0, 1]
__device__ __forceinline__ double spline_at(const double* y, const double* M, size_t stride, int i,
                                            double b, double h) {
  const double a = 1.0 - b;
  return a * y[i * stride] + b * y[(i + 1) * stride] +
         ((a * a * a - a) * M[i * stride] + (b * b * b - b) * M[(i + 1) * stride]) * (h * h / 6.0);
}

// second derivatives of the natural spline through y (stride `stride`), Thomas algorithm with
// the host's factors of the constant system M_{i-1} + 4 M_i + M_{i+1} = rhs_i: cp[i] (the
// modified super-diagonal) and den[i] (the pivot), i = 1..K-2
__device__ __forceinline__ void natural_spline(const double* y, double* M, size_t stride, int K,
                                               double h, const double* cp, const double* den) {
  M[0] = 0.0;
  M[(K - 1) * stride] = 0.0;
  if (K < 3) return;
  const double f = 6.0 / (h * h);
  // forward sweep: M holds d'_i
  double dprev = 0.0;
  for (int i = 1; i <= K - 2; ++i) {
    const double rhs = f * (y[(i + 1) * stride] - 2.0 * y[i * stride] + y[(i - 1) * stride]);
    const double d = (rhs - dprev) / den[i];
    M[i * stride] = d;
    dprev = d;
  }
  for (int i = K - 3; i >= 1; --i) M[i * stride] -= cp[i] * M[(i + 1) * stride];
}

// one thread per (atom, lm) of the handle: rho, M_rho (scratch), V, M_V laid out
// [atom][k][lm]; q [atom][lm]
template <int L>
__global__ void __launch_bounds__(256)
radial_kernel(int n_atoms, const int32_t* __restrict__ atom_sys, const HartreeSys* __restrict__ hs,
              const int32_t* __restrict__ edge, const double* __restrict__ cp,
              const double* __restrict__ den, const double* __restrict__ gl,
              const double* __restrict__ rho, double* __restrict__ Mr, double* __restrict__ V,
              double* __restrict__ MV, double* __restrict__ q, double4* __restrict__ Vc) {
  constexpr int NLM = (L + 1) * (L + 1);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_atoms * NLM) return;
  const int a = t / NLM, c = t - a * NLM;
  int l = 0;
  while ((l + 1) * (l + 1) <= c) ++l;
  const HartreeSys S = hs[atom_sys[a]];
  const int K = S.K, e = edge[a];            // nodes e..K-1 carry the spline (e <= K - 2)
  const double h = kPi / (double)(K + 1), rm = S.r_map;
  // node arrays of this atom: element (k, lm) at (a K_max + k) NLM + lm
  const double* y = rho + (size_t)a * S.K_max * NLM + c;
  double* My = Mr + (size_t)a * S.K_max * NLM + c;
  double* Vy = V + (size_t)a * S.K_max * NLM + c;
  double* MVy = MV + (size_t)a * S.K_max * NLM + c;
  // the Thomas factors of row i do not depend on the system size, so the spline over the
  // K - e nodes from e on uses the same cp / den
  natural_spline(y + (size_t)e * NLM, My + (size_t)e * NLM, NLM, K - e, h, cp + S.fac_off,
                 den + S.fac_off);
  // Poisson integrals per interval [theta_k, theta_k+1] (r from r_k+1 up to r_k): inner
  // (s^(l+2)) accumulated from the centre outwards, outer (s^(1-l)) from infinity inwards
  const double rmin = rm / (tan(0.5 * h * K) * tan(0.5 * h * K));
  double inner = y[(size_t)(K - 1) * NLM] * pow(rmin, l + 3) / (double)(2 * l + 3);
  // pass 1: inner integral at each node, stored in Vy temporarily
  Vy[(size_t)(K - 1) * NLM] = inner;
  for (int k = K - 2; k >= e; --k) {
    double A = 0.0;
    for (int g = 0; g < kGauss; ++g) {
      const double b = 0.5 + 0.5 * gl[g];
      const double tg = h * (double)(k + 1) + b * h;
      const double ct = 1.0 / tan(0.5 * tg), st = sin(0.5 * tg);
      const double s = rm * ct * ct, J = rm * ct / (st * st);
      A += gl[kGauss + g] * spline_at(y, My, NLM, k, b, h) * pow(s, l + 2) * J;
    }
    inner += 0.5 * h * A;
    Vy[(size_t)k * NLM] = inner;
  }
  q[(size_t)a * NLM + c] = inner;
  // pass 2: outer integral from the edge inwards and V at the nodes; outside the edge node V is
  // the exterior form
  double outer = 0.0;
  const double pref = 4.0 * kPi / (double)(2 * l + 1);
  for (int k = 0; k < e; ++k) {
    const double tk = h * (double)(k + 1);
    const double ctk = 1.0 / tan(0.5 * tk);
    Vy[(size_t)k * NLM] = pref * inner * pow(rm * ctk * ctk, -(l + 1));
  }
  for (int k = e; k < K; ++k) {
    if (k > e) {
      double B = 0.0;
      for (int g = 0; g < kGauss; ++g) {
        const double b = 0.5 + 0.5 * gl[g];
        const double tg = h * (double)k + b * h;
        const double ct = 1.0 / tan(0.5 * tg), st = sin(0.5 * tg);
        const double s = rm * ct * ct, J = rm * ct / (st * st);
        B += gl[kGauss + g] * spline_at(y, My, NLM, k - 1, b, h) * pow(s, 1 - l) * J;
      }
      outer += 0.5 * h * B;
    }
    const double tk = h * (double)(k + 1);
    const double ctk = 1.0 / tan(0.5 * tk);
    const double rk = rm * ctk * ctk;
    Vy[(size_t)k * NLM] = pref * (Vy[(size_t)k * NLM] * pow(rk, -(l + 1)) + outer * pow(rk, l));
  }
  natural_spline(Vy + (size_t)e * NLM, MVy + (size_t)e * NLM, NLM, K - e, h, cp + S.fac_off,
                 den + S.fac_off);
  // the same spline per interval as c0 + c1 b + c2 b^2 + c3 b^3 in the local b in [0, 1]:
  // a y_k + b y_k+1 + ((a^3 - a) M_k + (b^3 - b) M_k+1) h^2/6 with a = 1 - b, expanded
  double4* C = Vc + (size_t)a * S.K_max * NLM + c;
  const double h26 = h * h / 6.0;
  for (int k = e; k + 1 < K; ++k) {
    const double y0 = Vy[(size_t)k * NLM], y1 = Vy[(size_t)(k + 1) * NLM];
    const double m0 = MVy[(size_t)k * NLM], m1 = MVy[(size_t)(k + 1) * NLM];
    C[(size_t)k * NLM] = double4{y0, y1 - y0 - h26 * (2.0 * m0 + m1), 3.0 * h26 * m0, h26 * (m1 - m0)};
  }
}

template <int L>
__global__ void __launch_bounds__(256)
potential_kernel(const double4* __restrict__ pts, const int32_t* __restrict__ perm,
                 const int64_t* __restrict__ sys_pt_range, const SystemDesc* __restrict__ systems,
                 const int32_t* __restrict__ sys_natoms, const double* __restrict__ atom_xyz,
                 const HartreeSys* __restrict__ hs, const int32_t* __restrict__ edge,
                 const double* __restrict__ r_edge, const double* __restrict__ V,
                 const double4* __restrict__ Vc, const double* __restrict__ q,
                 const double* __restrict__ n_in, double* __restrict__ v_out,
                 double* __restrict__ part) {
  constexpr int NLM = (L + 1) * (L + 1);
  __shared__ double sh[4];
  const int s = blockIdx.y, nblk = gridDim.x;
  const int64_t p0 = sys_pt_range[2 * s], p1 = sys_pt_range[2 * s + 1];
  const int a0 = systems[s].atom_off, na = sys_natoms[s];
  const HartreeSys S = hs[s];
  const int K = S.K;
  const double h = kPi / (double)(K + 1), rm = S.r_map;
  const double ctK = 1.0 / tan(0.5 * h * K), rmin = rm * ctK * ctK;
  double se = 0.0;
  for (int64_t i = p0 + blockIdx.x * 256 + threadIdx.x; i < p1; i += (int64_t)nblk * 256) {
    const double4 P4 = pts[i];
    double v = 0.0;
    for (int a = a0; a < a0 + na; ++a) {
      const double dx = P4.x - atom_xyz[3 * a], dy = P4.y - atom_xyz[3 * a + 1],
                   dz = P4.z - atom_xyz[3 * a + 2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      const double ir = r > 0.0 ? 1.0 / r : 0.0;
      const double* Va = V + (size_t)a * S.K_max * NLM;
      double pw[L + 1];                     // running powers, indexed by the unrolled l
      if (r >= r_edge[a]) {                 // beyond the support: 4 pi q / ((2l+1) r^(l+1))
        const double* qa = q + (size_t)a * NLM;
        pw[0] = ir;
#pragma unroll
        for (int l = 1; l <= L; ++l) pw[l] = pw[l - 1] * ir;
        double sl[L + 1];                   // sum over m of q_lm Y_lm: one chain per l
#pragma unroll
        for (int l = 0; l <= L; ++l) sl[l] = 0.0;
        for_each_ylm<L>(dx * ir, dy * ir, dz * ir, [&](int l, int m, double Y) {
          sl[l] = fma(qa[l * l + l + m], Y, sl[l]);
        });
#pragma unroll
        for (int l = 0; l <= L; ++l) v = fma((4.0 * kPi / (double)(2 * l + 1)) * pw[l], sl[l], v);
      } else if (r < rmin) {                // inside the innermost node
        const double x = r / rmin;
        pw[0] = 1.0;
#pragma unroll
        for (int l = 1; l <= L; ++l) pw[l] = pw[l - 1] * x;
        for_each_ylm<L>(dx * ir, dy * ir, r > 0.0 ? dz * ir : 1.0, [&](int l, int m, double Y) {
          v += Va[(size_t)(K - 1) * NLM + l * l + l + m] * pw[l] * Y;
        });
      } else {
        const double t = 2.0 * atan(sqrt(rm / r));
        const int e = edge[a];
        int k = (int)floor(t / h) - 1;      // interval [theta_k, theta_k+1], theta_k = (k+1) h
        k = k < e ? e : (k > K - 2 ? K - 2 : k);
        const double b = (t - h * (double)(k + 1)) / h;
        const double4* Ck = Vc + ((size_t)a * S.K_max + k) * NLM;
        for_each_ylm<L>(dx * ir, dy * ir, dz * ir, [&](int l, int m, double Y) {
          const double4 cf = Ck[l * l + l + m];
          v += (((cf.w * b + cf.z) * b + cf.y) * b + cf.x) * Y;
        });
      }
    }
    const int qi = perm[i];
    v_out[qi] = v;
    se += P4.w * n_in[qi] * v;
  }
  for (int off = 32; off > 0; off >>= 1) se += __shfl_xor(se, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = se;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)s * nblk + blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ void __launch_bounds__(256) energy_kernel(const double* __restrict__ part, int nblk,
                                                     double* __restrict__ E) {
  __shared__ double sh[4];
  const int s = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) v += part[(size_t)s * nblk + b];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) E[s] = 0.5 * (((sh[0] + sh[1]) + sh[2]) + sh[3]);
}

template <int L>
hipError_t launch_all(const DeviceView& dv, const HartreeDev& hd, const double* n, double* v_out,
                      double* E_or_null, hipStream_t st) {
  constexpr int NLM = (L + 1) * (L + 1);
  if (hd.n_shells > 0) {
    hipLaunchKernelGGL(multipole_kernel<L>, dim3((hd.n_shells + 3) / 4), dim3(256), 0, st, hd.shells,
                       hd.n_shells, hd.shell_pts, dv.pts, dv.perm, dv.atom_xyz, n, hd.rho);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int nt = hd.n_atoms * NLM;
  hipLaunchKernelGGL(radial_kernel<L>, dim3((nt + 255) / 256), dim3(256), 0, st, hd.n_atoms,
                     dv.atom_sys, hd.sys, hd.edge, hd.cp, hd.den, hd.gl, hd.rho, hd.Mr, hd.V, hd.MV,
                     hd.q, hd.Vc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(potential_kernel<L>, dim3(kHartreeBlocks, dv.n_sys), dim3(256), 0, st, dv.pts,
                     dv.perm, dv.sys_pt_range, dv.systems, hd.sys_natoms, dv.atom_xyz, hd.sys,
                     hd.edge, hd.r_edge, hd.V, hd.Vc, hd.q, n, v_out, hd.part);
  e = hipGetLastError();
  if (e != hipSuccess || !E_or_null) return e;
  hipLaunchKernelGGL(energy_kernel, dim3(dv.n_sys), dim3(256), 0, st, hd.part, kHartreeBlocks,
                     E_or_null);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_hartree(const DeviceView& dv, const HartreeDev& hd, const double* n,
                          double* v_out, double* E_or_null, hipStream_t st) {
  switch (hd.l_max) {
    case 0: return launch_all<0>(dv, hd, n, v_out, E_or_null, st);
    case 1: return launch_all<1>(dv, hd, n, v_out, E_or_null, st);
    case 2: return launch_all<2>(dv, hd, n, v_out, E_or_null, st);
    case 3: return launch_all<3>(dv, hd, n, v_out, E_or_null, st);
    case 4: return launch_all<4>(dv, hd, n, v_out, E_or_null, st);
    case 5: return launch_all<5>(dv, hd, n, v_out, E_or_null, st);
    case 6: return launch_all<6>(dv, hd, n, v_out, E_or_null, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace aims
