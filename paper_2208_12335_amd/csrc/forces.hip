// gfx950 kernels of the total (moving-grid) energy gradient: the nuclear model potential on
// the grid, and the point-motion, partition-weight and potential terms added to the Pulay
// gradient (the basis-function terms come from the backward kernels).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "aims_internal.h"
#include "kernels.h"

namespace aims {

static inline int grid_for(size_t n, int per) {
  size_t g = (n + per - 1) / per;
  if (g > 65536) g = 65536;
  return (int)(g ? g : 1);
}

// ------------------------------------------------------------------------------------------
// Moving-grid terms of the total energy gradient.  Every grid point p belongs to the
// atom-centred grid of an owner atom o and moves with it; its weight is
//   w_p = g_p S_o(p) / sum_b S_b(p),  S_b = prod_{c != b} s(mu_bc),
//   mu_bc = (|p - R_b| - |p - R_c|) / |R_b - R_c|,  s(mu) = (1 - z(mu / a)) / 2,
//   z(x) = (35 x - 35 x^3 + 21 x^5 - 5 x^7) / 16 on [-1, 1], sign(x) beyond
// (Stratmann, Scuseria and Frisch), and the potential is v(p) = sum_a -Z_a erf(r_a / sigma) / r_a.
// ------------------------------------------------------------------------------------------

// v at every point (batch order in, caller order out) for the nuclear model of its system.
__global__ void __launch_bounds__(256)
vext_kernel(const double4* __restrict__ pts, const int32_t* __restrict__ perm, int64_t n,
            const int32_t* __restrict__ pt_sys, const SystemDesc* __restrict__ systems,
            const int32_t* __restrict__ sys_natoms, const double* __restrict__ atom_xyz,
            const double* __restrict__ atom_Z, const double* __restrict__ sys_model,
            double* __restrict__ v_out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double4 P4 = pts[i];
    const int sy = pt_sys[i];
    const int a0 = systems[sy].atom_off, na = sys_natoms[sy];
    const double sigma = sys_model[2 * sy];
    double v = 0.0;
    for (int a = a0; a < a0 + na; ++a) {
      const double dx = P4.x - atom_xyz[3 * a], dy = P4.y - atom_xyz[3 * a + 1],
                   dz = P4.z - atom_xyz[3 * a + 2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      // r -> 0 limit 2 / (sigma sqrt(pi)); grid points never sit on a nucleus
      v -= atom_Z[a] * (r > 1e-12 ? erf(r / sigma) / r : 2.0 / (sigma * 1.7724538509055160273));
    }
    v_out[perm[i]] = v;
  }
}

// Switching function s(x) = (1 - z(x)) / 2 of the partition on (-1, 1), with
// z(x) = (35 x - 35 x^3 + 21 x^5 - 5 x^7) / 16, written as (1 - x)^4 p(x) / 32 with
// p(x) = 16 + 29 x + 20 x^2 + 5 x^3 (> 0 on [-1, 1]): no cancellation as x -> 1, so s stays
// positive wherever x < 1.
__device__ __forceinline__ double switch_p(double x) { return 16.0 + x * (29.0 + x * (20.0 + 5.0 * x)); }
__device__ __forceinline__ double switch_s(double x) {
  const double u = 1.0 - x, u2 = u * u;
  return u2 * u2 * switch_p(x) * (1.0 / 32.0);
}
// s'(x) / s(x) = -35 (1 + x)^3 / ((1 - x) p(x)), finite for x < 1 (no division by s)
__device__ __forceinline__ double switch_dlns(double x) {
  const double v = 1.0 + x;
  return -35.0 * v * v * v / ((1.0 - x) * switch_p(x));
}

// One workgroup per batch, one thread per point (strided).  For a point p with owner o and
// F_p = v_p n_p + D_p (D_p = sum_ij P_ij phi_i tphi_j at p):
//   partition:  F_p dw_p/dR_a for every atom, with the point's own motion credited to o;
//   potential:  w_p n_p dv_p/dR_a likewise (for a != o the atom's own term, for o the others');
//   basis:      the point-motion sum G_p (from the Pulay pass) credited to o.
// Per-atom sums of the workgroup are kept in LDS and added to dE/dR (times gE) at the end.
__global__ void __launch_bounds__(256)
gridforce_kernel(const BatchDesc* __restrict__ batches, const double4* __restrict__ pts,
                 const int32_t* __restrict__ perm, const SystemDesc* __restrict__ systems,
                 const int32_t* __restrict__ sys_natoms, const double* __restrict__ atom_xyz,
                 const double* __restrict__ atom_Z, const double* __restrict__ sys_model,
                 const int32_t* __restrict__ pt_owner, const double* __restrict__ pt_wgrid,
                 const double* __restrict__ v_model, const double* __restrict__ n_sorted,
                 const double* __restrict__ d_sorted, const double* __restrict__ gpt,
                 const double* __restrict__ gE, double* __restrict__ dE_dR) {
  extern __shared__ double acc[];          // [na][3] of this batch's system
  const BatchDesc d = batches[blockIdx.x];
  const int a0 = systems[d.sys].atom_off, na = sys_natoms[d.sys];
  const double sigma = sys_model[2 * d.sys], pa = sys_model[2 * d.sys + 1];
  const double q = (1.0 + pa) / (1.0 - pa);
  for (int t = threadIdx.x; t < 3 * na; t += blockDim.x) acc[t] = 0.0;
  __syncthreads();
  const double* X = atom_xyz + 3 * (size_t)a0;
  const double* Z = atom_Z + a0;
  for (int p = threadIdx.x; p < d.n_p; p += blockDim.x) {
    const int i = d.pt_off + p;
    const double4 P4 = pts[i];
    const int o = pt_owner[i] - a0;
    const double n = n_sorted[i], F = v_model[perm[i]] * n + d_sorted[i];
    double go[3] = {0.0, 0.0, 0.0};      // owner's share (the point's own motion)
    // ---- potential: grad_p of each atom's term -Z erf(r/sigma)/r
    {
      const double wn = P4.w * n;
      for (int a = 0; a < na; ++a) {
        const double dx = P4.x - X[3 * a], dy = P4.y - X[3 * a + 1], dz = P4.z - X[3 * a + 2];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (!(r > 1e-12)) continue;
        const double e = erf(r / sigma);
        const double dfr = (1.1283791670955125739 / sigma) * exp(-(r * r) / (sigma * sigma)) / r - e / (r * r);
        const double c = -Z[a] * dfr / r * wn;     // w n grad_p(v_a) = c (p - R_a)
        const double gx = c * dx, gy = c * dy, gz = c * dz;
        if (a != o) {
          atomicAdd(&acc[3 * a], -gx);
          atomicAdd(&acc[3 * a + 1], -gy);
          atomicAdd(&acc[3 * a + 2], -gz);
          go[0] += gx;
          go[1] += gy;
          go[2] += gz;
        }
      }
    }
    // ---- partition weights: only atoms closer than dmin (1 + a) / (1 - a) have S_b > 0
    if (na > 1 && F != 0.0) {
      double dmin = 1e300;
      for (int b = 0; b < na; ++b) {
        const double dx = P4.x - X[3 * b], dy = P4.y - X[3 * b + 1], dz = P4.z - X[3 * b + 2];
        dmin = fmin(dmin, sqrt(dx * dx + dy * dy + dz * dz));
      }
      auto S_of = [&](int b, double rb) {      // prod_{c != b} s(mu_bc)
        double S = 1.0;
        for (int c = 0; c < na && S > 0.0; ++c) {
          if (c == b) continue;
          const double cx = P4.x - X[3 * c], cy = P4.y - X[3 * c + 1], cz = P4.z - X[3 * c + 2];
          const double rc_ = sqrt(cx * cx + cy * cy + cz * cz);
          const double ex = X[3 * b] - X[3 * c], ey = X[3 * b + 1] - X[3 * c + 1], ez = X[3 * b + 2] - X[3 * c + 2];
          const double x = (rb - rc_) / sqrt(ex * ex + ey * ey + ez * ez) / pa;
          S *= x >= 1.0 ? 0.0 : (x <= -1.0 ? 1.0 : switch_s(x));
        }
        return S;
      };
      double Ssum = 0.0, So = 0.0;
      for (int b = 0; b < na; ++b) {
        const double bx = P4.x - X[3 * b], by = P4.y - X[3 * b + 1], bz = P4.z - X[3 * b + 2];
        const double rb = sqrt(bx * bx + by * by + bz * bz);
        if (!(rb < dmin * q)) continue;
        const double S = S_of(b, rb);
        Ssum += S;
        if (b == o) So = S;
      }
      const double w = P4.w;        // = g_p So / Ssum, the weight the energy used
      if (w != 0.0 && So > 0.0 && Ssum > 0.0) {
        // dw = w sum_b (delta_bo - S_b / Ssum) dln S_b,  dln S_b = sum_c (s'/s)(mu_bc) dmu_bc
        for (int b = 0; b < na; ++b) {
          const double bx = P4.x - X[3 * b], by = P4.y - X[3 * b + 1], bz = P4.z - X[3 * b + 2];
          const double rb = sqrt(bx * bx + by * by + bz * bz);
          if (!(rb < dmin * q)) continue;
          const double Sb = S_of(b, rb);
          if (Sb <= 0.0) continue;
          const double kap = w * F * ((b == o ? 1.0 : 0.0) - Sb / Ssum);
          if (kap == 0.0) continue;
          const double ub[3] = {bx / rb, by / rb, bz / rb};
          for (int c = 0; c < na; ++c) {
            if (c == b) continue;
            const double cx = P4.x - X[3 * c], cy = P4.y - X[3 * c + 1], cz = P4.z - X[3 * c + 2];
            const double rc_ = sqrt(cx * cx + cy * cy + cz * cz);
            const double e3[3] = {X[3 * b] - X[3 * c], X[3 * b + 1] - X[3 * c + 1], X[3 * b + 2] - X[3 * c + 2]};
            const double Rbc = sqrt(e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2]);
            const double mu = (rb - rc_) / Rbc;
            const double x = mu / pa;
            if (x <= -1.0 || x >= 1.0) continue;             // s is constant there (s' = 0)
            const double t = kap * switch_dlns(x) / (pa * Rbc);
            const double uc[3] = {cx / rc_, cy / rc_, cz / rc_};
            for (int m = 0; m < 3; ++m) {
              const double e = e3[m] / Rbc;
              go[m] += t * (ub[m] - uc[m]);                      // via the point (moves with o)
              atomicAdd(&acc[3 * b + m], t * (-ub[m] - mu * e));  // via R_b
              atomicAdd(&acc[3 * c + m], t * (uc[m] + mu * e));   // via R_c
            }
          }
        }
      }
    }
    // ---- basis point motion (summed over all functions in the Pulay pass)
    go[0] += gpt[3 * (size_t)i];
    go[1] += gpt[3 * (size_t)i + 1];
    go[2] += gpt[3 * (size_t)i + 2];
    atomicAdd(&acc[3 * o], go[0]);
    atomicAdd(&acc[3 * o + 1], go[1]);
    atomicAdd(&acc[3 * o + 2], go[2]);
  }
  __syncthreads();
  const double ge = gE[0];
  for (int t = threadIdx.x; t < 3 * na; t += blockDim.x)
    if (acc[t] != 0.0) unsafeAtomicAdd(dE_dR + 3 * (size_t)a0 + t, ge * acc[t]);
}

// Wave-per-point form of the same terms, for systems of at most 64 K atoms.  Each workgroup
// takes a range of consecutive batches of one system; wave w handles points w, w + 4, ... of each
// batch.  Lane l owns atoms c = 64 j + l (j < K): it keeps their distances to the current point,
// their partition products S_c and their accumulated gradient in registers, so the potential term
// and the "via R_c" partition term need no atomics.  Per point:
//   * S_b is formed only for atoms with r_b < q r_min (others are exactly 0), and only if the
//     nearest atom n does not already switch b off (x_bn >= 1); the product over c is a wave
//     product;
//   * the "via R_b" term of atom b is a wave sum credited to b's lane;
//   * the point-motion share goes to the owner's lane, one wave sum per run of points with the
//     same owner.
// inv_aR holds 1 / (a |R_b - R_c|) per system (row b, column c).  Every workgroup writes its
// per-atom sums to its own slot of `part`; gridforce_reduce_kernel adds the slots in a fixed
// order, so the result does not depend on scheduling.
__device__ __forceinline__ double wave_sum_bcast(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return __shfl(v, 0);               // every lane takes lane 0's rounding
}
__device__ __forceinline__ double wave_prod_bcast(double v) {
  for (int off = 32; off > 0; off >>= 1) v *= __shfl_xor(v, off);
  return __shfl(v, 0);
}
__device__ __forceinline__ double wave_min(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}

template <int K>
__global__ void __launch_bounds__(256)
gridforce_wave_kernel(const ForceRange* __restrict__ ranges, const BatchDesc* __restrict__ batches,
                      const double4* __restrict__ pts, const int32_t* __restrict__ perm,
                      const SystemDesc* __restrict__ systems, const int32_t* __restrict__ sys_natoms,
                      const double* __restrict__ atom_xyz, const double* __restrict__ atom_Z,
                      const double* __restrict__ sys_model, const int64_t* __restrict__ sys_pair_off,
                      const double* __restrict__ inv_aR, const int32_t* __restrict__ pt_owner,
                      const double* __restrict__ v_model, const double* __restrict__ n_sorted,
                      const double* __restrict__ d_sorted, const double* __restrict__ gpt,
                      double* __restrict__ part) {
  extern __shared__ double wsum[];          // [4 waves][3 na]
  const ForceRange R = ranges[blockIdx.x];
  const int sy = R.sys;
  const int a0 = systems[sy].atom_off, na = sys_natoms[sy];
  const double sigma = sys_model[2 * sy], pa = sys_model[2 * sy + 1];
  const double q = (1.0 + pa) / (1.0 - pa), inv_sigma = 1.0 / sigma;
  const double* X = atom_xyz + 3 * (size_t)a0;
  const double* Z = atom_Z + a0;
  const double* T = inv_aR + sys_pair_off[sy];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  double acc[K][3];
#pragma unroll
  for (int j = 0; j < K; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.0;
  double go[3] = {0.0, 0.0, 0.0};          // lane share of the current owner's point-motion sum
  int cur_o = -1;
  auto flush_owner = [&]() {
    if (cur_o < 0) return;
    const double g0 = wave_sum_bcast(go[0]), g1 = wave_sum_bcast(go[1]), g2 = wave_sum_bcast(go[2]);
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (64 * j + lane == cur_o) {
        acc[j][0] += g0;
        acc[j][1] += g1;
        acc[j][2] += g2;
      }
    go[0] = go[1] = go[2] = 0.0;
  };

  for (int bt = R.b0; bt < R.b1; ++bt) {
    const BatchDesc d = batches[bt];
    for (int p = wave; p < d.n_p; p += 4) {
      const int i = d.pt_off + p;
      const double4 P4 = pts[i];
      const int o = pt_owner[i] - a0;
      if (o != cur_o) {
        flush_owner();
        cur_o = o;
      }
      const double n = n_sorted[i], F = v_model[perm[i]] * n + d_sorted[i];
      const double wn = P4.w * n;
      // ---- distances, and the potential term: grad_p of -Z_c erf(r / sigma) / r
      double rc[K];
      double dloc = 1e300;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int c = 64 * j + lane;
        rc[j] = 1e300;
        if (c < na) {
          const double dx = P4.x - X[3 * c], dy = P4.y - X[3 * c + 1], dz = P4.z - X[3 * c + 2];
          const double r = sqrt(dx * dx + dy * dy + dz * dz);
          rc[j] = r;
          dloc = fmin(dloc, r);
          if (c != o && r > 1e-12) {
            const double u = r * inv_sigma;
            // beyond u = 6.5, erf(u) = 1 and the Gaussian term is below 4e-18 of 1/r^2
            const double dfr = u > 6.5 ? -1.0 / (r * r)
                                       : (1.1283791670955125739 * inv_sigma) * exp(-u * u) / r - erf(u) / (r * r);
            const double cf = -Z[c] * dfr / r * wn;       // w n grad_p(v_c) = cf (p - R_c)
            acc[j][0] -= cf * dx;
            acc[j][1] -= cf * dy;
            acc[j][2] -= cf * dz;
            go[0] += cf * dx;
            go[1] += cf * dy;
            go[2] += cf * dz;
          }
        }
      }
      if (lane == 0) {                     // basis point motion (from the Pulay pass)
        go[0] += gpt[3 * (size_t)i];
        go[1] += gpt[3 * (size_t)i + 1];
        go[2] += gpt[3 * (size_t)i + 2];
      }
      if (na < 2 || F == 0.0 || P4.w == 0.0) continue;
      // ---- partition products of the candidate atoms
      const double dmin = wave_min(dloc), lim = dmin * q;
      int nn = -1;                          // nearest atom (lowest index on ties)
#pragma unroll
      for (int j = K - 1; j >= 0; --j) {
        const unsigned long long m = __ballot(rc[j] == dmin);
        if (m) nn = 64 * j + __ffsll((long long)m) - 1;
      }
      double Sreg[K];
      double Ssum = 0.0, So = 0.0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        Sreg[j] = 0.0;
        unsigned long long m = __ballot(rc[j] < lim);
        while (m) {
          const int l = __ffsll((long long)m) - 1;
          m &= m - 1;
          const int b = 64 * j + l;
          const double rb = __shfl(rc[j], l);
          const double* Tb = T + (size_t)b * na;
          if (b != nn && (rb - dmin) * Tb[nn] >= 1.0) continue;     // switched off by the nearest
          double f = 1.0;
#pragma unroll
          for (int jj = 0; jj < K; ++jj) {
            const int c = 64 * jj + lane;
            if (c < na && c != b) {
              const double x = (rb - rc[jj]) * Tb[c];
              f *= x >= 1.0 ? 0.0 : (x <= -1.0 ? 1.0 : switch_s(x));
            }
          }
          const double Sb = wave_prod_bcast(f);
          if (lane == l) Sreg[j] = Sb;
          Ssum += Sb;
          if (b == o) So = Sb;
        }
      }
      if (!(So > 0.0 && Ssum > 0.0)) continue;
      // ---- dw = w sum_b (delta_bo - S_b / Ssum) dln S_b
      const double wF = P4.w * F;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        unsigned long long m = __ballot(Sreg[j] > 0.0);
        while (m) {
          const int l = __ffsll((long long)m) - 1;
          m &= m - 1;
          const int b = 64 * j + l;
          const double Sb = __shfl(Sreg[j], l), rb = __shfl(rc[j], l);
          const double kap = wF * ((b == o ? 1.0 : 0.0) - Sb / Ssum);
          if (kap == 0.0) continue;
          const double Xb0 = X[3 * b], Xb1 = X[3 * b + 1], Xb2 = X[3 * b + 2];
          const double ub0 = (P4.x - Xb0) / rb, ub1 = (P4.y - Xb1) / rb, ub2 = (P4.z - Xb2) / rb;
          const double* Tb = T + (size_t)b * na;
          double ab0 = 0.0, ab1 = 0.0, ab2 = 0.0;
#pragma unroll
          for (int jj = 0; jj < K; ++jj) {
            const int c = 64 * jj + lane;
            if (c < na && c != b) {
              const double tinv = Tb[c];
              const double x = (rb - rc[jj]) * tinv;
              if (x > -1.0 && x < 1.0) {
                const double t = kap * switch_dlns(x) * tinv;
                const double mu = x * pa, es = tinv * pa;
                const double Xc0 = X[3 * c], Xc1 = X[3 * c + 1], Xc2 = X[3 * c + 2];
                const double ir = 1.0 / rc[jj];
                const double uc0 = (P4.x - Xc0) * ir, uc1 = (P4.y - Xc1) * ir, uc2 = (P4.z - Xc2) * ir;
                const double e0 = (Xb0 - Xc0) * es, e1 = (Xb1 - Xc1) * es, e2 = (Xb2 - Xc2) * es;
                go[0] += t * (ub0 - uc0);                 // via the point (moves with o)
                go[1] += t * (ub1 - uc1);
                go[2] += t * (ub2 - uc2);
                ab0 += t * (-ub0 - mu * e0);              // via R_b
                ab1 += t * (-ub1 - mu * e1);
                ab2 += t * (-ub2 - mu * e2);
                acc[jj][0] += t * (uc0 + mu * e0);        // via R_c
                acc[jj][1] += t * (uc1 + mu * e1);
                acc[jj][2] += t * (uc2 + mu * e2);
              }
            }
          }
          ab0 = wave_sum_bcast(ab0);
          ab1 = wave_sum_bcast(ab1);
          ab2 = wave_sum_bcast(ab2);
          if (lane == l) {
            acc[j][0] += ab0;
            acc[j][1] += ab1;
            acc[j][2] += ab2;
          }
        }
      }
    }
  }
  flush_owner();
  // ---- the four waves' sums, added in wave order, into this workgroup's slot
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int c = 64 * j + lane;
    if (c < na) {
      wsum[(size_t)wave * 3 * na + 3 * c] = acc[j][0];
      wsum[(size_t)wave * 3 * na + 3 * c + 1] = acc[j][1];
      wsum[(size_t)wave * 3 * na + 3 * c + 2] = acc[j][2];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 3 * na; t += blockDim.x)
    part[R.part_off + t] = ((wsum[t] + wsum[3 * na + t]) + wsum[6 * na + t]) + wsum[9 * na + t];
}

// dE/dR_a += gE sum over the system's workgroup slots: one workgroup per (component, system);
// thread k adds slots k, k + 256, ... and a fixed tree adds the 256 partial sums, so the order
// of additions never changes
__global__ void __launch_bounds__(256)
gridforce_reduce_kernel(const double* __restrict__ part, const int64_t* __restrict__ sys_part_off,
                        const int32_t* __restrict__ sys_nrange, const SystemDesc* __restrict__ systems,
                        const int32_t* __restrict__ sys_natoms, const double* __restrict__ gE,
                        double* __restrict__ dE_dR) {
  __shared__ double sh[256];
  const int sy = blockIdx.y, na = sys_natoms[sy];
  const int t = blockIdx.x;
  if (t >= 3 * na) return;                 // the whole workgroup
  const double* src = part + sys_part_off[sy] + t;
  const int nr = sys_nrange[sy];
  double s = 0.0;
  for (int r = threadIdx.x; r < nr; r += blockDim.x) s += src[(size_t)r * 3 * na];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) dE_dR[3 * (size_t)systems[sy].atom_off + t] += gE[0] * sh[0];
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
hipError_t launch_vext(const DeviceView& dv, int64_t n, const int32_t* pt_sys,
                       const int32_t* sys_natoms, const double* atom_Z, const double* sys_model,
                       double* v_out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(vext_kernel, dim3(grid_for((size_t)n, 256)), dim3(256), 0, st, dv.pts, dv.perm,
                     n, pt_sys, dv.systems, sys_natoms, dv.atom_xyz, atom_Z, sys_model, v_out);
  return hipGetLastError();
}

hipError_t launch_gridforce(const DeviceView& dv, int nbatch, int max_sys_atoms,
                            const int32_t* sys_natoms, const double* atom_Z, const double* sys_model,
                            const int32_t* pt_owner, const double* pt_wgrid, const double* v_model,
                            const double* n_sorted, const double* d_sorted, const double* gpt,
                            const double* gE, double* dE_dR, hipStream_t st) {
  if (nbatch == 0) return hipSuccess;
  const size_t lds = 3 * (size_t)max_sys_atoms * sizeof(double);
  hipLaunchKernelGGL(gridforce_kernel, dim3(nbatch), dim3(256), lds, st, dv.batches, dv.pts, dv.perm,
                     dv.systems, sys_natoms, dv.atom_xyz, atom_Z, sys_model, pt_owner, pt_wgrid,
                     v_model, n_sorted, d_sorted, gpt, gE, dE_dR);
  return hipGetLastError();
}

hipError_t launch_gridforce_wave(const DeviceView& dv, int k_chunks, const ForceRange* ranges,
                                 int n_ranges, int max_sys_atoms, const int32_t* sys_natoms,
                                 const double* atom_Z, const double* sys_model,
                                 const int64_t* sys_pair_off, const double* inv_aR,
                                 const int32_t* pt_owner, const double* v_model,
                                 const double* n_sorted, const double* d_sorted, const double* gpt,
                                 double* part, const int64_t* sys_part_off, const int32_t* sys_nrange,
                                 const double* gE, double* dE_dR, hipStream_t st) {
  if (max_sys_atoms > 64 * k_chunks) return hipErrorInvalidValue;
  if (n_ranges > 0) {
    const size_t lds = 4 * 3 * (size_t)max_sys_atoms * sizeof(double);
#define AIMS_GF_LAUNCH(KK)                                                                       \
  hipLaunchKernelGGL(gridforce_wave_kernel<KK>, dim3(n_ranges), dim3(256), lds, st, ranges,      \
                     dv.batches, dv.pts, dv.perm, dv.systems, sys_natoms, dv.atom_xyz, atom_Z,  \
                     sys_model, sys_pair_off, inv_aR, pt_owner, v_model, n_sorted, d_sorted,     \
                     gpt, part)
    switch (k_chunks) {
      case 1: AIMS_GF_LAUNCH(1); break;
      case 2: AIMS_GF_LAUNCH(2); break;
      case 4: AIMS_GF_LAUNCH(4); break;
      case 8: AIMS_GF_LAUNCH(8); break;
      default: return hipErrorInvalidValue;
    }
#undef AIMS_GF_LAUNCH
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(gridforce_reduce_kernel, dim3(3 * max_sys_atoms, dv.n_sys),
                     dim3(256), 0, st, part, sys_part_off, sys_nrange, dv.systems, sys_natoms, gE,
                     dE_dR);
  return hipGetLastError();
}

}  // namespace aims
