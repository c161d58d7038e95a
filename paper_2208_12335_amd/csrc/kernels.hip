// gfx950 kernels of the NAO grid-integration core.
//
//   phi_eval_kernel   basis values of one batch -> two slabs in HBM scratch (function-major,
//                     points contiguous): Phi^T and a second operand (t Phi^T, or
//                     w (v Phi + t Phi)^T for H, or w Phi^T for S)
//   density_kernel    per (batch, j-tile, p-tile): X^T = P_b Phi^T on MFMA, epilogue
//                     n_p += sum_j X_pj phi_j(p) and the E_T partial sum_p w_p sum_j X_pj tphi_j
//   hs_kernel         per (batch, i-tile, j-tile): C = Phi^T (second operand)^T on MFMA over the
//                     batch's points, scatter-added in FP64 into the dense H (or S)
//   finish kernels    caller-order scatter of n and deterministic FP64 sums N, E_V, E_T
//
// Precision policies: FP64 (double slabs, v_mfma_f64_16x16x4f64), FP32 (float slabs,
// v_mfma_f32_16x16x4f32); both accumulate per tile in the slab type and reduce across batches
// in FP64.
#include <hip/hip_runtime.h>

#include "aims_internal.h"
#include "basis.h"
#include "kernels.h"

namespace aims {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<double> { typedef d4_t type; };
template <> struct Acc<float> { typedef f4_t type; };

__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma16(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row of the 16 x 16 output block held in accumulator register r of a lane (the column is
// lane % 16).  Measured on gfx950: the FP64 instruction interleaves the rows of the four lane
// groups, the FP32 and BF16 instructions give each lane group four consecutive rows.
template <typename T>
__device__ __forceinline__ int acc_row(int lane, int r) {
  return sizeof(T) == 8 ? 4 * r + (lane >> 4) : 4 * (lane >> 4) + r;
}

// ------------------------------------------------------------------------------------------
// basis evaluation into slabs
// ------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void eval_atom_point(double dx, double dy, double dz,
                                                const SpeciesDesc& sd,
                                                const int32_t* __restrict__ shell_l,
                                                const T* __restrict__ spline,
                                                const RadialGrid& rg, int mode, T w, T wv,
                                                T* __restrict__ o1, T* __restrict__ o2, int ldp) {
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  if (!(r < rg.rc)) {
    for (int f = 0; f < sd.nfn; ++f) {
      o1[(size_t)f * ldp] = T(0);
      o2[(size_t)f * ldp] = T(0);
    }
    return;
  }
  const double rr = fmax(r, 1e-12);
  const double inv = 1.0 / rr;
  const T ux = T(dx * inv), uy = T(dy * inv), uz = T(dz * inv);
  const RadialPos rp = radial_pos(rr, rg);
  const T dt = T(rp.dt);
  const T* c = spline + sd.spline_off + (size_t)rp.k * sd.nshell * 8;
  int f = 0;
  for (int j = 0; j < sd.nshell; ++j) {
    const T R = cubic(c + j * 8, dt);
    const T K = cubic(c + j * 8 + 4, dt);
    const int l = shell_l[sd.shell_l_off + j];
    T Y[7];
    ylm_l<T>(l, ux, uy, uz, Y);
    const int nm = 2 * l + 1;
    for (int m = 0; m < nm; ++m) {
      const T phi = R * Y[m];
      const T tphi = K * Y[m];
      T second;
      if (mode == kModeDensity) second = tphi;
      else if (mode == kModeH) second = wv * phi + w * tphi;
      else second = w * phi;
      o1[(size_t)(f + m) * ldp] = phi;
      o2[(size_t)(f + m) * ldp] = second;
    }
    f += nm;
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
phi_eval_kernel(const BatchDesc* __restrict__ batches, int b0, const double4* __restrict__ pts,
                const int32_t* __restrict__ perm, const int32_t* __restrict__ batch_atoms,
                const int32_t* __restrict__ batch_acol, const double* __restrict__ atom_xyz,
                const int32_t* __restrict__ atom_species, const SpeciesDesc* __restrict__ species,
                const int32_t* __restrict__ shell_l, const T* __restrict__ spline, RadialGrid rg,
                const double* __restrict__ v, int mode, T* __restrict__ slab1,
                T* __restrict__ slab2) {
  const BatchDesc d = batches[b0 + blockIdx.x];
  const int np = d.n_p, na = d.n_atoms, ldp = d.ldp;
  T* s1 = slab1 + d.slab_off;
  T* s2 = slab2 + d.slab_off;
  const int pairs = np * na;
  for (int q = threadIdx.x; q < pairs; q += blockDim.x) {
    const int k = q / np;
    const int p = q - k * np;
    const int atom = batch_atoms[d.atom_off + k];
    const int col0 = batch_acol[d.atom_off + k];
    const SpeciesDesc sd = species[atom_species[atom]];
    const double4 P4 = pts[d.pt_off + p];
    double wv = 0.0;
    if (mode == kModeH) wv = P4.w * v[perm[d.pt_off + p]];
    eval_atom_point<T>(P4.x - atom_xyz[3 * atom], P4.y - atom_xyz[3 * atom + 1],
                       P4.z - atom_xyz[3 * atom + 2], sd, shell_l, spline, rg, mode, T(P4.w),
                       T(wv), s1 + (size_t)col0 * ldp + p, s2 + (size_t)col0 * ldp + p, ldp);
  }
  // zero the padding columns so that the K loops may run over whole padded rows
  const int padw = ldp - np;
  if (padw > 0) {
    const int tot = d.n_b * padw;
    for (int q = threadIdx.x; q < tot; q += blockDim.x) {
      const int row = q / padw;
      const int p = np + (q - row * padw);
      s1[(size_t)row * ldp + p] = T(0);
      s2[(size_t)row * ldp + p] = T(0);
    }
  }
}

// ------------------------------------------------------------------------------------------
// tiled MFMA kernels: 256 threads = 4 waves, 64 x 64 output tile, each wave a 32 x 32 quarter
// made of 2 x 2 blocks of 16 x 16 MFMA outputs; K staged through LDS in chunks of 16.
// ------------------------------------------------------------------------------------------
constexpr int kKC = 16;
constexpr int kLds = kTile + 16;   // padded LDS row length (elements)

// XCD-aware work order: the dispatcher places workgroup g on XCD g % 8, so consecutive work
// items (tiles of the same batch, which share its slab) are given workgroup ids that differ by
// multiples of 8 and stay in one XCD's L2.
__device__ __forceinline__ int xcd_item(int g, int n) {
  const int per = (n + 7) / 8;
  const int xcd = g & 7;
  const int slot = g >> 3;
  // items [xcd*per, (xcd+1)*per) go to this XCD; g runs over all n ids exactly once when the
  // grid is padded to a multiple of 8 and out-of-range ids are dropped
  return xcd * per + slot;
}

template <typename T>
__device__ __forceinline__ void mfma_chunk(const T (*As)[kLds], const T (*Bs)[kLds], int lane,
                                           int wm, int wn, typename Acc<T>::type (&acc)[2][2]) {
#pragma unroll
  for (int kk = 0; kk < kKC; kk += 4) {
    const int kr = kk + (lane >> 4);
    T a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = As[kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 2; ++i) b[i] = Bs[kr][wn * 32 + i * 16 + (lane & 15)];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = mfma16(a[mi], b[ni], acc[mi][ni]);
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
density_kernel(const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
               const SystemDesc* __restrict__ systems, const double4* __restrict__ pts,
               const int32_t* __restrict__ batch_cols, const T* __restrict__ Pmat,
               const T* __restrict__ slab1, const T* __restrict__ slab2,
               double* __restrict__ n_sorted, double* __restrict__ et_part) {
  const int item = xcd_item(blockIdx.x, n_items);
  if (item >= n_items) return;
  const TileItem it = items[item];
  const BatchDesc d = batches[it.batch];
  const SystemDesc sys = systems[d.sys];
  const int nb = d.n_b, ldp = d.ldp;
  const int j0 = it.ti * kTile;       // rows of X^T: basis functions
  const int p0 = it.tj * kTile;       // columns: points
  const int* cols = batch_cols + d.col_off;
  const T* S1 = slab1 + d.slab_off;
  const T* S2 = slab2 + d.slab_off;
  const T* Pm = Pmat + sys.mat_off;

  __shared__ T As[kKC][kLds];
  __shared__ T Bs[kKC][kLds];
  __shared__ double red_n[2][kTile];
  __shared__ double red_e[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  typedef typename Acc<T>::type acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = acc_t{0, 0, 0, 0};

  // rows of P_b this thread stages: m = e / 16 for e = tid + 256 q
  int grow[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = (tid + 256 * q) >> 4;
    grow[q] = (j0 + m < nb) ? cols[j0 + m] : -1;
  }
  const bool wave_live = (j0 + wm * 32 < nb) && (p0 + wn * 32 < d.n_p);

  for (int kc = 0; kc < nb; kc += kKC) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int m = e >> 4, kk = e & 15;
      T val = T(0);
      if (grow[q] >= 0 && kc + kk < nb) val = Pm[(size_t)grow[q] * sys.nb + cols[kc + kk]];
      As[kk][m] = val;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int kk = e >> 6, n = e & 63;
      T val = T(0);
      if (kc + kk < nb && p0 + n < ldp) val = S1[(size_t)(kc + kk) * ldp + p0 + n];
      Bs[kk][n] = val;
    }
    __syncthreads();
    if (wave_live) mfma_chunk<T>(As, Bs, lane, wm, wn, acc);
    __syncthreads();
  }

  // epilogue: column sums of X^T o Phi^T (density) and of w X^T o tPhi^T (kinetic energy)
  double sn[2] = {0.0, 0.0}, se = 0.0;
#pragma unroll
  for (int ni = 0; ni < 2; ++ni) {
    const int p = p0 + wn * 32 + ni * 16 + (lane & 15);
    double accn = 0.0, acce = 0.0;
    if (p < d.n_p) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = j0 + wm * 32 + mi * 16 + acc_row<T>(lane, r);
          if (j < nb) {
            const double x = (double)acc[mi][ni][r];
            accn += x * (double)S1[(size_t)j * ldp + p];
            acce += x * (double)S2[(size_t)j * ldp + p];
          }
        }
      acce *= pts[d.pt_off + p].w;
    }
    accn += __shfl_xor(accn, 16);
    accn += __shfl_xor(accn, 32);
    sn[ni] = accn;
    se += acce;
  }
  // wave-level sum of the energy part
  for (int off = 32; off > 0; off >>= 1) se += __shfl_xor(se, off);
  if (lane < 16) {
    red_n[wm][wn * 32 + lane] = sn[0];
    red_n[wm][wn * 32 + 16 + lane] = sn[1];
  }
  if (lane == 0) red_e[wave] = se;
  __syncthreads();
  if (tid < kTile) {
    const int p = p0 + tid;
    if (p < d.n_p) unsafeAtomicAdd(n_sorted + d.pt_off + p, red_n[0][tid] + red_n[1][tid]);
  }
  if (tid == 0) et_part[item] = (red_e[0] + red_e[1]) + (red_e[2] + red_e[3]);
}

template <typename T>
__global__ void __launch_bounds__(256)
hs_kernel(const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
          const SystemDesc* __restrict__ systems, const int32_t* __restrict__ batch_cols,
          const T* __restrict__ slab1, const T* __restrict__ slab2, double* __restrict__ out) {
  const int item = xcd_item(blockIdx.x, n_items);
  if (item >= n_items) return;
  const TileItem it = items[item];
  const BatchDesc d = batches[it.batch];
  const SystemDesc sys = systems[d.sys];
  const int nb = d.n_b, ldp = d.ldp;
  const int i0 = it.ti * kTile, jb = it.tj * kTile;
  const int* cols = batch_cols + d.col_off;
  const T* S1 = slab1 + d.slab_off;
  const T* S2 = slab2 + d.slab_off;

  __shared__ T As[kKC][kLds];
  __shared__ T Bs[kKC][kLds];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  typedef typename Acc<T>::type acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = acc_t{0, 0, 0, 0};
  const bool wave_live = (i0 + wm * 32 < nb) && (jb + wn * 32 < nb);

  for (int kc = 0; kc < ldp; kc += kKC) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int m = e >> 4, kk = e & 15;
      As[kk][m] = (i0 + m < nb) ? S1[(size_t)(i0 + m) * ldp + kc + kk] : T(0);
      Bs[kk][m] = (jb + m < nb) ? S2[(size_t)(jb + m) * ldp + kc + kk] : T(0);
    }
    __syncthreads();
    if (wave_live) mfma_chunk<T>(As, Bs, lane, wm, wn, acc);
    __syncthreads();
  }
  if (!wave_live) return;
  double* O = out + sys.mat_off;
#pragma unroll
  for (int ni = 0; ni < 2; ++ni) {
    const int j = jb + wn * 32 + ni * 16 + (lane & 15);
    if (j >= nb) continue;
    const size_t gj = (size_t)cols[j];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm * 32 + mi * 16 + acc_row<T>(lane, r);
        if (i < nb) unsafeAtomicAdd(O + (size_t)cols[i] * sys.nb + gj, (double)acc[mi][ni][r]);
      }
  }
}

// ------------------------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------------------------
__global__ void fill_kernel(double* __restrict__ x, size_t n, double val) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    x[i] = val;
}

template <typename T>
__global__ void convert_kernel(const double* __restrict__ x, T* __restrict__ y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    y[i] = T(x[i]);
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// Scatter n to caller order and form per-block partial sums of w n and w v n over the points
// [pt0, pt1) of one system (blockIdx.y = system).
__global__ void __launch_bounds__(256)
density_finish_kernel(const int64_t* __restrict__ sys_pt_range, const double4* __restrict__ pts,
                      const int32_t* __restrict__ perm, const double* __restrict__ n_sorted,
                      const double* __restrict__ v, double* __restrict__ n_out,
                      double* __restrict__ part, int nblk) {
  __shared__ double sh[4];
  const int s = blockIdx.y;
  const int64_t a = sys_pt_range[2 * s], b = sys_pt_range[2 * s + 1];
  double sn = 0.0, sv = 0.0;
  for (int64_t i = a + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < b;
       i += (int64_t)nblk * blockDim.x) {
    const double n = n_sorted[i];
    const int q = perm[i];
    n_out[q] = n;
    const double wn = pts[i].w * n;
    sn += wn;
    if (v) sv += wn * v[q];
  }
  sn = block_sum<256>(sn, sh);
  sv = block_sum<256>(sv, sh);
  if (threadIdx.x == 0) {
    part[(size_t)s * nblk * 2 + 2 * blockIdx.x] = sn;
    part[(size_t)s * nblk * 2 + 2 * blockIdx.x + 1] = sv;
  }
}

// One block per system: sums_out[3 s + (0, 1, 2)] = N, E_V, E_T in a fixed order.
__global__ void __launch_bounds__(256)
sums_finish_kernel(const double* __restrict__ part, int nblk, const int64_t* __restrict__ sys_item_range,
                   const double* __restrict__ et_part, double* __restrict__ sums_out) {
  __shared__ double sh[4];
  const int s = blockIdx.x;
  double sn = 0.0, sv = 0.0, se = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
    sn += part[(size_t)s * nblk * 2 + 2 * i];
    sv += part[(size_t)s * nblk * 2 + 2 * i + 1];
  }
  for (int64_t i = sys_item_range[2 * s] + threadIdx.x; i < sys_item_range[2 * s + 1]; i += blockDim.x)
    se += et_part[i];
  sn = block_sum<256>(sn, sh);
  sv = block_sum<256>(sv, sh);
  se = block_sum<256>(se, sh);
  if (threadIdx.x == 0) {
    sums_out[3 * s] = sn;
    sums_out[3 * s + 1] = sv;
    sums_out[3 * s + 2] = se;
  }
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
static inline int grid_for(size_t n, int per) {
  size_t g = (n + per - 1) / per;
  if (g > 65536) g = 65536;
  return (int)(g ? g : 1);
}

hipError_t launch_fill(double* x, size_t n, double val, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256 * 4)), dim3(256), 0, st, x, n, val);
  return hipGetLastError();
}

hipError_t launch_convert_f32(const double* x, float* y, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(convert_kernel<float>, dim3(grid_for(n, 256 * 4)), dim3(256), 0, st, x, y, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_phi_eval(const DeviceView& dv, int b0, int nbatch, int mode, const double* v,
                           T* slab1, T* slab2, hipStream_t st) {
  if (nbatch == 0) return hipSuccess;
  const T* spline = (const T*)(sizeof(T) == 8 ? (const void*)dv.spline64 : (const void*)dv.spline32);
  hipLaunchKernelGGL(phi_eval_kernel<T>, dim3(nbatch), dim3(256), 0, st, dv.batches, b0, dv.pts,
                     dv.perm, dv.batch_atoms, dv.batch_acol, dv.atom_xyz, dv.atom_species,
                     dv.species, dv.shell_l, spline, dv.rg, v, mode, slab1, slab2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_density(const DeviceView& dv, const TileItem* items, int n_items, const T* P,
                          const T* slab1, const T* slab2, double* n_sorted, double* et_part,
                          hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  const int grid = ((n_items + 7) / 8) * 8;
  hipLaunchKernelGGL(density_kernel<T>, dim3(grid), dim3(256), 0, st, items, n_items, dv.batches,
                     dv.systems, dv.pts, dv.batch_cols, P, slab1, slab2, n_sorted, et_part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_hs(const DeviceView& dv, const TileItem* items, int n_items, const T* slab1,
                     const T* slab2, double* out, hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  const int grid = ((n_items + 7) / 8) * 8;
  hipLaunchKernelGGL(hs_kernel<T>, dim3(grid), dim3(256), 0, st, items, n_items, dv.batches,
                     dv.systems, dv.batch_cols, slab1, slab2, out);
  return hipGetLastError();
}

hipError_t launch_density_finish(const DeviceView& dv, const double* n_sorted, const double* v,
                                 double* n_out, double* part, int nblk, const double* et_part,
                                 double* sums_out, hipStream_t st) {
  hipLaunchKernelGGL(density_finish_kernel, dim3(nblk, dv.n_sys), dim3(256), 0, st,
                     dv.sys_pt_range, dv.pts, dv.perm, n_sorted, v, n_out, part, nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sums_finish_kernel, dim3(dv.n_sys), dim3(256), 0, st, part, nblk,
                     dv.sys_item_range, et_part, sums_out);
  return hipGetLastError();
}

template hipError_t launch_phi_eval<double>(const DeviceView&, int, int, int, const double*,
                                            double*, double*, hipStream_t);
template hipError_t launch_phi_eval<float>(const DeviceView&, int, int, int, const double*,
                                           float*, float*, hipStream_t);
template hipError_t launch_density<double>(const DeviceView&, const TileItem*, int, const double*,
                                           const double*, const double*, double*, double*,
                                           hipStream_t);
template hipError_t launch_density<float>(const DeviceView&, const TileItem*, int, const float*,
                                          const float*, const float*, double*, double*,
                                          hipStream_t);
template hipError_t launch_hs<double>(const DeviceView&, const TileItem*, int, const double*,
                                      const double*, double*, hipStream_t);
template hipError_t launch_hs<float>(const DeviceView&, const TileItem*, int, const float*,
                                     const float*, double*, hipStream_t);

}  // namespace aims
