// gfx950 kernels around the density-matrix step: symmetrisation, column scaling, triangle
// fills, Gershgorin bounds and the trace-correcting purification bookkeeping.  The matrix
// products themselves are plain GEMMs (rocBLAS).
#include <hip/hip_runtime.h>

#include "scf.h"

namespace aims {

namespace {

constexpr int kT32 = 32;       // transpose tile

// out[i][j] = 0.5 (in[i][j] + in[j][i]) through a 32 x 32 LDS tile (coalesced both ways)
__global__ void __launch_bounds__(256) sym_part_kernel(const double* __restrict__ H,
                                                        double* __restrict__ A, int n) {
  __shared__ double tile[kT32][kT32 + 1];
  const int bx = blockIdx.x * kT32, by = blockIdx.y * kT32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;     // 32 x 8
  // tile of H^T at (by, bx): rows bx.., columns by..
  for (int r = ty; r < kT32; r += 8) {
    const int i = bx + r, j = by + tx;
    tile[r][tx] = (i < n && j < n) ? H[(size_t)i * n + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < kT32; r += 8) {
    const int i = by + r, j = bx + tx;
    if (i < n && j < n) A[(size_t)i * n + j] = 0.5 * (H[(size_t)i * n + j] + tile[tx][r]);
  }
}

__global__ void scale_cols_kernel(double* __restrict__ V, const double* __restrict__ s, int m,
                                  int n) {
  const size_t total = (size_t)m * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x)
    V[e] *= s[e / n];
}

// P[j][i] = P[i][j] for i > j in column-major storage (element (i, j) at P[i + j n])
__global__ void __launch_bounds__(256) mirror_lower_kernel(double* __restrict__ P, int n) {
  __shared__ double tile[kT32][kT32 + 1];
  const int bi = blockIdx.x * kT32, bj = blockIdx.y * kT32;   // source block rows bi, cols bj
  if (bi < bj) return;                                        // only blocks on/below the diagonal
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int c = ty; c < kT32; c += 8) {
    const int i = bi + tx, j = bj + c;
    tile[c][tx] = (i < n && j < n) ? P[(size_t)j * n + i] : 0.0;
  }
  __syncthreads();
  // destination (j, i) for source (i, j), i > j: column i, row j
  for (int c = ty; c < kT32; c += 8) {
    const int i = bi + c, j = bj + tx;
    if (i < n && j < n && i > j) P[(size_t)i * n + j] = tile[tx][c];
  }
}

__global__ void zero_upper_kernel(double* __restrict__ L, int n) {
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t j = e / n, i = e - j * n;     // column j, row i
    if (i < j) L[e] = 0.0;
  }
}

template <typename F>
__device__ __forceinline__ double block_reduce(double v, double* sh, F op) {
  for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  v = sh[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = op(v, sh[w]);
  return v;
}

// one workgroup per column (= row, X symmetric): rows[2 i] = X_ii - r_i, rows[2 i + 1] = X_ii + r_i
__global__ void __launch_bounds__(256) gershgorin_rows_kernel(const double* __restrict__ X, int n,
                                                               double* __restrict__ rows) {
  __shared__ double sh[4];
  const int i = blockIdx.x;
  const double* col = X + (size_t)i * n;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x)
    if (j != i) s += fabs(col[j]);
  s = block_reduce(s, sh, [](double a, double b) { return a + b; });
  if (threadIdx.x == 0) {
    rows[2 * i] = col[i] - s;
    rows[2 * i + 1] = col[i] + s;
  }
}

__global__ void __launch_bounds__(256) gershgorin_final_kernel(const double* __restrict__ rows,
                                                                int n, double* __restrict__ out) {
  __shared__ double sh[4];
  double lo = 1e300, hi = -1e300;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    lo = fmin(lo, rows[2 * i]);
    hi = fmax(hi, rows[2 * i + 1]);
  }
  lo = block_reduce(lo, sh, [](double a, double b) { return fmin(a, b); });
  hi = block_reduce(hi, sh, [](double a, double b) { return fmax(a, b); });
  if (threadIdx.x == 0) {
    out[0] = lo;
    out[1] = hi;
  }
}

__global__ void purify_init_kernel(const double* __restrict__ Hp, double* __restrict__ X, int n,
                                   const double* __restrict__ bounds) {
  const double lo = bounds[0], hi = bounds[1];
  const double inv = 1.0 / (hi - lo);
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t j = e / n, i = e - j * n;
    X[e] = ((i == j ? hi : 0.0) - Hp[e]) * inv;
  }
}

__global__ void __launch_bounds__(256) purify_coef_kernel(const double* __restrict__ X, int n,
                                                           double n_occ, double* __restrict__ ab,
                                                           double* __restrict__ hist, int it) {
  __shared__ double sh[4];
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) t += X[(size_t)i * n + i];
  t = block_reduce(t, sh, [](double a, double b) { return a + b; });
  if (threadIdx.x == 0) {
    hist[2 * it] = t;
    const bool square = t > n_occ;
    ab[0] = square ? 1.0 : -1.0;
    ab[1] = square ? 0.0 : 2.0;
  }
}

__global__ void __launch_bounds__(256) frob2_part_kernel(const double* __restrict__ X, size_t total,
                                                          double* __restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x)
    s += X[e] * X[e];
  s = block_reduce(s, sh, [](double a, double b) { return a + b; });
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) frob2_final_kernel(const double* __restrict__ part, int np,
                                                           double* __restrict__ hist, int it) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  s = block_reduce(s, sh, [](double a, double b) { return a + b; });
  if (threadIdx.x == 0) hist[2 * it + 1] = s;
}

inline int grid_1d(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  return (int)(g ? g : 1);
}

}  // namespace

hipError_t launch_sym_part(const double* H, double* A, int n, hipStream_t st) {
  const int t = (n + kT32 - 1) / kT32;
  hipLaunchKernelGGL(sym_part_kernel, dim3(t, t), dim3(256), 0, st, H, A, n);
  return hipGetLastError();
}

hipError_t launch_scale_cols(double* V, const double* s, int m, int n, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_cols_kernel, dim3(grid_1d((size_t)m * n)), dim3(256), 0, st, V, s, m, n);
  return hipGetLastError();
}

hipError_t launch_mirror_lower(double* P, int n, hipStream_t st) {
  const int t = (n + kT32 - 1) / kT32;
  hipLaunchKernelGGL(mirror_lower_kernel, dim3(t, t), dim3(256), 0, st, P, n);
  return hipGetLastError();
}

hipError_t launch_zero_upper(double* L, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_upper_kernel, dim3(grid_1d((size_t)n * n)), dim3(256), 0, st, L, n);
  return hipGetLastError();
}

hipError_t launch_gershgorin(const double* X, int n, double* rows, double* out, hipStream_t st) {
  hipLaunchKernelGGL(gershgorin_rows_kernel, dim3(n), dim3(256), 0, st, X, n, rows);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gershgorin_final_kernel, dim3(1), dim3(256), 0, st, rows, n, out);
  return hipGetLastError();
}

hipError_t launch_purify_init(const double* Hp, double* X, int n, const double* bounds,
                              hipStream_t st) {
  hipLaunchKernelGGL(purify_init_kernel, dim3(grid_1d((size_t)n * n)), dim3(256), 0, st, Hp, X, n,
                     bounds);
  return hipGetLastError();
}

hipError_t launch_purify_coef(const double* X, int n, double n_occ, double* ab, double* hist,
                              int it, hipStream_t st) {
  hipLaunchKernelGGL(purify_coef_kernel, dim3(1), dim3(256), 0, st, X, n, n_occ, ab, hist, it);
  return hipGetLastError();
}

hipError_t launch_frob2(const double* X, int n, double* part, double* hist, int it,
                        hipStream_t st) {
  const size_t total = (size_t)n * n;
  const int g = std::min(256, grid_1d(total));
  hipLaunchKernelGGL(frob2_part_kernel, dim3(g), dim3(256), 0, st, X, total, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(frob2_final_kernel, dim3(1), dim3(256), 0, st, part, g, hist, it);
  return hipGetLastError();
}

}  // namespace aims
