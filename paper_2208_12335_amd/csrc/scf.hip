// gfx950 kernels around the density-matrix step: symmetrisation, column scaling, triangle
// fills, Gershgorin bounds, and the trace-correcting purification: its symmetric products on
// the FP64 matrix cores with the trace and norm bookkeeping fused in.  The other matrix products
// of the step (Cholesky factor, inverse, congruence transforms) are rocSOLVER / rocBLAS calls.
#include <hip/hip_runtime.h>

#include "scf.h"
#include "tiles.h"

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

// X = (emax I - (Hp + Hp^T) / 2) / (emax - emin) on the leading n x n block of the ld x ld X
// (column-major), zero outside it; the symmetric part makes X exactly symmetric
__global__ void purify_init_kernel(const double* __restrict__ Hp, double* __restrict__ X, int n,
                                   int ld, const double* __restrict__ bounds) {
  const double lo = bounds[0], hi = bounds[1];
  const double inv = 1.0 / (hi - lo);
  const size_t total = (size_t)ld * ld;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / ld), i = (int)(e - (size_t)j * ld);
    double x = 0.0;
    if (i < n && j < n) {
      const double h = 0.5 * (Hp[(size_t)j * n + i] + Hp[(size_t)i * n + j]);
      x = ((i == j ? hi : 0.0) - h) * inv;
    }
    X[e] = x;
  }
}

// ------------------------------------------------------------------------------------------
// Purification products on the FP64 matrix cores.
//
// X is symmetric, column-major with leading dimension ld (a multiple of 64) and zero outside
// its n x n block.  Because X is symmetric, (X X)_ij is the dot product of columns i and j, so
// both MFMA operands are read along contiguous columns.  Only the 64 x 64 tiles on and below
// the diagonal are computed; each writes itself and its mirror image, so every output is
// exactly symmetric and the pad stays zero.  Each tile also leaves its share of tr Y and
// ||Y||_F^2, which the next product sums (in one fixed order in every workgroup) to choose its
// own coefficients: no host round trip and no atomics, so the iteration is deterministic.
// ------------------------------------------------------------------------------------------
constexpr int kPT = 64;       // output tile (4 waves of 32 x 32)

// lower-triangle tile b (row-major over the triangle) -> (ti, tj), tj <= ti
__device__ __forceinline__ void tri_tile(int b, int& ti, int& tj) {
  int i = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= b) ++i;
  while (i * (i + 1) / 2 > b) --i;
  ti = i;
  tj = b - i * (i + 1) / 2;
}

__device__ __forceinline__ double dsum(double a, double b) { return a + b; }

// per-tile shares of tr X and ||X||_F^2 for the starting matrix (the products leave their own)
__global__ void __launch_bounds__(256) purify_partials_kernel(const double* __restrict__ X, int ld,
                                                               double* __restrict__ part,
                                                               double* __restrict__ state) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  if (b == 0 && threadIdx.x == 0) {
    state[0] = -1.0;             // first product whose input was idempotent to the tolerance
    state[1] = -1.0;             // products done once converged
  }
  int ti, tj;
  tri_tile(b, ti, tj);
  const double w = ti == tj ? 1.0 : 2.0;       // an off-diagonal tile stands for its mirror too
  double t = 0.0, f = 0.0;
  for (int e = threadIdx.x; e < kPT * kPT; e += blockDim.x) {
    const int c = e / kPT, r = e % kPT;
    const int i = ti * kPT + r, j = tj * kPT + c;
    const double x = X[(size_t)j * ld + i];
    f += w * x * x;
    if (i == j) t += x;
  }
  t = block_reduce(t, sh, dsum);
  f = block_reduce(f, sh, dsum);
  if (threadIdx.x == 0) {
    part[2 * b] = t;
    part[2 * b + 1] = f;
  }
}

typedef double d2_t __attribute__((ext_vector_type(2)));
typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kPK = 32;            // k per main-loop chunk
constexpr int kPS = kPK + 2;       // doubles per staged column (the pad spreads the LDS banks)

// tr X and ||X||_F^2 from the n_tiles shares, summed in one fixed order in every workgroup
__device__ __forceinline__ void purify_totals(const double* __restrict__ part, int n_tiles,
                                              double* sh, double& t, double& f) {
  t = 0.0;
  f = 0.0;
  for (int k = threadIdx.x; k < n_tiles; k += blockDim.x) {
    t += part[2 * k];
    f += part[2 * k + 1];
  }
  t = block_reduce(t, sh, dsum);
  f = block_reduce(f, sh, dsum);
}

// The convergence rule on the device.  state[0] is the first product whose input X had
// |tr X - ||X||_F^2| < tol, state[1] the number of products once converged (else negative).
// The input of product it is final when it >= state[0] + 3 (quadratic convergence needs a few
// more products after the error is small); that product and all later ones do nothing.  Every
// workgroup reaches the same decision: state[0] can change during a launch only to it (which
// leaves it < state[0] + 3), and state[1] only in a launch where every workgroup is done.
__device__ __forceinline__ bool purify_done(const double* __restrict__ state, int it) {
  const double small_at = state[0];
  return state[1] >= 0.0 || (small_at >= 0.0 && it >= small_at + 3.0);
}

// Chunks [ch0, ch1) of K of the tile (ti, tj) by one workgroup: the 64 columns at I0 = 64 ti
// and at J0 = 64 tj are staged through LDS, [column][k] (32 k per chunk), double buffered, the
// next chunk's global loads in flight during this chunk's products.  Each staging load moves a
// whole 128-byte line segment of one column.  Wave (wm, wn) accumulates the 32 x 32 quadrant at
// rows I0 + 32 wm, columns J0 + 32 wn; the operand lane (c, q) holds column c at
// k = 8 h + 2 q + e of the chunk (the same k order for A and B).
__device__ __forceinline__ void purify_tile_k(const double* __restrict__ X, int ld, int ti, int tj,
                                              int ch0, int ch1, bool active,
                                              double (*lds)[2][64 * kPS], d4_t (&acc)[2][2]) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int scol = t >> 3, spc = t & 7;
  const double* ga = X + (size_t)(ti * kPT + scol) * ld + 2 * spc;
  const double* gb = X + (size_t)(tj * kPT + scol) * ld + 2 * spc;
  d2_t st[2][2][2];                              // [panel][column half][k half]
  auto gload = [&](int ch) {
    const int k = ch * kPK;
    for (int i = 0; i < 2; ++i)
      for (int h = 0; h < 2; ++h) {
        st[0][i][h] = *reinterpret_cast<const d2_t*>(ga + (size_t)32 * i * ld + k + 16 * h);
        st[1][i][h] = *reinterpret_cast<const d2_t*>(gb + (size_t)32 * i * ld + k + 16 * h);
      }
  };
  auto sstore = [&](int buf) {
    for (int pn = 0; pn < 2; ++pn)
      for (int i = 0; i < 2; ++i)
        for (int h = 0; h < 2; ++h)
          *reinterpret_cast<d2_t*>(&lds[buf][pn][(scol + 32 * i) * kPS + 2 * spc + 16 * h]) =
              st[pn][i][h];
  };
  const int wm = wave >> 1, wn = wave & 1, c = lane & 15, q = lane >> 4;
  gload(ch0);
  sstore(0);
  __syncthreads();
  for (int ch = ch0; ch < ch1; ++ch) {
    const int buf = (ch - ch0) & 1;
    gload(ch + 1 < ch1 ? ch + 1 : ch);           // the last reload is in bounds and unused
    if (active) {
      const double* la = &lds[buf][0][(32 * wm + c) * kPS + 2 * q];
      const double* lb = &lds[buf][1][(32 * wn + c) * kPS + 2 * q];
      for (int h = 0; h < 4; ++h) {
        const d2_t a0 = *reinterpret_cast<const d2_t*>(la + 8 * h);
        const d2_t a1 = *reinterpret_cast<const d2_t*>(la + 16 * kPS + 8 * h);
        const d2_t b0 = *reinterpret_cast<const d2_t*>(lb + 8 * h);
        const d2_t b1 = *reinterpret_cast<const d2_t*>(lb + 16 * kPS + 8 * h);
        for (int e = 0; e < 2; ++e) {
          acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[e], b0[e], acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[e], b1[e], acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[e], b0[e], acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[e], b1[e], acc[1][1], 0, 0, 0);
        }
      }
    }
    sstore(buf ^ 1);
    __syncthreads();
  }
}

// Y = ca acc + cb X on the quadrant, written with its mirror; the shares of tr Y and ||Y||_F^2
// (weight 2 off the diagonal, where the mirror is not computed) reduced over the workgroup.
// Output (row, col) of block (mi, ni) in accumulator r of a lane: row I + 16 mi + 4 r + q,
// column J + 16 ni + c.
__device__ __forceinline__ void purify_epilogue(const double* __restrict__ X,
                                                double* __restrict__ Y, int ld, int ti, int tj,
                                                bool square, const d4_t (&acc)[2][2], double* sh,
                                                double* __restrict__ share) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, c = lane & 15, q = lane >> 4;
  const int I = ti * kPT + 32 * (wave >> 1), J = tj * kPT + 32 * (wave & 1);
  const double ca = square ? 1.0 : -1.0, cb = square ? 0.0 : 2.0;
  double tr = 0.0, fr = 0.0;
  if (I >= J) {
    const bool diag = I == J;
    const double w = diag ? 1.0 : 2.0;
    for (int mi = 0; mi < 2; ++mi)
      for (int ni = 0; ni < 2; ++ni)
        for (int r = 0; r < 4; ++r) {
          const int i = I + 16 * mi + 4 * r + q, j = J + 16 * ni + c;
          double y = ca * acc[mi][ni][r];
          if (!square) y = fma(cb, X[(size_t)j * ld + i], y);
          Y[(size_t)j * ld + i] = y;
          if (!diag) Y[(size_t)i * ld + j] = y;
          fr += w * y * y;
          if (i == j) tr += y;
        }
  }
  tr = block_reduce(tr, sh, dsum);
  fr = block_reduce(fr, sh, dsum);
  if (threadIdx.x == 0) {
    share[0] = tr;
    share[1] = fr;
  }
}

// Y = X^2 if tr X > n_occ, else Y = 2 X - X^2.
// Work units: tiles [0, n_full) whole (epilogue included), then ks K parts of each of the r
// remaining tiles, whose partial sums go to W[unit - n_full] for purify_fixup_kernel.  With split
// tiles n_full is a multiple of 8, so both ranges keep the XCD-aware order.  hist[2 it], hist[2 it + 1] = tr X
// and ||X||_F^2 from workgroup 0; the shares of Y go to part_out[2 tile].
__global__ void __launch_bounds__(256) purify_step_kernel(const double* __restrict__ X,
                                                           double* __restrict__ Y, int ld,
                                                           double n_occ,
                                                           const double* __restrict__ part_in,
                                                           double* __restrict__ part_out,
                                                           int n_tiles, int n_full, int ks,
                                                           double* __restrict__ W,
                                                           double* __restrict__ hist, int it,
                                                           double tol,
                                                           double* __restrict__ state) {
  __shared__ __attribute__((aligned(16))) double lds[2][2][64 * kPS];
  __shared__ double sh[4];
  double t, f;
  purify_totals(part_in, n_tiles, sh, t, f);
  const bool done = purify_done(state, it);
  __syncthreads();                     // every thread has read the state before workgroup 0 writes
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hist[2 * it] = t;
    hist[2 * it + 1] = f;
    if (done) {
      if (state[1] < 0.0) state[1] = it;
    } else if (state[0] < 0.0 && fabs(t - f) < tol) {
      state[0] = it;
    }
  }
  if (done) return;
  const int g = blockIdx.x;
  const bool whole = g < n_full;
  int tile, u = 0, kp = 0;
  if (whole) {
    tile = xcd_item_exact(g, n_full);
  } else {
    u = xcd_item_exact(g - n_full, (n_tiles - n_full) * ks);
    tile = n_full + u / ks;
    kp = u - (u / ks) * ks;
  }
  int ti, tj;
  tri_tile(tile, ti, tj);
  const int wave = threadIdx.x >> 6;
  const bool active = ti * kPT + 32 * (wave >> 1) >= tj * kPT + 32 * (wave & 1);
  d4_t acc[2][2];
  for (int mi = 0; mi < 2; ++mi)
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = d4_t{0.0, 0.0, 0.0, 0.0};
  const int nch = ld / kPK;
  if (whole) {
    purify_tile_k(X, ld, ti, tj, 0, nch, active, lds, acc);
    purify_epilogue(X, Y, ld, ti, tj, t > n_occ, acc, sh, part_out + 2 * tile);
  } else {
    purify_tile_k(X, ld, ti, tj, kp * nch / ks, (kp + 1) * nch / ks, active, lds, acc);
    // partial sums: slot (mi, ni, r) of thread x at W[(unit 16 + slot) 256 + x]
    double* w = W + (size_t)u * 16 * 256 + threadIdx.x;
    if (active)
      for (int mi = 0; mi < 2; ++mi)
        for (int ni = 0; ni < 2; ++ni)
          for (int r = 0; r < 4; ++r) w[(mi * 8 + ni * 4 + r) * 256] = acc[mi][ni][r];
  }
}

// The split tiles: sum of the ks partial sums in part order, then the epilogue.  One workgroup
// per tile n_full + blockIdx.x.
__global__ void __launch_bounds__(256) purify_fixup_kernel(const double* __restrict__ X,
                                                            double* __restrict__ Y, int ld,
                                                            double n_occ,
                                                            const double* __restrict__ part_in,
                                                            double* __restrict__ part_out,
                                                            int n_tiles, int n_full, int ks,
                                                            const double* __restrict__ W, int it,
                                                            const double* __restrict__ state) {
  __shared__ double sh[4];
  double t, f;
  purify_totals(part_in, n_tiles, sh, t, f);
  if (purify_done(state, it)) return;
  const int tile = n_full + blockIdx.x;
  int ti, tj;
  tri_tile(tile, ti, tj);
  d4_t acc[2][2];
  for (int mi = 0; mi < 2; ++mi)
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = d4_t{0.0, 0.0, 0.0, 0.0};
  const int wave = threadIdx.x >> 6;
  if (ti * kPT + 32 * (wave >> 1) >= tj * kPT + 32 * (wave & 1)) {
    const double* w = W + (size_t)blockIdx.x * ks * 16 * 256 + threadIdx.x;
    for (int k = 0; k < ks; ++k)
      for (int mi = 0; mi < 2; ++mi)
        for (int ni = 0; ni < 2; ++ni)
          for (int r = 0; r < 4; ++r)
            acc[mi][ni][r] += w[((size_t)k * 16 + mi * 8 + ni * 4 + r) * 256];
  }
  purify_epilogue(X, Y, ld, ti, tj, t > n_occ, acc, sh, part_out + 2 * tile);
}

// *flag != 0 when a and b differ in any bit
__global__ void __launch_bounds__(256) differ_kernel(const unsigned long long* __restrict__ a,
                                                      const unsigned long long* __restrict__ b,
                                                      size_t n, int* __restrict__ flag) {
  int d = 0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    d |= a[e] != b[e];
  if (__any(d) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// Largest |P_ij - P_ji| and |P_ij| of one block.  Non-negative doubles order like their bit
// patterns, so the maxima are taken with integer atomics on those; an entry that is not finite
// makes the first one +inf.
__global__ void __launch_bounds__(256) asym_max_kernel(const double* __restrict__ P, int n,
                                                        unsigned long long* __restrict__ out) {
  double a = 0.0, m = 0.0;
  const size_t nn = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nn;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / n, j = e - i * n;
    const double x = P[e];
    if (!isfinite(x)) a = INFINITY;
    else a = fmax(a, fabs(x - P[j * n + i]));
    m = fmax(m, fabs(x));
  }
  for (int o = 32; o > 0; o >>= 1) {
    a = fmax(a, __shfl_xor(a, o));
    m = fmax(m, __shfl_xor(m, o));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out, (unsigned long long)__double_as_longlong(a));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(m));
  }
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

hipError_t launch_purify_init(const double* Hp, double* X, int n, int ld, const double* bounds,
                              hipStream_t st) {
  hipLaunchKernelGGL(purify_init_kernel, dim3(grid_1d((size_t)ld * ld)), dim3(256), 0, st, Hp, X, n,
                     ld, bounds);
  return hipGetLastError();
}

int purify_tiles(int ld) {
  const int t = ld / kPT;
  return t * (t + 1) / 2;
}

hipError_t launch_purify_partials(const double* X, int ld, double* part, double* state,
                                  hipStream_t st) {
  hipLaunchKernelGGL(purify_partials_kernel, dim3(purify_tiles(ld)), dim3(256), 0, st, X, ld, part,
                     state);
  return hipGetLastError();
}

hipError_t launch_asym_max(const double* P, int n, unsigned long long* out, hipStream_t st) {
  hipError_t e = hipMemsetAsync(out, 0, 2 * sizeof(unsigned long long), st);
  if (e != hipSuccess || n <= 0) return e;
  hipLaunchKernelGGL(asym_max_kernel, dim3(grid_1d((size_t)n * n)), dim3(256), 0, st, P, n, out);
  return hipGetLastError();
}

hipError_t launch_differ(const double* a, const double* b, size_t n, int* flag, hipStream_t st) {
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), st);
  if (e != hipSuccess || n == 0) return e;
  hipLaunchKernelGGL(differ_kernel, dim3(grid_1d(n)), dim3(256), 0, st,
                     reinterpret_cast<const unsigned long long*>(a),
                     reinterpret_cast<const unsigned long long*>(b), n, flag);
  return hipGetLastError();
}

PurifyPlan purify_plan(int ld, int cus) {
  PurifyPlan p;
  p.tiles = purify_tiles(ld);
  const int nch = ld / kPK;
  // whole tiles fill the compute units a whole number of times; the r left over are split in K
  // across all of them (at least two chunks per part), unless that would give under two parts
  const int c = cus / 8 * 8 > 8 ? cus / 8 * 8 : 8;
  p.n_full = p.tiles / c * c;
  const int r = p.tiles - p.n_full;
  p.ks = r > 0 ? c / r : 1;
  if (p.ks > nch / 2) p.ks = nch / 2;
  if (p.ks < 2) {
    p.n_full = p.tiles;
    p.ks = 1;
  }
  return p;
}

hipError_t launch_purify_step(const double* X, double* Y, int ld, double n_occ,
                              const double* part_in, double* part_out, const PurifyPlan& p,
                              double* W, double* hist, int it, double tol, double* state,
                              hipStream_t st) {
  const int r = p.tiles - p.n_full;
  if (r < 0 || (r > 0 && (p.n_full % 8 != 0 || p.ks < 2 || p.ks > ld / kPK)))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(purify_step_kernel, dim3(p.n_full + r * p.ks), dim3(256), 0, st, X, Y, ld,
                     n_occ, part_in, part_out, p.tiles, p.n_full, p.ks, W, hist, it, tol, state);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || r == 0) return e;
  hipLaunchKernelGGL(purify_fixup_kernel, dim3(r), dim3(256), 0, st, X, Y, ld, n_occ, part_in,
                     part_out, p.tiles, p.n_full, p.ks, W, it, state);
  return hipGetLastError();
}

}  // namespace aims
