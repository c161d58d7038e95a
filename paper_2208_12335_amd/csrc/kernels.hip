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

#include <type_traits>

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

__host__ __device__ __forceinline__ int round_up32(int x) { return (x + 31) & ~31; }

// ------------------------------------------------------------------------------------------
// basis evaluation into slabs
//
// Slab layouts (per batch, inside the group scratch; nbp = n_b rounded up to 32):
//   kLayoutDense   T values, function-major: [row][ldp], points contiguous
//   kLayoutBfFn    bf16 hi/lo splits, function-major: row = [ldp hi | ldp lo]
//   kLayoutBfPt    bf16 hi/lo splits, point-major:    row p = [nbp hi | nbp lo]
// A split is hi = bf16(x), lo = bf16(x - hi), so that hi + lo carries ~16 significant bits.
// ------------------------------------------------------------------------------------------
typedef __bf16 bf16_t;
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

enum { kLayoutDense = 0, kLayoutBfFn = 1, kLayoutBfPt = 2 };

__device__ __forceinline__ void split_bf16(float x, bf16_t& hi, bf16_t& lo) {
  hi = (bf16_t)x;
  lo = (bf16_t)(x - (float)hi);
}

template <typename T, int LAYOUT>
struct SlabStore {
  T* o1;
  T* o2;
  int ldp, nbp;
  __device__ __forceinline__ void operator()(int col, int p, T v1, T v2) const {
    o1[(size_t)col * ldp + p] = v1;
    o2[(size_t)col * ldp + p] = v2;
  }
};
template <>
struct SlabStore<float, kLayoutBfFn> {
  bf16_t* o1;
  bf16_t* o2;
  int ldp, nbp;
  __device__ __forceinline__ void operator()(int col, int p, float v1, float v2) const {
    bf16_t h, l;
    const size_t base = (size_t)col * 2 * ldp + p;
    split_bf16(v1, h, l);
    o1[base] = h;
    o1[base + ldp] = l;
    split_bf16(v2, h, l);
    o2[base] = h;
    o2[base + ldp] = l;
  }
};
template <>
struct SlabStore<float, kLayoutBfPt> {
  bf16_t* o1;
  bf16_t* o2;
  int ldp, nbp;
  __device__ __forceinline__ void operator()(int col, int p, float v1, float v2) const {
    bf16_t h, l;
    const size_t base = (size_t)p * 2 * nbp + col;
    split_bf16(v1, h, l);
    o1[base] = h;
    o1[base + nbp] = l;
    split_bf16(v2, h, l);
    o2[base] = h;
    o2[base + nbp] = l;
  }
};

template <typename T, typename Store>
__device__ __forceinline__ void eval_atom_point(double dx, double dy, double dz,
                                                const SpeciesDesc& sd,
                                                const int32_t* __restrict__ shell_l,
                                                const T* __restrict__ spline,
                                                const RadialGrid& rg, int mode, T w, T wv,
                                                int col0, int p, const Store& store) {
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  if (!(r < rg.rc)) {
    for (int f = 0; f < sd.nfn; ++f) store(col0 + f, p, T(0), T(0));
    return;
  }
  const double rr = fmax(r, 1e-12);
  const double inv = 1.0 / rr;
  const T ux = T(dx * inv), uy = T(dy * inv), uz = T(dz * inv);
  const RadialPos rp = radial_pos(rr, rg);
  const T dt = T(rp.dt);
  const T* c = spline + sd.spline_off + (size_t)rp.k * sd.nshell * 8;
  int f = col0;
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
      store(f + m, p, phi, second);
    }
    f += nm;
  }
}

template <typename T, int LAYOUT>
__global__ void __launch_bounds__(256)
phi_eval_kernel(const BatchDesc* __restrict__ batches, int b0, const double4* __restrict__ pts,
                const int32_t* __restrict__ perm, const int32_t* __restrict__ batch_atoms,
                const int32_t* __restrict__ batch_acol, const double* __restrict__ atom_xyz,
                const int32_t* __restrict__ atom_species, const SpeciesDesc* __restrict__ species,
                const int32_t* __restrict__ shell_l, const T* __restrict__ spline, RadialGrid rg,
                const double* __restrict__ v, int mode, void* __restrict__ slab1,
                void* __restrict__ slab2) {
  const BatchDesc d = batches[b0 + blockIdx.x];
  const int np = d.n_p, na = d.n_atoms, ldp = d.ldp, nbp = round_up32(d.n_b);
  typedef typename std::conditional<LAYOUT == kLayoutDense, T, bf16_t>::type S;
  const int64_t off = (LAYOUT == kLayoutDense ? 1 : 2) * d.slab_off;
  SlabStore<T, LAYOUT> store{(S*)slab1 + off, (S*)slab2 + off, ldp, nbp};
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
                       T(wv), col0, p, store);
  }
  // zero the padding so that the K loops may run over whole padded rows
  if (LAYOUT != kLayoutBfPt) {
    const int padw = ldp - np;
    if (padw > 0) {
      const int tot = d.n_b * padw;
      for (int q = threadIdx.x; q < tot; q += blockDim.x) {
        const int row = q / padw;
        store(row, np + (q - row * padw), T(0), T(0));
      }
    }
  } else {
    // point-major: columns n_b..nbp of every row, and whole rows n_p..ldp
    const int padc = nbp - d.n_b;
    for (int q = threadIdx.x; q < np * padc; q += blockDim.x) {
      const int p = q / padc;
      store(d.n_b + (q - p * padc), p, T(0), T(0));
    }
    for (int q = threadIdx.x; q < (ldp - np) * nbp; q += blockDim.x) {
      const int p = np + q / nbp;
      store(q - (p - np) * nbp, p, T(0), T(0));
    }
  }
}

// ------------------------------------------------------------------------------------------
// tiled MFMA kernels: 256 threads = 4 waves, 64 x 64 output tile, each wave a 32 x 32 quarter
// made of 2 x 2 blocks of 16 x 16 MFMA outputs.  K is staged through LDS in chunks of 16 with
// a two-stage pipeline (global -> registers for chunk c+1 while chunk c is multiplied).
//
// LDS layouts are chosen so that neither the staging stores nor the MFMA fragment reads
// conflict: operands whose K index is contiguous in HBM are kept K-contiguous with an odd row
// stride (kKC + 1), the point-contiguous slab operand of the density kernel is kept
// N-contiguous with a row stride of kTile + 16.
// ------------------------------------------------------------------------------------------
constexpr int kKC = 16;
constexpr int kLdK = kKC + 1;      // K-contiguous rows
constexpr int kLdN = kTile + 16;   // N-contiguous rows

// XCD-aware work order: the dispatcher places workgroup g on XCD g % 8, so consecutive work
// items (tiles of the same batch, which share its slab) are given workgroup ids that differ by
// multiples of 8 and stay in one XCD's L2.
__device__ __forceinline__ int xcd_item(int g, int n) {
  const int per = (n + 7) / 8;
  return (g & 7) * per + (g >> 3);
}

template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ p, T (&v)[4]);
template <>
__device__ __forceinline__ void load4<double>(const double* __restrict__ p, double (&v)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
template <>
__device__ __forceinline__ void load4<float>(const float* __restrict__ p, float (&v)[4]) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// One K chunk of MFMAs.  A fragments from a K-contiguous tile, B fragments from either a
// K-contiguous tile (B_KMAJOR = false: Bs[n][k]) or an N-contiguous tile (Bs[k][n]).
template <typename T, bool B_NCONTIG>
__device__ __forceinline__ void mfma_chunk(const T* __restrict__ As, const T* __restrict__ Bs,
                                           int lane, int wm, int wn,
                                           typename Acc<T>::type (&acc)[2][2]) {
#pragma unroll
  for (int kk = 0; kk < kKC; kk += 4) {
    const int kr = kk + (lane >> 4);
    T a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = As[(wm * 32 + i * 16 + (lane & 15)) * kLdK + kr];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int n = wn * 32 + i * 16 + (lane & 15);
      b[i] = B_NCONTIG ? Bs[kr * kLdN + n] : Bs[n * kLdK + kr];
    }
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

  __shared__ T As[2][kTile * kLdK];   // P_b[j][i], i contiguous
  __shared__ T Bs[2][kKC * kLdN];     // Phi^T[i][p], p contiguous
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

  // staging roles: A row ra (4 consecutive k at 4*sa), B row kb (4 consecutive p at 4*nbq)
  const int ra = tid >> 2, sa = tid & 3;
  const int kb = tid >> 4, nbq = tid & 15;
  const int grow = (j0 + ra < nb) ? cols[j0 + ra] : -1;
  const T* Prow = Pm + (size_t)(grow < 0 ? 0 : grow) * sys.nb;
  const bool bcol_ok = p0 + 4 * nbq < ldp;
  const bool wave_live = (j0 + wm * 32 < nb) && (p0 + wn * 32 < d.n_p);

  T ra_v[4], rb_v[4];
  // column indices of P_b are loaded one chunk ahead of the P values that need them
  int cidx[4];
  auto load_cols = [&](int kc) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k = kc + 4 * sa + c;
      cidx[c] = (k < nb) ? cols[k] : -1;
    }
  };
  auto fetch = [&](int kc) {
#pragma unroll
    for (int c = 0; c < 4; ++c) ra_v[c] = (grow >= 0 && cidx[c] >= 0) ? Prow[cidx[c]] : T(0);
    if (kc + kb < nb && bcol_ok) {
      load4<T>(S1 + (size_t)(kc + kb) * ldp + p0 + 4 * nbq, rb_v);
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) rb_v[c] = T(0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      As[buf][ra * kLdK + 4 * sa + c] = ra_v[c];
      Bs[buf][kb * kLdN + 4 * nbq + c] = rb_v[c];
    }
  };

  const int nchunk = (nb + kKC - 1) / kKC;
  load_cols(0);
  fetch(0);
  stash(0);
  load_cols(kKC);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) {
      fetch((c + 1) * kKC);
      load_cols((c + 2) * kKC);
    }
    if (wave_live) mfma_chunk<T, true>(As[buf], Bs[buf], lane, wm, wn, acc);
    if (c + 1 < nchunk) stash(buf ^ 1);
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

  __shared__ T As[2][kTile * kLdK];   // Phi^T[i][p], p contiguous (K)
  __shared__ T Bs[2][kTile * kLdK];   // second operand [j][p], p contiguous (K)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  typedef typename Acc<T>::type acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = acc_t{0, 0, 0, 0};
  const bool wave_live = (i0 + wm * 32 < nb) && (jb + wn * 32 < nb);

  const int row = tid >> 2, seg = tid & 3;
  const bool a_ok = i0 + row < nb, b_ok = jb + row < nb;
  const T* Ap = slab1 + d.slab_off + (size_t)(a_ok ? i0 + row : 0) * ldp + 4 * seg;
  const T* Bp = slab2 + d.slab_off + (size_t)(b_ok ? jb + row : 0) * ldp + 4 * seg;
  T av[4], bv[4];
  auto fetch = [&](int kc) {
    if (a_ok) load4<T>(Ap + kc, av);
    else for (int c = 0; c < 4; ++c) av[c] = T(0);
    if (b_ok) load4<T>(Bp + kc, bv);
    else for (int c = 0; c < 4; ++c) bv[c] = T(0);
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      As[buf][row * kLdK + 4 * seg + c] = av[c];
      Bs[buf][row * kLdK + 4 * seg + c] = bv[c];
    }
  };
  const int nchunk = ldp / kKC;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) fetch((c + 1) * kKC);
    if (wave_live) mfma_chunk<T, false>(As[buf], Bs[buf], lane, wm, wn, acc);
    if (c + 1 < nchunk) stash(buf ^ 1);
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
// BF16x3 kernels: per-batch contractions as three bf16 MFMA products of hi/lo splits
// (a_hi b_hi + a_hi b_lo + a_lo b_hi, v_mfma_f32_16x16x32_bf16, FP32 accumulation), with the
// same 64 x 64 tiling as above and K staged in chunks of 32 through LDS rows of 32 + 8 bf16.
// ------------------------------------------------------------------------------------------
constexpr int kKB = 32;            // K chunk
constexpr int kLdB = kKB + 8;      // LDS row length (bf16), keeps 16-byte alignment

__device__ __forceinline__ f4_t mfma_bf16(bf16x8_t a, bf16x8_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// A tile rows m (K contiguous), B tile rows n (K contiguous); each a hi and a lo plane.
__device__ __forceinline__ void mfma_chunk_bf16x3(const bf16_t* __restrict__ Ah, const bf16_t* __restrict__ Al,
                                                  const bf16_t* __restrict__ Bh, const bf16_t* __restrict__ Bl,
                                                  int lane, int wm, int wn, f4_t (&acc)[2][2]) {
  const int kq = 8 * (lane >> 4);
  bf16x8_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int ra = (wm * 32 + i * 16 + (lane & 15)) * kLdB + kq;
    const int rb = (wn * 32 + i * 16 + (lane & 15)) * kLdB + kq;
    ah[i] = *reinterpret_cast<const bf16x8_t*>(Ah + ra);
    al[i] = *reinterpret_cast<const bf16x8_t*>(Al + ra);
    bh[i] = *reinterpret_cast<const bf16x8_t*>(Bh + rb);
    bl[i] = *reinterpret_cast<const bf16x8_t*>(Bl + rb);
  }
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
      acc[mi][ni] = mfma_bf16(al[mi], bh[ni], acc[mi][ni]);
      acc[mi][ni] = mfma_bf16(ah[mi], bl[ni], acc[mi][ni]);
      acc[mi][ni] = mfma_bf16(ah[mi], bh[ni], acc[mi][ni]);
    }
}

__device__ __forceinline__ float bf_pair(const bf16_t* p, int lo_off) {
  return (float)p[0] + (float)p[lo_off];
}

// Density: X^T[j][p] = sum_i P_b[j][i] Phi[p][i]; P from the FP32 copy, split while staging;
// Phi (and t Phi) from point-major bf16 slabs.
__global__ void __launch_bounds__(256)
density_kernel_bf16(const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
                    const SystemDesc* __restrict__ systems, const double4* __restrict__ pts,
                    const int32_t* __restrict__ batch_cols, const float* __restrict__ Pmat,
                    const bf16_t* __restrict__ slab1, const bf16_t* __restrict__ slab2,
                    double* __restrict__ n_sorted, double* __restrict__ et_part) {
  const int item = xcd_item(blockIdx.x, n_items);
  if (item >= n_items) return;
  const TileItem it = items[item];
  const BatchDesc d = batches[it.batch];
  const SystemDesc sys = systems[d.sys];
  const int nb = d.n_b, ldp = d.ldp, nbp = round_up32(nb);
  const int j0 = it.ti * kTile, p0 = it.tj * kTile;
  const int* cols = batch_cols + d.col_off;
  const bf16_t* S1 = slab1 + 2 * d.slab_off;
  const bf16_t* S2 = slab2 + 2 * d.slab_off;
  const float* Pm = Pmat + sys.mat_off;

  __shared__ __attribute__((aligned(16))) bf16_t Ah[2][kTile * kLdB], Al[2][kTile * kLdB];
  __shared__ __attribute__((aligned(16))) bf16_t Bh[2][kTile * kLdB], Bl[2][kTile * kLdB];
  __shared__ double red_n[2][kTile];
  __shared__ double red_e[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  f4_t acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = f4_t{0, 0, 0, 0};

  // staging roles: row r = tid / 4 of both tiles, K segment 8 * (tid % 4)
  const int r = tid >> 2, sg = tid & 3;
  const int grow = (j0 + r < nb) ? cols[j0 + r] : -1;
  const float* Prow = Pm + (size_t)(grow < 0 ? 0 : grow) * sys.nb;
  const bool b_ok = p0 + r < ldp;
  const bf16_t* Bsrc1 = S1 + (size_t)(b_ok ? p0 + r : 0) * 2 * nbp + 8 * sg;
  const bool wave_live = (j0 + wm * 32 < nb) && (p0 + wn * 32 < d.n_p);

  int cidx[8];
  float pa[8];
  bf16x8_t bh, bl;
  auto load_cols = [&](int kc) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int k = kc + 8 * sg + c;
      cidx[c] = (k < nb) ? cols[k] : -1;
    }
  };
  auto fetch = [&](int kc) {
#pragma unroll
    for (int c = 0; c < 8; ++c) pa[c] = (grow >= 0 && cidx[c] >= 0) ? Prow[cidx[c]] : 0.f;
    if (b_ok) {
      bh = *reinterpret_cast<const bf16x8_t*>(Bsrc1 + kc);
      bl = *reinterpret_cast<const bf16x8_t*>(Bsrc1 + nbp + kc);
    } else {
      for (int c = 0; c < 8; ++c) { bh[c] = (bf16_t)0.f; bl[c] = (bf16_t)0.f; }
    }
  };
  auto stash = [&](int buf) {
    bf16x8_t h, l;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      bf16_t hh, ll;
      split_bf16(pa[c], hh, ll);
      h[c] = hh;
      l[c] = ll;
    }
    *reinterpret_cast<bf16x8_t*>(&Ah[buf][r * kLdB + 8 * sg]) = h;
    *reinterpret_cast<bf16x8_t*>(&Al[buf][r * kLdB + 8 * sg]) = l;
    *reinterpret_cast<bf16x8_t*>(&Bh[buf][r * kLdB + 8 * sg]) = bh;
    *reinterpret_cast<bf16x8_t*>(&Bl[buf][r * kLdB + 8 * sg]) = bl;
  };

  const int nchunk = (nb + kKB - 1) / kKB;
  load_cols(0);
  fetch(0);
  stash(0);
  load_cols(kKB);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) {
      fetch((c + 1) * kKB);
      load_cols((c + 2) * kKB);
    }
    if (wave_live) mfma_chunk_bf16x3(Ah[buf], Al[buf], Bh[buf], Bl[buf], lane, wm, wn, acc);
    if (c + 1 < nchunk) stash(buf ^ 1);
    __syncthreads();
  }

  double sn[2] = {0.0, 0.0}, se = 0.0;
#pragma unroll
  for (int ni = 0; ni < 2; ++ni) {
    const int p = p0 + wn * 32 + ni * 16 + (lane & 15);
    double accn = 0.0, acce = 0.0;
    if (p < d.n_p) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int j = j0 + wm * 32 + mi * 16 + acc_row<float>(lane, rr);
          if (j < nb) {
            const double x = (double)acc[mi][ni][rr];
            const size_t o = (size_t)p * 2 * nbp + j;
            accn += x * (double)bf_pair(S1 + o, nbp);
            acce += x * (double)bf_pair(S2 + o, nbp);
          }
        }
      acce *= pts[d.pt_off + p].w;
    }
    accn += __shfl_xor(accn, 16);
    accn += __shfl_xor(accn, 32);
    sn[ni] = accn;
    se += acce;
  }
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

// H/S: C[i][j] = sum_p slab1[i][p] slab2[j][p] from function-major bf16 slabs.
__global__ void __launch_bounds__(256)
hs_kernel_bf16(const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
               const SystemDesc* __restrict__ systems, const int32_t* __restrict__ batch_cols,
               const bf16_t* __restrict__ slab1, const bf16_t* __restrict__ slab2,
               double* __restrict__ out) {
  const int item = xcd_item(blockIdx.x, n_items);
  if (item >= n_items) return;
  const TileItem it = items[item];
  const BatchDesc d = batches[it.batch];
  const SystemDesc sys = systems[d.sys];
  const int nb = d.n_b, ldp = d.ldp;
  const int i0 = it.ti * kTile, jb = it.tj * kTile;
  const int* cols = batch_cols + d.col_off;

  __shared__ __attribute__((aligned(16))) bf16_t Ah[2][kTile * kLdB], Al[2][kTile * kLdB];
  __shared__ __attribute__((aligned(16))) bf16_t Bh[2][kTile * kLdB], Bl[2][kTile * kLdB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  f4_t acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = f4_t{0, 0, 0, 0};
  const bool wave_live = (i0 + wm * 32 < nb) && (jb + wn * 32 < nb);

  const int r = tid >> 2, sg = tid & 3;
  const bool a_ok = i0 + r < nb, b_ok = jb + r < nb;
  const bf16_t* Ap = slab1 + 2 * d.slab_off + (size_t)(a_ok ? i0 + r : 0) * 2 * ldp + 8 * sg;
  const bf16_t* Bp = slab2 + 2 * d.slab_off + (size_t)(b_ok ? jb + r : 0) * 2 * ldp + 8 * sg;
  bf16x8_t ah, al, bh, bl;
  auto fetch = [&](int kc) {
    if (a_ok) {
      ah = *reinterpret_cast<const bf16x8_t*>(Ap + kc);
      al = *reinterpret_cast<const bf16x8_t*>(Ap + ldp + kc);
    } else {
      for (int c = 0; c < 8; ++c) { ah[c] = (bf16_t)0.f; al[c] = (bf16_t)0.f; }
    }
    if (b_ok) {
      bh = *reinterpret_cast<const bf16x8_t*>(Bp + kc);
      bl = *reinterpret_cast<const bf16x8_t*>(Bp + ldp + kc);
    } else {
      for (int c = 0; c < 8; ++c) { bh[c] = (bf16_t)0.f; bl[c] = (bf16_t)0.f; }
    }
  };
  auto stash = [&](int buf) {
    *reinterpret_cast<bf16x8_t*>(&Ah[buf][r * kLdB + 8 * sg]) = ah;
    *reinterpret_cast<bf16x8_t*>(&Al[buf][r * kLdB + 8 * sg]) = al;
    *reinterpret_cast<bf16x8_t*>(&Bh[buf][r * kLdB + 8 * sg]) = bh;
    *reinterpret_cast<bf16x8_t*>(&Bl[buf][r * kLdB + 8 * sg]) = bl;
  };
  const int nchunk = ldp / kKB;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) fetch((c + 1) * kKB);
    if (wave_live) mfma_chunk_bf16x3(Ah[buf], Al[buf], Bh[buf], Bl[buf], lane, wm, wn, acc);
    if (c + 1 < nchunk) stash(buf ^ 1);
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
      for (int rr = 0; rr < 4; ++rr) {
        const int i = i0 + wm * 32 + mi * 16 + acc_row<float>(lane, rr);
        if (i < nb) unsafeAtomicAdd(O + (size_t)cols[i] * sys.nb + gj, (double)acc[mi][ni][rr]);
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
  hipLaunchKernelGGL((phi_eval_kernel<T, kLayoutDense>), dim3(nbatch), dim3(256), 0, st, dv.batches,
                     b0, dv.pts, dv.perm, dv.batch_atoms, dv.batch_acol, dv.atom_xyz,
                     dv.atom_species, dv.species, dv.shell_l, spline, dv.rg, v, mode,
                     (void*)slab1, (void*)slab2);
  return hipGetLastError();
}

hipError_t launch_phi_eval_bf16(const DeviceView& dv, int b0, int nbatch, int mode, bool point_major,
                                const double* v, void* slab1, void* slab2, hipStream_t st) {
  if (nbatch == 0) return hipSuccess;
  if (point_major)
    hipLaunchKernelGGL((phi_eval_kernel<float, kLayoutBfPt>), dim3(nbatch), dim3(256), 0, st,
                       dv.batches, b0, dv.pts, dv.perm, dv.batch_atoms, dv.batch_acol, dv.atom_xyz,
                       dv.atom_species, dv.species, dv.shell_l, dv.spline32, dv.rg, v, mode,
                       slab1, slab2);
  else
    hipLaunchKernelGGL((phi_eval_kernel<float, kLayoutBfFn>), dim3(nbatch), dim3(256), 0, st,
                       dv.batches, b0, dv.pts, dv.perm, dv.batch_atoms, dv.batch_acol, dv.atom_xyz,
                       dv.atom_species, dv.species, dv.shell_l, dv.spline32, dv.rg, v, mode,
                       slab1, slab2);
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

hipError_t launch_density_bf16(const DeviceView& dv, const TileItem* items, int n_items, const float* P,
                               const void* slab1, const void* slab2, double* n_sorted, double* et_part,
                               hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  const int grid = ((n_items + 7) / 8) * 8;
  hipLaunchKernelGGL(density_kernel_bf16, dim3(grid), dim3(256), 0, st, items, n_items, dv.batches,
                     dv.systems, dv.pts, dv.batch_cols, P, (const bf16_t*)slab1, (const bf16_t*)slab2,
                     n_sorted, et_part);
  return hipGetLastError();
}

hipError_t launch_hs_bf16(const DeviceView& dv, const TileItem* items, int n_items, const void* slab1,
                          const void* slab2, double* out, hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  const int grid = ((n_items + 7) / 8) * 8;
  hipLaunchKernelGGL(hs_kernel_bf16, dim3(grid), dim3(256), 0, st, items, n_items, dv.batches,
                     dv.systems, dv.batch_cols, (const bf16_t*)slab1, (const bf16_t*)slab2, out);
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
