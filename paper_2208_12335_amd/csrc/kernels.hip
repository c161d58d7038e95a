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
//   pulay_kernel      backward: per (point, relevant atom), gradients of phi and t phi
//                     contracted with X = Phi P_b and Y = (t Phi) P_b (both from the density
//                     kernel in store mode) into the Pulay-type dE/dR_a
//   dv_kernel         backward: dE/dv_p = gE w_p n_p in caller order
//
// Precision policies: FP64 (double slabs, v_mfma_f64_16x16x4f64), FP32 (float slabs,
// v_mfma_f32_16x16x4f32), BF16x3 (bf16 hi/lo splits of FP32 values, three
// v_mfma_f32_16x16x32_bf16 products).  Per-tile accumulation is in the MFMA's type; everything
// that crosses batches (n, H, S, N, E) is accumulated in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>
#include <type_traits>

#include "aims_internal.h"
#include "basis.h"
#include "kernels.h"
#include "tiles.h"

namespace aims {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16_t;
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

template <typename T> struct Acc;
template <> struct Acc<double> { typedef d4_t type; };
template <> struct Acc<float> { typedef f4_t type; };

__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma16(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_bf16(bf16x8_t a, bf16x8_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
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
//
// Slab layouts (per batch, inside the group scratch, n_b rows of ldp points):
//   kLayoutDense   T values, function-major: [row][ldp], points contiguous
//   kLayoutBfFn    bf16 hi/lo splits, function-major: row = [ldp hi | ldp lo]
// A split is hi = bf16(x), lo = bf16(x - hi), so that hi + lo carries ~16 significant bits.
// ------------------------------------------------------------------------------------------
enum { kLayoutDense = 0, kLayoutBfFn = 1 };

__device__ __forceinline__ void split_bf16(float x, bf16_t& hi, bf16_t& lo) {
  hi = (bf16_t)x;
  lo = (bf16_t)(x - (float)hi);
}

template <typename T, int LAYOUT>
struct SlabStore {
  T* o1;
  T* o2;
  int ldp;
  __device__ __forceinline__ void operator()(int col, int p, T v1, T v2) const {
    o1[(size_t)col * ldp + p] = v1;
    o2[(size_t)col * ldp + p] = v2;
  }
};
template <>
struct SlabStore<float, kLayoutBfFn> {
  bf16_t* o1;
  bf16_t* o2;
  int ldp;
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

// One shell of angular momentum L (compile-time, so only that harmonic's registers are live).
template <typename T, int L, typename Store>
__device__ __forceinline__ void eval_shell(const T* __restrict__ c, T dt, T ux, T uy, T uz, int mode,
                                           T w, T wv, int f, int p, const Store& store) {
  const T R = cubic(c, dt);
  const T K = cubic(c + 4, dt);
  T Y[7];
  ylm_l<T>(L, ux, uy, uz, Y);
#pragma unroll
  for (int m = 0; m < 2 * L + 1; ++m) {
    const T phi = R * Y[m];
    const T tphi = K * Y[m];
    T second;
    if (mode == kModeDensity) second = tphi;
    else if (mode == kModeH) second = wv * phi + w * tphi;
    else second = w * phi;
    store(f + m, p, phi, second);
  }
}

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
    const int l = shell_l[sd.shell_l_off + j];
    switch (l) {
      case 0: eval_shell<T, 0>(c + j * 8, dt, ux, uy, uz, mode, w, wv, f, p, store); break;
      case 1: eval_shell<T, 1>(c + j * 8, dt, ux, uy, uz, mode, w, wv, f, p, store); break;
      case 2: eval_shell<T, 2>(c + j * 8, dt, ux, uy, uz, mode, w, wv, f, p, store); break;
      default: eval_shell<T, 3>(c + j * 8, dt, ux, uy, uz, mode, w, wv, f, p, store); break;
    }
    f += 2 * l + 1;
  }
}

// Basis values of one batch: kPhiSlices workgroups of four waves per batch; workgroup s takes
// the batch's relevant atoms s, s + kPhiSlices, ...  Its waves take (atom, 64-point chunk)
// pairs in turn, chunk-minor, so every wave has work whatever the batch's point count (a
// 128-point batch keeps all four waves on two atoms) and the waves that share an atom write
// its slab rows together, in one burst per row.  The atom is wave-uniform, so the species,
// shell and table addressing is scalar; lanes past the batch's points write the zero padding
// of the atom's rows.
constexpr int kPhiSlices = 4;

template <typename T, int LAYOUT>
__global__ void __launch_bounds__(256)
phi_eval_kernel(const BatchDesc* __restrict__ batches, int b0, const double4* __restrict__ pts,
                const int32_t* __restrict__ perm, const int32_t* __restrict__ batch_atoms,
                const int32_t* __restrict__ batch_acol, const double* __restrict__ atom_xyz,
                const int32_t* __restrict__ atom_species, const SpeciesDesc* __restrict__ species,
                const int32_t* __restrict__ shell_l, const T* __restrict__ spline, RadialGrid rg,
                const double* __restrict__ v, int mode, void* __restrict__ slab1,
                void* __restrict__ slab2) {
  const int bi = blockIdx.x / kPhiSlices;
  const int slice = (int)(blockIdx.x % kPhiSlices);
  const int wq = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const BatchDesc d = batches[b0 + bi];
  const int np = d.n_p, na = d.n_atoms, ldp = d.ldp;
  typedef typename std::conditional<LAYOUT == kLayoutDense, T, bf16_t>::type S;
  const int64_t off = (LAYOUT == kLayoutDense ? 1 : 2) * d.slab_off;
  SlabStore<T, LAYOUT> store{(S*)slab1 + off, (S*)slab2 + off, ldp};
  const int nc = (ldp + 63) / 64;                               // 64-point chunks per row
  const int nk = (na - slice + kPhiSlices - 1) / kPhiSlices;    // this workgroup's atoms
  for (int q = wq; q < nk * nc; q += 4) {
    const int j = q / nc, c = q - j * nc;
    const int k = slice + j * kPhiSlices;
    const int atom = batch_atoms[d.atom_off + k];
    const int col0 = batch_acol[d.atom_off + k];
    const SpeciesDesc sd = species[atom_species[atom]];
    const double ax = atom_xyz[3 * atom], ay = atom_xyz[3 * atom + 1], az = atom_xyz[3 * atom + 2];
    const int p = 64 * c + lane;
    if (p < ldp) {
      if (p < np) {
        const double4 P4 = pts[d.pt_off + p];
        double wv = 0.0;
        if (mode == kModeH) wv = P4.w * v[perm[d.pt_off + p]];
        eval_atom_point<T>(P4.x - ax, P4.y - ay, P4.z - az, sd, shell_l, spline, rg, mode,
                           T(P4.w), T(wv), col0, p, store);
      } else {
        for (int f = 0; f < sd.nfn; ++f) store(col0 + f, p, T(0), T(0));
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Tiled MFMA kernels: 256 threads = 4 waves in a 2 (rows) x 2 (columns) arrangement.  Each
// wave owns 2 x NBN blocks of 16 x 16 outputs; blocks that lie wholly beyond the batch's rows
// or points are skipped (a wave-uniform branch).  K is staged through LDS with a two-stage
// pipeline (global -> registers for chunk c+1 while chunk c is multiplied; two chunks ahead in
// the FP64 density kernel with 64-point tiles), one barrier per chunk.
//
// LDS layouts avoid bank conflicts on both the staging stores and the MFMA fragment reads:
// operands whose K index is contiguous in HBM stay K-contiguous with an odd row stride
// (kKC + 1); the point-contiguous slab operand of the density kernel stays N-contiguous with a
// row stride of (tile width + 16).  The BF16 kernels keep every operand K-contiguous in rows
// of 32 + 8 bf16 (16-byte aligned for 128-bit fragment reads).
// ------------------------------------------------------------------------------------------
constexpr int kKC = 16;            // K chunk of the FP64/FP32 kernels
constexpr int kLdK = kKC + 1;      // K-contiguous LDS rows
constexpr int kKB = 32;            // K chunk of the BF16 kernels
constexpr int kLdB = kKB + 8;      // their LDS rows (bf16)

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

// Epilogue of the density kernels: given per-lane column sums sn[ni] (over the lane's rows)
// and the lane's energy partial se, reduce over the tile's rows and add into n (FP64 atomics,
// one per point and tile) and into the batch's E_T partial.
template <int NBN>
__device__ __forceinline__ void density_epilogue(double (&sn)[NBN], double (&sd)[NBN], double se,
                                                 int lane, int wave, int wm, int wn, int p0, int n_p,
                                                 int pt_off, double (*red_n)[32 * NBN],
                                                 double (*red_d)[32 * NBN], double* red_e,
                                                 double* __restrict__ n_sorted,
                                                 double* __restrict__ d_sorted,
                                                 double* __restrict__ et_batch, int batch) {
  constexpr int PT = 32 * NBN;
#pragma unroll
  for (int ni = 0; ni < NBN; ++ni) {
    sn[ni] += __shfl_xor(sn[ni], 16);
    sn[ni] += __shfl_xor(sn[ni], 32);
    if (d_sorted) {
      sd[ni] += __shfl_xor(sd[ni], 16);
      sd[ni] += __shfl_xor(sd[ni], 32);
    }
  }
  for (int off = 32; off > 0; off >>= 1) se += __shfl_xor(se, off);
  if (lane < 16) {
#pragma unroll
    for (int ni = 0; ni < NBN; ++ni) {
      red_n[wm][wn * 16 * NBN + ni * 16 + lane] = sn[ni];
      if (d_sorted) red_d[wm][wn * 16 * NBN + ni * 16 + lane] = sd[ni];
    }
  }
  if (lane == 0) red_e[wave] = se;
  __syncthreads();
  for (int t = threadIdx.x; t < PT; t += blockDim.x) {
    const int p = p0 + t;
    if (p < n_p) {
      unsafeAtomicAdd(n_sorted + pt_off + p, red_n[0][t] + red_n[1][t]);
      if (d_sorted) unsafeAtomicAdd(d_sorted + pt_off + p, red_d[0][t] + red_d[1][t]);
    }
  }
  if (threadIdx.x == 0)
    unsafeAtomicAdd(et_batch + batch, (red_e[0] + red_e[1]) + (red_e[2] + red_e[3]));
}

// Density, FP64 / FP32: X^T[j][p] = sum_i P_b[j][i] Phi^T[i][p] for 64 basis rows j and
// 32 * NBN points p of one batch.
template <typename T, int NBN>
__device__ __forceinline__ void
density_tile(int item, const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
               const SystemDesc* __restrict__ systems, const double4* __restrict__ pts,
               const int32_t* __restrict__ batch_cols, const T* __restrict__ Pmat,
               const T* __restrict__ slab1, const T* __restrict__ slab2,
               double* __restrict__ n_sorted, double* __restrict__ et_batch,
               T* __restrict__ xout, double* __restrict__ d_sorted) {
  constexpr int PT = 32 * NBN;          // points per tile
  constexpr int LDN = PT + 16;          // N-contiguous LDS rows
  constexpr int BW = PT / 4;            // 4-element units per B row
  constexpr int BU = kKC * BW;          // units of the B tile
  constexpr int BQ = (BU + 255) / 256;  // units per thread
  const TileItem it = items[item];
  const BatchDesc d = batches[it.batch];
  const SystemDesc sys = systems[d.sys];
  const int nb = d.n_b, ldp = d.ldp;
  const int j0 = it.ti * kTile;       // rows of X^T: basis functions
  const int p0 = it.tj * PT;          // columns: points
  const int* cols = batch_cols + d.col_off;
  const T* S1 = slab1 + d.slab_off;
  const T* S2 = slab2 + d.slab_off;
  const T* Pm = Pmat + sys.mat_off;

  __shared__ T As[2][kTile * kLdK];   // P_b[j][i], i contiguous
  __shared__ T Bs[2][kKC * LDN];      // Phi^T[i][p], p contiguous
  __shared__ double red_n[2][PT];
  __shared__ double red_d[2][PT];
  __shared__ double red_e[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int mrows = nb - (j0 + wm * 32);           // block mi is live if 16 mi < mrows
  const int ncols = d.n_p - (p0 + wn * 16 * NBN);  // block ni is live if 16 ni < ncols
  typedef typename Acc<T>::type acc_t;
  acc_t acc[2][NBN];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < NBN; ++ni) acc[mi][ni] = acc_t{0, 0, 0, 0};

  // A staging: thread (kk = tid % 16, rr = tid / 16) stages P_b[j0 + rr + 16 c][kc + kk] for
  // c = 0..3, so that the 16 lanes of one row read consecutive basis columns (one or two cache
  // lines per row and instruction).
  //
  // FP64 with 64-point tiles: a two-deep register pipeline.  Chunk m is loaded into register
  // set m & 1 two chunks before it is stashed, so its loads stay in flight across two
  // multiplies.  Its column index (ci[m & 1]) is loaded before the data loads of chunk m - 1:
  // memory loads retire in issue order, so waiting for an index never waits for the newer
  // chunk's data.  The fragments are read in two halves, which frees the registers of the
  // second set.  Other forms (FP32, FP64 with wider point tiles) have no registers to spare for
  // a second set: one set, loaded one chunk ahead.
  const int kk = tid & 15, rr = tid >> 4;
  uint32_t prow[4];                 // row offsets into the system's P (n_basis <= 65535)
  bool rok[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = j0 + rr + 16 * c;
    rok[c] = j < nb;
    prow[c] = (uint32_t)cols[rok[c] ? j : 0] * (uint32_t)sys.nb;
  }
  int ci[2];
  bool kv[2];
  T av[2][4], bv[2][BQ][4];
  bool aok[2][4], bok[2][BQ];
  auto load_cols = [&](auto S, int kc) {   // unconditional load of a clamped index (no branch)
    constexpr int s = decltype(S)::value;
    const int k = kc + kk;
    kv[s] = k < nb;
    ci[s] = cols[k < nb ? k : nb - 1];
  };
  // loads are issued unconditionally from clamped addresses (no branch, so they stay in flight
  // across the multiplies); invalid elements are zeroed when stashed
  auto fetch = [&](auto S, int kc) {
    constexpr int s = decltype(S)::value;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      aok[s][c] = rok[c] && kv[s];
      av[s][c] = Pm[prow[c] + (uint32_t)ci[s]];
    }
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
      const int u = tid + 256 * q;
      const int k = u / BW, n4 = u - k * BW;
      bok[s][q] = u < BU && kc + k < nb && p0 + 4 * n4 < ldp;
      load4<T>(S1 + (bok[s][q] ? (size_t)(kc + k) * ldp + p0 + 4 * n4 : 0), bv[s][q]);
    }
  };
  auto stash = [&](auto S, int buf) {
    constexpr int s = decltype(S)::value;
#pragma unroll
    for (int c = 0; c < 4; ++c) As[buf][(rr + 16 * c) * kLdK + kk] = aok[s][c] ? av[s][c] : T(0);
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
      const int u = tid + 256 * q;
      if (u < BU) {
        const int k = u / BW, n4 = u - k * BW;
#pragma unroll
        for (int c = 0; c < 4; ++c) Bs[buf][k * LDN + 4 * n4 + c] = bok[s][q] ? bv[s][q][c] : T(0);
      }
    }
  };
  const bool full = mrows >= 32 && ncols >= 16 * NBN;
  constexpr bool kDeep = sizeof(T) == 8 && NBN == 2;
  constexpr int kHalves = kDeep ? 2 : 1;   // fragment reads per chunk
  constexpr int kS = 4 / kHalves;          // k-steps of 4 per fragment read
  auto multiply = [&](int buf) {
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
      T a[kS][2], b[kS][NBN];
#pragma unroll
      for (int s2 = 0; s2 < kS; ++s2) {
        const int kr = 4 * (kS * h + s2) + (lane >> 4);
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) a[s2][mi] = As[buf][(wm * 32 + mi * 16 + (lane & 15)) * kLdK + kr];
#pragma unroll
        for (int ni = 0; ni < NBN; ++ni) b[s2][ni] = Bs[buf][kr * LDN + wn * 16 * NBN + ni * 16 + (lane & 15)];
      }
      if (full) {
#pragma unroll
        for (int s2 = 0; s2 < kS; ++s2)
#pragma unroll
          for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int ni = 0; ni < NBN; ++ni) acc[mi][ni] = mfma16(a[s2][mi], b[s2][ni], acc[mi][ni]);
      } else {
#pragma unroll
        for (int s2 = 0; s2 < kS; ++s2)
#pragma unroll
          for (int mi = 0; mi < 2; ++mi) {
            if (16 * mi >= mrows) continue;
#pragma unroll
            for (int ni = 0; ni < NBN; ++ni)
              if (16 * ni < ncols) acc[mi][ni] = mfma16(a[s2][mi], b[s2][ni], acc[mi][ni]);
          }
      }
    }
  };

  typedef std::integral_constant<int, 0> S0;
  typedef std::integral_constant<int, 1> S1_;
  const int nchunk = (nb + kKC - 1) / kKC;
  if constexpr (kDeep) {
    load_cols(S0{}, 0);
    load_cols(S1_{}, kKC);
    fetch(S0{}, 0);
    stash(S0{}, 0);
    if (nchunk > 1) {
      load_cols(S0{}, 2 * kKC);
      fetch(S1_{}, kKC);
    }
    if (nchunk > 2) {
      load_cols(S1_{}, 3 * kKC);
      fetch(S0{}, 2 * kKC);
    }
    __syncthreads();
    // iteration c: multiply chunk c, stash chunk c + 1 (register set (c + 1) & 1 = S) into the
    // other buffer, then load the index of chunk c + 4 and the data of chunk c + 3 into set S
    auto iter = [&](int c, auto S) {
      constexpr int s = decltype(S)::value;
      multiply(s ^ 1);
      if (c + 1 < nchunk) stash(S, s);
      if (c + 3 < nchunk) {
        load_cols(std::integral_constant<int, s ^ 1>{}, (c + 4) * kKC);
        fetch(S, (c + 3) * kKC);
      }
      __syncthreads();
    };
    for (int c = 0; c < nchunk; c += 2) {
      iter(c, S1_{});
      if (c + 1 < nchunk) iter(c + 1, S0{});
    }
  } else {
    load_cols(S0{}, 0);
    fetch(S0{}, 0);
    stash(S0{}, 0);
    load_cols(S0{}, kKC);
    __syncthreads();
    for (int c = 0; c < nchunk; ++c) {
      const int buf = c & 1;
      if (c + 1 < nchunk) {
        fetch(S0{}, (c + 1) * kKC);
        load_cols(S0{}, (c + 2) * kKC);
      }
      multiply(buf);
      if (c + 1 < nchunk) stash(S0{}, buf ^ 1);
      __syncthreads();
    }
  }

  if (xout) {   // store mode (backward): X^T[j][p] into a function-major slab, and, with a
                // density output, the epilogue as well
#pragma unroll
    for (int ni = 0; ni < NBN; ++ni) {
      const int p = p0 + wn * 16 * NBN + ni * 16 + (lane & 15);
      if (p >= d.n_p) continue;
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = j0 + wm * 32 + mi * 16 + acc_row<T>(lane, r);
          if (j < nb) xout[d.slab_off + (size_t)j * ldp + p] = acc[mi][ni][r];
        }
    }
    if (!n_sorted) return;      // else also the density epilogue below
  }
  // epilogue: column sums of X^T o Phi^T (density) and of w X^T o tPhi^T (kinetic energy)
  double sn[NBN], sd[NBN], se = 0.0;
#pragma unroll
  for (int ni = 0; ni < NBN; ++ni) {
    const int p = p0 + wn * 16 * NBN + ni * 16 + (lane & 15);
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
      sd[ni] = acce;
      acce *= pts[d.pt_off + p].w;
    } else {
      sd[ni] = 0.0;
    }
    sn[ni] = accn;
    se += acce;
  }
  density_epilogue<NBN>(sn, sd, se, lane, wave, wm, wn, p0, d.n_p, d.pt_off, red_n, red_d, red_e,
                        n_sorted, d_sorted, et_batch, it.batch);
}

template <typename T, int NBN>
__global__ void __launch_bounds__(256)
density_kernel(const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
               const SystemDesc* __restrict__ systems, const double4* __restrict__ pts,
               const int32_t* __restrict__ batch_cols, const T* __restrict__ Pmat,
               const T* __restrict__ slab1, const T* __restrict__ slab2,
               double* __restrict__ n_sorted, double* __restrict__ et_batch,
               T* __restrict__ xout, double* __restrict__ d_sorted,
    int* __restrict__ queue) {
  run_items(n_items, queue, [&](int item) {
    density_tile<T, NBN>(item, items, n_items, batches, systems, pts, batch_cols, Pmat, slab1, slab2, n_sorted, et_batch, xout, d_sorted);
  });
}


// H / S, FP64 / FP32: C[i][j] = sum_p slab1[i][p] slab2[j][p] over the batch's points, then a
// FP64 scatter-add into the dense output.  TE = 64: 64 x 64 tiles, each wave a 2 x 2 set of
// 16 x 16 blocks; TE = 32: 32 x 32 tiles (less padding on ragged basis counts), each wave one
// block, threads 0-127 staging the first operand and 128-255 the second.
template <typename T, int TE>
__device__ __forceinline__ void
hs_tile(int item, const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
          const SystemDesc* __restrict__ systems, const int32_t* __restrict__ batch_cols,
          const T* __restrict__ slab1, const T* __restrict__ slab2, double* __restrict__ out) {
  constexpr int NB = TE / 32;         // 16 x 16 blocks per wave and dimension
  const TileItem it = items[item];
  const BatchDesc d = batches[it.batch];
  const SystemDesc sys = systems[d.sys];
  const int nb = d.n_b, ldp = d.ldp;
  const int i0 = it.ti * TE, jb = it.tj * TE;
  const int* cols = batch_cols + d.col_off;

  __shared__ T As[2][TE * kLdK];      // Phi^T[i][p], p contiguous (K)
  __shared__ T Bs[2][TE * kLdK];      // second operand [j][p], p contiguous (K)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int mrows = nb - (i0 + wm * 16 * NB), ncols = nb - (jb + wn * 16 * NB);
  typedef typename Acc<T>::type acc_t;
  acc_t acc[NB][NB];
#pragma unroll
  for (int mi = 0; mi < NB; ++mi)
#pragma unroll
    for (int ni = 0; ni < NB; ++ni) acc[mi][ni] = acc_t{0, 0, 0, 0};

  // TE = 64: thread t stages row t / 4 of both operands; TE = 32: threads 0-127 stage row t / 4
  // of the first operand, threads 128-255 row (t - 128) / 4 of the second
  const int row = TE == 64 ? tid >> 2 : (tid & 127) >> 2, seg = tid & 3;
  const bool sa = TE == 64 || tid < 128, sb = TE == 64 || tid >= 128;
  const bool a_ok = sa && i0 + row < nb, b_ok = sb && jb + row < nb;
  const T* Ap = slab1 + d.slab_off + (size_t)(a_ok ? i0 + row : 0) * ldp + 4 * seg;
  const T* Bp = slab2 + d.slab_off + (size_t)(b_ok ? jb + row : 0) * ldp + 4 * seg;
  T av[4], bv[4];
  auto fetch = [&](int kc) {
    if (sa) load4<T>(Ap + kc, av);     // rows beyond n_b read row 0 and are zeroed when stashed
    if (sb) load4<T>(Bp + kc, bv);
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (sa) As[buf][row * kLdK + 4 * seg + c] = a_ok ? av[c] : T(0);
      if (sb) Bs[buf][row * kLdK + 4 * seg + c] = b_ok ? bv[c] : T(0);
    }
  };
  const bool full = mrows >= 16 * NB && ncols >= 16 * NB;
  auto multiply = [&](int buf) {
    T a[4][NB], b[4][NB];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int kr = 4 * s4 + (lane >> 4);
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        a[s4][i] = As[buf][(wm * 16 * NB + i * 16 + (lane & 15)) * kLdK + kr];
        b[s4][i] = Bs[buf][(wn * 16 * NB + i * 16 + (lane & 15)) * kLdK + kr];
      }
    }
    if (full) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int mi = 0; mi < NB; ++mi)
#pragma unroll
          for (int ni = 0; ni < NB; ++ni) acc[mi][ni] = mfma16(a[s4][mi], b[s4][ni], acc[mi][ni]);
    } else {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int mi = 0; mi < NB; ++mi) {
          if (16 * mi >= mrows) continue;
#pragma unroll
          for (int ni = 0; ni < NB; ++ni)
            if (16 * ni < ncols) acc[mi][ni] = mfma16(a[s4][mi], b[s4][ni], acc[mi][ni]);
        }
    }
  };
  const int nchunk = ldp / kKC;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) fetch((c + 1) * kKC);
    multiply(buf);
    if (c + 1 < nchunk) stash(buf ^ 1);
    __syncthreads();
  }
  if (mrows <= 0 || ncols <= 0) return;
  double* O = out + sys.mat_off;
#pragma unroll
  for (int ni = 0; ni < NB; ++ni) {
    const int j = jb + wn * 16 * NB + ni * 16 + (lane & 15);
    if (j >= nb) continue;
    const size_t gj = (size_t)cols[j];
#pragma unroll
    for (int mi = 0; mi < NB; ++mi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm * 16 * NB + mi * 16 + acc_row<T>(lane, r);
        if (i < nb) unsafeAtomicAdd(O + (size_t)cols[i] * sys.nb + gj, (double)acc[mi][ni][r]);
      }
  }
}

template <typename T, int TE>
__global__ void __launch_bounds__(256)
hs_kernel(const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
          const SystemDesc* __restrict__ systems, const int32_t* __restrict__ batch_cols,
          const T* __restrict__ slab1, const T* __restrict__ slab2, double* __restrict__ out,
    int* __restrict__ queue) {
  run_items(n_items, queue, [&](int item) {
    hs_tile<T, TE>(item, items, n_items, batches, systems, batch_cols, slab1, slab2, out);
  });
}


// ------------------------------------------------------------------------------------------
// BF16x3 kernels: a_hi b_hi + a_hi b_lo + a_lo b_hi on v_mfma_f32_16x16x32_bf16 (FP32
// accumulation), K chunks of 32, same 64-row tiles.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void mfma3(bf16x8_t ah, bf16x8_t al, bf16x8_t bh, bf16x8_t bl, f4_t& acc) {
  acc = mfma_bf16(al, bh, acc);
  acc = mfma_bf16(ah, bl, acc);
  acc = mfma_bf16(ah, bh, acc);
}

__device__ __forceinline__ float bf_pair(const bf16_t* p, int lo_off) {
  return (float)p[0] + (float)p[lo_off];
}

// Density: X^T[j][p] = sum_i P_b[j][i] Phi[p][i].  P comes from its FP32 copy and is split
// while staged; Phi comes from the function-major bf16 slab and is transposed into
// K-contiguous LDS rows while staged.
template <int NBN>
__device__ __forceinline__ void
density_tile_bf16(int item, const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
                    const SystemDesc* __restrict__ systems, const double4* __restrict__ pts,
                    const int32_t* __restrict__ batch_cols, const float* __restrict__ Pmat,
                    const bf16_t* __restrict__ slab1, const bf16_t* __restrict__ slab2,
                    double* __restrict__ n_sorted, double* __restrict__ et_batch,
                    float* __restrict__ xout) {
  constexpr int PT = 32 * NBN;
  constexpr int BW = PT / 8;            // 8-point units per slab row
  constexpr int BU = kKB * BW;          // units of the B tile
  constexpr int BQ = (BU + 255) / 256;
  const TileItem it = items[item];
  const BatchDesc d = batches[it.batch];
  const SystemDesc sys = systems[d.sys];
  const int nb = d.n_b, ldp = d.ldp;
  const int j0 = it.ti * kTile, p0 = it.tj * PT;
  const int* cols = batch_cols + d.col_off;
  const bf16_t* S1 = slab1 + 2 * d.slab_off;
  const bf16_t* S2 = slab2 + 2 * d.slab_off;
  const float* Pm = Pmat + sys.mat_off;

  __shared__ __attribute__((aligned(16))) bf16_t Ah[2][kTile * kLdB], Al[2][kTile * kLdB];
  __shared__ __attribute__((aligned(16))) bf16_t Bh[2][PT * kLdB], Bl[2][PT * kLdB];
  __shared__ double red_n[2][PT];
  __shared__ double red_e[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int mrows = nb - (j0 + wm * 32);
  const int ncols = d.n_p - (p0 + wn * 16 * NBN);
  f4_t acc[2][NBN];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < NBN; ++ni) acc[mi][ni] = f4_t{0, 0, 0, 0};

  // P_b staging: load c of a thread reads tile row 8 (tid / 32) + c at chunk column tid % 32, so
  // one load instruction covers two rows of 32 consecutive columns (two cache lines of P)
  // instead of sixteen rows
  const int kq = tid & 31, rb = 8 * (tid >> 5);
  uint32_t prow[8];                 // row offsets into the system's P (n_basis <= 65535)
  bool rok[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int j = j0 + rb + c;
    rok[c] = j < nb;
    prow[c] = (uint32_t)cols[rok[c] ? j : 0] * (uint32_t)sys.nb;
  }

  int cidx = 0;
  float pa[8];
  bf16x8_t bh[BQ], bl[BQ];
  const bool full = mrows >= 32 && ncols >= 16 * NBN;
  bool kval = false;
  auto load_cols = [&](int kc) {     // unconditional load of a clamped index (no branch)
    const int k = kc + kq;
    kval = k < nb;
    cidx = cols[k < nb ? k : nb - 1];
  };
  bool aok[8], bok[BQ];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      aok[c] = rok[c] && kval;
      pa[c] = Pm[prow[c] + (uint32_t)cidx];
    }
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
      const int u = tid + 256 * q;
      const int k = u & (kKB - 1), ps = u / kKB;
      bok[q] = u < BU && kc + k < nb && p0 + 8 * ps < ldp;
      const bf16_t* src = S1 + (bok[q] ? (size_t)(kc + k) * 2 * ldp + p0 + 8 * ps : 0);
      bh[q] = *reinterpret_cast<const bf16x8_t*>(src);
      bl[q] = *reinterpret_cast<const bf16x8_t*>(src + ldp);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      bf16_t hh, ll;
      split_bf16(aok[c] ? pa[c] : 0.f, hh, ll);
      Ah[buf][(rb + c) * kLdB + kq] = hh;
      Al[buf][(rb + c) * kLdB + kq] = ll;
    }
    const bf16_t zero = (bf16_t)0.f;
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
      const int u = tid + 256 * q;
      if (u < BU) {
        const int k = u & (kKB - 1), ps = u / kKB;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          Bh[buf][(8 * ps + c) * kLdB + k] = bok[q] ? bh[q][c] : zero;
          Bl[buf][(8 * ps + c) * kLdB + k] = bok[q] ? bl[q][c] : zero;
        }
      }
    }
  };
  auto multiply = [&](int buf) {
    const int kq = 8 * (lane >> 4);
    bf16x8_t ah[2], al[2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      const int o = (wm * 32 + mi * 16 + (lane & 15)) * kLdB + kq;
      ah[mi] = *reinterpret_cast<const bf16x8_t*>(&Ah[buf][o]);
      al[mi] = *reinterpret_cast<const bf16x8_t*>(&Al[buf][o]);
    }
    bf16x8_t bhv[NBN], blv[NBN];
#pragma unroll
    for (int ni = 0; ni < NBN; ++ni) {
      const int o = (wn * 16 * NBN + ni * 16 + (lane & 15)) * kLdB + kq;
      bhv[ni] = *reinterpret_cast<const bf16x8_t*>(&Bh[buf][o]);
      blv[ni] = *reinterpret_cast<const bf16x8_t*>(&Bl[buf][o]);
    }
    if (full) {
#pragma unroll
      for (int ni = 0; ni < NBN; ++ni)
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) mfma3(ah[mi], al[mi], bhv[ni], blv[ni], acc[mi][ni]);
    } else {
#pragma unroll
      for (int ni = 0; ni < NBN; ++ni) {
        if (16 * ni >= ncols) continue;
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
          if (16 * mi < mrows) mfma3(ah[mi], al[mi], bhv[ni], blv[ni], acc[mi][ni]);
      }
    }
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
    multiply(buf);
    if (c + 1 < nchunk) stash(buf ^ 1);
    __syncthreads();
  }

  if (xout) {   // store mode (backward): X^T[j][p] as FP32 into a function-major slab
#pragma unroll
    for (int ni = 0; ni < NBN; ++ni) {
      const int p = p0 + wn * 16 * NBN + ni * 16 + (lane & 15);
      if (p >= d.n_p) continue;
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int j = j0 + wm * 32 + mi * 16 + acc_row<float>(lane, rr);
          if (j < nb) xout[d.slab_off + (size_t)j * ldp + p] = acc[mi][ni][rr];
        }
    }
    if (!n_sorted) return;      // else also the density epilogue below
  }
  double sn[NBN], se = 0.0;
#pragma unroll
  for (int ni = 0; ni < NBN; ++ni) {
    const int p = p0 + wn * 16 * NBN + ni * 16 + (lane & 15);
    double accn = 0.0, acce = 0.0;
    if (p < d.n_p) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int j = j0 + wm * 32 + mi * 16 + acc_row<float>(lane, rr);
          if (j < nb) {
            const double x = (double)acc[mi][ni][rr];
            const size_t o = (size_t)j * 2 * ldp + p;
            accn += x * (double)bf_pair(S1 + o, ldp);
            acce += x * (double)bf_pair(S2 + o, ldp);
          }
        }
      acce *= pts[d.pt_off + p].w;
    }
    sn[ni] = accn;
    se += acce;
  }
  double sd[NBN];
  density_epilogue<NBN>(sn, sd, se, lane, wave, wm, wn, p0, d.n_p, d.pt_off, red_n, red_n, red_e,
                        n_sorted, nullptr, et_batch, it.batch);
}

template <int NBN>
__global__ void __launch_bounds__(256)
density_kernel_bf16(const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
                    const SystemDesc* __restrict__ systems, const double4* __restrict__ pts,
                    const int32_t* __restrict__ batch_cols, const float* __restrict__ Pmat,
                    const bf16_t* __restrict__ slab1, const bf16_t* __restrict__ slab2,
                    double* __restrict__ n_sorted, double* __restrict__ et_batch,
                    float* __restrict__ xout,
    int* __restrict__ queue) {
  run_items(n_items, queue, [&](int item) {
    density_tile_bf16<NBN>(item, items, n_items, batches, systems, pts, batch_cols, Pmat, slab1, slab2, n_sorted, et_batch, xout);
  });
}


// 16-byte segment of row `row` that holds k segment `seg` in the swizzled 64-byte LDS rows of
// the BF16 H kernel: rows are unpadded and the segment index is XORed with bits 1-2 of the
// row, so that the staging writes (four threads per row) and the fragment reads (16 rows per
// 16 lanes) fall on distinct 16-byte bank groups for 8- and 16-lane phases alike.
__device__ __forceinline__ int bf_seg(int row, int seg) { return seg ^ (((row >> 1) ^ (row >> 2)) & 3); }

// H/S: C[i][j] = sum_p slab1[i][p] slab2[j][p] from function-major bf16 slabs.
__device__ __forceinline__ void
hs_tile_bf16(int item, const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
               const SystemDesc* __restrict__ systems, const int32_t* __restrict__ batch_cols,
               const bf16_t* __restrict__ slab1, const bf16_t* __restrict__ slab2,
               double* __restrict__ out) {
  const TileItem it = items[item];
  const BatchDesc d = batches[it.batch];
  const SystemDesc sys = systems[d.sys];
  const int nb = d.n_b, ldp = d.ldp;
  const int i0 = it.ti * kTile, jb = it.tj * kTile;
  const int* cols = batch_cols + d.col_off;

  __shared__ __attribute__((aligned(16))) bf16_t Ah[2][kTile * kKB], Al[2][kTile * kKB];
  __shared__ __attribute__((aligned(16))) bf16_t Bh[2][kTile * kKB], Bl[2][kTile * kKB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int mrows = nb - (i0 + wm * 32), ncols = nb - (jb + wn * 32);
  f4_t acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = f4_t{0, 0, 0, 0};

  const int r = tid >> 2, sg = tid & 3;
  const bool a_ok = i0 + r < nb, b_ok = jb + r < nb;
  const bf16_t* Ap = slab1 + 2 * d.slab_off + (size_t)(a_ok ? i0 + r : 0) * 2 * ldp + 8 * sg;
  const bf16_t* Bp = slab2 + 2 * d.slab_off + (size_t)(b_ok ? jb + r : 0) * 2 * ldp + 8 * sg;
  bf16x8_t ah, al, bh, bl;
  auto fetch = [&](int kc) {
    ah = *reinterpret_cast<const bf16x8_t*>(Ap + kc);   // rows beyond n_b read row 0 and are
    al = *reinterpret_cast<const bf16x8_t*>(Ap + ldp + kc);   // zeroed when stashed
    bh = *reinterpret_cast<const bf16x8_t*>(Bp + kc);
    bl = *reinterpret_cast<const bf16x8_t*>(Bp + ldp + kc);
  };
  auto stash = [&](int buf) {
    const bf16x8_t z = {};
    const int o = r * kKB + 8 * bf_seg(r, sg);
    *reinterpret_cast<bf16x8_t*>(&Ah[buf][o]) = a_ok ? ah : z;
    *reinterpret_cast<bf16x8_t*>(&Al[buf][o]) = a_ok ? al : z;
    *reinterpret_cast<bf16x8_t*>(&Bh[buf][o]) = b_ok ? bh : z;
    *reinterpret_cast<bf16x8_t*>(&Bl[buf][o]) = b_ok ? bl : z;
  };
  const bool full = mrows >= 32 && ncols >= 32;
  auto multiply = [&](int buf) {
    const int kseg = lane >> 4;
    bf16x8_t a_h[2], a_l[2], b_h[2], b_l[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ra = wm * 32 + i * 16 + (lane & 15), rb = wn * 32 + i * 16 + (lane & 15);
      const int oa = ra * kKB + 8 * bf_seg(ra, kseg);
      const int ob = rb * kKB + 8 * bf_seg(rb, kseg);
      a_h[i] = *reinterpret_cast<const bf16x8_t*>(&Ah[buf][oa]);
      a_l[i] = *reinterpret_cast<const bf16x8_t*>(&Al[buf][oa]);
      b_h[i] = *reinterpret_cast<const bf16x8_t*>(&Bh[buf][ob]);
      b_l[i] = *reinterpret_cast<const bf16x8_t*>(&Bl[buf][ob]);
    }
    if (full) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) mfma3(a_h[mi], a_l[mi], b_h[ni], b_l[ni], acc[mi][ni]);
    } else {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) {
        if (16 * mi >= mrows) continue;
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          if (16 * ni < ncols) mfma3(a_h[mi], a_l[mi], b_h[ni], b_l[ni], acc[mi][ni]);
      }
    }
  };
  const int nchunk = ldp / kKB;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) fetch((c + 1) * kKB);
    multiply(buf);
    if (c + 1 < nchunk) stash(buf ^ 1);
    __syncthreads();
  }
  if (mrows <= 0 || ncols <= 0) return;
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

__global__ void __launch_bounds__(256)
hs_kernel_bf16(const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
               const SystemDesc* __restrict__ systems, const int32_t* __restrict__ batch_cols,
               const bf16_t* __restrict__ slab1, const bf16_t* __restrict__ slab2,
               double* __restrict__ out,
    int* __restrict__ queue) {
  run_items(n_items, queue, [&](int item) {
    hs_tile_bf16(item, items, n_items, batches, systems, batch_cols, slab1, slab2, out);
  });
}


// ------------------------------------------------------------------------------------------
// Backward: Pulay-type forces from basis gradients.  For every (point, relevant atom) pair the
// radial functions, their derivatives and the solid-harmonic gradients are recomputed and
//   g_a += w_p sum_{i on a} [(2 v_p X_pi + Y_pi) grad phi_i(p) + X_pi grad tphi_i(p)]
// with grad phi = (R' - l R/r) Y_lm u + (R/r) grad S_lm(u) (same with K for t phi); each
// atom's sum over a batch's points is reduced across a wave and dE/dR_a -= gE g_a is added
// with FP64 atomics.
// ------------------------------------------------------------------------------------------
// One shell of angular momentum L (a compile-time constant, so that only that harmonic's
// registers are live): adds its functions' terms of the per-point gradient sum.
template <typename T, int L>
__device__ __forceinline__ void pulay_shell(const T* __restrict__ c, T dt, T ir, T ux, T uy, T uz,
                                            T two_v, const T* __restrict__ X,
                                            const T* __restrict__ Y, size_t o0, int ldp, T& gx,
                                            T& gy, T& gz) {
  const T R = cubic(c, dt), dR = cubic_d(c, dt) * ir;
  const T K = cubic(c + 4, dt), dK = cubic_d(c + 4, dt) * ir;
  T Yl[7], Gx[7], Gy[7], Gz[7];
  ylm_l<T>(L, ux, uy, uz, Yl);
  ylm_grad_l<T>(L, ux, uy, uz, Gx, Gy, Gz);
  const T aR = dR - T(L) * R * ir, aK = dK - T(L) * K * ir;
  const T bR = R * ir, bK = K * ir;
#pragma unroll
  for (int m = 0; m < 2 * L + 1; ++m) {
    const size_t o = o0 + (size_t)m * ldp;
    const T xv = X[o], yv = Y[o];
    const T cp = two_v * xv + yv;        // multiplies grad phi
    const T ru = (cp * aR + xv * aK) * Yl[m];   // radial part, along u
    const T rs = cp * bR + xv * bK;             // angular part, along grad S
    gx += ru * ux + rs * Gx[m];
    gy += ru * uy + rs * Gy[m];
    gz += ru * uz + rs * Gz[m];
  }
}

// Work mapping as in the basis evaluation: kPhiSlices workgroups per batch, one relevant atom
// per wave at a time, lanes over the batch's points; each wave reduces its atom's gradient
// across lanes and adds -gE g_a to dE/dR_a with three FP64 atomics.
template <typename T>
__global__ void __launch_bounds__(256)
pulay_kernel(const BatchDesc* __restrict__ batches, int b0, const double4* __restrict__ pts,
             const int32_t* __restrict__ perm, const int32_t* __restrict__ batch_atoms,
             const int32_t* __restrict__ batch_acol, const double* __restrict__ atom_xyz,
             const int32_t* __restrict__ atom_species, const SpeciesDesc* __restrict__ species,
             const int32_t* __restrict__ shell_l, const T* __restrict__ spline, RadialGrid rg,
             const double* __restrict__ v, const T* __restrict__ Xs, const T* __restrict__ Ys,
             const double* __restrict__ gE, double* __restrict__ dE_dR, double* __restrict__ gpt) {
  const int bi = blockIdx.x / kPhiSlices;
  const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x % kPhiSlices) * 4 + (int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const BatchDesc d = batches[b0 + bi];
  const int np = d.n_p, na = d.n_atoms, ldp = d.ldp;
  const T* X = Xs + d.slab_off;
  const T* Y = Ys + d.slab_off;
  const double ge = gE[0];
  for (int k = wave; k < na; k += 4 * kPhiSlices) {
    const int atom = batch_atoms[d.atom_off + k];
    const int col0 = batch_acol[d.atom_off + k];
    const SpeciesDesc sd = species[atom_species[atom]];
    const double ax = atom_xyz[3 * atom], ay = atom_xyz[3 * atom + 1], az = atom_xyz[3 * atom + 2];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int p = lane; p < np; p += 64) {
      const double4 P4 = pts[d.pt_off + p];
      const double dx = P4.x - ax, dy = P4.y - ay, dz = P4.z - az;
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      if (!(r < rg.rc)) continue;
      const double rr = fmax(r, 1e-12);
      const double inv = 1.0 / rr;
      const T ux = T(dx * inv), uy = T(dy * inv), uz = T(dz * inv), ir = T(inv);
      const RadialPos rp = radial_pos(rr, rg);
      const T dt = T(rp.dt);
      const T* c = spline + sd.spline_off + (size_t)rp.k * sd.nshell * 8;
      const T two_v = T(2.0 * v[perm[d.pt_off + p]]);
      T gx = 0, gy = 0, gz = 0;
      int f = col0;
      for (int j = 0; j < sd.nshell; ++j) {
        const int l = shell_l[sd.shell_l_off + j];
        const size_t o0 = (size_t)f * ldp + p;
        switch (l) {
          case 0: pulay_shell<T, 0>(c + j * 8, dt, ir, ux, uy, uz, two_v, X, Y, o0, ldp, gx, gy, gz); break;
          case 1: pulay_shell<T, 1>(c + j * 8, dt, ir, ux, uy, uz, two_v, X, Y, o0, ldp, gx, gy, gz); break;
          case 2: pulay_shell<T, 2>(c + j * 8, dt, ir, ux, uy, uz, two_v, X, Y, o0, ldp, gx, gy, gz); break;
          default: pulay_shell<T, 3>(c + j * 8, dt, ir, ux, uy, uz, two_v, X, Y, o0, ldp, gx, gy, gz); break;
        }
        f += 2 * l + 1;
      }
      sx += P4.w * (double)gx;
      sy += P4.w * (double)gy;
      sz += P4.w * (double)gz;
      if (gpt) {     // the same terms summed over atoms per point: the point-motion term
        unsafeAtomicAdd(gpt + 3 * (size_t)(d.pt_off + p), P4.w * (double)gx);
        unsafeAtomicAdd(gpt + 3 * (size_t)(d.pt_off + p) + 1, P4.w * (double)gy);
        unsafeAtomicAdd(gpt + 3 * (size_t)(d.pt_off + p) + 2, P4.w * (double)gz);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      sx += __shfl_xor(sx, off);
      sy += __shfl_xor(sy, off);
      sz += __shfl_xor(sz, off);
    }
    if (lane == 0) {
      unsafeAtomicAdd(dE_dR + 3 * atom, -ge * sx);
      unsafeAtomicAdd(dE_dR + 3 * atom + 1, -ge * sy);
      unsafeAtomicAdd(dE_dR + 3 * atom + 2, -ge * sz);
    }
  }
}

// y[i] = gE * x[i]
__global__ void scale_kernel(double* __restrict__ y, const double* __restrict__ x, size_t n,
                             const double* __restrict__ gE) {
  const double s = gE[0];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    y[i] = s * x[i];
}

// dE/dv in caller order: gE w_p n_p
__global__ void dv_kernel(double* __restrict__ dv, const double* __restrict__ n_sorted,
                          const double4* __restrict__ pts, const int32_t* __restrict__ perm,
                          int64_t n, const double* __restrict__ gE) {
  const double s = gE[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dv[perm[i]] = s * pts[i].w * n_sorted[i];
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
// of one system (blockIdx.y = system).
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
sums_finish_kernel(const double* __restrict__ part, int nblk, const int64_t* __restrict__ sys_batch_range,
                   const double* __restrict__ et_batch, double* __restrict__ sums_out) {
  __shared__ double sh[4];
  const int s = blockIdx.x;
  double sn = 0.0, sv = 0.0, se = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
    sn += part[(size_t)s * nblk * 2 + 2 * i];
    sv += part[(size_t)s * nblk * 2 + 2 * i + 1];
  }
  for (int64_t i = sys_batch_range[2 * s] + threadIdx.x; i < sys_batch_range[2 * s + 1]; i += blockDim.x)
    se += et_batch[i];
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

static inline int item_grid(int n_items) { return ((n_items + 7) / 8) * 8; }

// Workgroups of a 256-thread kernel that are resident on the current device at once
// (occupancy x compute units), cached per kernel.
int resident_workgroups(const void* fn) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(fn);
  if (it != cache.end()) return it->second;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, 0) != hipSuccess)
    return 0;
  const int n = std::max(1, per) * std::max(1, cus);
  cache[fn] = n;
  return n;
}

// Grid of a tiled launch: one workgroup per item, or (persistent) the resident workgroup
// count rounded down to a multiple of the 8 XCDs.
int tile_grid(int n_items, const Queue& q, const void* fn) {
  const int g = item_grid(n_items);
  if (!q.counters) return g;
  const int res = q.workgroups > 0 ? q.workgroups : resident_workgroups(fn);
  return std::min(g, std::max(8, res / 8 * 8));
}

// Screening check of positions held on the device: flag = 1 if any atom is not finite or moved
// farther than the margin from its set-up position, else 0.  One workgroup.
__global__ void __launch_bounds__(256)
positions_check_kernel(const double* __restrict__ xyz, const double* __restrict__ xyz0, int n,
                       double margin2, int* __restrict__ flag) {
  int bad = 0;
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    double d2 = 0.0;
    bool fin = true;
    for (int c = 0; c < 3; ++c) {
      const double x = xyz[3 * a + c];
      fin = fin && isfinite(x);
      const double d = x - xyz0[3 * a + c];
      d2 += d * d;
    }
    if (!fin || !(d2 <= margin2)) bad = 1;
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) *flag = bad;
}

// The outputs of a call whose device positions failed the check become NaN (a no-op otherwise).
__global__ void poison_kernel(double* __restrict__ x, size_t n, const int* __restrict__ flag) {
  if (*flag == 0) return;
  const double nan = __builtin_nan("");
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[i] = nan;
}

hipError_t launch_positions_check(const double* xyz, const double* xyz0, int n, double margin,
                                  int* flag, hipStream_t st) {
  hipLaunchKernelGGL(positions_check_kernel, dim3(1), dim3(256), 0, st, xyz, xyz0, n, margin * margin, flag);
  return hipGetLastError();
}

hipError_t launch_poison(double* x, size_t n, const int* flag, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(poison_kernel, dim3(grid_for(n, 256 * 4)), dim3(256), 0, st, x, n, flag);
  return hipGetLastError();
}

__global__ void zero_int_kernel(int* __restrict__ x, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = 0;
}

hipError_t launch_zero_int(int* x, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_int_kernel, dim3(std::min(256, (n + 255) / 256)), dim3(256), 0, st, x, n);
  return hipGetLastError();
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
  hipLaunchKernelGGL((phi_eval_kernel<T, kLayoutDense>), dim3(nbatch * kPhiSlices), dim3(256), 0, st, dv.batches,
                     b0, dv.pts, dv.perm, dv.batch_atoms, dv.batch_acol, dv.atom_xyz,
                     dv.atom_species, dv.species, dv.shell_l, spline, dv.rg, v, mode,
                     (void*)slab1, (void*)slab2);
  return hipGetLastError();
}

hipError_t launch_phi_eval_bf16(const DeviceView& dv, int b0, int nbatch, int mode, const double* v,
                                void* slab1, void* slab2, hipStream_t st) {
  if (nbatch == 0) return hipSuccess;
  hipLaunchKernelGGL((phi_eval_kernel<float, kLayoutBfFn>), dim3(nbatch * kPhiSlices), dim3(256), 0, st,
                     dv.batches, b0, dv.pts, dv.perm, dv.batch_atoms, dv.batch_acol, dv.atom_xyz,
                     dv.atom_species, dv.species, dv.shell_l, dv.spline32, dv.rg, v, mode,
                     slab1, slab2);
  return hipGetLastError();
}

template <typename T, int NBN>
static void density_launch_nbn(const DeviceView& dv, const TileItem* items, int n_items, const T* P,
                               const T* slab1, const T* slab2, double* n_sorted, double* et_batch,
                               T* xout, double* d_sorted, const Queue& q, hipStream_t st) {
  hipLaunchKernelGGL((density_kernel<T, NBN>), dim3(tile_grid(n_items, q, (const void*)density_kernel<T, NBN>)), dim3(256), 0,
                     st, items, n_items, dv.batches, dv.systems, dv.pts, dv.batch_cols, P, slab1, slab2,
                     n_sorted, et_batch, xout, d_sorted, q.counters);
}

template <typename T>
hipError_t launch_density(const DeviceView& dv, int nbn, const TileItem* items, int n_items, const T* P,
                          const T* slab1, const T* slab2, double* n_sorted, double* et_batch,
                          hipStream_t st, T* xout, Queue q, double* d_sorted) {
  if (n_items == 0) return hipSuccess;
  switch (nbn) {
    case 2: density_launch_nbn<T, 2>(dv, items, n_items, P, slab1, slab2, n_sorted, et_batch, xout, d_sorted, q, st); break;
    case 3: density_launch_nbn<T, 3>(dv, items, n_items, P, slab1, slab2, n_sorted, et_batch, xout, d_sorted, q, st); break;
    case 4: density_launch_nbn<T, 4>(dv, items, n_items, P, slab1, slab2, n_sorted, et_batch, xout, d_sorted, q, st); break;
    case 5: density_launch_nbn<T, 5>(dv, items, n_items, P, slab1, slab2, n_sorted, et_batch, xout, d_sorted, q, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_hs(const DeviceView& dv, const TileItem* items, int n_items, const T* slab1,
                     const T* slab2, double* out, hipStream_t st, Queue q, int te) {
  if (n_items == 0) return hipSuccess;
  if (te == 32)
    hipLaunchKernelGGL((hs_kernel<T, 32>), dim3(tile_grid(n_items, q, (const void*)hs_kernel<T, 32>)), dim3(256), 0, st,
                       items, n_items, dv.batches, dv.systems, dv.batch_cols, slab1, slab2, out, q.counters);
  else
    hipLaunchKernelGGL((hs_kernel<T, 64>), dim3(tile_grid(n_items, q, (const void*)hs_kernel<T, 64>)), dim3(256), 0, st,
                       items, n_items, dv.batches, dv.systems, dv.batch_cols, slab1, slab2, out, q.counters);
  return hipGetLastError();
}

template <int NBN>
static void density_bf16_launch_nbn(const DeviceView& dv, const TileItem* items, int n_items,
                                    const float* P, const void* slab1, const void* slab2,
                                    double* n_sorted, double* et_batch, float* xout, const Queue& q,
                                    hipStream_t st) {
  hipLaunchKernelGGL((density_kernel_bf16<NBN>), dim3(tile_grid(n_items, q, (const void*)density_kernel_bf16<NBN>)), dim3(256), 0, st, items,
                     n_items, dv.batches, dv.systems, dv.pts, dv.batch_cols, P, (const bf16_t*)slab1,
                     (const bf16_t*)slab2, n_sorted, et_batch, xout, q.counters);
}

hipError_t launch_density_bf16(const DeviceView& dv, int nbn, const TileItem* items, int n_items,
                               const float* P, const void* slab1, const void* slab2, double* n_sorted,
                               double* et_batch, hipStream_t st, float* xout, Queue q) {
  if (n_items == 0) return hipSuccess;
  switch (nbn) {
    case 2: density_bf16_launch_nbn<2>(dv, items, n_items, P, slab1, slab2, n_sorted, et_batch, xout, q, st); break;
    case 3: density_bf16_launch_nbn<3>(dv, items, n_items, P, slab1, slab2, n_sorted, et_batch, xout, q, st); break;
    case 4: density_bf16_launch_nbn<4>(dv, items, n_items, P, slab1, slab2, n_sorted, et_batch, xout, q, st); break;
    case 5: density_bf16_launch_nbn<5>(dv, items, n_items, P, slab1, slab2, n_sorted, et_batch, xout, q, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pulay(const DeviceView& dv, int b0, int nbatch, const double* v, const T* X,
                        const T* Y, const double* gE, double* dE_dR, hipStream_t st, double* gpt) {
  if (nbatch == 0) return hipSuccess;
  const T* spline = (const T*)(sizeof(T) == 8 ? (const void*)dv.spline64 : (const void*)dv.spline32);
  hipLaunchKernelGGL(pulay_kernel<T>, dim3(nbatch * kPhiSlices), dim3(256), 0, st, dv.batches, b0, dv.pts,
                     dv.perm, dv.batch_atoms, dv.batch_acol, dv.atom_xyz, dv.atom_species,
                     dv.species, dv.shell_l, spline, dv.rg, v, X, Y, gE, dE_dR, gpt);
  return hipGetLastError();
}

hipError_t launch_scale(double* y, const double* x, size_t n, const double* gE, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n, 256 * 4)), dim3(256), 0, st, y, x, n, gE);
  return hipGetLastError();
}

hipError_t launch_dv(const DeviceView& dv, double* dE_dv, const double* n_sorted, int64_t n,
                     const double* gE, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(dv_kernel, dim3(grid_for(n, 256 * 4)), dim3(256), 0, st, dE_dv, n_sorted, dv.pts,
                     dv.perm, n, gE);
  return hipGetLastError();
}

hipError_t launch_hs_bf16(const DeviceView& dv, const TileItem* items, int n_items, const void* slab1,
                          const void* slab2, double* out, hipStream_t st, Queue q) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(hs_kernel_bf16, dim3(tile_grid(n_items, q, (const void*)hs_kernel_bf16)), dim3(256), 0, st, items, n_items,
                     dv.batches, dv.systems, dv.batch_cols, (const bf16_t*)slab1, (const bf16_t*)slab2,
                     out, q.counters);
  return hipGetLastError();
}

hipError_t launch_density_finish(const DeviceView& dv, const double* n_sorted, const double* v,
                                 double* n_out, double* part, int nblk, const double* et_batch,
                                 double* sums_out, hipStream_t st) {
  hipLaunchKernelGGL(density_finish_kernel, dim3(nblk, dv.n_sys), dim3(256), 0, st,
                     dv.sys_pt_range, dv.pts, dv.perm, n_sorted, v, n_out, part, nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sums_finish_kernel, dim3(dv.n_sys), dim3(256), 0, st, part, nblk,
                     dv.sys_batch_range, et_batch, sums_out);
  return hipGetLastError();
}

template hipError_t launch_phi_eval<double>(const DeviceView&, int, int, int, const double*,
                                            double*, double*, hipStream_t);
template hipError_t launch_phi_eval<float>(const DeviceView&, int, int, int, const double*,
                                           float*, float*, hipStream_t);
template hipError_t launch_density<double>(const DeviceView&, int, const TileItem*, int, const double*,
                                           const double*, const double*, double*, double*,
                                           hipStream_t, double*, Queue, double*);
template hipError_t launch_density<float>(const DeviceView&, int, const TileItem*, int, const float*,
                                          const float*, const float*, double*, double*,
                                          hipStream_t, float*, Queue, double*);
template hipError_t launch_pulay<double>(const DeviceView&, int, int, const double*, const double*,
                                         const double*, const double*, double*, hipStream_t, double*);
template hipError_t launch_pulay<float>(const DeviceView&, int, int, const double*, const float*,
                                        const float*, const double*, double*, hipStream_t, double*);
template hipError_t launch_hs<double>(const DeviceView&, const TileItem*, int, const double*,
                                      const double*, double*, hipStream_t, Queue, int);
template hipError_t launch_hs<float>(const DeviceView&, const TileItem*, int, const float*,
                                     const float*, double*, hipStream_t, Queue, int);

// Resident-workgroup counts of every tiled kernel, queried once on the current device
// (outside any stream capture, so that later persistent launches only read the cache).
hipError_t prepare_launch_configs() {
  const void* fns[] = {
      (const void*)density_kernel<double, 2>, (const void*)density_kernel<double, 3>,
      (const void*)density_kernel<double, 4>, (const void*)density_kernel<double, 5>,
      (const void*)density_kernel<float, 2>,  (const void*)density_kernel<float, 3>,
      (const void*)density_kernel<float, 4>,  (const void*)density_kernel<float, 5>,
      (const void*)density_kernel_bf16<2>,    (const void*)density_kernel_bf16<3>,
      (const void*)density_kernel_bf16<4>,    (const void*)density_kernel_bf16<5>,
      (const void*)hs_kernel<double, 64>,     (const void*)hs_kernel<float, 64>,
      (const void*)hs_kernel<double, 32>,     (const void*)hs_kernel<float, 32>,
      (const void*)hs_kernel_bf16};
  for (const void* f : fns)
    if (resident_workgroups(f) <= 0) return hipErrorInvalidDeviceFunction;
  return hipSuccess;
}

}  // namespace aims
