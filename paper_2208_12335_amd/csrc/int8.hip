// gfx950 kernels of the sliced integer form (AIMS_INT8X7): the per-batch contractions of the
// density and Hamiltonian passes on the int8 matrix cores, with results of FP64 quality.
//
// Every operand row (a row of P, one point's basis values, one function's values over a batch)
// gets a power-of-two scale 2^e with max|x| 2^-e < 1/2, and each value is written as seven
// balanced base-128 digits,
//
//     x = 2^e sum_{s=1..7} q_s 128^-s,   q_s in [-64, 64]  (round to nearest at every digit),
//
// held one per byte of a 64-bit word (byte s-1 = q_s).  A product of two such rows is
//
//     sum_k a_k b_k = 2^(e_a + e_b) sum_{s,t} 128^-(s+t) sum_k q^a_{s,k} q^b_{t,k},
//
// where each inner sum is an exact int32 MFMA accumulation (|q q| <= 2^12; seven pairs per level
// and up to 74,898 terms stay below 2^31).  The H and S passes keep the pairs with s + t <= 8 (28
// products on v_mfma_i32_32x32x32_i8), the density pass those with s + t <= 9 (34): its P rows
// carry large, cancelling entries when S is ill-conditioned.  Each level d = s + t has its own
// int32 accumulator; the levels are combined in FP64 once per tile.  In the density pass the K
// index is balanced first: P' = P D and Phi' = D^-1 Phi with D = diag(2^f_i), f_i the exponent of
// function i's largest magnitude, an exact rescaling that keeps a point's small functions from
// sitting in the low digits of its scale.  This is the error-free splitting of matrix products
// into fixed-point slices of Ozaki, Ogita, Oishi and Rump (2012), in the integer-unit form of
// Ootomo, Ozaki and Yokota (2024), laid out here for the 64-wide gfx950 wavefront.
//
//   slice_p_kernel          P -> digit words P8 and one exponent per row (once per call)
//   phi_eval_i8_kernel      basis values of one batch -> digit slabs; the scales come from a
//                           first sweep over the batch (radial bounds |R| Ymax_l), per point for
//                           the density pass and per function for the H / S pass.  The density
//                           pass's second slab (t phi, read only by its FP64 epilogue, never by
//                           the matrix cores) holds plain FP64 values
//   density_i8_kernel       X^T = P_b Phi^T (64 functions x 64 points per tile), epilogue
//                           n_p += sum_j X_jp phi_jp and the E_T partial, in FP64
//   hs_i8_kernel            C = Phi^T (second operand) over the batch's points (64 x 64 tiles),
//                           FP64 scatter-add into H or S
#include <hip/hip_runtime.h>

#include <cstdint>

#include "aims_internal.h"
#include "basis.h"
#include "kernels.h"
#include "tiles.h"

namespace aims {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kDigits = 7;        // base-128 digits per value
constexpr int kLevelsH = 7;       // H / S: kept levels d = s + t = 2..8
constexpr int kLevelsD = 8;       // density: levels 2..9
constexpr int kKI = 32;           // K chunk (the K of one v_mfma_i32_32x32x32_i8)

// max over m of |Y_lm| on the unit sphere is sqrt((2l + 1) / (4 pi)) (addition theorem), with a
// margin that covers the rounding of the evaluated harmonics
__device__ __forceinline__ double ymax(int l) {
  constexpr double m = 1.0 + 1.0 / (double)(1ll << 30);
  switch (l) {
    case 0: return 0.28209479177387814 * m;
    case 1: return 0.4886025119029199 * m;
    case 2: return 0.6307831305050401 * m;
    default: return 0.7463526651802308 * m;
  }
}

// Exponent e with m 2^-e < 1/2 (m = 0: any e works, 0 is taken).
__device__ __forceinline__ int digit_exp(double m) {
  if (!(m > 0.0)) return 0;
  int k;
  (void)frexp(m, &k);            // m = f 2^k, f in [1/2, 1)
  return k + 1;
}

// Seven balanced base-128 digits of x 2^-e, packed one per byte.  Every step is exact in FP64:
// t - rint(t) is exact and |t| < 64.5 throughout.
__device__ __forceinline__ uint64_t to_digits(double x, int e) {
  double t = ldexp(x, 7 - e);
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (int s = 0; s < kDigits; ++s) {
    const double q = rint(t);
    t = (t - q) * 128.0;
    const uint32_t b = (uint32_t)((int)q) & 0xffu;
    if (s < 4) lo |= b << (8 * s);
    else hi |= b << (8 * (s - 4));
  }
  return ((uint64_t)hi << 32) | lo;
}

// The value 2^e sum_s q_s 128^-s of a digit word (exact up to the final scaling).
__device__ __forceinline__ double from_digits(uint64_t u, int e) {
  const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
  const int q1 = (int)(int8_t)(lo & 0xff), q2 = (int)(int8_t)((lo >> 8) & 0xff);
  const int q3 = (int)(int8_t)((lo >> 16) & 0xff), q4 = (int)(int8_t)(lo >> 24);
  const int q5 = (int)(int8_t)(hi & 0xff), q6 = (int)(int8_t)((hi >> 8) & 0xff);
  const int q7 = (int)(int8_t)((hi >> 16) & 0xff);
  const int a = (q1 * 128 + q2) * 128 + q3;                   // |a| < 2^21
  const int b = ((q4 * 128 + q5) * 128 + q6) * 128 + q7;      // |b| < 2^28
  return ldexp(fma((double)a, 268435456.0, (double)b), e - 49);
}

// Digit planes of eight consecutive K elements: in[m] holds the digits of element m; out[s]
// holds digit s+1 of elements 0..7 (byte m).  v_perm_b32 picks bytes from two words.
__device__ __forceinline__ void digit_planes(const uint64_t (&in)[8], uint64_t (&out)[kDigits]) {
  uint32_t w[8][2];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    w[m][0] = (uint32_t)in[m];
    w[m][1] = (uint32_t)(in[m] >> 32);
  }
#pragma unroll
  for (int s = 0; s < kDigits; ++s) {
    const int h = s >> 2, b = s & 3;
    const uint32_t sel01 = (uint32_t)b | ((uint32_t)(b + 4) << 8) | 0x0c0c0000u;
    const uint32_t sel23 = 0x00000c0cu | ((uint32_t)b << 16) | ((uint32_t)(b + 4) << 24);
    const uint32_t lo = __builtin_amdgcn_perm(w[1][h], w[0][h], sel01) |
                        __builtin_amdgcn_perm(w[3][h], w[2][h], sel23);
    const uint32_t hi = __builtin_amdgcn_perm(w[5][h], w[4][h], sel01) |
                        __builtin_amdgcn_perm(w[7][h], w[6][h], sel23);
    out[s] = ((uint64_t)hi << 32) | lo;
  }
}

__device__ __forceinline__ v16i mfma_i8(v4i a, v4i b, v16i c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// Row of the 32 x 32 output block held in accumulator register r of a lane (the column is
// lane % 32): four groups of eight rows, each lane group holding four consecutive rows.
__device__ __forceinline__ int acc_row32(int lane, int r) {
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// LDS tile of one operand: [digit][k group of 16][row 0..63][16 bytes], as u64 pairs.  A lane's
// MFMA fragment (row lane % 32 of its half, k group lane / 32) is one 16-byte read; 32 lanes read
// 512 contiguous bytes.
constexpr int kOpWords = kDigits * 2 * 64 * 2;   // u64 per operand and stage (14 KiB)
__device__ __forceinline__ int op_index(int s, int kg, int row, int half) {
  return ((s * 2 + kg) * 64 + row) * 2 + half;
}

// The products of one K chunk: digit s of A times digit t of B into level d = s + t
// (acc[d - 2]) for d <= LV + 1.  Consecutive MFMAs write different accumulators.
template <int LV>
__device__ __forceinline__ void multiply_levels(const uint64_t* __restrict__ As,
                                                const uint64_t* __restrict__ Bs, int lane,
                                                int arow, int bcol, v16i (&acc)[LV]) {
  v4i b[kDigits];
  const int kg = lane >> 5, r = lane & 31;
#pragma unroll
  for (int t = 0; t < kDigits; ++t) b[t] = *reinterpret_cast<const v4i*>(Bs + op_index(t, kg, bcol + r, 0));
#pragma unroll
  for (int s = 0; s < kDigits; ++s) {
    const v4i a = *reinterpret_cast<const v4i*>(As + op_index(s, kg, arow + r, 0));
#pragma unroll
    for (int t = 0; t < kDigits; ++t)
      if (s + t < LV) acc[s + t] = mfma_i8(a, b[t], acc[s + t]);
  }
}

// sum_d acc_d 2^-7d of one output, in FP64 (Horner over the levels)
template <int LV>
__device__ __forceinline__ double level_sum(const v16i (&acc)[LV], int r) {
  double s = (double)acc[LV - 1][r];
#pragma unroll
  for (int L = LV - 2; L >= 0; --L) s = fma(s, 0.0078125, (double)acc[L][r]);
  return ldexp(s, -14);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// P D -> digit words, one exponent per (global) row
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
slice_p_kernel(const double* __restrict__ P, uint64_t* __restrict__ P8, int32_t* __restrict__ eP,
               const SystemDesc* __restrict__ systems, int n_sys, const int32_t* __restrict__ fexp) {
  const int64_t g = blockIdx.x;
  int lo = 0, hi = n_sys - 1;                        // system of this row
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (systems[mid].row_off <= g) lo = mid;
    else hi = mid - 1;
  }
  const SystemDesc sd = systems[lo];
  const int64_t off = sd.mat_off + (g - sd.row_off) * (int64_t)sd.nb;
  const int32_t* fx = fexp + sd.row_off;             // column c is scaled by 2^fx[c]
  double m = 0.0;
  for (int c = threadIdx.x; c < sd.nb; c += 256) m = fmax(m, fabs(ldexp(P[off + c], fx[c])));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  __shared__ double sm[4];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  const int e = digit_exp(fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3])));
  if (threadIdx.x == 0) eP[g] = e;
  for (int c = threadIdx.x; c < sd.nb; c += 256) P8[off + c] = to_digits(ldexp(P[off + c], fx[c]), e);
}

// ------------------------------------------------------------------------------------------
// basis values -> digit slabs
// ------------------------------------------------------------------------------------------
// One workgroup per batch; its waves take (atom, 64-point chunk) pairs.  The density pass's
// first slab holds phi_i 2^-f_i (the balanced K operand), its second t phi_i.  Sweep 1 bounds every
// value by |R_s(r)| Ymax_l (or |w v R + w K| Ymax_l for the H operand, |w R| Ymax_l for S): per
// point over all functions (density, LDS max per point) or per function over all points (H / S,
// wave max then LDS max per column).  The exponents go to ex1 / ex2 (per point in batch order,
// or per batch column) and stay in LDS for sweep 2, which evaluates the basis again and writes
// the digit words.  Dynamic LDS: 2 x (ldp or n_b) u64.
template <int MODE>
__global__ void __launch_bounds__(256)
phi_eval_i8_kernel(const BatchDesc* __restrict__ batches, int b0, const double4* __restrict__ pts,
                   const int32_t* __restrict__ perm, const int32_t* __restrict__ batch_atoms,
                   const int32_t* __restrict__ batch_acol, const double* __restrict__ atom_xyz,
                   const int32_t* __restrict__ atom_species, const SpeciesDesc* __restrict__ species,
                   const int32_t* __restrict__ shell_l, const int32_t* __restrict__ shell_fexp,
                   const double* __restrict__ spline, RadialGrid rg, const double* __restrict__ v,
                   uint64_t* __restrict__ slab1, uint64_t* __restrict__ slab2,
                   int32_t* __restrict__ ex1, int32_t* __restrict__ ex2) {
  extern __shared__ unsigned long long smax[];
  const int wq = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const BatchDesc d = batches[b0 + blockIdx.x];
  const int np = d.n_p, na = d.n_atoms, ldp = d.ldp, nb = d.n_b;
  const int nslot = MODE == kModeDensity ? ldp : nb;
  unsigned long long* m1 = smax;
  unsigned long long* m2 = smax + nslot;
  for (int i = threadIdx.x; i < 2 * nslot; i += 256) smax[i] = 0ull;
  __syncthreads();
  const int nc = (ldp + 63) / 64;

  // sweep 1: bounds
  for (int q = wq; q < na * nc; q += 4) {
    const int k = q / nc, c = q - k * nc;
    const int atom = batch_atoms[d.atom_off + k];
    const int col0 = batch_acol[d.atom_off + k];
    const SpeciesDesc sd = species[atom_species[atom]];
    const int p = 64 * c + lane;
    double w = 0.0, wv = 0.0, r = 1e300;
    if (p < np) {
      const double4 P4 = pts[d.pt_off + p];
      const double dx = P4.x - atom_xyz[3 * atom], dy = P4.y - atom_xyz[3 * atom + 1],
                   dz = P4.z - atom_xyz[3 * atom + 2];
      r = sqrt(dx * dx + dy * dy + dz * dz);
      w = P4.w;
      if (MODE == kModeH) wv = P4.w * v[perm[d.pt_off + p]];
    }
    const bool in = r < rg.rc;
    RadialPos rp{0, 0.0};
    if (in) rp = radial_pos(fmax(r, 1e-12), rg);
    const double* cf = spline + sd.spline_off + (size_t)rp.k * sd.nshell * 8;
    double b1 = 0.0, b2 = 0.0;                          // density: per-lane bounds of this atom
    int f = col0;
    for (int j = 0; j < sd.nshell; ++j) {
      const int l = shell_l[sd.shell_l_off + j];
      const double ym = ymax(l);
      double R = 0.0, K = 0.0;
      if (in) {
        R = cubic(cf + j * 8, rp.dt);
        K = cubic(cf + j * 8 + 4, rp.dt);
      }
      if (MODE == kModeDensity) {
        b1 = fmax(b1, ldexp(fabs(R) * ym, -shell_fexp[sd.shell_l_off + j]));
        b2 = fmax(b2, fabs(K) * ym);
      } else {
        double s1 = fabs(R) * ym;
        double s2 = (MODE == kModeH ? fabs(wv * R + w * K) : fabs(w * R)) * ym;
        for (int o = 32; o > 0; o >>= 1) {
          s1 = fmax(s1, __shfl_xor(s1, o));
          s2 = fmax(s2, __shfl_xor(s2, o));
        }
        if (lane < 2 * l + 1) {
          atomicMax(m1 + f + lane, (unsigned long long)__double_as_longlong(s1));
          atomicMax(m2 + f + lane, (unsigned long long)__double_as_longlong(s2));
        }
      }
      f += 2 * l + 1;
    }
    if (MODE == kModeDensity && p < np) {
      atomicMax(m1 + p, (unsigned long long)__double_as_longlong(b1));
      atomicMax(m2 + p, (unsigned long long)__double_as_longlong(b2));
    }
  }
  __syncthreads();
  // exponents, kept in LDS as one (x1, x2) pair per slot over the max words
  for (int i = threadIdx.x; i < nslot; i += 256) {
    const int x1 = digit_exp(__longlong_as_double((long long)m1[i]));
    const int x2 = digit_exp(__longlong_as_double((long long)m2[i]));
    if (MODE == kModeDensity) {
      if (i < np) {
        ex1[d.pt_off + i] = x1;
        ex2[d.pt_off + i] = x2;
      }
    } else {
      ex1[d.col_off + i] = x1;
      ex2[d.col_off + i] = x2;
    }
    smax[i] = ((unsigned long long)(uint32_t)x2 << 32) | (uint32_t)x1;   // pair per slot
  }
  __syncthreads();
  auto exps = [&](int i, int& x1, int& x2) {
    const unsigned long long u = smax[i];
    x1 = (int)(uint32_t)u;
    x2 = (int)(uint32_t)(u >> 32);
  };

  // sweep 2: digit words
  uint64_t* o1 = slab1 + d.slab_off;
  uint64_t* o2 = slab2 + d.slab_off;
  for (int q = wq; q < na * nc; q += 4) {
    const int k = q / nc, c = q - k * nc;
    const int atom = batch_atoms[d.atom_off + k];
    const int col0 = batch_acol[d.atom_off + k];
    const SpeciesDesc sd = species[atom_species[atom]];
    const int p = 64 * c + lane;
    if (p >= ldp) continue;
    double w = 0.0, wv = 0.0, r = 1e300, dx = 0.0, dy = 0.0, dz = 0.0;
    if (p < np) {
      const double4 P4 = pts[d.pt_off + p];
      dx = P4.x - atom_xyz[3 * atom];
      dy = P4.y - atom_xyz[3 * atom + 1];
      dz = P4.z - atom_xyz[3 * atom + 2];
      r = sqrt(dx * dx + dy * dy + dz * dz);
      w = P4.w;
      if (MODE == kModeH) wv = P4.w * v[perm[d.pt_off + p]];
    }
    const bool in = r < rg.rc;
    if (!in) {
      for (int f = 0; f < sd.nfn; ++f) {
        o1[(size_t)(col0 + f) * ldp + p] = 0ull;
        o2[(size_t)(col0 + f) * ldp + p] = 0ull;
      }
      continue;
    }
    const double rr = fmax(r, 1e-12);
    const double inv = 1.0 / rr;
    const double ux = dx * inv, uy = dy * inv, uz = dz * inv;
    const RadialPos rp = radial_pos(rr, rg);
    const double* cf = spline + sd.spline_off + (size_t)rp.k * sd.nshell * 8;
    int pe1 = 0, pe2 = 0;
    if (MODE == kModeDensity) exps(p, pe1, pe2);
    int f = col0;
    for (int j = 0; j < sd.nshell; ++j) {
      const int l = shell_l[sd.shell_l_off + j];
      const double R = cubic(cf + j * 8, rp.dt);
      const double K = cubic(cf + j * 8 + 4, rp.dt);
      const int fe = MODE == kModeDensity ? shell_fexp[sd.shell_l_off + j] : 0;
      double Y[7];
      ylm_l<double>(l, ux, uy, uz, Y);
      for (int m = 0; m < 2 * l + 1; ++m) {
        const double phi = R * Y[m], tphi = K * Y[m];
        double second;
        if (MODE == kModeDensity) second = tphi;
        else if (MODE == kModeH) second = wv * phi + w * tphi;
        else second = w * phi;
        int x1 = pe1, x2 = pe2;
        if (MODE != kModeDensity) exps(f + m, x1, x2);
        o1[(size_t)(f + m) * ldp + p] = to_digits(MODE == kModeDensity ? ldexp(phi, -fe) : phi, x1);
        // the density pass reads t phi only in its FP64 epilogue: kept as FP64 bits
        o2[(size_t)(f + m) * ldp + p] =
            MODE == kModeDensity ? (uint64_t)__double_as_longlong(second) : to_digits(second, x2);
      }
      f += 2 * l + 1;
    }
  }
}

// ------------------------------------------------------------------------------------------
// Tiled kernels: 256 threads = 4 waves, a 2 x 2 arrangement of 32 x 32 blocks over a 64 x 64
// output tile; K chunks of 32, staged through a double-buffered LDS tile (28 KiB per stage) with
// one barrier per chunk.  Staging threads load eight consecutive K elements (64-bit digit words)
// and split them into digit planes before the LDS store.
// ------------------------------------------------------------------------------------------
// Density: X^T[j][p] = sum_i P_b[j][i] Phi^T[i][p] for 64 functions j and 64 points p.
__device__ __forceinline__ void
density_i8_tile(int item, const TileItem* __restrict__ items, const BatchDesc* __restrict__ batches,
                const SystemDesc* __restrict__ systems, const double4* __restrict__ pts,
                const int32_t* __restrict__ batch_cols, const uint64_t* __restrict__ P8,
                const int32_t* __restrict__ eP, const uint64_t* __restrict__ slab1,
                const uint64_t* __restrict__ slab2, const int32_t* __restrict__ ex1,
                const int32_t* __restrict__ ex2, const int32_t* __restrict__ fexp,
                double* __restrict__ n_sorted, double* __restrict__ et_batch,
                uint64_t* __restrict__ lds, int* __restrict__ rowc) {
  const TileItem it = items[item];
  const BatchDesc d = batches[it.batch];
  const SystemDesc sys = systems[d.sys];
  const int nb = d.n_b, ldp = d.ldp;
  const int j0 = it.ti * 64, p0 = it.tj * 64;
  const int* cols = batch_cols + d.col_off;
  const uint64_t* S1 = slab1 + d.slab_off;
  const uint64_t* S2 = slab2 + d.slab_off;
  const uint64_t* Pm = P8 + sys.mat_off;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const bool live = j0 + 32 * wm < nb && p0 + 32 * wn < d.n_p;   // block holds outputs

  v16i acc[kLevelsD];
#pragma unroll
  for (int L = 0; L < kLevelsD; ++L) acc[L] = v16i{};

  // the epilogue's row constants, read once per tile: exponent of the row of P, and that plus
  // the row's balancing exponent (ordered before the epilogue by the K loop's barriers)
  if (tid < 64) {
    const int j = j0 + tid;
    const int gj = (int)sys.row_off + cols[j < nb ? j : 0];
    rowc[tid] = eP[gj];
    rowc[64 + tid] = eP[gj] + fexp[gj];
  }

  // A staging: row ra = tid / 4, k octet ka = tid % 4 (gathered P words; the batch's column
  // list starts 16-byte aligned and is padded, so its indices come in two 16-byte loads)
  const int ra = tid >> 2, ka = tid & 3;
  const bool rok = j0 + ra < nb;
  const uint32_t prow = (uint32_t)cols[rok ? j0 + ra : 0] * (uint32_t)sys.nb;
  // B staging: point pb = tid % 64, k octet kb = tid / 64 (coalesced slab rows)
  const int pb = tid & 63, kb = tid >> 6;
  const bool pok = p0 + pb < ldp;
  uint64_t av[8], bv[8];
  auto fetch = [&](int kc) {
    const int4 c0 = *reinterpret_cast<const int4*>(cols + kc + 8 * ka);
    const int4 c1 = *reinterpret_cast<const int4*>(cols + kc + 8 * ka + 4);
    const int ci[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int k = kc + 8 * ka + m;
      const bool ok = rok && k < nb;
      const uint64_t x = Pm[prow + (uint32_t)(k < nb ? ci[m] : cols[0])];
      av[m] = ok ? x : 0ull;
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int k = kc + 8 * kb + m;
      const bool ok = pok && k < nb;
      const uint64_t x = S1[(size_t)(k < nb ? k : nb - 1) * ldp + (pok ? p0 + pb : 0)];
      bv[m] = ok ? x : 0ull;
    }
  };
  auto stash = [&](int buf) {
    uint64_t* As = lds + buf * 2 * kOpWords;
    uint64_t* Bs = As + kOpWords;
    uint64_t pa[kDigits], pbv[kDigits];
    digit_planes(av, pa);
    digit_planes(bv, pbv);
#pragma unroll
    for (int s = 0; s < kDigits; ++s) {
      As[op_index(s, ka >> 1, ra, ka & 1)] = pa[s];
      Bs[op_index(s, kb >> 1, pb, kb & 1)] = pbv[s];
    }
  };
  const int nchunk = (nb + kKI - 1) / kKI;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) fetch((c + 1) * kKI);
    if (live) {
      const uint64_t* As = lds + buf * 2 * kOpWords;
      multiply_levels<kLevelsD>(As, As + kOpWords, lane, 32 * wm, 32 * wn, acc);
    }
    if (c + 1 < nchunk) stash(buf ^ 1);
    __syncthreads();
  }

  // epilogue: n_p += sum_j X_jp phi_jp, E_T partial sum_p w_p sum_j X_jp tphi_jp (FP64)
  double* red = reinterpret_cast<double*>(lds);       // [2][64] column sums, [4] energies
  const int p = p0 + 32 * wn + (lane & 31);
  double sn = 0.0, se = 0.0;
  if (live && p < d.n_p) {
    const int e1 = ex1[d.pt_off + p];
    uint64_t f1[16], f2[16];             // the epilogue's basis digits, loaded together
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int j = j0 + 32 * wm + acc_row32(lane, r);
      const size_t o = (size_t)(j < nb ? j : 0) * ldp + p;
      f1[r] = S1[o];
      f2[r] = S2[o];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int jl = 32 * wm + acc_row32(lane, r);
      if (j0 + jl < nb) {
        const double x = level_sum<kLevelsD>(acc, r);
        // X phi = 2^(eP + e1) x * 2^(e1 + f) digits(phi);  X t phi = 2^(eP + e1) x * t phi (FP64)
        sn += ldexp(x * from_digits(f1[r], 0), rowc[64 + jl] + 2 * e1);
        se += ldexp(x * __longlong_as_double((long long)f2[r]), rowc[jl] + e1);
      }
    }
    se *= pts[d.pt_off + p].w;
  }
  sn += __shfl_xor(sn, 32);
  for (int o = 32; o > 0; o >>= 1) se += __shfl_xor(se, o);
  if (lane < 32) red[wm * 64 + 32 * wn + lane] = sn;
  if (lane == 0) red[128 + wave] = se;
  __syncthreads();
  if (tid < 64 && p0 + tid < d.n_p)
    unsafeAtomicAdd(n_sorted + d.pt_off + p0 + tid, red[tid] + red[64 + tid]);
  if (tid == 0) unsafeAtomicAdd(et_batch + it.batch, (red[128] + red[129]) + (red[130] + red[131]));
}

__global__ void __launch_bounds__(256, 2)
density_i8_kernel(const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
                  const SystemDesc* __restrict__ systems, const double4* __restrict__ pts,
                  const int32_t* __restrict__ batch_cols, const uint64_t* __restrict__ P8,
                  const int32_t* __restrict__ eP, const uint64_t* __restrict__ slab1,
                  const uint64_t* __restrict__ slab2, const int32_t* __restrict__ ex1,
                  const int32_t* __restrict__ ex2, const int32_t* __restrict__ fexp,
                  double* __restrict__ n_sorted, double* __restrict__ et_batch,
                  int* __restrict__ queue) {
  __shared__ __attribute__((aligned(16))) uint64_t lds[4 * kOpWords];
  __shared__ int rowc[128];
  run_items(n_items, queue, [&](int item) {
    density_i8_tile(item, items, batches, systems, pts, batch_cols, P8, eP, slab1, slab2, ex1, ex2,
                    fexp, n_sorted, et_batch, lds, rowc);
  });
}

// H / S: C[i][j] = sum_p slab1[i][p] slab2[j][p] over the batch's points, FP64 scatter-add.
__device__ __forceinline__ void
hs_i8_tile(int item, const TileItem* __restrict__ items, const BatchDesc* __restrict__ batches,
           const SystemDesc* __restrict__ systems, const int32_t* __restrict__ batch_cols,
           const uint64_t* __restrict__ slab1, const uint64_t* __restrict__ slab2,
           const int32_t* __restrict__ ex1, const int32_t* __restrict__ ex2,
           double* __restrict__ out, uint64_t* __restrict__ lds, int* __restrict__ rowc) {
  const TileItem it = items[item];
  const BatchDesc d = batches[it.batch];
  const SystemDesc sys = systems[d.sys];
  const int nb = d.n_b, ldp = d.ldp;
  const int i0 = it.ti * 64, jb = it.tj * 64;
  const int* cols = batch_cols + d.col_off;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const bool live = i0 + 32 * wm < nb && jb + 32 * wn < nb;

  v16i acc[kLevelsH];
#pragma unroll
  for (int L = 0; L < kLevelsH; ++L) acc[L] = v16i{};
  if (tid < 64) {                       // row constants of the epilogue: H row, exponent
    const int i = i0 + tid < nb ? i0 + tid : 0;
    rowc[tid] = cols[i];
    rowc[64 + tid] = ex1[d.col_off + i];
  }

  // staging: row r = tid / 4 of both operands, point octet q = tid % 4 (64 contiguous bytes)
  const int r = tid >> 2, q = tid & 3;
  const bool a_ok = i0 + r < nb, b_ok = jb + r < nb;
  const uint64_t* Ap = slab1 + d.slab_off + (size_t)(a_ok ? i0 + r : 0) * ldp + 8 * q;
  const uint64_t* Bp = slab2 + d.slab_off + (size_t)(b_ok ? jb + r : 0) * ldp + 8 * q;
  uint64_t av[8], bv[8];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const ulonglong2 x = *reinterpret_cast<const ulonglong2*>(Ap + kc + 2 * h);
      const ulonglong2 y = *reinterpret_cast<const ulonglong2*>(Bp + kc + 2 * h);
      av[2 * h] = a_ok ? x.x : 0ull;
      av[2 * h + 1] = a_ok ? x.y : 0ull;
      bv[2 * h] = b_ok ? y.x : 0ull;
      bv[2 * h + 1] = b_ok ? y.y : 0ull;
    }
  };
  auto stash = [&](int buf) {
    uint64_t* As = lds + buf * 2 * kOpWords;
    uint64_t* Bs = As + kOpWords;
    uint64_t pa[kDigits], pbv[kDigits];
    digit_planes(av, pa);
    digit_planes(bv, pbv);
#pragma unroll
    for (int s = 0; s < kDigits; ++s) {
      As[op_index(s, q >> 1, r, q & 1)] = pa[s];
      Bs[op_index(s, q >> 1, r, q & 1)] = pbv[s];
    }
  };
  const int nchunk = ldp / kKI;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) fetch((c + 1) * kKI);
    if (live) {
      const uint64_t* As = lds + buf * 2 * kOpWords;
      multiply_levels<kLevelsH>(As, As + kOpWords, lane, 32 * wm, 32 * wn, acc);
    }
    if (c + 1 < nchunk) stash(buf ^ 1);
    __syncthreads();
  }
  if (!live) return;
  const int j = jb + 32 * wn + (lane & 31);
  if (j >= nb) return;
  double* O = out + sys.mat_off;
  const size_t gj = (size_t)cols[j];
  const int ej = ex2[d.col_off + j];
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    const int il = 32 * wm + acc_row32(lane, rr);
    if (i0 + il < nb)
      unsafeAtomicAdd(O + (size_t)rowc[il] * sys.nb + gj,
                      ldexp(level_sum<kLevelsH>(acc, rr), rowc[64 + il] + ej));
  }
}

__global__ void __launch_bounds__(256, 2)
hs_i8_kernel(const TileItem* __restrict__ items, int n_items, const BatchDesc* __restrict__ batches,
             const SystemDesc* __restrict__ systems, const int32_t* __restrict__ batch_cols,
             const uint64_t* __restrict__ slab1, const uint64_t* __restrict__ slab2,
             const int32_t* __restrict__ ex1, const int32_t* __restrict__ ex2,
             double* __restrict__ out, int* __restrict__ queue) {
  __shared__ __attribute__((aligned(16))) uint64_t lds[4 * kOpWords];
  __shared__ int rowc[128];
  run_items(n_items, queue, [&](int item) {
    hs_i8_tile(item, items, batches, systems, batch_cols, slab1, slab2, ex1, ex2, out, lds, rowc);
  });
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
hipError_t launch_slice_p(const DeviceView& dv, const double* P, uint64_t* P8, int32_t* eP,
                          int64_t n_rows, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(slice_p_kernel, dim3((unsigned)n_rows), dim3(256), 0, st, P, P8, eP, dv.systems,
                     dv.n_sys, dv.fn_fexp);
  return hipGetLastError();
}

hipError_t launch_phi_eval_i8(const DeviceView& dv, int b0, int nbatch, int mode, const double* v,
                              uint64_t* slab1, uint64_t* slab2, int32_t* ex1, int32_t* ex2,
                              int max_slots, hipStream_t st) {
  if (nbatch == 0) return hipSuccess;
  const size_t shmem = 2 * (size_t)max_slots * sizeof(unsigned long long);
  if (shmem > 64 * 1024) return hipErrorInvalidValue;
  switch (mode) {
    case kModeDensity:
      hipLaunchKernelGGL(phi_eval_i8_kernel<kModeDensity>, dim3(nbatch), dim3(256), shmem, st,
                         dv.batches, b0, dv.pts, dv.perm, dv.batch_atoms, dv.batch_acol, dv.atom_xyz,
                         dv.atom_species, dv.species, dv.shell_l, dv.shell_fexp, dv.spline64, dv.rg, v,
                         slab1, slab2, ex1, ex2);
      break;
    case kModeH:
      hipLaunchKernelGGL(phi_eval_i8_kernel<kModeH>, dim3(nbatch), dim3(256), shmem, st,
                         dv.batches, b0, dv.pts, dv.perm, dv.batch_atoms, dv.batch_acol, dv.atom_xyz,
                         dv.atom_species, dv.species, dv.shell_l, dv.shell_fexp, dv.spline64, dv.rg, v,
                         slab1, slab2, ex1, ex2);
      break;
    default:
      hipLaunchKernelGGL(phi_eval_i8_kernel<kModeS>, dim3(nbatch), dim3(256), shmem, st,
                         dv.batches, b0, dv.pts, dv.perm, dv.batch_atoms, dv.batch_acol, dv.atom_xyz,
                         dv.atom_species, dv.species, dv.shell_l, dv.shell_fexp, dv.spline64, dv.rg, v,
                         slab1, slab2, ex1, ex2);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_density_i8(const DeviceView& dv, const TileItem* items, int n_items,
                             const uint64_t* P8, const int32_t* eP, const uint64_t* slab1,
                             const uint64_t* slab2, const int32_t* ex1, const int32_t* ex2,
                             double* n_sorted, double* et_batch, hipStream_t st, Queue q) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(density_i8_kernel, dim3(tile_grid(n_items, q, (const void*)density_i8_kernel)),
                     dim3(256), 0, st, items, n_items, dv.batches, dv.systems, dv.pts, dv.batch_cols,
                     P8, eP, slab1, slab2, ex1, ex2, dv.fn_fexp, n_sorted, et_batch, q.counters);
  return hipGetLastError();
}

hipError_t launch_hs_i8(const DeviceView& dv, const TileItem* items, int n_items, const uint64_t* slab1,
                        const uint64_t* slab2, const int32_t* ex1, const int32_t* ex2, double* out,
                        hipStream_t st, Queue q) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(hs_i8_kernel, dim3(tile_grid(n_items, q, (const void*)hs_i8_kernel)), dim3(256), 0,
                     st, items, n_items, dv.batches, dv.systems, dv.batch_cols, slab1, slab2, ex1, ex2,
                     out, q.counters);
  return hipGetLastError();
}

hipError_t prepare_launch_configs_i8() {
  const void* fns[] = {(const void*)density_i8_kernel, (const void*)hs_i8_kernel};
  for (const void* f : fns)
    if (resident_workgroups(f) <= 0) return hipErrorInvalidDeviceFunction;
  return hipSuccess;
}

}  // namespace aims
