// Density matrix of the occupied subspace from H and S (the step after the H integration):
// device kernels (scf.hip) and the host-side solver (scf.cpp).  All matrices here are n x n,
// symmetric on input and output; the solver works in rocBLAS's column-major convention
// internally (for a symmetric matrix the two conventions coincide).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace aims {

// A = (H + H^T) / 2
hipError_t launch_sym_part(const double* H, double* A, int n, hipStream_t st);
// column k of the column-major V (k < m) times s[k]
hipError_t launch_scale_cols(double* V, const double* s, int m, int n, hipStream_t st);
// copy the lower triangle of the column-major P onto its upper triangle
hipError_t launch_mirror_lower(double* P, int n, hipStream_t st);
// zero the strictly upper triangle of the column-major L
hipError_t launch_zero_upper(double* L, int n, hipStream_t st);
// Gershgorin bounds of the symmetric X: out[0] = min_i (X_ii - r_i), out[1] = max_i (X_ii + r_i)
hipError_t launch_gershgorin(const double* X, int n, double* rows, double* out, hipStream_t st);
// X = (emax I - (Hp + Hp^T) / 2) / (emax - emin) with (emin, emax) = bounds[0..1] on the
// device, written as the leading n x n block of the ld x ld column-major X (zero elsewhere)
hipError_t launch_purify_init(const double* Hp, double* X, int n, int ld, const double* bounds,
                              hipStream_t st);
// Purification tiles (64 x 64, on and below the diagonal) of an ld x ld matrix, ld % 64 == 0;
// each tile leaves two doubles (its shares of the trace and of the squared Frobenius norm)
int purify_tiles(int ld);
// the shares of the starting X into part[2 purify_tiles(ld)]; resets the convergence state[2]
hipError_t launch_purify_partials(const double* X, int ld, double* part, double* state,
                                  hipStream_t st);
// *flag = 1 if the n doubles at a and b differ in any bit, else 0
hipError_t launch_differ(const double* a, const double* b, size_t n, int* flag, hipStream_t st);
// out[0] = bits of max |P_ij - P_ji|, out[1] = bits of max |P_ij| over the n x n row-major block P
// (out[0] = bits of +inf if an entry is not finite); out is cleared first
hipError_t launch_asym_max(const double* P, int n, unsigned long long* out, hipStream_t st);
// Work split of one product: tiles [0, n_full) whole, the remaining tiles in ks K parts each
// (ks >= 2, at most `cus` parts in all), summed by a second kernel
struct PurifyPlan {
  int tiles = 0, n_full = 0, ks = 1;
};
PurifyPlan purify_plan(int ld, int cus);
// Product `it` of the trace-correcting purification on the symmetric X (shares in part_in):
// Y = X^2 if tr X > n_occ, else Y = 2 X - X^2; the shares of Y go to part_out, tr X and
// ||X||_F^2 to hist[2 it], [2 it + 1].  W holds 4096 (tiles - n_full) ks doubles of partial sums.
// Convergence is decided on the device (state[2], reset by launch_purify_partials): once the
// input of a product is final (idempotency error below tol three products earlier), state[1]
// holds the number of products done and this and every later product return at once, so the
// final X is the input of product state[1].
hipError_t launch_purify_step(const double* X, double* Y, int ld, double n_occ,
                              const double* part_in, double* part_out, const PurifyPlan& p,
                              double* W, double* hist, int it, double tol, double* state,
                              hipStream_t st);

// Solver driver state: a rocBLAS handle on the stream and device buffers grown as needed.
struct DmSolver {
  void* blas = nullptr;           // rocblas_handle
  hipStream_t stream = nullptr;
  size_t cap = 0;                 // doubles per n x n buffer
  double* A = nullptr;
  double* B = nullptr;
  double* X = nullptr;
  double* Y = nullptr;
  double* T = nullptr;
  double* vec = nullptr;          // [n]: eigenvalues, scale factors, Gershgorin rows
  double* vec2 = nullptr;         // [n]: tridiagonal off-diagonals
  double* small = nullptr;        // [1024]: bounds, coefficients, history, partials
  double* part = nullptr;         // [4 purify_tiles(ld)]: two generations of purification shares
  double* W = nullptr;            // [4096 cus]: partial sums of the split purification tiles
  double* Lk = nullptr;           // L^{-1} of the overlap Sk (kept between calls)
  double* Sk = nullptr;           // the overlap matrix Lk belongs to
  int k_n = 0;                    // order of Sk / Lk (0: none kept)
  int last_factored = 0;          // 1 if the last purification factorised S, 0 if it reused Lk
  int cus = 0;                    // compute units of the device
  int ld = 0;                     // leading dimension of X and Y (n rounded up to 64)
  int* info = nullptr;
  int last_iterations = 0;        // purification iterations of the last system
};

enum { kDmEigen = 0, kDmPurify = 1 };

// One system: P (n x n) from H, S with n_elec electrons; eps_or_null receives the ascending
// eigenvalues (eigen method), mu the chemical potential.  Returns 0 on success, otherwise a
// status code (negative, as in aims_status) with a message in err.
int dm_solve(DmSolver& s, int method, int n, const double* H, const double* S, double n_elec,
             double kT, double* P, double* eps_or_null, double* mu, std::string& err);
void dm_release(DmSolver& s);

}  // namespace aims
