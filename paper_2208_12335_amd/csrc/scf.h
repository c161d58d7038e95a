// Density matrix of the occupied subspace from H and S (the step after the H integration):
// device kernels (scf.hip) and the solver driver (scf.cpp).  All matrices here are n x n,
// symmetric on input and output; the driver works in rocBLAS's column-major convention
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
// X = (emax I - Hp) / (emax - emin) with (emin, emax) = bounds[0..1] on the device
hipError_t launch_purify_init(const double* Hp, double* X, int n, const double* bounds,
                              hipStream_t st);
// One trace-correcting purification decision: trace t = tr(X), stored in hist[2 it]; the
// product coefficients ab = (1, 0) if t > n_occ (X <- X^2) else (-1, 2) (X <- 2 X - X^2)
hipError_t launch_purify_coef(const double* X, int n, double n_occ, double* ab, double* hist,
                              int it, hipStream_t st);
// hist[2 it + 1] = ||X||_F^2 (partials in `part`, one per workgroup)
hipError_t launch_frob2(const double* X, int n, double* part, double* hist, int it,
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
