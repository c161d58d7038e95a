// Density matrix of the occupied subspace from H and S, per system:
//
//   H_s = (H + H^T) / 2,   H_s C = S C diag(eps),   C^T S C = I,   P = C diag(f) C^T
//
// Two methods.
//  * Eigen: the generalised symmetric-definite eigensolver of rocSOLVER (sygvd: Cholesky
//    reduction and divide and conquer), occupations on the host (aufbau, or Fermi-Dirac with the
//    chemical potential found by bisection), then P = V V^T with V = C diag(sqrt f) on the
//    occupied columns (one rank-k update).
//  * Purify: no eigenvectors at all.  S = L L^T (Cholesky), H' = L^{-1} H_s L^{-T}, and the
//    spectral projector onto the N_e / 2 lowest states of H' by trace-correcting purification:
//    X_0 = (e_max I - H') / (e_max - e_min) from Gershgorin bounds, then repeatedly X <- X^2 when
//    tr X exceeds N_e / 2 and X <- 2 X - X^2 otherwise, until X^2 = X; P = 2 L^{-T} X L^{-1}.
//    Every step is one fused kernel (the symmetric product on the FP64 matrix cores, with the
//    choice between the two polynomials taken on the device from the trace the previous step
//    left), and the device also decides when to stop, so the host only reads a flag every few
//    products.  L^{-1} is kept between calls and reused while S is unchanged.  It needs an even
//    electron count, aufbau occupations and a gap at the Fermi level.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "scf.h"

namespace aims {

namespace {

constexpr int kStatusArg = -1, kStatusOom = -2, kStatusHip = -3, kStatusUnsupported = -5;
constexpr int kMaxPurify = 160;        // purification products before giving up
constexpr int kBatch = 8;              // products launched between reads of the device state

// layout of DmSolver::small
constexpr int kBounds = 0, kState = 4, kHist = 8;

int fail_msg(std::string& err, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  err = buf;
  return code;
}

#define DM_HIP(x, what)                                                              \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) return fail_msg(err, kStatusHip, "%s: %s", what, hipGetErrorString(e_)); \
  } while (0)
#define DM_BLAS(x, what)                                                              \
  do {                                                                                \
    rocblas_status s_ = (x);                                                          \
    if (s_ != rocblas_status_success)                                                 \
      return fail_msg(err, s_ == rocblas_status_memory_error ? kStatusOom : kStatusHip, \
                      "%s: %s", what, rocblas_status_to_string(s_));                  \
  } while (0)

void free_matrices(DmSolver& s) {
  for (double** p : {&s.A, &s.B, &s.X, &s.Y, &s.T, &s.vec, &s.vec2, &s.part, &s.W, &s.Lk, &s.Sk}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  s.k_n = 0;
  s.cap = 0;
}

int ensure(DmSolver& s, int n, std::string& err) {
  if (!s.blas) {
    rocblas_handle h = nullptr;
    DM_BLAS(rocblas_create_handle(&h), "rocblas_create_handle");
    s.blas = h;
  }
  DM_BLAS(rocblas_set_stream((rocblas_handle)s.blas, s.stream), "rocblas_set_stream");
  if (!s.cus) {
    int dev = 0;
    DM_HIP(hipGetDevice(&dev), "hipGetDevice");
    DM_HIP(hipDeviceGetAttribute(&s.cus, hipDeviceAttributeMultiprocessorCount, dev), "device attribute");
  }
  // every work matrix holds ld x ld (X and Y of the purification use that leading dimension)
  const int ld = (n + 63) / 64 * 64;
  const size_t need = std::max<size_t>(1, (size_t)ld * ld);
  if (need > s.cap) {
    free_matrices(s);
    bool ok = true;
    for (double** p : {&s.A, &s.B, &s.X, &s.Y, &s.T, &s.Lk, &s.Sk})
      ok = ok && hipMalloc(p, need * sizeof(double)) == hipSuccess;
    for (double** p : {&s.vec, &s.vec2})
      ok = ok && hipMalloc(p, 2 * std::max<size_t>(1, (size_t)ld) * sizeof(double)) == hipSuccess;
    const size_t nt = (size_t)std::max(1, purify_tiles(ld));
    ok = ok && hipMalloc(&s.part, 4 * nt * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&s.W, 4096 * (size_t)std::max(8, s.cus) * sizeof(double)) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      free_matrices(s);
      return fail_msg(err, kStatusOom, "device allocation of %d x %d work matrices failed", n, n);
    }
    s.cap = need;
  }
  if ((!s.small && hipMalloc(&s.small, 1024 * sizeof(double)) != hipSuccess) ||
      (!s.info && hipMalloc(&s.info, sizeof(int)) != hipSuccess)) {
    (void)hipGetLastError();
    return fail_msg(err, kStatusOom, "device allocation failed");
  }
  return 0;
}

// aufbau or Fermi-Dirac occupations of ascending eigenvalues (spin-restricted, f in [0, 2])
int occupations(const std::vector<double>& eps, double n_elec, double kT, std::vector<double>& f,
                double& mu, std::string& err) {
  const int n = (int)eps.size();
  f.assign(n, 0.0);
  if (!(n_elec >= 0.0 && n_elec <= 2.0 * n))
    return fail_msg(err, kStatusArg, "%g electrons do not fit %d states", n_elec, n);
  if (kT == 0.0) {
    const int full = (int)std::floor(n_elec / 2.0);
    for (int k = 0; k < full; ++k) f[k] = 2.0;
    const double rest = n_elec - 2.0 * full;
    if (rest > 0.0) f[full] = rest;
    if (rest > 0.0) {
      mu = eps[full];
    } else if (full > 0 && full < n) {
      mu = 0.5 * (eps[full - 1] + eps[full]);
    } else {
      mu = full == 0 ? (n ? eps[0] : 0.0) : eps[n - 1];
    }
    return 0;
  }
  auto fermi = [&](double m, bool fill) {
    double sum = 0.0;
    for (int k = 0; k < n; ++k) {
      const double x = (eps[k] - m) / kT;
      const double v = x > 0 ? 2.0 * std::exp(-x) / (1.0 + std::exp(-x)) : 2.0 / (1.0 + std::exp(x));
      if (fill) f[k] = v;
      sum += v;
    }
    return sum;
  };
  if (n_elec == 0.0) {
    mu = -HUGE_VAL;
    return 0;
  }
  if (n_elec == 2.0 * n) {
    for (auto& x : f) x = 2.0;
    mu = HUGE_VAL;
    return 0;
  }
  double a = eps[0] - 50.0 * kT - 1.0, b = eps[n - 1] + 50.0 * kT + 1.0;
  while (fermi(a, false) > n_elec) a -= (b - a);
  while (fermi(b, false) < n_elec) b += (b - a);
  for (int it = 0; it < 2000; ++it) {
    const double m = 0.5 * (a + b);
    if (m == a || m == b) break;
    if (fermi(m, false) < n_elec) a = m;
    else b = m;
  }
  mu = 0.5 * (a + b);
  fermi(mu, true);
  return 0;
}

int solve_eigen(DmSolver& s, int n, double n_elec, double kT, double* P, double* eps_out,
                double* mu, std::string& err) {
  rocblas_handle h = (rocblas_handle)s.blas;
  DM_BLAS(rocblas_set_pointer_mode(h, rocblas_pointer_mode_host), "pointer mode");
  // s.A = H_s (already), s.B = S (already): A <- C (columns = eigenvectors), vec <- eps
  DM_BLAS(rocsolver_dsygvd(h, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_upper, n, s.A,
                           n, s.B, n, s.vec, s.vec2, s.info),
          "rocsolver_dsygvd");
  int info = 0;
  std::vector<double> eps(n);
  DM_HIP(hipMemcpyAsync(&info, s.info, sizeof(int), hipMemcpyDeviceToHost, s.stream), "read info");
  DM_HIP(hipMemcpyAsync(eps.data(), s.vec, n * sizeof(double), hipMemcpyDeviceToHost, s.stream),
         "read eigenvalues");
  DM_HIP(hipStreamSynchronize(s.stream), "synchronize");
  if (info > n)
    return fail_msg(err, kStatusArg, "S is not positive definite (leading minor %d)", info - n);
  if (info != 0) return fail_msg(err, kStatusHip, "eigensolver did not converge (info %d)", info);
  std::vector<double> f;
  int rc = occupations(eps, n_elec, kT, f, *mu, err);
  if (rc) return rc;
  if (eps_out)
    DM_HIP(hipMemcpyAsync(eps_out, s.vec, n * sizeof(double), hipMemcpyDeviceToDevice, s.stream),
           "copy eigenvalues");
  int m = 0;                                       // occupied columns (f descending from the bottom)
  for (int k = 0; k < n; ++k)
    if (f[k] > 0.0) m = k + 1;
  std::vector<double> sf(std::max(1, m));
  for (int k = 0; k < m; ++k) sf[k] = std::sqrt(f[k]);
  if (m == 0) {
    DM_HIP(hipMemsetAsync(P, 0, (size_t)n * n * sizeof(double), s.stream), "clear P");
    return 0;
  }
  DM_HIP(hipMemcpyAsync(s.vec2, sf.data(), m * sizeof(double), hipMemcpyHostToDevice, s.stream),
         "upload occupations");
  DM_HIP(launch_scale_cols(s.A, s.vec2, m, n, s.stream), "scale");
  const double one = 1.0, zero = 0.0;
  // P = V V^T (lower triangle), V = A[:, :m] column-major n x m
  DM_BLAS(rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_none, n, m, &one, s.A, n, &zero, P,
                        n),
          "rocblas_dsyrk");
  DM_HIP(launch_mirror_lower(P, n, s.stream), "mirror");
  // the host vectors above must outlive the asynchronous copies
  DM_HIP(hipStreamSynchronize(s.stream), "synchronize");
  return 0;
}

// L^{-1} of S (lower, upper triangle zero) in s.Lk.  It is kept: while S is bitwise the matrix
// it came from (the overlap changes only with the geometry, so in an s.c.f. loop every iteration
// after the first) the Cholesky factorisation and the triangular inverse are skipped.
int inverse_factor(DmSolver& s, int n, const double* S, std::string& err) {
  rocblas_handle h = (rocblas_handle)s.blas;
  const size_t elems = (size_t)n * n;
  if (s.k_n == n) {
    DM_HIP(launch_differ(S, s.Sk, elems, s.info, s.stream), "compare S");
    int differ = 1;
    DM_HIP(hipMemcpyAsync(&differ, s.info, sizeof(int), hipMemcpyDeviceToHost, s.stream), "read flag");
    DM_HIP(hipStreamSynchronize(s.stream), "synchronize");
    if (!differ) {
      s.last_factored = 0;
      return 0;
    }
  }
  s.k_n = 0;
  s.last_factored = 1;
  DM_HIP(hipMemcpyAsync(s.Lk, S, elems * sizeof(double), hipMemcpyDeviceToDevice, s.stream), "copy S");
  DM_BLAS(rocblas_set_pointer_mode(h, rocblas_pointer_mode_host), "pointer mode");
  // S = L L^T (lower, column-major), then L <- L^{-1} with the upper triangle cleared
  DM_BLAS(rocsolver_dpotrf(h, rocblas_fill_lower, n, s.Lk, n, s.info), "rocsolver_dpotrf");
  int info = 0;
  DM_HIP(hipMemcpyAsync(&info, s.info, sizeof(int), hipMemcpyDeviceToHost, s.stream), "read info");
  DM_HIP(hipStreamSynchronize(s.stream), "synchronize");
  if (info != 0) return fail_msg(err, kStatusArg, "S is not positive definite (leading minor %d)", info);
  DM_BLAS(rocsolver_dtrtri(h, rocblas_fill_lower, rocblas_diagonal_non_unit, n, s.Lk, n, s.info),
          "rocsolver_dtrtri");
  DM_HIP(launch_zero_upper(s.Lk, n, s.stream), "clear triangle");
  DM_HIP(hipMemcpyAsync(s.Sk, S, elems * sizeof(double), hipMemcpyDeviceToDevice, s.stream), "keep S");
  s.k_n = n;
  return 0;
}

int solve_purify(DmSolver& s, int n, const double* S, double n_elec, double kT, double* P,
                 double* mu, std::string& err) {
  if (kT != 0.0) return fail_msg(err, kStatusUnsupported, "purification takes aufbau occupations (kT = 0)");
  const double n_occ = 0.5 * n_elec;
  if (n_occ != std::floor(n_occ))
    return fail_msg(err, kStatusUnsupported, "purification needs an even electron count (got %g)", n_elec);
  if (n_occ < 0 || n_occ > n) return fail_msg(err, kStatusArg, "%g electrons do not fit %d states", n_elec, n);
  rocblas_handle h = (rocblas_handle)s.blas;
  const double one = 1.0, zero = 0.0, two = 2.0;
  const size_t bytes = (size_t)n * n * sizeof(double);
  *mu = NAN;
  s.last_iterations = 0;
  if (n_occ == 0) {
    DM_HIP(hipMemsetAsync(P, 0, bytes, s.stream), "clear P");
    return 0;
  }
  int rc = inverse_factor(s, n, S, err);
  if (rc) return rc;
  const double* Li = s.Lk;
  DM_BLAS(rocblas_set_pointer_mode(h, rocblas_pointer_mode_host), "pointer mode");
  // H' = L^{-1} H_s L^{-T}: T = H_s L^{-T}, A = L^{-1} T
  DM_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, n, n, n, &one, s.A,
                        n, Li, n, &zero, s.T, n),
          "rocblas_dgemm");
  DM_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, Li, n,
                        s.T, n, &zero, s.A, n),
          "rocblas_dgemm");
  const int ld = (n + 63) / 64 * 64;             // X and Y: ld x ld, zero outside n x n
  double* X = s.X;
  if (n_occ == n) {                               // every state full: X = I
    DM_HIP(hipMemsetAsync(s.X, 0, (size_t)ld * ld * sizeof(double), s.stream), "clear X");
    std::vector<double> ones(n, 1.0);
    DM_HIP(hipMemcpy2DAsync(s.X, (ld + 1) * sizeof(double), ones.data(), sizeof(double),
                            sizeof(double), n, hipMemcpyHostToDevice, s.stream),
           "identity");
    DM_HIP(hipStreamSynchronize(s.stream), "synchronize");
  } else {
    double* sm = s.small;
    const int nt = purify_tiles(ld);
    double* part[2] = {s.part, s.part + 2 * nt};
    double* buf[2] = {s.X, s.Y};
    const PurifyPlan plan = purify_plan(ld, s.cus);
    const double tol = 1e-8 * std::max(1.0, n_occ);
    DM_HIP(launch_gershgorin(s.A, n, s.vec, sm + kBounds, s.stream), "bounds");
    DM_HIP(launch_purify_init(s.A, s.X, n, ld, sm + kBounds, s.stream), "purify init");
    DM_HIP(launch_purify_partials(s.X, ld, part[0], sm + kState, s.stream), "purify shares");
    // products in batches with no host round trip; the device stops the iteration itself
    double state[2] = {-1.0, -1.0};
    int it = 0;
    while (state[1] < 0.0) {
      if (it >= kMaxPurify) {
        double hist[2];
        DM_HIP(hipMemcpyAsync(hist, sm + kHist + 2 * (it - 1), sizeof(hist), hipMemcpyDeviceToHost,
                              s.stream),
               "read history");
        DM_HIP(hipStreamSynchronize(s.stream), "synchronize");
        return fail_msg(err, kStatusHip,
                        "purification did not converge in %d products (tr X %.17g, ||X||_F^2 %.17g; "
                        "no gap at the Fermi level?)",
                        kMaxPurify, hist[0], hist[1]);
      }
      const int batch = std::min(kBatch, kMaxPurify - it);
      for (int b = 0; b < batch; ++b, ++it)
        DM_HIP(launch_purify_step(buf[it & 1], buf[(it + 1) & 1], ld, n_occ, part[it & 1],
                                  part[(it + 1) & 1], plan, s.W, sm + kHist, it, tol, sm + kState,
                                  s.stream),
               "purification product");
      DM_HIP(hipMemcpyAsync(state, sm + kState, sizeof(state), hipMemcpyDeviceToHost, s.stream),
             "read state");
      DM_HIP(hipStreamSynchronize(s.stream), "synchronize");
    }
    s.last_iterations = (int)state[1];
    X = buf[s.last_iterations & 1];
  }
  // P = 2 L^{-T} X L^{-1}: T = X L^{-1}, P = 2 L^{-T} T
  DM_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, X, ld, Li,
                        n, &zero, s.T, n),
          "rocblas_dgemm");
  DM_BLAS(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, n, n, n, &two, Li,
                        n, s.T, n, &zero, s.B, n),
          "rocblas_dgemm");
  DM_HIP(launch_sym_part(s.B, P, n, s.stream), "symmetrise");
  DM_HIP(hipStreamSynchronize(s.stream), "synchronize");
  return 0;
}

}  // namespace

int dm_solve(DmSolver& s, int method, int n, const double* H, const double* S, double n_elec,
             double kT, double* P, double* eps_or_null, double* mu, std::string& err) {
  if (n <= 0) return 0;
  int rc = ensure(s, n, err);
  if (rc) return rc;
  DM_HIP(launch_sym_part(H, s.A, n, s.stream), "symmetrise");
  if (method == kDmEigen) {
    DM_HIP(hipMemcpyAsync(s.B, S, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, s.stream),
           "copy S");
    return solve_eigen(s, n, n_elec, kT, P, eps_or_null, mu, err);
  }
  if (eps_or_null) return fail_msg(err, kStatusUnsupported, "purification computes no eigenvalues");
  return solve_purify(s, n, S, n_elec, kT, P, mu, err);
}

void dm_release(DmSolver& s) {
  free_matrices(s);
  if (s.small) (void)hipFree(s.small);
  s.small = nullptr;
  if (s.info) (void)hipFree(s.info);
  s.info = nullptr;
  if (s.blas) rocblas_destroy_handle((rocblas_handle)s.blas);
  s.blas = nullptr;
}

}  // namespace aims
