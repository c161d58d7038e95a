/*
 * aims_grid.h -- C ABI of the MI355X NAO real-space grid-integration library.
 *
 * The library evaluates, for spatially compact batches of integration points, the nonzero
 * numeric atom-centred basis functions phi_i = R_s(r) Y_lm(r^) (cubic-spline radial function
 * times real spherical harmonic, l <= 3) and their kinetic terms t phi_i = -1/2 Laplacian phi_i
 * = K_s(r) Y_lm(r^), and from them
 *
 *     n(p)  = sum_ij P_ij phi_i(p) phi_j(p)                           (aims_update_density)
 *     H_ij  = sum_p w_p phi_i(p) [v(p) phi_j(p) + t phi_j(p)]           (aims_integrate_h)
 *     S_ij  = sum_p w_p phi_i(p) phi_j(p)
 *     E     = sum_p w_p v_p n(p) + sum_p w_p sum_ij P_ij phi_i tphi_j,  dE/dP, dE/dv, dE/dR
 *                                                                     (aims_integrate_h_backward)
 *
 * This is the grid-integration part of one self-consistent-field iteration of semilocal
 * all-electron DFT with numeric atom-centred orbitals (the method of the paper's "Background
 * and Current Status" and "Development Priorities" sections; the s.c.f. iteration timed in
 * its Figure 4).  The paper gives no formulas for it; the definitions above are the textbook
 * real-space quadrature of those matrix elements.
 *
 * Units: bohr and hartree.  Basis order (part of the contract): atom-major, then the shells of
 * the atom's species in the order given, then m = -l..l.  Real harmonics are orthonormal on the
 * sphere, without the Condon-Shortley phase (Y_1,-1 ~ y, Y_10 ~ z, Y_11 ~ x).
 *
 * Radial functions: for each shell the caller tabulates R and K at the logarithmic knots
 * r_k = r0 (rc/r0)^(k/(n_log-1)), k = 0..n_log-1.  The library interpolates them with the
 * natural cubic spline in s = ln r on those (uniform in s) knots, uses the first cubic below r0,
 * returns exactly 0 for r >= rc, and clamps r below 1e-12 bohr to 1e-12.
 *
 * Ownership: the caller owns every buffer it passes; the library owns the aims_grid handle
 * (tables, batch lists, scratch) until aims_grid_destroy and never frees caller memory.  No
 * pointer is retained after a call returns, except by a step graph (its buffers must outlive
 * it).  Calls are asynchronous on the stream given at setup; one handle must not be used from
 * two threads at once.  Errors: every call returns an aims_status; all argument validation
 * happens on the host before any launch, and aims_last_error() holds the message.
 *
 * Environment: AIMS_SCRATCH_MB sets the scratch budget that bounds a group of batches (default
 * 8192, minimum 16; read whenever a batch partition is built: at setup, and at the first call
 * with a new H partition).  A handle's scratch grows to the largest group it has needed; a
 * smaller scratch it outgrows is released unless a step graph has been captured on the handle.
 * Read at setup: AIMS_H_MERGE sets the initial h_merge of every precision (0..4);
 * AIMS_FORCES_THREAD_PATH=1 makes aims_total_forces use its thread-per-point kernel (otherwise
 * taken only above 512 atoms per system) for every system size.  Read at every device
 * allocation: AIMS_FAIL_ALLOC=1 makes it fail with AIMS_ERR_OOM (to test the error path).
 */
#ifndef AIMS_GRID_H
#define AIMS_GRID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aims_grid aims_grid;  /* opaque, library-owned */

typedef enum {
  AIMS_OK = 0,
  AIMS_ERR_ARG = -1,          /* invalid argument (null, wrong memory space, out of range)   */
  AIMS_ERR_OOM = -2,          /* device or host allocation failed                            */
  AIMS_ERR_HIP = -3,          /* a HIP runtime call or kernel launch failed                  */
  AIMS_ERR_STALE = -4,        /* an atom moved farther than screen_margin since setup        */
  AIMS_ERR_UNSUPPORTED = -5   /* l > 3, or a size beyond the documented limits               */
} aims_status;

typedef enum {
  AIMS_FP64 = 0,    /* everything in FP64                                                    */
  AIMS_FP32 = 1,    /* per-batch contractions on FP32 MFMA, FP32 basis values and tables;
                       FP64 cross-batch reduction of H/S/n and of the N/E sums               */
  AIMS_BF16X3 = 2,  /* per-batch contractions as three BF16 MFMA products of hi/lo splits
                       (x = hi + lo, hi = bf16(x), lo = bf16(x - hi); hi*hi + hi*lo + lo*hi)
                       with FP32 accumulation; FP64 cross-batch reduction as for AIMS_FP32   */
  AIMS_INT8X7 = 3   /* per-batch contractions on the int8 matrix cores: every operand row is
                       scaled by a power of two and written as seven balanced base-128 digits
                       (x = 2^e sum_s q_s 128^-s, q_s in [-64, 64]); the digit products with
                       s + t <= 8 (28 per product) accumulate exactly in int32 and combine in
                       FP64.  Basis values are evaluated in FP64.  Density, H and S passes only
                       (the backward, forces and the gradient term return
                       AIMS_ERR_UNSUPPORTED); at most 4096 functions per batch.  The products
                       follow the error-free slicing of Ozaki, Ogita, Oishi and Rump (2012),
                       the "Development Priorities" note on exploiting new GPU hardware.  */
} aims_precision;

/* One molecular system.  All pointers are HOST pointers; the library copies what it needs
 * during setup.  Sizes: n_atoms >= 1, n_species >= 1, 1 <= max_batch <= 512, n_log >= 4,
 * 0 < r0 < rc, 0 <= l <= 3.  n_points may be 0. */
typedef struct {
  int32_t n_atoms;
  const double *atom_xyz;        /* [n_atoms][3]                                             */
  const int32_t *atom_species;   /* [n_atoms], values 0..n_species-1                         */
  int32_t n_species;
  const int32_t *species_nshell; /* [n_species]                                              */
  const int32_t *shell_l;        /* [sum nshell], species-major, each 0..3                    */
  int32_t n_log;                 /* knots of the logarithmic radial grid                     */
  double r0, rc;                 /* first knot and cutoff radius (last knot)                 */
  const double *shell_R;         /* [sum nshell][n_log]: R(r_k)                              */
  const double *shell_K;         /* [sum nshell][n_log]: K(r_k) = -1/2[R''+2R'/r-l(l+1)R/r^2] */
  int64_t n_points;
  const double *pt_xyz;          /* [n_points][3]                                            */
  const double *pt_w;            /* [n_points] full quadrature weights                       */
  int32_t max_batch;             /* maximum points per batch                                 */
  double screen_margin;          /* bohr; atoms may later move this far (<= 0: 1e-2)         */
} aims_system;

/* Builds the splines (FP64 and FP32 copies), partitions the points into batches by recursive
 * bisection along the longest bounding-box axis until each holds <= max_batch points (a node of
 * 128 or more points splits at its median rounded to a multiple of 64 points, so that every
 * batch of a system but its last holds a multiple of 64 points),
 * keeps per batch the atoms closer than rc + screen_margin to at least one of its points (and
 * so every basis function that can be nonzero on it), and uploads everything to `device`.
 * `hip_stream` (a hipStream_t, NULL = default stream) is used by every later call.
 * At most 65535 basis functions per system (AIMS_ERR_UNSUPPORTED beyond).
 * On success *out receives a new handle. */
aims_status aims_grid_setup(const aims_system *sys, int device, void *hip_stream, aims_grid **out);

/* Several independent systems in one handle (the ensemble of independent calculations the
 * paper's "Concluding Remarks" describe, here on one GPU).  Their batches are processed
 * together in every call.  Per-system arrays passed to later calls are concatenated in system
 * order: points (n, v, dE/dv), atoms (atom_xyz, dE/dR), and the dense nb_s x nb_s matrices
 * (P, H, S, dE/dP) one after another at offsets sum_{t<s} nb_t^2.  At most 65535 systems
 * (AIMS_ERR_UNSUPPORTED beyond). */
aims_status aims_grid_setup_many(const aims_system *sys, int32_t n_sys, int device,
                                 void *hip_stream, aims_grid **out);

/* Density update: n_out[p] = sum_ij P_ij phi_i(p) phi_j(p) for every point (caller order) and
 * sums_out[3] = { N = sum w n, E_V = sum w v n, E_T = sum_p w_p sum_ij P_ij phi_i tphi_j }.
 * P: DEVICE, FP64, [nb][nb] row-major, symmetric (the caller's responsibility; with the
 * environment variable AIMS_DEBUG=1 at setup, every call that reads P checks it on the device,
 * max|P - P^T| <= 1e-12 max|P| and finite, and refuses it with AIMS_ERR_ARG).  v_or_null:
 * DEVICE [n_points] or NULL (then E_V = 0).  n_out: DEVICE [n_points].  sums_out: DEVICE [3].
 * atom_xyz: NULL (positions from setup) or a host or device [n_atoms][3] array within
 * screen_margin of the setup positions.  A host array is checked before any launch
 * (AIMS_ERR_STALE).  A device array is copied and checked on the device, with no host
 * synchronisation (so the call can be captured into a graph): if an atom moved beyond the
 * margin or is not finite, the call's outputs are set to NaN and aims_positions_status reports
 * AIMS_ERR_STALE.  The same holds for aims_integrate_h and aims_integrate_h_backward. */
aims_status aims_update_density(aims_grid *g, aims_precision prec, const double *atom_xyz,
                                const double *P, const double *v_or_null, double *n_out,
                                double *sums_out);

/* Result of the screening check of the last positions given as a device array (synchronous):
 * AIMS_OK, or AIMS_ERR_STALE when an atom had moved beyond screen_margin or was not finite (the
 * outputs of that call are NaN). */
aims_status aims_positions_status(aims_grid *g);

/* Allocation-free density update, for callers that cannot allocate device memory during the
 * call (code under stream capture, tight serving loops, hosts that forbid allocation): the
 * same result as aims_update_density with atom_xyz = NULL, computed by the same kernels, and no
 * hipMalloc, hipFree or allocating library routine inside the call.  The basis slabs of the
 * batches live in one static device array of 64 MiB (32 MiB per slab), held by every GPU the
 * library runs on until the process ends; the batches are processed in as many groups as that
 * takes.  AIMS_ERR_UNSUPPORTED if a single batch needs more than 32 MiB per slab (more than
 * 4M FP64 values: n_b rounded up to 32 times the batch's padded point count).  Every call on
 * one GPU shares that array, so calls that overlap on one GPU (other streams, other handles,
 * other host threads) race: the caller serialises them.  Positions are those of setup: a
 * handle moved by an earlier call is first restored, as with atom_xyz = NULL.  Arguments as
 * for aims_update_density. */
aims_status aims_update_density_noalloc(aims_grid *g, aims_precision prec, const double *P,
                                        const double *v_or_null, double *n_out, double *sums_out);

/* Hamiltonian (and optionally overlap) integration: H_ij = sum_p w_p phi_i (v_p phi_j + tphi_j)
 * (raw: not symmetrised), S_ij = sum_p w_p phi_i phi_j.  v: DEVICE [n_points].  H, S_or_null:
 * DEVICE FP64 [nb][nb] row-major, overwritten. */
aims_status aims_integrate_h(aims_grid *g, aims_precision prec, const double *atom_xyz,
                             const double *v, double *H, double *S_or_null);

/* Backward of E(P, v, R) = sum_p w_p v_p n(p) + sum_p w_p sum_ij P_ij phi_i tphi_j with an
 * incoming gradient gE (DEVICE, one double):
 *   dE/dP_ij = gE H_ij (independent entries),  dE/dv_p = gE w_p n(p),
 *   dE/dR_a  = -gE sum_p w_p sum_{i on a} [(2 v_p X_pi + Y_pi) grad phi_i(p) + X_pi grad tphi_i(p)]
 * with X = Phi P and Y = (T Phi) P per batch; basis values and gradients are recomputed, not
 * stored.  Only the basis centres move (grid points, weights and v are fixed).  Any output may
 * be NULL.  dE_dP: DEVICE [nb][nb]; dE_dv: DEVICE [n_points]; dE_dR: DEVICE [n_atoms][3];
 * all overwritten. */
aims_status aims_integrate_h_backward(aims_grid *g, aims_precision prec, const double *atom_xyz,
                                      const double *P, const double *v, const double *gE,
                                      double *dE_dP_or_null, double *dE_dv_or_null,
                                      double *dE_dR_or_null);

/* Moving-grid model of one system, for the total energy gradient (host arrays, copied):
 * every grid point belongs to the atom-centred grid of an owner atom and moves with it, its
 * weight is pt_wgrid times the Stratmann-Scuseria-Frisch partition with parameter
 * partition_a (Chem. Phys. Lett. 257, 213 (1996)), and the potential is the nuclear model
 * v(p) = sum_a -Z_a erf(|p - R_a| / nuc_sigma) / |p - R_a|.  The setup weights pt_w must be
 * pt_wgrid times that partition (exact products over all atoms).
 *   pt_owner   [n_points] owner atom, 0..n_atoms-1 of the system (caller point order)
 *   pt_wgrid   [n_points] radial x angular weight of the owner's grid (before the partition)
 *   atom_Z     [n_atoms]  nuclear charges
 * Errors: AIMS_ERR_ARG for out-of-range owners, non-finite values, sigma <= 0 or a outside
 * (0, 1). */
typedef struct {
  const int32_t *pt_owner;
  const double *pt_wgrid;
  const double *atom_Z;
  double nuc_sigma;
  double partition_a;
} aims_moving_grid;
aims_status aims_grid_set_moving(aims_grid *g, int32_t sys, const aims_moving_grid *m);

/* Total gradient (the extension of the backward to moving grids) of
 *     E(R) = sum_p w_p(R) [ v(p; R) n(p; R) + sum_ij P_ij phi_i(p) tphi_j(p) ]
 * at the setup positions, where the grid points, their partition weights, the nuclear model
 * potential and the basis centres all follow the atoms (P fixed):
 *     dE_dR[a] = gE * dE/dR_a = (Pulay term of aims_integrate_h_backward)
 *                + the point-motion, partition-weight and potential terms.
 * Every system needs aims_grid_set_moving first.  P: DEVICE [nb][nb]; gE: DEVICE [1];
 * dE_dR: DEVICE [n_atoms][3], overwritten; sums_out_or_null: DEVICE [n_sys][3] receives
 * (N, E_V, E_T) of that energy (v = the model potential).  AIMS_FP64 and AIMS_FP32 only
 * (AIMS_ERR_UNSUPPORTED otherwise); at most 2730 atoms per system. */
aims_status aims_total_forces(aims_grid *g, aims_precision prec, const double *P, const double *gE,
                              double *sums_out_or_null, double *dE_dR);

/* H with a gradient term, for gradient-corrected functionals:
 *     H_ij = sum_p w_p phi_i(p) [ v_p phi_j(p) + tphi_j(p) + u_p . grad phi_j(p) ]
 * The exchange-correlation part of a GGA Hamiltonian is
 *     sum_p w_p [ v_n phi_i phi_j + 2 v_sigma grad n . grad(phi_i phi_j) ] = V_n + B + B^T,
 *     B_ij = sum_p w_p phi_i 2 v_sigma grad n . grad phi_j    (v_sigma = d f_xc / d |grad n|^2)
 * and this raw form with v = v_nuc + v_n and u = 4 v_sigma grad n holds V_n + 2 B, whose
 * symmetric part is the same (the density-matrix step uses the symmetric part).  v: DEVICE [n_points]; u: DEVICE
 * [n_points][3] (caller order); H: DEVICE blocks as aims_integrate_h.  AIMS_FP64 or AIMS_FP32;
 * setup positions. */
aims_status aims_integrate_h_gga(aims_grid *g, aims_precision prec, const double *v,
                                 const double *u, double *H);

/* Density and its gradient at every point, the input of gradient-corrected functionals:
 *     n(p) = sum_ij P_ij phi_i(p) phi_j(p),   grad n(p) = 2 sum_ij P_ij phi_i(p) grad phi_j(p)
 * (P symmetric, the caller's responsibility), FP64, at the setup positions.  P: DEVICE
 * [nb][nb] blocks; grad_out: DEVICE [n_points][3] (caller order); n_out_or_null: DEVICE
 * [n_points]. */
aims_status aims_density_gradient(aims_grid *g, const double *P, double *n_out_or_null,
                                  double *grad_out);

/* Exchange-correlation potential on the grid, the step between the density and the H
 * integration of an s.c.f. iteration for the semilocal functionals the paper names
 * (Background and Current Status).  Spin-unpolarised LDA: Slater exchange
 * eps_x = -(3/4)(3 n/pi)^(1/3) and the Perdew-Wang 1992 correlation eps_c(rs), rs =
 * (3/(4 pi n))^(1/3); v_xc = d(n eps_xc)/dn.  Points with n <= 1e-14 (including negative
 * densities) get eps = v = 0.
 * n: DEVICE [n_points] (caller order, e.g. aims_update_density's output); v_xc_out: DEVICE
 * [n_points]; sums_out_or_null: DEVICE [n_sys][2] = (E_xc = sum_p w_p n_p eps_xc, sum_p w_p n_p
 * v_xc).  Asynchronous on the handle's stream. */
typedef enum { AIMS_XC_LDA_PW92 = 0, AIMS_XC_PBE = 1 } aims_xc_functional;
aims_status aims_xc(aims_grid *g, int32_t functional, const double *n, double *v_xc_out,
                    double *sums_out_or_null);
/* Gradient-corrected exchange-correlation (AIMS_XC_PBE, spin-unpolarised, PW92 correlation):
 * with sigma = |grad n|^2, s^2 = sigma / (4 k_F^2 n^2), t^2 = sigma / (4 k_s^2 n^2),
 *     f(n, sigma) = n eps_x(n) F_x(s) + n (eps_c(n) + H(rs, t))
 * (kappa = 0.804, beta = 0.06672455060314922, mu = beta pi^2 / 3).  Outputs per point (caller
 * order): v_out = df/dn, u_out [n_points][3] = 4 (df/dsigma) grad n, the vector field that
 * aims_integrate_h_gga takes; sums_out_or_null: DEVICE [n_sys][2] = (E_xc = sum w f,
 * sum w (n v_n + 2 sigma v_sigma) = tr(P H_xc)).  n, grad_n: DEVICE (aims_density_gradient's
 * output); n <= 1e-14 gives zeros. */
aims_status aims_xc_gga(aims_grid *g, int32_t functional, const double *n, const double *grad_n,
                        double *v_out, double *u_out, double *sums_out_or_null);

/* Hartree potential of the grid density by an atom-centred multipole expansion of the
 * partitioned density (the electrostatic step of an s.c.f. iteration, which the paper notes is
 * not yet accelerated on GPUs; Development Priorities).  The grid must be atom-centred product
 * grids on Becke's radial map r = r_map cot^2(theta/2), theta_k = (k+1) pi/(n_radial+1),
 * k = 0..n_radial-1, whose point weights are (radial weight with r^2) x (angular weight) x
 * (partition of the owner atom):
 *   rho_{a,lm}(r_k) = sum over the points of node k of atom a of w n Y_lm(u) / W_k,
 *   V_lm(r) = 4 pi/(2l+1) [ r^-(l+1) int_0^r rho_lm s^(l+2) ds + r^l int_r^inf rho_lm s^(1-l) ds ]
 *   (natural cubic splines of rho_lm and V_lm in theta, 6-point Gauss-Legendre per interval,
 *   (r/r_min)^l inside the innermost node),
 *   v_H(p) = sum_a sum_lm V_{a,lm}(|p - R_a|) Y_lm(u),  E_H = 1/2 sum w n v_H.
 * Support: atom a's piece lives on its own points.  With k_o its outermost node that holds a
 * point, its edge node is k_e = max(k_o - 1, 0) (0 for an atom without points); rho_lm is
 * splined over nodes k_e..n_radial-1 and is zero beyond r(k_e), where V_lm is exactly the
 * exterior field 4 pi q_lm / ((2l+1) r^(l+1)) with q_lm = int_0^r(k_e) rho_lm s^(l+2) ds: a
 * point beyond an atom's edge takes only that atom's moments (no spline evaluation).
 * aims_grid_set_hartree: per point (caller order of the system) the owner atom and the radial
 * node, plus n_radial, r_map and l_max (0..6, the same for every system of the handle).
 * aims_hartree: n: DEVICE [n_points] (caller order); v_out: DEVICE [n_points];
 * E_out_or_null: DEVICE [n_sys].  Setup positions. */
typedef struct {
  const int32_t *pt_owner;
  const int32_t *pt_node;
  int32_t n_radial;
  double r_map;
  int32_t l_max;
} aims_hartree_grid;
aims_status aims_grid_set_hartree(aims_grid *g, int32_t sys, const aims_hartree_grid *h);
aims_status aims_hartree(aims_grid *g, const double *n, double *v_out, double *E_out_or_null);

/* Density matrix of the occupied subspace: the step after the H integration in an s.c.f.
 * iteration, the eigensolver stage that the paper names as the bottleneck of large systems
 * (Development Priorities).  Per system s (basis size nb_s):
 *     H_sym = (H + H^T) / 2,   H_sym C = S C diag(eps),   C^T S C = I,   P = C diag(f) C^T
 * with spin-restricted occupations 0 <= f_k <= 2, sum f_k = n_electrons[s]: aufbau for kT = 0
 * (the lowest floor(N/2) states full, a remaining fraction in the next), Fermi-Dirac
 * f_k = 2 / (1 + exp((eps_k - mu) / kT)) for kT > 0 with mu fixed by the electron count.
 * method AIMS_DM_EIGEN: generalised eigensolver (rocSOLVER sygvd), eigenvalues available.
 * method AIMS_DM_PURIFY: Cholesky orthogonalisation and trace-correcting purification (X <- X^2
 *   or 2 X - X^2 by the trace; stop three products after |tr X - ||X||_F^2| < 1e-8 N_e/2,
 *   decided on the device), no eigenvectors; needs kT = 0, an even electron count and a gap at
 *   the Fermi level; no eigenvalues (eps_out must be NULL) and mu_out receives NaN.  The
 *   inverse Cholesky factor of S is kept by the handle and reused while a system's S is bitwise
 *   the one it came from (a device comparison per call); any change of S, in place or not,
 *   factorises it again.
 * H, S: DEVICE, the concatenated nb_s x nb_s blocks as aims_integrate_h writes them (H need not
 * be symmetric; S must be symmetric positive definite).  n_electrons: HOST [n_sys].  P_out:
 * DEVICE, same layout, symmetric.  eps_out_or_null: DEVICE [sum nb_s], ascending per system.
 * mu_out_or_null: HOST [n_sys].  Synchronous (it reads eigenvalues or convergence data back).
 * Errors: AIMS_ERR_ARG for counts that do not fit or an S that is not positive definite,
 * AIMS_ERR_UNSUPPORTED for the purification limits above, AIMS_ERR_HIP if the purification
 * does not converge. */
typedef enum { AIMS_DM_EIGEN = 0, AIMS_DM_PURIFY = 1 } aims_dm_method;
aims_status aims_density_matrix(aims_grid *g, int32_t method, const double *H, const double *S,
                                const double *n_electrons, double kT, double *P_out,
                                double *eps_out_or_null, double *mu_out_or_null);
/* Matrix products of the last purification (of the last system); 0 after AIMS_DM_EIGEN. */
int32_t aims_last_purify_products(const aims_grid *g);

/* One s.c.f. step (density update followed by H integration, setup positions) captured once
 * into a HIP graph on the handle's stream; aims_step_graph_launch replays it.  The buffers are
 * baked into the graph and must outlive it; update their contents in place between replays. */
typedef struct aims_step_graph aims_step_graph;
aims_status aims_step_graph_create(aims_grid *g, aims_precision prec, const double *P,
                                   const double *v, double *n_out, double *sums_out, double *H,
                                   aims_step_graph **out);
aims_status aims_step_graph_launch(aims_step_graph *graph);
void aims_step_graph_destroy(aims_step_graph *graph);

/* Tunable execution parameters of one precision (chosen by the project's autotuner, which
 * times candidates on the live device; see paper_2208_12335_amd.autotune).
 *   h_merge          the H/S pass uses batches of up to max_batch << h_merge points (the same
 *                    bisection stopped h_merge levels earlier): fewer FP64 scatter-adds into H
 *                    for slightly more flops.  0..4.
 *   density_pblocks  a density work tile covers 64 basis rows and up to 32 * density_pblocks
 *                    points of one batch (2..5); a batch of n_p points is cut into
 *                    ceil(n_p / (32 density_pblocks)) equal tiles.
 *   h_flops_per_atomic  0: the H/S batches are the fixed merge level above; R > 0: a cost
 *                    model chooses them (h_merge is then ignored): each node of the set-up
 *                    bisection, up to 4 x max_batch points, becomes one H batch when
 *                    2 n_p n_b^2 + R n_b^2 (flops plus R flop-equivalents per FP64 scatter-add)
 *                    is below the best cost of its two halves.  0..2^20.
 *   persistent       0: one workgroup per work tile (hardware dispatch order, XCD-interleaved);
 *                    1: the tiled density and H/S kernels launch as many workgroups as fit on
 *                    the device at once, and each pulls tiles from eight per-XCD work counters
 *                    (one atomic per tile, stealing from the other XCDs' counters when its
 *                    own is empty).  The counters are cleared by a kernel at the start of each
 *                    call, so calls in this mode can be captured into a step graph.
 * Setting a value builds its work lists once (device allocation), later calls reuse them;
 * buffers referenced by step graphs captured earlier stay allocated (a graph keeps replaying
 * the tuning it was captured with). */
typedef struct {
  int32_t h_merge;
  int32_t density_pblocks;
  int32_t persistent;
  int32_t h_flops_per_atomic;
  /* Tile shapes by (points, basis count) bucket.  A density batch of n_b functions falls in
   * bucket min(7, (n_b - 1) / 64); density_bucket_pblocks[b] (0, or 2..5) replaces
   * density_pblocks for the batches of bucket b.  An H / S batch falls in bucket
   * 2 min(7, (n_b - 1) / 64) + (1 if n_b mod 64 is in 1..32); bit b of h_tile32_mask runs that
   * bucket on 32 x 32 tiles instead of 64 x 64 (AIMS_FP64 and AIMS_FP32 only). */
  int32_t h_tile32_mask;
  int32_t density_bucket_pblocks[8];
} aims_tuning;
aims_status aims_get_tuning(const aims_grid *g, aims_precision prec, aims_tuning *out);
aims_status aims_set_tuning(aims_grid *g, aims_precision prec, const aims_tuning *t);

/* Batches and algorithmic flops (sum of 2 n_p n_b^2) per tile-shape bucket, for an autotuner:
 * which = 0, the density partition (8 buckets); which = 1, the precision's current H partition
 * (16 buckets).  batches_out and flops_out are HOST arrays of that many entries. */
aims_status aims_bucket_stats(aims_grid *g, aims_precision prec, int32_t which, int64_t *batches_out,
                              double *flops_out);

/* Work statistics: number of batches, sum_b n_p n_b^2 (flops = 4x this per s.c.f. step), and
 * sum_b n_b^2 (entries scattered into H per call); any pointer may be NULL. */
aims_status aims_work_stats(const aims_grid *g, int64_t *n_batches, double *sum_np_nb2,
                            double *sum_nb2);
int64_t aims_n_basis(const aims_grid *g);       /* total over systems                      */
int64_t aims_n_points(const aims_grid *g);      /* total over systems                      */
int32_t aims_n_atoms(const aims_grid *g);       /* total over systems                      */

/* Per-kernel timing: with profiling on, HIP events are recorded on the handle's stream around
 * every kernel launch.  aims_profile_read synchronizes the stream, then returns for one kernel
 * family ("phi_eval", "density", "hs", "backward", "finish") the number of launches since
 * profiling was enabled, their summed duration in milliseconds, and the algorithmic work they
 * did (flops of the per-batch contractions, 2 n_p n_b^2 per batch and GEMM).  Not for use while
 * a step graph is being captured. */
aims_status aims_profile_enable(aims_grid *g, int on);
aims_status aims_profile_read(aims_grid *g, const char *kernel, int64_t *launches,
                              double *total_ms, double *work);

/* Message of the last failure on this handle, or of the calling thread's last failed setup
 * when g is NULL.  Never NULL. */
const char *aims_last_error(const aims_grid *g);
void aims_grid_destroy(aims_grid *g);

#ifdef __cplusplus
}
#endif
#endif /* AIMS_GRID_H */
