"""FP64 CPU oracle for NAO real-space grid integration.  TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct reference that the HIP library is checked
against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may import it;
the library never does, and the two share no code (they meet only at the seeded inputs built
by the ``synth`` package).

What it computes is the direct quadrature of the method's definitions, in float64:

    phi_i(p)  = R_s(|p - R_a|) Y_lm(u),  u = (p - R_a)/|p - R_a|,  i = (atom a, shell s, m)
    tphi_i(p) = -1/2 Laplacian phi_i(p) = K_s(|p - R_a|) Y_lm(u)
    n(p)      = sum_ij P_ij phi_i(p) phi_j(p)
    S_ij      = sum_p w_p phi_i phi_j
    H_ij      = sum_p w_p phi_i (v_p phi_j + tphi_j)      (raw, not symmetrised)
    N = sum_p w_p n(p),  E_V = sum_p w_p v_p n(p),  E_T = sum_p w_p sum_ij P_ij phi_i tphi_j
    E = E_V + E_T,  dE/dP = H,  dE/dv_p = w_p n(p),  dE/dR_a by automatic differentiation

R_s and K_s are natural cubic splines in s = ln r through the tabulated knot values
(``scipy.interpolate.CubicSpline``), zero for r >= rc; Y_lm are the real, orthonormal spherical
harmonics without the Condon-Shortley phase, built from the general real-solid-harmonic sum.

``forces.moving_grid_gradient`` differentiates the same energy with every ingredient moving
with the atoms (atom-centred grid points, Stratmann partition weights, the erf nuclear
potential, the basis centres): the total analytic gradient, by torch autograd.

``xc.lda`` evaluates the exchange-correlation energy density and potential of the
spin-unpolarised gas (Slater exchange + Perdew-Wang 1992 correlation) pointwise.

``scf.density_matrix`` takes the step after the H integration: the generalised eigenproblem of
the symmetric part of H against S, aufbau or Fermi-Dirac occupations, and P = C diag(f) C^T.

Parity status: every function here is pinned by closed forms, invariants, library routines,
brute force or finite differences in ``tests/test_oracle_*.py``; none is "parity unpinned".
"""
from .harmonics import real_ylm, real_ylm_grad, ylm_terms  # noqa: F401
from .radial import RadialSplines  # noqa: F401
from .integrate import GridOracle  # noqa: F401
from .forces import moving_grid_gradient  # noqa: F401
from .scf import density_matrix  # noqa: F401
