"""Plain FP64 CPU oracle for the nested viscous-block solve of the SIP-DG Stokes
discretisation (Charrier, May & Schnepp, "Symmetric interior penalty
discontinuous Galerkin discretisations and block preconditioning for
heterogeneous Stokes flow").

THIS PACKAGE IS TEST INFRASTRUCTURE.  It is the slow, obviously-correct
reference that the HIP path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the GPU library: the forms are assembled by
Gauss-Legendre quadrature of the paper's bilinear forms (the GPU evaluates
closed modal formulas instead), and the solvers are plain numpy/scipy.

Modules
-------
legendre  : 1D Legendre polynomials, orthonormal scaling, Gauss rules.
mesh      : Cartesian grid, DoF numbering, face enumeration.
assemble  : sparse FP64 assembly of A (SIP form), B (divergence form),
            F, G, S* by quadrature (Section 4, eqs. stiffness_form,
            divergence_form, rhs_f; Section 5 for S*).
direct    : sparse direct solves of the viscous and Stokes systems.
multigrid : the hp-multilevel preconditioner of Section 6 (Algorithm 1,
            element-block Jacobi, Chebyshev, p-transfer, P_cd, Galerkin
            h-hierarchy) and the Krylov drivers of Section 8.
rng       : SplitMix64, the counter-based generator both sides use for the
            random start vector of the eigenvalue estimate.
"""
