"""FP64 CPU oracle for the screened-Laplace (Yukawa) double-layer solve.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The HIP library never
calls it and shares no code, header, table or constant with it.

It is a plain, slow, readable transcription of the method of Fu, Ryham,
Kloeckner, Wala, Jiang and Young, "Simulation of multiscale hydrophobic lipid
dynamics via efficient integral equation methods" (arXiv 1810.04131):

* the exterior Dirichlet problem for -rho^2 Lap u + u = 0 (eq. SL) with
  u = f on the particle boundaries and u -> 0 at infinity;
* the double-layer representation u = D[sigma] (eq. intrep) with the Yukawa
  Green's function G = K0(|x-y|/rho)/(2 pi) (eq. Gfunc) and the normal nu(y)
  pointing out of the particle into the water (section 4);
* the second-kind equation 1/2 sigma + D sigma = f (eq. bie);
* Nystrom discretisation on composite Gauss-Legendre panels and QBX local
  expansions from Graf's addition theorem (section 5, eqs. local-exp,
  graf-coefficient, graf-addition, Theorem qbx-accuracy);
* dense LU or GMRES for the discrete system (Algorithm 1);
* the hydrophobic stress, forces and torques (eqs. stress, force_torque,
  scalar-torque) and the energy of eq. main through Green's first identity;
* the excluded-volume repulsion of eq. repul with the three-circle ellipse
  model of supplementary section S1, and the constant-drag forward Euler step
  of eq. euler (Algorithm 1 without the Stokes mobility solve).

Modules: geometry (panels, nodes, weights), labels (boundary data f),
kernels (double-layer kernel and its gradient), qbx (near lists, QBX rows,
oversampled rows), operator (dense matrix and sampled rows), solve (LU and
MGS-GMRES), forces (surface gradient, traction, F, tau, energy), potential
(off-surface evaluation), dynamics (repulsion, Euler step).

Readings of points the paper leaves open are listed in each function's
docstring.  Parity pins live in tests/test_oracle_*.py.
"""
from .geometry import Params, Discretization, discretize, gauss_legendre  # noqa: F401
from .labels import arc_label, janus_label  # noqa: F401
from .kernels import dl_kernel, dl_grad_kernel  # noqa: F401
from .qbx import near_panels, qbx_row, operator_qbx_row, oversampled_row, interp_matrix  # noqa: F401
from .operator import build_matrices, apply_rows, far_rows  # noqa: F401
from .solve import lu_solve, gmres  # noqa: F401
from .forces import surface_fields, traction, forces_torques  # noqa: F401
from .potential import eval_potential  # noqa: F401
from .dynamics import circle_centres, repulsion, euler_update, time_step  # noqa: F401
