"""FP64 CPU oracle for the Darcy / Boussinesq / convection-diffusion state and adjoint solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or calls
this package; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the GPU path: the only thing the two sides have
in common is the seeded input generator, which holds none of the method's arithmetic.

What it computes (all in float64, plain and unblocked):

* the stabilised trilinear-hexahedron weak form of the paper's appendix A
  (eq. weakstable), with the Darcy velocity of Sec. 2.1 (eq. finaldarcy) and the
  Tezduyar SUPG weight of App. A, assembled element by element;
* RAMP interpolation of conductivity and permeability (Sec. 5.2,
  eqs. condRAMP / permRAMP), a cone density filter and the PDE (Helmholtz) density
  filter of Sec. 5.1, solved directly;
* a damped Newton iteration (Sec. 5.4) whose Jacobian is assembled from
  complex-step element Jacobians into a SciPy CSR matrix and solved directly
  with SuperLU;
* the adjoint solve with the transposed factorisation and the design
  sensitivities -lambda^T dR/dgamma (Sec. 5.1, adjoint sensitivity analysis);
* the Navier-Stokes / Brinkman flow model of the hybrid strategy (Sec. 6.4) on the
  same machinery, with equal-order SUPG / PSPG stabilisation;
* the closed-form permeability tuning of Sec. 3 (eqs. nusselt1-nusselt5);
* the Method of Moving Asymptotes for the volume-constrained design update (Sec. 5.1),
  and the design loop of Sec. 5 around it (continuation, warm starts, Q ramping).

Parity status: every function is pinned by tests under tests/ (closed forms,
invariants, brute-force finite differences, the paper's Table tab:2); the SUPG
parameter by the closed form of 1D advection-diffusion at three cell Peclet numbers,
and the centroid velocity of the SUPG weight by a pressure mode whose centroid
velocity vanishes (the energy row is then the Galerkin row).
"""

from .problem import Params, Mesh, default_constraints, patch_flux
from .material import ramp_k, ramp_kappa, ramp_k_deriv, ramp_kappa_deriv, cone_filter_matrix, kappa_f_tuning
from .element import element_residual, reference_element
from .pde_filter import PDEFilter, pde_length_scale
from .fem import Model
from .mma import MMA
from .navier_stokes import NSModel, ns_element_residual, ns_constraints, brinkman
from . import design

__all__ = [
    "Params", "Mesh", "default_constraints", "patch_flux",
    "ramp_k", "ramp_kappa", "ramp_k_deriv", "ramp_kappa_deriv", "cone_filter_matrix", "kappa_f_tuning",
    "element_residual", "reference_element", "Model", "PDEFilter", "pde_length_scale", "MMA",
    "NSModel", "ns_element_residual", "ns_constraints", "brinkman",
]
