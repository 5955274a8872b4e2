"""Oracle of the Navier-Stokes / Brinkman flow model: the full-flow model of the hybrid
strategy (Sec. 6.4), solved for the same five unknowns per node (u, v, w, P, T).
Test infrastructure only (see oracle/__init__.py).

Governing equations (Sec. 2.1 eq. app_NS with the modified pressure P and the
Boussinesq buoyancy of Sec. 2.1, plus a Brinkman friction that makes the solid
impermeable; the energy equation is the third line of eq. goveq):

    rho0 (u . grad) u - div(mu (grad u + grad u^T)) + grad P + a(gamma) u + rho0 alpha g T = 0
    div u = 0
    rho0 c_p u . grad T - div(k grad T) - Q = 0

with g = (0, 0, -g0) and T0 = 0 as in the Darcy model.

Discretisation (readings; the paper takes the Navier-Stokes formulation from earlier
work and prints no weak form for it): equal-order trilinear elements for all five
fields with the same 2x2x2 Gauss rule as the Darcy model,

  momentum  R_u,a = sum_q detJ [ W_a r_m + mu grad N_a . (grad u + grad u^T) ]
  continuity R_P,a = sum_q detJ [ N_a div u + (tau_m / rho0) grad N_a . r_m ]
  energy    R_T,a = sum_q detJ [ N*_a (rho0 c_p u . grad T - Q) + k grad N_a . grad T ]

where r_m = rho0 (u . grad) u + grad P + a u + rho0 alpha g T is the strong momentum
residual without the viscous term (zero-valued second derivatives of the trilinear
basis are dropped, and the mixed ones with them), W_a = N_a + tau_m u0 . grad N_a the
streamline-upwind weight (SUPG) and the second term of the continuity row the
pressure-stabilising one (PSPG).  u0 is the element's centroid velocity, h_e^2 = 3 h^2
and
    tau_m = (4 |u0|^2 / h_e^2 + 16 nu^2 / h_e^4 + (a / rho0)^2)^(-1/2),   nu = mu / rho0,
the momentum counterpart of the energy equation's parameter of App. A, which is kept:
N*_a = N_a + tau u0 . grad N_a with tau = (4 |u0|^2 / h_e^2 + 16 / h_e^4)^(-1/2).
The Brinkman coefficient interpolates the solid's impermeability: in the Navier-Stokes
stage of the hybrid strategy (the discussion of eq. contsch2) q_p interpolates the
impermeability of the solid and kappa_s is that impermeability (1e5), with the
interpolation of the cited Navier-Stokes work, written here for gamma = 1 solid:
    a(gamma) = kappa_s q_p gamma / (1 + q_p - gamma),
zero in the fluid (gamma = 0) and kappa_s in the solid.

Boundary conditions: no slip (u = 0) on every wall; on a symmetry plane of the quarter
domain only the normal velocity is held (the tangential rows keep their natural
condition, which for the symmetric-gradient form is the symmetry condition); T and
the pressure level as in the Darcy model.
"""

import numpy as np

from .problem import NFIELD, FIELD_P, FIELD_T
from .element import reference_element
from .material import ramp_k
from .fem import Model


def brinkman(gamma, prm):
    """Brinkman coefficient a(gamma) = kappa_s q_p gamma / (1 + q_p - gamma): kappa_s is the
    solid's impermeability in this model (complex-safe)."""
    return prm.kappa_s * prm.q_p * gamma / (1.0 + prm.q_p - gamma)


def _tau(u0, prm, a=None):
    """(tau_m, tau_T) of every element from its centroid velocity u0 (E, 3)."""
    he2 = 3.0 * prm.h * prm.h
    uu = np.einsum("ed,ed->e", u0, u0)
    nu = prm.mu / prm.rho0
    tm = 4.0 * uu / he2 + 16.0 * nu * nu / (he2 * he2)
    if a is not None:
        tm = tm + (a / prm.rho0) ** 2
    tt = 4.0 * uu / he2 + 16.0 / (he2 * he2)
    return tm ** (-0.5), tt ** (-0.5)


def ns_element_residual(Ue, Pe, Te, k, a, prm, Qe=None, src_U=None, src_T=None, x0=None):
    """Element rows of the Navier-Stokes / Brinkman residual for every element.

    Ue (E, 8, 3), Pe, Te (E, 8): nodal unknowns; k, a (E,): conductivity and Brinkman
    coefficient; Qe (E,) volumetric source (default prm.Q); src_U, src_T: optional
    callables of the physical Gauss points (E, 8, 3) giving a body force (E, 8, 3) and a
    heat source (E, 8), x0 (E, 3) the element origins.  Returns RU (E, 8, 3), RP, RT
    (E, 8).  Complex-safe.
    """
    N, G, Nc, _, detJ, xq = reference_element(prm.h)
    buoy = prm.rho0 * prm.alpha * np.array([0.0, 0.0, -prm.g0])
    uq = np.einsum("qa,eai->eqi", N, Ue)
    Gu = np.einsum("qaj,eai->eqij", G, Ue)               # d u_i / d x_j at q
    GP = np.einsum("qad,ea->eqd", G, Pe)
    Tq = np.einsum("qa,ea->eq", N, Te)
    GT = np.einsum("qad,ea->eqd", G, Te)
    rm = prm.rho0 * np.einsum("eqj,eqij->eqi", uq, Gu) + GP + a[:, None, None] * uq + Tq[..., None] * buoy
    xg = None
    if src_U is not None or src_T is not None:
        xg = x0[:, None, :] + xq[None, :, :]
    if src_U is not None:
        rm = rm - src_U(xg)
    div = np.einsum("eqii->eq", Gu)
    u0 = np.einsum("a,eai->ei", Nc, Ue)
    tau_m, tau_t = _tau(u0, prm, a)
    adv = np.einsum("ed,qad->eqa", u0, G)                # u0 . grad N_a at q
    Wm = N[None, :, :] + tau_m[:, None, None] * adv
    Wt = N[None, :, :] + tau_t[:, None, None] * adv
    S = Gu + np.swapaxes(Gu, -1, -2)
    RU = detJ * (np.einsum("eqa,eqi->eai", Wm, rm) + prm.mu * np.einsum("qaj,eqij->eai", G, S))
    RP = detJ * (np.einsum("qa,eq->ea", N, div) + (tau_m / prm.rho0)[:, None] * np.einsum("qad,eqd->ea", G, rm))
    Q = prm.Q if Qe is None else np.asarray(Qe)[:, None]
    cT = prm.rho0 * prm.cp * np.einsum("eqd,eqd->eq", uq, GT) - Q
    if src_T is not None:
        cT = cT - src_T(xg)
    RT = detJ * (np.einsum("eqa,eq->ea", Wt, cT) + k[:, None] * np.einsum("qad,eqd->ea", G, GT))
    return RU, RP, RT


def ns_supg_weights(Ue, prm):
    """Integrated energy weights int_e N*_a (E, 8) at the centroid velocity of the nodal
    velocity field (the weight of the volumetric heat load, App. A f_tQ)."""
    N, G, Nc, _, detJ, _ = reference_element(prm.h)
    u0 = np.einsum("a,eai->ei", Nc, Ue)
    _, tau_t = _tau(u0, prm)
    Nstar = N[None, :, :] + tau_t[:, None, None] * np.einsum("ed,qad->eqa", u0, G)
    return detJ * Nstar.sum(axis=1)


def ns_constraints(mesh, p):
    """Dirichlet mask [N, 5] and values: no slip on the walls (only u.n on a symmetry
    plane), T and the pressure level as in the Darcy model."""
    i, j, k = mesh.node_ijk[:, 0], mesh.node_ijk[:, 1], mesh.node_ijk[:, 2]
    sx, sy = bool(p.sym_x), bool(p.sym_y)
    wall = (i == 0) | (j == 0) | (k == 0) | (k == mesh.nz)
    wall |= (i == mesh.nx) & (not sx)
    wall |= (j == mesh.ny) & (not sy)
    mask = np.zeros((mesh.n_nodes, NFIELD), dtype=bool)
    mask[:, 0:3] = wall[:, None]
    if sx:
        mask[:, 0] |= i == mesh.nx
    if sy:
        mask[:, 1] |= j == mesh.ny
    mask[:, FIELD_T] = (i == 0) | ((i == mesh.nx) & (not sx)) | (j == 0) | ((j == mesh.ny) & (not sy)) | (k == mesh.nz)
    mask[mesh.node_id(0, 0, mesh.nz), FIELD_P] = True
    return mask, np.zeros((mesh.n_nodes, NFIELD))


class NSModel(Model):
    """The Navier-Stokes / Brinkman model on the machinery of the Darcy oracle: the same
    design chain, constraint convention, complex-step Jacobians, damped Newton, SuperLU
    adjoint and sensitivities; only the element rows, the default constraints and the
    state dependence of the volumetric objective differ."""

    objective_fields = (0, 1, 2, FIELD_T)

    def __init__(self, prm, x, constraints=None, flux=None, src_U=None, src_T=None, gamma=None):
        super().__init__(prm, x, constraints=constraints, flux=flux, gamma=gamma)
        if constraints is None:
            self.mask, self.sbar = ns_constraints(self.mesh, prm)
        self.src_U, self.src_T_ns = src_U, src_T
        self.a = brinkman(self.gamma, prm)

    def _elem_rows(self, se, k=None, a=None):
        v = se.reshape(se.shape[0], 8, NFIELD)
        k = self.k if k is None else k
        a = self.a if a is None else a
        RU, RP, RT = ns_element_residual(v[:, :, 0:3], v[:, :, FIELD_P], v[:, :, FIELD_T], k, a, self.prm,
                                         self.Qe, self.src_U, self.src_T_ns, self.x0)
        out = np.empty(v.shape, dtype=np.result_type(se, k, a))
        out[:, :, 0:3] = RU
        out[:, :, FIELD_P] = RP
        out[:, :, FIELD_T] = RT
        return out.reshape(se.shape[0], 8 * NFIELD)

    def elem_dR_dgamma(self, s):
        """d R_e / d gamma_e through the conductivity RAMP and the Brinkman coefficient, by
        the complex step, (E, 40)."""
        s = np.asarray(s, dtype=float).reshape(-1)
        g = self.gamma.astype(complex) + 1j * 1e-30
        p = self.prm
        k = ramp_k(g, p.k_f, p.k_s, p.q_c)
        return self._elem_rows(s[self.ldof].astype(complex), k, brinkman(g, p)).imag / 1e-30

    def dfdgamma_explicit(self, s):
        """The compliance's weight does not depend on the design in this model."""
        return np.zeros(self.mesh.n_elems)

    def _objective_q(self, s, kap=None):
        """Volumetric compliance sum_e Q_e int_e N*^T t_e with the weight at the element's
        centroid velocity (the permeability does not enter)."""
        s = np.asarray(s).reshape(-1, NFIELD)
        src = np.nonzero(self.Qe != 0.0)[0]
        if src.size == 0:
            return 0.0
        conn = self.mesh.conn[src]
        w = ns_supg_weights(s[:, 0:3][conn], self.prm)
        return np.sum(self.Qe[src][:, None] * w * s[:, FIELD_T][conn])
