"""Oracle element residual of the stabilised weak form, App. A eq. weakstable.
Test infrastructure only (see oracle/__init__.py).

Written in the dense textbook form: shape-function values and gradients are
tabulated at the eight 2x2x2 Gauss points and every integral is a plain sum over
those points.  The routine is vectorised over elements and is complex-safe, so the
caller can differentiate it by the complex step.
"""

import numpy as np

GAUSS = 1.0 / np.sqrt(3.0)
# reference coordinates (+-1) of local node a = ia + 2 ja + 4 ka
NODE_SIGN = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1] for a in range(8)], dtype=float)


def _shape(xi):
    """Trilinear shape functions N_a(xi) = prod_d (1 + s_ad xi_d) / 2 and their
    reference gradients at one point xi of [-1, 1]^3."""
    lin = 0.5 * (1.0 + NODE_SIGN * xi[None, :])        # (8, 3): factors per direction
    N = lin.prod(axis=1)
    dN = np.empty((8, 3))
    for d in range(3):
        others = [o for o in range(3) if o != d]
        dN[:, d] = 0.5 * NODE_SIGN[:, d] * lin[:, others[0]] * lin[:, others[1]]
    return N, dN


def supg_weights(Pe, Te, kap, prm):
    """Integrated SUPG weights int_e N*_a = int_e (N_a + tau u0 . grad N_a), (E, 8), at
    the centroid velocity u0 of each element (App. A); complex-safe."""
    h = prm.h
    N, G, Nc, Gc, detJ, _ = reference_element(h)
    buoy = prm.rho0 * prm.alpha * np.array([0.0, 0.0, -prm.g0])
    gradPc = np.einsum("ad,ea->ed", Gc, Pe)
    Tc = np.einsum("a,ea->e", Nc, Te)
    u0 = -(kap / prm.mu)[:, None] * (gradPc + Tc[:, None] * buoy)
    he2 = 3.0 * h * h
    tau = (4.0 * np.einsum("ed,ed->e", u0, u0) / he2 + 16.0 / (he2 * he2)) ** (-0.5)
    Nstar = N[None, :, :] + tau[:, None, None] * np.einsum("ed,qad->eqa", u0, G)
    return detJ * Nstar.sum(axis=1)


def reference_element(h):
    """Gauss points, weights and shape data of a cube of edge h.

    Returns (N, G, Nc, Gc, detJ, xq) with N[q, a], physical gradients G[q, a, d]
    = (2/h) dN/dxi at Gauss point q (q numbered like the nodes, point = sign * 1/sqrt3),
    the centroid values Nc[a] and gradients Gc[a, d], the Jacobian determinant
    h^3 / 8 (unit Gauss weights) and the Gauss points in [0, h]^3.
    """
    N = np.empty((8, 8))
    G = np.empty((8, 8, 3))
    for q in range(8):
        n, dn = _shape(GAUSS * NODE_SIGN[q])
        N[q] = n
        G[q] = dn * (2.0 / h)
    nc, dnc = _shape(np.zeros(3))
    xq = 0.5 * h * (1.0 + GAUSS * NODE_SIGN)
    return N, G, nc, dnc * (2.0 / h), h ** 3 / 8.0, xq


def element_residual(Pe, Te, Ue, k, kap, prm, src_P=None, src_T=None, x0=None, Qe=None):
    """Element rows of R(s) for every element at once.

    Pe, Te : (E, 8) nodal modified pressure and temperature
    Ue     : (E, 8, 3) nodal velocity unknowns
    k, kap : (E,) element conductivity and permeability
    Qe     : optional (E,) volumetric source per element (default: prm.Q everywhere)
    src_P, src_T : optional callables f(x) -> (E, 8) giving volumetric sources at the
             physical Gauss points x (E, 8, 3); x0 (E, 3) is each element's origin.
    Returns RP (E, 8), RT (E, 8), RU (E, 8, 3).

    Rows (sums over Gauss points q with weight detJ):
      Darcy velocity, Sec. 2.1 eq. finaldarcy with T0 = 0 and g = (0, 0, -g0):
          u_q = -(kappa/mu) (grad P_q + rho0 alpha g T_q)
      pressure row, first line of eq. weakstable (q_u = 0 on all walls):
          R_P,a = sum_q detJ (kappa/mu) grad N_a . (grad P_q + rho0 alpha g T_q)
      energy row, second and third lines of eq. weakstable with the SUPG weight of
      App. A, N*_a = N_a + tau u0 . grad N_a, u0 the Darcy velocity at the centroid:
          R_T,a = sum_q detJ [ N*_a (rho0 c_p u_q . grad T_q - Q) + k grad N_a . grad T_q ]
        (the boundary flux is added by the caller)
      SUPG parameter: tau = (tau1^-2 + tau3^-2)^(-1/2), tau1 = h_e / (2 |u0|),
        tau3 = h_e^2 / 4, h_e = sqrt(dx^2 + dy^2 + dz^2); written without the
        division by |u0| so that u0 = 0 is regular and the complex step works.
      velocity rows (nodal lumped projection of the Darcy velocity):
          R_U,a = sum_q detJ N_a(q) (U_a - u_q)
    """
    h = prm.h
    N, G, Nc, Gc, detJ, xq = reference_element(h)
    gvec = np.array([0.0, 0.0, -prm.g0])
    buoy = prm.rho0 * prm.alpha * gvec                       # rho0 alpha g

    gradP = np.einsum("qad,ea->eqd", G, Pe)
    Tq = np.einsum("qa,ea->eq", N, Te)
    gradT = np.einsum("qad,ea->eqd", G, Te)
    kmu = (kap / prm.mu)[:, None, None]
    uq = -kmu * (gradP + Tq[..., None] * buoy)

    gradPc = np.einsum("ad,ea->ed", Gc, Pe)
    Tc = np.einsum("a,ea->e", Nc, Te)
    u0 = -(kap / prm.mu)[:, None] * (gradPc + Tc[:, None] * buoy)
    he2 = 3.0 * h * h                                        # dx = dy = dz = h
    tau = (4.0 * np.einsum("ed,ed->e", u0, u0) / he2 + 16.0 / (he2 * he2)) ** (-0.5)
    Nstar = N[None, :, :] + tau[:, None, None] * np.einsum("ed,qad->eqa", u0, G)

    Q = prm.Q if Qe is None else np.asarray(Qe)[:, None]
    conv = prm.rho0 * prm.cp * np.einsum("eqd,eqd->eq", uq, gradT) - Q
    RP = detJ * np.einsum("qad,eqd->ea", G, -uq)
    RT = detJ * (np.einsum("eqa,eq->ea", Nstar, conv) + k[:, None] * np.einsum("qad,eqd->ea", G, gradT))
    mass = detJ * N.sum(axis=0)                              # lumped element mass per node
    RU = mass[None, :, None] * Ue - detJ * np.einsum("qa,eqd->ead", N, uq)

    if src_P is not None or src_T is not None:
        xg = x0[:, None, :] + xq[None, :, :]
        if src_P is not None:
            RP = RP - detJ * np.einsum("qa,eq->ea", N, src_P(xg))
        if src_T is not None:
            RT = RT - detJ * np.einsum("eqa,eq->ea", Nstar, src_T(xg))
    return RP, RT, RU
