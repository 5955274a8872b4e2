"""Pins of the oracle's Navier-Stokes / Brinkman model (the full-flow model of the hybrid
strategy, Sec. 6.4) against exact solutions, hand-derived element integrals, a 1D
reduction, a symmetry reduction, the sign structure of the saddle-point Jacobian and
brute-force finite differences."""

import numpy as np
import pytest

from oracle import Params, Mesh, NSModel, ns_element_residual, ns_constraints, brinkman
from oracle.problem import FIELD_P, FIELD_T, NFIELD
from paper_1904_00182_amd.inputs import noise_design, rng

from test_oracle_pins import _benchmark_boxes, _quarter, rel


def _interior(mesh):
    i, j, k = mesh.node_ijk[:, 0], mesh.node_ijk[:, 1], mesh.node_ijk[:, 2]
    return (i > 0) & (i < mesh.nx) & (j > 0) & (j < mesh.ny) & (k > 0) & (k < mesh.nz)


def _boundary_data_model(p, gamma, s_exact, src_T=None):
    """Every boundary node's u, v, w and T held at the exact field, P at one node."""
    m = Mesh(p)
    inner = _interior(m)
    mask = np.zeros((m.n_nodes, NFIELD), dtype=bool)
    mask[:, 0:3] = ~inner[:, None]
    mask[:, FIELD_T] = ~inner
    mask[m.node_id(0, 0, m.nz), FIELD_P] = True
    return NSModel(p, np.zeros(m.n_elems), constraints=(mask, s_exact.copy()), src_T=src_T, flux=np.zeros(m.n_nodes),
                   gamma=gamma)


# --------------------------------------------------------------------------- P18
def test_exact_shear_flow_with_convection():
    """u = (c1 z + c2 y + b_x, b_y, b_z) is divergence free with constant convective
    acceleration (b_y c2 + b_z c1, 0, 0), balanced by a linear P; with no Brinkman
    friction (pure fluid) and no buoyancy every term of the momentum and continuity rows
    is exact at the Gauss points, the stabilising terms vanish with the strong residual,
    and T = t1 x with the heat source rho0 c_p u . grad T makes the energy rows exact.
    Interior rows vanish to round-off, and Newton from zero with the exact boundary data
    returns the exact nodal fields.  A transposed convective term ((grad u)^T u), a
    dropped viscous half of the symmetric gradient or a wrong pressure sign all fail."""
    p = Params(4, 3, 5, h=0.2, alpha=0.0, rho0=1.3, mu=0.7, cp=1.1, q_h=0.0)
    m = Mesh(p)
    c1, c2, b = 0.9, -0.6, np.array([0.4, 0.7, -0.5])
    t1 = 0.8
    X = m.node_xyz
    s = np.zeros((m.n_nodes, NFIELD))
    s[:, 0] = c1 * X[:, 2] + c2 * X[:, 1] + b[0]
    s[:, 1] = b[1]
    s[:, 2] = b[2]
    s[:, FIELD_P] = -p.rho0 * (b[1] * c2 + b[2] * c1) * X[:, 0]
    s[:, FIELD_T] = t1 * X[:, 0]

    def src_T(xg):
        ux = c1 * xg[..., 2] + c2 * xg[..., 1] + b[0]
        return p.rho0 * p.cp * ux * t1

    model = _boundary_data_model(p, np.zeros(m.n_elems), s, src_T=src_T)
    R = model.residual_unconstrained(s)
    inner = _interior(m)
    assert np.abs(R[inner]).max() <= 1e-13, np.abs(R[inner]).max(axis=0)
    # every term is active: the rows are not small term by term
    R_wrong = model.residual_unconstrained(s + 0.01 * rng(1).standard_normal(s.shape))
    assert np.abs(R_wrong[inner]).max() > 1e-5
    sol, hist = model.solve_state()
    assert hist["converged"]
    for f in range(NFIELD):
        assert np.abs(sol[:, f] - s[:, f]).max() <= 1e-12 * max(np.abs(s[:, f]).max(), 1.0), f


def test_exact_brinkman_flow_with_buoyancy():
    """A uniform velocity b through a uniform porous medium (Brinkman coefficient a of the
    impermeability interpolation) under uniform temperature t0: grad P = -a b - rho0 alpha g t0
    (P linear), no convection or viscous stress, T rows trivially exact.  Interior rows
    vanish; Newton returns the fields.  Checks the Brinkman and buoyancy signs against the
    pressure gradient."""
    p = Params(3, 4, 3, h=0.25, alpha=300.0, q_h=0.0, kappa_s=1e3)
    m = Mesh(p)
    gam = 0.3
    a = brinkman(np.array([gam]), p)[0]
    assert abs(a - 1e3 * 8.0 * 0.3 / 8.7) <= 1e-12 * a
    b, t0 = np.array([0.02, -0.03, 0.05]), 0.7
    X = m.node_xyz
    s = np.zeros((m.n_nodes, NFIELD))
    s[:, 0:3] = b
    s[:, FIELD_T] = t0
    s[:, FIELD_P] = -a * (X @ b) + p.rho0 * p.alpha * p.g0 * t0 * X[:, 2]
    model = _boundary_data_model(p, np.full(m.n_elems, gam), s)
    R = model.residual_unconstrained(s)
    inner = _interior(m)
    assert np.abs(R[inner]).max() <= 1e-12 * a * np.abs(b).max() * p.h ** 3, np.abs(R[inner]).max(axis=0)
    sol, hist = model.solve_state()
    assert hist["converged"]
    for f in range(NFIELD):
        assert np.abs(sol[:, f] - s[:, f]).max() <= 1e-11 * max(np.abs(s[:, f]).max(), 1.0), f


# --------------------------------------------------------------------------- P19
def _signs(a):
    return np.array([2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1], dtype=float)


def _one_element(p, U, P, T, a=0.0, k=1.0, Q=0.0):
    RU, RP, RT = ns_element_residual(U[None], P[None], T[None], np.array([k]), np.array([a]), p,
                                     Qe=np.array([Q]))
    return RU[0], RP[0], RT[0]


def test_element_integrals_closed_form():
    """Single element of edge h with hand-integrated rows (int N_a = h^3/8 and
    int dN_a/dx_j = s_aj h^2/4 exactly; the strong residual is constant):

    * u = (U, 0, w1 x/h): convective acceleration (0, 0, U w1/h), centroid velocity
      (U, 0, w1/2), tau_m = (4 (U^2 + w1^2/4)/h_e^2 + 16 nu^2/h_e^4)^(-1/2), h_e^2 = 3 h^2:
        R_w,a = rho U w1 h^2/8 + tau_m rho U w1 h (U s_ax + w1 s_az / 2)/4 + mu s_ax w1 h/4
        R_u,a = mu s_az w1 h/4,  R_v,a = 0,  R_P,a = tau_m U w1 s_az h/4
    * uniform u = (U, 0, 0) with Brinkman coefficient a (tau_m gains (a/rho)^2):
        R_u,a = a U (h^3/8 + tau_m U s_ax h^2/4),  R_P,a = tau_m a U s_ax h^2/(4 rho)
    * rest, uniform T = t0: R_w,a = -rho alpha g0 t0 h^3/8, R_P,a = -tau_m alpha g0 t0 s_az h^2/4
    * rest, P = p1 x: R_u,a = p1 h^3/8, R_P,a = tau_m p1 s_ax h^2/(4 rho)
    * u = (U, 0, 0), T = t1 x/h, no buoyancy: the energy row with
      tau = (4 U^2/h_e^2 + 16/h_e^4)^(-1/2):
        R_T,a = (h^3/8 + tau U s_ax h^2/4)(rho c_p U t1/h - Q) + k s_ax h t1/4
    """
    h = 0.5
    p = Params(1, 1, 1, h=h, rho0=1.2, mu=0.8, cp=1.5, alpha=40.0, g0=1.0)
    rho, mu = p.rho0, p.mu
    nu = mu / rho
    he2 = 3 * h * h
    S = np.array([_signs(a) for a in range(8)])
    xa = h * (S + 1) / 2                                     # node coordinates
    zero8 = np.zeros(8)

    U, w1 = 0.7, -1.3
    Ue = np.zeros((8, 3))
    Ue[:, 0] = U
    Ue[:, 2] = w1 * xa[:, 0] / h
    RU, RP, RT = _one_element(Params(1, 1, 1, h=h, rho0=rho, mu=mu, cp=1.5, alpha=0.0), Ue, zero8, zero8)
    tau = (4 * (U * U + w1 * w1 / 4) / he2 + 16 * nu * nu / he2 ** 2) ** -0.5
    Rw = rho * U * w1 * h * h / 8 + tau * rho * U * w1 * h * (U * S[:, 0] + w1 * S[:, 2] / 2) / 4 \
        + mu * S[:, 0] * w1 * h / 4
    assert np.abs(RU[:, 2] - Rw).max() <= 1e-14
    assert np.abs(RU[:, 0] - mu * S[:, 2] * w1 * h / 4).max() <= 1e-14
    assert np.abs(RU[:, 1]).max() <= 1e-15
    assert np.abs(RP - tau * U * w1 * S[:, 2] * h / 4).max() <= 1e-14
    assert np.abs(RT).max() <= 1e-15

    a = 250.0
    Ue = np.zeros((8, 3))
    Ue[:, 0] = U
    RU, RP, _ = _one_element(Params(1, 1, 1, h=h, rho0=rho, mu=mu, alpha=0.0), Ue, zero8, zero8, a=a)
    tau = (4 * U * U / he2 + 16 * nu * nu / he2 ** 2 + (a / rho) ** 2) ** -0.5
    assert np.abs(RU[:, 0] - a * U * (h ** 3 / 8 + tau * U * S[:, 0] * h * h / 4)).max() <= 1e-13
    assert np.abs(RU[:, 1:]).max() <= 1e-15
    assert np.abs(RP - tau * a * U * S[:, 0] * h * h / (4 * rho)).max() <= 1e-14

    t0 = 0.6
    RU, RP, RT = _one_element(p, np.zeros((8, 3)), zero8, np.full(8, t0), a=a)
    tau = (16 * nu * nu / he2 ** 2 + (a / rho) ** 2) ** -0.5
    assert np.abs(RU[:, 2] + rho * p.alpha * p.g0 * t0 * h ** 3 / 8).max() <= 1e-13
    assert np.abs(RU[:, :2]).max() <= 1e-15
    assert np.abs(RP + tau * p.alpha * p.g0 * t0 * S[:, 2] * h * h / 4).max() <= 1e-14
    assert np.abs(RT).max() <= 1e-15

    p1 = 2.1
    RU, RP, _ = _one_element(p, np.zeros((8, 3)), p1 * xa[:, 0], zero8)
    tau = (16 * nu * nu / he2 ** 2) ** -0.5
    assert np.abs(RU[:, 0] - p1 * h ** 3 / 8).max() <= 1e-14
    assert np.abs(RP - tau * p1 * S[:, 0] * h * h / (4 * rho)).max() <= 1e-14

    t1, k, Q = 0.9, 3.0, 2.5
    Ue = np.zeros((8, 3))
    Ue[:, 0] = U
    pT = Params(1, 1, 1, h=h, rho0=rho, mu=mu, cp=1.5, alpha=0.0)
    _, _, RT = _one_element(pT, Ue, zero8, t1 * xa[:, 0] / h, k=k, Q=Q)
    tauT = (4 * U * U / he2 + 16 / he2 ** 2) ** -0.5
    ref = (h ** 3 / 8 + tauT * U * S[:, 0] * h * h / 4) * (rho * 1.5 * U * t1 / h - Q) + k * S[:, 0] * h * t1 / 4
    assert np.abs(RT - ref).max() <= 1e-14


# --------------------------------------------------------------------------- P20
def test_hydrostatic_pressure_from_the_pspg_rows():
    """With the velocity held at zero everywhere and T = z held everywhere, only the
    continuity rows remain, and they reduce to tau_m int grad N . (grad P - rho0 alpha g0 T
    e_z) = 0: the pressure-stabilising term alone fixes P.  Its nodal solution is exact,
    P = rho0 alpha g0 (z^2 - Lz^2)/2 (P = 0 on the top corner), even though P is
    quadratic: each element's integral vanishes once dP/dz equals the layer mean of
    rho0 alpha g0 T, whatever the element's tau_m (here varying with a random design)."""
    p = Params(3, 2, 6, alpha=500.0, rho0=1.4, g0=0.9)
    m = Mesh(p)
    mask = np.zeros((m.n_nodes, NFIELD), dtype=bool)
    mask[:, 0:3] = True
    mask[:, FIELD_T] = True
    mask[m.node_id(0, 0, m.nz), FIELD_P] = True
    sbar = np.zeros((m.n_nodes, NFIELD))
    z = m.node_xyz[:, 2]
    sbar[:, FIELD_T] = z
    model = NSModel(p, noise_design(m.n_elems, 31), constraints=(mask, sbar), flux=np.zeros(m.n_nodes))
    s, hist = model.solve_state()
    assert hist["converged"]
    Lz = m.nz * p.h
    exact = p.rho0 * p.alpha * p.g0 * (z * z - Lz * Lz) / 2
    assert np.abs(s[:, FIELD_P] - exact).max() <= 1e-12 * np.abs(exact).max()


# --------------------------------------------------------------------------- P21
def test_quarter_domain_with_symmetry_planes_equals_full_domain():
    """The symmetric-gradient viscous term makes the natural condition of the tangential
    rows on a symmetry plane the symmetry condition, so the quarter cavity with u.n = 0
    on its mirror planes reproduces the full cavity node for node (heat-source block,
    passive solid and fluid, design mirror-symmetric in x and y), adjoint and
    sensitivities included."""
    L, n = 1.0, 8
    src, des = _benchmark_boxes(L)
    kw = dict(alpha=1e4, q_h=0.0, Q=40.0, kappa_s=1e5)
    pf = Params(n, n, n, q_box=src, solid_box=src, design_box=des, **kw)
    x = noise_design(n ** 3, 41).reshape(n, n, n)
    x = 0.25 * (x + x[:, :, ::-1] + x[:, ::-1, :] + x[:, ::-1, ::-1])
    mf = NSModel(pf, x.ravel())
    sf, hf = mf.solve_state()
    assert hf["converged"]
    lf = mf.solve_adjoint(sf, mf.dfds(sf))
    gf, _ = mf.sensitivity(sf, lf, explicit=True)
    pq = Params(n // 2, n // 2, n, h=pf.h, q_box=_quarter(src, L), solid_box=_quarter(src, L),
                design_box=_quarter(des, L), sym_x=True, sym_y=True, **kw)
    mq = NSModel(pq, x[:, : n // 2, : n // 2].ravel())
    sq, hq = mq.solve_state()
    assert hq["converged"]
    lq = mq.solve_adjoint(sq, mq.dfds(sq))
    gq, _ = mq.sensitivity(sq, lq, explicit=True)
    ijk = mq.mesh.node_ijk
    full_ids = mf.mesh.node_id(ijk[:, 0], ijk[:, 1], ijk[:, 2])
    for f in range(NFIELD):
        assert np.abs(sq[:, f] - sf[full_ids, f]).max() <= 1e-10 * np.abs(sf[:, f]).max(), f
        assert np.abs(lq[:, f] - lf[full_ids, f]).max() <= 1e-9 * np.abs(lf[:, f]).max(), f
    e = mq.mesh.elem_ijk
    assert np.abs(gq - gf[mf.mesh.elem_id(e[:, 0], e[:, 1], e[:, 2])]).max() <= 1e-9 * np.abs(gf).max()
    assert abs(4 * mq.objective(sq) - mf.objective(sf)) <= 1e-11 * abs(mf.objective(sf))
    # the flow is real: the velocity is not negligible next to the no-slip scale
    assert np.abs(sf[:, 2]).max() > 1e-3


# --------------------------------------------------------------------------- P22
def test_saddle_point_sign_structure_at_rest():
    """At rest, in pure fluid and without buoyancy, the Galerkin pressure-gradient and
    divergence blocks are negative transposes of each other on the free dofs, so the
    symmetric part of the Jacobian is block diagonal: the symmetric-gradient viscous
    stiffness, tau_m times the pressure Laplacian (PSPG) and the conduction stiffness --
    positive semidefinite, with a positive pressure block.  A flipped continuity row,
    PSPG or viscous sign makes it indefinite."""
    p = Params(3, 3, 3, alpha=0.0, q_h=0.0)
    m = Mesh(p)
    model = NSModel(p, np.zeros(m.n_elems))
    J = model.jacobian(np.zeros((m.n_nodes, NFIELD))).toarray()
    free = ~model.mask.reshape(-1)
    Jf = J[np.ix_(free, free)]
    Sym = 0.5 * (Jf + Jf.T)
    ev = np.linalg.eigvalsh(Sym)
    assert ev.min() >= -1e-13 * ev.max(), ev.min()
    fld = np.tile(np.arange(NFIELD), m.n_nodes)[free]
    u = fld < 3
    P = fld == FIELD_P
    assert np.abs(Sym[np.ix_(u, P)]).max() <= 1e-15 * np.abs(Jf[np.ix_(u, P)]).max()
    assert np.abs(Jf[np.ix_(u, P)]).max() > 0
    assert np.linalg.eigvalsh(Sym[np.ix_(P, P)]).max() > 0


# --------------------------------------------------------------------------- P23
@pytest.mark.parametrize("filt", [0.0, 1.5])
def test_adjoint_gradient_vs_brute_force_fd(filt):
    """df/dx of the compliance with a patch flux and a volumetric source block (whose
    SUPG weight depends on the velocity unknowns) from the adjoint, against central
    differences of f(x) over full Newton solves."""
    n = 4
    src = (0.25, 0.75, 0.25, 0.75, 0.0, 0.25)
    p = Params(n, n, n, alpha=1e3, q_h=5.0, Q=40.0, q_box=src, filter_radius=filt, kappa_s=1e4)
    m = Mesh(p)
    x = noise_design(m.n_elems, 51)
    model = NSModel(p, x)
    s, _ = model.solve_state()
    g = model.dfds(s)
    assert np.abs(g[:, 0:3]).max() > 0          # the weight's velocity dependence enters
    lam = model.solve_adjoint(s, g)
    _, dfdx = model.sensitivity(s, lam, explicit=True)
    eps = 1e-5
    for j in rng(52).choice(m.n_elems, 12, replace=False):
        vals = []
        for sgn in (1, -1):
            xx = x.copy()
            xx[j] += sgn * eps
            mm = NSModel(p, xx)
            ss, _ = mm.solve_state(s0=s)
            vals.append(mm.objective(ss))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - dfdx[j]) <= 1e-6 * np.abs(dfdx).max() + 1e-6 * abs(dfdx[j]), (j, fd, dfdx[j])
