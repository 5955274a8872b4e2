"""Oracle global model: assembly, Newton state solve, adjoint solve and sensitivities.
Test infrastructure only (see oracle/__init__.py).

Constraint convention.  With the free dofs f and the constrained dofs c (values
s_bar), the constrained system is
    R~_f(s) = R_f(s),        R~_c(s) = s_c - s_bar_c,
and its Jacobian is taken with the constrained columns eliminated,
    J~ = [[J_ff, 0], [0, I]].
Newton corrections are then zero on c, and the adjoint J~^T lambda = df/ds (with the
right-hand side zeroed on c) gives lambda_c = 0 and lambda_f = J_ff^-T df/ds_f, the
adjoint of the problem restricted to the free dofs (Sec. 5.1, adjoint sensitivity
analysis of eq. optprob).
"""

import time
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .problem import Mesh, default_constraints, patch_flux, element_regions, NFIELD, FIELD_P, FIELD_T
from .material import cone_filter_matrix, ramp_k, ramp_kappa
from .pde_filter import PDEFilter
from .element import element_residual, supg_weights

CSTEP = 1.0e-30     # complex-step size: derivative exact to round-off


class Model:
    # fields through which the volumetric objective depends on the state (the SUPG
    # weight's velocity is the Darcy velocity of P and T)
    objective_fields = (FIELD_P, FIELD_T)

    def __init__(self, prm, x, constraints=None, flux=None, src_P=None, src_T=None, gamma=None):
        """prm: Params; x: raw design per element (E,) in [0, 1].  The filtered density
        gamma = F x feeds RAMP (if `gamma` is given it is used as is, without a filter)."""
        self.prm = prm
        self.mesh = Mesh(prm)
        if prm.filter_kind == "pde" and prm.filter_radius > 0.0:
            self.F = PDEFilter(self.mesh, prm.filter_radius)         # Sec. 5.1 PDE filter
        else:
            self.F = cone_filter_matrix(self.mesh, prm.filter_radius)
        self.x = np.asarray(x, dtype=float)
        # passive regions of Sec. 6.1 (heat-source block solid, outside the design domain
        # fluid) and the volumetric source per element
        self.Qe, self.solid, self.fluid = element_regions(self.mesh, prm)
        self.design = ~(self.solid | self.fluid)
        if gamma is not None:
            self.gamma = np.asarray(gamma, dtype=float)
        else:
            self.gamma = self.F @ self.x
            self.gamma[self.solid] = 1.0
            self.gamma[self.fluid] = 0.0
        self.k = ramp_k(self.gamma, prm.k_f, prm.k_s, prm.q_c)
        self.kap = ramp_kappa(self.gamma, prm.kappa_f, prm.kappa_s, prm.q_p)
        if constraints is None:
            constraints = default_constraints(self.mesh, prm)
        self.mask, self.sbar = constraints
        self.flux = patch_flux(self.mesh, prm) if flux is None else np.asarray(flux, dtype=float)
        self.src_P, self.src_T = src_P, src_T
        m = self.mesh
        self.ndof = m.n_nodes * NFIELD
        # global dof of local dof (a, f): node * 5 + f, local index a * 5 + f
        self.ldof = (m.conn[:, :, None] * NFIELD + np.arange(NFIELD)[None, None, :]).reshape(m.n_elems, 8 * NFIELD)
        self.x0 = m.elem_ijk * m.h
        self.timing = {}

    # ---------------------------------------------------------------- residual
    def _elem_rows(self, se, k=None, kap=None):
        """se: (E, 40) local dofs -> (E, 40) element residual rows (complex-safe)."""
        v = se.reshape(se.shape[0], 8, NFIELD)
        k = self.k if k is None else k
        kap = self.kap if kap is None else kap
        RP, RT, RU = element_residual(v[:, :, FIELD_P], v[:, :, FIELD_T], v[:, :, 0:3], k, kap, self.prm,
                                      self.src_P, self.src_T, self.x0, self.Qe)
        out = np.empty(v.shape, dtype=np.result_type(se, k, kap))
        out[:, :, 0:3] = RU
        out[:, :, FIELD_P] = RP
        out[:, :, FIELD_T] = RT
        return out.reshape(se.shape[0], 8 * NFIELD)

    def residual_unconstrained(self, s):
        """R(s) = M(s) s - f of eq. finalsyseq for every row, as (N, 5)."""
        s = np.asarray(s, dtype=float).reshape(-1)
        re = self._elem_rows(s[self.ldof])
        R = np.zeros(self.ndof)
        np.add.at(R, self.ldof.ravel(), re.ravel())
        R = R.reshape(-1, NFIELD)
        R[:, FIELD_T] -= self.flux
        return R

    def residual(self, s):
        s = np.asarray(s, dtype=float).reshape(-1, NFIELD)
        R = self.residual_unconstrained(s)
        R[self.mask] = s[self.mask] - self.sbar[self.mask]
        return R

    # ---------------------------------------------------------------- Jacobian
    def element_jacobians(self, s):
        """Complex-step element Jacobians Je (E, 40, 40), Je[e, i, j] = d R_e,i / d s_e,j."""
        s = np.asarray(s, dtype=float).reshape(-1)
        se = s[self.ldof]
        E = se.shape[0]
        Je = np.empty((E, 8 * NFIELD, 8 * NFIELD))
        for j in range(8 * NFIELD):
            pert = se.astype(complex)
            pert[:, j] += 1j * CSTEP
            Je[:, :, j] = self._elem_rows(pert).imag / CSTEP
        return Je

    def jacobian(self, s):
        """Assembled constrained Jacobian J~ (CSR)."""
        Je = self.element_jacobians(s)
        nz = np.any(Je != 0.0, axis=0)                      # structural pattern of the element block
        li, lj = np.nonzero(nz)
        rows = self.ldof[:, li].ravel()
        cols = self.ldof[:, lj].ravel()
        vals = Je[:, li, lj].ravel()
        J = sp.csr_matrix((vals, (rows, cols)), shape=(self.ndof, self.ndof))
        free = (~self.mask).reshape(-1).astype(float)
        Df = sp.diags(free)
        return (Df @ J @ Df + sp.diags(1.0 - free)).tocsr()

    def jac_apply(self, s, v):
        return (self.jacobian(s) @ np.asarray(v, dtype=float).reshape(-1)).reshape(-1, NFIELD)

    def jacT_apply(self, s, w):
        return (self.jacobian(s).T @ np.asarray(w, dtype=float).reshape(-1)).reshape(-1, NFIELD)

    # ---------------------------------------------------------------- Newton
    def solve_state(self, s0=None, step_rtol=1e-12, maxit=50, verbose=False):
        """Damped Newton (Sec. 5.4): full step unless it increases ||R~||_2, then halve.

        Stops after a full step whose every field-block is below step_rtol relative to
        that field of the iterate (quadratic convergence makes the following error
        round-off); such a step is taken undamped (reading of the paper's stopping rule for
        the float64 floor).  Returns s (N, 5) and a history dict.
        """
        s = np.zeros((self.mesh.n_nodes, NFIELD)) if s0 is None else np.array(s0, dtype=float).reshape(-1, NFIELD)
        s[self.mask] = self.sbar[self.mask]
        R = self.residual(s)
        hist = {"res": [np.linalg.norm(R)], "lam": [], "step": []}
        t_asm = t_fac = t_sol = 0.0
        for it in range(maxit):
            t0 = time.perf_counter()
            J = self.jacobian(s)
            t1 = time.perf_counter()
            lu = spla.splu(J.tocsc())
            t2 = time.perf_counter()
            d = lu.solve(-R.reshape(-1)).reshape(-1, NFIELD)
            t3 = time.perf_counter()
            t_asm, t_fac, t_sol = t_asm + t1 - t0, t_fac + t2 - t1, t_sol + t3 - t2
            nrm = np.linalg.norm(R)
            lam = 1.0
            # a full step already below step_rtol in every field is at the round-off level of
            # the root, where the residual norm is noise and no longer orders the iterates:
            # it is taken undamped and ends the iteration
            full = [np.linalg.norm(d[:, f]) / max(np.linalg.norm(s[:, f] + d[:, f]), 1e-300) for f in range(NFIELD)]
            tiny = max(full) <= step_rtol
            while not tiny:
                st = s + lam * d
                Rt = self.residual(st)
                if np.linalg.norm(Rt) <= nrm or lam < 1.0 / 64:
                    break
                lam *= 0.5
            if tiny:
                st = s + d
                Rt = self.residual(st)
            s, R = st, Rt
            rel = [np.linalg.norm(d[:, f]) / max(np.linalg.norm(s[:, f]), 1e-300) for f in range(NFIELD)]
            hist["res"].append(np.linalg.norm(R))
            hist["lam"].append(lam)
            hist["step"].append(max(rel))
            if verbose:
                print(f"newton {it}: |R|={hist['res'][-1]:.3e} lam={lam} step={max(rel):.3e}")
            if lam == 1.0 and max(rel) <= step_rtol:
                hist["converged"] = True
                break
        hist["its"] = it + 1
        hist.setdefault("converged", False)
        self.timing.update(state_assembly=t_asm, state_factor=t_fac, state_solve=t_sol)
        return s, hist

    # ---------------------------------------------------------------- objective / adjoint
    def _objective_q(self, s, kap=None):
        """Volumetric part of the thermal compliance, sum_e f_tQ,e^T t_e (Sec. 5.1
        eq. objdiscr; f_tQ,e = int N*^T Q of App. A, with the SUPG weight); complex-safe."""
        s = np.asarray(s).reshape(-1, NFIELD)
        src = np.nonzero(self.Qe != 0.0)[0]
        if src.size == 0:
            return 0.0
        conn = self.mesh.conn[src]
        kap = self.kap if kap is None else kap
        w = supg_weights(s[:, FIELD_P][conn], s[:, FIELD_T][conn], kap[src], self.prm)
        return np.sum(self.Qe[src][:, None] * w * s[:, FIELD_T][conn])

    def objective(self, s):
        """Thermal compliance f = f_qh^T t + sum_e f_tQ,e^T t_e (Sec. 5.1 eq. objdiscr with
        the volumetric load of App. A, plus the boundary-flux load)."""
        q = self._objective_q(s)
        return float(self.flux @ np.asarray(s).reshape(-1, NFIELD)[:, FIELD_T] + np.real(q))

    def dfds(self, s=None):
        """d f / d s: the flux load on the T entries, plus the derivative of the volumetric
        part (which depends on P and T through the SUPG weight) by the complex step."""
        g = np.zeros((self.mesh.n_nodes, NFIELD))
        g[:, FIELD_T] = self.flux
        src = np.nonzero(self.Qe != 0.0)[0]
        if src.size:
            if s is None:
                raise ValueError("the volumetric objective's gradient depends on the state")
            s = np.asarray(s, dtype=float).reshape(-1, NFIELD)
            nodes = np.unique(self.mesh.conn[src])
            for f in self.objective_fields:
                for n in nodes:
                    sc = s.astype(complex)
                    sc[n, f] += 1j * CSTEP
                    g[n, f] += self._objective_q(sc).imag / CSTEP
        g[self.mask] = 0.0
        return g

    def dfdgamma_explicit(self, s):
        """Explicit d f / d gamma_e (the volumetric objective depends on the permeability
        through the SUPG weight), by the complex step through RAMP, element by element."""
        out = np.zeros(self.mesh.n_elems)
        p = self.prm
        for e in np.nonzero(self.Qe != 0.0)[0]:
            g = self.gamma.astype(complex)
            g[e] += 1j * CSTEP
            kap = ramp_kappa(g, p.kappa_f, p.kappa_s, p.q_p)
            out[e] = self._objective_q(s, kap).imag / CSTEP
        return out

    def volume(self):
        """Volume constraint of Sec. 5.1 (eq. constr): g = sum_D gamma_e v_e / sum_D v_e - g*
        is returned without g*, as the solid fraction of the design domain D, with its
        gradient with respect to the raw design x (through the filter; zero off D)."""
        D = self.design
        frac = float(self.gamma[D].sum() / D.sum())
        dg = np.where(D, 1.0 / D.sum(), 0.0)
        dx = self.F.T @ dg
        dx[~D] = 0.0
        return frac, dx

    def solve_adjoint(self, s, rhs):
        """Solve J~^T lambda = rhs (rhs zeroed on constrained dofs) with SuperLU."""
        t0 = time.perf_counter()
        J = self.jacobian(s)
        t1 = time.perf_counter()
        lu = spla.splu(J.tocsc())
        t2 = time.perf_counter()
        b = np.array(rhs, dtype=float).reshape(-1, NFIELD)
        b[self.mask] = 0.0
        lam = lu.solve(b.reshape(-1), trans="T").reshape(-1, NFIELD)
        t3 = time.perf_counter()
        self.timing.update(adjoint_assembly=t1 - t0, adjoint_factor=t2 - t1, adjoint_solve=t3 - t2)
        return lam

    def elem_dR_dgamma(self, s):
        """d R_e / d gamma_e for every element by the complex step through RAMP, (E, 40)."""
        s = np.asarray(s, dtype=float).reshape(-1)
        g = self.gamma.astype(complex) + 1j * CSTEP
        p = self.prm
        k = ramp_k(g, p.k_f, p.k_s, p.q_c)
        kap = ramp_kappa(g, p.kappa_f, p.kappa_s, p.q_p)
        return self._elem_rows(s[self.ldof].astype(complex), k, kap).imag / CSTEP

    def sensitivity(self, s, lam, explicit=False):
        """Returns (dfdgamma, dfdx): -lambda_e^T dR_e/dgamma_e per element (plus the
        objective's explicit d f/d gamma_e when `explicit`), zero on passive elements, and
        its image under the filter transpose (the design chain gamma = F x), zero off the
        design domain (passive elements are not design variables)."""
        lam = np.asarray(lam, dtype=float).reshape(-1)
        dR = self.elem_dR_dgamma(s)
        dfdg = -np.einsum("ej,ej->e", lam[self.ldof], dR)
        if explicit:
            dfdg = dfdg + self.dfdgamma_explicit(s)
        dfdg[~self.design] = 0.0
        dfdx = self.F.T @ dfdg
        dfdx[~self.design] = 0.0
        return dfdg, dfdx
