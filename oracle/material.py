"""Oracle design chain: RAMP interpolation, cone density filter and the closed-form
permeability tuning.  Test infrastructure only (see oracle/__init__.py).
"""

import numpy as np
import scipy.sparse as sp


def ramp_k(gam, k_f, k_s, q_c):
    """Conductivity RAMP, Sec. 5.2 eq. condRAMP: gamma = 0 fluid, gamma = 1 solid."""
    return k_f + gam / (1.0 + q_c * (1.0 - gam)) * (k_s - k_f)


def ramp_kappa(gam, kappa_f, kappa_s, q_p):
    """Permeability RAMP, Sec. 5.2 eq. permRAMP."""
    return kappa_s + (1.0 - gam) / (1.0 + q_p * gam) * (kappa_f - kappa_s)


def ramp_k_deriv(gam, k_f, k_s, q_c):
    """d k / d gamma of eq. condRAMP (quotient rule)."""
    return (k_s - k_f) * (1.0 + q_c) / (1.0 + q_c * (1.0 - gam)) ** 2


def ramp_kappa_deriv(gam, kappa_f, kappa_s, q_p):
    """d kappa / d gamma of eq. permRAMP (quotient rule)."""
    return -(kappa_f - kappa_s) * (1.0 + q_p) / (1.0 + q_p * gam) ** 2


def cone_filter_matrix(mesh, radius):
    """Normalised cone ("hat") density filter as an explicit sparse matrix F (E x E).

    gamma_tilde_e = sum_j w_ej x_j / sum_j w_ej with w_ej = max(0, R - |c_e - c_j| / h),
    the sum running over elements of the grid (no padding outside).  The paper
    regularises with a PDE filter (Sec. 5.1); this cone filter is the density
    filter of the workloads built here.  radius <= 0 gives the identity.
    Built by brute force over every element and every offset within the radius.
    """
    E = mesh.n_elems
    if radius <= 0.0:
        return sp.identity(E, format="csr")
    r = int(np.ceil(radius))
    rows, cols, vals = [], [], []
    ijk = mesh.elem_ijk
    for dk in range(-r, r + 1):
        for dj in range(-r, r + 1):
            for di in range(-r, r + 1):
                w = radius - np.sqrt(di * di + dj * dj + dk * dk)
                if w <= 0.0:
                    continue
                ni, nj, nk = ijk[:, 0] + di, ijk[:, 1] + dj, ijk[:, 2] + dk
                ok = (ni >= 0) & (ni < mesh.nx) & (nj >= 0) & (nj < mesh.ny) & (nk >= 0) & (nk < mesh.nz)
                e = np.nonzero(ok)[0]
                rows.append(e)
                cols.append(mesh.elem_id(ni[ok], nj[ok], nk[ok]))
                vals.append(np.full(e.size, w))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    Wm = sp.csr_matrix((vals, (rows, cols)), shape=(E, E))
    rowsum = np.asarray(Wm.sum(axis=1)).ravel()
    return sp.diags(1.0 / rowsum) @ Wm


def kappa_f_tuning(alpha, dT, H=1.0, L=0.5, g=1.0, nu=1.0, beta=1.0, beta_m=1.0):
    """Fluid permeability from equal average Nusselt numbers, Sec. 3.

    Sets the pure-fluid enclosure correlation (eqs. nusselt1, nusselt2) equal to the
    porous-enclosure estimate (eqs. nusselt3, nusselt4) and solves for kappa.
    Worked from those two relations directly:
        (L/H)^2 g alpha kappa H dT / (nu beta_m)
            = 0.18^2 (Pr/(0.2+Pr))^0.58 (g alpha dT H^3 / (nu beta))^0.58
    which gives the printed eq. nusselt5 except that the height enters as H^2.74 (the
    printed H^1.74 is irrelevant at H = 1, the only value used).
    """
    Pr = nu / beta
    ra_h = g * alpha * dT * H ** 3 / (nu * beta)           # Ra_H = Gr_H Pr
    nu_fluid = 0.18 * (Pr / (0.2 + Pr) * ra_h) ** 0.29      # eq. nusselt1
    # eq. nusselt3: Nu = (L/H) Ra^0.5 with Ra = g alpha kappa H dT / (nu beta_m)  (eq. nusselt4)
    ra_needed = (nu_fluid * H / L) ** 2
    return ra_needed * nu * beta_m / (g * alpha * H * dT)
