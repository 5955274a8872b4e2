"""Glue shared by the GPU tests: oracle models with the same parameters and inputs."""

import numpy as np
import torch

import oracle
from oracle.problem import NFIELD
from paper_1904_00182_amd import nc, inputs

DEV = "cuda:0"


def _box(b):
    b = tuple(float(v) for v in b)
    return b if (b[1] > b[0] and b[3] > b[2] and b[5] > b[4]) else None


def oracle_params(p):
    """oracle.Params mirroring an NCProblem."""
    return oracle.Params(p.nx, p.ny, p.nz, h=p.h, rho0=p.rho0, mu=p.mu, cp=p.cp, g0=p.g0, alpha=p.alpha,
                         k_f=p.k_f, k_s=p.k_s, kappa_f=p.kappa_f, kappa_s=p.kappa_s, q_c=p.q_c, q_p=p.q_p,
                         q_h=p.q_h, patch=(p.patch_x0, p.patch_x1, p.patch_y0, p.patch_y1), Q=p.Q,
                         filter_radius=p.filter_radius, filter_kind="pde" if p.filter_kind == nc.NC_FILTER_PDE else "cone",
                         q_box=_box(p.q_box), solid_box=_box(p.solid_box), design_box=_box(p.design_box),
                         sym_x=bool(p.sym_x), sym_y=bool(p.sym_y))


def oracle_blob_design(grid, seed):
    """The 'blobs' recipe with the oracle's own cone filter (radius 2, threshold 0.5)."""
    prm = oracle.Params(*grid)
    F = oracle.cone_filter_matrix(oracle.Mesh(prm), 2.0)
    x0 = inputs.uniform_design(prm.nx * prm.ny * prm.nz, seed)
    return (F @ x0 >= 0.5).astype(np.float64)


def random_state(model, seed, pscale=20.0, scale=0.05):
    s = inputs.rng(seed).standard_normal((model.mesh.n_nodes, NFIELD)) * scale
    s[:, 3] *= pscale
    s[model.mask] = 0.0
    return s


def rel_fields(a, b):
    a = np.asarray(a).reshape(-1, NFIELD)
    b = np.asarray(b).reshape(-1, NFIELD)
    return [float(np.linalg.norm(a[:, f] - b[:, f]) / max(np.linalg.norm(b[:, f]), 1e-300)) for f in range(NFIELD)]


def field_errors(a, b):
    """Per field of [N][F] arrays: (relative l2 error, element-wise max|a - b| / max|b|);
    None for a field that is zero in b (it must then be zero in a as well)."""
    a = np.asarray(a)
    b = np.asarray(b)
    a = a.reshape(len(a), -1)
    b = b.reshape(len(b), -1)
    out = []
    for f in range(b.shape[1]):
        nb = np.linalg.norm(b[:, f])
        if nb == 0.0:
            assert np.abs(a[:, f]).max() == 0.0, ("field", f, "must be zero")
            out.append(None)
            continue
        d = a[:, f] - b[:, f]
        out.append((float(np.linalg.norm(d) / nb), float(np.abs(d).max() / np.abs(b[:, f]).max())))
    return out


def check_fields(a, b, tol, what="", max_tol=None):
    """Asserts relative l2 <= tol and element-wise max|a - b| / max|b| <= max_tol (default
    tol) in every field that is not identically zero in b; returns the errors."""
    max_tol = tol if max_tol is None else max_tol
    errs = field_errors(a, b)
    for f, e in enumerate(errs):
        if e is not None:
            assert e[0] <= tol and e[1] <= max_tol, (what, "field", f, "l2, max", e, "tol", tol, max_tol)
    print(what, "errors (l2, max) per field:", errs, flush=True)
    return errs


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def local_rows(p, s, k, kap, nodes, v=None, transpose_w=None):
    """Oracle rows at a few nodes of a large grid, computed from the elements around
    each node only (oracle.element_residual, complex step for the Jacobian).

    Returns an array (len(nodes), 5): R~ at those nodes, or (J~ v) when v is given.
    s, v: (N, 5) float64; k, kap: (E,) element coefficients; nodes: list of (i, j, k).
    """
    prm = oracle_params(p)
    mesh = oracle.Mesh(prm)
    mask, _ = oracle.default_constraints(mesh, prm)
    out = np.zeros((len(nodes), NFIELD))
    h = 1e-30
    for r, (i, j, kk) in enumerate(nodes):
        n = mesh.node_id(i, j, kk)
        elems, corner = [], []
        for c in range(8):
            ei, ej, ek = i - (c & 1), j - ((c >> 1) & 1), kk - ((c >> 2) & 1)
            if 0 <= ei < p.nx and 0 <= ej < p.ny and 0 <= ek < p.nz:
                elems.append(mesh.elem_id(ei, ej, ek))
                corner.append(c)
        elems = np.array(elems)
        conn = mesh.conn[elems]
        se = s[conn]                                    # (Ee, 8, 5)
        if transpose_w is not None:
            wm = transpose_w.copy()
            wm[mask] = 0.0
            we = wm[conn]
            for f in range(NFIELD):
                if mask[n, f]:
                    out[r, f] = transpose_w[n, f]
                    continue
                sp = se.astype(complex)
                for e_loc, c in enumerate(corner):
                    sp[e_loc, c, f] += 1j * h
                RP, RT, RU = oracle.element_residual(sp[:, :, 3], sp[:, :, 4], sp[:, :, 0:3], k[elems], kap[elems], prm)
                col = (np.einsum("ea,ea->", RP.imag, we[:, :, 3]) + np.einsum("ea,ea->", RT.imag, we[:, :, 4])
                       + np.einsum("ead,ead->", RU.imag, we[:, :, 0:3])) / h
                out[r, f] = col
            continue
        if v is not None:
            vm = v.copy()
            vm[mask] = 0.0
            se = se.astype(complex) + 1j * h * vm[conn]
        RP, RT, RU = oracle.element_residual(se[:, :, 3], se[:, :, 4], se[:, :, 0:3], k[elems], kap[elems], prm)
        row = np.zeros(NFIELD, dtype=se.dtype)
        for e_loc, c in enumerate(corner):
            row[0:3] += RU[e_loc, c]
            row[3] += RP[e_loc, c]
            row[4] += RT[e_loc, c]
        if v is None:
            row = row.real
            # flux load of the patch faces around a bottom node
            if kk == 0:
                x0, x1, y0, y1 = prm.patch
                for c in range(4):
                    fi, fj = i - (c & 1), j - (c >> 1)
                    if 0 <= fi < p.nx and 0 <= fj < p.ny:
                        xc, yc = (fi + 0.5) * prm.h, (fj + 0.5) * prm.h
                        if x0 <= xc <= x1 and y0 <= yc <= y1:
                            row[4] -= prm.q_h * prm.h * prm.h / 4
            for f in range(NFIELD):
                if mask[n, f]:
                    row[f] = s[n, f]
        else:
            row = row.imag / h
            for f in range(NFIELD):
                if mask[n, f]:
                    row[f] = v[n, f]
        out[r] = row
    return out


def sample_nodes(p, count, seed):
    """Random nodes plus corners, wall, top, pinned and patch nodes."""
    g = inputs.rng(seed)
    pts = {(0, 0, 0), (p.nx, p.ny, p.nz), (0, 0, p.nz), (p.nx, 0, 0), (0, p.ny, 0),
           (p.nx // 2, p.ny // 2, 0), (p.nx // 2, p.ny // 4, 0), (p.nx // 2 + 1, p.ny // 4, 0),
           (1, 1, p.nz - 1), (p.nx - 1, p.ny - 1, 1), (p.nx // 2, p.ny // 2, p.nz // 2)}
    while len(pts) < count:
        pts.add((int(g.integers(p.nx + 1)), int(g.integers(p.ny + 1)), int(g.integers(p.nz + 1))))
    return sorted(pts)
