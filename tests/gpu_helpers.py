"""Glue shared by the GPU tests: oracle models with the same parameters and inputs."""

import numpy as np
import torch

import oracle
from oracle.problem import NFIELD
from paper_1904_00182_amd import nc, inputs

DEV = "cuda:0"


def oracle_params(p):
    """oracle.Params mirroring an NCProblem."""
    return oracle.Params(p.nx, p.ny, p.nz, h=p.h, rho0=p.rho0, mu=p.mu, cp=p.cp, g0=p.g0, alpha=p.alpha,
                         k_f=p.k_f, k_s=p.k_s, kappa_f=p.kappa_f, kappa_s=p.kappa_s, q_c=p.q_c, q_p=p.q_p,
                         q_h=p.q_h, patch=(p.patch_x0, p.patch_x1, p.patch_y0, p.patch_y1), Q=p.Q,
                         filter_radius=p.filter_radius)


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


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)
