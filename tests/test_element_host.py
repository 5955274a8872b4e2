"""Host build of the library's element header checked against the oracle.

The GPU kernels call the same element header; this test catches mistakes in the
element math on the CPU, before any GPU run.  The oracle is independent code (dense
shape-function tables, complex-step Jacobians)."""

import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import Params, Model, ramp_k_deriv, ramp_kappa_deriv
from oracle.problem import NFIELD
from paper_1904_00182_amd.inputs import noise_design, rng

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        out = os.path.join(tempfile.mkdtemp(prefix="nc_hostcheck_"), "libhostcheck.so")
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", out,
                               os.path.join(HERE, "native", "host_check.cpp")])
        _LIB = ctypes.CDLL(out)
    return _LIB


def ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def args(p):
    dims = np.array([p.nx, p.ny, p.nz], dtype=np.int32)
    prm = np.array([p.h, p.rho0, p.mu, p.cp, p.g0, p.alpha, p.Q, p.q_h, *p.patch], dtype=np.float64)
    return dims, prm


def setup(grid=(8, 4, 8), seed=0, **kw):
    p = Params(*grid, **kw)
    x = noise_design(p.nx * p.ny * p.nz, seed)
    m = Model(p, x)
    s = rng(seed + 100).standard_normal((m.mesh.n_nodes, NFIELD)) * 0.05
    s[:, 3] *= 20.0
    s[m.mask] = 0.0
    return p, m, s


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(params=[0, 1], ids=["gauss", "modal"])
def variant(request):
    lib().hc_set_variant(request.param)
    yield request.param
    lib().hc_set_variant(0)


@pytest.mark.parametrize("kw", [dict(alpha=1e3), dict(alpha=1e4, kappa_f=0.00206, Q=0.7, q_h=3.0)])
def test_host_residual_matches_oracle(kw, variant):
    p, m, s = setup(**kw)
    dims, prm = args(p)
    r = np.zeros_like(s)
    lib().hc_residual(ptr(dims), ptr(prm), ptr(m.k), ptr(m.kap), ptr(s), ptr(r))
    ro = m.residual(s)
    for f in range(NFIELD):
        assert rel(r[:, f], ro[:, f]) < 1e-13, f


@pytest.mark.parametrize("kw", [dict(alpha=1e3), dict(alpha=1e4, kappa_f=0.00206, Q=0.7)])
def test_host_jacobian_and_transpose_match_oracle(kw, variant):
    p, m, s = setup(**kw)
    dims, prm = args(p)
    J = m.jacobian(s)
    v = rng(5).standard_normal(s.shape)
    y = np.zeros_like(s)
    lib().hc_jv(ptr(dims), ptr(prm), ptr(m.k), ptr(m.kap), ptr(s), ptr(v), ptr(y))
    yo = (J @ v.reshape(-1)).reshape(-1, NFIELD)
    for f in range(NFIELD):
        assert rel(y[:, f], yo[:, f]) < 1e-13, ("Jv", f)
    y = np.zeros_like(s)
    lib().hc_jtw(ptr(dims), ptr(prm), ptr(m.k), ptr(m.kap), ptr(s), ptr(v), ptr(y))
    yo = (J.T @ v.reshape(-1)).reshape(-1, NFIELD)
    for f in range(NFIELD):
        assert rel(y[:, f], yo[:, f]) < 1e-13, ("JTw", f)


def test_host_sensitivity_matches_oracle():
    p, m, s = setup(alpha=1e4, kappa_f=0.00206, Q=0.3)
    dims, prm = args(p)
    lam = rng(9).standard_normal(s.shape)
    lam[m.mask] = 0.0
    dk = ramp_k_deriv(m.gamma, p.k_f, p.k_s, p.q_c)
    dkap = ramp_kappa_deriv(m.gamma, p.kappa_f, p.kappa_s, p.q_p)
    g = np.zeros(m.mesh.n_elems)
    lib().hc_sens(ptr(args(p)[0]), ptr(prm), ptr(m.k), ptr(m.kap), ptr(dk), ptr(dkap), ptr(s), ptr(lam), ptr(g))
    go, _ = m.sensitivity(s, lam)
    assert rel(g, go) < 1e-12
