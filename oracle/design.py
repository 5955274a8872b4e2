"""Oracle design loop of Sec. 5: the volume-constrained compliance minimisation of
eq. optprob by MMA, with the continuation of Sec. 5.3 and the solver practice of
Sec. 5.4.  Test infrastructure only (see oracle/__init__.py).

One design iteration: filter and passive regions (gamma), RAMP at the current continuation
stage, the state solve warm-started from the previous design's state (Sec. 5.4), with a
ramp of the heat source Q when that Newton solve fails (Sec. 5.4), the compliance and its
adjoint sensitivities, the volume constraint g = frac - g* and its gradient (eq. constr),
then one MMA update of the design elements (move limit of Sec. 6.1).  The objective is
passed to MMA as f / f0 (f0 the first iteration's compliance): the paper does not state a
scaling.
"""

from dataclasses import replace

import numpy as np

from .fem import Model
from .mma import MMA

# eq. contsch1: (q_c, q_p, kappa_s) of the five stages, advanced every `every` iterations
CONTINUATION = ((0.881, 8.0, 1e-5), (8.81, 8.0, 1e-5), (88.1, 8.0, 1e-5), (88.1, 98.0, 1e-6), (881.0, 998.0, 1e-7))
Q_RAMP = (0.25, 0.5, 0.75, 1.0)


def stage_params(prm, it, every, continuation=CONTINUATION):
    q_c, q_p, kappa_s = continuation[min(it // every, len(continuation) - 1)]
    return replace(prm, q_c=q_c, q_p=q_p, kappa_s=kappa_s)


def solve_with_ramp(prm, x, s0):
    """Newton from s0; if it fails, the heat source is ramped up through Q_RAMP, each stage
    warm-started from the last.  Returns (model at the full Q, state, ramped?)."""
    m = Model(prm, x)
    s, h = m.solve_state(s0=s0)
    if h["converged"]:
        return m, s, False
    s = s0
    for frac in Q_RAMP:
        mr = Model(replace(prm, Q=frac * prm.Q), x)
        s, h = mr.solve_state(s0=s)
    return mr, s, True


def optimize(prm, x0, iterations, g_star=0.05, move=0.2, every=100, continuation=CONTINUATION):
    """Runs the design loop from the raw design x0 (passive entries are kept).  Returns the
    final design, the last state and a history of (f, volume fraction, MMA multiplier,
    ramped) per iteration, with the designs after every update."""
    x = np.array(x0, dtype=float)
    s = None
    f0 = None
    opt = None
    hist = []
    for it in range(iterations):
        p = stage_params(prm, it, every, continuation)
        m, s, ramped = solve_with_ramp(p, x, s)
        D = m.design
        if opt is None:
            opt = MMA(int(D.sum()), move=move)
        f = m.objective(s)
        lam = m.solve_adjoint(s, m.dfds(s))
        _, dfdx = m.sensitivity(s, lam, explicit=True)
        frac, dg = m.volume()
        if f0 is None:
            f0 = f
        xd, mult = opt.update(x[D], dfdx[D] / f0, frac - g_star, dg[D])
        x = x.copy()
        x[D] = xd
        hist.append(dict(f=f, frac=frac, lam=mult, ramped=ramped, x=x.copy()))
    return x, s, hist
