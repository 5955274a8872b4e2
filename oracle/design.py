"""Oracle design loop of Sec. 5: the volume-constrained compliance minimisation of
eq. optprob by MMA, with the continuation of Sec. 5.3 and the solver practice of
Sec. 5.4.  Test infrastructure only (see oracle/__init__.py).

One design iteration: filter and passive regions (gamma), RAMP at the current continuation
stage, the state solve warm-started from the previous design's state (Sec. 5.4), with a
ramp of the heat source Q when that Newton solve fails (Sec. 5.4), the compliance and its
adjoint sensitivities, the volume constraint g = frac - g* and its gradient (eq. constr),
then one MMA update of the design elements (move limit of Sec. 6.1).  The objective is
passed to MMA as f / f0 (f0 the first iteration's compliance): the paper does not state a
scaling.  A continuation may name the flow model per stage (the hybrid strategy of Sec. 6.4).
"""

from dataclasses import replace

import numpy as np

from .fem import Model
from .mma import MMA
from .navier_stokes import NSModel

# eq. contsch1: (q_c, q_p, kappa_s) of the five stages, advanced every `every` iterations
CONTINUATION = ((0.881, 8.0, 1e-5), (8.81, 8.0, 1e-5), (88.1, 8.0, 1e-5), (88.1, 98.0, 1e-6), (881.0, 998.0, 1e-7))
# eq. contsch2, the hybrid strategy of Sec. 6.4 (NS-D of Table tab:hybridapproaches): two
# stages with the Navier-Stokes model (q_p and kappa_s interpolate the solid's
# impermeability there), then three with the Darcy model
HYBRID_NS_D = (("ns", 0.881, 8.0, 1e5), ("ns", 8.81, 8.0, 1e5), ("darcy", 88.1, 8.0, 1e-5),
               ("darcy", 88.1, 98.0, 1e-6), ("darcy", 881.0, 998.0, 1e-7))
Q_RAMP = (0.25, 0.5, 0.75, 1.0)
MODELS = {"darcy": Model, "ns": NSModel}


def stage(continuation, it, every):
    """(model kind, q_c, q_p, kappa_s) of iteration it; plain triples are Darcy stages."""
    st = continuation[min(it // every, len(continuation) - 1)]
    return st if len(st) == 4 else ("darcy",) + tuple(st)


def stage_params(prm, it, every, continuation=CONTINUATION):
    _, q_c, q_p, kappa_s = stage(continuation, it, every)
    return replace(prm, q_c=q_c, q_p=q_p, kappa_s=kappa_s)


def solve_with_ramp(prm, x, s0, kind="darcy"):
    """Newton from s0; if it fails, the heat source is ramped up through Q_RAMP, each stage
    warm-started from the last.  Returns (model at the full Q, state, ramped?)."""
    M = MODELS[kind]
    m = M(prm, x)
    s, h = m.solve_state(s0=s0)
    if h["converged"]:
        return m, s, False
    s = s0
    for frac in Q_RAMP:
        mr = M(replace(prm, Q=frac * prm.Q), x)
        s, h = mr.solve_state(s0=s)
    return mr, s, True


def optimize(prm, x0, iterations, g_star=0.05, move=0.2, every=100, continuation=CONTINUATION):
    """Runs the design loop from the raw design x0 (passive entries are kept).  Returns the
    final design, the last state and a history of (f, volume fraction, MMA multiplier,
    ramped, model) per iteration, with the designs after every update.  A change of flow
    model starts its first state solve from zero (the other model's state is no warm start
    for it); MMA carries on across the change."""
    x = np.array(x0, dtype=float)
    s = None
    f0 = None
    opt = None
    kind_prev = None
    hist = []
    for it in range(iterations):
        p = stage_params(prm, it, every, continuation)
        kind = stage(continuation, it, every)[0]
        if kind != kind_prev:
            s = None
            kind_prev = kind
        m, s, ramped = solve_with_ramp(p, x, s, kind)
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
        hist.append(dict(f=f, frac=frac, lam=mult, ramped=ramped, model=kind, x=x.copy()))
    return x, s, hist
