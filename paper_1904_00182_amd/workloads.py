"""Workload definitions: the unit-constant cavity (Sec. 3, Sec. 6.1) at the grid sizes,
Grashof numbers and design recipes of the benchmark configurations, on the GPU path.

Designs are built from the seeded noise of `inputs` with the library's own cone
filter (nc_cone_filter) and, where a 0/1 design is wanted, a threshold at 0.5 taken
in float64 (ties go to solid).
"""

import torch

from . import inputs
from . import nc

# permeability from Table tab:2 per Grashof number (alpha with unit constants)
KAPPA_F = {1e3: 0.00513, 1e4: 0.00206, 1e5: 0.00085, 1e6: 0.00036}

CONFIGS = {
    # name: grid, Gr, precision, design recipe, in-chain filter radius, seed
    "cavity16": dict(grid=(16, 8, 16), gr=1e3, precision=nc.NC_FP64, design="noise", radius=0.0, seed=0),
    "cavity64": dict(grid=(64, 32, 64), gr=1e3, precision=nc.NC_FP64, design="blobs", radius=0.0, seed=1),
    "cavity32": dict(grid=(32, 16, 32), gr=1e3, precision=nc.NC_FP64, design="blobs", radius=0.0, seed=1),
    "cavity128mixed": dict(grid=(128, 64, 128), gr=1e4, precision=nc.NC_MIXED, design="blobs", radius=0.0, seed=2),
    "cavity128": dict(grid=(128, 64, 128), gr=1e4, precision=nc.NC_FP64, design="blobs", radius=0.0, seed=2),
    "cavity96filtered": dict(grid=(96, 48, 96), gr=1e3, precision=nc.NC_FP64, design="noise", radius=1.5, seed=3),
    "cavity24filtered": dict(grid=(24, 12, 24), gr=1e3, precision=nc.NC_FP64, design="noise", radius=1.5, seed=3),
    # the paper's PDE filter with radius 2.5 element lengths (Sec. 6.3, Sec. 7.1)
    "cavity24pde": dict(grid=(24, 12, 24), gr=1e3, precision=nc.NC_FP64, design="noise", radius=2.5, seed=3,
                        filter="pde"),
    "cavity96pde": dict(grid=(96, 48, 96), gr=1e3, precision=nc.NC_FP64, design="noise", radius=2.5, seed=3,
                        filter="pde"),
    "cavity128pde": dict(grid=(128, 64, 128), gr=1e4, precision=nc.NC_MIXED, design="noise", radius=2.5, seed=2,
                         filter="pde"),
}


def problem(grid, gr=1e3, precision=nc.NC_FP64, radius=0.0, q_h=1.0, **over):
    """Cavity problem at Grashof number gr (alpha = gr, kappa_f from Table tab:2); keyword
    overrides replace any field (e.g. alpha=0 for pure conduction)."""
    nx, ny, nz = grid
    fields = dict(alpha=float(gr), kappa_f=KAPPA_F[float(gr)], precision=precision, filter_radius=float(radius),
                  q_h=float(q_h))
    fields.update(over)
    return nc.default_problem(nx, ny, nz, **fields)


def design(grid, recipe, seed, device="cuda:0"):
    """Raw design x for the solver: 'noise' = 0.5 + 0.1 U(-1,1); 'blobs' = U(0,1) smoothed
    by a radius-2 cone filter and thresholded at 0.5 (1 = solid)."""
    nx, ny, nz = grid
    E = nx * ny * nz
    if recipe == "noise":
        return torch.as_tensor(inputs.noise_design(E, seed), device=device)
    if recipe == "blobs":
        x0 = torch.as_tensor(inputs.uniform_design(E, seed), device=device)
        y = nc.cone_filter(x0, nx, ny, nz, 2.0)
        return (y >= 0.5).to(torch.float64)
    raise ValueError(recipe)


def config(name, device="cuda:0", **over):
    c = dict(CONFIGS[name])
    c.update(over)
    fk = nc.NC_FILTER_PDE if c.get("filter") == "pde" else nc.NC_FILTER_CONE
    p = problem(c["grid"], c["gr"], c["precision"], c["radius"], filter_kind=fk)
    x = design(c["grid"], c["design"], c["seed"], device)
    return p, x, c


# The benchmark of Sec. 6.1 on a quarter of the 1 m cavity with symmetry planes at x = y =
# 0.5: heat-source block 0.1 x 0.1 x 0.05 m (Q = 1e4, passive solid) on the floor at the
# centre, design domain 0.75 x 0.75 x 0.75 m on top of it, fluid elsewhere.
BENCH_Q = 1e4
BENCH_SOURCE = (0.45, 0.5, 0.45, 0.5, 0.0, 0.05)
BENCH_DESIGN = (0.125, 0.5, 0.125, 0.5, 0.05, 0.8)


# multigrid smoothing of the strongly convective regime (alpha >= 1e5 on the benchmark)
CONVECTIVE_SMOOTHING = dict(smooth_omega=0.5, smooth_pre=4, smooth_post=4, smooth_pre_coarse=2, smooth_post_coarse=2)


def benchmark_problem(n, alpha=1e3, precision=nc.NC_FP64, kappa_s=1e-5, q_c=8.81, q_p=8.0, filter_radius=2.5,
                      **over):
    """Quarter cavity of Sec. 6.1 with n x n x 2n elements (h = 0.5 / n), the Table tab:2
    permeability for alpha, the PDE filter of radius 2.5 elements and the penalties of the
    performance study (q_c = 8.81, q_p = 8).  From alpha = 1e5 on the multigrid smooths
    harder (damping 0.5, four sweeps before and after the coarse correction on the finest
    level, two on the others): with the default two undamped sweeps the Krylov solves of
    this strongly convective regime stagnate.  There, too, a mixed-precision context
    reserves a float64 Krylov basis: on grids where the source block is one or two
    elements wide the V-cycle amplifies the pressure inside it by orders of magnitude, and
    float32 Krylov solves stagnate; the context then goes on in float64 Krylov with the
    float32 V-cycle."""
    fields = dict(h=0.5 / n, alpha=float(alpha), kappa_f=KAPPA_F[float(alpha)], kappa_s=kappa_s, q_c=q_c, q_p=q_p,
                  q_h=0.0, Q=BENCH_Q, precision=precision, filter_radius=float(filter_radius),
                  filter_kind=nc.NC_FILTER_PDE, sym_x=1, sym_y=1, q_box=BENCH_SOURCE, solid_box=BENCH_SOURCE,
                  design_box=BENCH_DESIGN)
    if alpha >= 1e5:
        fields.update(CONVECTIVE_SMOOTHING)
        fields["f64_krylov_fallback"] = 1
    fields.update(over)
    return nc.default_problem(n, n, 2 * n, **fields)


def benchmark_start_design(p, device="cuda:0"):
    """The paper's initial design for the benchmark (Sec. 6.1): 0.05 on the design elements,
    1 on the passive solid block, 0 on the passive fluid (membership by element centre)."""
    import numpy as np
    nx, ny, nz, h = p.nx, p.ny, p.nz, p.h
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = np.stack([(i.ravel() + 0.5) * h, (j.ravel() + 0.5) * h, (k.ravel() + 0.5) * h], axis=1)

    def inside(box):
        b = [float(v) for v in box]
        return ((c[:, 0] >= b[0]) & (c[:, 0] <= b[1]) & (c[:, 1] >= b[2]) & (c[:, 1] <= b[3])
                & (c[:, 2] >= b[4]) & (c[:, 2] <= b[5]))

    solid = inside(p.solid_box)
    des = inside(p.design_box) & ~solid
    x = np.where(solid, 1.0, np.where(des, 0.05, 0.0))
    return torch.as_tensor(x, device=device)
