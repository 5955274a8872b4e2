"""Oracle problem data: parameters, the structured hexahedral grid, constraints and the
boundary heat-flux load.  Test infrastructure only (see oracle/__init__.py).

Numbering (shared convention of the whole project, restated here independently):
  node  n = i + (nx+1) * (j + (ny+1) * k),   0 <= i <= nx, ...
  elem  e = i + nx * (j + ny * k),           0 <= i < nx, ...
  local node a = ia + 2*ja + 4*ka of element (i,j,k) is node (i+ia, j+ja, k+ka)
  fields per node: 0,1,2 = velocity (u,v,w); 3 = modified pressure P; 4 = temperature T
The z axis is vertical; gravity is (0, 0, -g0) (Sec. 2.1: buoyancy points against g).
"""

from dataclasses import dataclass
import numpy as np

FIELD_U, FIELD_V, FIELD_W, FIELD_P, FIELD_T = 0, 1, 2, 3, 4
NFIELD = 5


@dataclass
class Params:
    """Physical and discretisation parameters.

    Defaults follow Sec. 6.1 (k_s = 100, k_f = 1, rho0 = mu = c_p = 1) and Sec. 3
    (all remaining constants one, alpha equal to the Grashof number).
    """
    nx: int
    ny: int
    nz: int
    h: float = 0.0              # element edge; 0 means 1/nx
    rho0: float = 1.0
    mu: float = 1.0
    cp: float = 1.0
    g0: float = 1.0
    alpha: float = 1.0e3        # thermal expansion coefficient (= Gr with unit constants)
    k_f: float = 1.0
    k_s: float = 100.0
    kappa_f: float = 0.00513    # Table tab:2 value for alpha = 1e3
    kappa_s: float = 1.0e-4
    q_c: float = 8.0
    q_p: float = 8.0
    q_h: float = 1.0            # heat flux into the bottom patch
    patch: tuple = (0.375, 0.625, 0.125, 0.375)   # x0, x1, y0, y1 of the bottom heated patch
    Q: float = 0.0              # volumetric heat source (on q_box, or everywhere if q_box is None)
    q_box: tuple = None         # (x0, x1, y0, y1, z0, z1): elements whose centre is inside carry Q
    solid_box: tuple = None     # passive solid: gamma = 1 on elements whose centre is inside
    design_box: tuple = None    # design domain; elements outside it (and outside solid_box) are
                                # passive fluid, gamma = 0.  None: every element is a design element
    sym_x: bool = False         # the wall x = Lx is a symmetry plane (insulated, u.n = 0), not T = 0
    sym_y: bool = False         # the wall y = Ly likewise
    filter_radius: float = 0.0  # density-filter radius in element lengths; 0 = identity
    filter_kind: str = "cone"   # "cone" (normalised hat weights) or "pde" (Helmholtz, Sec. 5.1)

    def __post_init__(self):
        if self.h <= 0.0:
            self.h = 1.0 / self.nx


class Mesh:
    """Index bookkeeping for the nx * ny * nz grid of cubes of edge h."""

    def __init__(self, p: Params):
        self.nx, self.ny, self.nz, self.h = p.nx, p.ny, p.nz, p.h
        self.NX, self.NY, self.NZ = p.nx + 1, p.ny + 1, p.nz + 1
        self.n_nodes = self.NX * self.NY * self.NZ
        self.n_elems = p.nx * p.ny * p.nz
        ii, jj, kk = np.meshgrid(np.arange(p.nx), np.arange(p.ny), np.arange(p.nz), indexing="ij")
        # element order e = i + nx*(j + ny*k): flatten with k slowest
        ie = ii.transpose(2, 1, 0).ravel()
        je = jj.transpose(2, 1, 0).ravel()
        ke = kk.transpose(2, 1, 0).ravel()
        self.elem_ijk = np.stack([ie, je, ke], axis=1)
        conn = np.empty((self.n_elems, 8), dtype=np.int64)
        for a in range(8):
            ia, ja, ka = a & 1, (a >> 1) & 1, (a >> 2) & 1
            conn[:, a] = self.node_id(ie + ia, je + ja, ke + ka)
        self.conn = conn
        n = np.arange(self.n_nodes)
        self.node_ijk = np.stack([n % self.NX, (n // self.NX) % self.NY, n // (self.NX * self.NY)], axis=1)
        self.node_xyz = self.node_ijk * self.h
        self.elem_centre = (self.elem_ijk + 0.5) * self.h

    def node_id(self, i, j, k):
        return i + self.NX * (j + self.NY * k)

    def elem_id(self, i, j, k):
        return i + self.nx * (j + self.ny * k)


def in_box(points, box):
    """Points (n, 3) inside the closed box (x0, x1, y0, y1, z0, z1)."""
    x0, x1, y0, y1, z0, z1 = box
    x, y, z = points[:, 0], points[:, 1], points[:, 2]
    return (x >= x0) & (x <= x1) & (y >= y0) & (y <= y1) & (z >= z0) & (z <= z1)


def element_regions(mesh: Mesh, p: Params):
    """Per element: volumetric source Q_e, passive-solid mask, passive-fluid mask (Sec. 6.1:
    the heat source block is solid and carries Q, the region outside the design domain is
    fluid; membership by element centre)."""
    c = mesh.elem_centre
    Qe = np.full(mesh.n_elems, p.Q) if p.q_box is None else np.where(in_box(c, p.q_box), p.Q, 0.0)
    solid = np.zeros(mesh.n_elems, dtype=bool) if p.solid_box is None else in_box(c, p.solid_box)
    fluid = np.zeros(mesh.n_elems, dtype=bool) if p.design_box is None else ~in_box(c, p.design_box) & ~solid
    return Qe, solid, fluid


def default_constraints(mesh: Mesh, p: Params = None):
    """Dirichlet mask [N, 5] and prescribed values for the cavity of Sec. 6.1.

    T = 0 on the vertical walls and the top (the bottom is insulated except for the
    heated patch); the pressure level is fixed by P = 0 at the single top corner node
    (0, 0, nz), where T is fixed as well.  With the quarter domain of Sec. 6.1 the walls
    x = Lx and y = Ly can be symmetry planes instead (p.sym_x, p.sym_y): insulated, u.n = 0.  Velocity is never constrained: it is the
    lumped projection of the Darcy velocity and the walls carry u.n = 0 naturally.
    """
    i, j, k = mesh.node_ijk[:, 0], mesh.node_ijk[:, 1], mesh.node_ijk[:, 2]
    sx = p is not None and p.sym_x
    sy = p is not None and p.sym_y
    mask = np.zeros((mesh.n_nodes, NFIELD), dtype=bool)
    # a symmetry plane is insulated (natural condition), so T stays free there
    mask[:, FIELD_T] = (i == 0) | ((i == mesh.nx) & (not sx)) | (j == 0) | ((j == mesh.ny) & (not sy)) | (k == mesh.nz)
    # u.n = 0 on a symmetry plane: the normal velocity is odd across it, so its nodal
    # projection there (the mean over both sides) is zero; the tangential components are
    # even, so the one-sided projection is already the mean over both sides
    if sx:
        mask[:, 0] = i == mesh.nx
    if sy:
        mask[:, 1] = j == mesh.ny
    mask[mesh.node_id(0, 0, mesh.nz), FIELD_P] = True
    values = np.zeros((mesh.n_nodes, NFIELD))
    return mask, values


def patch_flux(mesh: Mesh, p: Params):
    """Consistent nodal load of a uniform flux q_h on the bottom patch (boundary term of
    eq. weakstable, f_{t q_h} of App. A).

    A bottom element face belongs to the patch when its centre lies inside
    [x0, x1] x [y0, y1].  The integral of a bilinear face shape function over a square
    face of edge h is h^2 / 4, so each patch face adds q_h h^2 / 4 to its four nodes.
    """
    x0, x1, y0, y1 = p.patch
    f = np.zeros(mesh.n_nodes)
    h = mesh.h
    for i in range(mesh.nx):
        xc = (i + 0.5) * h
        if not (x0 <= xc <= x1):
            continue
        for j in range(mesh.ny):
            yc = (j + 0.5) * h
            if not (y0 <= yc <= y1):
                continue
            for di in (0, 1):
                for dj in (0, 1):
                    f[mesh.node_id(i + di, j + dj, 0)] += p.q_h * h * h / 4.0
    return f
