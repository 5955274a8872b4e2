"""Oracle PDE (Helmholtz) density filter of Sec. 5.1.  Test infrastructure only (see
oracle/__init__.py).

The paper regularises the design with a PDE-based filter (Sec. 5.1; the filter of
Lazarov and Sigmund), with radius 2.5 element lengths (Sec. 6.3, Sec. 7.1).  Written out:

    -r^2 lap(y) + y = x  in the domain,   grad(y) . n = 0 on its boundary,

with r = R / (2 sqrt 3) for a filter radius R (the length scale that matches a cone
filter of radius R).  Discretisation: trilinear (Q1) nodal y on the element grid,
Galerkin with the consistent mass matrix,

    K_F y = B x,   K_F = int (r^2 grad N_a . grad N_b + N_a N_b),   B_ae = int_e N_a = h^3 / 8,

and the filtered density of an element is the mean of y over the element, which for a
trilinear y is the average of its eight nodal values: gamma = (1/h^3) B^T y.  The filter
F = (1/h^3) B^T K_F^-1 B is symmetric (K_F is), so the sensitivity map F^T is F itself.
Element matrices come from 2x2x2 Gauss quadrature (exact for these polynomial
integrands); K_F is factorised once by SuperLU.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .element import reference_element


def pde_length_scale(radius, h):
    """r = R h / (2 sqrt 3) for a radius of R element lengths."""
    return radius * h / (2.0 * np.sqrt(3.0))


class PDEFilter:
    """y = F x and F^T x (F = F^T) by a direct solve with the assembled K_F."""

    def __init__(self, mesh, radius):
        h = mesh.h
        r = pde_length_scale(radius, h)
        N, G, _, _, detJ, _ = reference_element(h)
        Ke = detJ * (r * r * np.einsum("qad,qbd->ab", G, G) + np.einsum("qa,qb->ab", N, N))
        E, Nn = mesh.n_elems, mesh.n_nodes
        rows = np.repeat(mesh.conn, 8, axis=1).ravel()
        cols = np.tile(mesh.conn, (1, 8)).ravel()
        vals = np.tile(Ke.ravel(), E)
        self.K = sp.csr_matrix((vals, (rows, cols)), shape=(Nn, Nn))
        be = detJ * N.sum(axis=0)                                  # int_e N_a = h^3 / 8
        self.B = sp.csr_matrix((np.tile(be, E), (mesh.conn.ravel(), np.repeat(np.arange(E), 8))), shape=(Nn, E))
        self.vol = h ** 3
        self.lu = spla.splu(self.K.tocsc())
        self.shape = (E, E)

    def __matmul__(self, x):
        y = self.lu.solve(self.B @ np.asarray(x, dtype=float))
        return (self.B.T @ y) / self.vol

    @property
    def T(self):
        return self                                                # F is symmetric
