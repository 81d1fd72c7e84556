"""Level transfers of the h-multigrid hierarchy (test infrastructure only).

Sec. 3.3: the pressure Poisson preconditioner is a geometric multigrid
V-cycle with matrix-free level transfers.  Between a periodic mesh and the
mesh with every element split in two per direction (same degree k), the
prolongation is the embedding of the coarse DG space in the fine one: the
fine nodal values are the coarse element's polynomial evaluated at the fine
nodes.  The restriction is its transpose.  Each fine element's values are a
dense matrix (rows: fine nodes, columns: coarse basis functions, every entry
a product of three Lagrange evaluations) times its parent's values.
"""
from functools import lru_cache

import numpy as np

from . import basis
from .mesh import Mesh


def fine_mesh(coarse):
    return Mesh(tuple(2 * n for n in coarse.n_el), coarse.length)


@lru_cache(maxsize=64)
def child_matrix(k, child):
    """Phi[i, a] = l_a(x_i) over the 3D nodes: fine node i of the child
    (cx, cy, cz) mapped into the parent's reference cube, coarse basis a; the
    tensor product of the three 1D evaluation matrices (rows i + n(j + n l),
    columns a + n(b + n c))."""
    xi = basis.lgl_nodes(k)
    n = k + 1
    L = [basis.lagrange_values(xi, (xi + c) / 2.0) for c in child]   # per direction: [fine node, coarse basis]
    # Phi[(l, j, i), (c, b, a)] = Lz[l, c] Ly[j, b] Lx[i, a]
    return np.einsum("lc,jb,ia->ljicba", L[2], L[1], L[0]).reshape(n ** 3, n ** 3)


def _children(coarse):
    """For every fine element: its parent and child index."""
    fine = fine_mesh(coarse)
    c = fine.coords()
    parent = coarse.index(c // 2)
    child = c % 2
    return fine, parent, child


def prolongate(u, k, coarse):
    """u: [..., N_el coarse, n^3] -> [..., N_el fine, n^3]."""
    u = np.asarray(u, dtype=np.float64)
    fine, parent, child = _children(coarse)
    out = np.zeros(u.shape[:-2] + (fine.N, u.shape[-1]))
    for cx in range(2):
        for cy in range(2):
            for cz in range(2):
                sel = np.nonzero((child[:, 0] == cx) & (child[:, 1] == cy) & (child[:, 2] == cz))[0]
                PhiT = np.ascontiguousarray(child_matrix(k, (cx, cy, cz)).T)
                out[..., sel, :] = u[..., parent[sel], :] @ PhiT
    return out


def restrict(r, k, coarse):
    """Transpose of prolongate: r: [..., N_el fine, n^3] -> [..., N_el coarse, n^3]."""
    r = np.asarray(r, dtype=np.float64)
    fine, parent, child = _children(coarse)
    out = np.zeros(r.shape[:-2] + (coarse.N, r.shape[-1]))
    for cx in range(2):
        for cy in range(2):
            for cz in range(2):
                sel = np.nonzero((child[:, 0] == cx) & (child[:, 1] == cy) & (child[:, 2] == cz))[0]
                Phi = child_matrix(k, (cx, cy, cz))
                # each coarse element has exactly one child of each index
                out[..., parent[sel], :] += r[..., sel, :] @ Phi
    return out
