"""Pressure gradient g_h with central flux (test infrastructure only).

Sec. 3.2, weak form of g_h, tested with a vector function v:

    g_h(v, p) = -(div v, p)_K + (v . n, {{p}})_dK

Row i of component j is g_h(phi_i e_j, p): the volume term -(d_j phi_i, p)_K
and, on the two faces normal to e_j, n_j (phi_i, 1/2 (p^- + p^+)).  It enters
the projection step's right-hand side (Sec. 3.1) and the paper leaves it in the
same space as the velocity.  Gauss rule with k+1 points per direction (exact on
affine cells) unless n_q says otherwise.
"""
import numpy as np

from .basis import default_laplace_nq
from .tables import tables


def gradient_apply(p, k, mesh, n_q=0, elems=None):
    """y[j]_i = g_h(phi_i e_j, p); p: [N_el, (k+1)^3] -> y: [3, N_el, (k+1)^3]
    (or the rows of the elements in elems)."""
    m = n_q or default_laplace_nq(k)
    T = tables(k, m)
    h = mesh.h
    vol = float(np.prod(h))
    E = np.arange(mesh.N) if elems is None else np.asarray(elems)
    p = np.asarray(p, dtype=np.float64)
    pe = p[E]
    pq = pe @ T.B.T                                   # p at the cell points
    y = np.zeros((3,) + pe.shape)
    for j in range(3):
        # -(d_j phi_i, p)_K: reference derivative over h_j, cell volume
        y[j] -= (vol / h[j]) * ((T.W * pq) @ T.G[j])
        area = vol / h[j]
        for s in range(2):
            nj = 1.0 if s == 1 else -1.0               # outward normal component
            nb = mesh.neighbor(j, s, E)
            pm = pe @ T.FV[j][s].T
            pp = p[nb] @ T.FV[j][1 - s].T
            y[j] += area * ((T.WF * (nj * 0.5 * (pm + pp))) @ T.FV[j][s])
    return y
