"""Velocity-pressure coupling terms between the mixed-order spaces (test
infrastructure only).

Sec. 3.2: the velocity has tensor degree k and the pressure degree k - 1
(inf-sup stable pair).  With central fluxes on a periodic mesh:

    d_h(q, u) = -(grad q, u)_K + (q, {{u}} . n)_dK        q of degree k - 1,
    g_h(v, p) = -(div v, p)_K + (v . n, {{p}})_dK         v of degree k.

d_h maps the velocity (k) into the pressure test space (k - 1): it is the
right-hand side of the pressure Poisson step; g_h maps the pressure (k - 1)
into the velocity test space (k): it enters the projection step (Sec. 3.1).
Both are explicit Gauss sums with k + 1 points per direction (the integrands
have degree at most 2k - 1 per direction: exact) against the dense 3D tables
of the two bases, no sum factorisation.
"""
import numpy as np

from .tables import tables


def _tabs(k):
    m = k + 1
    return tables(k, m), tables(k - 1, m)


def mixed_divergence_apply(u, k, mesh, elems=None):
    """b_i = d_h(q_i, u) for the degree-(k-1) pressure basis q_i;
    u: [3, N_el, (k+1)^3] -> b: [N_el, k^3] (or the rows of elems)."""
    Tu, Tp = _tabs(k)
    h = mesh.h
    vol = float(np.prod(h))
    E = np.arange(mesh.N) if elems is None else np.asarray(elems)
    u = np.asarray(u, dtype=np.float64)
    ue = u[:, E, :]
    b = np.zeros((len(E), k ** 3))
    for j in range(3):
        uq = ue[j] @ Tu.B.T                                  # u_j at the cell points
        b -= (vol / h[j]) * ((Tp.W * uq) @ Tp.G[j])          # -(d_j q_i, u_j)
    for d in range(3):
        area = vol / h[d]
        for s in range(2):
            sgn = 1.0 if s == 1 else -1.0                      # outward normal component
            nb = mesh.neighbor(d, s, E)
            um = ue[d] @ Tu.FV[d][s].T
            up = u[d][nb] @ Tu.FV[d][1 - s].T
            b += area * ((Tp.WF * (sgn * 0.5 * (um + up))) @ Tp.FV[d][s])
    return b


def mixed_gradient_apply(p, k, mesh, elems=None):
    """y[j]_i = g_h(phi_i e_j, p) for the degree-k velocity basis phi_i;
    p: [N_el, k^3] -> y: [3, N_el, (k+1)^3] (or the rows of elems)."""
    Tu, Tp = _tabs(k)
    h = mesh.h
    vol = float(np.prod(h))
    E = np.arange(mesh.N) if elems is None else np.asarray(elems)
    p = np.asarray(p, dtype=np.float64)
    pe = p[E]
    pq = pe @ Tp.B.T                                           # p at the cell points
    y = np.zeros((3, len(E), (k + 1) ** 3))
    for j in range(3):
        y[j] -= (vol / h[j]) * ((Tu.W * pq) @ Tu.G[j])       # -(d_j phi_i, p)
        area = vol / h[j]
        for s in range(2):
            nj = 1.0 if s == 1 else -1.0
            nb = mesh.neighbor(j, s, E)
            pm = pe @ Tp.FV[j][s].T
            pp = p[nb] @ Tp.FV[j][1 - s].T
            y[j] += area * ((Tu.WF * (nj * 0.5 * (pm + pp))) @ Tu.FV[j][s])
    return y
