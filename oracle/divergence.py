"""Velocity divergence d_h with central flux (test infrastructure only).

Sec. 3.2, weak form of d_h:

    d_h(q, u) = -(grad q, u)_K + (q, {{u}} . n)_dK

It forms the right-hand side of the pressure Poisson step (Sec. 3.1/3.3,
L P = -gamma_0/dt D U).  The oracle evaluates it in the same degree-k space as
the operator it feeds and leaves out the factor -gamma_0/dt.  Gauss rule with
k+1 points per direction (exact on affine cells).
"""
import numpy as np

from .basis import default_laplace_nq
from .tables import tables


def divergence_apply(u, k, mesh, n_q=0, elems=None):
    """b_i = d_h(phi_i, u); u: [3, N_el, (k+1)^3] -> b: [N_el, (k+1)^3]."""
    m = n_q or default_laplace_nq(k)
    T = tables(k, m)
    h = mesh.h
    vol = float(np.prod(h))
    E = np.arange(mesh.N) if elems is None else np.asarray(elems)
    u = np.asarray(u, dtype=np.float64)
    ue = u[:, E, :]
    b = np.zeros(ue.shape[1:])
    for j in range(3):
        b -= (vol / h[j]) * ((T.W * (ue[j] @ T.B.T)) @ T.G[j])
    for d in range(3):
        area = vol / h[d]
        for s in range(2):
            sgn = 1.0 if s == 1 else -1.0
            nb = mesh.neighbor(d, s, E)
            um = ue[d] @ T.FV[d][s].T
            up = u[d][nb] @ T.FV[d][1 - s].T
            b += area * ((T.WF * (sgn * 0.5 * (um + up))) @ T.FV[d][s])
    return b


def poisson_rhs(u, k, mesh, n_q=0):
    """d_h(phi_i, u) with its Euclidean coefficient mean removed (periodic solvability)."""
    b = divergence_apply(u, k, mesh, n_q)
    return b - b.mean()
