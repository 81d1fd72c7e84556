"""SIPG negative Laplacian l_h, evaluated the plain way (test infrastructure only).

Sec. 3.2, weak form of l_h (symmetric interior penalty):

    l_h(q, p) = (grad q, grad p)_K - (grad q, 1/2 [[p]])_dK
                - (q, {{grad p}} . n)_dK + (q, tau [[p]] . n)_dK

with [[p]] = p^- n^- + p^+ n^+ (Sec. 3.2), so on a face with outward normal n
of the own element: (grad q, 1/2 [[p]]) = 1/2 (grad q . n)(p^- - p^+) and
tau [[p]] . n = tau (p^- - p^+).  The paper leaves tau unspecified; this
oracle uses tau = penalty_factor * (k+1)^2 / h_d on faces normal to
direction d.  The viscous term v_h of the same section is nu times this form
applied to each velocity component; ``scale`` carries nu and leading array
dimensions carry components.

Every integral is an explicit Gauss sum over the (k+1)^3 cell points and the
(k+1)^2 points of each face, against dense 3D basis tables.
"""
import numpy as np

from .basis import default_laplace_nq
from .tables import tables


def laplace_apply(u, k, mesh, n_q=0, penalty_factor=1.0, scale=1.0, elems=None):
    """y = A u for the SIPG form above.

    u has shape [..., N_el, (k+1)^3]; leading dimensions (components, batches)
    are independent.  ``elems`` restricts the output to a subset of elements
    (the input must still cover the whole mesh).
    """
    m = n_q or default_laplace_nq(k)
    T = tables(k, m)
    h = mesh.h
    vol = float(np.prod(h))
    E = np.arange(mesh.N) if elems is None else np.asarray(elems)
    u = np.asarray(u, dtype=np.float64)
    ue = u[..., E, :]
    y = np.zeros(ue.shape)
    # cell term: sum_d (1/h_d^2) * vol * sum_q W_q d_d(phi_i) d_d(u)
    for d in range(3):
        gd = ue @ T.G[d].T
        y += (vol / h[d] ** 2) * ((gd * T.W) @ T.G[d])
    # face terms, element by element over its six faces
    for d in range(3):
        area = vol / h[d]
        tau = penalty_factor * (k + 1) ** 2 / h[d]
        for s in range(2):
            sgn = 1.0 if s == 1 else -1.0          # outward normal n = sgn * e_d
            nb = mesh.neighbor(d, s, E)
            un = u[..., nb, :]
            u_m = ue @ T.FV[d][s].T                 # own trace u^-
            u_p = un @ T.FV[d][1 - s].T             # neighbour trace u^+
            dn_m = (sgn / h[d]) * (ue @ T.FG[d][s][d].T)       # grad u^- . n
            dn_p = (sgn / h[d]) * (un @ T.FG[d][1 - s][d].T)   # grad u^+ . n
            jump = u_m - u_p
            coef_val = tau * jump - 0.5 * (dn_m + dn_p)   # multiplies q
            coef_grad = -0.5 * jump                       # multiplies grad q . n
            y += area * ((T.WF * coef_val) @ T.FV[d][s]
                         + (T.WF * coef_grad) @ ((sgn / h[d]) * T.FG[d][s][d]))
    return scale * y


def laplace_matrix(k, mesh, n_q=0, penalty_factor=1.0, scale=1.0):
    """Dense matrix of the form on a small mesh, column by column."""
    n3 = (k + 1) ** 3
    ndof = mesh.N * n3
    I = np.eye(ndof).reshape(ndof, mesh.N, n3)
    cols = laplace_apply(I, k, mesh, n_q, penalty_factor, scale)
    return cols.reshape(ndof, ndof).T


def laplace_diagonal(k, mesh, n_q=0, penalty_factor=1.0, scale=1.0, elem=0):
    """diag(A) on one element (the same on every element of a uniform mesh)."""
    n3 = (k + 1) ** 3
    d = np.zeros(n3)
    for i in range(n3):
        u = np.zeros((mesh.N, n3))
        u[elem, i] = 1.0
        d[i] = laplace_apply(u, k, mesh, n_q, penalty_factor, scale, elems=[elem])[0, i]
    return d


def mass_apply(u, k, mesh, n_q=0, elems=None):
    """y = M u, the DG mass matrix m_h(v, u) = (v, u) (Sec. 3.2)."""
    m = n_q or default_laplace_nq(k)
    T = tables(k, m)
    vol = float(np.prod(mesh.h))
    E = np.arange(mesh.N) if elems is None else np.asarray(elems)
    ue = np.asarray(u, dtype=np.float64)[..., E, :]
    return vol * ((ue @ T.B.T) * T.W) @ T.B
