"""Operator of the projection step, M + A_D + A_C, evaluated the plain way
(test infrastructure only).

Sec. 3.2 (divergence and continuity penalty terms added to the projection
step) and Sec. 3.3 (the projection equation (M + A_D + A_C) u = rhs):
    (v, u)_K
  + (div v, tau_D div u)_K                                     divergence penalty
  + sum over the faces of K (v . n, {tau_C} [[u]] . n)          continuity penalty
with n the outward normal of the own element, [[u]] = u^- - u^+ and
{tau_C} the mean of the two elements' values.  tau_D and tau_C are given per
element (the paper forms them from the extrapolated velocity, the element
size and the time step; here they are inputs).  On a face normal to e_d,
(v . n)([[u]] . n) = v_d (u^-_d - u^+_d): only the normal component couples.
Every integral is an explicit Gauss sum (k+1 points per direction, exact)
against the dense 3D tables.
"""
import numpy as np

from .tables import tables


def projection_apply(u, k, mesh, tau_d, tau_c, elems=None):
    """y = (M + A_D + A_C) u; u: [3, N_el, (k+1)^3]; tau_d, tau_c: [N_el].
    With elems, only the rows of those elements: [3, len(elems), (k+1)^3]."""
    T = tables(k, k + 1)
    h = mesh.h
    vol = float(np.prod(h))
    u = np.asarray(u, dtype=np.float64)
    tau_d = np.asarray(tau_d, dtype=np.float64)
    tau_c = np.asarray(tau_c, dtype=np.float64)
    el = np.arange(mesh.N) if elems is None else np.asarray(elems)
    ue = u[:, el]
    # mass
    Mb = vol * (T.B.T * T.W) @ T.B
    y = ue @ Mb.T
    # divergence penalty: div u at the cell points, tested with div v
    div = sum((ue[j] @ T.G[j].T) / h[j] for j in range(3))         # [elements, points]
    dw = div * T.W[None, :] * (vol * tau_d[el])[:, None]
    for i in range(3):
        y[i] += (dw @ T.G[i]) / h[i]
    # continuity penalty on the normal component
    for d in range(3):
        area = vol / h[d]
        for s in range(2):
            nb = mesh.neighbor(d, s, el)
            own = ue[d] @ T.FV[d][s].T
            other = u[d][nb] @ T.FV[d][1 - s].T
            tau = 0.5 * (tau_c[el] + tau_c[nb])
            y[d] += area * ((tau[:, None] * T.WF[None, :] * (own - other)) @ T.FV[d][s])
    return y
