"""Convective term c_h with local Lax-Friedrichs flux (test infrastructure only).

Sec. 3.2, weak form of c_h with F_c(u) = u (x) u (Sec. 3):

    c_h(v, u) = -(grad v, u (x) u)_K
                + (v, ({{u (x) u}} + max(|u^- . n|, |u^+ . n|) [[u]]) . n)_dK

With [[u]] = u^- (x) n^- + u^+ (x) n^+ and n = n^- the own outward normal,
[[u]] . n = u^- - u^+, so the numerical flux at a face point is

    F*_c = 1/2 (u^-_c (u^- . n) + u^+_c (u^+ . n)) + lf * L (u^-_c - u^+_c),
    L    = max(|u^- . n|, |u^+ . n|)   (pointwise at the quadrature point).

The paper writes no factor 1/2 in front of the dissipative term; ``lf``
(default 1) is that coefficient.  Quadrature: floor(3k/2)+1 Gauss points per
direction (the 3/2 rule, Sec. 3.2) unless ``n_q`` says otherwise.

The Jacobian is assembled explicitly as a sparse matrix from the
linearisation of every Gauss sum; its transpose product is the reference for
the vector-Jacobian product.  At the kinks of L the derivative takes 1/2 of
each side on exact ties |u^-.n| = |u^+.n| and sign(0) = 0.
"""
import numpy as np
import scipy.sparse as sp

from .basis import default_convective_nq
from .tables import tables


def _setup(k, mesh, n_q, elems):
    m = n_q or default_convective_nq(k)
    T = tables(k, m)
    h = mesh.h
    vol = float(np.prod(h))
    E = np.arange(mesh.N) if elems is None else np.asarray(elems)
    return T, h, vol, E


def convective_apply(u, k, mesh, n_q=0, lf_factor=1.0, elems=None):
    """R_c = c_h(phi_i e_c, u) for every basis function; u, R: [3, N_el, (k+1)^3]."""
    T, h, vol, E = _setup(k, mesh, n_q, elems)
    u = np.asarray(u, dtype=np.float64)
    ue = u[:, E, :]
    U = ue @ T.B.T                      # values at the cell points
    R = np.zeros(ue.shape)
    for c in range(3):
        for j in range(3):
            R[c] -= (vol / h[j]) * ((T.W * U[c] * U[j]) @ T.G[j])
    for d in range(3):
        area = vol / h[d]
        for s in range(2):
            sgn = 1.0 if s == 1 else -1.0
            nb = mesh.neighbor(d, s, E)
            um = ue @ T.FV[d][s].T
            up = u[:, nb, :] @ T.FV[d][1 - s].T
            unm, unp = sgn * um[d], sgn * up[d]
            lam = np.maximum(np.abs(unm), np.abs(unp))
            for c in range(3):
                F = 0.5 * (um[c] * unm + up[c] * unp) + lf_factor * lam * (um[c] - up[c])
                R[c] += area * ((T.WF * F) @ T.FV[d][s])
    return R


def _flux_derivs(um, up, d, sgn, lf):
    """dF*_c/du^-_j and dF*_c/du^+_j at face points: arrays [3(c), 3(j), ..., m^2]."""
    unm, unp = sgn * um[d], sgn * up[d]
    a_m, a_p = np.abs(unm), np.abs(unp)
    lam = np.maximum(a_m, a_p)
    s_m = np.where(a_m > a_p, 1.0, np.where(a_m == a_p, 0.5, 0.0))
    s_p = 1.0 - s_m
    dm = np.zeros((3, 3) + um.shape[1:])
    dp = np.zeros((3, 3) + um.shape[1:])
    for c in range(3):
        jmp = um[c] - up[c]
        for j in range(3):
            if c == j:
                dm[c, j] += 0.5 * unm + lf * lam
                dp[c, j] += 0.5 * unp - lf * lam
            if j == d:
                dm[c, j] += 0.5 * um[c] * sgn + lf * jmp * s_m * np.sign(unm) * sgn
                dp[c, j] += 0.5 * up[c] * sgn + lf * jmp * s_p * np.sign(unp) * sgn
    return dm, dp


def convective_jvp(u, v, k, mesh, n_q=0, lf_factor=1.0, elems=None):
    """J(u) v computed point by point from the linearised integrands (no matrix)."""
    T, h, vol, E = _setup(k, mesh, n_q, elems)
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    U = u[:, E, :] @ T.B.T
    V = v[:, E, :] @ T.B.T
    out = np.zeros((3, len(E), u.shape[2]))
    for c in range(3):
        for j in range(3):
            out[c] -= (vol / h[j]) * ((T.W * (V[c] * U[j] + U[c] * V[j])) @ T.G[j])
    for d in range(3):
        area = vol / h[d]
        for s in range(2):
            sgn = 1.0 if s == 1 else -1.0
            nb = mesh.neighbor(d, s, E)
            um = u[:, E, :] @ T.FV[d][s].T
            up = u[:, nb, :] @ T.FV[d][1 - s].T
            vm = v[:, E, :] @ T.FV[d][s].T
            vp = v[:, nb, :] @ T.FV[d][1 - s].T
            dm, dp = _flux_derivs(um, up, d, sgn, lf_factor)
            for c in range(3):
                dF = sum(dm[c, j] * vm[j] + dp[c, j] * vp[j] for j in range(3))
                out[c] += area * ((T.WF * dF) @ T.FV[d][s])
    return out


def convective_jacobian(u, k, mesh, n_q=0, lf_factor=1.0):
    """Sparse Jacobian dR/du; row/column index (c * N_el + e) * (k+1)^3 + i."""
    T, h, vol, E = _setup(k, mesh, n_q, None)
    n = k + 1
    n3 = n ** 3
    N = mesh.N
    u = np.asarray(u, dtype=np.float64)
    U = u @ T.B.T                                  # 3 x N x m3
    rows, cols, vals = [], [], []
    loc = np.arange(n3)

    def add_blocks(c, cp, e_row, e_col, li, lj, blocks):
        # blocks: [N, len(li), len(lj)]
        r = ((c * N + e_row)[:, None, None] * n3 + li[None, :, None])
        q = ((cp * N + e_col)[:, None, None] * n3 + lj[None, None, :])
        r, q = np.broadcast_arrays(r, q)
        rows.append(r.ravel())
        cols.append(q.ravel())
        vals.append(blocks.ravel())

    # cell blocks: d/du_{c'} of -sum_j s_j G_j^T W U_c U_j
    for c in range(3):
        for cp in range(3):
            blk = np.zeros((N, n3, n3))
            for j in range(3):
                s_j = vol / h[j]
                w = np.zeros((N, T.B.shape[0]))
                if c == cp:
                    w += U[j]
                if j == cp:
                    w += U[c]
                if np.any(w):
                    blk -= s_j * ((T.G[j].T[None, :, :] * (T.W * w)[:, None, :]) @ T.B)
            add_blocks(c, cp, E, E, loc, loc, blk)

    # face blocks: only face-layer basis functions are non-zero on a face
    idx = np.arange(n3).reshape(n, n, n)           # [c, b, a]
    for d in range(3):
        area = vol / h[d]
        for s in range(2):
            sgn = 1.0 if s == 1 else -1.0
            nb = mesh.neighbor(d, s)
            layer = [np.take(idx, 0, axis=2 - d).ravel(), np.take(idx, n - 1, axis=2 - d).ravel()]
            own_nodes, nb_nodes = layer[s], layer[1 - s]
            Fo = T.FV[d][s][:, own_nodes]           # m2 x n2
            Fn = T.FV[d][1 - s][:, nb_nodes]
            um = u @ T.FV[d][s].T
            up = u[:, nb, :] @ T.FV[d][1 - s].T
            dm, dp = _flux_derivs(um, up, d, sgn, lf_factor)
            for c in range(3):
                for j in range(3):
                    bo = area * ((Fo.T[None] * (T.WF * dm[c, j])[:, None, :]) @ Fo)
                    bn = area * ((Fo.T[None] * (T.WF * dp[c, j])[:, None, :]) @ Fn)
                    add_blocks(c, j, E, E, own_nodes, own_nodes, bo)
                    add_blocks(c, j, E, nb, own_nodes, nb_nodes, bn)
    ndof = 3 * N * n3
    J = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(ndof, ndof))
    return J.tocsr()


def convective_vjp(u, w, k, mesh, n_q=0, lf_factor=1.0):
    """J(u)^T w through the explicitly assembled Jacobian."""
    J = convective_jacobian(u, k, mesh, n_q, lf_factor)
    return (J.T @ np.asarray(w, dtype=np.float64).ravel()).reshape(np.shape(u))
