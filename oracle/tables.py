"""Explicit 3D basis tables on the reference hexahedron (test infrastructure only).

The oracle never factorises: each table is a dense matrix whose row is a
quadrature point of the cell (or of one face) and whose column is one of the
(k+1)^3 tensor-product basis functions (Sec. 3.2).  Entry [q, i] with
i = a + n*(b + n*c) is l_a(x_q) * l_b(y_q) * l_c(z_q) (or one factor replaced by
its derivative).  ``np.kron`` only fills these dense tables; applying them is
a plain matrix product per element batch.
"""
from functools import lru_cache

import numpy as np

from . import basis


class Tables:
    def __init__(self, k, m):
        self.k, self.n, self.m = k, k + 1, m
        nodes = basis.lgl_nodes(k)
        zq, wq = basis.gauss_rule(m)
        L = basis.lagrange_values(nodes, zq)        # m x n
        Ld = basis.lagrange_derivs(nodes, zq)       # m x n
        Le = [basis.lagrange_values(nodes, [0.0]), basis.lagrange_values(nodes, [1.0])]   # 1 x n
        Lde = [basis.lagrange_derivs(nodes, [0.0]), basis.lagrange_derivs(nodes, [1.0])]  # 1 x n
        self.nodes = nodes
        self.qpts, self.qw = zq, wq

        def k3(fz, fy, fx):
            return np.kron(fz, np.kron(fy, fx))

        # cell tables: rows are points (qx fastest), columns basis functions
        self.B = k3(L, L, L)
        self.G = [k3(L, L, Ld), k3(L, Ld, L), k3(Ld, L, L)]
        self.W = k3(wq[:, None], wq[:, None], wq[:, None])[:, 0]

        # face tables: face (d, s); rows are the m^2 points of the two
        # tangential directions, lower-numbered direction fastest
        self.FV = [[None, None] for _ in range(3)]
        self.FG = [[[None] * 3 for _ in range(2)] for _ in range(3)]
        for s in range(2):
            for d in range(3):
                f = [L, L, L]
                f[d] = Le[s]
                self.FV[d][s] = k3(f[2], f[1], f[0])
                for g in range(3):
                    fg = list(f)
                    fg[g] = Lde[s] if g == d else Ld
                    self.FG[d][s][g] = k3(fg[2], fg[1], fg[0])
        self.WF = np.kron(wq[:, None], wq[:, None])[:, 0]


@lru_cache(maxsize=32)
def tables(k, m):
    return Tables(k, m)
