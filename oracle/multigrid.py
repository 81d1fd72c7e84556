"""Geometric multigrid V-cycle for the SIPG Laplacian (test infrastructure
only).

Sec. 3.3: the pressure Poisson equation is preconditioned by one V-cycle of
geometric multigrid with a Chebyshev smoother of D^-1 A (pre- and
post-smoothing of the same degree, smoothing range 20) and a Chebyshev
method with a fixed number of steps on the coarsest level.  Levels here:
the periodic mesh and its coarsenings by two per direction, same degree,
each level with its own SIPG operator (re-discretised) and diagonal; level
transfers from transfer.py.  Post-smoothing smooths the residual equation
from zero, so the smoother is always the zero-start Chebyshev of solvers.py.
"""
import numpy as np

from .laplace import laplace_apply, laplace_diagonal
from .mesh import Mesh
from .solvers import chebyshev
from .transfer import prolongate, restrict


def level_meshes(fine, levels):
    out = [fine]
    for l in range(1, levels):
        n = tuple(m // 2 ** l for m in fine.n_el)
        if any(m < 1 or m * 2 ** l != f for m, f in zip(n, fine.n_el)):
            raise ValueError("element counts must be divisible by 2^(levels-1)")
        out.append(Mesh(n, fine.length))
    return out


def vcycle(r, k, fine, levels, lam_max, degree=5, smoothing_range=20.0, coarse_degree=10,
           penalty_factor=1.0, scale=1.0):
    """z = V r on the fine mesh; r: [N_el, (k+1)^3]; lam_max[l]: the largest
    eigenvalue bound of D_l^-1 A_l used by level l's Chebyshev smoother."""
    meshes = level_meshes(fine, levels)

    def cycle(b, l):
        msh = meshes[l]

        def A(v):
            return laplace_apply(v, k, msh, penalty_factor=penalty_factor, scale=scale)

        dinv = (1.0 / laplace_diagonal(k, msh, penalty_factor=penalty_factor, scale=scale))[None, :]
        lmax = lam_max[l]
        lmin = lmax / smoothing_range
        if l == levels - 1:
            return chebyshev(A, dinv, b, coarse_degree, lmin, lmax)
        x = chebyshev(A, dinv, b, degree, lmin, lmax)                  # pre-smoothing
        x = x + prolongate(cycle(restrict(b - A(x), k, meshes[l + 1]), l + 1), k, meshes[l + 1])
        return x + chebyshev(A, dinv, b - A(x), degree, lmin, lmax)    # post-smoothing

    return cycle(np.asarray(r, dtype=np.float64), 0)
