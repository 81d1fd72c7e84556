"""Pins of the oracle's multigrid V-cycle (CPU)."""
import numpy as np

from oracle import mesh as M
from oracle.laplace import laplace_apply, laplace_diagonal
from oracle.multigrid import level_meshes, vcycle
from oracle.solvers import lanczos_max_eig, pcg


def _lams(k, fine, levels):
    out = []
    for msh in level_meshes(fine, levels):
        dinv = np.tile(1.0 / laplace_diagonal(k, msh), msh.N)
        A = lambda v, msh=msh: laplace_apply(v.reshape(msh.N, -1), k, msh).ravel()
        out.append(1.1 * lanczos_max_eig(A, dinv, msh.N * (k + 1) ** 3, steps=25, project=True))
    return out


def test_vcycle_is_symmetric():
    # pre- and post-smoother are the same symmetric polynomial in D^-1 A times
    # D^-1, restriction is the transpose of prolongation: V = V^T
    k, fine, levels = 2, M.cube(4), 2
    lam = _lams(k, fine, levels)
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal((2, fine.N, (k + 1) ** 3))
    a = np.vdot(v, vcycle(u, k, fine, levels, lam))
    b = np.vdot(u, vcycle(v, k, fine, levels, lam))
    assert abs(a - b) < 1e-11 * abs(a)


def test_vcycle_contracts_the_error():
    # one cycle as an iteration x <- x + V (b - A x) reduces the A-norm of a
    # zero-mean error by well over half (the smoother alone: about 0.2 per
    # sweep on the high frequencies, nothing on the smooth ones)
    k, fine, levels = 3, M.cube(8), 3
    lam = _lams(k, fine, levels)
    e = np.random.default_rng(2).standard_normal((fine.N, (k + 1) ** 3))
    e -= e.mean()
    Ae = laplace_apply(e, k, fine)
    e2 = e - vcycle(Ae, k, fine, levels, lam)
    e2 -= e2.mean()
    ratio = np.sqrt(np.vdot(e2, laplace_apply(e2, k, fine)) / np.vdot(e, Ae))
    assert ratio < 0.5, ratio


def test_vcycle_preconditioned_cg_iterations():
    # the paper's range for its GMG-preconditioned pressure CG is 6-12
    # iterations; on this small periodic problem the V-cycle PCG converges to
    # 1e-10 within 15, where Jacobi-PCG needs several times as many
    k, fine, levels = 3, M.cube(8), 3
    lam = _lams(k, fine, levels)
    b = np.random.default_rng(3).standard_normal((fine.N, (k + 1) ** 3))
    b -= b.mean()
    A = lambda v: laplace_apply(v, k, fine)
    _, info = pcg(A, b, precond=lambda r: vcycle(r, k, fine, levels, lam), rtol=1e-10, project=True)
    dinv = (1.0 / laplace_diagonal(k, fine))[None, :]
    _, info_j = pcg(A, b, precond=lambda r: dinv * r, rtol=1e-10, project=True)
    assert info["iterations"] <= 15 and 3 * info["iterations"] < info_j["iterations"], (info["iterations"],
                                                                                        info_j["iterations"])
