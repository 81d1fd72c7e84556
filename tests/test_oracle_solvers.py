"""Pins of the oracle's divergence right-hand side and solvers (CPU only).

S1 fast diagonalisation solves A x = b with the 3D oracle operator; S3 the
Chebyshev iteration reproduces its closed-form error polynomial on a diagonal
matrix; S4 Jacobi- and Chebyshev-preconditioned CG agree with the direct
solve modulo the constant; the divergence form vanishes on constants, sums to
zero and is consistent with div u.
"""
import numpy as np
import pytest

from oracle import basis, mesh as M
from oracle.divergence import divergence_apply, poisson_rhs
from oracle.laplace import laplace_apply, laplace_diagonal
from oracle.solvers import chebyshev, fdm_solve, lanczos_max_eig, pcg
from oracle.tables import tables
from paper_1802_01439_amd.inputs import node_positions, tgv_plus_noise


def test_divergence_of_constant_is_zero_and_sums_vanish():
    k = 3
    msh = M.Mesh((3, 2, 4), (2 * np.pi, 2.0, 3.0))
    n3 = (k + 1) ** 3
    uc = np.ones((3, msh.N, n3)) * np.array([1.5, -0.2, 0.7])[:, None, None]
    assert np.abs(divergence_apply(uc, k, msh)).max() < 1e-13
    u = np.random.default_rng(0).uniform(-1, 1, (3, msh.N, n3))
    b = divergence_apply(u, k, msh)
    assert abs(b.sum()) < 1e-13 * np.abs(b).sum()


def test_divergence_consistency():
    k = 3
    errs = []
    for N in (4, 8, 16):
        msh = M.cube(N)
        x, y, z = node_positions(basis.lgl_nodes(k), msh.n_el, msh.length)
        u = np.stack([np.sin(x) * np.cos(z), np.sin(2 * y), np.cos(x + z)])
        divu = np.cos(x) * np.cos(z) + 2 * np.cos(2 * y) - np.sin(x + z)
        b = divergence_apply(u, k, msh)
        T = tables(k, k + 1)
        Me = np.prod(msh.h) * (T.B.T * T.W) @ T.B
        g = np.linalg.solve(Me, b.T).T
        errs.append(np.abs(g - divu).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 0.02 and rates.min() > k - 0.5


@pytest.mark.parametrize("k,msh", [(3, M.cube(4)), (2, M.Mesh((3, 4, 2), (2 * np.pi, 1.0, 2.0)))])
def test_S1_fdm_solves_the_3d_operator(k, msh):
    b = np.random.default_rng(5).standard_normal((msh.N, (k + 1) ** 3))
    b -= b.mean()
    x = fdm_solve(b, k, msh)
    r = laplace_apply(x, k, msh) - b
    assert np.linalg.norm(r) < 1e-11 * np.linalg.norm(b)


def test_S3_chebyshev_closed_form():
    lam = np.linspace(0.05, 1.0, 40)
    lmax, lmin = 1.0, 1.0 / 20
    b = np.random.default_rng(2).standard_normal(40)
    x = chebyshev(lambda v: lam * v, np.ones(40), b, 5, lmin, lmax)
    theta, delta = (lmax + lmin) / 2, (lmax - lmin) / 2
    T5 = lambda t: np.cos(5 * np.arccos(np.clip(t, -1, 1))) if np.all(np.abs(t) <= 1) else np.cosh(5 * np.arccosh(t))
    Rpoly = np.array([T5((theta - l) / delta) for l in lam]) / T5(np.array(theta / delta))
    np.testing.assert_allclose(1.0 - lam * x / b, Rpoly, atol=1e-13)
    # contraction factor on the interval: 1 / T5(21/19) = 0.2035 for range 20
    assert abs(1.0 / T5(np.array(21.0 / 19.0)) - 0.2035) < 1e-4


def test_lanczos_estimate_bounds_true_eigenvalue():
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    ev = np.linspace(0.1, 7.0, 60)
    A = (Q * ev) @ Q.T
    d = np.diag(A).copy()
    est = lanczos_max_eig(lambda v: A @ v, 1.0 / d, 60, steps=20)
    true = np.linalg.eigvals(A / d[:, None]).real.max()
    assert 0.97 * true <= est <= true * (1 + 1e-10)


def test_pcg_on_dense_spd():
    rng = np.random.default_rng(6)
    B = rng.standard_normal((50, 50))
    A = B @ B.T + 50 * np.eye(50)
    b = rng.standard_normal(50)
    x, info = pcg(lambda v: A @ v, b, lambda r: r / np.diag(A), rtol=1e-12)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10)


def test_S4_cg_jacobi_and_chebyshev_match_fdm():
    k = 3
    msh = M.cube(4)
    u = tgv_plus_noise(basis.lgl_nodes(k), msh.n_el, msh.length, seed=104)
    b = poisson_rhs(u, k, msh)
    x_ref = fdm_solve(b, k, msh)
    A = lambda v: laplace_apply(v, k, msh)
    dinv = 1.0 / np.tile(laplace_diagonal(k, msh), (msh.N, 1))
    xj, ij = pcg(A, b, lambda r: dinv * r, rtol=1e-10, project=True)
    lmax = 1.1 * lanczos_max_eig(lambda v: A(v.reshape(b.shape)).ravel(), dinv.ravel(), b.size,
                                 project=True)
    cheb = lambda r: chebyshev(A, dinv, r, 5, lmax / 20, lmax)
    xc, ic = pcg(A, b, cheb, rtol=1e-10, project=True)
    for x in (xj, xc):
        e = (x - x.mean()) - (x_ref - x_ref.mean())
        assert np.linalg.norm(e) < 1e-8 * np.linalg.norm(x_ref)
    assert ic["iterations"] < ij["iterations"] / 2
