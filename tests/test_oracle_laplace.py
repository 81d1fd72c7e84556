"""Pins of the oracle's SIPG Laplace operator (CPU only).

Each check is fixed by the mathematics of the weak form (Sec. 3.2) rather
than by the oracle: A 1 = 0, symmetry, semi-definiteness with a one-dimensional
null space, the Kronecker-sum identity against an independently written 1D
textbook SIPG matrix, the spectrum of the continuous operator and consistency
with -Laplace on smooth data.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import basis, mesh as M
from oracle.laplace import laplace_apply, laplace_diagonal, laplace_matrix, mass_apply
from oracle.solvers import mass_1d, sipg_1d, to_tensor
from oracle.tables import tables

ANISO = M.Mesh((2, 3, 2), (2 * np.pi, 1.7, 3.1))


@pytest.mark.parametrize("k", [2, 3, 5, 7])
def test_P1_constant_in_null_space(k):
    msh = M.Mesh((3, 2, 4), (2 * np.pi, 2.0, 5.0))
    u = np.ones((msh.N, (k + 1) ** 3))
    y = laplace_apply(u, k, msh)
    assert np.abs(y).max() < 1e-11 * np.abs(laplace_diagonal(k, msh)).max()


@pytest.mark.parametrize("k,msh", [(2, M.cube(3)), (3, M.cube(2)), (2, ANISO)])
def test_P2_symmetric(k, msh):
    A = laplace_matrix(k, msh)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()


@pytest.mark.parametrize("k", [2, 3, 4])
def test_P3_psd_one_zero_eigenvalue(k):
    msh = M.cube(2) if k > 2 else M.cube(3)
    A = laplace_matrix(k, msh)
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    tol = 1e-12 * ev[-1]
    assert ev[0] > -tol
    assert abs(ev[0]) < tol
    assert ev[1] > 1e3 * tol


def _kron_sum(k, msh, penalty=1.0):
    h = msh.h
    K = [sipg_1d(k, msh.n_el[d], h[d], penalty) for d in range(3)]
    Mm = [mass_1d(k, msh.n_el[d], h[d]) for d in range(3)]
    return (np.kron(K[2], np.kron(Mm[1], Mm[0])) + np.kron(Mm[2], np.kron(K[1], Mm[0]))
            + np.kron(Mm[2], np.kron(Mm[1], K[0])))


@pytest.mark.parametrize("k,msh,pen", [(2, M.cube(3), 1.0), (3, ANISO, 1.0), (4, M.cube(2), 2.5),
                                       (5, M.Mesh((1, 2, 2), (1.0, 2.0, 1.5)), 1.0)])
def test_P4_kronecker_identity(k, msh, pen):
    """A = K(x)M(x)M + M(x)K(x)M + M(x)M(x)K with the 1D textbook matrices."""
    A = laplace_matrix(k, msh, penalty_factor=pen)
    n3 = (k + 1) ** 3
    perm = to_tensor(np.arange(msh.N * n3).reshape(msh.N, n3), msh, k).ravel()
    Ap = A[np.ix_(perm, perm)]
    A3 = _kron_sum(k, msh, pen)
    assert np.abs(Ap - A3).max() <= 1e-13 * np.abs(A3).max()


def test_1d_textbook_sipg_is_a_consistent_laplacian():
    """The 1D matrix used above is pinned on its own: symmetric, K 1 = 0,
    generalised eigenvalues of (K, M) approach the continuous kappa^2."""
    k, N = 4, 6
    h = 2 * np.pi / N
    K = sipg_1d(k, N, h)
    Mm = mass_1d(k, N, h)
    assert np.abs(K - K.T).max() < 1e-13 * np.abs(K).max()
    assert np.abs(K.sum(1)).max() < 1e-12 * np.abs(K).max()
    w = sla.eigh(K, Mm, eigvals_only=True)
    np.testing.assert_allclose(w[:7], [0, 1, 1, 4, 4, 9, 9], rtol=1e-3, atol=1e-10)


@pytest.mark.parametrize("k", [2, 3, 5])
def test_P6_smallest_eigenvalues_of_A_M(k):
    """Smallest non-zero generalised eigenvalue of (A, M) ~ |kappa|^2 = 1 on [-pi, pi]^3."""
    msh = M.cube(2 if k >= 3 else 3)
    A = laplace_matrix(k, msh)
    n3 = (k + 1) ** 3
    Mm = mass_apply(np.eye(msh.N * n3).reshape(-1, msh.N, n3), k, msh).reshape(msh.N * n3, -1).T
    w = sla.eigh(0.5 * (A + A.T), 0.5 * (Mm + Mm.T), eigvals_only=True)
    assert abs(w[0]) < 1e-10
    np.testing.assert_allclose(w[1:7], 1.0, rtol=2e-2 if k <= 3 else 1e-4)


def _interp(f, k, msh):
    from paper_1802_01439_amd.inputs import node_positions
    x, y, z = node_positions(basis.lgl_nodes(k), msh.n_el, msh.length)
    return f(x, y, z)


def test_P7_consistency_with_minus_laplace():
    """M^-1 A I(f) -> -Laplace(f) = 3 f for f = sin x sin y sin z, at rate >= k-1."""
    k = 3
    errs = []
    for N in (4, 8, 16):
        msh = M.cube(N)
        f = _interp(lambda x, y, z: np.sin(x) * np.sin(y) * np.sin(z), k, msh)
        y = laplace_apply(f, k, msh)
        T = tables(k, k + 1)
        Me = np.prod(msh.h) * (T.B.T * T.W) @ T.B
        g = np.linalg.solve(Me, y.T).T
        errs.append(np.abs(g - 3 * f).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 0.01
    assert rates.min() > k - 1.3


def test_diagonal_matches_kronecker_formula():
    k = 4
    msh = M.cube(3)
    d = laplace_diagonal(k, msh, penalty_factor=1.5, scale=0.7)
    h = msh.h[0]
    K = sipg_1d(k, 3, h, 1.5)[:k + 1, :k + 1]
    Mm = mass_1d(k, 3, h)[:k + 1, :k + 1]
    kd, md = np.diag(K), np.diag(Mm)
    n = k + 1
    i = np.arange(n ** 3)
    a, b, c = i % n, (i // n) % n, i // (n * n)
    ref = kd[a] * md[b] * md[c] + md[a] * kd[b] * md[c] + md[a] * md[b] * kd[c]
    np.testing.assert_allclose(d, 0.7 * ref, rtol=1e-13)


def test_scale_and_components_are_linear():
    k = 2
    msh = M.cube(3)
    rng = np.random.default_rng(3)
    u = rng.uniform(-1, 1, (3, msh.N, (k + 1) ** 3))
    y3 = laplace_apply(u, k, msh, scale=0.25)
    for c in range(3):
        np.testing.assert_allclose(y3[c], 0.25 * laplace_apply(u[c], k, msh), rtol=1e-15, atol=1e-15)


def test_elems_subset_matches_full():
    k = 3
    msh = M.Mesh((3, 4, 2), (1.0, 2.0, 3.0))
    u = np.random.default_rng(1).uniform(-1, 1, (msh.N, 64))
    full = laplace_apply(u, k, msh)
    sub = [0, 5, 23, 11]
    np.testing.assert_allclose(laplace_apply(u, k, msh, elems=sub), full[sub], rtol=1e-14, atol=1e-14)
