"""Pins of the oracle's convective operator, its Jacobian, JVP and VJP (CPU only).

C1 constants give zero residual element by element; C2 momentum is conserved
on periodic meshes; C3 the 3D operator reduces to a textbook 1D DG scheme for
(u^2)_x with the LLF flux; C4 consistency with div(u (x) u) for the
Taylor-Green field (closed form).  V1 central differences, V2 matrix-free JVP
against the assembled Jacobian, V4 the Euler identity of a 2-homogeneous
operator, V5 zero velocity.
"""
import numpy as np
import pytest

from oracle import basis, mesh as M
from oracle.convective import convective_apply, convective_jacobian, convective_jvp, convective_vjp
from oracle.tables import tables
from paper_1802_01439_amd.inputs import node_positions, taylor_green

MSH = M.Mesh((3, 2, 4), (2 * np.pi, 2.0, 3.0))


def _rand(shape, seed):
    return np.random.default_rng(seed).uniform(-1, 1, shape)


@pytest.mark.parametrize("k", [2, 3, 5])
def test_C1_constant_gives_zero(k):
    n3 = (k + 1) ** 3
    u = np.ones((3, MSH.N, n3)) * np.array([0.3, -0.7, 1.1])[:, None, None]
    R = convective_apply(u, k, MSH)
    assert np.abs(R).max() < 1e-13


@pytest.mark.parametrize("k,lf", [(2, 1.0), (3, 0.5), (4, 1.0)])
def test_C2_momentum_conservation(k, lf):
    u = _rand((3, MSH.N, (k + 1) ** 3), k)
    R = convective_apply(u, k, MSH, lf_factor=lf)
    # sum_i phi_i = 1, so sum over all coefficients of R_c is c_h(e_c, u) = 0
    assert np.abs(R.sum(axis=(1, 2))).max() < 1e-13 * np.abs(R).max() * R[0].size ** 0.5


def _textbook_1d(u1, k, N, h, lf):
    """1D DG residual of (u^2)_x: -int l_a' u^2 + l_a(1) f(u_e(1), u_e+1(0)) - l_a(0) f(u_e-1(1), u_e(0)),
    f(uL, uR) = (uL^2 + uR^2)/2 + lf * max(|uL|, |uR|) (uL - uR)."""
    nodes = basis.lgl_nodes(k)
    z, w = basis.gauss_rule(2 * k + 2)
    L = basis.lagrange_values(nodes, z)
    Ld = basis.lagrange_derivs(nodes, z) / h
    u_q = u1 @ L.T
    R = -h * (u_q ** 2 * w) @ Ld
    uR = u1[:, -1]       # value at right end of each element
    uL = u1[:, 0]
    def f(a, b):
        return 0.5 * (a * a + b * b) + lf * np.maximum(np.abs(a), np.abs(b)) * (a - b)
    right = f(uR, np.roll(uL, -1))
    left = f(np.roll(uR, 1), uL)
    R[:, -1] += right
    R[:, 0] -= left
    return R


@pytest.mark.parametrize("k,lf", [(2, 1.0), (3, 1.0), (5, 0.5)])
def test_C3_one_dimensional_reduction(k, lf):
    n = k + 1
    msh = M.Mesh((4, 2, 3), (2 * np.pi, 1.5, 2.5))
    Nx, Ny, Nz = msh.n_el
    u1d = _rand((Nx, n), 7 + k)
    e = np.arange(msh.N)
    i = np.arange(n ** 3)
    ex = e % Nx
    a = i % n
    u = np.zeros((3, msh.N, n ** 3))
    u[0] = u1d[ex][:, a]
    R = convective_apply(u, k, msh, lf_factor=lf)
    R1 = _textbook_1d(u1d, k, Nx, msh.h[0], lf)
    z, w = basis.gauss_rule(n)
    wb = [msh.h[d] * w @ basis.lagrange_values(basis.lgl_nodes(k), z) for d in range(3)]
    b, c = (i // n) % n, i // (n * n)
    ref = R1[ex][:, a] * wb[1][b][None, :] * wb[2][c][None, :]
    np.testing.assert_allclose(R[0], ref, atol=1e-13)
    assert np.abs(R[1:]).max() < 1e-14


def test_C4_taylor_green_consistency():
    """M^-1 R(I u) -> div(u (x) u) = (sin2x cos^2 z / 2, sin2y cos^2 z / 2, 0)."""
    k = 3
    errs = []
    for N in (4, 8, 16):
        msh = M.cube(N)
        x, y, z = node_positions(basis.lgl_nodes(k), msh.n_el, msh.length)
        u = taylor_green(x, y, z)
        R = convective_apply(u, k, msh)
        T = tables(k, k + 1)
        Me = np.prod(msh.h) * (T.B.T * T.W) @ T.B
        g = np.stack([np.linalg.solve(Me, R[c].T).T for c in range(3)])
        ref = np.stack([0.5 * np.sin(2 * x) * np.cos(z) ** 2, 0.5 * np.sin(2 * y) * np.cos(z) ** 2, 0 * x])
        errs.append(np.abs(g - ref).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 2e-3
    assert rates.min() > k - 0.5


@pytest.mark.parametrize("k", [2, 4])
def test_V1_central_differences(k):
    u = _rand((3, MSH.N, (k + 1) ** 3), 11)
    v = np.random.default_rng(1011).standard_normal(u.shape)
    w = np.random.default_rng(2011).standard_normal(u.shape)
    eps = 1e-6
    fd = (convective_apply(u + eps * v, k, MSH) - convective_apply(u - eps * v, k, MSH)) / (2 * eps)
    lhs = (w * fd).sum()
    rhs = (convective_vjp(u, w, k, MSH) * v).sum()
    assert abs(lhs - rhs) <= 1e-7 * abs(rhs) + 1e-9
    jvp = convective_jvp(u, v, k, MSH)
    assert np.abs(fd - jvp).max() <= 1e-7 * np.abs(jvp).max()


@pytest.mark.parametrize("k,lf", [(2, 1.0), (3, 0.3)])
def test_V2_assembled_jacobian_matches_matrix_free_jvp(k, lf):
    u = _rand((3, MSH.N, (k + 1) ** 3), 12)
    v = _rand(u.shape, 13)
    J = convective_jacobian(u, k, MSH, lf_factor=lf)
    np.testing.assert_allclose((J @ v.ravel()).reshape(u.shape), convective_jvp(u, v, k, MSH, lf_factor=lf),
                               atol=1e-13 * np.abs(v).max() * 10)


@pytest.mark.parametrize("k", [2, 3])
def test_V4_euler_identity(k):
    """R is positively 2-homogeneous: J(u) u = 2 R(u), hence <J^T w, u> = 2 <w, R(u)>."""
    u = _rand((3, MSH.N, (k + 1) ** 3), 14)
    w = _rand(u.shape, 15)
    R = convective_apply(u, k, MSH)
    g = convective_vjp(u, w, k, MSH)
    assert abs((g * u).sum() - 2 * (w * R).sum()) < 1e-12 * np.abs(R).sum()


def test_V4_euler_identity_at_exact_ties():
    """Ties |u^-.n| = |u^+.n| on every face: the half-half convention keeps J u = 2 R(u)."""
    k = 2
    n3 = (k + 1) ** 3
    msh = M.cube(2)
    u = np.zeros((3, msh.N, n3))
    u[0] = 0.5
    u[0, ::2] = -0.5    # alternating sign in x: u.n flips sign across x-faces, |.| ties
    u[1] = 0.25
    J = convective_jacobian(u, k, msh)
    R = convective_apply(u, k, msh)
    np.testing.assert_allclose((J @ u.ravel()).reshape(u.shape), 2 * R, atol=1e-13)


def test_V5_zero_velocity():
    k = 3
    u = np.zeros((3, MSH.N, (k + 1) ** 3))
    w = _rand(u.shape, 16)
    assert np.abs(convective_vjp(u, w, k, MSH)).max() == 0.0
