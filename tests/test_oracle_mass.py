"""Pins of the oracle's mass matrix and its inverse (CPU)."""
import numpy as np
import pytest
from numpy.polynomial import legendre

from oracle import basis, mesh as M
from oracle.mass import inverse_mass_apply, mass_apply, mass_block


def _poly(coef, x):
    return np.polynomial.polynomial.polyval(x, coef)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7])
def test_inverse_mass_recovers_polynomials_of_the_space(k):
    """b_i = (phi_i, f) for f in Q_k, integrated with an independent Gauss-Legendre
    rule of k+3 points per direction; M^-1 b is then f at the element's nodes
    (the L2 projection onto the DG space reproduces its own members)."""
    rng = np.random.default_rng(7 + k)
    msh = M.Mesh((2, 3, 2), (1.0, 2.0, 1.5))
    cx, cy, cz = (rng.standard_normal(k + 1) for _ in range(3))
    nodes = basis.lgl_nodes(k)
    xg, wg = legendre.leggauss(k + 3)
    xg, wg = 0.5 * (xg + 1.0), 0.5 * wg                      # on [0, 1]
    Lg = basis.lagrange_values(nodes, xg)                    # (k+3) x (k+1)
    n = k + 1
    b = np.zeros((msh.N, n ** 3))
    f_nodes = np.zeros((msh.N, n ** 3))
    h = msh.h
    for e in range(msh.N):
        ex, ey, ez = e % msh.n_el[0], (e // msh.n_el[0]) % msh.n_el[1], e // (msh.n_el[0] * msh.n_el[1])
        x0 = np.array([ex * h[0], ey * h[1], ez * h[2]])
        fx = _poly(cx, x0[0] + h[0] * xg) * wg * h[0]
        fy = _poly(cy, x0[1] + h[1] * xg) * wg * h[1]
        fz = _poly(cz, x0[2] + h[2] * xg) * wg * h[2]
        bx, by, bz = Lg.T @ fx, Lg.T @ fy, Lg.T @ fz           # 1D moments
        b[e] = np.kron(bz, np.kron(by, bx))
        f_nodes[e] = np.kron(_poly(cz, x0[2] + h[2] * nodes),
                             np.kron(_poly(cy, x0[1] + h[1] * nodes), _poly(cx, x0[0] + h[0] * nodes)))
    x = inverse_mass_apply(b, k, msh)
    assert np.max(np.abs(x - f_nodes)) < 1e-10 * np.max(np.abs(f_nodes))


def test_mass_block_is_spd_with_volume_trace_of_partition_of_unity():
    k = 4
    msh = M.Mesh((3, 3, 3), (1.0, 2.0, 3.0))
    Mb = mass_block(k, msh)
    assert np.allclose(Mb, Mb.T, atol=1e-15)
    assert np.min(np.linalg.eigvalsh(Mb)) > 0
    # sum_ij M_ij = (1, 1) = element volume
    assert abs(Mb.sum() - np.prod(msh.h)) < 1e-13


def test_inverse_undoes_mass_and_scales_with_the_cell():
    k = 3
    rng = np.random.default_rng(3)
    m1 = M.cube(2)
    m2 = M.cube(2, length=2 * 2 * np.pi)                      # cells twice as large
    u = rng.standard_normal((3, m1.N, (k + 1) ** 3))
    assert np.allclose(inverse_mass_apply(mass_apply(u, k, m1), k, m1), u, atol=1e-11)
    assert np.allclose(inverse_mass_apply(u, k, m2), inverse_mass_apply(u, k, m1) / 8.0, rtol=1e-12)
