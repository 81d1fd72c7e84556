"""Pins of the oracle's multigrid level transfers (CPU)."""
import numpy as np

from oracle import basis, mesh as M
from oracle.mass import inverse_mass_apply, mass_apply
from oracle.transfer import fine_mesh, prolongate, restrict


def test_prolongation_reproduces_elementwise_polynomials():
    # a different Q_k polynomial on every coarse element, evaluated at the
    # coarse nodes and, independently, at the nodes of its eight children
    for k in (1, 3, 5):
        coarse = M.Mesh((2, 3, 1), (1.0, 1.5, 0.8))
        fine = fine_mesh(coarse)
        rng = np.random.default_rng(20 + k)
        n = k + 1
        coef = rng.standard_normal((coarse.N, n, n, n))
        xi = basis.lgl_nodes(k)
        a = np.arange(n)
        ia, ib, ic = [g.transpose(2, 1, 0).ravel() for g in np.meshgrid(a, a, a, indexing="ij")]
        hc, hf = coarse.h, fine.h

        def evaluate(e, X, Y, Z):
            # X, Y, Z relative to the coarse element's origin, scaled by its size
            x, y, z = X / hc[0], Y / hc[1], Z / hc[2]
            return np.einsum("ijl,pi,pj,pl->p", coef[e], np.vander(x, n, increasing=True),
                             np.vander(y, n, increasing=True), np.vander(z, n, increasing=True))

        uc = np.zeros((coarse.N, n ** 3))
        for e in range(coarse.N):
            uc[e] = evaluate(e, xi[ia] * hc[0], xi[ib] * hc[1], xi[ic] * hc[2])
        uf = np.zeros((fine.N, n ** 3))
        fc = fine.coords()
        for f in range(fine.N):
            e = coarse.index(fc[f] // 2)
            ch = fc[f] % 2
            uf[f] = evaluate(e, (xi[ia] + ch[0]) * hf[0], (xi[ib] + ch[1]) * hf[1], (xi[ic] + ch[2]) * hf[2])
        assert np.max(np.abs(prolongate(uc, k, coarse) - uf)) < 1e-11 * np.max(np.abs(uf))


def test_restriction_is_the_transpose():
    k = 2
    coarse = M.Mesh((2, 1, 2), (1.0, 1.0, 1.0))
    rng = np.random.default_rng(3)
    n3 = (k + 1) ** 3
    u = rng.standard_normal((coarse.N, n3))
    r = rng.standard_normal((8 * coarse.N, n3))
    assert abs(np.vdot(prolongate(u, k, coarse), r) - np.vdot(u, restrict(r, k, coarse))) < 1e-12 * np.linalg.norm(r)


def test_mass_weighted_restriction_inverts_the_prolongation():
    # the fine space contains the coarse one: M_c^-1 P^T M_f P = I
    for k in (2, 4):
        coarse = M.Mesh((3, 2, 2), (1.2, 0.7, 1.0))
        fine = fine_mesh(coarse)
        u = np.random.default_rng(7 + k).standard_normal((3, coarse.N, (k + 1) ** 3))
        back = inverse_mass_apply(restrict(mass_apply(prolongate(u, k, coarse), k, fine), k, coarse), k, coarse)
        assert np.max(np.abs(back - u)) < 1e-11 * np.max(np.abs(u))
