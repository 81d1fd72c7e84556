"""Pins of the oracle's 1D basis and its explicit 3D tables (CPU only).

Pinned against closed forms (tests/golden), polynomial exactness and
monomial integrals, never against the oracle itself.
"""
import os
from math import sqrt  # noqa: F401  (used by the golden expressions)

import numpy as np
import pytest

from oracle import basis
from oracle.tables import tables

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            rows.append((int(tok[0]), [eval(t, {"sqrt": sqrt}) for t in tok[1:]]))
    return rows


def test_lgl_nodes_closed_form():
    for k, vals in _read_golden("lgl_nodes.txt"):
        ref = (np.array(vals) + 1.0) / 2.0
        np.testing.assert_allclose(basis.lgl_nodes(k), ref, rtol=0, atol=2e-16 * 8)


def test_lgl_nodes_are_lobatto_for_high_degree():
    # for every degree used: end points exact, interior = roots of P_k', symmetric
    from numpy.polynomial import legendre as L
    for k in range(2, 16):
        x = basis.lgl_nodes(k)
        assert x[0] == 0.0 and x[-1] == 1.0
        np.testing.assert_allclose(x + x[::-1], 1.0, atol=1e-15)
        c = np.zeros(k + 1)
        c[k] = 1
        d = L.legder(c)
        assert np.abs(L.legval(2 * x[1:-1] - 1, d)).max() < 1e-11 * k ** 2


def test_gauss_rule_closed_form():
    rows = _read_golden("gauss_rules.txt")
    for (m, pts), (m2, wts) in zip(rows[0::2], rows[1::2]):
        assert m == m2
        z, w = basis.gauss_rule(m)
        np.testing.assert_allclose(z, (np.array(pts) + 1) / 2, atol=1e-15)
        np.testing.assert_allclose(w, np.array(wts) / 2, atol=1e-15)


@pytest.mark.parametrize("m", [1, 3, 5, 8, 13, 17])
def test_gauss_exact_for_monomials(m):
    z, w = basis.gauss_rule(m)
    for p in range(2 * m):
        assert abs((w * z ** p).sum() - 1.0 / (p + 1)) < 1e-14


@pytest.mark.parametrize("k", [2, 3, 5, 8, 11])
def test_lagrange_cardinal_and_reproduction(k):
    x = basis.lgl_nodes(k)
    np.testing.assert_allclose(basis.lagrange_values(x, x), np.eye(k + 1), atol=1e-13)
    t = np.linspace(-0.3, 1.2, 37)
    for p in range(k + 1):
        # interpolation of t^p is exact; so is its derivative
        np.testing.assert_allclose(basis.lagrange_values(x, t) @ x ** p, t ** p, atol=1e-11)
        dref = p * t ** (p - 1) if p > 0 else 0 * t
        np.testing.assert_allclose(basis.lagrange_derivs(x, t) @ x ** p, dref, atol=1e-9 * k ** 2)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_3d_tables_integrate_polynomials_exactly(k):
    """P5: cell mass/stiffness entries of degree <= k data agree with
    a (2k+5)-point rule and with closed-form monomial integrals."""
    m = k + 1
    T = tables(k, m)
    Tr = tables(k, 2 * k + 5)
    np.testing.assert_allclose((T.B.T * T.W) @ T.B, (Tr.B.T * Tr.W) @ Tr.B, atol=1e-14)
    for d in range(3):
        np.testing.assert_allclose((T.G[d].T * T.W) @ T.G[d], (Tr.G[d].T * Tr.W) @ Tr.G[d],
                                   atol=1e-12 * k ** 4)
    # integral of x^p y^q z^r over [0,1]^3 from nodal coefficients
    x = basis.lgl_nodes(k)
    n = k + 1
    i = np.arange(n ** 3)
    a, b, c = i % n, (i // n) % n, i // (n * n)
    for (p, q, r) in [(0, 0, 0), (k, 0, 1), (1, k, k), (k, k, k)]:
        coeff = x[a] ** p * x[b] ** q * x[c] ** r
        val = T.W @ (T.B @ coeff)
        assert abs(val - 1.0 / ((p + 1) * (q + 1) * (r + 1))) < 1e-14
        # d/dx integral: p x^(p-1) y^q z^r
        dval = T.W @ (T.G[0] @ coeff)
        ref = (1.0 if p > 0 else 0.0) / ((q + 1) * (r + 1))
        assert abs(dval - ref) < 1e-13


def test_face_tables_pick_the_face_layer():
    k, m = 3, 4
    T = tables(k, m)
    n = k + 1
    idx = np.arange(n ** 3).reshape(n, n, n)       # [c, b, a]
    for d in range(3):
        for s in range(2):
            layer = np.take(idx, 0 if s == 0 else n - 1, axis=2 - d).ravel()
            mask = np.zeros(n ** 3, bool)
            mask[layer] = True
            assert np.abs(T.FV[d][s][:, ~mask]).max() == 0.0
            # values on the face: partition of unity
            np.testing.assert_allclose(T.FV[d][s].sum(1), 1.0, atol=1e-14)
            np.testing.assert_allclose(T.FG[d][s][d].sum(1), 0.0, atol=1e-12)
