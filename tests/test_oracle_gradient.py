"""Pins of the oracle's pressure gradient g_h (CPU)."""
import numpy as np

from oracle import basis, mesh as M
from oracle.divergence import divergence_apply
from oracle.gradient import gradient_apply
from oracle.mass import inverse_mass_apply


def test_gradient_is_minus_the_transpose_of_the_divergence():
    # with central fluxes on a periodic mesh, integration by parts element by
    # element and [[p u]] = {{p}}[[u]] + [[p]]{{u}} give g_h(v, p) = -d_h(p, v)
    k = 2
    msh = M.Mesh((3, 2, 2), (1.3, 0.8, 1.1))
    n3 = (k + 1) ** 3
    nu, npr = 3 * msh.N * n3, msh.N * n3
    D = np.zeros((npr, nu))
    for i in range(nu):
        e = np.zeros(nu)
        e[i] = 1.0
        D[:, i] = divergence_apply(e.reshape(3, msh.N, n3), k, msh).ravel()
    G = np.zeros((nu, npr))
    for i in range(npr):
        e = np.zeros(npr)
        e[i] = 1.0
        G[:, i] = gradient_apply(e.reshape(msh.N, n3), k, msh).ravel()
    assert np.max(np.abs(G + D.T)) < 1e-13 * np.max(np.abs(D))


def test_gradient_of_a_constant_is_zero():
    k = 3
    msh = M.Mesh((3, 3, 2), (1.0, 2.0, 1.5))
    y = gradient_apply(np.full((msh.N, (k + 1) ** 3), 2.5), k, msh)
    assert np.max(np.abs(y)) < 1e-13


def test_gradient_consistency_on_a_smooth_field():
    # M^-1 g_h(., p) of the nodal interpolant of p = sin x cos 2y sin z tends to grad p
    errs = []
    for k in (3, 5, 7):
        msh = M.cube(4)
        n = k + 1
        xi = basis.lgl_nodes(k)
        c = msh.coords()
        h = msh.h
        a = np.arange(n)
        ia, ib, ic = [g.transpose(2, 1, 0).ravel() for g in np.meshgrid(a, a, a, indexing="ij")]
        X = (c[:, 0:1] + xi[ia][None, :]) * h[0]
        Y = (c[:, 1:2] + xi[ib][None, :]) * h[1]
        Z = (c[:, 2:3] + xi[ic][None, :]) * h[2]
        p = np.sin(X) * np.cos(2 * Y) * np.sin(Z)
        g = np.stack([np.cos(X) * np.cos(2 * Y) * np.sin(Z), -2 * np.sin(X) * np.sin(2 * Y) * np.sin(Z),
                      np.sin(X) * np.cos(2 * Y) * np.cos(Z)])
        y = inverse_mass_apply(gradient_apply(p, k, msh), k, msh)
        errs.append(np.max(np.abs(y - g)))
    # spectral convergence on the fixed 4^3 mesh (0.14, 4e-3, 6e-5)
    assert errs[0] < 0.2 and errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10 and errs[2] < 1e-4
