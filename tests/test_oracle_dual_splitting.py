"""Pins of the oracle's mixed-order coupling terms, Taylor-Green diagnostics
and dual-splitting step (Sec. 3.1-3.3, Sec. 4), none of which re-types an
oracle formula:

* the mixed gradient (pressure degree k-1 -> velocity test space k) is minus
  the transpose of the mixed divergence (integration by parts with central
  fluxes on a periodic mesh);
* both vanish on constants and converge to the continuous divergence and
  gradient of smooth fields (interpolated, then divided by the mass matrix of
  the test space);
* e_k of the Taylor-Green field tends to 1/8 and eps to 3 nu / 4 (closed
  forms of (1/V) int u.u/2 and (nu/V) int grad u : grad u);
* the pressure of one step from the Taylor-Green field tends to the analytic
  pressure (cos 2x + cos 2y)(cos 2z + 2)/16 (a sign, factor or orientation
  error in the convective, divergence or pressure step fails it);
* the projection step removes most of the divergence the convective step
  introduces;
* a constant state is kept exactly, and a shear flow (0, 0, sin x), on which
  the convective term, the divergence and the penalties vanish, decays by the
  factor of the viscous step, 1/(1 + nu dt / gamma_0), for BDF1 and BDF2.
"""
import numpy as np
import pytest

from oracle import basis, mesh as M
from oracle.dual_splitting import bdf_coefficients, dual_splitting_step, tgv_diagnostics
from oracle.mass import inverse_mass_apply
from oracle.mixed import mixed_divergence_apply, mixed_gradient_apply
from paper_1802_01439_amd import inputs


def _xyz(k, msh):
    return inputs.node_positions(basis.lgl_nodes(k), msh.n_el, msh.length)


def test_mixed_gradient_is_minus_transpose_of_mixed_divergence():
    k = 2
    msh = M.Mesh((2, 2, 3), (2 * np.pi, 1.5, 2.0))
    nu, npr = 3 * msh.N * (k + 1) ** 3, msh.N * k ** 3
    D = np.stack([mixed_divergence_apply(e.reshape(3, msh.N, (k + 1) ** 3), k, msh).ravel()
                  for e in np.eye(nu)], axis=1)
    G = np.stack([mixed_gradient_apply(e.reshape(msh.N, k ** 3), k, msh).ravel() for e in np.eye(npr)], axis=1)
    assert D.shape == (npr, nu) and G.shape == (nu, npr)
    assert np.abs(G + D.T).max() < 1e-13 * np.abs(G).max()


def test_mixed_operators_vanish_on_constants():
    k = 4
    msh = M.Mesh((3, 2, 2), (1.0, 2.0, 3.0))
    c = np.ones((3, msh.N, (k + 1) ** 3)) * np.array([0.3, -1.2, 2.0])[:, None, None]
    assert np.abs(mixed_divergence_apply(c, k, msh)).max() < 1e-13
    assert np.abs(mixed_gradient_apply(np.full((msh.N, k ** 3), 1.7), k, msh)).max() < 1e-13


@pytest.mark.parametrize("k,meshes", [(2, (6, 12)), (3, (6, 12)), (5, (3, 6))])
def test_mixed_operators_converge_to_divergence_and_gradient(k, meshes):
    errs_d, errs_g = [], []
    for N in meshes:
        msh = M.cube(N)
        x, y, z = _xyz(k, msh)
        u = np.stack([np.sin(x) * np.cos(y), np.sin(y) * np.cos(z), np.sin(z) * np.cos(x)])
        xp, yp, zp = _xyz(k - 1, msh)
        div = np.cos(xp) * np.cos(yp) + np.cos(yp) * np.cos(zp) + np.cos(zp) * np.cos(xp)
        got = inverse_mass_apply(mixed_divergence_apply(u, k, msh), k - 1, msh)
        errs_d.append(np.abs(got - div).max())
        p = np.sin(xp) * np.cos(yp) * np.sin(zp)
        grad = np.stack([np.cos(x) * np.cos(y) * np.sin(z), -np.sin(x) * np.sin(y) * np.sin(z),
                         np.sin(x) * np.cos(y) * np.cos(z)])
        got = inverse_mass_apply(mixed_gradient_apply(p, k, msh), k, msh)
        errs_g.append(np.abs(got - grad).max())
    # halving h divides the error by about 2^(k-1) at least (the pressure
    # space has degree k-1)
    rate = lambda e: np.log2(e[0] / e[1])
    assert rate(errs_d) > k - 1.3 and errs_d[1] < 0.2, errs_d
    assert rate(errs_g) > k - 1.3 and errs_g[1] < 0.3, errs_g


def test_taylor_green_diagnostics_closed_forms():
    k, N, nu = 4, 6, 1.0 / 1600
    msh = M.cube(N)
    u = inputs.taylor_green(*_xyz(k, msh))
    ek, eps = tgv_diagnostics(u, k, msh, nu)
    assert abs(ek / 0.125 - 1) < 1e-6
    assert abs(eps / (0.75 * nu) - 1) < 1e-6


def test_step_pressure_tends_to_the_taylor_green_pressure():
    k, nu = 3, 1.0 / 1600
    errs = []
    for N in (4, 6, 8):
        msh = M.cube(N)
        u = inputs.taylor_green(*_xyz(k, msh))
        dt = 0.125 / k ** 1.5 * (2 * np.pi / N)
        r = dual_splitting_step([u], k, msh, dt, nu, order=1)
        xp, yp, zp = _xyz(k - 1, msh)
        p_ex = (np.cos(2 * xp) + np.cos(2 * yp)) * (np.cos(2 * zp) + 2) / 16
        p_ex -= p_ex.mean()
        errs.append(np.abs(r["p"] - p_ex).max() / np.abs(p_ex).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.03, errs


def test_projection_removes_the_divergence_of_the_convective_step():
    k, N = 3, 4
    msh = M.cube(N)
    u = inputs.taylor_green(*_xyz(k, msh))
    r = dual_splitting_step([u], k, msh, 0.125 / k ** 1.5 * (2 * np.pi / N), 1.0 / 1600, order=1)
    d_hat = np.linalg.norm(mixed_divergence_apply(r["u_hat"], k, msh))
    d_hh = np.linalg.norm(mixed_divergence_apply(r["u_hathat"], k, msh))
    assert d_hh < 0.1 * d_hat, (d_hat, d_hh)


@pytest.mark.parametrize("order", [1, 2])
def test_step_keeps_a_constant_state(order):
    k, N = 3, 3
    msh = M.cube(N)
    c = np.ones((3, msh.N, (k + 1) ** 3)) * np.array([0.3, -0.7, 1.1])[:, None, None]
    r = dual_splitting_step([c, c][:order], k, msh, 0.05, 0.01, order=order)
    assert np.abs(r["u"] - c).max() < 1e-13
    assert np.abs(r["p"]).max() < 1e-12


@pytest.mark.parametrize("order", [1, 2])
def test_step_shear_flow_decays_by_the_viscous_factor(order):
    k, N, nu, dt = 3, 6, 0.5, 0.1
    msh = M.cube(N)
    x, _, _ = _xyz(k, msh)
    u = np.stack([np.zeros_like(x), np.zeros_like(x), np.sin(x)])
    g0 = bdf_coefficients(order)[0]
    r = dual_splitting_step([u, u][:order], k, msh, dt, nu, order=order)
    assert np.abs(r["p"]).max() < 1e-12
    ref = u / (1 + nu * dt / g0)
    assert np.abs(r["u"] - ref).max() < 2e-4 * np.abs(u).max()
