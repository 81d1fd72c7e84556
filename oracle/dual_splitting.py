"""One time step of the dual splitting scheme and the Taylor-Green
diagnostics, composed from the oracle operators (test infrastructure only).

Sec. 3.1, the four substeps in matrix form (Sec. 3.3), BDF of order J with
coefficients gamma_0, alpha_i and the extrapolation beta_i of the convective
term, no body force, periodic mesh (no inhomogeneous boundary terms):

  1. convective step   M (gamma_0 U^ - sum_i alpha_i U^{n-i}) / dt = -sum_i beta_i C(U^{n-i})
  2. pressure step     L P = -(gamma_0 / dt) D U^            (pressure degree k - 1)
  3. projection step   (M + A_D + A_C) U^^ = M U^ - (dt / gamma_0) G P
  4. viscous step      (gamma_0 / dt M + V) U^{n+1} = (gamma_0 / dt) M U^^

with C the convective form, D and G the mixed-order divergence and gradient,
L the SIPG Laplacian of the pressure space, V = nu times the SIPG Laplacian
per velocity component, and the penalty factors of A_D and A_C from the
extrapolated velocity (Sec. 3.2): tau_D = zeta_D |u_ex|_e h / (k + 1) dt,
tau_C = zeta_C |u_ex|_e dt, |u_ex|_e the volume average of the velocity
magnitude over the element, h = V_e^(1/3).  The linear systems are solved to
a tight tolerance (the pressure exactly, by fast diagonalisation), so the
result is the step's discrete solution up to rounding.

Diagnostics (Sec. 4.2): e_k = (1/V) int 1/2 u.u and
eps = (nu/V) int grad u : grad u (element by element).
"""
import numpy as np

from .convective import convective_apply
from .laplace import laplace_apply
from .mass import inverse_mass_apply, mass_apply
from .mixed import mixed_divergence_apply, mixed_gradient_apply
from .projection import projection_apply
from .solvers import fdm_solve, pcg
from .tables import tables


def bdf_coefficients(order):
    """(gamma_0, alpha, beta) of BDF1/BDF2 with the extrapolation of the
    same order (Sec. 3.1; BDF2 in the paper's runs, BDF1 as the start-up)."""
    if order == 1:
        return 1.0, (1.0,), (1.0,)
    if order == 2:
        return 1.5, (2.0, -0.5), (2.0, -1.0)
    raise ValueError("order must be 1 or 2")


def element_mean_speed(u, k, mesh):
    """(1/V_e) int_e |u| per element, by the (k+1)-point Gauss rule."""
    T = tables(k, k + 1)
    u = np.asarray(u, dtype=np.float64)
    uq = np.stack([u[j] @ T.B.T for j in range(3)])       # [3, N_el, points]
    return np.sqrt((uq ** 2).sum(axis=0)) @ T.W


def penalty_parameters(u_ex, k, mesh, dt, zeta_d=1.0, zeta_c=1.0):
    """tau_D and tau_C per element from the extrapolated velocity (Sec. 3.2)."""
    s = element_mean_speed(u_ex, k, mesh)
    h = float(np.prod(mesh.h)) ** (1.0 / 3.0)
    return zeta_d * s * h / (k + 1) * dt, zeta_c * s * dt


def tgv_diagnostics(u, k, mesh, nu):
    """(e_k, eps) of a velocity field u: [3, N_el, (k+1)^3] (Sec. 4.2)."""
    T = tables(k, k + 1)
    h = mesh.h
    vol = float(np.prod(h))
    V = vol * mesh.N
    u = np.asarray(u, dtype=np.float64)
    ek = 0.5 * sum(float(np.vdot(u[j], mass_apply(u[j], k, mesh))) for j in range(3)) / V
    g2 = 0.0
    for j in range(3):
        for d in range(3):
            gq = (u[j] @ T.G[d].T) / h[d]                   # d_d u_j at the cell points
            g2 += vol * float(((gq ** 2) @ T.W).sum())
    return ek, nu * g2 / V


def dual_splitting_step(u_hist, k, mesh, dt, nu, order=2, penalty_factor=1.0, lf_factor=1.0,
                        zeta_d=1.0, zeta_c=1.0, rtol=1e-13):
    """u_hist = [u^n, u^{n-1}, ...] (at least `order` fields, [3, N_el, (k+1)^3]).
    Returns dict(u_hat, p, u_hathat, u, tau_d, tau_c); p has zero coefficient mean."""
    g0, alpha, beta = bdf_coefficients(order)
    u_hist = [np.asarray(v, dtype=np.float64) for v in u_hist[:order]]
    # 1. convective step
    conv = sum(b * convective_apply(v, k, mesh, lf_factor=lf_factor) for b, v in zip(beta, u_hist))
    u_hat = (sum(a * v for a, v in zip(alpha, u_hist)) - dt * inverse_mass_apply(conv, k, mesh)) / g0
    # 2. pressure Poisson step (degree k - 1, periodic: zero-mean right-hand side)
    rhs = -(g0 / dt) * mixed_divergence_apply(u_hat, k, mesh)
    rhs -= rhs.mean()
    p = fdm_solve(rhs, k - 1, mesh, penalty_factor=penalty_factor)
    p -= p.mean()
    # 3. projection step
    u_ex = sum(b * v for b, v in zip(beta, u_hist))
    tau_d, tau_c = penalty_parameters(u_ex, k, mesh, dt, zeta_d, zeta_c)
    rhs3 = mass_apply(u_hat, k, mesh) - (dt / g0) * mixed_gradient_apply(p, k, mesh)
    u_hh, _ = pcg(lambda v: projection_apply(v, k, mesh, tau_d, tau_c), rhs3,
                  precond=lambda r: inverse_mass_apply(r, k, mesh), rtol=rtol)
    # 4. viscous step, each component with the Laplacian scaled by nu
    rhs4 = (g0 / dt) * mass_apply(u_hh, k, mesh)

    def helm(v):
        return (g0 / dt) * mass_apply(v, k, mesh) + laplace_apply(v, k, mesh, penalty_factor=penalty_factor,
                                                                 scale=nu)
    u_new, _ = pcg(helm, rhs4, precond=lambda r: inverse_mass_apply(r, k, mesh), rtol=rtol)
    return dict(u_hat=u_hat, p=p, u_hathat=u_hh, u=u_new, tau_d=tau_d, tau_c=tau_c)
