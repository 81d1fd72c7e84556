"""Pins of the oracle's projection-step operator (CPU)."""
import numpy as np
from numpy.polynomial import legendre

from oracle import basis, mesh as M
from oracle.mass import mass_apply
from oracle.projection import projection_apply


def _nodal_field(k, msh, fns):
    """[3, N_el, n^3] nodal values of the functions fns[j](x, y, z)."""
    nodes = basis.lgl_nodes(k)
    n = k + 1
    c = msh.coords()
    h = msh.h
    a = np.arange(n)
    ia, ib, ic = np.meshgrid(a, a, a, indexing="ij")
    ia, ib, ic = ia.transpose(2, 1, 0).ravel(), ib.transpose(2, 1, 0).ravel(), ic.transpose(2, 1, 0).ravel()
    X = (c[:, 0:1] + nodes[ia][None, :]) * h[0]
    Y = (c[:, 1:2] + nodes[ib][None, :]) * h[1]
    Z = (c[:, 2:3] + nodes[ic][None, :]) * h[2]
    return np.stack([f(X, Y, Z) for f in fns])


def test_divergence_penalty_vanishes_on_divergence_free_fields():
    # u = (y, z, x): linear, divergence free; tau_C = 0 leaves mass + A_D
    k = 3
    msh = M.Mesh((3, 2, 2), (3.0, 2.0, 2.0))
    u = _nodal_field(k, msh, [lambda x, y, z: y, lambda x, y, z: z, lambda x, y, z: x])
    td = np.linspace(0.5, 2.0, msh.N)
    y = projection_apply(u, k, msh, td, np.zeros(msh.N))
    assert np.allclose(y, mass_apply(u, k, msh), atol=1e-12)


def test_continuity_penalty_vanishes_on_continuous_fields():
    # periodic smooth field: traces agree at the shared LGL face nodes
    k = 4
    msh = M.cube(3)
    u = _nodal_field(k, msh, [lambda x, y, z: np.sin(x) * np.cos(z), lambda x, y, z: np.cos(y + z),
                              lambda x, y, z: np.sin(x + y)])
    tc = np.linspace(0.3, 3.0, msh.N)
    y = projection_apply(u, k, msh, np.zeros(msh.N), tc)
    assert np.allclose(y, mass_apply(u, k, msh), atol=1e-12)


def test_divergence_penalty_energy_against_an_independent_rule():
    # u^T A_D u = sum_e tau_e int_K (div u)^2, integrated with k+3 Gauss points
    k = 2
    rng = np.random.default_rng(5)
    msh = M.Mesh((2, 2, 1), (1.0, 1.5, 0.8))
    n = k + 1
    u = rng.standard_normal((3, msh.N, n ** 3))
    td = rng.uniform(0.5, 2.0, msh.N)
    AD = projection_apply(u, k, msh, td, np.zeros(msh.N)) - mass_apply(u, k, msh)
    lhs = float(np.sum(u * AD))
    nodes = basis.lgl_nodes(k)
    xg, wg = legendre.leggauss(k + 3)
    xg, wg = 0.5 * (xg + 1.0), 0.5 * wg
    L = basis.lagrange_values(nodes, xg)
    Ld = basis.lagrange_derivs(nodes, xg)
    h = msh.h
    rhs = 0.0
    for e in range(msh.N):
        div = 0.0
        for j in range(3):
            f = [L, L, L]
            f[j] = Ld
            U = u[j, e].reshape(n, n, n)                       # [c, b, a]
            vals = np.einsum("za,yb,xc,cba->zyx", f[0], f[1], f[2], U)  # [x pt, y pt, z pt]
            div = div + vals / h[j]
        wq = np.einsum("i,j,k->ijk", wg, wg, wg)
        rhs += td[e] * np.prod(h) * float(np.sum(wq * div ** 2))
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)


def test_operator_is_symmetric_positive_definite():
    k = 2
    rng = np.random.default_rng(8)
    msh = M.Mesh((3, 2, 2), (1.0, 1.0, 1.0))
    n3 = (k + 1) ** 3
    td, tc = rng.uniform(0.1, 1.0, msh.N), rng.uniform(0.1, 1.0, msh.N)
    u, v = rng.standard_normal((2, 3, msh.N, n3))
    pu, pv = projection_apply(u, k, msh, td, tc), projection_apply(v, k, msh, td, tc)
    assert abs(np.sum(v * pu) - np.sum(u * pv)) < 1e-12 * np.linalg.norm(pu) * np.linalg.norm(v)
    assert np.sum(u * pu) > 0


def test_continuity_penalty_energy_against_an_independent_rule():
    # u^T A_C u = sum over the faces (each once) of {tau_C} int_F (u^-_d - u^+_d)^2:
    # the two elements of a face contribute u^- (u^- - u^+) and u^+ (u^+ - u^-).
    # Traces from the Lagrange basis at xi_d = 0, 1, integrated with k+3 Gauss points.
    k = 3
    rng = np.random.default_rng(6)
    msh = M.Mesh((3, 2, 2), (1.2, 0.9, 1.5))
    n = k + 1
    u = rng.standard_normal((3, msh.N, n ** 3))
    tc = rng.uniform(0.5, 2.0, msh.N)
    AC = projection_apply(u, k, msh, np.zeros(msh.N), tc) - mass_apply(u, k, msh)
    lhs = float(np.sum(u * AC))
    nodes = basis.lgl_nodes(k)
    xg, wg = legendre.leggauss(k + 3)
    xg, wg = 0.5 * (xg + 1.0), 0.5 * wg
    L = basis.lagrange_values(nodes, xg)
    ends = [basis.lagrange_values(nodes, [0.0]), basis.lagrange_values(nodes, [1.0])]
    h = msh.h
    vol = float(np.prod(h))
    rhs = 0.0
    for d in range(3):
        up = msh.neighbor(d, 1)
        for e in range(msh.N):
            def trace(el, s):
                f = [L, L, L]
                f[d] = ends[s]
                U = u[d, el].reshape(n, n, n)                  # [c, b, a]
                return np.einsum("pa,qb,rc,cba->pqr", f[0], f[1], f[2], U).squeeze(axis=d)
            jump = trace(e, 1) - trace(up[e], 0)
            rhs += 0.5 * (tc[e] + tc[up[e]]) * (vol / h[d]) * float(np.sum(np.outer(wg, wg) * jump ** 2))
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)


def _dense(apply, shape):
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        A[:, i] = apply(e.reshape(shape)).ravel()
    return A


def test_mass_preconditioned_cg_solves_the_projection_and_helmholtz_equations():
    # the oracle's PCG with the inverse mass as preconditioner (Sec. 3.3)
    # against a dense direct solve of the assembled operators
    from oracle.mass import helmholtz_apply, inverse_mass_apply
    from oracle.solvers import pcg
    k = 1
    msh = M.Mesh((2, 2, 1), (1.0, 0.8, 0.6))
    rng = np.random.default_rng(9)
    td, tc = rng.uniform(0.1, 1.0, msh.N), rng.uniform(0.1, 1.0, msh.N)
    shape = (3, msh.N, (k + 1) ** 3)
    cases = [lambda v: projection_apply(v, k, msh, td, tc), lambda v: helmholtz_apply(v, k, msh, 5.0)]
    for apply in cases:
        b = rng.standard_normal(shape)
        A = _dense(apply, shape)
        x_direct = np.linalg.solve(A, b.ravel()).reshape(shape)
        x, info = pcg(apply, b, precond=lambda r: inverse_mass_apply(r, k, msh), rtol=1e-13, flexible=False)
        assert np.linalg.norm(x - x_direct) < 1e-10 * np.linalg.norm(x_direct)
        assert info["iterations"] < 60


def test_sampled_rows_equal_the_full_apply():
    k = 2
    rng = np.random.default_rng(11)
    msh = M.Mesh((3, 4, 2), (1.0, 2.0, 1.5))
    u = rng.standard_normal((3, msh.N, (k + 1) ** 3))
    td, tc = rng.uniform(0.1, 1.0, msh.N), rng.uniform(0.1, 1.0, msh.N)
    full = projection_apply(u, k, msh, td, tc)
    el = np.array([0, 5, 23, 7, 7])
    part = projection_apply(u, k, msh, td, tc, elems=el)
    # the same sums; a matrix product over fewer rows may round differently
    assert np.max(np.abs(part - full[:, el])) <= 1e-14 * np.max(np.abs(full))
