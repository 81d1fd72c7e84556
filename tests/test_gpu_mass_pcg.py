"""GPU parity of dg_mass_pcg_solve (CG preconditioned with the inverse mass
matrix for the projection and Helmholtz equations) against the oracle's PCG
with the same preconditioner, through the C ABI.

Both solve to rtol = 1e-12; the solutions agree within 1e-9 relative
(2-norm) and the iteration counts within one; the true residual of the GPU
solution is at most 1e-11.  Ragged batches, anisotropic boxes, random
per-element penalty parameters, one and three components, a non-zero initial
guess, b = 0, the iteration limit and argument errors.
"""
import numpy as np
import pytest
import torch

from gpu_common import announce, rel_err, to_dev
from oracle import mesh as M
from oracle.mass import helmholtz_apply, inverse_mass_apply
from oracle.projection import projection_apply
from oracle.solvers import pcg
from paper_1802_01439_amd import dgmf, inputs

pytestmark = pytest.mark.gpu


def _projection_case(k, n_el, seed):
    msh = M.Mesh(n_el, (1.0 * n_el[0], 0.7 * n_el[1], 1.3 * n_el[2]))
    h2 = float(np.min(msh.h)) ** 2
    td = inputs.uniform((msh.N,), seed=seed + 1, lo=0.1, hi=1.0) * h2
    tc = inputs.uniform((msh.N,), seed=seed + 2, lo=0.1, hi=1.0) * h2
    b = inputs.uniform((3, msh.N, (k + 1) ** 3), seed=seed)
    return msh, td, tc, b


def _oracle(apply, b, k, msh):
    return pcg(apply, b, precond=lambda r: inverse_mass_apply(r, k, msh), rtol=1e-12, flexible=False)


@pytest.mark.parametrize("k,n_el", [(2, (11, 2, 1)), (4, (5, 3, 2)), (7, (3, 2, 2))])
def test_projection_solve_parity(k, n_el):
    msh, td, tc, b = _projection_case(k, n_el, 900 + k)
    announce(f"mass-preconditioned CG, projection, k={k} n_el={n_el}")
    d = dgmf.make_desc(k, n_el, tuple(msh.length), n_comp=3)
    x, rep, rc = dgmf.mass_pcg_solve(d, dgmf.DG_OP_PROJECTION, to_dev(b), tau_d=to_dev(td), tau_c=to_dev(tc),
                                     rtol=1e-12)
    assert rc == dgmf.DG_OK
    xr, info = _oracle(lambda v: projection_apply(v, k, msh, td, tc), b, k, msh)
    assert rel_err(x.cpu().numpy(), xr) < 1e-9
    assert abs(rep["iterations"] - info["iterations"]) <= 1
    assert rep["true_rel_res"] < 1e-11
    # initial and true residual, plus at most 7 no-op iterations that end a batch
    assert rep["iterations"] + 2 <= rep["matvec_f64"] <= rep["iterations"] + 9


@pytest.mark.parametrize("k,n_comp", [(3, 1), (6, 3)])
def test_helmholtz_solve_parity(k, n_comp):
    n_el = (7, 3, 2)
    msh = M.Mesh(n_el, (2.0, 1.1, 0.9))
    shape = (msh.N, (k + 1) ** 3) if n_comp == 1 else (3, msh.N, (k + 1) ** 3)
    b = inputs.uniform(shape, seed=920 + k)
    mass_factor = 20.0
    announce(f"mass-preconditioned CG, Helmholtz, k={k} n_comp={n_comp}")
    d = dgmf.make_desc(k, n_el, tuple(msh.length), n_comp=n_comp)
    x, rep, rc = dgmf.mass_pcg_solve(d, dgmf.DG_OP_HELMHOLTZ, to_dev(b), mass_factor=mass_factor, rtol=1e-12)
    assert rc == dgmf.DG_OK
    xr, info = _oracle(lambda v: helmholtz_apply(v, k, msh, mass_factor), b, k, msh)
    assert rel_err(x.cpu().numpy(), xr) < 1e-9
    assert abs(rep["iterations"] - info["iterations"]) <= 1
    assert rep["true_rel_res"] < 1e-11


def test_initial_guess_zero_rhs_and_iteration_limit():
    k, n_el = 3, (4, 3, 2)
    msh, td, tc, b = _projection_case(k, n_el, 940)
    d = dgmf.make_desc(k, n_el, tuple(msh.length), n_comp=3)
    tdd, tcd = to_dev(td), to_dev(tc)
    announce("mass-preconditioned CG: initial guess, b = 0, iteration limit")
    x0, _, rc0 = dgmf.mass_pcg_solve(d, dgmf.DG_OP_PROJECTION, to_dev(b), tau_d=tdd, tau_c=tcd, rtol=1e-12)
    assert rc0 == dgmf.DG_OK
    guess = to_dev(inputs.normal(b.shape, seed=941))
    x1, rep1, rc1 = dgmf.mass_pcg_solve(d, dgmf.DG_OP_PROJECTION, to_dev(b), x=guess, tau_d=tdd, tau_c=tcd,
                                        rtol=1e-12)
    assert rc1 == dgmf.DG_OK
    assert rel_err(x1.cpu().numpy(), x0.cpu().numpy()) < 1e-9
    z, rep0, rcz = dgmf.mass_pcg_solve(d, dgmf.DG_OP_PROJECTION, torch.zeros_like(x0),
                                       x=to_dev(inputs.normal(b.shape, seed=942)), tau_d=tdd, tau_c=tcd)
    assert rcz == dgmf.DG_OK and float(z.abs().max()) == 0.0 and rep0["iterations"] == 0
    _, repl, rcl = dgmf.mass_pcg_solve(d, dgmf.DG_OP_PROJECTION, to_dev(b), tau_d=tdd, tau_c=tcd, rtol=1e-14,
                                       max_iter=1)
    assert rcl == dgmf.DG_NOT_CONVERGED and repl["iterations"] == 1


def test_argument_errors():
    k = 2
    d1 = dgmf.make_desc(k, 3)
    d3 = dgmf.make_desc(k, 3, n_comp=3)
    b1 = torch.ones(27, 27, dtype=torch.float64, device="cuda")
    b3 = torch.ones(3, 27, 27, dtype=torch.float64, device="cuda")
    t = torch.ones(27, dtype=torch.float64, device="cuda")
    with pytest.raises(dgmf.DgError):   # mass_factor must be > 0
        dgmf.mass_pcg_solve(d1, dgmf.DG_OP_HELMHOLTZ, b1, mass_factor=0.0)
    with pytest.raises(dgmf.DgError):   # bad op
        dgmf.mass_pcg_solve(d1, 7, b1, mass_factor=1.0)
    with pytest.raises(dgmf.DgError):   # x aliases b
        dgmf.mass_pcg_solve(d3, dgmf.DG_OP_PROJECTION, b3, x=b3, tau_d=t, tau_c=t)


def test_projection_solve_at_the_benchmark_size():
    # k = 5, 16^3, TGV + noise velocity, tau from the CFL time step (Cr = 0.2,
    # r = 1.5), rhs M u: the GPU solution has a small residual under the
    # oracle's operator
    from oracle import basis
    from oracle.mass import mass_apply
    k, N = 5, 16
    L = 2 * np.pi
    h = L / N
    dt = 0.2 / k ** 1.5 * h
    msh = M.cube(N)
    u = inputs.tgv_plus_noise(basis.lgl_nodes(k), (N, N, N), (L,) * 3, seed=inputs.FIELD_SEED_BASE + 2)
    umag = np.sqrt((u ** 2).sum(axis=0)).mean(axis=1)
    td, tc = umag * h / (k + 1) * dt, umag * dt
    b = mass_apply(u, k, msh)
    announce("mass-preconditioned CG, projection, k=5 16^3")
    d = dgmf.make_desc(k, N, n_comp=3)
    x, rep, rc = dgmf.mass_pcg_solve(d, dgmf.DG_OP_PROJECTION, to_dev(b), tau_d=to_dev(td), tau_c=to_dev(tc),
                                     rtol=1e-10)
    assert rc == dgmf.DG_OK and rep["iterations"] < 60
    res = b - projection_apply(x.cpu().numpy(), k, msh, td, tc)
    assert np.linalg.norm(res) < 1e-9 * np.linalg.norm(b)
