"""GPU parity of the dual-splitting pieces through the C ABI: the mixed-order
divergence and gradient (velocity degree k, pressure k-1; FP64 within 1e-12,
FP32 within 1e-5 against the oracle on the FP32-rounded input), the
Taylor-Green diagnostics, and one BDF1 step followed by one BDF2 step against
the oracle's step (all solves to tight tolerances), plus a constant state
and the argument checks."""
import numpy as np
import pytest
import torch

from gpu_common import announce, rel_err, round_f32, to_dev
from oracle import basis, mesh as M
from oracle.dual_splitting import dual_splitting_step, tgv_diagnostics
from oracle.mixed import mixed_divergence_apply, mixed_gradient_apply
from paper_1802_01439_amd import dgmf, inputs

pytestmark = pytest.mark.gpu


def _mesh_for(k):
    # several workgroups (E = floor(256/(k+1)^2) elements each) and a ragged last one
    return (3, 4, 3) if k <= 4 else (3, 2, 3)


@pytest.mark.parametrize("k", list(range(2, 12)))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_mixed_divergence_and_gradient(k, dtype):
    n_el = _mesh_for(k)
    length = (2 * np.pi, 2.5, 1.5)
    msh = M.Mesh(n_el, length)
    u = inputs.uniform((3, msh.N, (k + 1) ** 3), seed=1300 + k)
    p = inputs.uniform((msh.N, k ** 3), seed=1350 + k)
    if dtype == torch.float32:
        u, p = round_f32(u), round_f32(p)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    d = dgmf.make_desc(k, n_el, length)
    announce(f"mixed divergence k={k} {dtype}")
    b = dgmf.apply_divergence_mixed(d, to_dev(u, dtype)).double().cpu().numpy()
    assert rel_err(b, mixed_divergence_apply(u, k, msh)) < tol
    announce(f"mixed gradient k={k} {dtype}")
    y = dgmf.apply_gradient_mixed(d, to_dev(p, dtype)).double().cpu().numpy()
    assert rel_err(y, mixed_gradient_apply(p, k, msh)) < tol


def test_mixed_operators_one_element_per_direction():
    k, n_el = 3, (1, 2, 1)
    msh = M.Mesh(n_el, (1.0, 2.0, 3.0))
    u = inputs.uniform((3, msh.N, 64), seed=1401)
    p = inputs.uniform((msh.N, 27), seed=1402)
    d = dgmf.make_desc(k, n_el, msh.length)
    announce("mixed operators, one element per direction")
    assert rel_err(dgmf.apply_divergence_mixed(d, to_dev(u)).cpu().numpy(), mixed_divergence_apply(u, k, msh)) < 1e-12
    assert rel_err(dgmf.apply_gradient_mixed(d, to_dev(p)).cpu().numpy(), mixed_gradient_apply(p, k, msh)) < 1e-12


@pytest.mark.parametrize("k,N", [(2, 3), (3, 4), (7, 2), (11, 2)])
def test_diagnostics(k, N):
    msh = M.Mesh((N, N + 1, N), (2 * np.pi, 2 * np.pi, 3.0))
    u = inputs.tgv_plus_noise(basis.lgl_nodes(k), msh.n_el, msh.length, seed=1450 + k, noise_std=0.1)
    announce(f"diagnostics k={k}")
    ek, eps = dgmf.tgv_diagnostics(dgmf.make_desc(k, msh.n_el, msh.length), to_dev(u), 0.01)
    rk, re = tgv_diagnostics(u, k, msh, 0.01)
    assert abs(ek - rk) < 1e-12 * abs(rk) and abs(eps - re) < 1e-12 * abs(re)


@pytest.mark.parametrize("pc", [dgmf.DG_STEP_PC_CHEB_F32, dgmf.DG_STEP_PC_GMG_F32])
@pytest.mark.parametrize("k,N", [(3, 3), (5, 2), (2, 4), (2, 8)])
def test_bdf1_then_bdf2_step_against_oracle(k, N, pc):
    """Taylor-Green + noise velocity, dt from the CFL condition (Cr = 0.2),
    nu = 0.01; the GPU solves to 1e-12 (pressure CG with the Chebyshev or the
    V-cycle preconditioner: 1, 1, 2 and 3 levels on these meshes), the
    oracle's to 1e-13 (pressure: exact)."""
    msh = M.cube(N)
    d = dgmf.make_desc(k, N)
    h = 2 * np.pi / N
    dt, nu = 0.2 / k ** 1.5 * h, 0.01
    u0 = inputs.tgv_plus_noise(basis.lgl_nodes(k), msh.n_el, msh.length, seed=1500 + k, noise_std=0.05)
    announce(f"step BDF1 k={k} N={N} pc={pc}")
    u1, p1, rep1, rc1 = dgmf.dual_splitting_step(d, to_dev(u0), dt=dt, nu=nu, order=1, rtol=1e-12,
                                                 atol_pressure=0.0, pressure_precond=pc)
    assert rc1 == dgmf.DG_OK, rep1
    r1 = dual_splitting_step([u0], k, msh, dt, nu, order=1)
    assert rel_err(u1.cpu().numpy(), r1["u"]) < 1e-9
    pg = p1.cpu().numpy()
    assert rel_err(pg - pg.mean(), r1["p"]) < 1e-8
    announce(f"step BDF2 k={k} N={N} pc={pc}")
    u2, p2, rep2, rc2 = dgmf.dual_splitting_step(d, u1, to_dev(u0), p=p1.clone(), dt=dt, nu=nu, order=2,
                                                 rtol=1e-12, atol_pressure=0.0, pressure_precond=pc)
    assert rc2 == dgmf.DG_OK, rep2
    r2 = dual_splitting_step([r1["u"], u0], k, msh, dt, nu, order=2)
    assert rel_err(u2.cpu().numpy(), r2["u"]) < 1e-8
    pg = p2.cpu().numpy()
    assert rel_err(pg - pg.mean(), r2["p"]) < 1e-7
    ek, eps = tgv_diagnostics(r2["u"], k, msh, nu)
    assert abs(rep2["kinetic_energy"] - ek) < 1e-9 * ek and abs(rep2["dissipation"] - eps) < 1e-8 * eps
    assert rep2["it_pressure"] > 0 and rep2["it_projection"] > 0 and rep2["it_viscous"] > 0


def test_step_keeps_a_constant_state():
    k, N = 4, 3
    d = dgmf.make_desc(k, N)
    c = torch.ones((3, N ** 3, (k + 1) ** 3), dtype=torch.float64, device="cuda")
    c *= torch.tensor([0.3, -0.7, 1.1], dtype=torch.float64, device="cuda")[:, None, None]
    announce("step constant state")
    u1, p1, rep, rc = dgmf.dual_splitting_step(d, c, c.clone(), dt=0.05, nu=0.01, order=2, rtol=1e-10)
    # the pressure right-hand side is rounding noise: the absolute tolerance stops its solve at once
    assert rc == dgmf.DG_OK, rep
    assert (u1 - c).abs().max().item() < 1e-12 and p1.abs().max().item() < 1e-12


def test_step_argument_errors():
    k, N = 3, 2
    d = dgmf.make_desc(k, N)
    u = torch.zeros((3, N ** 3, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        dgmf.dual_splitting_step(d, u, order=2)
    with pytest.raises(dgmf.DgError) as ei:
        dgmf.dual_splitting_step(d, u, dt=-1.0, order=1)
    assert ei.value.code == dgmf.DG_ERR_INVALID_ARG
    with pytest.raises(dgmf.DgError) as ei:
        dgmf.dual_splitting_step(d, u, u, out=u, order=2)
    assert ei.value.code == dgmf.DG_ERR_ALIAS
    with pytest.raises(dgmf.DgError) as ei:
        dgmf.dual_splitting_step(d, u, order=1, pressure_precond=7)
    assert ei.value.code == dgmf.DG_ERR_INVALID_ARG
    d1 = dgmf.make_desc(1, N)
    with pytest.raises(dgmf.DgError) as ei:
        dgmf.apply_divergence_mixed(d1, torch.zeros((3, N ** 3, 8), dtype=torch.float64, device="cuda"))
    assert ei.value.code == dgmf.DG_ERR_UNSUPPORTED


@pytest.mark.parametrize("pc", [dgmf.DG_STEP_PC_GMG_F32, dgmf.DG_STEP_PC_CHEB_F32])
def test_step_with_kept_convective_term_is_bit_identical(pc):
    """dg_dual_splitting_step_conv: three steps (BDF1, then BDF2 twice) that
    hand C(u_n) to the next step give bit-for-bit the steps of
    dg_dual_splitting_step, which recompute C(u_nm1)."""
    k, N = 5, 4
    msh = M.Mesh((N, N, N), (2 * np.pi,) * 3)
    u0 = to_dev(inputs.tgv_plus_noise(basis.lgl_nodes(k), msh.n_el, msh.length, seed=1560 + k, noise_std=0.05))
    d = dgmf.make_desc(k, N)
    announce(f"step with kept convective term k={k} N={N} pc={pc}")
    kw = dict(dt=2e-2, nu=1 / 1600, pressure_precond=pc)
    ref = [u0]
    p = None
    for n in range(3):
        u, p, _, rc = dgmf.dual_splitting_step(d, ref[-1], ref[-2] if n else None, p=p, order=2 if n else 1, **kw)
        assert rc == dgmf.DG_OK
        ref.append(u.clone())
        p = p.clone()
    pref = p
    got = [u0]
    p = None
    conv = [torch.empty_like(u0), torch.empty_like(u0)]
    for n in range(3):
        u, p, _, rc = dgmf.dual_splitting_step(d, got[-1], got[-2] if n else None, p=p, order=2 if n else 1,
                                               conv_prev=conv[(n + 1) % 2] if n else None, conv_out=conv[n % 2], **kw)
        assert rc == dgmf.DG_OK
        got.append(u.clone())
        p = p.clone()
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    assert torch.equal(pref, p)
    # the kept term is C(u_n) of the last step's input
    c = dgmf.apply_convective(d, got[-2])
    assert torch.equal(c, conv[2 % 2])
    with pytest.raises(dgmf.DgError) as ei:
        dgmf.dual_splitting_step(d, got[-1], got[-2], p=p, order=2, conv_prev=conv[0], conv_out=conv[0], **kw)
    assert ei.value.code == dgmf.DG_ERR_ALIAS
