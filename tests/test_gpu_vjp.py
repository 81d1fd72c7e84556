"""GPU parity of dg_vjp_convective and the autograd wrappers.

Against the oracle's explicitly assembled Jacobian transpose on the 4^3
sub-mesh (k=4) and on small ragged meshes for every supported degree
(FP64 1e-12, FP32 1e-5 relative); at the full 32^3, k=4 size through
properties that hold at any size: central differences of the GPU forward
operator (step 1e-6), the Euler identity <J^T w, u> = 2 <w, R(u)> of the
2-homogeneous operator, and u = 0.  The Laplace backward equals its forward.
"""
import numpy as np
import pytest
import torch

from gpu_common import announce, rel_err, round_f32, to_dev
from oracle import basis, mesh as M
from oracle.convective import convective_vjp
from paper_1802_01439_amd import autograd, dgmf, inputs

pytestmark = pytest.mark.gpu


def _tgv(k, n_el, seed):
    msh = M.Mesh(n_el, (2 * np.pi,) * 3)
    return msh, inputs.tgv_plus_noise(basis.lgl_nodes(k), n_el, msh.length, seed=seed)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_config4_submesh_against_assembled_jacobian(dtype):
    k = 4
    msh, u = _tgv(k, (4, 4, 4), inputs.FIELD_SEED_BASE + 3)
    w = inputs.normal(u.shape, seed=inputs.FIELD_SEED_BASE + 3 + inputs.COTANGENT_OFFSET)
    if dtype == torch.float32:
        u, w = round_f32(u), round_f32(w)
    announce(f"vjp config4 4^3 k=4 {dtype}")
    d = dgmf.make_desc(k, 4)
    g = dgmf.vjp_convective(d, to_dev(u, dtype), to_dev(w, dtype)).double().cpu().numpy()
    ref = convective_vjp(u, w, k, msh)
    assert rel_err(g, ref) < (1e-12 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("k", list(range(1, 8)))
def test_low_degrees_fp64(k):
    # 27 elements: several workgroups of several elements and a ragged last one
    n_el = (3, 3, 3) if k <= 4 else (3, 2, 2)
    length = (2 * np.pi, 1.5, 2.5)
    msh = M.Mesh(n_el, length)
    u = inputs.uniform((3, msh.N, (k + 1) ** 3), seed=600 + k)
    w = inputs.uniform(u.shape, seed=700 + k)
    announce(f"vjp fp64 k={k} n_el={n_el}")
    d = dgmf.make_desc(k, n_el, length, lf_factor=0.7)
    g = dgmf.vjp_convective(d, to_dev(u), to_dev(w)).cpu().numpy()
    assert rel_err(g, convective_vjp(u, w, k, msh, lf_factor=0.7)) < 1e-12


@pytest.mark.parametrize("k", list(range(1, 8)))
def test_low_degrees_fp32(k):
    n_el = (3, 3, 3) if k <= 5 else (3, 2, 2)
    msh = M.Mesh(n_el, (2 * np.pi,) * 3)
    u = round_f32(inputs.uniform((3, msh.N, (k + 1) ** 3), seed=800 + k))
    w = round_f32(inputs.uniform(u.shape, seed=900 + k))
    announce(f"vjp fp32 k={k}")
    d = dgmf.make_desc(k, n_el)
    g = dgmf.vjp_convective(d, to_dev(u, torch.float32), to_dev(w, torch.float32)).double().cpu().numpy()
    assert rel_err(g, convective_vjp(u, w, k, msh)) < 1e-5


@pytest.mark.parametrize("k", [8, 9, 10, 11])
def test_high_degrees(k):
    """FP64 (where built) and FP32 against one oracle evaluation on inputs
    that FP32 holds exactly; 2^3 and 3x2x2 meshes (the assembled Jacobian of
    a 3^3 mesh at k = 11 takes minutes on the host)."""
    n_el = (3, 2, 2) if k <= 9 else (2, 2, 2)
    length = (2 * np.pi, 1.5, 2.5)
    msh = M.Mesh(n_el, length)
    u = round_f32(inputs.uniform((3, msh.N, (k + 1) ** 3), seed=620 + k))
    w = round_f32(inputs.uniform(u.shape, seed=720 + k))
    d = dgmf.make_desc(k, n_el, length, lf_factor=0.7)
    ref = convective_vjp(u, w, k, msh, lf_factor=0.7)
    if k <= dgmf.vjp_max_degree(torch.float64):
        announce(f"vjp fp64 k={k} n_el={n_el}")
        g = dgmf.vjp_convective(d, to_dev(u), to_dev(w)).cpu().numpy()
        assert rel_err(g, ref) < 1e-12
    announce(f"vjp fp32 k={k} n_el={n_el}")
    g = dgmf.vjp_convective(d, to_dev(u, torch.float32), to_dev(w, torch.float32)).double().cpu().numpy()
    assert rel_err(g, ref) < 1e-5


@pytest.mark.parametrize("k", [3, 7])
def test_input_alignment_fp32(k):
    """FP32 pencils of contiguous values are read in 16-byte loads when u and
    w are 16-byte aligned; inputs one value (4 bytes) off that take the plain
    loads and give the same result bit for bit; both match the oracle."""
    n_el = (3, 2, 2)
    msh = M.Mesh(n_el, (2 * np.pi,) * 3)
    u = round_f32(inputs.uniform((3, msh.N, (k + 1) ** 3), seed=1400 + k))
    w = round_f32(inputs.uniform(u.shape, seed=1500 + k))
    d = dgmf.make_desc(k, n_el)
    ua, wa = to_dev(u, torch.float32), to_dev(w, torch.float32)
    def shifted(x):
        base = torch.empty(x.numel() + 1, dtype=x.dtype, device=x.device)
        y = base[1:].view(x.shape)
        y.copy_(x)
        return y
    um, wm = shifted(ua), shifted(wa)
    assert ua.data_ptr() % 16 == 0 and um.data_ptr() % 16 != 0
    announce(f"vjp alignment fp32 k={k}")
    ga = dgmf.vjp_convective(d, ua, wa)
    gm = dgmf.vjp_convective(d, um, wm)
    assert torch.equal(ga, gm)
    assert rel_err(ga.double().cpu().numpy(), convective_vjp(u, w, k, msh)) < 1e-5


def test_exact_ties_follow_half_half_convention():
    k = 2
    msh = M.cube(2)
    n3 = (k + 1) ** 3
    u = np.zeros((3, msh.N, n3))
    u[0] = 0.5
    u[0, ::2] = -0.5
    u[1] = 0.25
    w = inputs.uniform(u.shape, seed=31)
    announce("vjp ties")
    g = dgmf.vjp_convective(dgmf.make_desc(k, 2), to_dev(u), to_dev(w)).cpu().numpy()
    assert rel_err(g, convective_vjp(u, w, k, msh)) < 1e-12


def test_full_size_properties():
    """32^3 elements, k=4 (12.3M DoFs): central differences (step 1e-6), the
    Euler identity, u = 0, FP32 against FP64.

    The LLF term max(|u-.n|, |u+.n|) is not differentiable: among the ~5e6
    face quadrature points a few lie within the step of a kink, where the
    difference quotient and the one-sided derivative differ by O(1).  The
    smooth part of the operator (lf_factor = 0) is therefore checked to 1e-7;
    with the dissipative term the kink points limit the agreement to ~1e-5.
    """
    k, N = 4, 32
    msh, u = _tgv(k, (N, N, N), inputs.FIELD_SEED_BASE + 3)
    w = inputs.normal(u.shape, seed=inputs.FIELD_SEED_BASE + 3 + inputs.COTANGENT_OFFSET)
    v = inputs.normal(u.shape, seed=inputs.FIELD_SEED_BASE + 3 + 2 * inputs.COTANGENT_OFFSET)
    ut, wt, vt = to_dev(u), to_dev(w), to_dev(v)
    eps = 1e-6
    for lf, tol in ((0.0, 1e-7), (1.0, 1e-4)):
        d = dgmf.make_desc(k, N, lf_factor=lf)
        announce(f"vjp full size 32^3 k=4 lf={lf}")
        g = dgmf.vjp_convective(d, ut, wt)
        R = dgmf.apply_convective(d, ut)
        fd = (dgmf.apply_convective(d, ut + eps * vt) - dgmf.apply_convective(d, ut - eps * vt)) / (2 * eps)
        lhs, rhs = (wt * fd).sum().item(), (g * vt).sum().item()
        assert abs(lhs - rhs) <= tol * abs(rhs), (lf, lhs, rhs)
        e1, e2 = (g * ut).sum().item(), 2 * (wt * R).sum().item()
        assert abs(e1 - e2) <= 1e-12 * (g * ut).abs().sum().item()
    z = dgmf.vjp_convective(d, torch.zeros_like(ut), wt)
    assert z.abs().max().item() == 0.0
    g32 = dgmf.vjp_convective(d, ut.float(), wt.float()).double()
    assert ((g32 - g).norm() / g.norm()).item() < 1e-5


def test_autograd_convective_and_laplace():
    k, N = 2, 2
    msh, u = _tgv(k, (N, N, N), 41)
    ut = to_dev(u).requires_grad_(True)
    announce("autograd gradcheck convective")
    f = lambda x: autograd.convective(x, k, N)
    assert torch.autograd.gradcheck(f, (ut,), eps=1e-6, atol=1e-7, rtol=1e-5)
    p = to_dev(inputs.uniform((N ** 3, 27), seed=42)).requires_grad_(True)
    y = autograd.laplace(p, k, N)
    gout = to_dev(inputs.uniform((N ** 3, 27), seed=43))
    (gp,) = torch.autograd.grad(y, p, gout)
    assert torch.allclose(gp, dgmf.apply_laplace(dgmf.make_desc(k, N), gout), rtol=0, atol=0)


def test_unsupported_degree_and_alias():
    if dgmf.vjp_max_degree(torch.float64) < 11:
        d = dgmf.make_desc(11, 2)
        u = torch.zeros((3, 8, 12 ** 3), dtype=torch.float64, device="cuda")
        with pytest.raises(dgmf.DgError) as ei:
            dgmf.vjp_convective(d, u, u)
        assert ei.value.code == dgmf.DG_ERR_UNSUPPORTED
    d = dgmf.make_desc(2, 2)
    u = torch.zeros((3, 8, 27), dtype=torch.float64, device="cuda")
    with pytest.raises(dgmf.DgError) as ei:
        dgmf.vjp_convective(d, u, u.clone(), out=u)
    assert ei.value.code == dgmf.DG_ERR_ALIAS
