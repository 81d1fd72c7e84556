"""GPU parity of dg_apply_gradient (central-flux pressure gradient g_h)
against the CPU oracle, through the C ABI.

FP64 within 1e-12 relative (2-norm), FP32 within 1e-5 relative against the
oracle applied to the FP32-rounded input.  Every degree on meshes that span
several workgroup batches with a ragged last batch, anisotropic boxes,
one-element directions, over-integration, the degree-sweep full size on
sampled elements, and -D^T adjointness with the GPU divergence at 16^3.
"""
import numpy as np
import pytest
import torch

from gpu_common import announce, rel_err, round_f32, to_dev
from oracle import mesh as M
from oracle.gradient import gradient_apply
from paper_1802_01439_amd import dgmf, inputs

pytestmark = pytest.mark.gpu


def _mesh_for(k):
    E = max(1, 256 // (k + 1) ** 2)
    nx = 2 * E + 3
    return (nx, 2, 1) if nx < 40 else (nx, 1, 1)


@pytest.mark.parametrize("k", list(range(1, 12)))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_gradient_parity(k, dtype):
    n_el = _mesh_for(k)
    msh = M.Mesh(n_el, (1.0 * n_el[0], 0.7 * n_el[1], 1.3 * n_el[2]))
    p = inputs.uniform((msh.N, (k + 1) ** 3), seed=960 + k)
    if dtype == torch.float32:
        p = round_f32(p)
    announce(f"gradient k={k} {dtype} n_el={n_el}")
    d = dgmf.make_desc(k, n_el, tuple(msh.length))
    y = dgmf.apply_gradient(d, to_dev(p, dtype)).double().cpu().numpy()
    assert rel_err(y, gradient_apply(p, k, msh)) < (1e-12 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("k,n_el,n_q", [(2, (1, 3, 2), 0), (4, (1, 1, 1), 0), (5, (3, 2, 2), 9)])
def test_gradient_small_meshes_and_over_integration(k, n_el, n_q):
    msh = M.Mesh(n_el, (0.9, 1.2, 1.0))
    p = inputs.normal((msh.N, (k + 1) ** 3), seed=975 + k)
    announce(f"gradient k={k} n_el={n_el} n_q={n_q}")
    d = dgmf.make_desc(k, n_el, tuple(msh.length), n_q=n_q)
    y = dgmf.apply_gradient(d, to_dev(p)).cpu().numpy()
    assert rel_err(y, gradient_apply(p, k, msh, n_q=n_q)) < 1e-12


@pytest.mark.parametrize("k", [3, 7])
def test_gradient_full_size_sampled(k):
    N = int(round(256.0 / (k + 1)))
    msh = M.cube(N)
    p = inputs.uniform((msh.N, (k + 1) ** 3), seed=985 + k)
    announce(f"gradient full size k={k} N={N}")
    y = dgmf.apply_gradient(dgmf.make_desc(k, N), to_dev(p)).cpu().numpy()
    rng = np.random.default_rng(986 + k)
    el = np.concatenate([[0, msh.N - 1], rng.choice(msh.N, 62, replace=False)])
    assert rel_err(y[:, el], gradient_apply(p, k, msh, elems=el)) < 1e-12


@pytest.mark.parametrize("k", [2, 6])
def test_gradient_is_minus_divergence_transpose(k):
    N = 16
    d = dgmf.make_desc(k, N)
    p = to_dev(inputs.normal((N ** 3, (k + 1) ** 3), seed=990 + k))
    v = to_dev(inputs.normal((3, N ** 3, (k + 1) ** 3), seed=991 + k))
    announce(f"gradient adjointness k={k} 16^3")
    a = float(torch.vdot(v.flatten(), dgmf.apply_gradient(d, p).flatten()))
    b = float(torch.vdot(p.flatten(), dgmf.apply_divergence(d, v).flatten()))
    assert abs(a + b) <= 1e-11 * abs(a)


def test_gradient_rejects_aliasing():
    d = dgmf.make_desc(2, 3)
    y = torch.zeros(3, 27, 27, dtype=torch.float64, device="cuda")
    with pytest.raises(dgmf.DgError):
        dgmf.apply_gradient(d, y[0], out=y)
