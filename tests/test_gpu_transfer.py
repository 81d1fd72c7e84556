"""GPU parity of dg_prolongate and dg_restrict (h-multigrid level transfers)
against the CPU oracle, through the C ABI.

FP64 within 1e-12 relative (2-norm), FP32 within 1e-5 relative against the
oracle applied to the FP32-rounded input.  Every degree, coarse meshes whose
fine and coarse element counts leave a ragged last workgroup, one and three
components, one-element directions, both launch forms of the prolongation
(one child per workgroup below 1024 workgroups, the loop over the children
above), and the adjointness of the two GPU kernels at a larger size.
"""
import numpy as np
import pytest
import torch

from gpu_common import announce, rel_err, round_f32, to_dev
from oracle import mesh as M
from oracle.transfer import prolongate, restrict
from paper_1802_01439_amd import dgmf, inputs

pytestmark = pytest.mark.gpu


def _coarse_for(k):
    E = max(1, 256 // (k + 1) ** 2)
    nx = E + 3          # 8 nx ny fine elements: several ragged batches either way
    return (nx, 2, 1) if nx < 20 else (nx, 1, 1)


@pytest.mark.parametrize("k", list(range(1, 12)))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_transfer_parity(k, dtype):
    n_el = _coarse_for(k)
    coarse = M.Mesh(n_el, (1.0, 0.8, 1.2))
    n3 = (k + 1) ** 3
    uc = inputs.uniform((coarse.N, n3), seed=1000 + k)
    rf = inputs.uniform((8 * coarse.N, n3), seed=1020 + k)
    if dtype == torch.float32:
        uc, rf = round_f32(uc), round_f32(rf)
    d = dgmf.make_desc(k, n_el, tuple(coarse.length))
    announce(f"transfer k={k} {dtype} coarse={n_el}")
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    uf = dgmf.prolongate(d, to_dev(uc, dtype)).double().cpu().numpy()
    assert rel_err(uf, prolongate(uc, k, coarse)) < tol
    rc = dgmf.restrict(d, to_dev(rf, dtype)).double().cpu().numpy()
    assert rel_err(rc, restrict(rf, k, coarse)) < tol


@pytest.mark.parametrize("k,n_el", [(2, (1, 1, 1)), (3, (2, 1, 3)), (6, (1, 2, 1))])
def test_transfer_three_components_small_meshes(k, n_el):
    coarse = M.Mesh(n_el, (1.0, 1.0, 1.0))
    n3 = (k + 1) ** 3
    uc = inputs.normal((3, coarse.N, n3), seed=1040 + k)
    rf = inputs.normal((3, 8 * coarse.N, n3), seed=1041 + k)
    d = dgmf.make_desc(k, n_el, n_comp=3)
    announce(f"transfer 3 components k={k} coarse={n_el}")
    assert rel_err(dgmf.prolongate(d, to_dev(uc)).cpu().numpy(), prolongate(uc, k, coarse)) < 1e-12
    assert rel_err(dgmf.restrict(d, to_dev(rf)).cpu().numpy(), restrict(rf, k, coarse)) < 1e-12


@pytest.mark.parametrize("k", [3, 7])
def test_transfer_adjoint_at_larger_size(k):
    N = 12
    d = dgmf.make_desc(k, N)
    n3 = (k + 1) ** 3
    u = to_dev(inputs.normal((N ** 3, n3), seed=1050 + k))
    r = to_dev(inputs.normal((8 * N ** 3, n3), seed=1051 + k))
    announce(f"transfer adjointness k={k} coarse {N}^3")
    a = float(torch.vdot(dgmf.prolongate(d, u).flatten(), r.flatten()))
    b = float(torch.vdot(u.flatten(), dgmf.restrict(d, r).flatten()))
    assert abs(a - b) <= 1e-12 * abs(a) * 10


@pytest.mark.parametrize("k,n_el,n_comp,dtype", [(2, (24, 24, 17), 3, torch.float64), (2, (24, 24, 17), 3, torch.float32),
                                                 (7, (16, 16, 16), 1, torch.float64)])
def test_transfer_parity_serial_children(k, n_el, n_comp, dtype):
    """Meshes whose launch has at least 1024 workgroups (batches x components),
    where the prolongation loops over the eight children inside each
    workgroup; the smaller meshes above take one child per workgroup."""
    E = max(1, 256 // (k + 1) ** 2)
    nc = n_el[0] * n_el[1] * n_el[2]
    assert (nc + E - 1) // E * n_comp >= 1024
    coarse = M.Mesh(n_el, (1.0, 1.0, 1.0))
    n3 = (k + 1) ** 3
    lead = (n_comp,) if n_comp > 1 else ()
    uc = inputs.uniform(lead + (coarse.N, n3), seed=1060 + k)
    rf = inputs.uniform(lead + (8 * coarse.N, n3), seed=1061 + k)
    if dtype == torch.float32:
        uc, rf = round_f32(uc), round_f32(rf)
    d = dgmf.make_desc(k, n_el, n_comp=n_comp)
    announce(f"transfer k={k} {dtype} coarse={n_el} n_comp={n_comp}")
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    uf = dgmf.prolongate(d, to_dev(uc, dtype)).double().cpu().numpy()
    assert rel_err(uf, prolongate(uc, k, coarse)) < tol
    rc = dgmf.restrict(d, to_dev(rf, dtype)).double().cpu().numpy()
    assert rel_err(rc, restrict(rf, k, coarse)) < tol
