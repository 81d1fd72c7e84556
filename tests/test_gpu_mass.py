"""GPU parity of dg_apply_inverse_mass against the CPU oracle (through the C ABI).

FP64 within 1e-12 relative (2-norm), FP32 within 1e-5 relative against the
oracle applied to the FP32-rounded input.  Meshes span several workgroup
batches with a ragged last batch; anisotropic boxes, three components, in
place; the degree-sweep full size on sampled elements.
"""
import numpy as np
import pytest
import torch

from gpu_common import announce, rel_err, round_f32, to_dev
from oracle import mesh as M
from oracle.mass import inverse_mass_apply, mass_apply
from paper_1802_01439_amd import dgmf, inputs

pytestmark = pytest.mark.gpu


def _mesh_for(k):
    # E = floor(256/n^2) element blocks per workgroup; N_el > 2E and not a multiple of E
    E = max(1, 256 // (k + 1) ** 2)
    nx = 2 * E + 3
    return (nx, 2, 1) if nx < 40 else (nx, 1, 1)


@pytest.mark.parametrize("k", list(range(1, 12)))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_inverse_mass_parity(k, dtype):
    n_el = _mesh_for(k)
    length = (1.0 * n_el[0], 0.7 * n_el[1], 1.3 * n_el[2])
    msh = M.Mesh(n_el, length)
    u = inputs.uniform((msh.N, (k + 1) ** 3), seed=700 + k)
    if dtype == torch.float32:
        u = round_f32(u)
    announce(f"inverse mass k={k} {dtype} n_el={n_el}")
    d = dgmf.make_desc(k, n_el, length)
    y = dgmf.apply_inverse_mass(d, to_dev(u, dtype)).double().cpu().numpy()
    assert rel_err(y, inverse_mass_apply(u, k, msh)) < (1e-12 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("k", [2, 5, 8])
def test_three_components_in_place_and_mass_round_trip(k):
    n_el = (5, 3, 2)
    msh = M.Mesh(n_el, (2 * np.pi,) * 3)
    u = inputs.normal((3, msh.N, (k + 1) ** 3), seed=720 + k)
    d = dgmf.make_desc(k, n_el, n_comp=3)
    announce(f"inverse mass 3 components in place k={k}")
    t = to_dev(u)
    dgmf.apply_inverse_mass(d, t, out=t)
    torch.cuda.synchronize()
    y = t.cpu().numpy()
    assert rel_err(y, inverse_mass_apply(u, k, msh)) < 1e-12
    # M (M^-1 b) = b with the oracle's mass
    assert rel_err(mass_apply(y, k, msh), u) < 1e-12


@pytest.mark.parametrize("k", [3, 7])
def test_full_size_sampled(k):
    N = int(round(256.0 / (k + 1)))
    msh = M.cube(N)
    u = inputs.uniform((msh.N, (k + 1) ** 3), seed=102 + 10 * k)
    announce(f"inverse mass full size k={k} N={N}")
    y = dgmf.apply_inverse_mass(dgmf.make_desc(k, N), to_dev(u)).cpu().numpy()
    sample = np.arange(0, msh.N, 1009)
    assert rel_err(y[sample], inverse_mass_apply(u, k, msh, elems=sample)) < 1e-12


def test_unsupported_and_alias():
    d = dgmf.make_desc(3, 4, n_q=3)
    u = to_dev(inputs.uniform((64, 64), seed=1))
    with pytest.raises(dgmf.DgError) as ei:
        dgmf.apply_inverse_mass(d, u)
    assert ei.value.code == dgmf.DG_ERR_UNSUPPORTED
    d = dgmf.make_desc(3, 4)
    big = to_dev(inputs.uniform((65, 64), seed=2))
    with pytest.raises(dgmf.DgError) as ei:
        dgmf.apply_inverse_mass(d, big[:64], out=big[1:])
    assert ei.value.code == dgmf.DG_ERR_ALIAS


@pytest.mark.parametrize("k,dtype,ncomp", [(2, torch.float64, 1), (4, torch.float64, 3), (7, torch.float64, 1),
                                           (11, torch.float64, 1), (3, torch.float32, 1), (8, torch.float32, 3)])
def test_helmholtz_parity(k, dtype, ncomp):
    from oracle.mass import helmholtz_apply
    E = max(1, 256 // (k + 1) ** 2)
    n_el = (2 * E + 3, 2, 2) if 2 * E + 3 < 30 else (2 * E + 3, 1, 2)
    length = (0.9 * n_el[0], 1.1 * n_el[1], 1.0 * n_el[2])
    msh = M.Mesh(n_el, length)
    shape = (msh.N, (k + 1) ** 3) if ncomp == 1 else (3, msh.N, (k + 1) ** 3)
    u = inputs.uniform(shape, seed=740 + k)
    if dtype == torch.float32:
        u = round_f32(u)
    mass_factor, nu = 37.5, 0.02          # gamma_0 / dt and nu of a viscous step
    announce(f"helmholtz k={k} {dtype} ncomp={ncomp}")
    d = dgmf.make_desc(k, n_el, length, scale=nu, n_comp=ncomp)
    y = dgmf.apply_helmholtz(d, to_dev(u, dtype), mass_factor).double().cpu().numpy()
    ref = helmholtz_apply(u, k, msh, mass_factor, scale=nu)
    assert rel_err(y, ref) < (1e-12 if dtype == torch.float64 else 1e-5)


def test_helmholtz_without_mass_is_the_laplace_and_bad_factor():
    k, n_el = 3, (5, 4, 3)
    d = dgmf.make_desc(k, n_el, scale=0.5)
    u = to_dev(inputs.uniform((60, 64), seed=9))
    announce("helmholtz mass_factor 0")
    a = dgmf.apply_helmholtz(d, u, 0.0)
    b = dgmf.apply_laplace(d, u)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    with pytest.raises(dgmf.DgError) as ei:
        dgmf.apply_helmholtz(d, u, -1.0)
    assert ei.value.code == dgmf.DG_ERR_INVALID_ARG
