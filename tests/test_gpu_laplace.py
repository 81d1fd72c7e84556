"""GPU parity of dg_apply_laplace against the CPU oracle (through the C ABI).

FP64 within 1e-12 relative (2-norm), FP32 within 1e-5 relative against the
oracle applied to the FP32-rounded input.  Meshes span several workgroup
batches with a ragged last batch; edge cases: one and two elements per
direction, anisotropic boxes, three components, penalty and scale factors.
The full-size case (degree sweep size, k=3, 64^3) is checked on sampled
elements, plus invariants that hold at any size.
"""
import numpy as np
import pytest
import torch

from gpu_common import announce, rel_err, round_f32, to_dev
from oracle import mesh as M
from oracle.laplace import laplace_apply, laplace_diagonal
from paper_1802_01439_amd import dgmf, inputs

pytestmark = pytest.mark.gpu


def _run(k, n_el, length, u, dtype=torch.float64, **kw):
    d = dgmf.make_desc(k, n_el, length, n_comp=3 if u.ndim == 3 else 1, **kw)
    y = dgmf.apply_laplace(d, to_dev(u, dtype))
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def _mesh_for(k):
    # E = floor(256/n^2) elements per workgroup; pick N_el > 2E, not a multiple of E
    E = max(1, 256 // (k + 1) ** 2)
    nx = 5
    ny = 3
    nz = max(2, (2 * E) // (nx * ny) + 1)
    if (nx * ny * nz) % E == 0:
        nz += 1
    return (nx, ny, nz)


def test_config1_fp64():
    """4^3 elements, k=3, tau=(k+1)^2/h, U[-1,1] from seed (the small parity case)."""
    k, N = 3, 4
    msh = M.cube(N)
    u = inputs.uniform((msh.N, 64), seed=inputs.FIELD_SEED_BASE + 0)
    announce("laplace config1 k=3 N=4 fp64")
    y = _run(k, N, msh.length, u)
    ref = laplace_apply(u, k, msh)
    assert rel_err(y, ref) < 1e-12
    assert np.abs(y - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("k", list(range(1, 12)))
def test_all_degrees_fp64(k):
    n_el = _mesh_for(k)
    length = (2 * np.pi, 2.0, 3.5)
    msh = M.Mesh(n_el, length)
    u = inputs.uniform((msh.N, (k + 1) ** 3), seed=200 + k)
    announce(f"laplace fp64 k={k} n_el={n_el}")
    y = _run(k, n_el, length, u)
    assert rel_err(y, laplace_apply(u, k, msh)) < 1e-12


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7, 11])
def test_all_degrees_fp32(k):
    n_el = _mesh_for(k)
    length = (2 * np.pi,) * 3
    msh = M.Mesh(n_el, length)
    u = round_f32(inputs.uniform((msh.N, (k + 1) ** 3), seed=300 + k))
    announce(f"laplace fp32 k={k} n_el={n_el}")
    y = _run(k, n_el, length, u, dtype=torch.float32)
    assert rel_err(y, laplace_apply(u, k, msh)) < 1e-5


@pytest.mark.parametrize("n_el", [(1, 1, 1), (1, 2, 3), (2, 2, 2), (7, 1, 2)])
def test_one_and_two_elements_per_direction(n_el):
    k = 4
    length = (1.0, 2.0, 3.0)
    msh = M.Mesh(n_el, length)
    u = inputs.uniform((msh.N, 125), seed=17)
    announce(f"laplace small mesh n_el={n_el}")
    y = _run(k, n_el, length, u)
    assert rel_err(y, laplace_apply(u, k, msh)) < 1e-12


def test_three_components_penalty_scale_nq():
    k = 5
    n_el = (3, 4, 2)
    length = (2 * np.pi, 1.0, 2.0)
    msh = M.Mesh(n_el, length)
    u = inputs.uniform((3, msh.N, 216), seed=18)
    announce("laplace n_comp=3 penalty=2.5 scale=1/1600 n_q=9")
    y = _run(k, n_el, length, u, penalty_factor=2.5, scale=1 / 1600, n_q=9)
    ref = laplace_apply(u, k, msh, n_q=9, penalty_factor=2.5, scale=1 / 1600)
    assert rel_err(y, ref) < 1e-12
    announce("laplace over-integrated n_q=12 for k=5")
    y = _run(k, n_el, length, u[0], n_q=12)
    assert rel_err(y, laplace_apply(u[0], k, msh, n_q=12)) < 1e-12
    with pytest.raises(dgmf.DgError) as ei:
        _run(k, n_el, length, u[0], n_q=4)
    assert ei.value.code == dgmf.DG_ERR_UNSUPPORTED


def test_invariants_on_gpu_output():
    """A 1 = 0, symmetry v.Au = u.Av, bitwise determinism."""
    k, N = 4, 6
    d = dgmf.make_desc(k, N)
    n3 = 125
    ones = torch.ones((N ** 3, n3), dtype=torch.float64, device="cuda")
    announce("laplace invariants")
    y1 = dgmf.apply_laplace(d, ones)
    diag = laplace_diagonal(k, M.cube(N))
    assert y1.abs().max().item() < 1e-12 * np.abs(diag).max()
    u = to_dev(inputs.uniform((N ** 3, n3), seed=19))
    v = to_dev(inputs.uniform((N ** 3, n3), seed=20))
    Au, Av = dgmf.apply_laplace(d, u), dgmf.apply_laplace(d, v)
    a, b = (v * Au).sum().item(), (u * Av).sum().item()
    assert abs(a - b) < 1e-13 * (Au.abs().sum().item())
    Au2 = dgmf.apply_laplace(d, u)
    assert torch.equal(Au, Au2)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_full_size_sampled(dtype):
    """Degree-sweep size (k=3, 64^3 elements, 16.8M DoFs), sampled elements."""
    k, N = 3, 64
    msh = M.cube(N)
    u = inputs.uniform((msh.N, 64), seed=inputs.FIELD_SEED_BASE + 2)
    if dtype == torch.float32:
        u = round_f32(u)
    announce(f"laplace full size k=3 N=64 {dtype}")
    y = _run(k, N, msh.length, u, dtype=dtype)
    rng = np.random.default_rng(7)
    sample = np.unique(np.concatenate([rng.integers(0, msh.N, 200), [0, N - 1, N * N - 1, msh.N - 1]]))
    ref = laplace_apply(u, k, msh, elems=sample)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert rel_err(y[sample], ref) < tol


def test_alias_error_on_gpu():
    d = dgmf.make_desc(3, 4)
    u = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(dgmf.DgError) as ei:
        dgmf.apply_laplace(d, u, out=u)
    assert ei.value.code == dgmf.DG_ERR_ALIAS


@pytest.mark.parametrize("k,dtype", [(3, torch.float64), (2, torch.float32), (4, torch.float64)])
def test_partial_tiles_and_short_last_z_segment(k, dtype):
    """47 x 46 x 47 elements: the low-degree kernel's x-y tiles do not divide
    the mesh and its last z segment is shorter than the others; sampled
    elements at tile and segment borders, corners and wrap-around."""
    n_el = (47, 46, 47)
    msh = M.Mesh(n_el, (2 * np.pi,) * 3)
    n3 = (k + 1) ** 3
    u = inputs.uniform((msh.N, n3), seed=400 + k)
    if dtype == torch.float32:
        u = round_f32(u)
    announce(f"laplace partial tiles k={k} {dtype}")
    y = _run(k, n_el, msh.length, u, dtype=dtype)
    nx, ny, nz = n_el
    rng = np.random.default_rng(11)
    ex = np.concatenate([[0, 1, 3, 4, 7, 8, nx - 2, nx - 1], rng.integers(0, nx, 12)])
    ey = np.concatenate([[0, 3, 4, 7, 8, ny - 2, ny - 1], rng.integers(0, ny, 12)])
    ez = np.concatenate([[0, 1, 2, 3, 4, nz - 4, nz - 3, nz - 2, nz - 1], rng.integers(0, nz, 12)])
    sample = np.unique((ex[:, None, None] + nx * (ey[None, :, None] + ny * ez[None, None, :])).ravel())
    sample = sample[rng.permutation(len(sample))[:400]]
    ref = laplace_apply(u, k, msh, elems=np.sort(sample))
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert rel_err(y[np.sort(sample)], ref) < tol


def test_three_components_low_degree():
    """n_comp = 3 through the low-degree (marching) kernel, full oracle check."""
    k, n_el = 3, (6, 5, 7)
    msh = M.Mesh(n_el, (1.0, 2.0, 3.0))
    u = inputs.uniform((3, msh.N, 64), seed=21)
    announce("laplace n_comp=3 k=3")
    y = _run(k, n_el, msh.length, u, penalty_factor=1.5, scale=0.25)
    ref = laplace_apply(u, k, msh, penalty_factor=1.5, scale=0.25)
    assert rel_err(y, ref) < 1e-12
