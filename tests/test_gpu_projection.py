"""GPU parity of dg_apply_projection (M + A_D + A_C of the projection step)
against the CPU oracle, through the C ABI.

FP64 within 1e-12 relative (2-norm), FP32 within 1e-5 relative against the
oracle applied to the FP32-rounded inputs.  Meshes span several workgroup
batches with a ragged last batch, on anisotropic boxes, with random
per-element penalty parameters; one-element directions (the element is its
own neighbour); the special cases tau = 0 (the mass matrix) and the symmetry
of the operator at a larger size; the degree-sweep meshes the benchmark
times, on 64 sampled elements (the first and last among them).
"""
import numpy as np
import pytest
import torch

from gpu_common import announce, rel_err, round_f32, to_dev
from oracle import mesh as M
from oracle.mass import mass_apply
from oracle.projection import projection_apply
from paper_1802_01439_amd import dgmf, inputs

pytestmark = pytest.mark.gpu


def _mesh_for(k):
    # E = floor(256 / (3 n^2)) elements per workgroup; N_el > 2E and not a multiple of E
    E = max(1, 256 // (3 * (k + 1) ** 2))
    nx = 2 * E + 3
    return (nx, 2, 1) if nx < 30 else (nx, 1, 1)


def _case(k, n_el, length, seed, dtype):
    msh = M.Mesh(n_el, length)
    u = inputs.uniform((3, msh.N, (k + 1) ** 3), seed=seed)
    h2 = float(np.min(msh.h)) ** 2
    td = inputs.uniform((msh.N,), seed=seed + 1, lo=0.1, hi=1.0) * h2
    tc = inputs.uniform((msh.N,), seed=seed + 2, lo=0.1, hi=1.0) * h2
    if dtype == torch.float32:
        u, td, tc = round_f32(u), round_f32(td), round_f32(tc)
    return msh, u, td, tc


def _run(k, msh, u, td, tc, dtype):
    d = dgmf.make_desc(k, msh.n_el, tuple(msh.length), n_comp=3)
    y = dgmf.apply_projection(d, to_dev(u, dtype), to_dev(td, dtype), to_dev(tc, dtype))
    return y.double().cpu().numpy()


@pytest.mark.parametrize("k", list(range(1, 12)))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_projection_parity(k, dtype):
    n_el = _mesh_for(k)
    length = (1.0 * n_el[0], 0.7 * n_el[1], 1.3 * n_el[2])
    msh, u, td, tc = _case(k, n_el, length, 800 + k, dtype)
    announce(f"projection k={k} {dtype} n_el={n_el}")
    y = _run(k, msh, u, td, tc, dtype)
    assert rel_err(y, projection_apply(u, k, msh, td, tc)) < (1e-12 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("k,n_el", [(2, (3, 1, 2)), (4, (1, 1, 1)), (6, (2, 3, 1))])
def test_projection_one_element_directions(k, n_el):
    msh, u, td, tc = _case(k, n_el, (1.1, 0.9, 1.4), 830 + k, torch.float64)
    announce(f"projection k={k} n_el={n_el}")
    y = _run(k, msh, u, td, tc, torch.float64)
    assert rel_err(y, projection_apply(u, k, msh, td, tc)) < 1e-12


@pytest.mark.parametrize("k", [3, 8])
def test_projection_zero_penalty_is_the_mass_matrix(k):
    msh, u, _, _ = _case(k, (4, 3, 2), (2.0, 1.5, 1.0), 850 + k, torch.float64)
    z = np.zeros(msh.N)
    announce(f"projection tau=0 k={k}")
    y = _run(k, msh, u, z, z, torch.float64)
    assert rel_err(y, mass_apply(u, k, msh)) < 1e-12


@pytest.mark.parametrize("k", [2, 5])
def test_projection_symmetric_at_larger_size(k):
    n = 16 if k == 5 else 24
    msh, u, td, tc = _case(k, (n, n, n), (2 * np.pi,) * 3, 870 + k, torch.float64)
    v = inputs.normal(u.shape, seed=880 + k)
    announce(f"projection symmetry k={k} n_el={n}^3")
    au = _run(k, msh, u, td, tc, torch.float64)
    av = _run(k, msh, v, td, tc, torch.float64)
    a, b = float(np.vdot(v, au)), float(np.vdot(u, av))
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0) * 10
    # positive definite: the mass is, both penalties are positive semi-definite
    assert float(np.vdot(u, au)) > 0


def test_projection_rejects_bad_arguments():
    k = 2
    dev = torch.device("cuda:0")
    d1 = dgmf.make_desc(k, 3)
    u1 = torch.zeros(1, 27, 27, dtype=torch.float64, device=dev)
    t = torch.zeros(27, dtype=torch.float64, device=dev)
    rc = dgmf.lib().dg_apply_projection(dgmf.ctypes.byref(d1), dgmf.DG_F64, dgmf.ctypes.c_void_p(u1.data_ptr()),
                                        dgmf.ctypes.c_void_p(t.data_ptr()), dgmf.ctypes.c_void_p(t.data_ptr()),
                                        dgmf.ctypes.c_void_p(u1.data_ptr() + 8 * 27 * 27), None)
    assert rc == dgmf.DG_ERR_INVALID_ARG            # n_comp must be 3
    d3 = dgmf.make_desc(k, 3, n_comp=3)
    u = torch.zeros(3, 27, 27, dtype=torch.float64, device=dev)
    rc = dgmf.lib().dg_apply_projection(dgmf.ctypes.byref(d3), dgmf.DG_F64, dgmf.ctypes.c_void_p(u.data_ptr()),
                                        dgmf.ctypes.c_void_p(t.data_ptr()), dgmf.ctypes.c_void_p(t.data_ptr()),
                                        dgmf.ctypes.c_void_p(u.data_ptr()), None)
    assert rc == dgmf.DG_ERR_ALIAS
    with pytest.raises(TypeError):
        dgmf.apply_projection(d3, u, t.float(), t)


@pytest.mark.parametrize("k,dtype", [(3, torch.float64), (7, torch.float64), (9, torch.float32)])
def test_projection_full_size_sampled(k, dtype):
    # the degree-sweep mesh the benchmark times: N = round(256/(k+1)) elements
    # per direction on [-pi, pi]^3, three components, tau ~ U[0.1, 1] h^2
    N = int(round(256.0 / (k + 1)))
    msh = M.cube(N)
    u = inputs.uniform((3, msh.N, (k + 1) ** 3), seed=890 + k)
    h2 = float(msh.h[0]) ** 2
    td = inputs.uniform((msh.N,), seed=891 + k, lo=0.1, hi=1.0) * h2
    tc = inputs.uniform((msh.N,), seed=892 + k, lo=0.1, hi=1.0) * h2
    if dtype == torch.float32:
        u, td, tc = round_f32(u), round_f32(td), round_f32(tc)
    announce(f"projection full size k={k} N={N} {dtype}")
    y = _run(k, msh, u, td, tc, dtype)
    rng = np.random.default_rng(893 + k)
    el = np.concatenate([[0, msh.N - 1], rng.choice(msh.N, 62, replace=False)])
    ref = projection_apply(u, k, msh, td, tc, elems=el)
    assert rel_err(y[:, el], ref) < (1e-12 if dtype == torch.float64 else 1e-5)
