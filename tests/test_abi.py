"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/dgmf.h, and its host-only logic (validation, LGL nodes,
the SIPG diagonal) behaves.  No compute kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import basis, mesh as M
from oracle.laplace import laplace_diagonal
from paper_1802_01439_amd import dgmf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgmf.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = dgmf.lib()
    names = declared_functions()
    assert "dg_apply_laplace" in names and "dg_cg_solve" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(dgmf.EXPORTS) >= set(names)


def test_error_strings():
    L = dgmf.lib()
    for code in (0, -1, -2, -3, -4, 1, 2):
        assert L.dg_error_string(code).decode()


def _call_laplace(desc, src, dst, dtype=dgmf.DG_F64):
    return dgmf.lib().dg_apply_laplace(desc, dtype, ctypes.c_void_p(src), ctypes.c_void_p(dst), None)


def test_validation_errors_without_gpu():
    L = dgmf.lib()
    d = dgmf.make_desc(3, 4)
    fake_a, fake_b = 0x10000000, 0x20000000      # never dereferenced: validation fails first
    assert L.dg_apply_laplace(None, 0, ctypes.c_void_p(fake_a), ctypes.c_void_p(fake_b), None) == dgmf.DG_ERR_INVALID_ARG
    bad = dgmf.make_desc(12, 4)
    assert _call_laplace(ctypes.byref(bad), fake_a, fake_b) == dgmf.DG_ERR_UNSUPPORTED
    bad = dgmf.make_desc(0, 4)
    assert _call_laplace(ctypes.byref(bad), fake_a, fake_b) == dgmf.DG_ERR_UNSUPPORTED
    bad = dgmf.make_desc(3, (4, 0, 4))
    assert _call_laplace(ctypes.byref(bad), fake_a, fake_b) == dgmf.DG_ERR_INVALID_ARG
    bad = dgmf.make_desc(3, 4, length=-1.0)
    assert _call_laplace(ctypes.byref(bad), fake_a, fake_b) == dgmf.DG_ERR_INVALID_ARG
    bad = dgmf.make_desc(3, 4, penalty_factor=float("nan"))
    assert _call_laplace(ctypes.byref(bad), fake_a, fake_b) == dgmf.DG_ERR_INVALID_ARG
    bad = dgmf.make_desc(3, 4, n_comp=2)
    assert _call_laplace(ctypes.byref(bad), fake_a, fake_b) == dgmf.DG_ERR_INVALID_ARG
    assert _call_laplace(ctypes.byref(d), fake_a, 0) == dgmf.DG_ERR_INVALID_ARG
    assert _call_laplace(ctypes.byref(d), fake_a, fake_b, dtype=7) == dgmf.DG_ERR_INVALID_ARG
    # overlapping ranges: dst starts inside src
    assert _call_laplace(ctypes.byref(d), fake_a, fake_a + 8) == dgmf.DG_ERR_ALIAS
    assert "overlap" in L.dg_last_error().decode()


def test_lgl_nodes_match_oracle():
    for k in range(1, 12):
        np.testing.assert_allclose(dgmf.lgl_nodes(k), basis.lgl_nodes(k), atol=4e-16)


@pytest.mark.parametrize("k,n_el,pen,scale", [(3, (4, 4, 4), 1.0, 1.0), (5, (3, 2, 4), 2.0, 0.01),
                                              (2, (1, 3, 2), 1.0, 1.0), (7, (2, 2, 2), 1.0, 1.0)])
def test_host_diagonal_matches_oracle(k, n_el, pen, scale):
    length = (2 * np.pi, 1.5, 3.0)
    msh = M.Mesh(n_el, length)
    ref = laplace_diagonal(k, msh, penalty_factor=pen, scale=scale)
    got = dgmf.laplace_diagonal(dgmf.make_desc(k, n_el, length, penalty_factor=pen, scale=scale))
    np.testing.assert_allclose(got, ref, rtol=1e-13)


def test_validation_errors_of_the_widening_entry_points_without_gpu():
    L = dgmf.lib()
    vp = ctypes.c_void_p
    fa, fb, fc, fd = 0x10000000, 0x20000000, 0x30000000, 0x40000000   # never dereferenced
    d1 = dgmf.make_desc(3, 4)
    d3 = dgmf.make_desc(3, 4, n_comp=3)
    # projection operator: three components, n_q = k+1, no aliasing
    assert L.dg_apply_projection(ctypes.byref(d1), 0, vp(fa), vp(fb), vp(fc), vp(fd), None) == dgmf.DG_ERR_INVALID_ARG
    dq = dgmf.make_desc(3, 4, n_comp=3, n_q=6)
    assert L.dg_apply_projection(ctypes.byref(dq), 0, vp(fa), vp(fb), vp(fc), vp(fd), None) == dgmf.DG_ERR_UNSUPPORTED
    assert L.dg_apply_projection(ctypes.byref(d3), 0, vp(fa), vp(fb), None, vp(fd), None) == dgmf.DG_ERR_INVALID_ARG
    assert L.dg_apply_projection(ctypes.byref(d3), 0, vp(fa), vp(fb), vp(fc), vp(fa + 8), None) == dgmf.DG_ERR_ALIAS
    # gradient: y (3 components) must not overlap p
    assert L.dg_apply_gradient(ctypes.byref(d1), 0, vp(fa), None, None) == dgmf.DG_ERR_INVALID_ARG
    assert L.dg_apply_gradient(ctypes.byref(d1), 0, vp(fa + 8), vp(fa), None) == dgmf.DG_ERR_ALIAS
    # Helmholtz and inverse mass
    assert L.dg_apply_helmholtz(ctypes.byref(d1), 0, -1.0, vp(fa), vp(fb), None) == dgmf.DG_ERR_INVALID_ARG
    assert L.dg_apply_inverse_mass(ctypes.byref(d1), 0, vp(fa), vp(fa + 8), None) == dgmf.DG_ERR_ALIAS
    # mass-preconditioned CG
    def solve(desc, op, mf, td, tc, b, x, rtol=1e-10, it=10):
        return L.dg_mass_pcg_solve(ctypes.byref(desc), op, mf, td, tc, vp(b), vp(x), rtol, it, None, None)
    assert solve(d1, 7, 1.0, None, None, fa, fb) == dgmf.DG_ERR_INVALID_ARG
    assert solve(d1, dgmf.DG_OP_HELMHOLTZ, 0.0, None, None, fa, fb) == dgmf.DG_ERR_INVALID_ARG
    assert solve(d1, dgmf.DG_OP_HELMHOLTZ, 1.0, None, None, fa, fb, rtol=0.0) == dgmf.DG_ERR_INVALID_ARG
    assert solve(d1, dgmf.DG_OP_HELMHOLTZ, 1.0, None, None, fa, fb, it=-1) == dgmf.DG_ERR_INVALID_ARG
    assert solve(d1, dgmf.DG_OP_PROJECTION, 0.0, vp(fc), vp(fd), fa, fb) == dgmf.DG_ERR_INVALID_ARG
    assert solve(d3, dgmf.DG_OP_PROJECTION, 0.0, None, vp(fd), fa, fb) == dgmf.DG_ERR_INVALID_ARG
    assert solve(d3, dgmf.DG_OP_PROJECTION, 0.0, vp(fc), vp(fd), fa, fa + 8) == dgmf.DG_ERR_ALIAS
    assert solve(d1, dgmf.DG_OP_HELMHOLTZ, 1.0, None, None, fa, fa) == dgmf.DG_ERR_ALIAS


def test_validation_errors_of_the_multigrid_entry_points_without_gpu():
    L = dgmf.lib()
    vp = ctypes.c_void_p
    fa, fb = 0x10000000, 0x20000000      # never dereferenced
    lam2 = (ctypes.c_double * 2)(2.5, 2.5)
    bad = (ctypes.c_double * 2)(2.5, float("nan"))
    d = dgmf.make_desc(2, (8, 4, 4))
    d6 = dgmf.make_desc(2, (6, 4, 4))
    d3 = dgmf.make_desc(2, 4, n_comp=3)

    def vc(desc, levels, lam, r, z, degree=5, rng=20.0, coarse=10):
        return L.dg_gmg_vcycle(ctypes.byref(desc), levels, degree, rng, coarse, lam, dgmf.DG_F64, vp(r), vp(z), None)
    assert vc(d3, 2, lam2, fa, fb) == dgmf.DG_ERR_INVALID_ARG            # n_comp must be 1
    assert vc(d6, 3, (ctypes.c_double * 3)(1, 1, 1), fa, fb) == dgmf.DG_ERR_INVALID_ARG   # 6 not divisible by 4
    assert vc(d, 2, bad, fa, fb) == dgmf.DG_ERR_INVALID_ARG              # non-finite bound
    assert vc(d, 0, lam2, fa, fb) == dgmf.DG_ERR_INVALID_ARG             # no level
    assert vc(d, 2, lam2, fa, fb, rng=1.0) == dgmf.DG_ERR_INVALID_ARG    # smoothing range must exceed 1
    assert vc(d, 2, lam2, fa, fa + 8) == dgmf.DG_ERR_ALIAS
    assert L.dg_gmg_vcycle(ctypes.byref(d), 2, 5, 20.0, 10, lam2, 7, vp(fa), vp(fb), None) == dgmf.DG_ERR_INVALID_ARG
    # FP32: 4-byte values, so an offset of 4 bytes still overlaps
    assert L.dg_gmg_vcycle(ctypes.byref(d), 2, 5, 20.0, 10, lam2, dgmf.DG_F32, vp(fa), vp(fa + 4),
                           None) == dgmf.DG_ERR_ALIAS
    rep = dgmf.CgReport()

    def cg(desc, levels, lam, b, x, rtol=1e-10, it=10, cycle=dgmf.DG_F64, deg=5, rng=20.0, cdeg=10):
        return L.dg_gmg_cg_solve(ctypes.byref(desc), levels, deg, rng, cdeg, lam, cycle, vp(b), vp(x), rtol, it,
                                 ctypes.byref(rep), None)
    assert cg(d, 2, lam2, fa, fb, rtol=0.0) == dgmf.DG_ERR_INVALID_ARG
    assert cg(d, 2, lam2, fa, fb, cycle=7) == dgmf.DG_ERR_INVALID_ARG       # cycle precision F64 or F32
    assert cg(d, 2, lam2, fa, fa + 8, cycle=dgmf.DG_F32) == dgmf.DG_ERR_ALIAS
    assert cg(d, 2, lam2, fa, fb, it=-1) == dgmf.DG_ERR_INVALID_ARG
    assert cg(d, 2, bad, fa, fb) == dgmf.DG_ERR_INVALID_ARG
    assert cg(d, 2, lam2, fa, fb, deg=0) == dgmf.DG_ERR_INVALID_ARG          # smoother degrees >= 1
    assert cg(d, 2, lam2, fa, fb, rng=0.5) == dgmf.DG_ERR_INVALID_ARG        # smoothing range > 1
    assert cg(d, 2, lam2, fa, fa + 8) == dgmf.DG_ERR_ALIAS


def test_binding_checks_dtype_before_any_launch():
    """An output or solution tensor of another dtype than the call's would be
    written past its end by the kernel (the C ABI takes one dtype per call):
    the binding raises TypeError before calling the library.  Shapes match
    here, so the dtype check is the one that fires (host tensors: nothing
    reaches a GPU)."""
    import torch
    k, N = 2, 2
    n3 = (k + 1) ** 3
    d1, d3 = dgmf.make_desc(k, N), dgmf.make_desc(k, N, n_comp=3)
    s64 = torch.zeros((N ** 3, n3), dtype=torch.float64)
    v64 = torch.zeros((3, N ** 3, n3), dtype=torch.float64)
    s32, v32 = s64.float(), v64.float()
    tau32 = torch.zeros(N ** 3, dtype=torch.float32)
    cases = [
        lambda: dgmf.apply_laplace(d1, s64, out=s32),
        lambda: dgmf.apply_convective(d1, v64, out=v32),
        lambda: dgmf.vjp_convective(d1, v64, v32),
        lambda: dgmf.vjp_convective(d1, v64, v64, out=v32),
        lambda: dgmf.apply_divergence(d1, v64, out=s32),
        lambda: dgmf.apply_gradient(d1, s64, out=v32),
        lambda: dgmf.apply_helmholtz(d1, s64, 1.0, out=s32),
        lambda: dgmf.apply_projection(d3, v64, tau32, tau32),
        lambda: dgmf.apply_inverse_mass(d1, s32, out=s64),
        lambda: dgmf.prolongate(dgmf.make_desc(k, 1), s64[:1], out=s32),
        lambda: dgmf.restrict(dgmf.make_desc(k, 1), s64, out=s32[:1]),
        lambda: dgmf.gmg_vcycle(d1, s32, [1.0], out=s64),
        lambda: dgmf.cg_solve(d1, s32),
        lambda: dgmf.cg_solve(d1, s64, x=s32),
        lambda: dgmf.gmg_cg_solve(d1, s64, [1.0], x=s32),
        lambda: dgmf.mass_pcg_solve(d3, dgmf.DG_OP_HELMHOLTZ, v64, x=v32, mass_factor=1.0),
        lambda: dgmf.mass_pcg_solve(d3, dgmf.DG_OP_PROJECTION, v64, tau_d=tau32, tau_c=tau32),
    ]
    for i, call in enumerate(cases):
        with pytest.raises(TypeError):
            call()


def test_noalloc_cg_refuses_problems_beyond_its_static_array_without_gpu():
    """68 bytes per DoF in a 64 MiB array: 1.1e6 DoFs (k = 3, 20 x 20 x 43
    elements) no longer fit and are refused before any HIP call; the
    argument checks are those of dg_cg_solve."""
    L = dgmf.lib()
    vp = ctypes.c_void_p
    fa, fb = 0x10000000, 0x40000000      # never dereferenced
    o = dgmf.CgOpts()
    o.precond, o.cheb_degree, o.cheb_range, o.rtol, o.atol, o.max_iter, o.project_mean = 1, 5, 20.0, 1e-10, 0.0, 10, 1
    big = dgmf.make_desc(3, (20, 20, 43))
    assert L.dg_cg_solve_noalloc(ctypes.byref(big), ctypes.byref(o), vp(fa), vp(fb), None, None) == \
        dgmf.DG_ERR_INVALID_ARG
    assert "scratch" in L.dg_last_error().decode()
    small = dgmf.make_desc(3, 4)
    assert L.dg_cg_solve_noalloc(ctypes.byref(small), ctypes.byref(o), vp(fa), vp(fa + 8), None, None) == \
        dgmf.DG_ERR_ALIAS
    o.max_iter = 0
    assert L.dg_cg_solve_noalloc(ctypes.byref(small), ctypes.byref(o), vp(fa), vp(fb), None, None) == \
        dgmf.DG_ERR_INVALID_ARG
