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
