"""dg_cg_solve_noalloc (work memory from the library's static array) against
dg_cg_solve (work memory the library allocates), through the C ABI: two
calls in a row, the second on a smaller problem, for the FP32 Chebyshev and
the FP64 Jacobi preconditioners.  Both run the same kernels on the same
data, so the solutions agree to the FP64 parity bound and the iteration
counts and eigenvalue bounds are equal."""
import numpy as np
import pytest
import torch

from gpu_common import announce, rel_err, to_dev
from oracle import basis, mesh as M
from oracle.divergence import poisson_rhs
from paper_1802_01439_amd import dgmf, inputs

pytestmark = pytest.mark.gpu


def _rhs(k, N, seed):
    msh = M.cube(N)
    u = inputs.tgv_plus_noise(basis.lgl_nodes(k), msh.n_el, msh.length, seed=seed)
    return to_dev(poisson_rhs(u, k, msh))


@pytest.mark.parametrize("precond", [dgmf.DG_PC_CHEB_F32, dgmf.DG_PC_JACOBI_F64])
def test_noalloc_solve_matches_the_allocating_solve(precond):
    cases = [(3, 6), (2, 4)]             # the second call is smaller than the first
    bs = [_rhs(k, N, 700 + k) for k, N in cases]
    refs = []
    for (k, N), b in zip(cases, bs):
        announce(f"cg reference k={k} N={N} precond={precond}")
        refs.append(dgmf.cg_solve(dgmf.make_desc(k, N), b, precond=precond, rtol=1e-10))
    got = []
    for (k, N), b in zip(cases, bs):
        announce(f"cg noalloc k={k} N={N} precond={precond}")
        x = torch.zeros_like(b)
        got.append(dgmf.cg_solve(dgmf.make_desc(k, N), b, x=x, precond=precond, rtol=1e-10, noalloc=True))
    for (k, N), (x_ref, rep_ref, rc_ref), (x, rep, rc) in zip(cases, refs, got):
        assert rc == rc_ref == dgmf.DG_OK, (rep, rep_ref)
        assert rep["iterations"] == rep_ref["iterations"], (rep, rep_ref)
        assert rep["matvec_f32"] == rep_ref["matvec_f32"]
        assert abs(rep["lambda_max"] - rep_ref["lambda_max"]) <= 1e-12 * abs(rep_ref["lambda_max"])
        assert rep["true_rel_res"] < 1e-9
        assert rel_err(x.cpu().numpy(), x_ref.cpu().numpy()) < 1e-12, (k, N)
