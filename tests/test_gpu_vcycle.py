"""GPU parity of dg_gmg_vcycle (one FP64 multigrid V-cycle for the SIPG
Laplacian) against the oracle's V-cycle, through the C ABI.

Both sides take the same per-level eigenvalue bounds (from the oracle's
Lanczos estimate), so the two cycles are the same linear operator; FP64
within 1e-11 relative (2-norm).  Two and three levels, a single level (the
coarse Chebyshev alone), anisotropic meshes, penalty and scale factors.
"""
import numpy as np
import pytest
import torch

from gpu_common import announce, rel_err, to_dev
from oracle import mesh as M
from oracle.laplace import laplace_apply, laplace_diagonal
from oracle.multigrid import level_meshes, vcycle
from oracle.solvers import lanczos_max_eig
from paper_1802_01439_amd import dgmf, inputs

pytestmark = pytest.mark.gpu


def _lams(k, fine, levels, pen, scale):
    out = []
    for msh in level_meshes(fine, levels):
        dinv = np.tile(1.0 / laplace_diagonal(k, msh, penalty_factor=pen, scale=scale), msh.N)
        A = lambda v, msh=msh: laplace_apply(v.reshape(msh.N, -1), k, msh, penalty_factor=pen, scale=scale).ravel()
        out.append(1.1 * lanczos_max_eig(A, dinv, msh.N * (k + 1) ** 3, steps=25, project=True))
    return out


@pytest.mark.parametrize("k,n_el,length,levels,pen,scale", [
    (3, (8, 8, 8), (2 * np.pi,) * 3, 3, 1.0, 1.0),
    (2, (8, 4, 4), (2.0, 1.0, 1.5), 2, 1.0, 1.0),
    (5, (4, 4, 4), (1.0, 1.0, 1.0), 2, 2.0, 0.5),
    (4, (4, 2, 6), (1.0, 0.7, 1.3), 1, 1.0, 1.0),
])
def test_vcycle_parity(k, n_el, length, levels, pen, scale):
    fine = M.Mesh(n_el, length)
    lam = _lams(k, fine, levels, pen, scale)
    r = inputs.uniform((fine.N, (k + 1) ** 3), seed=1100 + k)
    r -= r.mean()
    announce(f"V-cycle k={k} n_el={n_el} levels={levels}")
    d = dgmf.make_desc(k, n_el, length, penalty_factor=pen, scale=scale)
    z = dgmf.gmg_vcycle(d, to_dev(r), lam).cpu().numpy()
    ref = vcycle(r, k, fine, levels, lam, penalty_factor=pen, scale=scale)
    assert rel_err(z, ref) < 1e-11


def test_vcycle_rejects_bad_arguments():
    d = dgmf.make_desc(2, (6, 4, 4))
    r = torch.zeros(96, 27, dtype=torch.float64, device="cuda")
    with pytest.raises(dgmf.DgError):      # 6 is not divisible by 4
        dgmf.gmg_vcycle(d, r, [1.0, 1.0, 1.0])
    with pytest.raises(dgmf.DgError):      # lambda_max must be positive
        dgmf.gmg_vcycle(d, r, [1.0, -1.0])
    with pytest.raises(dgmf.DgError):      # z aliases r
        dgmf.gmg_vcycle(d, r, [1.0, 1.0], out=r)
