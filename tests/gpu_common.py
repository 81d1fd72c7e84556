"""Helpers for the GPU parity tests (imported by tests marked ``gpu``)."""
import sys

import numpy as np


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm GPU")
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device())


def rel_err(got, ref):
    """The larger of the relative 2-norm error ||got - ref|| / ||ref|| and the
    element-wise error max|got - ref| / max|ref|, so that one entry far off
    cannot hide in the norm of a large array."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    nrm = np.linalg.norm(ref)
    top = np.abs(ref).max() if ref.size else 0.0
    e2 = np.linalg.norm(got - ref) / (nrm if nrm > 0 else 1.0)
    emax = np.abs(got - ref).max() / (top if top > 0 else 1.0) if ref.size else 0.0
    return max(e2, emax)


def announce(msg):
    """Name the case before a GPU step so a failure points at it."""
    print(msg, file=sys.stderr, flush=True)


def round_f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)
