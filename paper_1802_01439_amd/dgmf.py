"""Thin ctypes binding of libdgmf.so (the C ABI in include/dgmf.h).

Argument marshalling only: every step of every operator runs in the HIP
library.  Tensors must be contiguous CUDA (ROCm) tensors of float64 or
float32; the call is enqueued on torch's current stream.  If the library has
not been built, every entry point raises.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdgmf.so")

DG_OK = 0
DG_ERR_INVALID_ARG = -1
DG_ERR_UNSUPPORTED = -2
DG_ERR_ALIAS = -3
DG_ERR_HIP = -4
DG_NOT_CONVERGED = 1
DG_ERR_BREAKDOWN = 2
DG_F64, DG_F32 = 0, 1
DG_PC_JACOBI_F64, DG_PC_CHEB_F32 = 0, 1
DG_OP_HELMHOLTZ, DG_OP_PROJECTION = 0, 1
DG_STEP_PC_GMG_F32, DG_STEP_PC_CHEB_F32 = 0, 1

EXPORTS = ("dg_apply_laplace", "dg_apply_convective", "dg_vjp_convective", "dg_apply_divergence",
           "dg_apply_inverse_mass", "dg_apply_helmholtz", "dg_apply_projection", "dg_apply_gradient", "dg_prolongate", "dg_restrict", "dg_gmg_vcycle", "dg_gmg_cg_solve", "dg_cg_solve", "dg_cg_solve_noalloc", "dg_mass_pcg_solve", "dg_apply_divergence_mixed", "dg_apply_gradient_mixed",
           "dg_tgv_diagnostics", "dg_dual_splitting_step", "dg_dual_splitting_step_conv", "dg_laplace_diagonal",
           "dg_lgl_nodes", "dg_error_string", "dg_last_error")


class OpDesc(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("n_el", ctypes.c_int32 * 3), ("length", ctypes.c_double * 3),
                ("n_q", ctypes.c_int32), ("penalty_factor", ctypes.c_double), ("scale", ctypes.c_double),
                ("n_comp", ctypes.c_int32), ("lf_factor", ctypes.c_double)]


class CgOpts(ctypes.Structure):
    _fields_ = [("precond", ctypes.c_int32), ("cheb_degree", ctypes.c_int32), ("cheb_range", ctypes.c_double),
                ("rtol", ctypes.c_double), ("atol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("project_mean", ctypes.c_int32)]


class CgReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("matvec_f64", ctypes.c_int32), ("matvec_f32", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("seconds_solve", ctypes.c_double), ("seconds_setup", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class StepOpts(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("dt", ctypes.c_double), ("nu", ctypes.c_double),
                ("zeta_d", ctypes.c_double), ("zeta_c", ctypes.c_double), ("rtol_pressure", ctypes.c_double),
                ("rtol_projection", ctypes.c_double), ("rtol_viscous", ctypes.c_double),
                ("atol_pressure", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("pressure_precond", ctypes.c_int32)]


class StepReport(ctypes.Structure):
    _fields_ = [("it_pressure", ctypes.c_int32), ("it_projection", ctypes.c_int32), ("it_viscous", ctypes.c_int32),
                ("kinetic_energy", ctypes.c_double), ("dissipation", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class DgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdgmf error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libdgmf.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                               "(python -m paper_1802_01439_amd.build) first")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, i32 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32
        pd = ctypes.POINTER(OpDesc)
        L.dg_apply_laplace.argtypes = [pd, ctypes.c_int, vp, vp, vp]
        L.dg_apply_convective.argtypes = [pd, ctypes.c_int, vp, vp, vp]
        L.dg_vjp_convective.argtypes = [pd, ctypes.c_int, vp, vp, vp, vp]
        L.dg_apply_divergence.argtypes = [pd, ctypes.c_int, vp, vp, vp]
        L.dg_apply_inverse_mass.argtypes = [pd, ctypes.c_int, vp, vp, vp]
        L.dg_apply_helmholtz.argtypes = [pd, ctypes.c_int, ctypes.c_double, vp, vp, vp]
        L.dg_apply_projection.argtypes = [pd, ctypes.c_int, vp, vp, vp, vp, vp]
        L.dg_apply_gradient.argtypes = [pd, ctypes.c_int, vp, vp, vp]
        L.dg_prolongate.argtypes = [pd, ctypes.c_int, vp, vp, vp]
        L.dg_gmg_vcycle.argtypes = [pd, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_int32, vp, vp, vp]
        L.dg_gmg_cg_solve.argtypes = [pd, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_int32, vp, vp, ctypes.c_double,
                                       ctypes.c_int32, ctypes.POINTER(CgReport), vp]
        L.dg_restrict.argtypes = [pd, ctypes.c_int, vp, vp, vp]
        L.dg_cg_solve.argtypes = [pd, ctypes.POINTER(CgOpts), vp, vp, ctypes.POINTER(CgReport), vp]
        L.dg_cg_solve_noalloc.argtypes = [pd, ctypes.POINTER(CgOpts), vp, vp, ctypes.POINTER(CgReport), vp]
        L.dg_mass_pcg_solve.argtypes = [pd, ctypes.c_int32, ctypes.c_double, vp, vp, vp, vp, ctypes.c_double,
                                         ctypes.c_int32, ctypes.POINTER(CgReport), vp]
        L.dg_apply_divergence_mixed.argtypes = [pd, ctypes.c_int, vp, vp, vp]
        L.dg_apply_gradient_mixed.argtypes = [pd, ctypes.c_int, vp, vp, vp]
        L.dg_tgv_diagnostics.argtypes = [pd, vp, ctypes.c_double, dp, vp]
        L.dg_dual_splitting_step.argtypes = [pd, ctypes.POINTER(StepOpts), vp, vp, vp, vp,
                                             ctypes.POINTER(StepReport), vp]
        L.dg_dual_splitting_step_conv.argtypes = [pd, ctypes.POINTER(StepOpts), vp, vp, vp, vp, vp, vp,
                                                  ctypes.POINTER(StepReport), vp]
        L.dg_laplace_diagonal.argtypes = [pd, dp]
        L.dg_lgl_nodes.argtypes = [i32, dp]
        L.dg_error_string.argtypes = [ctypes.c_int]
        L.dg_error_string.restype = ctypes.c_char_p
        L.dg_last_error.argtypes = []
        L.dg_last_error.restype = ctypes.c_char_p
        for name in ("dg_apply_laplace", "dg_apply_convective", "dg_vjp_convective", "dg_apply_divergence",
                     "dg_apply_inverse_mass", "dg_apply_helmholtz", "dg_apply_projection", "dg_apply_gradient", "dg_prolongate", "dg_restrict", "dg_gmg_vcycle", "dg_gmg_cg_solve", "dg_cg_solve", "dg_cg_solve_noalloc", "dg_mass_pcg_solve",
                     "dg_apply_divergence_mixed", "dg_apply_gradient_mixed", "dg_tgv_diagnostics",
                     "dg_dual_splitting_step", "dg_dual_splitting_step_conv", "dg_laplace_diagonal", "dg_lgl_nodes"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc, soft_ok=False):
    if rc == DG_OK or (soft_ok and rc > 0):
        return rc
    L = lib()
    raise DgError(rc, f"{L.dg_error_string(rc).decode()}: {L.dg_last_error().decode()}")


def make_desc(degree, n_el, length=None, n_q=0, penalty_factor=1.0, scale=1.0, n_comp=1, lf_factor=1.0):
    if isinstance(n_el, int):
        n_el = (n_el, n_el, n_el)
    if length is None:
        length = (2 * np.pi,) * 3
    elif np.isscalar(length):
        length = (float(length),) * 3
    d = OpDesc()
    d.degree = int(degree)
    for i in range(3):
        d.n_el[i] = int(n_el[i])
        d.length[i] = float(length[i])
    d.n_q = int(n_q)
    d.penalty_factor = float(penalty_factor)
    d.scale = float(scale)
    d.n_comp = int(n_comp)
    d.lf_factor = float(lf_factor)
    return d


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return DG_F64
    if t.dtype == torch.float32:
        return DG_F32
    raise TypeError(f"unsupported dtype {t.dtype}; use float64 or float32")


def _check_tensor(t, name, shape, like=None, dtype=None):
    """Shape and dtype of one argument.  The C ABI takes one dtype per call
    and raw pointers, so an output of another dtype would be written past its
    end: every argument is checked before any launch.  like: a tensor whose
    dtype t must share; dtype: the dtype t must have.  Device and layout are
    checked by _placed, after every shape and dtype."""
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if dtype is None and like is not None:
        dtype = like.dtype
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")


def _placed(first, *others):
    """Every tensor is a contiguous GPU tensor on first's device."""
    for t in (first,) + others:
        if not t.is_cuda:
            raise ValueError("every tensor argument must be a GPU tensor")
        if t.device != first.device:
            raise ValueError(f"tensor arguments on {first.device} and {t.device}: use one device")
        if not t.is_contiguous():
            raise ValueError("every tensor argument must be contiguous")


def _stream(t):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _nel(desc):
    return desc.n_el[0] * desc.n_el[1] * desc.n_el[2]


def apply_laplace(desc, u, out=None):
    """SIPG Laplace apply; u: [N_el, n^3] (n_comp=1) or [3, N_el, n^3] (n_comp=3)."""
    torch = _torch()
    n3 = (desc.degree + 1) ** 3
    shape = (_nel(desc), n3) if desc.n_comp == 1 else (3, _nel(desc), n3)
    _check_tensor(u, "u", shape)
    if out is None:
        out = torch.empty_like(u)
    _check_tensor(out, "out", shape, like=u)
    _placed(u, out)
    _check(lib().dg_apply_laplace(ctypes.byref(desc), _dtype_code(u), ctypes.c_void_p(u.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), _stream(u)))
    return out


def apply_convective(desc, u, out=None):
    """Convective LLF apply; u, out: [3, N_el, n^3]."""
    torch = _torch()
    shape = (3, _nel(desc), (desc.degree + 1) ** 3)
    _check_tensor(u, "u", shape)
    if out is None:
        out = torch.empty_like(u)
    _check_tensor(out, "out", shape, like=u)
    _placed(u, out)
    _check(lib().dg_apply_convective(ctypes.byref(desc), _dtype_code(u), ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), _stream(u)))
    return out


def vjp_max_degree(dtype):
    """Highest degree dg_vjp_convective is built for: 11 in FP64 and FP32."""
    return 11


def vjp_convective(desc, u, w, out=None):
    """J(u)^T w for the convective apply; all [3, N_el, n^3]."""
    torch = _torch()
    shape = (3, _nel(desc), (desc.degree + 1) ** 3)
    _check_tensor(u, "u", shape)
    _check_tensor(w, "w", shape, like=u)
    if out is None:
        out = torch.empty_like(u)
    _check_tensor(out, "out", shape, like=u)
    _placed(u, w, out)
    _check(lib().dg_vjp_convective(ctypes.byref(desc), _dtype_code(u), ctypes.c_void_p(u.data_ptr()),
                                   ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(out.data_ptr()), _stream(u)))
    return out


def apply_divergence(desc, u, out=None):
    """Central-flux divergence d_h(phi_i, u); u: [3, N_el, n^3] -> [N_el, n^3]."""
    torch = _torch()
    n3 = (desc.degree + 1) ** 3
    _check_tensor(u, "u", (3, _nel(desc), n3))
    if out is None:
        out = torch.empty((_nel(desc), n3), dtype=u.dtype, device=u.device)
    _check_tensor(out, "out", (_nel(desc), n3), like=u)
    _placed(u, out)
    _check(lib().dg_apply_divergence(ctypes.byref(desc), _dtype_code(u), ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), _stream(u)))
    return out


def apply_gradient(desc, p, out=None):
    """Central-flux pressure gradient g_h(phi_i e_j, p); p: [N_el, n^3] -> [3, N_el, n^3]."""
    torch = _torch()
    n3 = (desc.degree + 1) ** 3
    _check_tensor(p, "p", (_nel(desc), n3))
    if out is None:
        out = torch.empty((3, _nel(desc), n3), dtype=p.dtype, device=p.device)
    _check_tensor(out, "out", (3, _nel(desc), n3), like=p)
    _placed(p, out)
    _check(lib().dg_apply_gradient(ctypes.byref(desc), _dtype_code(p), ctypes.c_void_p(p.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), _stream(p)))
    return out


def _level_shapes(coarse):
    n3 = (coarse.degree + 1) ** 3
    nc = _nel(coarse)
    if coarse.n_comp == 1:
        return (nc, n3), (8 * nc, n3)
    return (coarse.n_comp, nc, n3), (coarse.n_comp, 8 * nc, n3)


def prolongate(coarse, uc, out=None):
    """Coarse -> fine (every element split in two per direction); coarse describes the coarse mesh."""
    torch = _torch()
    sc, sf = _level_shapes(coarse)
    _check_tensor(uc, "uc", sc)
    if out is None:
        out = torch.empty(sf, dtype=uc.dtype, device=uc.device)
    _check_tensor(out, "out", sf, like=uc)
    _placed(uc, out)
    _check(lib().dg_prolongate(ctypes.byref(coarse), _dtype_code(uc), ctypes.c_void_p(uc.data_ptr()),
                               ctypes.c_void_p(out.data_ptr()), _stream(uc)))
    return out


def restrict(coarse, rf, out=None):
    """Fine -> coarse, the transpose of prolongate."""
    torch = _torch()
    sc, sf = _level_shapes(coarse)
    _check_tensor(rf, "rf", sf)
    if out is None:
        out = torch.empty(sc, dtype=rf.dtype, device=rf.device)
    _check_tensor(out, "out", sc, like=rf)
    _placed(rf, out)
    _check(lib().dg_restrict(ctypes.byref(coarse), _dtype_code(rf), ctypes.c_void_p(rf.data_ptr()),
                             ctypes.c_void_p(out.data_ptr()), _stream(rf)))
    return out


def _levels_and_bounds(lambda_max, levels):
    if lambda_max is None:
        if levels is None:
            raise ValueError("give lambda_max or levels")
        return int(levels), None
    lam = np.ascontiguousarray(lambda_max, dtype=np.float64)
    if levels is not None and int(levels) != len(lam):
        raise ValueError("levels does not match len(lambda_max)")
    return len(lam), lam


def gmg_vcycle(desc, r, lambda_max=None, degree=5, smoothing_range=20.0, coarse_degree=10, out=None, levels=None):
    """z = V r, one V-cycle in r's precision (float64 or float32);
    lambda_max: one bound of D^-1 A per level (finest first), or None: the
    library estimates them (then `levels` gives the number of levels)."""
    torch = _torch()
    shape = (_nel(desc), (desc.degree + 1) ** 3)
    _check_tensor(r, "r", shape)
    if r.dtype not in (torch.float64, torch.float32):
        raise TypeError("r must be float64 or float32")
    if out is None:
        out = torch.empty_like(r)
    _check_tensor(out, "out", shape, like=r)
    nlev, lam = _levels_and_bounds(lambda_max, levels)
    _placed(r, out)
    _check(lib().dg_gmg_vcycle(ctypes.byref(desc), nlev, int(degree), float(smoothing_range),
                               int(coarse_degree), None if lam is None else lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               DG_F32 if r.dtype == torch.float32 else DG_F64, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(out.data_ptr()), _stream(r)))
    return out


def gmg_cg_solve(desc, b, lambda_max=None, x=None, rtol=1e-10, max_iter=200, cycle_dtype=DG_F64, levels=None,
                 degree=5, smoothing_range=20.0, coarse_degree=10):
    """FP64 CG with one V-cycle per iteration (periodic: zero-mean iterates),
    the cycle in FP64 (DG_F64) or FP32 (DG_F32) with the smoother of
    gmg_vcycle; lambda_max: per-level bounds, or None with `levels`
    (estimated by the library); returns (x, report dict, return code)."""
    torch = _torch()
    shape = (_nel(desc), (desc.degree + 1) ** 3)
    _check_tensor(b, "b", shape, dtype=torch.float64)
    if x is None:
        x = torch.zeros_like(b)
    _check_tensor(x, "x", shape, like=b)
    nlev, lam = _levels_and_bounds(lambda_max, levels)
    rep = CgReport()
    _placed(b, x)
    rc = _check(lib().dg_gmg_cg_solve(ctypes.byref(desc), nlev, int(degree), float(smoothing_range),
                                      int(coarse_degree),
                                      None if lam is None else lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      int(cycle_dtype),
                                      ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), float(rtol),
                                      int(max_iter), ctypes.byref(rep), _stream(b)), soft_ok=True)
    return x, rep.as_dict(), rc


def apply_helmholtz(desc, u, mass_factor, out=None):
    """mass_factor M u + scale L u (viscous step); u: [N_el, n^3] or [3, N_el, n^3]."""
    torch = _torch()
    n3 = (desc.degree + 1) ** 3
    shape = (_nel(desc), n3) if desc.n_comp == 1 else (3, _nel(desc), n3)
    _check_tensor(u, "u", shape)
    if out is None:
        out = torch.empty_like(u)
    _check_tensor(out, "out", shape, like=u)
    _placed(u, out)
    _check(lib().dg_apply_helmholtz(ctypes.byref(desc), _dtype_code(u), float(mass_factor),
                                    ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()), _stream(u)))
    return out


def apply_projection(desc, u, tau_d, tau_c, out=None):
    """(M + A_D + A_C) u of the projection step; u: [3, N_el, n^3]; tau_d, tau_c: [N_el]."""
    torch = _torch()
    shape = (3, _nel(desc), (desc.degree + 1) ** 3)
    _check_tensor(u, "u", shape)
    _check_tensor(tau_d, "tau_d", (_nel(desc),), like=u)
    _check_tensor(tau_c, "tau_c", (_nel(desc),), like=u)
    if out is None:
        out = torch.empty_like(u)
    _check_tensor(out, "out", shape, like=u)
    _placed(u, tau_d, tau_c, out)
    _check(lib().dg_apply_projection(ctypes.byref(desc), _dtype_code(u), ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(tau_d.data_ptr()), ctypes.c_void_p(tau_c.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), _stream(u)))
    return out


def apply_inverse_mass(desc, u, out=None):
    """x = M^-1 u, element by element; u: [N_el, n^3] (n_comp=1) or [3, N_el, n^3] (n_comp=3).
    out may be u itself (in place)."""
    torch = _torch()
    n3 = (desc.degree + 1) ** 3
    shape = (_nel(desc), n3) if desc.n_comp == 1 else (3, _nel(desc), n3)
    _check_tensor(u, "u", shape)
    if out is None:
        out = torch.empty_like(u)
    _check_tensor(out, "out", shape, like=u)
    _placed(u, out)
    _check(lib().dg_apply_inverse_mass(ctypes.byref(desc), _dtype_code(u), ctypes.c_void_p(u.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), _stream(u)))
    return out


def cg_solve(desc, b, x=None, precond=DG_PC_CHEB_F32, cheb_degree=5, cheb_range=20.0, rtol=1e-10,
             atol=0.0, max_iter=5000, project_mean=True, noalloc=False):
    """FP64 CG on the SIPG Laplacian; returns (x, report dict, return code).
    noalloc: call dg_cg_solve_noalloc (work memory from the library's static
    array, no device allocation by the library; x must be given then if the
    caller allocates nothing either)."""
    torch = _torch()
    n3 = (desc.degree + 1) ** 3
    _check_tensor(b, "b", (_nel(desc), n3), dtype=torch.float64)
    if x is None:
        x = torch.zeros_like(b)
    _check_tensor(x, "x", (_nel(desc), n3), like=b)
    o = CgOpts()
    o.precond, o.cheb_degree, o.cheb_range = int(precond), int(cheb_degree), float(cheb_range)
    o.rtol, o.atol, o.max_iter, o.project_mean = float(rtol), float(atol), int(max_iter), int(project_mean)
    rep = CgReport()
    _placed(b, x)
    fn = lib().dg_cg_solve_noalloc if noalloc else lib().dg_cg_solve
    rc = _check(fn(ctypes.byref(desc), ctypes.byref(o), ctypes.c_void_p(b.data_ptr()),
                   ctypes.c_void_p(x.data_ptr()), ctypes.byref(rep), _stream(b)), soft_ok=True)
    return x, rep.as_dict(), rc


def mass_pcg_solve(desc, op, b, x=None, mass_factor=0.0, tau_d=None, tau_c=None, rtol=1e-10, max_iter=1000):
    """FP64 CG preconditioned with the inverse mass matrix for the Helmholtz
    (op = DG_OP_HELMHOLTZ) or projection (DG_OP_PROJECTION) equation; returns
    (x, report dict, return code)."""
    torch = _torch()
    shape = (desc.n_comp, _nel(desc), (desc.degree + 1) ** 3) if desc.n_comp > 1 else (_nel(desc), (desc.degree + 1) ** 3)
    _check_tensor(b, "b", shape, dtype=torch.float64)
    if x is None:
        x = torch.zeros_like(b)
    _check_tensor(x, "x", shape, like=b)
    ptr = [None, None]
    if op == DG_OP_PROJECTION:
        for i, t in enumerate((tau_d, tau_c)):
            _check_tensor(t, "tau", (_nel(desc),), like=b)
            ptr[i] = ctypes.c_void_p(t.data_ptr())
    rep = CgReport()
    _placed(b, x, *[t for t in (tau_d, tau_c) if op == DG_OP_PROJECTION])
    rc = _check(lib().dg_mass_pcg_solve(ctypes.byref(desc), int(op), float(mass_factor), ptr[0], ptr[1],
                                        ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), float(rtol),
                                        int(max_iter), ctypes.byref(rep), _stream(b)), soft_ok=True)
    return x, rep.as_dict(), rc


def apply_divergence_mixed(desc, u, out=None):
    """d_h(q_i, u) for the degree-(k-1) pressure basis; u: [3, N_el, (k+1)^3] -> [N_el, k^3]."""
    torch = _torch()
    k = desc.degree
    _check_tensor(u, "u", (3, _nel(desc), (k + 1) ** 3))
    if out is None:
        out = torch.empty((_nel(desc), k ** 3), dtype=u.dtype, device=u.device)
    _check_tensor(out, "out", (_nel(desc), k ** 3), like=u)
    _placed(u, out)
    _check(lib().dg_apply_divergence_mixed(ctypes.byref(desc), _dtype_code(u), ctypes.c_void_p(u.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), _stream(u)))
    return out


def apply_gradient_mixed(desc, p, out=None):
    """g_h(phi_i e_j, p) for the degree-k velocity basis; p: [N_el, k^3] -> [3, N_el, (k+1)^3]."""
    torch = _torch()
    k = desc.degree
    _check_tensor(p, "p", (_nel(desc), k ** 3))
    if out is None:
        out = torch.empty((3, _nel(desc), (k + 1) ** 3), dtype=p.dtype, device=p.device)
    _check_tensor(out, "out", (3, _nel(desc), (k + 1) ** 3), like=p)
    _placed(p, out)
    _check(lib().dg_apply_gradient_mixed(ctypes.byref(desc), _dtype_code(p), ctypes.c_void_p(p.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), _stream(p)))
    return out


def tgv_diagnostics(desc, u, nu):
    """(e_k, eps) of a float64 velocity field u: [3, N_el, (k+1)^3]."""
    torch = _torch()
    _check_tensor(u, "u", (3, _nel(desc), (desc.degree + 1) ** 3), dtype=torch.float64)
    _placed(u)
    out = np.zeros(2)
    _check(lib().dg_tgv_diagnostics(ctypes.byref(desc), ctypes.c_void_p(u.data_ptr()), float(nu),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(u)))
    return float(out[0]), float(out[1])


def dual_splitting_step(desc, u_n, u_nm1=None, p=None, out=None, dt=1e-3, nu=1.0 / 1600, order=2,
                        zeta_d=1.0, zeta_c=1.0, rtol=1e-6, rtol_pressure=None, rtol_projection=None,
                        rtol_viscous=None, atol_pressure=1e-12, max_iter=2000, pressure_precond=DG_STEP_PC_GMG_F32,
                        conv_prev=None, conv_out=None):
    """One dual-splitting step; u_n, u_nm1, out: float64 [3, N_el, (k+1)^3];
    p: float64 [N_el, k^3], initial guess in, P^{n+1} out (zeros if None);
    pressure_precond: DG_STEP_PC_GMG_F32 (one FP32 V-cycle per pressure CG
    iteration, the default) or DG_STEP_PC_CHEB_F32 (FP32 Chebyshev(5)).
    conv_prev: C(u_nm1) from the previous step's conv_out (order 2), or None;
    conv_out: a [3, N_el, (k+1)^3] float64 tensor that receives C(u_n), or
    None (dg_dual_splitting_step_conv when either is given).
    Returns (u_np1, p, report dict, return code)."""
    torch = _torch()
    k = desc.degree
    vshape, pshape = (3, _nel(desc), (k + 1) ** 3), (_nel(desc), k ** 3)
    _check_tensor(u_n, "u_n", vshape, dtype=torch.float64)
    if order == 2:
        if u_nm1 is None:
            raise ValueError("order 2 needs u_nm1")
        _check_tensor(u_nm1, "u_nm1", vshape, like=u_n)
    if p is None:
        p = torch.zeros(pshape, dtype=torch.float64, device=u_n.device)
    _check_tensor(p, "p", pshape, like=u_n)
    if out is None:
        out = torch.empty_like(u_n)
    _check_tensor(out, "out", vshape, like=u_n)
    _placed(u_n, p, out, *([u_nm1] if order == 2 else []))
    o = StepOpts()
    o.order, o.dt, o.nu, o.zeta_d, o.zeta_c = int(order), float(dt), float(nu), float(zeta_d), float(zeta_c)
    o.rtol_pressure = float(rtol if rtol_pressure is None else rtol_pressure)
    o.rtol_projection = float(rtol if rtol_projection is None else rtol_projection)
    o.rtol_viscous = float(rtol if rtol_viscous is None else rtol_viscous)
    o.atol_pressure = float(atol_pressure)
    o.max_iter = int(max_iter)
    o.pressure_precond = int(pressure_precond)
    rep = StepReport()
    nm1 = ctypes.c_void_p(u_nm1.data_ptr()) if order == 2 else None
    if conv_prev is None and conv_out is None:
        rc = _check(lib().dg_dual_splitting_step(ctypes.byref(desc), ctypes.byref(o), ctypes.c_void_p(u_n.data_ptr()),
                                                 nm1, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(p.data_ptr()),
                                                 ctypes.byref(rep), _stream(u_n)), soft_ok=True)
        return out, p, rep.as_dict(), rc
    for t, nm in ((conv_prev, "conv_prev"), (conv_out, "conv_out")):
        if t is not None:
            _check_tensor(t, nm, vshape, like=u_n)
            _placed(u_n, t)
    cp = ctypes.c_void_p(conv_prev.data_ptr()) if conv_prev is not None and order == 2 else None
    co = ctypes.c_void_p(conv_out.data_ptr()) if conv_out is not None else None
    rc = _check(lib().dg_dual_splitting_step_conv(ctypes.byref(desc), ctypes.byref(o), ctypes.c_void_p(u_n.data_ptr()),
                                                  nm1, cp, co, ctypes.c_void_p(out.data_ptr()),
                                                  ctypes.c_void_p(p.data_ptr()), ctypes.byref(rep), _stream(u_n)),
                soft_ok=True)
    return out, p, rep.as_dict(), rc


def laplace_diagonal(desc):
    n3 = (desc.degree + 1) ** 3
    out = np.zeros(n3)
    _check(lib().dg_laplace_diagonal(ctypes.byref(desc), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def lgl_nodes(degree):
    out = np.zeros(degree + 1)
    _check(lib().dg_lgl_nodes(int(degree), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out
