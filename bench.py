#!/usr/bin/env python3
"""Throughput of the matrix-free DG operator applies on one MI355X.

Metric: DoFs/s per operator apply against degree k, FP64 and FP32, with the
fraction of the HBM roofline.  One step is one pass over the degree sweep:
for k = 2..11 on a periodic cube of N = round(256/(k+1)) elements per
direction (about 1.7e7 DoFs per component), the SIPG Laplace apply and the
convective (LLF) apply, each in FP64 and FP32.  Inputs are seeded U[-1,1]
fields resident in HBM before timing starts.  `value` is the total DoFs
processed in a step divided by the step time.

Also measured once, outside the timed steps: the convective VJP on 32^3
elements at k=4 (FP64, FP32) and the pressure-Poisson CG (k=7, 24^3) with the
FP32 Chebyshev preconditioner against FP64 Jacobi-CG.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--kmin 2 --kmax 11]
                    [--ops laplace,convective] [--no-cpu-baseline] [--no-extras]
                    [--sweep-out FILE] [--full-out FILE] [--only OP:K:DTYPE]

stdout gets one compact JSON line (under SUMMARY_MAX_CHARS): the headline,
the roofline of the dominant kernel, the oracle baseline and one GDoF/s and
HBM fraction per operator, dtype and degree; --full-out writes the full
record (every case, every extra) to a file.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DoFs/sec per operator apply vs degree k (FP64, FP32); % HBM roofline"
HBM_PEAK_GBS = 8000.0
# vector ALU peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz =
# 78.6 TFLOP/s, for FP64 and for unpacked FP32 alike (the published FP32
# figure, 157.3, counts packed FP32 instructions, which this code never uses)
ALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 78.6}
# the final stdout line stays under this many characters (a log tail holds it)
SUMMARY_MAX_CHARS = 4096
# algorithmic bytes per DoF of one apply: read the input once, write the output once
BYTES_PER_DOF = {("laplace", "f64"): 16, ("laplace", "f32"): 8,
                 ("convective", "f64"): 16, ("convective", "f32"): 8,
                 ("vjp", "f64"): 24, ("vjp", "f32"): 12}
KERNEL_NAME = {"laplace": "laplace_march_kernel|laplace_batch_kernel", "convective": "convective_kernel", "vjp": "convective_vjp_kernel"}
# every source file that defines each kernel (the traffic record is keyed by their hash)
SOURCES = {"laplace": ("laplace.hip", "laplace_kernels.h", "common.h"),
           "convective": ("convective.hip", "conv_common.h", "basis_ct.h", "common.h"),
           "vjp": ("convective_vjp.hip", "conv_common.h", "basis_ct.h", "common.h")}


def sweep_mesh(k):
    return int(round(256.0 / (k + 1)))


def conv_flops_per_element(k):
    """Algorithmic flops of one element of the convective apply: plain sum
    factorisation (no even-odd savings), each face flux formed by both of its
    elements.  n = k+1 nodes, m = floor(3k/2)+1 Gauss points per direction."""
    n, m = k + 1, (3 * k) // 2 + 1
    fwd = 3 * 2 * (n ** 3 * m + n ** 2 * m ** 2 + n * m ** 3)          # u -> Gauss points
    flux = 21 * m ** 3                                                 # F_cj = s_j W u_c u_j
    back = 3 * 2 * (3 * m ** 3 * n + 3 * m ** 2 * n ** 2 + 2 * m * n ** 3)
    face_sweep = 2 * (n * n * m + n * m * m)                           # 2D sweep of one face layer
    faces = 6 * (2 * 3 * face_sweep + 28 * m * m + 3 * face_sweep)     # traces, LLF flux, integral
    return fwd + flux + back + faces


def source_hash(op):
    h = hashlib.sha256()
    for name in SOURCES[op]:
        with open(os.path.join(ROOT, "paper_1802_01439_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(op, k, dtype):
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    or None if there is none for this kernel or its source has changed."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        tab = json.load(f)
    e = tab.get(f"{op}:k{k}:{dtype}")
    if not e or e.get("source_sha") != source_hash(op):
        return None
    return e.get("bytes_per_launch")


class Case:
    def __init__(self, op, k, N, dtype, dgmf, torch, base):
        self.op, self.k, self.N, self.dtype = op, k, N, dtype
        ncomp = 1 if op == "laplace" else 3
        self.desc = dgmf.make_desc(k, N, n_comp=1)
        tdt = torch.float64 if dtype == "f64" else torch.float32
        n3 = (k + 1) ** 3
        src = base[:ncomp].reshape(ncomp, N ** 3, n3) if ncomp == 3 else base[0]
        self.u = src.to(tdt).contiguous()
        self.out = torch.empty_like(self.u)
        self.dofs = ncomp * N ** 3 * n3
        self.bytes = BYTES_PER_DOF[(op, dtype)] * self.dofs
        self.flops = conv_flops_per_element(k) * N ** 3 if op == "convective" else None
        self.fn = dgmf.apply_laplace if op == "laplace" else dgmf.apply_convective
        self.times = []

    def launch(self):
        self.fn(self.desc, self.u, self.out)

    def name(self):
        return f"{self.op}:k{self.k}:{self.dtype}"


def build_cases(args, torch, dgmf, inputs, dev):
    cases = []
    only = set(args.only.split(",")) if args.only else None
    for k in range(args.kmin, args.kmax + 1):
        N = sweep_mesh(k)
        n3 = (k + 1) ** 3
        need3 = "convective" in args.ops
        shape = (3 if need3 else 1, N ** 3, n3)
        # seeded U[-1,1] (the degree-sweep input), generated once per degree
        base = torch.from_numpy(inputs.uniform(shape, seed=inputs.FIELD_SEED_BASE + 2 + 10 * k)).to(dev)
        for op in args.ops:
            for dtype in ("f64", "f32"):
                c = Case(op, k, N, dtype, dgmf, torch, base)
                if only and c.name() not in only:
                    continue
                cases.append(c)
        del base
    return cases


def config5_against_oracle(solutions, k=7, N=24):
    """Final error of each GPU pressure-Poisson solve (k=7, 24^3, tolerance
    1e-10) against the oracle's FP64 direct solve (fast diagonalisation of the
    Kronecker-sum operator, exact on this mesh) of the same right-hand side:
    relative 2-norm of the difference after removing the constant."""
    from oracle import mesh as M
    from oracle.solvers import fdm_solve
    b = solutions["b"]
    t0 = time.perf_counter()
    x_ref = fdm_solve(b, k, M.cube(N))
    t_fdm = time.perf_counter() - t0
    x_ref = x_ref - x_ref.mean()
    nrm = np.linalg.norm(x_ref)
    err = {name: float(np.linalg.norm((x - x.mean()) - x_ref) / nrm)
           for name, x in solutions.items() if name != "b"}
    return {"rel_err_vs_oracle_fdm": err, "oracle_fdm_seconds": t_fdm}


def cpu_baseline(args, solutions=None):
    """The oracle (plain NumPy, explicit 3D tables) on a bounded sample of the
    sweep: every degree, both operators, a fixed number of elements each.
    With solutions (from the CG extras): also the final errors of the GPU
    solves against the oracle's direct solve."""
    from oracle import mesh as M
    from oracle.convective import convective_apply
    from oracle.laplace import laplace_apply
    from paper_1802_01439_amd import inputs
    try:
        import threadpoolctl
        cores = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    tot_dofs, tot_t, parts = 0, 0.0, []
    budget = 0.6   # seconds of oracle work per (operator, degree), at least
    for k in range(args.kmin, args.kmax + 1):
        N = sweep_mesh(k)
        msh = M.cube(N)
        n3 = (k + 1) ** 3
        u = inputs.uniform((3, msh.N, n3), seed=inputs.FIELD_SEED_BASE + 2 + 10 * k)
        for op in ("laplace", "convective"):
            if op not in args.ops:
                continue
            per_el = n3 if op == "laplace" else 3 * n3
            # calls on doubling runs of consecutive elements until the budget is spent
            ne = max(2, int((2e5 if op == "laplace" else 2e4) / per_el))
            done, t_op = 0, 0.0
            while t_op < budget and done < msh.N:
                E = np.arange(done, min(msh.N, done + ne))
                t0 = time.perf_counter()
                if op == "laplace":
                    laplace_apply(u[0], k, msh, elems=E)
                else:
                    convective_apply(u, k, msh, elems=E)
                t_op += time.perf_counter() - t0
                done += len(E)
                ne *= 2
            tot_dofs += done * per_el
            tot_t += t_op
            parts.append(f"{op} k={k}: {done} el")
    return {"value": tot_dofs / tot_t, "unit": "DoFs/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"oracle (float64, explicit 3D tables) FP64 applies on the first elements of each "
                       f"degree-sweep mesh, k={args.kmin}..{args.kmax}, Laplace and convective, at least "
                       f"{budget} s of oracle work each ({tot_dofs} DoFs in {tot_t:.1f} s; "
                       + ", ".join(parts) + ")"),
            "rows": oracle_rows(args),
            "config5": config5_against_oracle(solutions) if solutions and "b" in solutions else None}


def oracle_rows(args, budget=0.15):
    """The oracle beside the other measured rows: DoFs/s of its FP64 inverse
    mass, gradient, divergence and projection operator on the first elements
    of each degree-sweep mesh (at least `budget` s of work per row and
    degree, one call at the least), for comparison with the GPU figures of the
    same rows in `extras`."""
    from oracle import mesh as M
    from oracle.divergence import divergence_apply
    from oracle.gradient import gradient_apply
    from oracle.mass import inverse_mass_apply
    from oracle.projection import projection_apply
    from paper_1802_01439_amd import inputs
    names = ("inverse_mass", "gradient", "divergence", "projection")
    dofs = dict.fromkeys(names, 0)
    secs = dict.fromkeys(names, 0.0)
    for k in range(args.kmin, args.kmax + 1):
        N = sweep_mesh(k)
        msh = M.cube(N)
        n3 = (k + 1) ** 3
        ne = max(2, int(1e4 / n3))
        nel = min(msh.N, 32 * ne)
        full = np.zeros((3, msh.N, n3))
        full[:, :nel] = inputs.uniform((3, nel, n3), seed=inputs.FIELD_SEED_BASE + 30 + k)
        tau = np.full(msh.N, 1e-3)
        for name in names:
            done, t_k = 0, 0.0
            while (t_k < budget or done == 0) and done + ne <= nel:
                E = np.arange(done, done + ne)
                t0 = time.perf_counter()
                if name == "inverse_mass":
                    inverse_mass_apply(full[0], k, msh, elems=E)
                elif name == "gradient":
                    gradient_apply(full[0], k, msh, elems=E)
                elif name == "divergence":
                    divergence_apply(full, k, msh, elems=E)
                else:
                    projection_apply(full, k, msh, tau, tau, elems=E)
                t_k += time.perf_counter() - t0
                done += ne
            dofs[name] += done * n3 * (3 if name == "projection" else 1)
            secs[name] += t_k
        del full
    out = {name: {"dofs_per_s": dofs[name] / secs[name],
                  "sample": f"k={args.kmin}..{args.kmax}, {dofs[name]} DoFs in {secs[name]:.1f} s"}
           for name in names}
    # prolongation (fine DoFs per second) on a 4 x 2 x 2 coarse mesh per degree
    from oracle.transfer import prolongate
    fd, ft = 0, 0.0
    for k in range(args.kmin, args.kmax + 1):
        coarse = M.Mesh((4, 2, 2), (1.0, 1.0, 1.0))
        n3 = (k + 1) ** 3
        u = inputs.uniform((coarse.N, n3), seed=inputs.FIELD_SEED_BASE + 50 + k)
        prolongate(u, k, coarse)          # the child matrices are built once per degree
        t0 = time.perf_counter()
        prolongate(u, k, coarse)
        ft += time.perf_counter() - t0
        fd += 8 * coarse.N * n3
    out["prolongation"] = {"dofs_per_s": fd / ft, "sample": f"k={args.kmin}..{args.kmax}, 4x2x2 coarse meshes, "
                                                            f"{fd} fine DoFs in {ft:.2f} s"}
    return out


def extras(torch, dgmf, inputs, dev, args, which=("vjp", "cg", "mass", "proj", "mpcg", "grad", "xfer", "vcycle",
                                                  "step"),
           keep=None):
    """Rows measured once per run, outside the timed steps.  keep: a dict that
    receives the pressure-Poisson right-hand side and each solver's solution
    (host arrays), for the comparison with the oracle's direct solve."""
    out = {}
    # inverse mass (element-local, memory bound) and the projection-step
    # operator (M + A_D + A_C, three components, seeded per-element penalty
    # parameters), degree-sweep meshes, seeded U[-1,1]
    if "mass" in which:
        out["inverse_mass_sweep"] = _sweep_extra(torch, dgmf, dev, args, 1, 102, lambda d, x, y, tau:
                                                 dgmf.apply_inverse_mass(d, x, y))
    if "vcycle" in which:
        out["vcycle_k7_24cubed"] = _vcycle_extra(torch, dgmf, inputs, dev)
    if "step" in which:
        try:
            out["dual_splitting_k7_24cubed"] = step_extra(torch, dgmf, inputs, dev)
        except dgmf.DgError as ex:
            out["dual_splitting_k7_24cubed"] = {"error": str(ex)}
    if "xfer" in which:
        out["transfer_sweep"] = _xfer_sweep(torch, dgmf, dev, args)
    if "grad" in which:
        out["gradient_sweep"] = _grad_sweep(torch, dgmf, dev, args, "gradient")
        out["divergence_sweep"] = _grad_sweep(torch, dgmf, dev, args, "divergence")
    if "proj" in which:
        out["projection_sweep"] = _sweep_extra(torch, dgmf, dev, args, 3, 103, lambda d, x, y, tau:
                                               dgmf.apply_projection(d, x, tau[0], tau[1], y))
    # the projection and Helmholtz equations of one time step, k=5, 16^3,
    # solved by CG with the inverse mass as preconditioner (Sec. 3.3)
    try:
        if "mpcg" not in which:
            raise _Skip
        out["mass_pcg_k5_16cubed"] = mass_pcg_extra(torch, dgmf, inputs, dev)
    except _Skip:
        pass
    except dgmf.DgError as ex:
        out["mass_pcg_k5_16cubed"] = {"error": str(ex)}
    # convective VJP, k=4, 32^3, TGV + noise velocity and N(0,1) cotangent
    try:
        if "vjp" not in which:
            raise _Skip
        k, N = 4, 32
        d = dgmf.make_desc(k, N)
        nodes = dgmf.lgl_nodes(k)
        u = inputs.tgv_plus_noise(nodes, (N, N, N), (2 * np.pi,) * 3, seed=inputs.FIELD_SEED_BASE + 3)
        w = inputs.normal(u.shape, seed=inputs.FIELD_SEED_BASE + 3 + inputs.COTANGENT_OFFSET)
        res = {}
        for dtype, tdt in (("f64", torch.float64), ("f32", torch.float32)):
            ut, wt = torch.from_numpy(u).to(dev, tdt), torch.from_numpy(w).to(dev, tdt)
            g = torch.empty_like(ut)
            for _ in range(3):
                dgmf.vjp_convective(d, ut, wt, g)
            torch.cuda.synchronize()
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 20
            s.record()
            for _ in range(reps):
                dgmf.vjp_convective(d, ut, wt, g)
            e.record()
            torch.cuda.synchronize()
            t = s.elapsed_time(e) / 1e3 / reps
            dofs = u.size
            res[dtype] = {"dofs_per_s": dofs / t, "us": t * 1e6,
                          "hbm_frac": BYTES_PER_DOF[("vjp", dtype)] * dofs / t / (HBM_PEAK_GBS * 1e9)}
        out["vjp_k4_32cubed"] = res
        out["vjp_sweep"] = _vjp_sweep(torch, dgmf, dev, args)
    except _Skip:
        pass
    except dgmf.DgError as ex:
        out["vjp_k4_32cubed"] = {"error": str(ex)}
    # pressure Poisson CG, k=7, 24^3, rhs = d_h(TGV + noise), zero mean
    try:
        if "cg" not in which:
            raise _Skip
        k, N = 7, 24
        d = dgmf.make_desc(k, N)
        nodes = dgmf.lgl_nodes(k)
        u = inputs.tgv_plus_noise(nodes, (N, N, N), (2 * np.pi,) * 3, seed=inputs.FIELD_SEED_BASE + 4)
        b = dgmf.apply_divergence(d, torch.from_numpy(u).to(dev))
        b -= b.mean()
        res = {}
        if keep is not None:
            keep["b"] = b.cpu().numpy()
        for name, pc in (("jacobi_f64", dgmf.DG_PC_JACOBI_F64), ("chebyshev5_f32", dgmf.DG_PC_CHEB_F32)):
            x, rep, rc = dgmf.cg_solve(d, b, precond=pc, rtol=1e-10, max_iter=20000)
            rep["rc"] = rc
            res[name] = rep
            if keep is not None:
                keep[name] = x.cpu().numpy()
        res["speedup_solve"] = res["jacobi_f64"]["seconds_solve"] / res["chebyshev5_f32"]["seconds_solve"]
        # CG with one V-cycle per iteration (24^3 -> 3^3, four levels); the
        # library estimates the level bounds of D^-1 A (the Chebyshev CG's
        # Lanczos bound, kept per operator)
        for cyc, cdt in (("f64", dgmf.DG_F64), ("f32", dgmf.DG_F32)):
            for rtol in (1e-10, 1e-6):
                dgmf.gmg_cg_solve(d, b, levels=4, rtol=rtol, cycle_dtype=cdt)       # warm-up
                x, rep, rc = dgmf.gmg_cg_solve(d, b, levels=4, rtol=rtol, cycle_dtype=cdt)
                rep["rc"] = rc
                res[f"gmg_vcycle_{cyc}_rtol{rtol:g}"] = rep
                if keep is not None and rtol == 1e-10:
                    keep[f"gmg_vcycle_{cyc}"] = x.cpu().numpy()
        res["speedup_gmg_vs_jacobi"] = (res["jacobi_f64"]["seconds_solve"]
                                        / res["gmg_vcycle_f64_rtol1e-10"]["seconds_solve"])
        res["speedup_gmg_f32_vs_jacobi"] = (res["jacobi_f64"]["seconds_solve"]
                                            / res["gmg_vcycle_f32_rtol1e-10"]["seconds_solve"])
        out["cg_k7_24cubed"] = res
    except _Skip:
        pass
    except dgmf.DgError as ex:
        out["cg_k7_24cubed"] = {"error": str(ex)}
    return out


def step_extra(torch, dgmf, inputs, dev, k=7, N=24, steps=5):
    """Dual-splitting time steps of the Taylor-Green vortex (Sec. 4: Re = 1600,
    U0 = L = 1, no noise), velocity degree k = 7, pressure 6, on 24^3
    elements; dt from the CFL condition with Cr = 0.125 and r = 1.5
    (Sec. 4.1); the paper's solver tolerances (relative 1e-6, absolute 1e-12
    for the pressure).  One BDF1 start-up step, then `steps` BDF2 steps, each
    timed on the host around the blocking call (three CG solves, the
    convective, divergence, gradient and mass applies, the penalty
    parameters and the diagnostics); each step hands its C(u_n) to the next
    (dg_dual_splitting_step_conv), so a BDF2 step applies the convective
    operator once."""
    L = 2 * np.pi
    h = L / N
    dt, nu = 0.125 / k ** 1.5 * h, 1.0 / 1600
    x, y, z = inputs.node_positions(dgmf.lgl_nodes(k), (N, N, N), (L,) * 3)
    u0 = torch.from_numpy(inputs.taylor_green(x, y, z)).to(dev)
    d = dgmf.make_desc(k, N)

    def run(pc):
        bufs = [u0.clone(), torch.empty_like(u0), torch.empty_like(u0)]
        # C(u_n) of each step is kept for the next one (its C(u_{n-1}))
        conv = [torch.empty_like(u0), torch.empty_like(u0)]
        _, p, rep0, rc = dgmf.dual_splitting_step(d, bufs[0], out=bufs[1], dt=dt, nu=nu, order=1, pressure_precond=pc,
                                                  conv_out=conv[0])
        res = {"dt": dt, "dofs": N ** 3 * (3 * (k + 1) ** 3 + k ** 3), "startup": rep0, "rc": [rc], "steps": []}
        cur, prev, nxt = 1, 0, 2
        for j in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, p, rep, rc = dgmf.dual_splitting_step(d, bufs[cur], bufs[prev], p=p, out=bufs[nxt], dt=dt, nu=nu,
                                                     order=2, pressure_precond=pc, conv_prev=conv[j % 2],
                                                     conv_out=conv[(j + 1) % 2])
            res["steps"].append(dict(rep, wall_s=time.perf_counter() - t0))
            res["rc"].append(rc)
            cur, prev, nxt = nxt, cur, prev
        w = [r["wall_s"] for r in res["steps"]]
        res["ms_per_step"] = 1e3 * float(np.median(w))
        res["dofs_steps_per_s"] = res["dofs"] / float(np.median(w))
        return res

    # pressure CG with one FP32 V-cycle per iteration (24^3 -> 3^3, four
    # levels; Sec. 3.3), then with the FP32 Chebyshev(5) smoother
    res = run(dgmf.DG_STEP_PC_GMG_F32)
    res["chebyshev_pressure"] = run(dgmf.DG_STEP_PC_CHEB_F32)
    return res


def mass_pcg_extra(torch, dgmf, inputs, dev, k=5, N=16):
    """Velocity = TGV + N(0, 0.01) noise at the LGL nodes; time step from the
    CFL condition with Cr = 0.2, r = 1.5, U0 = 1; penalty parameters
    tau_D = |u|_e h/(k+1) dt, tau_C = |u|_e dt (zeta = 1) with |u|_e the mean
    nodal velocity magnitude of the element; Helmholtz with gamma_0 = 3/2
    (BDF2) and nu = 1/1600.  Right-hand sides M u and (1/dt) M u, zero start,
    relative tolerance 1e-6 (the paper's) and 1e-10.  Bytes per iteration:
    112 per DoF (operator 16, p.q 16, the fused x/r update, inverse mass and
    r.r, r.z 56, direction update 24)."""
    L = 2 * np.pi
    h = L / N
    dt = 0.2 / k ** 1.5 * h / 1.0
    nodes = dgmf.lgl_nodes(k)
    u = inputs.tgv_plus_noise(nodes, (N, N, N), (L,) * 3, seed=inputs.FIELD_SEED_BASE + 2)
    umag = np.sqrt((u ** 2).sum(axis=0)).mean(axis=1)
    td = umag * h / (k + 1) * dt
    tc = umag * dt
    d3 = dgmf.make_desc(k, N, n_comp=3)
    ut = torch.from_numpy(u).to(dev)
    b = torch.empty_like(ut)
    dm = dgmf.make_desc(k, N, n_comp=3, scale=0.0)   # Helmholtz with a zero Laplace scale: M u
    dgmf.apply_helmholtz(dm, ut, 1.0, b)
    tdd, tcd = torch.from_numpy(td).to(dev), torch.from_numpy(tc).to(dev)
    dofs = u.size
    res = {"dt": dt, "dofs": dofs}
    dh = dgmf.make_desc(k, N, n_comp=3, scale=1.0 / 1600)
    for rtol in (1e-6, 1e-10):
        for name, call in (
                ("projection", lambda: dgmf.mass_pcg_solve(d3, dgmf.DG_OP_PROJECTION, b, tau_d=tdd, tau_c=tcd,
                                                           rtol=rtol)),
                ("helmholtz", lambda: dgmf.mass_pcg_solve(dh, dgmf.DG_OP_HELMHOLTZ, b / dt, mass_factor=1.5 / dt,
                                                          rtol=rtol))):
            call()   # warm-up (tables, work vectors)
            torch.cuda.synchronize()
            x, rep, rc = call()
            it = max(rep["iterations"], 1)
            per_it = rep["seconds_solve"] / it
            res[f"{name}_rtol{rtol:g}"] = {"rc": rc, "iterations": rep["iterations"],
                                          "seconds_solve": rep["seconds_solve"],
                                          "us_per_iteration": per_it * 1e6,
                                          "true_rel_res": rep["true_rel_res"],
                                          "hbm_frac_per_iteration": 112 * dofs / per_it / (HBM_PEAK_GBS * 1e9)}
    return res


def _vcycle_extra(torch, dgmf, inputs, dev, k=7, N=24, levels=4, reps=5):
    """One V-cycle, FP64 and FP32, on the pressure Poisson size (k=7, 24^3 ->
    12^3 -> 6^3 -> 3^3), Chebyshev degree 5, coarse degree 10.  The per-level bounds
    of D^-1 A are the library's own Lanczos estimates (computed once per
    operator and kept).  Wall time per cycle includes the cycle's set-up
    (level diagonals, work vectors) and its final synchronisation."""
    d = dgmf.make_desc(k, N)
    g = torch.Generator(device=dev)
    g.manual_seed(108)
    r = torch.rand((N ** 3, (k + 1) ** 3), generator=g, dtype=torch.float64, device=dev) - 0.5
    r -= r.mean()
    res = {"levels": levels, "fine_operator_applications": 2 * (5 - 1) + 2}
    for name, rr in (("f64", r), ("f32", r.float())):
        z = dgmf.gmg_vcycle(d, rr, levels=levels)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            dgmf.gmg_vcycle(d, rr, levels=levels, out=z)
        t = (time.perf_counter() - t0) / reps
        res["ms_per_cycle" if name == "f64" else "ms_per_cycle_f32"] = t * 1e3
    return res


def _xfer_sweep(torch, dgmf, dev, args):
    """h-multigrid prolongation and restriction between the mesh of N/2 and N
    elements per direction, N = the degree-sweep mesh rounded to even;
    seeded U[-1,1] input, 4 input/output pairs in rotation.  Algorithmic
    bytes: 9/8 values per fine DoF either way (coarse read or written once,
    fine written or read once)."""
    res = {}
    R = 4
    for k in range(args.kmin, args.kmax + 1):
        Nc = sweep_mesh(k) // 2
        d = dgmf.make_desc(k, Nc)
        n3 = (k + 1) ** 3
        g = torch.Generator(device=dev)
        g.manual_seed(106 + 10 * k)
        coarse = torch.rand((Nc ** 3, n3), generator=g, dtype=torch.float64, device=dev) * 2 - 1
        fine = torch.rand((8 * Nc ** 3, n3), generator=g, dtype=torch.float64, device=dev) * 2 - 1
        nf = fine.numel()
        for dtype, tdt in (("f64", torch.float64), ("f32", torch.float32)):
            es = 8 if dtype == "f64" else 4
            for name, src, call in (("prolongate", coarse, dgmf.prolongate), ("restrict", fine, dgmf.restrict)):
                xs = [src.to(tdt) for _ in range(R)]
                ys = [call(d, xs[i]) for i in range(R)]
                torch.cuda.synchronize()
                s0, e0 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                reps = 5 * R
                s0.record()
                for i in range(reps):
                    call(d, xs[i % R], ys[i % R])
                e0.record()
                torch.cuda.synchronize()
                t = s0.elapsed_time(e0) / 1e3 / reps
                res[f"{name}_k{k}_{dtype}"] = {"us": t * 1e6, "fine_dofs_per_s": nf / t,
                                               "hbm_frac": 9 / 8 * es * nf / t / (HBM_PEAK_GBS * 1e9)}
                del xs, ys
        del coarse, fine
    return res


def _grad_sweep(torch, dgmf, dev, args, op):
    """Pressure gradient (scalar -> 3 components) or velocity divergence
    (3 components -> scalar) on the degree-sweep meshes, seeded U[-1,1] input;
    4 input/output pairs in rotation.  Algorithmic bytes: input read once,
    output written once, 4 values per pressure DoF either way."""
    res = {}
    R = 4
    grad = op == "gradient"
    for k in range(args.kmin, args.kmax + 1):
        N = sweep_mesh(k)
        d = dgmf.make_desc(k, N)
        g = torch.Generator(device=dev)
        g.manual_seed((104 if grad else 105) + 10 * k)
        scalar = (N ** 3, (k + 1) ** 3)
        vector = (3,) + scalar
        base = torch.rand(scalar if grad else vector, generator=g, dtype=torch.float64, device=dev) * 2 - 1
        for dtype, tdt in (("f64", torch.float64), ("f32", torch.float32)):
            xs = [base.to(tdt) for _ in range(R)]
            ys = [torch.empty(vector if grad else scalar, dtype=tdt, device=dev) for _ in range(R)]
            call = dgmf.apply_gradient if grad else dgmf.apply_divergence
            for i in range(R):
                call(d, xs[i], ys[i])
            torch.cuda.synchronize()
            s0, e0 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 5 * R
            s0.record()
            for i in range(reps):
                call(d, xs[i % R], ys[i % R])
            e0.record()
            torch.cuda.synchronize()
            t = s0.elapsed_time(e0) / 1e3 / reps
            n = N ** 3 * (k + 1) ** 3
            nbytes = 4 * (8 if dtype == "f64" else 4) * n
            res[f"k{k}_{dtype}"] = {"us": t * 1e6, "dofs_per_s": n / t,
                                    "hbm_frac": nbytes / t / (HBM_PEAK_GBS * 1e9)}
            del xs, ys
        del base
    return res


def _sweep_extra(torch, dgmf, dev, args, comps, seed, apply):
    """Time one element-local operator over the degree-sweep meshes.  4 input/
    output pairs in rotation, so that the 256 MB Infinity Cache does not hold
    a pair between its repeats.  Algorithmic bytes: read and write every DoF
    once, plus the two per-element penalty parameters (projection only)."""
    res = {}
    R = 4
    for k in range(args.kmin, args.kmax + 1):
        N = sweep_mesh(k)
        d = dgmf.make_desc(k, N, n_comp=comps)
        g = torch.Generator(device=dev)
        g.manual_seed(seed + 10 * k)
        shape = (N ** 3, (k + 1) ** 3) if comps == 1 else (comps, N ** 3, (k + 1) ** 3)
        base = torch.rand(shape, generator=g, dtype=torch.float64, device=dev) * 2 - 1
        h2 = (2 * np.pi / N) ** 2
        taus = [(0.1 + 0.9 * torch.rand(N ** 3, generator=g, dtype=torch.float64, device=dev)) * h2
                for _ in range(2)]
        for dtype, tdt in (("f64", torch.float64), ("f32", torch.float32)):
            xs = [base.to(tdt) for _ in range(R)]
            ys = [torch.empty_like(xs[0]) for _ in range(R)]
            tau = [t.to(tdt) for t in taus]
            for i in range(R):
                apply(d, xs[i], ys[i], tau)
            torch.cuda.synchronize()
            s0, e0 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 5 * R
            s0.record()
            for i in range(reps):
                apply(d, xs[i % R], ys[i % R], tau)
            e0.record()
            torch.cuda.synchronize()
            t = s0.elapsed_time(e0) / 1e3 / reps
            n = xs[0].numel()
            es = 8 if dtype == "f64" else 4
            nbytes = 2 * es * n + (2 * es * N ** 3 if comps == 3 else 0)
            res[f"k{k}_{dtype}"] = {"us": t * 1e6, "dofs_per_s": n / t,
                                    "hbm_frac": nbytes / t / (HBM_PEAK_GBS * 1e9)}
            del xs, ys, tau
        del base, taus
    return res


def _vjp_sweep(torch, dgmf, dev, args):
    """dg_vjp_convective over the degree-sweep meshes: seeded U[-1,1] velocity
    and cotangent, two input sets in rotation.  Algorithmic bytes: u and w
    read once, g written once (24 B per DoF in FP64, 12 B in FP32)."""
    res = {}
    R = 2
    for k in range(args.kmin, args.kmax + 1):
        N = sweep_mesh(k)
        d = dgmf.make_desc(k, N)
        g = torch.Generator(device=dev)
        g.manual_seed(910 + k)
        shape = (3, N ** 3, (k + 1) ** 3)
        for dtype, tdt in (("f64", torch.float64), ("f32", torch.float32)):
            us = [(torch.rand(shape, generator=g, dtype=torch.float64, device=dev) * 2 - 1).to(tdt) for _ in range(R)]
            ws = [(torch.rand(shape, generator=g, dtype=torch.float64, device=dev) * 2 - 1).to(tdt) for _ in range(R)]
            gs = [torch.empty_like(us[0]) for _ in range(R)]
            for i in range(R):
                dgmf.vjp_convective(d, us[i], ws[i], gs[i])
            torch.cuda.synchronize()
            s0, e0 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 3 * R
            s0.record()
            for i in range(reps):
                dgmf.vjp_convective(d, us[i % R], ws[i % R], gs[i % R])
            e0.record()
            torch.cuda.synchronize()
            t = s0.elapsed_time(e0) / 1e3 / reps
            n = us[0].numel()
            res[f"k{k}_{dtype}"] = {"us": t * 1e6, "dofs_per_s": n / t,
                                    "hbm_frac": BYTES_PER_DOF[("vjp", dtype)] * n / t / (HBM_PEAK_GBS * 1e9)}
            del us, ws, gs
    return res


class _Skip(Exception):
    pass


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kmin", type=int, default=2)
    ap.add_argument("--kmax", type=int, default=11)
    ap.add_argument("--ops", default="laplace,convective")
    ap.add_argument("--only", default="", help="comma list of op:kK:dtype cases to run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--sweep-out", default="")
    ap.add_argument("--full-out", default="", help="write the full record (every case, all extras) to this file")
    ap.add_argument("--extras-only", default="",
                    help="diagnostic: run only these extras (vjp,cg,mass,proj,mpcg,grad,xfer,vcycle,step), print them as one JSON line, no sweep")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="also run one plain device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    args.ops = [o for o in args.ops.split(",") if o]
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1802_01439_amd import dgmf, inputs
    dgmf.lib()   # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.extras_only:
        which = tuple(w for w in args.extras_only.split(",") if w)
        if args.calib_copy:
            a = torch.ones(args.calib_copy // 8, dtype=torch.float64, device=dev)
            c = torch.empty_like(a)
            c.copy_(a)
            torch.cuda.synchronize()
            del a, c
        print(json.dumps({"extras": extras(torch, dgmf, inputs, dev, args, which)}), flush=True)
        return
    print(f"[bench] building inputs for k={args.kmin}..{args.kmax} ops={args.ops}", file=sys.stderr, flush=True)
    cases = build_cases(args, torch, dgmf, inputs, dev)
    torch.cuda.synchronize()
    if args.calib_copy:
        a = torch.ones(args.calib_copy // 8, dtype=torch.float64, device=dev)
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        del a, c
    stream = torch.cuda.current_stream()
    for w in range(args.warmup):
        for c in cases:
            c.launch()
    torch.cuda.synchronize()
    print(f"[bench] {len(cases)} applies per step; warmup done", file=sys.stderr, flush=True)
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in cases]
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        for c, (a, b) in zip(cases, evs[s]):
            a.record(stream)
            c.launch()
            b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for s in range(args.steps):
        for c, (a, b) in zip(cases, evs[s]):
            c.times.append(a.elapsed_time(b) / 1e3)
    dofs_step = sum(c.dofs for c in cases)
    ms_step = wall / args.steps * 1e3
    sweep = []
    for c in cases:
        t = float(np.mean(c.times))
        row = {"op": c.op, "k": c.k, "N": c.N, "dtype": c.dtype, "dofs": c.dofs, "us": t * 1e6,
               "dofs_per_s": c.dofs / t, "gbs": c.bytes / t / 1e9,
               "hbm_frac": c.bytes / t / 1e9 / HBM_PEAK_GBS}
        if c.flops:
            row["tflops"] = c.flops / t / 1e12
            row["alu_frac"] = c.flops / t / 1e12 / ALU_PEAK_TFLOPS[c.dtype]
        sweep.append(row)
    dom = max(cases, key=lambda c: np.mean(c.times))
    tdom = float(np.mean(dom.times))
    traffic = load_traffic(dom.op, dom.k, dom.dtype)
    roofline = {"bound": "hbm", "achieved": dom.bytes / tdom / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dom.bytes / tdom / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": f"{KERNEL_NAME[dom.op]} k={dom.k} {dom.dtype} N={dom.N}",
                "algorithmic_bytes_per_launch": dom.bytes, "avg_launch_us": tdom * 1e6}
    if dom.flops:   # the convective apply also has a vector-ALU roofline
        roofline["alu_frac"] = dom.flops / tdom / 1e12 / ALU_PEAK_TFLOPS[dom.dtype]
        roofline["alu_peak_tflops"] = ALU_PEAK_TFLOPS[dom.dtype]
        roofline["algorithmic_flops_per_launch"] = dom.flops
    res = {"metric": METRIC, "value": dofs_step / (ms_step / 1e3), "unit": "DoFs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
           "config": {"workload": (f"degree sweep k={args.kmin}..{args.kmax}: SIPG Laplace and LLF convective "
                                   f"applies, FP64 and FP32, periodic cube N=round(256/(k+1)), ~1.7e7 "
                                   f"DoFs per component, seeded U[-1,1]"),
                      "ops": args.ops, "applies_per_step": len(cases), "dofs_per_step": dofs_step},
           "roofline": roofline}
    if args.sweep_out:
        with open(args.sweep_out, "w") as f:
            json.dump(sweep, f, indent=1)
    res["sweep"] = [{k_: (round(v, 4) if isinstance(v, float) else v) for k_, v in r.items()} for r in sweep]
    del cases
    torch.cuda.empty_cache()
    solutions = {}
    if not args.no_extras:
        print("[bench] extras: inverse mass, gradient, projection, mass-preconditioned solves, VJP, CG",
              file=sys.stderr, flush=True)
        res["extras"] = extras(torch, dgmf, inputs, dev, args, keep=solutions)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(args, solutions)
    if args.full_out:
        with open(args.full_out, "w") as f:
            json.dump(res, f, indent=1)
    sys.stderr.flush()
    print(json.dumps(summary(res)), flush=True)


def _r(x, nd=3):
    return None if x is None else float(f"{x:.{nd}g}")


def summary(res):
    """The one stdout line: the contract's fields, the roofline of the
    dominant kernel, the oracle baseline, one GDoF/s and one HBM fraction per
    (operator, dtype) and degree, and a few figures of the extras.  The full
    record (every per-case number, all extras) goes to --full-out."""
    out = {k: res[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                               "higher_is_better", "scaling", "vs_baseline", "dtype", "data")}
    out["config"] = {"workload": res["config"]["workload"], "applies_per_step": res["config"]["applies_per_step"],
                     "dofs_per_step": res["config"]["dofs_per_step"]}
    rf = res["roofline"]
    out["roofline"] = {k: (_r(v, 4) if isinstance(v, float) else v) for k, v in rf.items()
                       if k not in ("algorithmic_flops_per_launch",)}
    gd, hf, ks = {}, {}, {}
    for r in res.get("sweep", []):
        key = f"{r['op']}_{r['dtype']}"
        gd.setdefault(key, []).append(round(r["dofs_per_s"] / 1e9, 1))
        hf.setdefault(key, []).append(round(r["hbm_frac"], 3))
        ks.setdefault(key, []).append(r["k"])
    ks_all = sorted({k for v in ks.values() for k in v})
    out["sweep"] = {"k": ks_all, "gdofs_per_s": gd, "hbm_frac": hf}
    ex = res.get("extras") or {}
    xs = {}
    v = ex.get("vjp_k4_32cubed") or {}
    for dt in ("f64", "f32"):
        if dt in v:
            xs[f"vjp_k4_32cubed_{dt}"] = {"us": _r(v[dt]["us"]), "hbm_frac": _r(v[dt]["hbm_frac"])}
    cg = ex.get("cg_k7_24cubed") or {}
    if "jacobi_f64" in cg:
        xs["cg_k7_24cubed_seconds_to_1e-10"] = {
            n: _r(cg[key]["seconds_solve"]) for n, key in (("jacobi_f64", "jacobi_f64"),
                                                           ("chebyshev5_f32", "chebyshev5_f32"),
                                                           ("gmg_f64", "gmg_vcycle_f64_rtol1e-10"),
                                                           ("gmg_f32", "gmg_vcycle_f32_rtol1e-10")) if key in cg}
        xs["cg_k7_24cubed_iterations"] = {n: cg[n]["iterations"] for n in
                                          ("jacobi_f64", "chebyshev5_f32", "gmg_vcycle_f64_rtol1e-10",
                                           "gmg_vcycle_f32_rtol1e-10") if n in cg}
    st = ex.get("dual_splitting_k7_24cubed") or {}
    if "ms_per_step" in st:
        last = st["steps"][-1]
        xs["dual_splitting_k7_24cubed"] = {"ms_per_step": _r(st["ms_per_step"]),
                                           "iterations_p_proj_visc": [last["it_pressure"], last["it_projection"],
                                                                      last["it_viscous"]],
                                           "e_k": _r(last["kinetic_energy"], 6), "eps": _r(last["dissipation"], 4)}
        g = st.get("chebyshev_pressure") or {}
        if "ms_per_step" in g:
            xs["dual_splitting_k7_24cubed"]["chebyshev_pressure"] = {"ms_per_step": _r(g["ms_per_step"]),
                                                                     "it_pressure": g["steps"][-1]["it_pressure"]}
    for name in ("vjp_sweep", "inverse_mass_sweep", "projection_sweep", "gradient_sweep", "divergence_sweep"):
        v = ex.get(name)
        if isinstance(v, dict) and v:
            fr = [e["hbm_frac"] for e in v.values() if isinstance(e, dict) and "hbm_frac" in e]
            if fr:
                xs[name + "_hbm_frac_range"] = [_r(min(fr), 2), _r(max(fr), 2)]
    if xs:
        out["extras"] = xs
    cb = res.get("cpu_baseline")
    if cb:
        out["cpu_baseline"] = {"value": _r(cb["value"]), "unit": cb["unit"], "cores": cb["cores"], "kind": cb["kind"],
                               "sample": ("oracle FP64 applies on the first elements of each degree-sweep mesh, "
                                          "Laplace and convective, k=2..11 (full description in the full record)")}
        c5 = cb.get("config5")
        if c5:
            out["cpu_baseline"]["config5_rel_err_vs_oracle_fdm"] = {k: _r(v, 2) for k, v in
                                                                    c5["rel_err_vs_oracle_fdm"].items()}
    return out

if __name__ == "__main__":
    main()
