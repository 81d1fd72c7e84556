"""Host logic of bench.py (no GPU): the one-GPU contract, the degree-sweep
meshes and the traffic records keyed by kernel source."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_sweep_meshes_hold_about_1_7e7_dofs_per_component():
    # N = round(256/(k+1)) elements per direction for k = 2..11
    assert [bench.sweep_mesh(k) for k in range(2, 12)] == [85, 64, 51, 43, 37, 32, 28, 26, 23, 21]
    for k in range(2, 12):
        dofs = (bench.sweep_mesh(k) * (k + 1)) ** 3
        assert 1.55e7 < dofs < 1.8e7


def test_convective_flop_count_per_dof():
    # algorithmic flops per component DoF (3 components per element)
    per_dof = {k: bench.conv_flops_per_element(k) / (3 * (k + 1) ** 3) for k in range(2, 12)}
    for k, v in ((2, 285), (5, 392), (7, 502), (11, 720)):
        assert abs(per_dof[k] - v) < 1.0, (k, per_dof[k])
    # grows with the degree over every step of m = floor(3k/2) + 1
    assert all(per_dof[k + 2] > per_dof[k] for k in range(2, 10))


def test_traffic_record_needs_matching_sources(tmp_path, monkeypatch):
    import shutil
    csrc = tmp_path / "paper_1802_01439_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in set(bench.SOURCES["laplace"]) | set(bench.SOURCES["convective"]):
        shutil.copy(os.path.join(ROOT, "paper_1802_01439_amd", "csrc", name), csrc / name)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    tab = {"laplace:k3:f64": {"bytes_per_launch": 123.0, "source_sha": bench.source_hash("laplace")},
           "convective:k3:f64": {"bytes_per_launch": 456.0, "source_sha": "0" * 16}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(tab))
    assert bench.load_traffic("laplace", 3, "f64") == 123.0
    assert bench.load_traffic("convective", 3, "f64") is None     # stale record
    assert bench.load_traffic("laplace", 4, "f64") is None        # no record
    # any change to a file that defines the kernel invalidates the record
    (csrc / "common.h").write_text((csrc / "common.h").read_text() + "\n")
    assert bench.load_traffic("laplace", 3, "f64") is None


@pytest.mark.parametrize("op", ["laplace", "convective", "vjp"])
def test_source_hash_covers_every_defining_file(op):
    for name in bench.SOURCES[op]:
        assert os.path.exists(os.path.join(ROOT, "paper_1802_01439_amd", "csrc", name)), name
    assert len(bench.source_hash(op)) == 16


def _full_record():
    """A record shaped like bench.py's full one at the default sizes: 40
    sweep cases and every extra."""
    sweep = []
    for k in range(2, 12):
        for op in ("laplace", "convective"):
            for dt in ("f64", "f32"):
                row = {"op": op, "k": k, "N": bench.sweep_mesh(k), "dtype": dt, "dofs": 17_000_000,
                       "us": 123.4567, "dofs_per_s": 1.234567e11, "gbs": 1234.5678, "hbm_frac": 0.123456}
                if op == "convective":
                    row.update(tflops=12.3456, alu_frac=0.345678)
                sweep.append(row)
    per_k = {f"k{k}_{dt}": {"us": 100.123, "dofs_per_s": 1.5e11, "hbm_frac": 0.412345}
             for k in range(2, 12) for dt in ("f64", "f32")}
    rep = {"iterations": 203, "matvec_f64": 204, "matvec_f32": 816, "rel_res": 9.9e-11, "true_rel_res": 9.9e-11,
           "lambda_max": 2.345, "seconds_solve": 0.0567, "seconds_setup": 0.01, "rc": 0}
    cg = {"jacobi_f64": rep, "chebyshev5_f32": rep, "speedup_solve": 1.8}
    for cyc in ("f64", "f32"):
        for rt in ("1e-10", "1e-06"):
            cg[f"gmg_vcycle_{cyc}_rtol{rt}"] = rep
    extras = {"inverse_mass_sweep": per_k, "projection_sweep": per_k, "gradient_sweep": per_k,
              "divergence_sweep": per_k, "transfer_sweep": per_k, "cg_k7_24cubed": cg,
              "vjp_k4_32cubed": {"f64": {"dofs_per_s": 2e10, "us": 608.5, "hbm_frac": 0.061},
                                 "f32": {"dofs_per_s": 4e10, "us": 266.0, "hbm_frac": 0.069}},
              "dual_splitting_k7_24cubed": {
                  "dt": 0.01, "dofs": 22_643_712, "ms_per_step": 45.6789, "dofs_steps_per_s": 5e8,
                  "steps": [{"it_pressure": 30, "it_projection": 12, "it_viscous": 3, "kinetic_energy": 0.1249876,
                             "dissipation": 4.6877e-4, "seconds": 0.045, "wall_s": 0.0456}] * 5}}
    return {"metric": bench.METRIC, "value": 8.3e10, "unit": "DoFs/s", "n_gpus": 1, "steps": 20, "warmup": 5,
            "ms_per_step": 16.1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64+f32", "data": "synthetic",
            "config": {"workload": "degree sweep k=2..11: " + "x" * 150, "ops": ["laplace", "convective"],
                       "applies_per_step": 40, "dofs_per_step": 1_360_000_000},
            "roofline": {"bound": "hbm", "achieved": 569.123456, "peak": 8000.0, "unit": "GB/s",
                         "frac": 0.0711234, "traffic": 1.234e9, "kernel": "convective_kernel k=9 f64 N=26",
                         "algorithmic_bytes_per_launch": 843_648_000, "avg_launch_us": 1481.12345,
                         "alu_frac": 0.27712, "alu_peak_tflops": 78.6, "algorithmic_flops_per_launch": 3.2e10},
            "sweep": sweep, "extras": extras,
            "cpu_baseline": {"value": 4.5e6, "unit": "DoFs/s", "cores": 16, "kind": "oracle", "sample": "s" * 2000,
                             "rows": {"inverse_mass": {"dofs_per_s": 1e6, "sample": "x" * 100}},
                             "config5": {"rel_err_vs_oracle_fdm": {"jacobi_f64": 1.23e-11,
                                                                   "chebyshev5_f32": 2.34e-11,
                                                                   "gmg_vcycle_f64": 3.4e-11,
                                                                   "gmg_vcycle_f32": 4.5e-11},
                                         "oracle_fdm_seconds": 1.5}}}


def test_summary_line_is_compact_and_complete():
    full = _full_record()
    line = json.dumps(bench.summary(full))
    assert len(line) < bench.SUMMARY_MAX_CHARS, len(line)
    assert "\n" not in line
    s = json.loads(line)
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in s, key
    assert s["config"]["workload"].startswith("degree sweep")
    rf = s["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert {"value", "unit", "cores", "kind", "sample"} <= set(s["cpu_baseline"])
    assert set(s["sweep"]["hbm_frac"]) == {"laplace_f64", "laplace_f32", "convective_f64", "convective_f32"}
    assert all(len(v) == 10 for v in s["sweep"]["gdofs_per_s"].values())
    assert s["sweep"]["k"] == list(range(2, 12))
    assert s["cpu_baseline"]["config5_rel_err_vs_oracle_fdm"]["chebyshev5_f32"] == 2.3e-11
    assert s["extras"]["dual_splitting_k7_24cubed"]["iterations_p_proj_visc"] == [30, 12, 3]


def test_alu_peak_is_the_unpacked_vector_rate():
    # no packed FP32 instruction is ever generated, so FP32 and FP64 share it
    assert bench.ALU_PEAK_TFLOPS["f32"] == bench.ALU_PEAK_TFLOPS["f64"] == 78.6
