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
