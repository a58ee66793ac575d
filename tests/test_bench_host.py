"""Host logic of bench.py (no GPU): the one-GPU guard, the roofline arithmetic on the
method's own work, and the validity rule of the stored traffic record."""
import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def _res(form, kms, nonzero, tile, dense):
    return {"form": form, "kms": kms, "chunk": 4,
            "work": {"nonzero_flops": nonzero, "tile_flops": tile, "dense_flops": dense}}


def test_roofline_is_eight_bytes_per_update_over_the_kernel_time():
    spec = types.SimpleNamespace(cells=1024 * 1024, q=2048, nx=1024, ny=1024, n_azim=64)
    res = _res("banded", {"contraction": 7.2}, 1.546e11, 1.57e11, 2 * 2048.0 ** 2 * 1024 ** 2)
    r = bench.roofline(res, spec, "f32")
    cq = spec.cells * spec.q
    assert r["kernel"] == "banded_euler_kernel<64, true>" and r["bound"] == "hbm"
    assert r["achieved"] == pytest.approx(8 * cq / 7.2e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["method_TFLOPs"] == pytest.approx(1.546e11 / 7.2e-3 / 1e12)
    assert r["intensity_flop_per_byte"] == pytest.approx(1.546e11 / (8 * cq))
    assert r["ridge_flop_per_byte"] == pytest.approx(78.6e12 / 8e12)   # FP32 VALU
    assert r["executed_over_nonzero"] == pytest.approx(1.57 / 1.546)


def test_separate_form_takes_the_slower_of_its_two_kernels():
    spec = types.SimpleNamespace(cells=400 * 400, q=512, nx=400, ny=400, n_azim=32)
    res = _res("separate", {"contraction": 0.24, "stream_collide": 0.19}, 1.0, 2.0, 4.0)
    assert bench.roofline(res, spec, "f32")["kernel"] == "gemm_f32_kernel<false>"
    k = bench.roofline(res, spec, "f32")["kernels"]
    cq = spec.cells * spec.q
    assert k["stream_collide"]["frac"] == pytest.approx(12 * cq / 0.19e-3 / 8e12)
    assert k["contraction"]["executed_frac"] == pytest.approx(2.0 / 0.24e-3 / 157.3e12)
    assert k["contraction"]["nonzero_frac"] == pytest.approx(1.0 / 0.24e-3 / 157.3e12)
    res["kms"] = {"contraction": 0.10, "stream_collide": 0.19}
    assert bench.roofline(res, spec, "f32")["kernel"] == "stream_collide_flat_kernel<false>"
    assert bench.roofline(_res("fused", {"contraction": 0.4}, 1.0, 1.0, 1.0), spec,
                          "bf16")["ridge_flop_per_byte"] == pytest.approx(2500e12 / 8e12)


def test_traffic_record_is_void_once_the_kernel_code_changes(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("int a; // note\n/* block */ int b;\n")
    h0 = bench.kernel_source_hash(str(src))
    src.write_text("int  a;   // other note\n\nint b;\n")
    assert bench.kernel_source_hash(str(src)) == h0          # comments and blank space only
    src.write_text("int a; int c;\n")
    assert bench.kernel_source_hash(str(src)) != h0
    rec = {"kernel_code_sha256": h0, "workload_nx_ny_q": [4, 4, 8],
           "kernels": {"k<1>": {"fetch_bytes": 3.0, "write_bytes": 2.0}}}
    f = tmp_path / "t.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    spec = types.SimpleNamespace(nx=4, ny=4, q=8)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda path=None: h0)
    assert bench.measured_traffic("k<1>", spec) == 5.0
    assert bench.measured_traffic("k<1>", types.SimpleNamespace(nx=4, ny=4, q=16)) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda path=None: "other")
    assert bench.measured_traffic("k<1>", spec) is None



def test_banded_kernel_instance_follows_the_row_width():
    res = _res("banded", {"contraction": 0.3}, 1e9, 1e9, 1e12)
    narrow = types.SimpleNamespace(cells=400 * 400, q=512, nx=400, ny=400, n_azim=32)
    wide = types.SimpleNamespace(cells=1024 * 4, q=512, nx=1024, ny=4, n_azim=32)
    assert bench.dominant_kernel(res, narrow, "f32")[0] == "banded_euler_kernel<32, false>"
    assert bench.dominant_kernel(res, wide, "f32")[0] == "banded_euler_kernel<32, true>"


def test_banded_reduced_precision_kernel_named_by_family():
    spec = types.SimpleNamespace(cells=1024 * 1024, q=2048, nx=1024, ny=1024, n_azim=64)
    res = _res("banded", {"contraction": 10.7}, 1.5e11, 8.8e12, 2 * 2048.0 ** 2 * 1024 ** 2)
    r = bench.roofline(res, spec, "bf16")
    assert r["kernel"] == "banded_lp_kernel<64, 1, R>"
    assert r["compute_peak_TFLOPs"] == 2500.0
    assert r["frac"] == pytest.approx(8 * spec.cells * spec.q / 10.7e-3 / 1e9 / 8000.0)
