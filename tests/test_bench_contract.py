"""The benchmark's contract, on the CPU: one GPU only (a message and exit status 2
for more), HBM traffic taken from a counter record only while the kernel source it
was taken on is unchanged, the stage byte model, and the committed headline record's
keys and internal consistency."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_follows_kernel_source(tmp_path, monkeypatch):
    src = tmp_path / "paper_1510_00903_amd" / "csrc"
    src.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (src / "kernels.hip").write_bytes(b"kernel source A")
    sha = hashlib.sha256(b"kernel source A").hexdigest()
    rec = {"kernel": "k", "bytes_per_dispatch": 123456789, "kernels_sha256": sha}
    (tmp_path / "profiles" / "traffic_contract_f64_16c.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_for("contract", "f64", 16) == 123456789
    assert bench.traffic_for("contract", "f64", 32) is None          # no record for that lattice
    assert bench.traffic_for("contract", "f32", 16) is None          # nor for that form
    (src / "kernels.hip").write_bytes(b"kernel source B")             # the kernels changed since
    assert bench.traffic_for("contract", "f64", 16) is None


def test_stage_model_bytes():
    # 16^3, 8,280 components per sink spin, FP64: the grouped field is 2 x 8280 x 4096 x 16 B
    nc, L, b = 8280, 16, 16
    field = 2 * nc * L ** 3 * b
    assert field == 1_085_276_160
    assert bench.stage_model("blocks", L, nc, 52, b) == L ** 3 * 2 * 144 * b + field
    assert bench.stage_model("fft_forward", L, nc, 52, b) == 2 * field
    assert bench.stage_model("fft_inverse", L, nc, 52, b) == 2 * 52 * 16 * L ** 3 * b
    assert bench.stage_model("no such stage", L, nc, 52, b) is None


def test_committed_headline_record():
    path = os.path.join(ROOT, "profiles", "bench_16c32_52ch_f64.json")
    d = json.load(open(path))
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["higher_is_better"] is True and d["dtype"] == "f64"
    assert "workload" in d["config"]
    # value = site-channels per step / seconds per step
    spc = d["config"]["site_channels_per_step"]
    assert spc == 16 ** 3 * 32 * 52
    assert d["value"] == pytest.approx(spc / (d["ms_per_step"] * 1e-3), rel=1e-3)
    r = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-3)
    assert r["peak"] == 78.6 and r["unit"] == "TFLOP/s"
    c = d["cpu_baseline"]
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in c, k
    assert c["kind"] == "oracle" and c["cores"] >= 1
