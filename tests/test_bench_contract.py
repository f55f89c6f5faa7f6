"""The bench's command-line contract: one JSON line with the metric, the
throughput, the roofline object of the dominant kernel and the CPU oracle
baseline; a request for more than one GPU is refused with a message; the
counter traffic is read from a committed profile only when that profile was
taken on the current kernel sources."""
import json
import os
import sys

import pytest

import bench


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    assert bench.main() == 2
    d = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert "error" in d and "one GPU" in d["error"]


def test_counter_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    for f in bench.KERNEL_SOURCES:
        os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
        with open(os.path.join(bench.ROOT, f), "rb") as src, open(tmp_path / f, "wb") as dst:
            dst.write(src.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    t, note = bench.counter_traffic("column_50cm", "fp64")
    assert t is None and "no counter profile" in note
    rec = dict(source_sha16=bench.kernel_source_sha16(), fetch_kib=1000.0, write_kib=500.0,
               fetch_factor=1.5, write_factor=1.0)
    body = "# counters\n\n```json\n" + json.dumps(rec) + "\n```\n"
    (tmp_path / "profiles" / "hbm_counters_push_column_50cm_fp64.md").write_text(body)
    t, note = bench.counter_traffic("column_50cm", "fp64")
    assert t == (1000.0 * 1.5 + 500.0) * 1024.0
    with open(tmp_path / bench.KERNEL_SOURCES[0], "a") as f:
        f.write("\n// changed\n")
    t, note = bench.counter_traffic("column_50cm", "fp64")
    assert t is None and "not the current" in note


def test_algorithmic_bytes_per_electron():
    assert bench.electron_bytes_per_step(0.0) == 36.0
    assert bench.electron_bytes_per_step(0.5) == 52.0
    assert bench.electron_bytes_per_step(0.5, fp32=True) == 36.0


@pytest.mark.gpu
def test_json_line(torch_cuda, monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--steps", "40", "--warmup", "40", "--cpu-steps", "2",
                                      "--no-batch", "--no-fluid", "--no-pair", "--no-section-v", "--no-fp32",
                                      "--no-20cm", "--probe-mib", "256"])
    assert bench.main() == 0
    d = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 40 and d["warmup"] == 40
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["config"]["workload"] == "column_50cm" and d["metric"] == bench.METRIC
    r = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert 0.0 < r["frac"] < 1.0 and abs(r["frac"] - r["achieved"] / r["peak"]) <= 1e-12
    c = d["cpu_baseline"]
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in c, k
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1
    assert c["serial"]["value"] > 0 and c["host"]["cpus"] >= 1
    p = d["stream_probe"]
    assert p["copy_ok"] and p["GB_s"] > 0
    assert abs(r["frac_of_measured_copy"] - r["achieved"] / p["GB_s"]) <= 1e-12


def test_counter_traffic_scales_with_electrons(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    for f in bench.KERNEL_SOURCES:
        os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
        with open(os.path.join(bench.ROOT, f), "rb") as src, open(tmp_path / f, "wb") as dst:
            dst.write(src.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = dict(source_sha16=bench.kernel_source_sha16(), fetch_kib=1000.0, write_kib=500.0, fetch_factor=2.0,
               write_factor=1.0, electrons_per_launch=4.0e6)
    body = "```json\n" + json.dumps(rec) + "\n```\n"
    (tmp_path / "profiles" / "hbm_counters_push_column_50cm_fp64.md").write_text(body)
    t0, _ = bench.counter_traffic("column_50cm", "fp64")
    t1, note = bench.counter_traffic("column_50cm", "fp64", 5.0e6)
    assert t0 == 2500.0 * 1024.0 and abs(t1 / t0 - 1.25) < 1e-12 and "scaled" in note
