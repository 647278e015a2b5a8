"""Host-side parts of the benchmark: the one-GPU guard, the roofline record and
the HBM counter summary (no GPU needed)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "--gpus must be 1" in (r.stdout + r.stderr)


def test_roofline_record_fields():
    dom = dict(launches=4, ms=2.0, bytes=4 * 1.0e9)          # 1 GB per launch, 0.5 ms per launch
    rl = bench.roofline(dom, "xelast32", 256)
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert rl["achieved"] == pytest.approx(2000.0)
    assert rl["frac"] == pytest.approx(0.25)
    assert rl["kernel"] == "k_xelast<float, 256>"
    assert rl["bytes_per_launch"] == 10 ** 9 and rl["mean_launch_us"] == pytest.approx(500.0)
    assert bench.roofline(dict(launches=0, ms=0.0, bytes=0.0), "xelast32") is None


def _counter_csv(path, counter, rows):
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(cols)
        for i, (name, value, dur_ns) in enumerate(rows):
            w.writerow([i + 1, name, counter, value, 1000, 1000 + dur_ns])


def test_counter_summary_calibrates_and_drops_early_exit_launches(tmp_path):
    probe = "void at::native::elementwise_kernel<MulFunctor<double>>(int)"
    kern = "void tumor::k_xelast<float, 256>(tumor::XElastArgs, tumor::cplx<float> const*)"
    # the probe reads and writes 1 MiB; FETCH_SIZE reports half of it (factor 2)
    _counter_csv(tmp_path / "f", "FETCH_SIZE", [(probe, 512.0, 50000), (kern, 900.0, 300000),
                                               (kern, 1100.0, 290000), (kern, 3.0, 3000)])
    _counter_csv(tmp_path / "w", "WRITE_SIZE", [(probe, 1024.0, 50000), (kern, 500.0, 300000),
                                               (kern, 700.0, 290000), (kern, 0.5, 3000)])
    out = tmp_path / "c.json"
    bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), 1, str(out))
    d = json.load(open(out))
    assert d["fetch_factor"] == pytest.approx(2.0) and d["write_factor"] == pytest.approx(1.0)
    k = d["kernels"]["k_xelast<float, 256>"]
    assert k["launches"] == 2                      # the 3 us launch is dropped
    assert k["fetch_kib"] == pytest.approx(1000.0) and k["write_kib"] == pytest.approx(600.0)
    assert d["sources_sha256"] == bench.kernel_sources_digest()


def test_source_digest_ignores_comments_and_layout(tmp_path, monkeypatch):
    src = tmp_path / "paper_1810_05370_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "a.hip").write_text("int f(int x) {\n  return x + 1;  // one\n}\n/* block\n comment */\n")
    (src / "engine.hip").write_text("host only\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.kernel_sources_digest()
    (src / "a.hip").write_text("// a note\nint f(int x) {   return x + 1; }\n")
    assert bench.kernel_sources_digest() == d0
    (src / "engine.hip").write_text("host only, changed\n")
    assert bench.kernel_sources_digest() == d0
    (src / "a.hip").write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_sources_digest() != d0
