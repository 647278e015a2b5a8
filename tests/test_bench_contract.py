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


def test_cycle_plan_splits_into_runs_no_longer_than_the_window():
    assert bench.cycle_plan(20, 10) == [10, 10]
    assert bench.cycle_plan(25, 10) == [10, 10, 5]
    assert bench.cycle_plan(5, 10) == [5]
    assert bench.cycle_plan(0, 10) == []
    for total in range(0, 60):
        runs = bench.cycle_plan(total, 7)
        assert sum(runs) == total and all(1 <= r <= 7 for r in runs)
    with pytest.raises(ValueError):
        bench.cycle_plan(3, 0)


class _FakeEvent:
    def __init__(self, **kw):
        pass

    def record(self, stream=None):
        pass

    def synchronize(self):
        pass

    def elapsed_time(self, other):
        return 1.0


class _FakeCuda:
    Event = _FakeEvent

    @staticmethod
    def synchronize():
        pass


class _FakeTorch:
    cuda = _FakeCuda


class _FakeSim:
    """Counts the trajectory step each call reaches: steps since t = 0 for the
    prefix, then since the snapshot the window restarts from."""

    def __init__(self, limit):
        self.limit = limit
        self.pos = 0
        self.snap_pos = None
        self.max_pos = 0
        self.steps = 0
        self.stream = None

    def step(self, k=1):
        assert k == 1
        self.pos += 1
        self.steps += 1
        self.max_pos = max(self.max_pos, self.pos)
        if self.pos > self.limit:
            raise AssertionError(f"step {self.pos} lies past the stable window (last step {self.limit})")
        return dict(it_elast=30, outer_elast=2, it_diff=[1, 1, 1])

    def save_state(self):
        self.snap_pos = self.pos
        return "snapshot"

    def load_state(self, snap):
        assert snap == "snapshot"
        self.pos = self.snap_pos

    def kernel_timer(self, name, enable=True):
        pass

    def kernel_timer_read(self, name):
        return dict(launches=1, ms=1.0 if name == "xelast32" else 0.5, bytes=1e9)

    def substep_timer(self, enable=True):
        pass

    def substep_timer_read(self):
        return self.steps, dict(transport=1.0, diffusion=1.0, reaction=1.0, elasticity=1.0)

    def diagnose(self, thr):
        return dict(max_disp=1.0)

    def get(self, name):
        return name

    def close(self):
        pass


@pytest.mark.parametrize("steps,warmup", [(20, 5), (10, 3), (1, 0), (37, 11)])
def test_the_timed_steps_never_leave_the_stable_window(steps, warmup):
    """The driver's --steps 20 --warmup 5 (and any other counts) queue no step
    past the last step of the window; the timed count is exact."""
    start, span = bench.WINDOWS["seeds3_n256"]
    sims = []

    class _TM:
        F_DEFAULT = 0x7

        @staticmethod
        def from_inputs(inp, P, **kw):
            sims.append(_FakeSim(start + span))
            return sims[-1]

    r = bench.run_form(_TM, _FakeTorch, {}, {}, "mixed", steps, warmup, (start, span), keep_fields=True)
    sim = sims[0]
    assert sim.max_pos <= start + span
    assert len(r["stats"]) == steps
    assert r["dominant"] == "xelast32"
    s = bench.run_single(_TM, _FakeTorch, {}, {}, "mixed", steps, warmup, (start, span))
    assert sims[1].max_pos <= start + span and len(s["elasticity_iterations"]) == steps


def test_every_workload_the_benchmark_can_time_has_a_window():
    import synthetic
    for name in synthetic.WORKLOADS:
        start, span = bench.WINDOWS[name]
        assert start >= 0 and span >= 1
