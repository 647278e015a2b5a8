#!/usr/bin/env python3
"""Throughput of the operator-split multispecies glioblastoma step on one MI355X.

A "step" is one whole split step (transport, three Crank-Nicolson solves,
reaction/oxygen/edema, coefficient refresh, force and the elasticity solve)
on the 256^3 synthetic workload (three tumour seeds, tissue maps smoothed
over 8 cells, dt = 0.01, PCG rtol 1e-8) in the mixed precision.  The FP64
form of the same workload is timed as well and reported beside it.

Prints one JSON line.  value = split steps per second (inputs resident in
HBM).  roofline = the dominant kernel class of the timed steps (by HIP-event
time), its algorithmic bytes per launch over its mean launch duration,
measured live with events on the library's stream.  cpu_baseline = the CPU
oracle timed on a bounded sample of the same step (see --help).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "split time steps/s at 256³ (fwd, fwd+adjoint), mixed vs FP64 on one GPU"
HBM_PEAK_GBS = 8000.0
CLASSES = ("colinv64", "colfwd64", "colinv32", "colfwd32", "colinv32z", "colfwd32z", "xelast64", "xelast32",
           "xdiff64", "xdiff32", "xother", "sl", "react", "krylov64", "krylov32", "zinvp64", "zinvp32",
           "zinvp64c1", "zinvp32c1", "zinvpb64", "zinvpb32", "coldot64", "coldot32")
# classes that time exactly one kernel symbol, so that the roofline's kernel can
# be matched to a rocprofv3 summary line (xother, sl and krylov group several)
SINGLE_KERNEL = ("colinv64", "colfwd64", "colinv32", "colfwd32", "colinv32z", "colfwd32z", "coldot64",
                 "coldot32", "xelast64", "xelast32", "xdiff64", "xdiff32", "zinvp64", "zinvp32", "zinvp64c1",
                 "zinvp32c1", "zinvpb64", "zinvpb32", "react")

# Stable windows of the 256^3 forward workloads: (steps from t = 0 before the
# window, longest run from the window's start).  The coupled transport /
# elasticity of these synthetic inputs loses stability after about 18 steps
# (seeds3_n256); every timed step lies in steps 4..13, where the trajectory is
# smooth.  Each run of at most `span` steps starts from a device snapshot of the
# state after step `start` (bit-exact restore, outside the timed region).
WINDOWS = {"seeds3_n256": (3, 10), "seeds3_n128": (3, 10), "seed1_n32": (0, 10),
           "lattice_n256": (0, 4), "lattice_n128": (0, 4)}


def cycle_plan(total, span):
    """Lengths of the runs that make up `total` steps, each at most `span` long
    (every run restarts from the window snapshot, so no step leaves the window)."""
    if span < 1 or total < 0:
        raise ValueError("span must be >= 1 and total >= 0")
    runs = []
    while total > 0:
        k = min(span, total)
        runs.append(k)
        total -= k
    return runs


def log(*a):
    print(*a, file=sys.stderr, flush=True)


SPECIES = ("p", "i", "n", "o", "l", "g", "w", "f")


def window_end_fields(sim, snap, span):
    """State after a full window run (snapshot + span steps): species and u."""
    sim.load_state(snap)
    for _ in range(span):
        sim.step(1)
    return {k: sim.get(k) for k in SPECIES + ("u",)}


def timed_cycles(torch, sim, snap, steps, span):
    """Time `steps` steps in runs of at most `span` from the snapshot.  Returns
    (event ms summed over the runs, wall s including the restores, stats)."""
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    stats, gpu_ms = [], 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for run in cycle_plan(steps, span):
        sim.load_state(snap)                   # restore: outside the event-timed region
        ev0.record(sim.stream)
        for k in range(run):
            stats.append(sim.step(1))
        ev1.record(sim.stream)
        ev1.synchronize()
        gpu_ms += ev0.elapsed_time(ev1)
    torch.cuda.synchronize()
    return gpu_ms, time.perf_counter() - t0, stats


def run_form(tm, torch, inp, P, precision, steps, warmup, window, keep_fields=False):
    """Reach the window, warm up, find the dominant kernel class, then time
    `steps` steps (all inside the window)."""
    start, span = window
    sim = tm.from_inputs(inp, P, precision=precision)
    for k in range(start):
        sim.step(1)
    snap = sim.save_state()
    for c in CLASSES:
        sim.kernel_timer(c, True)
    # W warm-up steps in window runs; with W = 0 one untimed run of the window
    # still profiles the kernel classes (to pick the roofline's kernel)
    wstats = []
    for run in cycle_plan(warmup, span) or [min(span, 3)]:
        sim.load_state(snap)
        for k in range(run):
            wstats.append(sim.step(1))
            log(f"[{precision}] warm-up step {len(wstats)} (window step {start + k + 1}): elast it "
                f"{wstats[-1]['it_elast']} (outer {wstats[-1]['outer_elast']}), diff it {wstats[-1]['it_diff']}")
    prof = {c: sim.kernel_timer_read(c) for c in CLASSES}
    # the roofline is reported for the single kernel with the largest share of time
    dominant = max(SINGLE_KERNEL, key=lambda c: prof[c]["ms"])
    for c in CLASSES:
        sim.kernel_timer(c, c == dominant)       # only the dominant class inside the timed region
    sim.substep_timer(True)                      # six events per step at the sub-step boundaries
    gpu_ms, wall, stats = timed_cycles(torch, sim, snap, steps, span)
    dom = sim.kernel_timer_read(dominant)
    sim.kernel_timer(dominant, False)
    nsub, sub = sim.substep_timer_read()
    sim.substep_timer(False)
    substeps = {k: round(v / max(nsub, 1), 3) for k, v in sub.items()}
    # algorithmic bytes of the timed steps: the same runs again (bit-exact from
    # the snapshot, so the same iterations) with every kernel class counting;
    # the timed region above ran with one class only
    for c in CLASSES:
        sim.kernel_timer(c, True)
    timed_cycles(torch, sim, snap, steps, span)
    step_bytes = sum(sim.kernel_timer_read(c)["bytes"] for c in CLASSES) / max(steps, 1)
    for c in CLASSES:
        sim.kernel_timer(c, False)
    log(f"[{precision}] {steps} steps in runs {cycle_plan(steps, span)}: events {gpu_ms / 1e3:.3f} s, wall {wall:.3f} s;"
        f" dominant {dominant}: {dom['launches']} launches, {dom['ms']:.1f} ms")
    # mass-effect diagnostics (scalars) of the displacement the timed runs ended with
    sim.diagnose(0.1)                                    # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        diag = sim.diagnose(0.1)
    torch.cuda.synchronize()
    diag_ms = (time.perf_counter() - t0) / reps * 1e3
    fields = window_end_fields(sim, snap, span) if keep_fields else None
    sim.close()
    return dict(wall=wall, gpu_ms=gpu_ms, stats=stats, warm_profile=prof, dominant=dominant, dom=dom,
                diag=diag, diag_ms=diag_ms, fields=fields, substeps=substeps, step_bytes=step_bytes)


def step_roofline(run, steps):
    """Per-step roofline: the algorithmic bytes of the timed steps (every
    kernel class) over their event-timed duration, against the 8 TB/s peak."""
    ms = run["gpu_ms"] / steps
    gbs = run["step_bytes"] / (ms / 1e3) / 1e9
    return dict(bytes_per_step=round(run["step_bytes"]), ms_per_step=round(ms, 3), achieved=round(gbs, 1),
                peak=HBM_PEAK_GBS, unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4),
                note="bytes: each kernel's input and output arrays once per launch, summed over every kernel "
                     "class; device-to-device state copies and fills are not counted")


def run_single(tm, torch, inp, P, precision, steps, warmup, window, model="single", flags=None):
    """Split steps/s of a model variant (the single-species model, the
    multispecies model on masked inputs, or the symmetric step) on the 256^3
    inputs, timed inside the same window as the main form."""
    start, span = window
    sim = tm.from_inputs(inp, P, precision=precision, model=model,
                         flags=tm.F_DEFAULT if flags is None else flags)
    for _ in range(start):
        sim.step(1)
    snap = sim.save_state()
    for run in cycle_plan(warmup, span):
        sim.load_state(snap)
        for _ in range(run):
            sim.step(1)
    ms, _, its = timed_cycles(torch, sim, snap, steps, span)
    sim.close()
    log(f"[{model} {precision} flags {flags}] {steps} steps: {ms / steps:.1f} ms/step, elasticity it {[s['it_elast'] for s in its]}")
    return dict(steps_per_s=round(steps / (ms / 1e3), 4), ms_per_step=round(ms / steps, 3),
                elasticity_iterations=[s["it_elast"] for s in its], diffusion_iterations=[s["it_diff"][0] for s in its])


def run_adjoint(tm, torch, inp, P, precision, steps, warmup, ckpt):
    """Forward + adjoint throughput: `steps` recorded steps then their reverse sweep."""
    import numpy as np
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    free0, total = torch.cuda.mem_get_info()
    sim = tm.from_inputs(inp, P, precision=precision, flags=tm.F_DEFAULT | tm.F_ADJOINT)
    for k in range(warmup):
        sim.step(1)
    sim.record(steps, ckpt)
    n = inp["n"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tau = sim.get("p") + sim.get("i") + sim.get("n")
    lam = torch.zeros((14, n, n, n), dtype=torch.float64, device=tau.device)
    h3 = (2 * np.pi / n) ** 3
    for k in range(3):
        lam[k].copy_(h3 * 0.1 * tau)          # seed of 1/2 h^3 ||tau - 0.9 tau||^2
    del tau
    grad = np.zeros(5 + len(inp["weights"]))
    free1, _ = torch.cuda.mem_get_info()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for k in range(steps):
        sim.adjoint_step(lam, grad)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    peak = torch.cuda.max_memory_allocated() / 2 ** 30
    log(f"[{precision} adjoint] {steps} recorded steps {t1 - t0:.2f} s, reverse sweep {t3 - t2:.2f} s "
        f"(checkpoint every {ckpt}); peak allocated {peak:.1f} GiB")
    sim.close()
    del sim, lam
    torch.cuda.empty_cache()
    return dict(fwd_s=t1 - t0, adj_s=t3 - t2, steps_per_s=steps / ((t1 - t0) + (t3 - t2)), peak_gib=peak,
                device_used_gib=(free0 - free1) / 2 ** 30, grad_head=[float(v) for v in grad[:5]], grad=grad)


def copy_ceiling(torch, tm, mib=1024, reps=10):
    """Achievable HBM bandwidth of plain device copies of `mib` MiB: the
    library's streaming copy (one 16-byte load and store per thread), torch's
    device-to-device copy and a one-read-one-write torch elementwise kernel,
    each timed with events; bytes moved = read + written."""
    n = mib * 2 ** 20 // 8
    src = torch.empty(n, dtype=torch.float64, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    out = {}
    for name, fn in (("stream_copy", lambda: tm.stream_copy(src, dst)), ("torch_copy", lambda: dst.copy_(src)),
                     ("torch_scale", lambda: torch.mul(src, 2.0, out=dst))):
        for _ in range(3):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        ms = sorted(a.elapsed_time(b) for a, b in ev)
        gbs = 2 * n * 8 / (ms[len(ms) // 2] * 1e-3) / 1e9
        out[name] = round(gbs, 1)
    del src, dst
    torch.cuda.empty_cache()
    best = max(out.values())
    return dict(gbs=best, frac_of_peak=round(best / HBM_PEAK_GBS, 4), mib=mib, by_kernel=out,
                note="median of %d event-timed launches, bytes = read + written" % reps)


def lockstep_differences(tm, torch, inp, P, steps, form_a, form_b):
    """Two contexts stepped side by side from t = 0; the relative L2 difference
    of every species and of u after each step.  form = (precision, weight
    factor of the initial condition)."""
    sims = []
    for prec, wfac in (form_a, form_b):
        d = dict(inp)
        d["weights"] = [w * wfac for w in inp["weights"]]
        sims.append(tm.from_inputs(d, P, precision=prec))
    out = []
    for k in range(steps):
        for sim in sims:
            sim.step(1)
        errs = rel_l2_errors({f: sims[0].get(f) for f in SPECIES + ("u",)},
                             {f: sims[1].get(f) for f in SPECIES + ("u",)})
        out.append({f: float(f"{v:.3e}") for f, v in errs.items()})
    for sim in sims:
        sim.close()
    torch.cuda.empty_cache()
    return out


def rel_l2_errors(mixed, ref):
    """Relative L2 error of each field of the mixed form against the FP64 form."""
    out = {}
    for k in ref:
        d = (mixed[k] - ref[k]).double().norm().item()
        r = ref[k].double().norm().item()
        out[k] = d / r if r > 0 else d
    return out


COUNTERS_FILE = os.path.join(ROOT, "profiles", "hbm_counters_256.json")


def kernel_sources_digest():
    """SHA-256 over the library's device sources: every HIP source and header
    (sorted by name) except engine.hip, which holds host-side control only (no
    kernel and no launch configuration).  Comments and blank space are
    stripped first, so only code changes invalidate the counters."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1810_05370_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")) and f != "engine.hip":
            text = open(os.path.join(csrc, f), encoding="utf-8").read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
            h.update(f.encode())
            h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc summary.

    None when no summary exists, when it has no entry for the kernel, or when
    the kernel sources changed after the counters were taken."""
    if kernel is None or not os.path.exists(COUNTERS_FILE):
        return None
    d = json.load(open(COUNTERS_FILE))
    if d.get("sources_sha256") != kernel_sources_digest():
        return None
    k = d["kernels"].get(kernel)
    if k is None:
        return None
    return round(k["fetch_kib"] * 1024 * d["fetch_factor"] + k["write_kib"] * 1024 * d["write_factor"])


def summarize_counters(fetch_dir, write_dir, probe_mib, out_path):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) into the
    per-kernel summary read by counter_traffic().

    Each run's counter_collection CSV holds one row per dispatch; rows are
    averaged per kernel (name up to the argument list) over the dispatches
    that did work: longer than 20 us, since PCG launches queued after
    convergence exit at once (the library's timers drop them too).  A kernel
    with no such dispatch is averaged over all of them.  The first torch
    multiply dispatch is the copy probe (--copy-probe-mib): it reads and writes
    probe_mib MiB, which fixes the factor from counter KiB to bytes."""
    import csv
    import glob

    def load(d, counter):
        path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not path:
            raise SystemExit(f"no counter_collection.csv under {d}")
        rows = [r for r in csv.DictReader(open(path[0])) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        probe = next(r for r in rows if "MulFunctor" in r["Kernel_Name"])
        per = {}
        for r in rows:
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("tumor::", "").strip()
            worked = int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) >= 20000
            acc = per.setdefault(name, [0.0, 0, 0.0, 0])
            acc[0] += float(r["Counter_Value"])
            acc[1] += 1
            if worked:
                acc[2] += float(r["Counter_Value"])
                acc[3] += 1
        return float(probe["Counter_Value"]), {
            k: ((v[2] / v[3], v[3]) if v[3] else (v[0] / v[1], v[1])) for k, v in per.items()}

    probe_bytes = probe_mib * 2.0 ** 20
    pf, fetch = load(fetch_dir, "FETCH_SIZE")
    pw, write = load(write_dir, "WRITE_SIZE")
    kernels = {k: dict(fetch_kib=round(fetch[k][0], 1), write_kib=round(write.get(k, (0.0, 0))[0], 1),
                       launches=fetch[k][1])
               for k in fetch if not k.startswith("at::")}
    out = dict(counters=["FETCH_SIZE", "WRITE_SIZE"], probe_mib=probe_mib,
               probe_fetch_kib=pf, probe_write_kib=pw,
               fetch_factor=probe_bytes / (pf * 1024.0), write_factor=probe_bytes / (pw * 1024.0),
               sources_sha256=kernel_sources_digest(), kernels=kernels)
    json.dump(out, open(out_path, "w"), indent=1, sort_keys=True)
    print(f"wrote {out_path}: fetch factor {out['fetch_factor']:.4f}, write factor {out['write_factor']:.4f}, "
          f"{len(kernels)} kernels")


def roofline(dom, name=None, n=256):
    import paper_1810_05370_amd as tm
    if dom["launches"] == 0 or dom["ms"] <= 0:
        return None
    per_launch = dom["bytes"] / dom["launches"]
    mean_ms = dom["ms"] / dom["launches"]
    achieved = per_launch / (mean_ms * 1e-3) / 1e9
    kernel = tm.KERNEL_NAMES.get(name, name).format(n=n) if name else None
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=counter_traffic(kernel),
                kernel=kernel, bytes_per_launch=round(per_launch), mean_launch_us=round(mean_ms * 1e3, 2))


def cpu_baseline(inp, P, iters_e, iters_d):
    """Time the FP64 CPU oracle on a bounded sample of one 256^3 step.

    Sample: one elasticity operator apply + one elasticity preconditioner
    (one PCG iteration's operator work), one CN diffusion apply + its
    preconditioner, the reaction/oxygen/edema/refresh sub-steps on the whole
    grid, the force, and the semi-Lagrangian interpolations on 4 z-planes.
    The step time is reconstructed as
    SL * (N / 4) + reaction + force + (n_e + 1) * elasticity-iteration
    + (n_d + 3) * CN-iteration, with n_e the elasticity iterations and n_d
    the iterations of the three CN solves together, per step of the same
    workload (FP64 run); the +1 and +3 are the initial residuals.
    """
    import numpy as np

    from oracle import model, reaction as rx, solvers, transport
    from oracle.spectral import Grid

    n = inp["n"]
    t_all = time.perf_counter()
    st = model.init_state(P, n, inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"], inp["weights"])
    g = st.grid
    co = st.coef
    F = st.f
    rng = np.random.default_rng(7)
    u = 1e-3 * rng.standard_normal((3, n, n, n))

    t = time.perf_counter()
    Au = solvers.elasticity_op(g, co["mu"], co["lam"], co["eta"], u)
    solvers.elasticity_precond(g, co["mubar"], co["lambar"], co["etabar"], Au)
    t_e = time.perf_counter() - t
    del Au
    t = time.perf_counter()
    q = solvers.cn_matrix(g, co["K"], 0.01, F["p"])
    solvers.cn_precond(g, co["Kbar"], 0.01, q)
    t_d = time.perf_counter() - t
    del q
    t = time.perf_counter()
    z = np.zeros_like(F["p"])
    p1, i1, n1, g1, w1 = rx.species_reaction(P, 0.01, F["p"], F["i"], F["n"], F["g"], F["w"], F["o"],
                                             co["rho_p"], co["rho_i"], z)
    o1 = rx.oxygen_reaction(P, 0.01, F["o"], p1, g1, w1)
    rx.edema_reaction(P, 0.01, F["l"], i1)
    rx.refresh(P, p1, i1, n1, g1, w1, F["f"])
    t_r = time.perf_counter() - t
    t = time.perf_counter()
    b = rx.elastic_force(g, P["zeta"], p1, n1)
    v = u / 0.01
    delta = g.div(v)
    t_f = time.perf_counter() - t
    del b, o1
    slab = 4
    t = time.perf_counter()
    r = np.arange(n, dtype=np.float64)
    jz, jy, jx = np.meshgrid(r[:slab], r, r, indexing="ij")
    s = 0.01 / g.h
    xs = (jx - s * v[0, :slab], jy - s * v[1, :slab], jz - s * v[2, :slab])
    vs = [transport.interp(v[a], *xs) for a in range(3)]
    X = tuple(j - 0.5 * s * (v[a, :slab] + vs[a]) for a, j in enumerate((jx, jy, jz)))
    for name in ("p", "i", "n", "g", "w", "f"):
        transport.interp(F[name], *X)
    transport.interp(delta, *X)
    t_sl = (time.perf_counter() - t) * (n / slab)
    step_s = t_sl + t_r + t_f + (iters_e + 1) * t_e + (iters_d + 3) * t_d
    cores = len(os.sched_getaffinity(0))
    log(f"cpu sample: elast iter {t_e:.2f} s, cn iter {t_d:.2f} s, reaction {t_r:.2f} s, force {t_f:.2f} s,"
        f" SL (scaled) {t_sl:.2f} s; sample wall {time.perf_counter() - t_all:.1f} s")
    return dict(value=round(1.0 / step_s, 6), unit="steps/s", cores=cores, kind="oracle",
                sample=(f"FP64 NumPy/SciPy oracle at 256^3 on {cores} host threads (scipy.fft workers; NumPy "
                        f"elementwise single-threaded): one elasticity apply+preconditioner ({t_e:.2f} s), one CN "
                        f"apply+preconditioner ({t_d:.2f} s), reaction+refresh ({t_r:.2f} s), force+velocity "
                        f"divergence ({t_f:.2f} s), SL interpolation on {slab} of {n} z-planes scaled x{n // slab} "
                        f"({t_sl:.2f} s); step = SL + reaction + force + (n_e+1) elasticity + (n_d+3) CN "
                        f"iterations with n_e={iters_e:.1f}, n_d={iters_d:.1f} per step of the FP64 run"))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed steps, in runs of at most the window length from the window snapshot")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="seeds3_n256", help="synthetic workload name (default: the 256^3 case)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward+adjoint form")
    ap.add_argument("--no-single", action="store_true", help="skip the single-species model")
    ap.add_argument("--no-strang", action="store_true", help="skip the symmetric (Strang) form of the step")
    ap.add_argument("--no-masked", action="store_true",
                    help="skip the fictitious-domain form (brain mask and background material)")
    ap.add_argument("--no-lockstep", action="store_true",
                    help="skip the step-by-step mixed-vs-FP64 and perturbation comparisons")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size kernel that calibrates "
                         "the HBM byte counters of a rocprofv3 --pmc run)")
    ap.add_argument("--adjoint-workload", default="lattice_n256", help="workload of the forward+adjoint form")
    ap.add_argument("--adjoint-steps", type=int, default=4,
                    help="recorded steps of the forward+adjoint form (from t = 0).  The lattice workload's "
                         "coupled transport/elasticity loses stability after about 9 steps at 256^3, and its "
                         "gradient stops being smooth (central differences disagree) near step 8; over 4 steps "
                         "the adjoint gradient matches central differences")
    ap.add_argument("--ckpt-every", type=int, default=1,
                    help="checkpoint interval of the forward+adjoint form; 1 keeps every state and the step "
                         "intermediates on the tape (about 14 GB at 256^3 for 4 steps), so the reverse sweep "
                         "recomputes no forward step")
    ap.add_argument("--ckpt-steps", type=int, default=8,
                    help="recorded steps of the checkpointed forward+adjoint form (0 skips it)")
    ap.add_argument("--ckpt-k", type=int, default=4, help="checkpoint interval of that form")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "PROBE_MIB"),
                    help="no GPU work: write the HBM counter summary from two rocprofv3 --pmc output folders")
    args = ap.parse_args()
    if args.summarize_counters:
        fd, wd, mib = args.summarize_counters
        summarize_counters(fd, wd, int(mib), COUNTERS_FILE)
        return
    if args.gpus != 1:
        print("bench.py: one simulation runs on exactly one GPU, so --gpus must be 1 "
              "(several GPUs would run independent simulations, which this benchmark does not time)",
              file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1810_05370_amd as tm
    import synthetic

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    tm.load_library()
    if args.copy_probe_mib > 0:
        src = torch.empty(args.copy_probe_mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.mul(src, 2.0, out=dst)          # the probe: one read and one write of the buffer
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst
    P = synthetic.params()
    t = time.perf_counter()
    inp = synthetic.workload_inputs(args.workload)
    n = inp["n"]
    log(f"inputs {args.workload} n={n} generated in {time.perf_counter() - t:.1f} s")
    precision = inp["precision"]

    if args.workload not in WINDOWS:
        raise SystemExit(f"bench.py: no stable window is known for workload {args.workload!r}")
    window = WINDOWS[args.workload]
    start, span = window
    extra = {}
    # achievable HBM bandwidth of a plain device copy, the practical ceiling
    extra["copy_ceiling"] = copy_ceiling(torch, tm)
    log(f"copy ceiling: {extra['copy_ceiling']}")
    compare = not args.no_fp64 and precision != "fp64" and not args.no_lockstep
    main_run = run_form(tm, torch, inp, P, precision, args.steps, args.warmup, window)
    ms_per_step = main_run["gpu_ms"] / args.steps
    value = args.steps / (main_run["gpu_ms"] / 1e3)
    fp64_run = None
    if not args.no_fp64 and precision != "fp64":
        torch.cuda.empty_cache()
        fp64_run = run_form(tm, torch, inp, P, "fp64", args.steps, args.warmup, window)
        v64 = args.steps / (fp64_run["gpu_ms"] / 1e3)
        extra["fp64_steps_per_s"] = round(v64, 4)
        extra["mixed_speedup_over_fp64"] = round(value / v64, 3)
        extra["fp64_roofline"] = roofline(fp64_run["dom"], fp64_run["dominant"], n)
        extra["fp64_step_roofline"] = step_roofline(fp64_run, args.steps)
        extra["fp64_substep_ms_per_step"] = fp64_run["substeps"]
    extra["substep_ms_per_step"] = main_run["substeps"]
    extra["step_roofline"] = step_roofline(main_run, args.steps)
    extra["step_roofline"]["frac_of_copy_ceiling"] = round(
        extra["step_roofline"]["achieved"] / extra["copy_ceiling"]["gbs"], 4)
    if compare:
        # error of the mixed form against the FP64 form (itself held to the FP64
        # oracle at 1e-10 by the parity tests), after every step from t = 0 to the
        # window's end; beside it, how far two FP64 runs whose initial tumour
        # differs by 1e-12 (relative) drift apart over the same steps: the
        # trajectory's own amplification of a small perturbation
        by_step = lockstep_differences(tm, torch, inp, P, start + span, ("mixed", 1.0), ("fp64", 1.0))
        extra["mixed_vs_fp64_rel_l2"] = dict(after_step=start + span, **by_step[-1])
        extra["mixed_vs_fp64_rel_l2_by_step"] = {f: [e[f] for e in by_step] for f in ("p", "i", "o", "u")}
        pert = lockstep_differences(tm, torch, inp, P, start + span, ("fp64", 1.0 + 1e-12), ("fp64", 1.0))
        extra["fp64_ic_perturbation_1e-12_rel_l2_by_step"] = {f: [e[f] for e in pert] for f in ("p", "i", "o", "u")}
        log(f"mixed vs FP64 relative L2 by step: {extra['mixed_vs_fp64_rel_l2_by_step']}")
        log(f"FP64 1e-12 IC perturbation by step: {extra['fp64_ic_perturbation_1e-12_rel_l2_by_step']}")
    it_e = [s["it_elast"] for s in main_run["stats"]]
    extra["timed_runs"] = dict(window_steps=[start + 1, start + span], runs=cycle_plan(args.steps, span),
                               note="each run restarts from a device snapshot of the state after step "
                                    f"{start} (restore outside the timed region)")
    extra["elasticity_iterations_per_step"] = it_e
    extra["elasticity_outer_per_step"] = [s["outer_elast"] for s in main_run["stats"]]
    extra["diffusion_iterations_last_step"] = main_run["stats"][-1]["it_diff"]
    extra["warmup_kernel_ms"] = {c: round(v["ms"], 2) for c, v in main_run["warm_profile"].items() if v["ms"] > 0}
    # algorithmic HBM rate of every kernel class over the warm-up steps (launches
    # that exit early after convergence are not counted), against the 8 TB/s peak
    extra["warmup_class_rates"] = {
        c: dict(launches=v["launches"], gbs=round(v["bytes"] / v["ms"] / 1e6, 1),
                frac=round(v["bytes"] / v["ms"] / 1e6 / HBM_PEAK_GBS, 3))
        for c, v in main_run["warm_profile"].items() if v["ms"] > 0 and v["launches"] > 0}
    extra["wall_s"] = round(main_run["wall"], 4)
    extra["diagnostics"] = dict(ms=round(main_run["diag_ms"], 3), threshold_voxels=0.1,
                                **{k: round(v, 6) for k, v in main_run["diag"].items()})
    rl = roofline(main_run["dom"], main_run["dominant"], n)
    if rl is not None:
        rl["frac_of_copy_ceiling"] = round(rl["achieved"] / extra["copy_ceiling"]["gbs"], 4)

    if not args.no_single:
        extra["single_species"] = {prec: run_single(tm, torch, inp, P, prec, args.steps, args.warmup, window)
                                   for prec in (("mixed", "fp64") if not args.no_fp64 else ("mixed",))}

    if not args.no_strang:
        extra["strang"] = {prec: run_single(tm, torch, inp, P, prec, args.steps, args.warmup, window, "multispecies",
                                            tm.F_DEFAULT | tm.F_STRANG)
                           for prec in (("mixed", "fp64") if not args.no_fp64 else ("mixed",))}

    if not args.no_masked:
        minp = synthetic.workload_inputs(args.workload, masked=True)
        extra["masked"] = dict(workload=f"{args.workload} with the brain mask and background material",
                               **run_single(tm, torch, minp, P, precision, args.steps, args.warmup, window,
                                            "multispecies"))

    if not args.no_adjoint:
        ainp = synthetic.workload_inputs(args.adjoint_workload)
        grads = {}
        for prec in (("mixed", "fp64") if not args.no_fp64 else ("mixed",)):
            r = run_adjoint(tm, torch, ainp, P, prec, args.adjoint_steps, 0, args.ckpt_every)
            grads[prec] = r["grad"]
            key = "fwd_adjoint_steps_per_s" if prec == "mixed" else "fwd_adjoint_fp64_steps_per_s"
            extra[key] = round(r["steps_per_s"], 4)
            extra[key.replace("steps_per_s", "detail")] = dict(
                workload=f"{args.adjoint_workload}: {ainp['n']}^3, {len(ainp['weights'])} initial-condition weights",
                recorded_steps=args.adjoint_steps, ckpt_every=args.ckpt_every, forward_s=round(r["fwd_s"], 3),
                reverse_s=round(r["adj_s"], 3), peak_allocated_gib=round(r["peak_gib"], 2),
                device_used_gib=round(r["device_used_gib"], 2), grad_rho_kw_kg_kf_scale=r["grad_head"])
        if len(grads) == 2:
            import numpy as np
            g64 = grads["fp64"]
            extra["fwd_adjoint_mixed_vs_fp64_grad_rel_l2"] = float(
                f"{np.linalg.norm(grads['mixed'] - g64) / np.linalg.norm(g64):.3e}")
        if args.ckpt_steps > 0:
            # the checkpointed tape: a checkpoint every K steps, each reversed step
            # recomputes its window from the nearest checkpoint
            r = run_adjoint(tm, torch, ainp, P, precision, args.ckpt_steps, 0, args.ckpt_k)
            extra["fwd_adjoint_checkpointed"] = dict(
                precision=precision, recorded_steps=args.ckpt_steps, ckpt_every=args.ckpt_k,
                steps_per_s=round(r["steps_per_s"], 4), forward_s=round(r["fwd_s"], 3), reverse_s=round(r["adj_s"], 3),
                peak_allocated_gib=round(r["peak_gib"], 2), device_used_gib=round(r["device_used_gib"], 2))

    cpu = None
    if not args.no_cpu_baseline:
        ref = fp64_run if fp64_run is not None else main_run
        ne = sum(s["it_elast"] for s in ref["stats"]) / len(ref["stats"])
        nd = sum(sum(s["it_diff"]) for s in ref["stats"]) / len(ref["stats"])
        cpu = cpu_baseline(inp, P, ne, nd)

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n}^3 periodic grid, {precision} precision, full multispecies "
                               f"split step (transport, CN diffusion of i/o/l, reaction, oxygen, edema, elasticity); "
                               f"timed steps lie in steps {start + 1}-{start + span} of the trajectory from t = 0, in "
                               f"runs of at most {span} steps that each restart from a device snapshot of the state "
                               f"after step {start}",
                   "window": [start + 1, start + span],
                   "n": n, "precision": precision, "dt": inp["dt"], "rtol": inp["rtol"],
                   "tumour_seeds": int(len(inp["weights"])), "forward_only": True},
        "roofline": rl,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
