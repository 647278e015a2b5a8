"""Whole split steps on the GPU against the FP64 CPU oracle, through the C ABI.

Iteration lockstep: the oracle runs first with its tolerance-based stopping;
its per-solve iteration counts are then imposed on the GPU run
(tumor_force_iterations), so both sides execute the same algorithm for the
same number of iterations and differ only by floating-point rounding.  The
GPU's own counts (free run) must agree with the oracle's to within one
iteration.  Bar: relative L2 <= 1e-10 per species and for the displacement
in FP64, <= 1e-5 in the mixed precision.
"""
import numpy as np
import pytest

import paper_1810_05370_amd as tm
import synthetic
from gpu_common import need_gpu, rel_l2, say
from oracle import model

pytestmark = pytest.mark.gpu

SPECIES = ("p", "i", "n", "o", "l", "g", "w", "f")


def _oracle(P, inp, steps, cfg=None):
    st = model.init_state(P, inp["n"], inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"],
                          inp["weights"])
    stats = [model.step(st, cfg) for _ in range(steps)]
    return st, stats


def _iters(s):
    return [s["it_diff"][0], s["it_diff"][1], s["it_diff"][2], s["it_elast"]]


def _compare(sim, st, tol, label):
    worst = {}
    for k in SPECIES:
        got = sim.get(k).cpu().numpy()
        ref = st.f[k]
        if np.linalg.norm(ref) == 0.0:
            worst[k] = float(np.abs(got).max())
        else:
            worst[k] = rel_l2(got, ref)
    for k, ref in (("u", st.u), ("u_prev", st.u_prev)):
        got = sim.get(k).cpu().numpy()
        worst[k] = rel_l2(got, ref) if np.linalg.norm(ref) > 0 else float(np.abs(got).max())
    say(label, {k: f"{v:.2e}" for k, v in worst.items()})
    for k, v in worst.items():
        assert v <= tol, (label, k, v)
    return worst


def _run_case(P, inp, steps, flags=tm.F_DEFAULT, cfg=None, tol=1e-10):
    need_gpu()
    say(f"case n={inp['n']} steps={steps} flags={flags}")
    st, stats = _oracle(P, inp, steps, cfg)
    free = tm.from_inputs(inp, P, flags=flags)
    lock = tm.from_inputs(inp, P, flags=flags)
    for k in range(steps):
        sf = free.step(1)
        lock.force_iterations(_iters(stats[k]))
        lock.step(1)
        diff = np.abs(np.array(_iters(sf)) - np.array(_iters(stats[k])))
        assert diff.max() <= 1, (k, _iters(sf), _iters(stats[k]))
    _compare(lock, st, tol, f"lockstep n={inp['n']}")
    free.close()
    lock.close()
    return st, stats


def test_small_grid_two_steps():
    P = synthetic.params()
    _run_case(P, synthetic.workload_inputs("seed1_n32", n=16), 2)


def test_single_seed_workload_ten_steps_32():
    # The 32^3, 10-step FP64 workload.
    P = synthetic.params()
    _run_case(P, synthetic.workload_inputs("seed1_n32"), 10)


def test_hypoxic_regime_exercises_invasion_necrosis_and_edema():
    # Strong oxygen consumption drives the tumour core hypoxic within a few
    # steps, so the p -> i switch, necrosis and the edema source are active.
    P = synthetic.params(delta_p=60.0)
    st, stats = _run_case(P, synthetic.workload_inputs("seed1_n32", n=32), 6)
    assert st.f["i"].max() > 1e-3 and st.f["n"].max() > 1e-3 and st.f["l"].max() > 1e-4


def test_three_seed_workload_at_64():
    P = synthetic.params()
    inp = synthetic.workload_inputs("seeds3_n128", n=64)
    _run_case(P, inp, 3)


def test_sub_step_switches():
    P = synthetic.params(delta_p=60.0)
    inp = synthetic.workload_inputs("seed1_n32", n=16)
    _run_case(P, inp, 3, flags=tm.F_ELASTICITY, cfg=dict(advection=False, edema=False))
    _run_case(P, inp, 3, flags=tm.F_ADVECTION | tm.F_EDEMA, cfg=dict(elasticity=False))


def test_no_tumour_is_a_steady_state_of_the_tissue():
    need_gpu()
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32", n=16)
    inp = dict(inp, centers=np.zeros((0, 3)), sigmas=np.zeros(0), weights=np.zeros(0))
    sim = tm.from_inputs(inp, P)
    sim.step(2)
    # Only the (exponentially small) necrosis of healthy tissue acts: the
    # tissue maps are unchanged to the last bit and the mass effect vanishes.
    for k in ("g", "w", "f"):
        assert np.array_equal(sim.get(k).cpu().numpy(), inp[{"g": "gm", "w": "wm", "f": "csf"}[k]])
    assert not sim.get("p").cpu().numpy().any() and not sim.get("i").cpu().numpy().any()
    assert np.abs(sim.get("u").cpu().numpy()).max() < 1e-60
    sim.close()


def test_mixed_precision_matches_fp64_oracle():
    need_gpu()
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32")
    steps = 10
    st, stats = _oracle(P, inp, steps)
    sim = tm.from_inputs(inp, P, precision="mixed")
    for k in range(steps):
        s = sim.step(1)
        assert s["relres_elast"] <= 1e-8 and max(s["relres_diff"]) <= 1e-8
    _compare(sim, st, 1e-5, "mixed n=32")
    sim.close()


def test_mixed_precision_with_fields_below_fp32_range():
    """A tumour of amplitude 5e-31: forces, residuals and the necrotic cells lie
    far below FP32's normal range, so the FP32 stages work on power-of-two
    scaled copies; the result must still match the FP64 oracle."""
    need_gpu()
    P = synthetic.params(delta_p=60.0)
    inp = synthetic.workload_inputs("seed1_n32", n=16)
    inp = dict(inp, weights=1e-30 * np.asarray(inp["weights"]))
    steps = 4
    st, stats = _oracle(P, inp, steps)
    assert 0.0 < np.abs(st.u).max() < 1e-40
    sim = tm.from_inputs(inp, P, precision="mixed")
    for k in range(steps):
        s = sim.step(1)
        assert s["relres_elast"] <= 1e-8 and max(s["relres_diff"]) <= 1e-8, s
    _compare(sim, st, 1e-5, "mixed tiny n=16")
    sim.close()


def test_elasticity_solve_entry_point():
    need_gpu()
    import torch
    from oracle import reaction as rx, solvers
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32", n=32)
    sim = tm.from_inputs(inp, P)
    st = model.init_state(P, 32, inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"], inp["weights"])
    co = st.coef
    force = rx.elastic_force(st.grid, P["zeta"], st.f["p"], st.f["n"])
    ref, it, rr, ok = solvers.solve_elasticity(st.grid, co["mu"], co["lam"], co["eta"],
                                               (co["mubar"], co["lambar"], co["etabar"]), force,
                                               np.zeros_like(force), 1e-8, 1000)
    u, git, grr = sim.solve_elasticity()
    assert abs(git - it) <= 1 and grr <= 1e-8
    assert rel_l2(u.cpu().numpy(), ref) < 1e-9
    # explicit force argument gives the same solve
    u2, git2, _ = sim.solve_elasticity(torch.as_tensor(force).cuda())
    assert git2 == git and rel_l2(u2.cpu().numpy(), u.cpu().numpy()) < 1e-12
    sim.close()


def test_invalid_arguments_on_a_live_context():
    need_gpu()
    P = synthetic.params()
    sim = tm.from_inputs(synthetic.workload_inputs("seed1_n32", n=16), P)
    lib = sim.lib
    assert lib.tumor_get_field(sim.ctx, 99, None) == tm.EINVAL
    assert lib.tumor_apply_op(sim.ctx, 42, None, None) == tm.EINVAL
    assert lib.tumor_step(sim.ctx, -1, None) == tm.EINVAL
    assert lib.tumor_set_field(sim.ctx, tm.FIELDS["K"], None) == tm.EINVAL
    with pytest.raises(tm.TumorError):
        sim.force_iterations([1, 1, 1, 10 ** 7])
    sim.close()


def test_max_it_reports_no_convergence():
    need_gpu()
    P = synthetic.params()
    sim = tm.from_inputs(synthetic.workload_inputs("seed1_n32", n=16), P, max_it=2)
    with pytest.raises(tm.TumorError) as e:
        sim.step(1)
    assert e.value.code == tm.ENOCONV
    s = sim.step(1, allow_noconv=True)
    assert s["it_elast"] == 2
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_state_snapshot_restores_the_trajectory_bit_for_bit(precision):
    """tumor_save_state / tumor_load_state: steps taken after a restore repeat
    the saved trajectory exactly (the benchmark's timed runs rely on this)."""
    torch = need_gpu()
    P = synthetic.params()
    inp = synthetic.workload_inputs("seeds3_n128", n=32)
    say(f"snapshot case n=32 precision={precision}")
    sim = tm.from_inputs(inp, P, precision=precision)
    sim.step(2)
    snap = sim.save_state()
    assert snap.numel() == sim.state_bytes() >= 14 * 32 ** 3 * 8
    a_stats = [sim.step(1) for _ in range(3)]
    a = {k: sim.get(k) for k in SPECIES + ("u", "u_prev", "mu")}
    sim.load_state(snap)
    # an equal state gives a byte-identical snapshot, header included, whatever
    # the buffer held before
    again = sim.save_state(torch.full_like(snap, 0xA5))
    assert torch.equal(again, snap)
    b_stats = [sim.step(1) for _ in range(3)]
    b = {k: sim.get(k) for k in SPECIES + ("u", "u_prev", "mu")}
    for k in a:
        assert torch.equal(a[k], b[k]), k
    assert [s["it_elast"] for s in a_stats] == [s["it_elast"] for s in b_stats]
    assert [s["it_diff"] for s in a_stats] == [s["it_diff"] for s in b_stats]
    # a snapshot too small for the state is refused before any device work
    with pytest.raises(tm.TumorError):
        sim.load_state(snap[:-1])
    # a snapshot of another grid, padded to this grid's size, is refused by its
    # header and leaves the state as it was
    other = tm.from_inputs(synthetic.workload_inputs("seeds3_n128", n=16), P, precision=precision)
    small = other.save_state()
    other.close()
    padded = torch.zeros(snap.numel(), dtype=torch.uint8, device="cuda")
    padded[:small.numel()].copy_(small)
    with pytest.raises(tm.TumorError) as e:
        sim.load_state(padded)
    assert e.value.code == tm.EINVAL
    assert torch.equal(sim.get("p"), b["p"])
    sim.close()


def test_substep_timer_accounts_for_the_step():
    """The sub-step events cover the step: their sum is the step's event time
    (within the launch gaps before the first and after the last boundary)."""
    torch = need_gpu()
    P = synthetic.params()
    inp = synthetic.workload_inputs("seeds3_n128", n=64)
    sim = tm.from_inputs(inp, P, precision="mixed")
    sim.step(2)
    sim.substep_timer(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(sim.stream)
    sim.step(3)
    ev[1].record(sim.stream)
    torch.cuda.synchronize()
    n, sub = sim.substep_timer_read()
    sim.close()
    total = ev[0].elapsed_time(ev[1])
    say(f"sub-steps over {n} steps: {sub}, step events {total:.2f} ms")
    assert n == 3
    assert all(v > 0.0 for v in sub.values())
    assert 0.9 * total <= sum(sub.values()) <= total * 1.001


def test_batched_cn_kernel_timers_count_the_systems_still_iterating():
    """The batched CN solve's passes carry i, o and l while each iterates.  The
    kernel timers count, per launch, the bytes of the systems it computed: for
    the fused first pass 7 array passes per system, for the x pass K once plus
    6 per system.  So the mean bytes per launch lie between one and three
    systems' worth, and below three since o converges first."""
    need_gpu()
    P = synthetic.params()
    n = 64
    inp = synthetic.workload_inputs("seeds3_n128", n=n)
    sim = tm.from_inputs(inp, P, precision="mixed")
    sim.step(3)   # i and l nonzero: all three systems iterate
    for c in ("zinvpb32", "xdiff32"):
        sim.kernel_timer(c, True)
    stats = sim.step(2)
    reads = {c: sim.kernel_timer_read(c) for c in ("zinvpb32", "xdiff32")}
    sim.close()
    V, fb = n ** 3, 4
    say(f"batched timers: {reads}, diffusion iterations {stats['it_diff']}")
    its = stats["it_diff"]
    assert min(its) < max(its)
    for c, (fixed, per) in {"zinvpb32": (0, 7), "xdiff32": (1, 6)}.items():
        r = reads[c]
        assert r["launches"] > 0
        b = r["bytes"] / r["launches"]
        assert (fixed + per) * V * fb <= b < (fixed + 3 * per) * V * fb, (c, b)
