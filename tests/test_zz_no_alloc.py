"""The allocation-free context (tumor_init_static, the library's own fixed
device workspace) against the workspace context of tumor_init, through the C
ABI: the same split steps must give the same fields, on two contexts in a row
(the second on a smaller grid, reusing the array the first one left)."""
import pytest

import paper_1810_05370_amd as tm
import synthetic
from gpu_common import need_gpu, rel_l2, say

pytestmark = pytest.mark.gpu

FIELDS = ("p", "i", "n", "o", "l", "g", "w", "f", "u", "u_prev")


def _run(inp, P, precision, no_alloc, steps):
    sim = tm.from_inputs(inp, P, precision=precision, no_alloc=no_alloc)
    try:
        stats = [sim.step(1) for _ in range(steps)]
        out = {k: sim.get(k).cpu().numpy() for k in FIELDS}
    finally:
        sim.close()
    return stats, out


def test_static_context_matches_the_workspace_context_on_two_calls():
    need_gpu()
    P = synthetic.params()
    # second call: smaller grid on the array the first call left behind
    for n, precision in ((32, "mixed"), (16, "fp64")):
        say(f"allocation-free case n={n} precision={precision}")
        inp = synthetic.workload_inputs("seeds3_n128", n=n)
        ref_stats, ref = _run(inp, P, precision, False, 3)
        got_stats, got = _run(inp, P, precision, True, 3)
        assert [s["it_elast"] for s in got_stats] == [s["it_elast"] for s in ref_stats]
        assert [s["it_diff"] for s in got_stats] == [s["it_diff"] for s in ref_stats]
        for k in FIELDS:
            err = rel_l2(got[k], ref[k])
            # identical kernels on identical inputs: equal up to rounding order at most
            assert err <= 1e-12, (n, precision, k, err)


def test_one_live_static_context_per_device():
    torch = need_gpu()
    P = synthetic.params()
    inp = synthetic.workload_inputs("seeds3_n128", n=16)
    say("allocation-free: second live context refused")
    a = tm.from_inputs(inp, P, no_alloc=True)
    try:
        with pytest.raises(tm.TumorError) as e:
            tm.from_inputs(inp, P, no_alloc=True)
        assert e.value.code == tm.ESTATE
    finally:
        a.close()
    b = tm.from_inputs(inp, P, no_alloc=True)      # released by close()
    b.step(1)
    assert torch.isfinite(b.get("p")).all()
    b.close()
