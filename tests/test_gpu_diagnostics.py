"""GPU mass-effect diagnostics against the FP64 oracle, through the C ABI.

After a few split steps (so that the displacement and the Lame fields are
non-trivial), tumor_diagnose's fields (stress trace, Mohr shear, Jacobian)
are compared element by element with the oracle's and its scalars with the
oracle's scalars.  The threshold of d_max is chosen away from every voxel's
displacement so that both sides select the same voxels.
"""
import numpy as np
import pytest

import paper_1810_05370_amd as tm
import synthetic
from gpu_common import need_gpu, rel_l2, say
from oracle import diagnostics as dg
from oracle.spectral import Grid

pytestmark = pytest.mark.gpu


def _threshold_away_from_voxels(umag, want):
    vals = np.sort(umag.ravel())
    t = want
    for _ in range(50):
        if np.min(np.abs(vals - t)) > 1e-6 * max(t, 1e-12):
            return t
        t *= 1.0137
    return t


def _check(sim, inp, label, tol=1e-10):
    n = inp["n"]
    g = Grid(n)
    u = sim.get("u").cpu().numpy()
    mu, lam = sim.get("mu").cpu().numpy(), sim.get("lambda").cpu().numpy()
    umag = np.sqrt((u ** 2).sum(axis=0)) / g.h
    thr = _threshold_away_from_voxels(umag, 0.1 * umag.max())
    ref_f, ref_s = dg.diagnose(g, mu, lam, u, inp["centers"], thr)
    s, f = sim.diagnose(thr, fields=True)
    f = f.cpu().numpy()
    for k, name in enumerate(("trace", "shear", "jac")):
        ref = ref_f[name] - (1.0 if name == "jac" else 0.0)
        got = f[k] - (1.0 if name == "jac" else 0.0)
        err = rel_l2(got, ref)
        say(f"{label} {name}: relL2 {err:.2e}")
        assert err < tol, name
    for key in ref_s:
        r, v = ref_s[key], s[key]
        scale = max(abs(r), 1e-300)
        if key in ("jac_min", "jac_max"):
            r, v, scale = r - 1.0, v - 1.0, max(abs(ref_s["jac_max"] - 1.0), abs(ref_s["jac_min"] - 1.0))
        say(f"  {key}: {v:.12e} (oracle {ref_s[key]:.12e})")
        assert abs(v - r) <= tol * scale, key
    assert s["d_max"] > 0.0


@pytest.mark.parametrize("n", [32, 64])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_diagnostics_match_the_oracle(n, precision):
    need_gpu()
    P = synthetic.params()
    inp = synthetic.workload_inputs("seeds3_n128", n=n)
    sim = tm.from_inputs(inp, P, precision=precision)
    sim.step(3)
    _check(sim, inp, f"n={n} {precision}")
    sim.close()


def test_no_displacement_gives_identity():
    need_gpu()
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32", n=16)
    sim = tm.from_inputs(inp, P)
    s = sim.diagnose(0.1)
    assert s["max_disp"] == 0.0 and s["jac_min"] == 1.0 and s["jac_max"] == 1.0 and s["jac_l2"] == 0.0
    assert s["d_max"] == 0.0 and s["shear_max"] == 0.0
    with pytest.raises(tm.TumorError):
        sim.diagnose(-1.0)
    sim.close()
