"""C-ABI checks that need no GPU: the library loads, exports every entry point
the header declares, agrees with the header on struct layouts, and rejects
invalid arguments before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1810_05370_amd as tm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tumor.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tumor_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return tm.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_abi_version(lib):
    assert lib.tumor_abi_version() == 3


def test_struct_layouts_match_the_header(tmp_path):
    probe = tmp_path / "probe.c"
    probe.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "tumor.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(tumor_params), sizeof(tumor_config), sizeof(tumor_step_stats));
  printf("%zu %zu %zu %zu\n", offsetof(tumor_config, dt), offsetof(tumor_config, max_it),
         offsetof(tumor_config, reserved), offsetof(tumor_params, heaviside_eps));
  printf("%zu %zu %zu\n", offsetof(tumor_step_stats, relres_diff), offsetof(tumor_step_stats, mass),
         offsetof(tumor_step_stats, max_cfl));
  printf("%zu %zu %zu\n", sizeof(tumor_diagnostics), offsetof(tumor_diagnostics, jac_l2),
         offsetof(tumor_diagnostics, d_max));
  return 0;
}
''')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = [int(v) for v in out]
    c = ctypes
    want = [c.sizeof(tm.TumorParams), c.sizeof(tm.TumorConfig), c.sizeof(tm.TumorStepStats),
            tm.TumorConfig.dt.offset, tm.TumorConfig.max_it.offset, tm.TumorConfig.reserved.offset,
            tm.TumorParams.heaviside_eps.offset, tm.TumorStepStats.relres_diff.offset,
            tm.TumorStepStats.mass.offset, tm.TumorStepStats.max_cfl.offset,
            c.sizeof(tm.TumorDiagnostics), tm.TumorDiagnostics.jac_l2.offset, tm.TumorDiagnostics.d_max.offset]
    assert got == want


def test_param_names_cover_the_synthetic_presets():
    import synthetic
    assert set(tm.PARAM_FIELDS) == set(synthetic.TABLE_SETUP)


def test_workspace_size_and_validation(lib):
    b64 = tm.workspace_bytes(tm.make_config(64))
    bmx = tm.workspace_bytes(tm.make_config(64, "mixed"))
    assert b64 > 60 * 64 ** 3 * 8 and bmx > b64
    for bad in (dict(n=100), dict(n=8), dict(n=1024), dict(n=32, dt=0.0), dict(n=32, rtol_diff=1.0),
                dict(n=32, max_it=0), dict(n=32, flags=0x20), dict(n=32, model="nonsense"),
                dict(n=32, model="single", flags=0x7 | 0x8), dict(n=32, flags=0x7 | 0x8 | 0x10)):
        with pytest.raises(tm.TumorError) as e:
            tm.workspace_bytes(tm.make_config(**bad))
        assert e.value.code == tm.EINVAL
    assert tm.workspace_bytes(tm.make_config(32, flags=tm.F_DEFAULT | tm.F_STRANG)) == tm.workspace_bytes(
        tm.make_config(32))
    cfg = tm.make_config(32)
    cfg.reserved[1] = 3
    with pytest.raises(tm.TumorError):
        tm.workspace_bytes(cfg)
    assert lib.tumor_workspace_bytes(ctypes.byref(tm.make_config(32)), None) == tm.EINVAL


def test_calls_reject_null_context_before_device_work(lib):
    assert lib.tumor_step(None, 1, None) == tm.EINVAL
    assert lib.tumor_get_field(None, 0, None) == tm.EINVAL
    assert lib.tumor_set_field(None, 0, None) == tm.EINVAL
    assert lib.tumor_apply_op(None, 0, None, None) == tm.EINVAL
    assert lib.tumor_solve_elasticity(None, None, None, None, None) == tm.EINVAL
    assert lib.tumor_interp(None, None, None, None, None, 0, None) == tm.EINVAL
    assert lib.tumor_refresh(None) == tm.EINVAL
    assert lib.tumor_adjoint_step(None, None, None) == tm.EINVAL
    lib.tumor_destroy(None)
    assert b"ctx" in lib.tumor_last_error()


def test_init_validates_arguments_before_the_device(lib):
    import synthetic
    cfg = tm.make_config(16)
    prm = tm.make_params(synthetic.params())
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    # NULL workspace
    assert lib.tumor_init(ctypes.byref(ctx), ctypes.byref(cfg), ctypes.byref(prm), None, 1 << 30,
                          fake, fake, fake, 0, None, None, None, None) == tm.EINVAL
    # misaligned workspace
    assert lib.tumor_init(ctypes.byref(ctx), ctypes.byref(cfg), ctypes.byref(prm), ctypes.c_void_p(0x1008),
                          1 << 30, fake, fake, fake, 0, None, None, None, None) == tm.EINVAL
    # too small workspace
    assert lib.tumor_init(ctypes.byref(ctx), ctypes.byref(cfg), ctypes.byref(prm), fake, 1024,
                          fake, fake, fake, 0, None, None, None, None) == tm.ENOMEM
    # invalid parameters (Poisson ratio 0.5, non-positive Heaviside width)
    bad = synthetic.params(nu_tumor=0.5)
    assert lib.tumor_init(ctypes.byref(ctx), ctypes.byref(cfg), ctypes.byref(tm.make_params(bad)), fake,
                          1 << 30, fake, fake, fake, 0, None, None, None, None) == tm.EINVAL
    bad = synthetic.params(heaviside_eps=0.0)
    assert lib.tumor_init(ctypes.byref(ctx), ctypes.byref(cfg), ctypes.byref(tm.make_params(bad)), fake,
                          1 << 30, fake, fake, fake, 0, None, None, None, None) == tm.EINVAL
    # no screening at all (e:screening): the elasticity system would have no solution
    bad = synthetic.params(eta_tumor=0.0, eta_healthy=0.0, eta_bg=0.0)
    assert lib.tumor_init(ctypes.byref(ctx), ctypes.byref(cfg), ctypes.byref(tm.make_params(bad)), fake,
                          1 << 30, fake, fake, fake, 0, None, None, None, None) == tm.EINVAL
    # negative width of a tumour seed
    s = (ctypes.c_double * 1)(-0.3)
    c3 = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    w = (ctypes.c_double * 1)(0.5)
    assert lib.tumor_init(ctypes.byref(ctx), ctypes.byref(cfg), ctypes.byref(prm), fake, 1 << 30,
                          fake, fake, fake, 1, ctypes.cast(c3, ctypes.c_void_p), ctypes.cast(s, ctypes.c_void_p),
                          ctypes.cast(w, ctypes.c_void_p), None) == tm.EINVAL
    assert not ctx.value


def test_static_init_rejects_oversize_configurations_before_the_device(lib):
    """tumor_init_static: a workspace beyond TUMOR_STATIC_WS_BYTES (n > 32) or
    more than 256 seeds is refused with a message, before any device call."""
    import synthetic
    prm = tm.make_params(synthetic.params())
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    for n, prec in ((64, "fp64"), (64, "mixed"), (128, "fp64")):
        cfg = tm.make_config(n, prec)
        assert lib.tumor_init_static(ctypes.byref(ctx), ctypes.byref(cfg), ctypes.byref(prm), fake, fake, fake,
                                     0, None, None, None, None) == tm.EINVAL
        assert b"allocation-free" in lib.tumor_last_error()
    # every n <= 32 fits, in both precisions and with the adjoint scratch
    for prec in ("fp64", "mixed"):
        assert tm.workspace_bytes(tm.make_config(32, prec, flags=tm.F_DEFAULT | tm.F_ADJOINT)) <= 32 << 20
    k = 257
    c3 = (ctypes.c_double * (3 * k))(*([1.0] * 3 * k))
    s = (ctypes.c_double * k)(*([0.2] * k))
    w = (ctypes.c_double * k)(*([0.1] * k))
    cfg = tm.make_config(32)
    assert lib.tumor_init_static(ctypes.byref(ctx), ctypes.byref(cfg), ctypes.byref(prm), fake, fake, fake, k,
                                 ctypes.cast(c3, ctypes.c_void_p), ctypes.cast(s, ctypes.c_void_p),
                                 ctypes.cast(w, ctypes.c_void_p), None) == tm.EINVAL
    assert lib.tumor_init_static(None, ctypes.byref(cfg), ctypes.byref(prm), fake, fake, fake, 0,
                                 None, None, None, None) == tm.EINVAL
    assert not ctx.value


def test_stream_copy_validates_before_the_device(lib):
    fake = ctypes.c_void_p(0x1000)
    assert lib.tumor_stream_copy(None, fake, 16, None) == tm.EINVAL
    assert lib.tumor_stream_copy(fake, fake, 24, None) == tm.EINVAL             # not a multiple of 16
    assert lib.tumor_stream_copy(ctypes.c_void_p(0x1008), fake, 32, None) == tm.EINVAL   # misaligned
