"""Python binding of libtumor: the MI355X split step of the multispecies
glioblastoma model with mass effect (Subramanian, Gholami & Biros).

Argument marshalling only.  Every step of the method runs in the HIP kernels
of ``libtumor.so``; PyTorch supplies device memory (the workspace and field
tensors) and the stream.  There is no CPU fallback: if the library is not
built, or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtumor.so")

# tumor_params, in the C struct order (include/tumor.h)
PARAM_FIELDS = (
    "k_w", "k_g", "k_f", "rho_w", "rho_g", "rho_inv_frac",
    "alpha0", "beta0", "gamma", "sigma_b", "o_hyp", "o_inv", "o_heal", "delta_s", "delta_p",
    "delta_e", "delta_half", "delta_l", "eta_tumor", "eta_healthy",
    "E_wm", "E_gm", "E_csf", "E_tumor", "nu_wm", "nu_gm", "nu_csf", "nu_tumor",
    "lame_scale", "zeta", "heaviside_eps", "E_bg", "nu_bg", "eta_bg",
)

OK, EINVAL, ENOMEM, ENOCONV, EDEVICE, ENAN, ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "TUMOR_OK", -1: "TUMOR_EINVAL", -2: "TUMOR_ENOMEM", -3: "TUMOR_ENOCONV",
                -4: "TUMOR_EDEVICE", -5: "TUMOR_ENAN", -6: "TUMOR_ESTATE"}
PREC = {"fp64": 0, "mixed": 1}
F_ADVECTION, F_ELASTICITY, F_EDEMA = 0x1, 0x2, 0x4
F_DEFAULT = F_ADVECTION | F_ELASTICITY | F_EDEMA
F_ADJOINT = 0x8
F_STRANG = 0x10
GRAD_NAMES = ("rho", "k_w", "k_g", "k_f", "lame_scale")
FIELDS = {"p": 0, "i": 1, "n": 2, "o": 3, "l": 4, "g": 5, "w": 6, "f": 7, "u": 8, "u_prev": 9,
          "K": 10, "rho": 11, "mu": 12, "lambda": 13, "eta": 14, "bg": 15}
OPS = {"deriv_x": 0, "deriv_y": 1, "deriv_z": 2, "diffusion": 3, "elasticity": 4,
       "elast_precond": 5, "cn_precond": 6, "force": 7}
VECTOR_OPS = ("elasticity", "elast_precond", "force")
KERNEL_CLASSES = {"colinv64": 0, "colfwd64": 1, "colinv32": 2, "colfwd32": 3, "xelast64": 4, "xelast32": 5,
                  "xdiff64": 6, "xdiff32": 7, "xother": 8, "sl": 9, "react": 10, "krylov64": 11, "krylov32": 12,
                  "zinvp64": 13, "zinvp32": 14, "coldot64": 15, "coldot32": 16, "colinv32z": 17,
                  "colfwd32z": 18, "zinvp64c1": 19, "zinvp32c1": 20, "zinvpb64": 21, "zinvpb32": 22}
# rocprofv3 kernel names of each class (for cross-checking event timings against traces)
KERNEL_NAMES = {"colinv64": "k_col_pass<double, {n}, true, false, 256>",
                "colfwd64": "k_col_pass<double, {n}, false, false, 256>",
                "colinv32": "k_col_pass<float, {n}, true, false, 128>",
                "colfwd32": "k_col_pass<float, {n}, false, false, 128>",
                "colinv32z": "k_col_pass<float, {n}, true, false, 256>",
                "colfwd32z": "k_col_pass<float, {n}, false, false, 256>",
                "coldot64": "k_col_pass<double, {n}, false, true, 256>",
                "coldot32": "k_col_pass<float, {n}, false, true, 256>",
                "zinvp64": "k_zinv_pupdate<double, {n}, 3>", "zinvp32": "k_zinv_pupdate<float, {n}, 3>",
                "zinvp64c1": "k_zinv_pupdate<double, {n}, 1>", "zinvp32c1": "k_zinv_pupdate<float, {n}, 1>",
                "zinvpb64": "k_zinv_pupdate_b<double, {n}>", "zinvpb32": "k_zinv_pupdate_b<float, {n}>",
                "xelast64": "k_xelast<double, {n}>", "xelast32": "k_xelast<float, {n}>",
                "xdiff64": "k_xdiff<double, {n}>", "xdiff32": "k_xdiff<float, {n}>", "sl": "k_sl",
                "react": "k_react"}


class TumorParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in PARAM_FIELDS]


class TumorConfig(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("precision", ctypes.c_int32), ("dt", ctypes.c_double),
                ("rtol_diff", ctypes.c_double), ("rtol_elast", ctypes.c_double),
                ("max_it", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("model", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class TumorDiagnostics(ctypes.Structure):
    _fields_ = [("max_disp", ctypes.c_double), ("trace_min", ctypes.c_double), ("trace_max", ctypes.c_double),
                ("shear_max", ctypes.c_double), ("jac_min", ctypes.c_double), ("jac_max", ctypes.c_double),
                ("jac_l2", ctypes.c_double), ("d_max", ctypes.c_double)]


class TumorStepStats(ctypes.Structure):
    _fields_ = [("it_diff", ctypes.c_int32 * 3), ("it_elast", ctypes.c_int32),
                ("outer_elast", ctypes.c_int32), ("outer_diff", ctypes.c_int32 * 3),
                ("relres_diff", ctypes.c_double * 3), ("relres_elast", ctypes.c_double),
                ("mass", ctypes.c_double * 8), ("max_cfl", ctypes.c_double)]

    def as_dict(self):
        return dict(it_diff=list(self.it_diff), it_elast=self.it_elast, outer_elast=self.outer_elast,
                    outer_diff=list(self.outer_diff), relres_diff=list(self.relres_diff),
                    relres_elast=self.relres_elast, mass=list(self.mass), max_cfl=self.max_cfl)


class TumorError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None
P = ctypes.c_void_p


def load_library(path: Optional[str] = None):
    """Load libtumor.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with __graft_entry__.build() "
                          "(python -m paper_1810_05370_amd._build)")
    lib = ctypes.CDLL(p)
    sig = {
        "tumor_abi_version": (ctypes.c_int, []),
        "tumor_last_error": (ctypes.c_char_p, []),
        "tumor_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(TumorConfig), ctypes.POINTER(ctypes.c_size_t)]),
        "tumor_init": (ctypes.c_int, [ctypes.POINTER(P), ctypes.POINTER(TumorConfig), ctypes.POINTER(TumorParams),
                                      P, ctypes.c_size_t, P, P, P, ctypes.c_int32, P, P, P, P]),
        "tumor_init_static": (ctypes.c_int, [ctypes.POINTER(P), ctypes.POINTER(TumorConfig),
                                             ctypes.POINTER(TumorParams), P, P, P, ctypes.c_int32, P, P, P, P]),
        "tumor_step": (ctypes.c_int, [P, ctypes.c_int32, ctypes.POINTER(TumorStepStats)]),
        "tumor_solve_elasticity": (ctypes.c_int, [P, P, P, ctypes.POINTER(ctypes.c_int32),
                                                  ctypes.POINTER(ctypes.c_double)]),
        "tumor_transport": (ctypes.c_int, [P, P, ctypes.POINTER(ctypes.c_double)]),
        "tumor_diagnose": (ctypes.c_int, [P, ctypes.c_double, P, ctypes.POINTER(TumorDiagnostics)]),
        "tumor_adjoint_step": (ctypes.c_int, [P, P, P]),
        "tumor_tape_bytes": (ctypes.c_int, [ctypes.POINTER(TumorConfig), ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_size_t)]),
        "tumor_record": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_size_t]),
        "tumor_state_bytes": (ctypes.c_int, [ctypes.POINTER(TumorConfig), ctypes.POINTER(ctypes.c_size_t)]),
        "tumor_save_state": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "tumor_load_state": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "tumor_get_field": (ctypes.c_int, [P, ctypes.c_int32, P]),
        "tumor_set_field": (ctypes.c_int, [P, ctypes.c_int32, P]),
        "tumor_refresh": (ctypes.c_int, [P]),
        "tumor_apply_op": (ctypes.c_int, [P, ctypes.c_int32, P, P]),
        "tumor_interp": (ctypes.c_int, [P, P, P, P, P, ctypes.c_int64, P]),
        "tumor_force_iterations": (ctypes.c_int, [P, P]),
        "tumor_kernel_timer": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32]),
        "tumor_kernel_timer_read": (ctypes.c_int, [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                                   ctypes.POINTER(ctypes.c_double),
                                                   ctypes.POINTER(ctypes.c_double)]),
        "tumor_stream_copy": (ctypes.c_int, [P, P, ctypes.c_size_t, P]),
        "tumor_substep_timer": (ctypes.c_int, [P, ctypes.c_int32]),
        "tumor_substep_timer_read": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int64), P]),
        "tumor_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(code):
    if code != OK:
        msg = load_library().tumor_last_error()
        raise TumorError(code, msg.decode() if msg else "")


def make_params(values: dict) -> TumorParams:
    missing = [k for k in PARAM_FIELDS if k not in values]
    if missing:
        raise KeyError(f"missing parameters: {missing}")
    return TumorParams(*[float(values[k]) for k in PARAM_FIELDS])


MODELS = {"multispecies": 0, "single": 1}


def make_config(n, precision="fp64", dt=0.01, rtol_diff=1e-8, rtol_elast=1e-8, max_it=1000,
                flags=F_DEFAULT, model="multispecies") -> TumorConfig:
    """model: "multispecies" or "single" (an unknown name gives an invalid code)."""
    return TumorConfig(int(n), PREC[precision], float(dt), float(rtol_diff), float(rtol_elast),
                       int(max_it), int(flags), MODELS.get(model, -1), (ctypes.c_int32 * 3)(0, 0, 0))


def workspace_bytes(cfg: TumorConfig) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().tumor_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)))
    return out.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _host_array(vals):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(vals, dtype=np.float64).ravel())
    return a, a.ctypes.data_as(ctypes.c_void_p)


class Tumor:
    """One simulation context on the current CUDA/HIP device.

    wm, gm, csf: float64 device tensors of shape (n, n, n), [z][y][x].
    centers (k, 3) as (x, y, z), sigmas (k,), weights (k,): host arrays.
    no_alloc: create the context with tumor_init_static (the library's own
    fixed workspace on the device, n <= 32; one such context per GPU at a time)
    instead of a workspace tensor.
    """

    def __init__(self, n, params: dict, wm, gm, csf, centers=(), sigmas=(), weights=(),
                 precision="fp64", dt=0.01, rtol_diff=1e-8, rtol_elast=1e-8, max_it=1000,
                 flags=F_DEFAULT, stream=None, model="multispecies", no_alloc=False):
        import torch
        self._torch = torch
        lib = load_library()
        self.lib = lib
        self.n = int(n)
        self.cfg = make_config(n, precision, dt, rtol_diff, rtol_elast, max_it, flags, model)
        self.prm = make_params(params)
        dev = wm.device
        self.device = dev
        if no_alloc:
            self.workspace = None
        else:
            nb = workspace_bytes(self.cfg)
            self.workspace = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
            base = self.workspace.data_ptr()
            off = (-base) % 256
            self._ws_ptr = ctypes.c_void_p(base + off)
            self._ws_bytes = nb
        for t in (wm, gm, csf):
            if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != (n, n, n):
                raise ValueError("tissue maps must be contiguous float64 (n, n, n) device tensors")
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        c, cp = _host_array(centers)
        s, sp = _host_array(sigmas)
        w, wp = _host_array(weights)
        nic = s.size
        if c.size != 3 * nic or w.size != nic:
            raise ValueError("centers must be (k, 3), sigmas and weights (k,)")
        ctx = ctypes.c_void_p()
        torch.cuda.synchronize(dev)
        ic = (cp if nic else None, sp if nic else None, wp if nic else None)
        if no_alloc:
            code = lib.tumor_init_static(ctypes.byref(ctx), ctypes.byref(self.cfg), ctypes.byref(self.prm),
                                         _ptr(wm), _ptr(gm), _ptr(csf), nic, *ic,
                                         ctypes.c_void_p(self.stream.cuda_stream))
        else:
            code = lib.tumor_init(ctypes.byref(ctx), ctypes.byref(self.cfg), ctypes.byref(self.prm),
                                  self._ws_ptr, self._ws_bytes, _ptr(wm), _ptr(gm), _ptr(csf), nic, *ic,
                                  ctypes.c_void_p(self.stream.cuda_stream))
        _check(code)
        self.ctx = ctx
        self.n_ic = nic

    # -- lifetime ------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            self.lib.tumor_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- method --------------------------------------------------------
    def step(self, nsteps=1, allow_noconv=False):
        st = TumorStepStats()
        code = self.lib.tumor_step(self.ctx, int(nsteps), ctypes.byref(st))
        if code == ENOCONV and allow_noconv:
            return st.as_dict()
        _check(code)
        return st.as_dict()

    def solve_elasticity(self, force=None):
        torch = self._torch
        n = self.n
        u = torch.empty((3, n, n, n), dtype=torch.float64, device=self.device)
        it = ctypes.c_int32(0)
        rr = ctypes.c_double(0)
        if force is not None:
            force = force.contiguous()
        _check(self.lib.tumor_solve_elasticity(self.ctx, _ptr(force) if force is not None else None,
                                               _ptr(u), ctypes.byref(it), ctypes.byref(rr)))
        return u, it.value, rr.value

    def transport(self):
        """The transport sub-step alone: (6, N, N, N) tensor of the transported
        p, i, n, g, w, f, and max |dt v| / h.  The state is unchanged."""
        torch = self._torch
        n = self.n
        out = torch.empty((6, n, n, n), dtype=torch.float64, device=self.device)
        cfl = ctypes.c_double(0)
        _check(self.lib.tumor_transport(self.ctx, _ptr(out), ctypes.byref(cfl)))
        return out, cfl.value

    def diagnose(self, threshold=0.1, fields=False):
        """Mass-effect diagnostics of the current displacement: a dict of the
        scalars, plus a (3, N, N, N) tensor (stress trace, Mohr shear,
        Jacobian) when fields is true."""
        torch = self._torch
        n = self.n
        out = TumorDiagnostics()
        f = torch.empty((3, n, n, n), dtype=torch.float64, device=self.device) if fields else None
        _check(self.lib.tumor_diagnose(self.ctx, float(threshold), _ptr(f) if fields else None, ctypes.byref(out)))
        d = {k: getattr(out, k) for k, _ in TumorDiagnostics._fields_}
        return (d, f) if fields else d

    def state_bytes(self):
        out = ctypes.c_size_t(0)
        _check(self.lib.tumor_state_bytes(ctypes.byref(self.cfg), ctypes.byref(out)))
        return out.value

    def save_state(self, dst=None):
        """Snapshot of the time-stepping state (species, u^n, u^{n-1}) in a
        device uint8 tensor (``dst`` if given)."""
        nb = self.state_bytes()
        if dst is None:
            dst = self._torch.empty(nb, dtype=self._torch.uint8, device=self.device)
        if dst.numel() * dst.element_size() < nb or not dst.is_contiguous():
            raise ValueError("snapshot buffer too small or not contiguous")
        _check(self.lib.tumor_save_state(self.ctx, _ptr(dst), nb))
        return dst

    def load_state(self, src):
        """Restore a snapshot taken by save_state (the coefficients are refreshed)."""
        nb = src.numel() * src.element_size()
        _check(self.lib.tumor_load_state(self.ctx, _ptr(src.contiguous()), nb))

    def get(self, name):
        torch = self._torch
        n = self.n
        fid = FIELDS[name]
        shape = (3, n, n, n) if name in ("u", "u_prev") else (n, n, n)
        out = torch.empty(shape, dtype=torch.float64, device=self.device)
        _check(self.lib.tumor_get_field(self.ctx, fid, _ptr(out)))
        return out

    def set(self, name, value):
        v = value.to(device=self.device, dtype=self._torch.float64).contiguous()
        _check(self.lib.tumor_set_field(self.ctx, FIELDS[name], _ptr(v)))

    def refresh(self):
        _check(self.lib.tumor_refresh(self.ctx))

    def apply_op(self, name, x):
        torch = self._torch
        n = self.n
        x = x.to(device=self.device, dtype=torch.float64).contiguous()
        shape = (3, n, n, n) if name in VECTOR_OPS else (n, n, n)
        out = torch.empty(shape, dtype=torch.float64, device=self.device)
        _check(self.lib.tumor_apply_op(self.ctx, OPS[name], _ptr(x), _ptr(out)))
        return out

    def interp(self, q, jx, jy, jz):
        torch = self._torch
        q = q.to(device=self.device, dtype=torch.float64).contiguous()
        pts = [a.to(device=self.device, dtype=torch.float64).contiguous() for a in (jx, jy, jz)]
        out = torch.empty(pts[0].shape, dtype=torch.float64, device=self.device)
        _check(self.lib.tumor_interp(self.ctx, _ptr(q), _ptr(pts[0]), _ptr(pts[1]), _ptr(pts[2]),
                                     pts[0].numel(), _ptr(out)))
        return out

    def kernel_timer(self, name, enable=True):
        _check(self.lib.tumor_kernel_timer(self.ctx, KERNEL_CLASSES[name], 1 if enable else 0))

    def kernel_timer_read(self, name):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0)
        b = ctypes.c_double(0)
        _check(self.lib.tumor_kernel_timer_read(self.ctx, KERNEL_CLASSES[name], ctypes.byref(n),
                                                ctypes.byref(ms), ctypes.byref(b)))
        return dict(launches=n.value, ms=ms.value, bytes=b.value)

    SUBSTEPS = ("transport", "diffusion", "reaction", "elasticity")

    def substep_timer(self, enable=True):
        _check(self.lib.tumor_substep_timer(self.ctx, 1 if enable else 0))

    def substep_timer_read(self):
        """(steps timed, {sub-step: summed ms})."""
        import numpy as np
        n = ctypes.c_int64(0)
        ms = np.zeros(4)
        _check(self.lib.tumor_substep_timer_read(self.ctx, ctypes.byref(n), ms.ctypes.data_as(ctypes.c_void_p)))
        return n.value, dict(zip(self.SUBSTEPS, (float(v) for v in ms)))

    # -- adjoint ---------------------------------------------------------
    def record(self, nsteps, ckpt_every=1):
        """Record the next ``nsteps`` steps for the adjoint (checkpoint every ``ckpt_every``)."""
        torch = self._torch
        nb = ctypes.c_size_t(0)
        _check(self.lib.tumor_tape_bytes(ctypes.byref(self.cfg), int(nsteps), int(ckpt_every), ctypes.byref(nb)))
        self.tape = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        base = self.tape.data_ptr()
        ptr = base + ((-base) % 256)
        _check(self.lib.tumor_record(self.ctx, int(nsteps), int(ckpt_every), ctypes.c_void_p(ptr), nb.value))
        self.tape_bytes = nb.value

    def adjoint_step(self, adj, grad):
        """Reverse one recorded step.  adj: (14, n, n, n) float64 device tensor, updated in
        place.  grad: float64 numpy array of 5 + n_ic entries, accumulated in place."""
        import numpy as np
        assert adj.dtype == self._torch.float64 and adj.is_contiguous() and adj.numel() == 14 * self.n ** 3
        assert isinstance(grad, np.ndarray) and grad.dtype == np.float64 and grad.size == 5 + self.n_ic
        _check(self.lib.tumor_adjoint_step(self.ctx, _ptr(adj), grad.ctypes.data_as(ctypes.c_void_p)))

    def force_iterations(self, iters=None):
        if iters is None:
            _check(self.lib.tumor_force_iterations(self.ctx, None))
            return
        arr = (ctypes.c_int32 * 4)(*[int(v) for v in iters])
        _check(self.lib.tumor_force_iterations(self.ctx, ctypes.cast(arr, ctypes.c_void_p)))


def stream_copy(src, dst, stream=None):
    """Copy the bytes of device tensor src into dst with the library's streaming
    copy kernel (measurement hook; queued on `stream`, torch's current if None)."""
    import torch
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nb or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("dst must be contiguous and hold src")
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    _check(load_library().tumor_stream_copy(_ptr(src), _ptr(dst), nb, ctypes.c_void_p(st.cuda_stream)))


def from_inputs(inputs: dict, params: dict, device="cuda", **kw) -> Tumor:
    """Build a context from a ``synthetic.workload_inputs`` dictionary (with
    the background fraction set and the coefficients refreshed when the
    inputs carry one)."""
    import torch
    n = inputs["n"]
    t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
    sim = Tumor(n, params, t(inputs["wm"]), t(inputs["gm"]), t(inputs["csf"]),
                inputs["centers"], inputs["sigmas"], inputs["weights"], **kw)
    if inputs.get("bg") is not None:
        sim.set("bg", t(inputs["bg"]))
        sim.refresh()
    return sim
