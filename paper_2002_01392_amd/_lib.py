"""ctypes binding of libfcns.so (argument marshalling only).

Every computation runs in the HIP kernels behind the C ABI declared in
``include/fcns.h``; this module only converts torch device tensors to
pointers, keeps the context alive and raises on error codes.  There is no
CPU fallback: without the built library or a HIP device it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfcns.so")

FCNS_OK, FCNS_EINVAL, FCNS_ENOMEM, FCNS_EDEVICE, FCNS_ENONFINITE, FCNS_ESTATE = 0, -1, -2, -3, -4, -5
FCNS_ECANCELED = -6
FCNS_CHECK_OFF, FCNS_CHECK_SYNC, FCNS_CHECK_DEFERRED = 0, 1, 2
FCNS_FP64, FCNS_MIXED = 0, 1
_PRECISIONS = {"fp64": FCNS_FP64, "mixed": FCNS_MIXED}


class FcnsProblem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
        ("fc_d", ctypes.c_int32), ("fc_C", ctypes.c_int32),
        ("fc_table", ctypes.POINTER(ctypes.c_double)),
        ("nu", ctypes.c_double), ("forcing_x", ctypes.c_double),
        ("boussinesq", ctypes.c_int32),
        ("kappa", ctypes.c_double), ("gamma", ctypes.c_double),
        ("rk_order", ctypes.c_int32),
        ("filter_beta", ctypes.c_double), ("filter_2p", ctypes.c_double),
        ("precision", ctypes.c_int32), ("keep_pressure", ctypes.c_int32),
    ]


# name -> (restype, argtypes)
_P, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
SIGNATURES = {
    "fcns_create": (ctypes.c_int, [ctypes.POINTER(FcnsProblem), _P, ctypes.POINTER(_P)]),
    "fcns_destroy": (ctypes.c_int, [_P]),
    "fcns_fc_extend": (ctypes.c_int, [_P, _P, _I64, _I64, _I64, _P, _I64, _I64]),
    "fcns_fc_derivative": (ctypes.c_int, [_P, _I32, _P, _I64, _I64, _I64, _P]),
    "fcns_fc_derivative_noalloc": (ctypes.c_int, [_I32, _D, _I32, _I32, _P, _I32, _P, _I64,
                                                  _I64, _I64, _P, _P]),
    "fcns_rhs_nonlinear": (ctypes.c_int, [_P, _P, _P, _I32, _P, _P]),
    "fcns_pressure_project": (ctypes.c_int, [_P, _P, _D, _P, _P]),
    "fcns_set_state": (ctypes.c_int, [_P, _P, _P]),
    "fcns_rk_step": (ctypes.c_int, [_P, _D, _I32]),
    "fcns_rk_graph": (ctypes.c_int, [_P, _D, _I32]),
    "fcns_set_finite_check": (ctypes.c_int, [_P, _I32]),
    "fcns_set_z_fused": (ctypes.c_int, [_P, _I32]),
    "fcns_set_slab": (ctypes.c_int, [_P, _I32]),
    "fcns_set_blocked": (ctypes.c_int, [_P, _I32]),
    "fcns_set_y_lines": (ctypes.c_int, [_P, _I32]),
    "fcns_get_choices": (ctypes.c_int, [_P, ctypes.c_char_p, _I32]),
    "fcns_set_choices": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "fcns_check_finite": (ctypes.c_int, [_P]),
    "fcns_nonfinite_flag": (ctypes.c_int32, [_P]),
    "fcns_autotune": (ctypes.c_int, [_P, ctypes.c_char_p, _I32]),
    "fcns_batch_step": (ctypes.c_int, [ctypes.POINTER(_P), _I32, ctypes.POINTER(_D),
                                       ctypes.POINTER(_I32)]),
    "fcns_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), _I32, ctypes.POINTER(_D),
                                         ctypes.POINTER(_P)]),
    "fcns_batch_run": (ctypes.c_int, [_P, _I32]),
    "fcns_batch_destroy": (ctypes.c_int, [_P]),
    "fcns_get_state": (ctypes.c_int, [_P, _P, _P, _P]),
    "fcns_get_spectral": (ctypes.c_int, [_P, _I32, _P]),
    "fcns_set_spectral": (ctypes.c_int, [_P, ctypes.POINTER(_P), _P]),
    "fcns_get_wall_grad": (ctypes.c_int, [_P, _P]),
    "fcns_npr": (ctypes.c_int32, [_P]),
    "fcns_set_timing": (ctypes.c_int, [_P, _I32]),
    "fcns_set_timing_mask": (ctypes.c_int, [_P, _I32]),
    "fcns_timing_reset": (ctypes.c_int, [_P]),
    "fcns_timing_report": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_I32), _P, _P, _P]),
    "fcns_last_error": (ctypes.c_char_p, [_P]),
    "fcns_footprint": (ctypes.c_int, [ctypes.POINTER(FcnsProblem), ctypes.POINTER(_I64)]),
    "fcns_diagnostics": (ctypes.c_int, [_P, _P, _I32]),
    "fcns_spectra": (ctypes.c_int, [_P, _I32, _I32, _P, _P]),
    "fcns_set_params": (ctypes.c_int, [_P, _D, _D, _D, _D]),
    "fcns_stream": (_P, [_P]),
    "fcns_server_create": (ctypes.c_int, [_I32, _I64, ctypes.POINTER(_P)]),
    "fcns_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(FcnsProblem), _P, _P, _D, _I32,
                                          _P, _P, ctypes.POINTER(_I64)]),
    "fcns_server_poll": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                        ctypes.POINTER(_I64)]),
    "fcns_server_now": (_D, [_P]),
    "fcns_server_result": (ctypes.c_int, [_P, _I64, _P]),
    "fcns_server_step_times": (ctypes.c_int, [_P, _I64, _I32, _P, ctypes.POINTER(_I32)]),
    "fcns_server_release": (ctypes.c_int, [_P, _I64]),
    "fcns_server_cancel": (ctypes.c_int, [_P, _I64]),
    "fcns_server_set_choices": (ctypes.c_int, [_P, ctypes.POINTER(FcnsProblem), ctypes.c_char_p]),
    "fcns_server_set_mix": (ctypes.c_int, [_P, _I32, _I64]),
    "fcns_server_destroy": (ctypes.c_int, [_P]),
    "fcns_server_last_error": (ctypes.c_char_p, [_P]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libfcns.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2002_01392_amd.build.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class FcnsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fcns error {code}: {msg}")
        self.code = code


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def make_problem(nx, ny, nz, lx, ly, lz, nu, d=5, C=25, forcing_x=0.0, boussinesq=False,
                 kappa=0.0, gamma=0.0, keep_pressure=False, filter_beta=0.0, filter_2p=0.0,
                 rk_order=2, precision="fp64", table=None):
    """The fcns_problem struct and the FC table array it points to (keep the
    array alive as long as the struct is used)."""
    from . import fctable
    tab = np.ascontiguousarray(table if table is not None else fctable.load(d, C),
                               dtype=np.float64)
    prob = FcnsProblem(nx, ny, nz, lx, ly, lz, d, C,
                       tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       nu, forcing_x, int(bool(boussinesq)), kappa, gamma, int(rk_order),
                       filter_beta, filter_2p, _PRECISIONS[precision], int(bool(keep_pressure)))
    return prob, tab


def workload_problem(w, **kw):
    return make_problem(w.nx, w.ny, w.nz, w.lx, w.ly, w.lz, w.nu, d=w.d, C=w.C,
                        forcing_x=w.forcing_x, boussinesq=w.boussinesq, kappa=w.kappa,
                        gamma=w.gamma, **kw)


def batch_step(solvers, dts, nsteps):
    """Step several solvers together (fcns_batch_step): their launches are
    interleaved step by step, each on the solver's own stream."""
    lib = load_library()
    n = len(solvers)
    ctxs = (_P * n)(*[s.ctx for s in solvers])
    dt = (_D * n)(*[float(x) for x in dts])
    ns = (_I32 * n)(*[int(x) for x in nsteps])
    st = lib.fcns_batch_step(ctxs, n, dt, ns)
    if st != FCNS_OK:
        raise FcnsError(st, "batch_step")


class Batch:
    """Several solvers (FP64, N' <= 288, one rk_order, any shapes) stepped
    together with one fused z-pass launch per RK stage for all of them
    (fcns_batch_*)."""

    def __init__(self, solvers, dts):
        self.lib = load_library()
        self.solvers = list(solvers)
        n = len(self.solvers)
        ctxs = (_P * n)(*[s.ctx for s in self.solvers])
        dt = (_D * n)(*[float(x) for x in dts])
        h = _P()
        st = self.lib.fcns_batch_create(ctxs, n, dt, ctypes.byref(h))
        if st != FCNS_OK:
            raise FcnsError(st, self.lib.fcns_last_error(self.solvers[0].ctx).decode()
                            or self.lib.fcns_last_error(None).decode())
        self.h = h

    def run(self, nsteps):
        st = self.lib.fcns_batch_run(self.h, int(nsteps))
        if st != FCNS_OK:
            raise FcnsError(st, "batch_run")

    def close(self):
        if getattr(self, "h", None):
            self.lib.fcns_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint(prob):
    lib = load_library()
    b = ctypes.c_int64()
    st = lib.fcns_footprint(ctypes.byref(prob), ctypes.byref(b))
    if st != FCNS_OK:
        raise FcnsError(st, "footprint")
    return b.value


class Server:
    """The library's request loop (fcns_server_*): host numpy in and out."""

    def __init__(self, max_active=8, max_bytes=64 << 30):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the server runs only on the GPU")
        self.lib = load_library()
        h = ctypes.c_void_p()
        st = self.lib.fcns_server_create(int(max_active), int(max_bytes), ctypes.byref(h))
        if st != FCNS_OK:
            raise FcnsError(st, "server_create")
        self.srv = h
        self.arrays = {}   # per request: inputs and outputs the library reads / writes

    def _check(self, st):
        if st != FCNS_OK:
            raise FcnsError(st, self.lib.fcns_server_last_error(self.srv).decode())

    def set_mix(self, max_large, large_points):
        """At most max_large running requests of >= large_points grid points."""
        self._check(self.lib.fcns_server_set_mix(self.srv, int(max_large), int(large_points)))

    def set_choices(self, prob, text):
        """Launch choices for every context of prob's shape created from now on."""
        self._check(self.lib.fcns_server_set_choices(self.srv, ctypes.byref(prob),
                                                     text.encode()))

    def submit(self, prob, v0, theta0, dt, nsteps):
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        th = None if theta0 is None else np.ascontiguousarray(theta0, dtype=np.float64)
        vo = np.empty_like(v0)
        tho = None if th is None else np.empty_like(th)
        addr = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        rid = ctypes.c_int64()
        self._check(self.lib.fcns_server_submit(
            self.srv, ctypes.byref(prob), addr(v0), addr(th), float(dt), int(nsteps), addr(vo),
            addr(tho), ctypes.byref(rid)))
        self.arrays[rid.value] = (v0, th, vo, tho)
        return rid.value

    def poll(self):
        q, a, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        self._check(self.lib.fcns_server_poll(self.srv, ctypes.byref(q), ctypes.byref(a),
                                              ctypes.byref(d)))
        return q.value, a.value, d.value

    def now(self):
        return self.lib.fcns_server_now(self.srv)

    def result(self, rid):
        _, _, v, th = self.arrays[rid]
        stats = np.zeros(6)
        st = self.lib.fcns_server_result(self.srv, rid, stats.ctypes.data_as(ctypes.c_void_p))
        if st not in (FCNS_OK, FCNS_ENONFINITE, FCNS_ECANCELED):
            self._check(st)
        keys = ("t_submit", "t_admit", "t_done", "step_ms_mean", "step_ms_p50", "step_ms_max")
        info = dict(zip(keys, stats.tolist()))
        info["finite"] = st == FCNS_OK
        info["status"] = st
        return v, th, info

    def cancel(self, rid):
        self._check(self.lib.fcns_server_cancel(self.srv, rid))

    def step_times(self, rid, maxn=1 << 16):
        ms = np.zeros(maxn, dtype=np.float32)
        n = ctypes.c_int32()
        self._check(self.lib.fcns_server_step_times(self.srv, rid, maxn,
                                                    ms.ctypes.data_as(ctypes.c_void_p),
                                                    ctypes.byref(n)))
        return ms[:n.value].copy()

    def release(self, rid):
        self._check(self.lib.fcns_server_release(self.srv, rid))
        self.arrays.pop(rid, None)

    def close(self):
        if getattr(self, "srv", None):
            self.lib.fcns_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """One solver context on the current torch stream of `device`.

    Inputs and outputs are float64 torch tensors on the HIP device:
    physical fields (nz, ny, nx); vectors (3, nz, ny, nx).
    """

    def __init__(self, nx, ny, nz, lx, ly, lz, nu, d=5, C=25, forcing_x=0.0,
                 boussinesq=False, kappa=0.0, gamma=0.0, keep_pressure=False,
                 filter_beta=0.0, filter_2p=0.0, rk_order=2, precision="fp64", table=None,
                 device="cuda:0", stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the solver runs only on the GPU")
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        prob, tab = make_problem(nx, ny, nz, lx, ly, lz, nu, d=d, C=C, forcing_x=forcing_x,
                                 boussinesq=boussinesq, kappa=kappa, gamma=gamma,
                                 keep_pressure=keep_pressure, filter_beta=filter_beta,
                                 filter_2p=filter_2p, rk_order=rk_order, precision=precision,
                                 table=table)
        self._table = tab
        self.shape = (nz, ny, nx)
        self.nx, self.ny, self.nz, self.d, self.C = nx, ny, nz, d, C
        self.npr = nz + C
        self.boussinesq = bool(boussinesq)
        self.rk_order = int(rk_order)
        self.precision = precision
        self.lx, self.ly, self.lz = lx, ly, lz
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.fcns_create(ctypes.byref(prob), ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(h))
        if st != FCNS_OK:
            raise FcnsError(st, self.lib.fcns_last_error(None).decode())
        self.ctx = h

    @classmethod
    def from_workload(cls, w, **kw):
        return cls(w.nx, w.ny, w.nz, w.lx, w.ly, w.lz, w.nu, d=w.d, C=w.C,
                   forcing_x=w.forcing_x, boussinesq=w.boussinesq, kappa=w.kappa,
                   gamma=w.gamma, **kw)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.fcns_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -----------------------------------------------------------
    def _check(self, st):
        if st != FCNS_OK:
            raise FcnsError(st, self.lib.fcns_last_error(self.ctx).decode())

    # Inputs are staged and outputs allocated on the solver's stream, so the
    # library's work on that stream is ordered after the copies and the
    # allocator keeps the buffers until that stream is done with them.
    def _dev(self, a, shape=None):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        with t.cuda.stream(self.stream):
            a = a.to(device=self.device, dtype=t.float64).contiguous()
        if shape is not None and tuple(a.shape) != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {tuple(a.shape)}")
        return a

    def _empty(self, *shape):
        with self.torch.cuda.stream(self.stream):
            return self.torch.empty(shape, dtype=self.torch.float64, device=self.device)

    # -- entry points ----------------------------------------------------------
    def fc_extend(self, lines):
        f = self._dev(lines)
        nl = f.shape[0]
        if f.shape[1] != self.nz:
            raise ValueError("lines must have nz points")
        out = self._empty(nl, self.npr)
        self._check(self.lib.fcns_fc_extend(self.ctx, _ptr(f), nl, 1, self.nz, _ptr(out), 1,
                                            self.npr))
        self._keep = (f, out)
        return out

    def fc_derivative(self, lines, order=1):
        f = self._dev(lines)
        nl = f.shape[0]
        out = self._empty(nl, self.nz)
        self._check(self.lib.fcns_fc_derivative(self.ctx, order, _ptr(f), nl, 1, self.nz,
                                                _ptr(out)))
        self._keep = (f, out)
        return out

    def set_state(self, v, theta=None):
        v = self._dev(v, (3,) + self.shape)
        th = self._dev(theta, self.shape) if theta is not None else None
        self._check(self.lib.fcns_set_state(self.ctx, _ptr(v), _ptr(th)))
        self._keep = (v, th)

    def rk_step(self, dt, nsteps=1):
        self._check(self.lib.fcns_rk_step(self.ctx, float(dt), int(nsteps)))

    def set_finite_check(self, mode):
        """"off", "sync" (rk_step waits and raises on a non-finite state) or
        "deferred" (check_finite reports)."""
        modes = {"off": FCNS_CHECK_OFF, "sync": FCNS_CHECK_SYNC, "deferred": FCNS_CHECK_DEFERRED}
        self._check(self.lib.fcns_set_finite_check(self.ctx, modes[mode]))

    def check_finite(self):
        self._check(self.lib.fcns_check_finite(self.ctx))

    def set_z_fused(self, on=True):
        """Run each stage's z pass as one fused kernel (FP64, N' <= 288)."""
        self._check(self.lib.fcns_set_z_fused(self.ctx, int(bool(on))))

    def set_slab(self, planes):
        """Run rk_step's y and x passes slab by slab, `planes` z planes at a
        time (0: whole arrays)."""
        self._check(self.lib.fcns_set_slab(self.ctx, int(planes)))

    def set_blocked(self, on=True):
        """Keep rk_step's (kx, y) intermediates in the blocked layout."""
        self._check(self.lib.fcns_set_blocked(self.ctx, int(bool(on))))

    def set_y_lines(self, lines):
        """Lines per y-transform tile: 4, or 8 at ny = 512."""
        self._check(self.lib.fcns_set_y_lines(self.ctx, int(lines)))

    def choices(self):
        """The launch choices as text (see set_choices)."""
        buf = ctypes.create_string_buffer(512)
        self._check(self.lib.fcns_get_choices(self.ctx, buf, len(buf)))
        return buf.value.decode()

    def set_choices(self, text):
        """Apply launch choices saved by choices() (no autotuning)."""
        self._check(self.lib.fcns_set_choices(self.ctx, text.encode()))

    def autotune(self):
        """Pick the fastest launch choices for this shape; returns the summary."""
        buf = ctypes.create_string_buffer(1024)
        self._check(self.lib.fcns_autotune(self.ctx, buf, len(buf)))
        return buf.value.decode()

    def rk_graph(self, dt, nsteps=1):
        self._check(self.lib.fcns_rk_graph(self.ctx, float(dt), int(nsteps)))

    def get_state(self, pressure=False):
        v = self._empty(3, *self.shape)
        th = self._empty(*self.shape) if self.boussinesq else None
        p = self._empty(*self.shape) if pressure else None
        self._check(self.lib.fcns_get_state(self.ctx, _ptr(v), _ptr(th), _ptr(p)))
        return v, th, p

    def rhs_nonlinear(self, v, theta=None, filtered=False):
        v = self._dev(v, (3,) + self.shape)
        th = self._dev(theta, self.shape) if theta is not None else None
        nlv = self._empty(3, *self.shape)
        nlt = self._empty(*self.shape) if th is not None else None
        self._check(self.lib.fcns_rhs_nonlinear(self.ctx, _ptr(v), _ptr(th), int(bool(filtered)),
                                                _ptr(nlv), _ptr(nlt)))
        self._keep = (v, th)
        return nlv, nlt

    def pressure_project(self, v_star, c):
        vs = self._dev(v_star, (3,) + self.shape)
        vo = self._empty(3, *self.shape)
        gp = self._empty(2, 2, self.ny, self.nx)
        self._check(self.lib.fcns_pressure_project(self.ctx, _ptr(vs), float(c), _ptr(vo),
                                                   _ptr(gp)))
        self._keep = (vs,)
        return vo, gp

    DIAG_NAMES = ("energy", "div2", "slip_bottom", "slip_top", "w2_bottom", "w2_top",
                  "dudz_bottom", "dudz_top", "re_tau_bottom", "re_tau_top", "nu_bottom",
                  "nu_top", "theta2")

    def diagnostics(self):
        out = np.zeros(len(self.DIAG_NAMES))
        self._check(self.lib.fcns_diagnostics(self.ctx, out.ctypes.data_as(ctypes.c_void_p),
                                              len(out)))
        return dict(zip(self.DIAG_NAMES, out.tolist()))

    def spectra(self, field, z):
        ex = np.zeros(self.nx // 2 + 1)
        ey = np.zeros(self.ny)
        self._check(self.lib.fcns_spectra(self.ctx, int(field), int(z),
                                          ex.ctypes.data_as(ctypes.c_void_p),
                                          ey.ctypes.data_as(ctypes.c_void_p)))
        return ex, ey

    def _cempty(self, *shape):
        with self.torch.cuda.stream(self.stream):
            return self.torch.empty(shape, dtype=self.torch.complex128, device=self.device)

    def get_spectral(self, field):
        out = self._cempty(self.npr, self.ny, self.nx // 2 + 1)
        self._check(self.lib.fcns_get_spectral(self.ctx, int(field), _ptr(out)))
        return out

    def get_wall_grad(self):
        out = self._cempty(2, 2, self.ny, self.nx // 2 + 1)
        self._check(self.lib.fcns_get_wall_grad(self.ctx, _ptr(out)))
        return out

    def set_spectral(self, fields, wall_grad=None):
        with self.torch.cuda.stream(self.stream):
            fs = [f.to(self.device).contiguous() for f in fields]
            wg = wall_grad.to(self.device).contiguous() if wall_grad is not None else None
        arr = (ctypes.c_void_p * len(fs))(*[f.data_ptr() for f in fs])
        self._check(self.lib.fcns_set_spectral(self.ctx, arr, _ptr(wg)))
        self._keep = (fs, wg)

    TIMING_CLASSES = ("y_back_dy", "y_back_dz", "x_nl", "y_fwd", "z_stageA", "z_stageB",
                      "z_back", "z_pass", "xy_slabs")

    def set_timing(self, enable=True, classes=None):
        """Event-time rk_step's kernels: every class, or only those named in
        `classes` (fewer events perturb the step less)."""
        if classes is None or not enable:
            self._check(self.lib.fcns_set_timing(self.ctx, int(bool(enable))))
            return
        mask = 0
        for nm in classes:
            mask |= 1 << self.TIMING_CLASSES.index(nm)
        self._check(self.lib.fcns_set_timing_mask(self.ctx, mask))

    def timing_reset(self):
        self._check(self.lib.fcns_timing_reset(self.ctx))

    def timing_report(self):
        """{kernel class: (launches, total ms)} since the last reset."""
        n = ctypes.c_int32()
        names = ctypes.create_string_buffer(32 * 16)
        counts = (ctypes.c_int64 * 16)()
        ms = (ctypes.c_double * 16)()
        self._check(self.lib.fcns_timing_report(self.ctx, 16, ctypes.byref(n), names, counts, ms))
        out = {}
        for i in range(n.value):
            nm = names.raw[32 * i:32 * (i + 1)].split(b"\0")[0].decode()
            out[nm] = (int(counts[i]), float(ms[i]))
        return out

    def synchronize(self):
        self.stream.synchronize()


def problem_bytes(nx, ny, nz, C, nfields, d=5):
    """Device memory a context of this shape allocates (bytes), from the
    library (no device needed)."""
    prob, _tab = make_problem(nx, ny, nz, 1.0, 1.0, 1.0, 0.0, d=d, C=C,
                              boussinesq=nfields == 4)
    return footprint(prob)

