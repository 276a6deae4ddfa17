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
    "fcns_rhs_nonlinear": (ctypes.c_int, [_P, _P, _P, _I32, _P, _P]),
    "fcns_pressure_project": (ctypes.c_int, [_P, _P, _D, _P, _P]),
    "fcns_set_state": (ctypes.c_int, [_P, _P, _P]),
    "fcns_rk_step": (ctypes.c_int, [_P, _D, _I32]),
    "fcns_get_state": (ctypes.c_int, [_P, _P, _P, _P]),
    "fcns_get_spectral": (ctypes.c_int, [_P, _I32, _P]),
    "fcns_set_spectral": (ctypes.c_int, [_P, ctypes.POINTER(_P), _P]),
    "fcns_get_wall_grad": (ctypes.c_int, [_P, _P]),
    "fcns_npr": (ctypes.c_int32, [_P]),
    "fcns_set_timing": (ctypes.c_int, [_P, _I32]),
    "fcns_timing_reset": (ctypes.c_int, [_P]),
    "fcns_timing_report": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_I32), _P, _P, _P]),
    "fcns_last_error": (ctypes.c_char_p, [_P]),
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
        from . import fctable

        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the solver runs only on the GPU")
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        tab = np.ascontiguousarray(table if table is not None else fctable.load(d, C),
                                   dtype=np.float64)
        self._table = tab
        prob = FcnsProblem(nx, ny, nz, lx, ly, lz, d, C,
                           tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           nu, forcing_x, int(bool(boussinesq)), kappa, gamma, int(rk_order),
                           filter_beta, filter_2p, _PRECISIONS[precision],
                           int(bool(keep_pressure)))
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

    def _dev(self, a, shape=None):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        a = a.to(device=self.device, dtype=t.float64).contiguous()
        if shape is not None and tuple(a.shape) != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {tuple(a.shape)}")
        return a

    def _empty(self, *shape):
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

    def get_spectral(self, field):
        out = self.torch.empty((self.npr, self.ny, self.nx // 2 + 1), dtype=self.torch.complex128,
                               device=self.device)
        self._check(self.lib.fcns_get_spectral(self.ctx, int(field), _ptr(out)))
        return out

    def get_wall_grad(self):
        out = self.torch.empty((2, 2, self.ny, self.nx // 2 + 1), dtype=self.torch.complex128,
                               device=self.device)
        self._check(self.lib.fcns_get_wall_grad(self.ctx, _ptr(out)))
        return out

    def set_spectral(self, fields, wall_grad=None):
        fs = [f.to(self.device).contiguous() for f in fields]
        arr = (ctypes.c_void_p * len(fs))(*[f.data_ptr() for f in fs])
        wg = wall_grad.to(self.device).contiguous() if wall_grad is not None else None
        self._check(self.lib.fcns_set_spectral(self.ctx, arr, _ptr(wg)))
        self._keep = (fs, wg)

    def set_timing(self, enable=True):
        self._check(self.lib.fcns_set_timing(self.ctx, int(bool(enable))))

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


def problem_bytes(nx, ny, nz, C, nfields):
    """Device memory the context allocates (bytes)."""
    nkx = nx // 2 + 1
    S = (nz + C) * ny * nkx * 16
    M = nz * ny * nkx * 16
    return 3 * nfields * S + (2 + 2 + 3 + 1) * nfields * M + M + 8 * ny * nkx * 16

