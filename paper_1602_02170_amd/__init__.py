"""Python binding of librmb, the MI355X rigid-multiblob mobility library.

Argument marshalling only: every step of the computation runs in the HIP
kernels of librmb.so.  PyTorch provides device memory and streams.  The
binding fails loudly when the library has not been built; there is no CPU
fallback.

Layouts follow include/rmb.h: blob arrays (Nb, 3), body arrays (N, 3) or
(N, 6), all float64 CUDA (HIP) tensors on the context's device; body offsets
are a host int64 array of length N + 1.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librmb.so")

RMB_OK, RMB_EINVAL, RMB_ENOTSPD, RMB_ENOCONV, RMB_ENOMEM, RMB_EDEVICE, RMB_EBUSY = range(7)
STATUS_NAMES = {0: "RMB_OK", 1: "RMB_EINVAL", 2: "RMB_ENOTSPD", 3: "RMB_ENOCONV", 4: "RMB_ENOMEM",
                5: "RMB_EDEVICE", 6: "RMB_EBUSY"}
GEOM_FREE, GEOM_WALL = 0, 1
PREC_FP64, PREC_FP32_PAIRS = 0, 1

# Exported symbols, as declared in include/rmb.h.
EXPORTS = ["rmb_ctx_create", "rmb_ctx_destroy", "rmb_last_error", "rmb_version",
           "rmb_mobility_matvec"]


class RmbError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class rmb_system(ctypes.Structure):
    _fields_ = [("n_blobs", ctypes.c_int64), ("n_bodies", ctypes.c_int64),
                ("pos", ctypes.c_void_p), ("body_off", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("a", ctypes.c_double), ("eta", ctypes.c_double), ("geometry", ctypes.c_int32)]


_LIB = None


def library(path: str = LIB_PATH):
    """Loads librmb.so (after torch, so that both share one HIP runtime)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(path):
            raise RuntimeError(f"librmb.so is not built ({path}); run __graft_entry__.build()")
        L = ctypes.CDLL(path)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sysp = ctypes.POINTER(rmb_system)
        L.rmb_ctx_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.rmb_ctx_destroy.argtypes = [vp]
        L.rmb_ctx_destroy.restype = None
        L.rmb_last_error.argtypes = [vp]
        L.rmb_last_error.restype = ctypes.c_char_p
        L.rmb_version.restype = ctypes.c_char_p
        L.rmb_mobility_matvec.argtypes = [vp, sysp, i32, vp, vp, vp]
        _LIB = L
    return _LIB


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, name: str, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """An rmb context on one device (device memory budget in bytes, 0 = 16 GiB)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self.lib = library()
        self.device = device
        h = ctypes.c_void_p()
        st = self.lib.rmb_ctx_create(device, hbm_budget, ctypes.byref(h))
        if st != RMB_OK:
            raise RmbError(st, "rmb_ctx_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.rmb_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st):
        if st != RMB_OK:
            raise RmbError(st, self.lib.rmb_last_error(self.h).decode())
        return st


class System:
    """Holds the tensors of one suspension and its rmb_system struct."""

    def __init__(self, pos: torch.Tensor, a: float, eta: float = 1.0, wall: bool = False,
                 body_off=None, q: torch.Tensor = None):
        self.pos = pos
        self.q = q
        self.a, self.eta, self.wall = float(a), float(eta), bool(wall)
        self.body_off = None if body_off is None else np.ascontiguousarray(body_off, dtype=np.int64)
        n_b = 0 if self.body_off is None else len(self.body_off) - 1
        self.n_blobs = int(pos.shape[0])
        self.n_bodies = n_b
        self.c = rmb_system(self.n_blobs, n_b, _dev(pos, "pos", (self.n_blobs, 3)).value,
                            None if self.body_off is None else self.body_off.ctypes.data,
                            None if q is None else _dev(q, "q", (n_b, 3)).value,
                            self.a, self.eta, GEOM_WALL if self.wall else GEOM_FREE)

    @classmethod
    def from_suspension(cls, sus, device="cuda"):
        pos = torch.as_tensor(sus.pos, dtype=torch.float64, device=device).contiguous()
        q = torch.as_tensor(sus.q, dtype=torch.float64, device=device).contiguous()
        return cls(pos, sus.a, sus.eta, sus.wall, sus.body_off, q)


def _prec(p):
    if p in ("fp64", PREC_FP64):
        return PREC_FP64
    if p in ("fp32", "fp32_pairs", PREC_FP32_PAIRS):
        return PREC_FP32_PAIRS
    raise ValueError(f"unknown precision {p!r}")


def mobility_matvec(ctx: Context, system: System, lam: torch.Tensor, precision="fp64",
                    out: torch.Tensor = None, stream=None) -> torch.Tensor:
    """v = M lambda (free-space or wall-corrected RPY), (Nb, 3) float64."""
    n = system.n_blobs
    lp = _dev(lam, "lambda", (n, 3))
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device=lam.device)
    op = _dev(out, "out", (n, 3))
    ctx.check(ctx.lib.rmb_mobility_matvec(ctx.h, ctypes.byref(system.c), _prec(precision), lp, op,
                                          _stream(stream)))
    return out
