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
PREC_FP64, PREC_FP32_PAIRS, PREC_RELAXED = 0, 1, 2

# Exported symbols, as declared in include/rmb.h.
EXPORTS = ["rmb_ctx_create", "rmb_ctx_destroy", "rmb_last_error", "rmb_version",
           "rmb_mobility_matvec", "rmb_precond_factor", "rmb_precond_apply", "rmb_precond_destroy",
           "rmb_solve_mobility", "rmb_solve_batch", "rmb_server_create", "rmb_server_submit",
           "rmb_server_step", "rmb_server_poll", "rmb_server_destroy", "rmb_ctx_set_timing",
           "rmb_ctx_kernel_time", "rmb_ctx_tuned_panel", "rmb_ctx_tune_log", "rmb_pair_plan",
           "rmb_flow_field", "rmb_precond_factor_shapes", "rmb_precond_set_orientations",
           "rmb_solve_resistance", "rmb_mobility_matvec_noalloc", "rmb_noalloc_workspace_bytes",
           "rmb_tile_shape_count", "rmb_tile_shape_info", "rmb_ctx_set_tile_shape",
           "rmb_mobility_matvec_f32"]
KERNELS = {"pair_f32_wall": 0, "pair_f32_free": 1, "pair_f64_wall": 2, "pair_f64_free": 3}


class RmbError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class rmb_system(ctypes.Structure):
    _fields_ = [("n_blobs", ctypes.c_int64), ("n_bodies", ctypes.c_int64),
                ("pos", ctypes.c_void_p), ("body_off", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("a", ctypes.c_double), ("eta", ctypes.c_double), ("geometry", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("blob_shift", ctypes.c_void_p)]


class rmb_shapes(ctypes.Structure):
    _fields_ = [("n_shapes", ctypes.c_int32), ("reserved", ctypes.c_int32), ("shape_off", ctypes.c_void_p),
                ("ref_pos", ctypes.c_void_p)]


class rmb_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("precision", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("pad", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("u_tol", ctypes.c_double)]


class rmb_tune_record(ctypes.Structure):
    _fields_ = [("padded_dim", ctypes.c_int32), ("panel", ctypes.c_int32), ("row_tiles", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("ms", ctypes.c_double), ("chosen", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class rmb_solve_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("matvecs_fp64", ctypes.c_int32), ("matvecs_fp32", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("tol_internal", ctypes.c_double), ("u_err_est", ctypes.c_double), ("gamma", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


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
        L.rmb_mobility_matvec_noalloc.argtypes = [vp, sysp, i32, vp, vp, i32, vp]
        L.rmb_mobility_matvec_f32.argtypes = [vp, sysp, vp, vp, vp]
        L.rmb_noalloc_workspace_bytes.argtypes = []
        L.rmb_noalloc_workspace_bytes.restype = ctypes.c_size_t
        L.rmb_flow_field.argtypes = [vp, sysp, i32, vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                     ctypes.c_int64, vp, vp, vp]
        optp, infop = ctypes.POINTER(rmb_solve_opts), ctypes.POINTER(rmb_solve_info)
        L.rmb_precond_factor.argtypes = [vp, sysp, ctypes.POINTER(vp), vp]
        L.rmb_precond_apply.argtypes = [vp, vp, i32, vp, vp, vp]
        L.rmb_precond_factor_shapes.argtypes = [vp, sysp, ctypes.POINTER(rmb_shapes), vp, vp, ctypes.POINTER(vp),
                                                vp]
        L.rmb_precond_set_orientations.argtypes = [vp, vp, vp, vp]
        L.rmb_precond_destroy.argtypes = [vp]
        L.rmb_precond_destroy.restype = None
        L.rmb_solve_mobility.argtypes = [vp, sysp, vp, vp, vp, vp, vp, optp, infop, vp]
        L.rmb_solve_resistance.argtypes = [vp, sysp, vp, vp, vp, vp, vp, optp, infop, vp]
        L.rmb_solve_batch.argtypes = [vp, i32, sysp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), ctypes.POINTER(vp), optp, infop, vp]
        L.rmb_server_create.argtypes = [vp, i32, vp, ctypes.POINTER(vp)]
        L.rmb_server_submit.argtypes = [vp, sysp, vp, vp, vp, vp, optp, i64]
        L.rmb_server_step.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.rmb_server_poll.argtypes = [vp, i32, ctypes.POINTER(i64), infop, ctypes.POINTER(i32)]
        L.rmb_server_destroy.argtypes = [vp]
        L.rmb_server_destroy.restype = None
        L.rmb_ctx_set_timing.argtypes = [vp, i32]
        L.rmb_ctx_kernel_time.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
        L.rmb_ctx_tuned_panel.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.rmb_tile_shape_count.argtypes = []
        L.rmb_tile_shape_count.restype = i32
        L.rmb_tile_shape_info.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.rmb_ctx_set_tile_shape.argtypes = [vp, i32, i32]
        L.rmb_ctx_tune_log.argtypes = [vp, i32, ctypes.POINTER(rmb_tune_record), ctypes.POINTER(i32)]
        L.rmb_pair_plan.argtypes = [i64, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        _LIB = L
    return _LIB


def tile_shapes() -> list:
    """Every tile shape of the large-body factorisation: dicts with panel,
    row_tiles and chunk, indexed by shape number."""
    L = library()
    out = []
    for k in range(L.rmb_tile_shape_count()):
        p, g, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        if L.rmb_tile_shape_info(k, ctypes.byref(p), ctypes.byref(g), ctypes.byref(c)) != RMB_OK:
            raise RmbError(RMB_EINVAL, f"rmb_tile_shape_info({k}) failed")
        out.append({"panel": p.value, "row_tiles": g.value, "chunk": c.value})
    return out


def pair_plan(nb: int):
    """(symmetric, block) of the mobility product of nb blobs (see rmb_pair_plan)."""
    sym, blk = ctypes.c_int32(), ctypes.c_int32()
    st = library().rmb_pair_plan(int(nb), ctypes.byref(sym), ctypes.byref(blk))
    if st != RMB_OK:
        raise RmbError(st, "rmb_pair_plan failed")
    return bool(sym.value), blk.value


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, name: str, shape=None, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {str(dtype).replace('torch.', '')}")
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
        self._children = []  # objects holding device memory of this context

    def _adopt(self, obj):
        import weakref
        self._children.append(weakref.ref(obj))

    def close(self):
        if getattr(self, "h", None):
            for ref in getattr(self, "_children", []):
                child = ref()
                if child is not None:
                    child.close()
            self.lib.rmb_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, enable: bool):
        """Bracket every pair-kernel launch with HIP events (resets totals)."""
        self.check(self.lib.rmb_ctx_set_timing(self.h, 1 if enable else 0))

    def kernel_time(self, kernel: str):
        """(total ms, launches) of a pair kernel since timing was enabled."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self.check(self.lib.rmb_ctx_kernel_time(self.h, KERNELS[kernel], ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def tuned_panel(self, padded_dim: int) -> int:
        """Panel width the autotuner chose for this padded block size (0: none yet)."""
        w = ctypes.c_int32()
        self.check(self.lib.rmb_ctx_tuned_panel(self.h, int(padded_dim), ctypes.byref(w)))
        return w.value

    def set_tile_shape(self, padded_dim: int, shape: int):
        """Force a tile shape of the large-body factorisation for one padded
        size on this context (-1: back to the autotuner)."""
        self.check(self.lib.rmb_ctx_set_tile_shape(self.h, int(padded_dim), int(shape)))

    def tune_log(self) -> list:
        """Every timing the large-body autotuner took on this context:
        dicts with padded_dim, panel, row_tiles, chunk, ms, chosen."""
        n = ctypes.c_int32()
        self.check(self.lib.rmb_ctx_tune_log(self.h, 0, None, ctypes.byref(n)))
        recs = (rmb_tune_record * max(n.value, 1))()
        self.check(self.lib.rmb_ctx_tune_log(self.h, n.value, recs, ctypes.byref(n)))
        return [{"padded_dim": r.padded_dim, "panel": r.panel, "row_tiles": r.row_tiles, "chunk": r.chunk,
                 "ms": r.ms, "chosen": bool(r.chosen)} for r in recs[:n.value]]

    def check(self, st):
        if st != RMB_OK:
            raise RmbError(st, self.lib.rmb_last_error(self.h).decode())
        return st


class System:
    """Holds the tensors of one suspension and its rmb_system struct."""

    def __init__(self, pos: torch.Tensor, a: float, eta: float = 1.0, wall: bool = False,
                 body_off=None, q: torch.Tensor = None, blob_shift: torch.Tensor = None):
        """blob_shift: optional (Nb,) device tensor of permeability shifts
        d_i = kappa_p / (eta dV_i) added to the diagonal of M."""
        self.pos = pos
        self.q = q
        self.blob_shift = blob_shift
        self.a, self.eta, self.wall = float(a), float(eta), bool(wall)
        self.body_off = None if body_off is None else np.ascontiguousarray(body_off, dtype=np.int64)
        n_b = 0 if self.body_off is None else len(self.body_off) - 1
        self.n_blobs = int(pos.shape[0])
        self.n_bodies = n_b
        self.c = rmb_system(self.n_blobs, n_b, _dev(pos, "pos", (self.n_blobs, 3)).value,
                            None if self.body_off is None else self.body_off.ctypes.data,
                            None if q is None else _dev(q, "q", (n_b, 3)).value,
                            self.a, self.eta, GEOM_WALL if self.wall else GEOM_FREE, 0,
                            None if blob_shift is None else _dev(blob_shift, "blob_shift", (self.n_blobs,)).value)

    @classmethod
    def from_suspension(cls, sus, device="cuda"):
        pos = torch.as_tensor(sus.pos, dtype=torch.float64, device=device).contiguous()
        q = torch.as_tensor(sus.q, dtype=torch.float64, device=device).contiguous()
        shift = getattr(sus, "blob_shift", None)
        if shift is not None:
            shift = torch.as_tensor(shift, dtype=torch.float64, device=device).contiguous()
        return cls(pos, sus.a, sus.eta, sus.wall, sus.body_off, q, shift)


def _prec(p):
    if p in ("fp64", PREC_FP64):
        return PREC_FP64
    if p in ("fp32", "fp32_pairs", PREC_FP32_PAIRS):
        return PREC_FP32_PAIRS
    if p in ("relaxed", PREC_RELAXED):
        return PREC_RELAXED
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


def mobility_matvec_f32(ctx: Context, system: System, lam: torch.Tensor, out: torch.Tensor = None,
                        stream=None) -> torch.Tensor:
    """v = M lambda for float32 forces (Nb, 3), FP32 pairs with FP64
    accumulation, velocities rounded to float32 (rmb_mobility_matvec_f32)."""
    n = system.n_blobs
    lp = _dev(lam, "lambda", (n, 3), torch.float32)
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=lam.device)
    op = _dev(out, "out", (n, 3), torch.float32)
    ctx.check(ctx.lib.rmb_mobility_matvec_f32(ctx.h, ctypes.byref(system.c), lp, op, _stream(stream)))
    return out


def mobility_matvec_noalloc(ctx: Context, system: System, lam: torch.Tensor, out: torch.Tensor,
                            precision="fp64", validate: bool = True, stream=None) -> torch.Tensor:
    """v = M lambda through the entry point that allocates nothing
    (rmb_mobility_matvec_noalloc): the output tensor is the caller's, the
    workspace a static device array shared by every call on the device."""
    n = system.n_blobs
    lp = _dev(lam, "lambda", (n, 3))
    op = _dev(out, "out", (n, 3))
    ctx.check(ctx.lib.rmb_mobility_matvec_noalloc(ctx.h, ctypes.byref(system.c), _prec(precision), lp, op,
                                                  1 if validate else 0, _stream(stream)))
    return out


def noalloc_workspace_bytes() -> int:
    return int(library().rmb_noalloc_workspace_bytes())


def flow_field(ctx: Context, system: System, lam: torch.Tensor, sub_offsets, tracer_a: float,
               targets: torch.Tensor, precision="fp64", out: torch.Tensor = None, stream=None) -> torch.Tensor:
    """Fluid velocity at `targets` (n, 3) from blob forces `lam` (Nb, 3): each
    blob replaced by len(sub_offsets) blobs of radius tracer_a at
    r_i + a * sub_offsets[k] carrying lam_i / n_sub (rmb_flow_field)."""
    import numpy as np
    n = system.n_blobs
    lp = _dev(lam, "lambda", (n, 3))
    offs = np.ascontiguousarray(np.asarray(sub_offsets, dtype=np.float64).reshape(-1, 3))
    nt = int(targets.shape[0])
    tp = _dev(targets, "targets", (nt, 3))
    if out is None:
        out = torch.empty((nt, 3), dtype=torch.float64, device=targets.device)
    op = _dev(out, "out", (nt, 3))
    ctx.check(ctx.lib.rmb_flow_field(ctx.h, ctypes.byref(system.c), _prec(precision), lp, int(offs.shape[0]),
                                     offs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(tracer_a), nt,
                                     tp, op, _stream(stream)))
    return out


def solve_opts(tol=1e-8, precision="fp64", restart=100, max_iters=1000, inner_tol=1e-5, u_tol=0.0):
    """u_tol > 0 bounds the forward error of the body velocities as well
    (see rmb_solve_opts in include/rmb.h)."""
    return rmb_solve_opts(float(tol), _prec(precision), int(restart), int(max_iters), 0, float(inner_tol),
                          float(u_tol))


def _vec(t, name, n):
    if t is None:
        return None
    return _dev(t, name, (n, 3) if name in ("slip", "lambda") else (n, 6))


class Precond:
    """Block-diagonal preconditioner factors of one system (rmb_precond)."""

    def __init__(self, ctx: Context, system: System, stream=None, _handle=None):
        self.ctx, self.system = ctx, system
        h = ctypes.c_void_p()
        if _handle is None:
            ctx.check(ctx.lib.rmb_precond_factor(ctx.h, ctypes.byref(system.c), ctypes.byref(h),
                                                 _stream(stream)))
        else:
            h = _handle
        self.h = h
        ctx._adopt(self)

    @classmethod
    def from_shapes(cls, ctx: Context, system: System, shapes, body_shape, quat: torch.Tensor, stream=None):
        """One factorisation per reference shape (rmb_precond_factor_shapes):
        shapes is a list of (n_k, 3) body-frame blob positions relative to the
        tracking point, body_shape the shape index of every body, quat the
        (N, 4) device orientations (w, x, y, z)."""
        import numpy as np
        refs = [np.asarray(r, dtype=np.float64).reshape(-1, 3) for r in shapes]
        off = np.ascontiguousarray(np.concatenate([[0], np.cumsum([len(r) for r in refs])]).astype(np.int64))
        ref = np.ascontiguousarray(np.concatenate(refs, axis=0))
        bs = np.ascontiguousarray(np.asarray(body_shape, dtype=np.int32).reshape(-1))
        if bs.shape[0] != system.n_bodies:
            raise ValueError(f"body_shape has {bs.shape[0]} entries for {system.n_bodies} bodies")
        qp = _dev(quat, "quat", (system.n_bodies, 4))
        sh = rmb_shapes(len(refs), 0, off.ctypes.data, ref.ctypes.data)
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.rmb_precond_factor_shapes(ctx.h, ctypes.byref(system.c), ctypes.byref(sh),
                                                    bs.ctypes.data, qp, ctypes.byref(h), _stream(stream)))
        return cls(ctx, system, _handle=h)

    def set_orientations(self, quat: torch.Tensor, stream=None):
        """New (N, 4) device orientations for a shared-shape preconditioner."""
        qp = _dev(quat, "quat", (self.system.n_bodies, 4))
        self.ctx.check(self.ctx.lib.rmb_precond_set_orientations(self.ctx.h, self.h, qp, _stream(stream)))

    def apply(self, rhs: torch.Tensor, out: torch.Tensor = None, stream=None) -> torch.Tensor:
        """P^-1 applied to each row of rhs (nrhs, 3 Nb + 6 N)."""
        n = 3 * self.system.n_blobs + 6 * self.system.n_bodies
        if rhs.dim() == 1:
            rhs = rhs.reshape(1, -1)
        _dev(rhs, "rhs", (rhs.shape[0], n))
        if out is None:
            out = torch.empty_like(rhs)
        _dev(out, "out", tuple(rhs.shape))
        self.ctx.check(self.ctx.lib.rmb_precond_apply(self.ctx.h, self.h, rhs.shape[0],
                                                      ctypes.c_void_p(rhs.data_ptr()),
                                                      ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self.ctx.lib.rmb_precond_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_mobility(ctx: Context, system: System, FT: torch.Tensor, slip: torch.Tensor = None,
                   precond: Precond = None, stream=None, raise_on_noconv=False, **opts):
    """Mobility problem (eq:saddle_M) by preconditioned GMRES.  Returns
    (U (N, 6), lambda (Nb, 3), info dict)."""
    nb, N = system.n_blobs, system.n_bodies
    FTp = _dev(FT, "FT", (N, 6))
    sp = _vec(slip, "slip", nb)
    U = torch.empty((N, 6), dtype=torch.float64, device=FT.device)
    lam = torch.empty((nb, 3), dtype=torch.float64, device=FT.device)
    o = solve_opts(**opts)
    info = rmb_solve_info()
    st = ctx.lib.rmb_solve_mobility(ctx.h, ctypes.byref(system.c), precond.h if precond else None, FTp, sp,
                                    ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                    ctypes.byref(o), ctypes.byref(info), _stream(stream))
    if st != RMB_OK and (st != RMB_ENOCONV or raise_on_noconv):
        ctx.check(st)
    return U, lam, info.as_dict()


def solve_resistance(ctx: Context, system: System, U: torch.Tensor, slip: torch.Tensor = None,
                     precond: Precond = None, stream=None, raise_on_noconv=False, **opts):
    """Resistance problem (eq:resistance_problem): M lambda = K U + slip,
    F = K^T lambda.  Returns (F (N, 6), lambda (Nb, 3), info dict)."""
    nb, N = system.n_blobs, system.n_bodies
    Up = _dev(U, "U", (N, 6))
    sp = _vec(slip, "slip", nb)
    F = torch.empty((N, 6), dtype=torch.float64, device=U.device)
    lam = torch.empty((nb, 3), dtype=torch.float64, device=U.device)
    o = solve_opts(**opts)
    info = rmb_solve_info()
    st = ctx.lib.rmb_solve_resistance(ctx.h, ctypes.byref(system.c), precond.h if precond else None, Up, sp,
                                      ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                      ctypes.byref(o), ctypes.byref(info), _stream(stream))
    if st != RMB_OK and (st != RMB_ENOCONV or raise_on_noconv):
        ctx.check(st)
    return F, lam, info.as_dict()


def solve_batch(ctx: Context, systems, FTs, slips=None, stream=None, **opts):
    """Independent mobility problems solved together.  Returns a list of
    (U, lambda, info) in input order; failed solves carry their status in
    info['status']."""
    k = len(systems)
    arr = (rmb_system * k)(*[s.c for s in systems])
    Us = [torch.empty((s.n_bodies, 6), dtype=torch.float64, device=FTs[i].device) for i, s in enumerate(systems)]
    Ls = [torch.empty((s.n_blobs, 3), dtype=torch.float64, device=FTs[i].device) for i, s in enumerate(systems)]
    vp = ctypes.c_void_p
    FTa = (vp * k)(*[_dev(FTs[i], "FT", (s.n_bodies, 6)).value for i, s in enumerate(systems)])
    Sa = None
    if slips is not None:
        Sa = (vp * k)(*[None if slips[i] is None else _dev(slips[i], "slip", (s.n_blobs, 3)).value
                        for i, s in enumerate(systems)])
    Ua = (vp * k)(*[u.data_ptr() for u in Us])
    La = (vp * k)(*[l.data_ptr() for l in Ls])
    infos = (rmb_solve_info * k)()
    o = solve_opts(**opts)
    st = ctx.lib.rmb_solve_batch(ctx.h, k, arr, FTa, Sa, Ua, La, ctypes.byref(o), infos, _stream(stream))
    if st not in (RMB_OK, RMB_ENOCONV, RMB_ENOTSPD, RMB_EINVAL):
        ctx.check(st)
    return [(Us[i], Ls[i], infos[i].as_dict()) for i in range(k)]


class Server:
    """Continuous-batching request loop (rmb_server).  Keeps each request's
    tensors alive until it is polled."""

    def __init__(self, ctx: Context, max_active: int = 0, stream=None):
        self.ctx = ctx
        self.stream = stream
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.rmb_server_create(ctx.h, max_active, _stream(stream), ctypes.byref(h)))
        self.h = h
        self.live = {}
        ctx._adopt(self)

    def submit(self, tag: int, system: System, FT: torch.Tensor, slip: torch.Tensor = None, **opts):
        """Queues one request.  Tags must be unique among requests not yet
        polled: the output tensors of a request are kept alive under its tag
        until poll() returns it."""
        if int(tag) in self.live:
            raise ValueError(f"tag {int(tag)} is already in flight")
        nb, N = system.n_blobs, system.n_bodies
        U = torch.empty((N, 6), dtype=torch.float64, device=FT.device)
        lam = torch.empty((nb, 3), dtype=torch.float64, device=FT.device)
        o = solve_opts(**opts)
        self.ctx.check(self.ctx.lib.rmb_server_submit(self.h, ctypes.byref(system.c), _dev(FT, "FT", (N, 6)),
                                                      _vec(slip, "slip", nb), ctypes.c_void_p(U.data_ptr()),
                                                      ctypes.c_void_p(lam.data_ptr()), ctypes.byref(o), int(tag)))
        self.live[int(tag)] = (system, FT, slip, U, lam)

    def step(self):
        a, q = ctypes.c_int32(), ctypes.c_int32()
        self.ctx.check(self.ctx.lib.rmb_server_step(self.h, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def poll(self, max_out: int = 1024):
        tags = (ctypes.c_int64 * max_out)()
        infos = (rmb_solve_info * max_out)()
        n = ctypes.c_int32()
        self.ctx.check(self.ctx.lib.rmb_server_poll(self.h, max_out, tags, infos, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            t = int(tags[i])
            system, FT, slip, U, lam = self.live.pop(t)
            out.append((t, U, lam, infos[i].as_dict()))
        return out

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self.ctx.lib.rmb_server_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
