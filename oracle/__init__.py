"""CPU FP64 oracle of the rigid-multiblob mobility solve (test infrastructure).

Test infrastructure only: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the GPU library never does, and the two
share no code.  Everything here is plain FP64, written from the paper's
definitions, with library primitives (numpy/scipy dense solves) as steps.

  pair blocks, dense M, mobility product M lambda
        -> librmb_oracle.so (rmb_oracle.c): free-space RPY (eq:RPYTensor) and
           the wall-corrected RPY (Sec. 2.1.1, Sec. 5)
  K U, K^T lambda            -> rigid no-slip kinematics (eq:noslip_rigid,
                                eq:rigidSystem)
  saddle operator A [lambda; U] = [M lambda - K U; -K^T lambda] (eq:saddle_M);
  permeable bodies (eq:permeable_slip) put d_i on the diagonal of M in the
  operator, the dense solve and the per-body blocks
  dense_solve                -> U = N (F - K^T M^-1 slip), N = (K^T M^-1 K)^-1,
                                lambda = M^-1 (K U + slip)  (Schur complement
                                below eq:saddle_M, eq:BodyMob)
  BlockPreconditioner        -> indefinite block-diagonal preconditioner
                                (eq:M_tilde_block_diag, eq:indef_block_P,
                                eq:saddle_M_precon)
  ShapePreconditioner        -> the same with one free-space block per
                                reference shape, rotated per body (Sec. 2.2.2
                                after eq:saddle_M_precon; Sec. 5.4)
  resistance_dense,          -> resistance problem M lambda = K U + slip,
  solve_resistance              F = K^T lambda (eq:resistance_problem), dense
                                and by GMRES with the blocks M_pp^-1
  gmres                      -> right-preconditioned GMRES (Sec. 2.2.2; right
                                preconditioning so the monitored residual is
                                the true one, Sec. 3.3)
  velocity_at, flow_field    -> rectangular product at arbitrary points and
                                the flow field of the appendix on computing
                                flow fields (blobs split into tracer-size
                                blobs carrying equal shares of the force)

Vector layout of a saddle-point vector: [lambda (Nb x 3, blob-major);
U (N x 6: u then omega)], flattened.
"""
from __future__ import annotations

import ctypes
import os
import time

import numpy as np
import scipy.linalg as sla

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "librmb_oracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_pair_block.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.oracle_wall_block.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp]
        L.oracle_matvec.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, dp]
        L.oracle_matvec_rows.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_int64, ctypes.c_int64, dp,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.oracle_assemble.argtypes = [ctypes.c_int64, dp, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, dp]
        L.oracle_num_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _p(x):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


# ----------------------------------------------------------------------------
# blob mobility
# ----------------------------------------------------------------------------

def pair_block(ri, rj, a, eta=1.0, wall=False) -> np.ndarray:
    """3x3 block M_ij: velocity of blob i (rows) per force on blob j (cols)."""
    ri, rj = _c(ri), _c(rj)
    out = np.empty(9)
    lib().oracle_pair_block(_p(ri), _p(rj), a, eta, int(bool(wall)), _p(out))
    return out.reshape(3, 3)


def wall_block(ri, rj, a, eta=1.0) -> np.ndarray:
    """The wall correction part of M_ij alone."""
    ri, rj = _c(ri), _c(rj)
    out = np.empty(9)
    lib().oracle_wall_block(_p(ri), _p(rj), a, eta, _p(out))
    return out.reshape(3, 3)


def matvec(pos, lam, a, eta=1.0, wall=False) -> np.ndarray:
    """v = M lambda over all blobs (Nb x 3 in, Nb x 3 out)."""
    pos, lam = _c(pos), _c(lam)
    v = np.empty_like(pos)
    lib().oracle_matvec(pos.shape[0], _p(pos), _p(lam), a, eta, int(bool(wall)), _p(v))
    return v


def matvec_rows(pos, lam, rows, a, eta=1.0, wall=False) -> np.ndarray:
    """(M lambda)_i for the target blobs i in `rows` only (1-D index array)."""
    pos, lam = _c(pos), _c(lam)
    rows = np.asarray(rows, dtype=np.int64)
    tgt = _c(pos[rows])
    v = np.empty_like(tgt)
    lib().oracle_matvec_rows(pos.shape[0], _p(pos), _p(lam), 0, len(rows), _p(tgt), a, eta,
                             int(bool(wall)), _p(v))
    return v


def velocity_at(src_pos, src_lam, targets, a, eta=1.0, wall=False) -> np.ndarray:
    """sum_j M(t, r_j) lambda_j at arbitrary target points t (rectangular
    product; every point is a blob of radius a)."""
    src_pos, src_lam, targets = _c(src_pos), _c(src_lam), _c(targets)
    v = np.empty_like(targets)
    lib().oracle_matvec_rows(src_pos.shape[0], _p(src_pos), _p(src_lam), 0, targets.shape[0], _p(targets), a,
                             eta, int(bool(wall)), _p(v))
    return v


def flow_field(pos, lam, a, sub_offsets, tracer_a, targets, eta=1.0, wall=False) -> np.ndarray:
    """Flow field of the appendix on computing flow fields: blob i is
    replaced by n_sub blobs of radius tracer_a at r_i + a * u_k, each carrying
    lambda_i / n_sub; the velocity at t is the blob-blob mobility of radius
    tracer_a summed over all of them."""
    pos, lam = np.asarray(pos, dtype=np.float64), np.asarray(lam, dtype=np.float64)
    u = np.asarray(sub_offsets, dtype=np.float64).reshape(-1, 3)
    sub_pos = (pos[:, None, :] + a * u[None, :, :]).reshape(-1, 3)
    sub_lam = np.repeat(lam / len(u), len(u), axis=0)
    return velocity_at(sub_pos, sub_lam, targets, tracer_a, eta, wall)


def assemble(pos, a, eta=1.0, wall=False) -> np.ndarray:
    """Dense (3 Nb x 3 Nb) mobility matrix."""
    pos = _c(pos)
    n = pos.shape[0]
    M = np.empty((3 * n, 3 * n))
    lib().oracle_assemble(n, _p(pos), a, eta, int(bool(wall)), _p(M))
    return M


# ----------------------------------------------------------------------------
# rigid kinematics
# ----------------------------------------------------------------------------

def K_apply(pos, off, q, U) -> np.ndarray:
    """Blob velocities u_p + omega_p x (r_i - q_p) of rigid motions U (N x 6)."""
    U = np.asarray(U, dtype=np.float64).reshape(-1, 6)
    out = np.empty((pos.shape[0], 3))
    for p in range(len(off) - 1):
        s, e = off[p], off[p + 1]
        out[s:e] = U[p, 0:3] + np.cross(U[p, 3:6], pos[s:e] - q[p])
    return out


def KT_apply(pos, off, q, lam) -> np.ndarray:
    """Per-body force sum and torque about q_p of blob forces (-> N x 6)."""
    lam = np.asarray(lam, dtype=np.float64).reshape(-1, 3)
    out = np.empty((len(off) - 1, 6))
    for p in range(len(off) - 1):
        s, e = off[p], off[p + 1]
        out[p, 0:3] = lam[s:e].sum(axis=0)
        out[p, 3:6] = np.cross(pos[s:e] - q[p], lam[s:e]).sum(axis=0)
    return out


def K_dense(pos, off, q) -> np.ndarray:
    """Dense K (3 Nb x 6 N), built column by column from K_apply."""
    n_b = len(off) - 1
    K = np.zeros((3 * pos.shape[0], 6 * n_b))
    for p in range(n_b):
        for c in range(6):
            U = np.zeros((n_b, 6))
            U[p, c] = 1.0
            K[:, 6 * p + c] = K_apply(pos, off, q, U).ravel()
    return K


# ----------------------------------------------------------------------------
# saddle-point system (eq:saddle_M)
# ----------------------------------------------------------------------------

def _shift3(sus):
    """Permeable bodies (eq:permeable_slip): the slip -d_i lambda_i, i.e.
    d_i added to the three diagonal entries of blob i in M; None if the
    bodies are impermeable."""
    d = getattr(sus, "blob_shift", None)
    return None if d is None else np.repeat(np.asarray(d, dtype=np.float64), 3)


def split(sus, x):
    nb3 = 3 * sus.n_blobs
    return x[:nb3].reshape(-1, 3), x[nb3:].reshape(-1, 6)


def rhs(sus, FT, slip=None) -> np.ndarray:
    """b = [slip; -F]."""
    top = np.zeros((sus.n_blobs, 3)) if slip is None else np.asarray(slip, dtype=np.float64)
    return np.concatenate([top.ravel(), -np.asarray(FT, dtype=np.float64).ravel()])


def saddle_apply(sus, x) -> np.ndarray:
    """A [lambda; U] = [M lambda - K U; -K^T lambda]."""
    lam, U = split(sus, x)
    top = matvec(sus.pos, lam, sus.a, sus.eta, sus.wall) - K_apply(sus.pos, sus.body_off, sus.q, U)
    d3 = _shift3(sus)
    if d3 is not None:
        top = top + (d3 * lam.ravel()).reshape(-1, 3)
    bot = -KT_apply(sus.pos, sus.body_off, sus.q, lam)
    return np.concatenate([top.ravel(), bot.ravel()])


def relative_residual(sus, FT, slip, U, lam) -> float:
    """||b - A x|| / ||b|| with the FP64 oracle operator."""
    b = rhs(sus, FT, slip)
    x = np.concatenate([np.asarray(lam, dtype=np.float64).ravel(),
                        np.asarray(U, dtype=np.float64).ravel()])
    r = b - saddle_apply(sus, x)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def dense_solve(sus, FT, slip=None):
    """Exact solution of eq:saddle_M through the Schur complement:
    U = N (F - K^T M^-1 slip), N = (K^T M^-1 K)^-1, lambda = M^-1 (K U + slip).
    Returns (U (N x 6), lambda (Nb x 3))."""
    M = assemble(sus.pos, sus.a, sus.eta, sus.wall)
    d3 = _shift3(sus)
    if d3 is not None:
        M[np.diag_indices_from(M)] += d3
    K = K_dense(sus.pos, sus.body_off, sus.q)
    cf = sla.cho_factor(M, lower=True)
    MinvK = sla.cho_solve(cf, K)
    s = np.zeros(3 * sus.n_blobs) if slip is None else np.asarray(slip, dtype=np.float64).ravel()
    Minvs = sla.cho_solve(cf, s)
    S = K.T @ MinvK
    U = np.linalg.solve(S, np.asarray(FT, dtype=np.float64).ravel() - K.T @ Minvs)
    lam = Minvs + MinvK @ U
    return U.reshape(-1, 6), lam.reshape(-1, 3)


def resistance_dense(sus, U, slip=None):
    """Resistance problem (eq:resistance_problem) by a dense Cholesky solve:
    lambda = M^-1 (K U + slip), F = K^T lambda.  Returns (F (N x 6),
    lambda (Nb x 3))."""
    M = assemble(sus.pos, sus.a, sus.eta, sus.wall)
    d3 = _shift3(sus)
    if d3 is not None:
        M[np.diag_indices_from(M)] += d3
    rhs_ = K_apply(sus.pos, sus.body_off, sus.q, U).ravel()
    if slip is not None:
        rhs_ = rhs_ + np.asarray(slip, dtype=np.float64).ravel()
    lam = sla.cho_solve(sla.cho_factor(M, lower=True), rhs_).reshape(-1, 3)
    return KT_apply(sus.pos, sus.body_off, sus.q, lam), lam


def body_mobility(sus) -> np.ndarray:
    """Dense body mobility N = (K^T M^-1 K)^-1 (6N x 6N), eq:BodyMob."""
    M = assemble(sus.pos, sus.a, sus.eta, sus.wall)
    d3 = _shift3(sus)
    if d3 is not None:
        M[np.diag_indices_from(M)] += d3
    K = K_dense(sus.pos, sus.body_off, sus.q)
    MinvK = sla.cho_solve(sla.cho_factor(M, lower=True), K)
    return np.linalg.inv(K.T @ MinvK)


# ----------------------------------------------------------------------------
# block-diagonal preconditioner (eq:indef_block_P, eq:saddle_M_precon)
# ----------------------------------------------------------------------------

class BlockPreconditioner:
    """P^-1 of the indefinite block-diagonal preconditioner: per body p solve
    [M_pp -K_p; -K_p^T 0][lambda_p; U_p] = [s_p; -F_p] by
    U_p = (K_p^T M_pp^-1 K_p)^-1 (F_p - K_p^T M_pp^-1 s_p),
    lambda_p = M_pp^-1 (s_p + K_p U_p)."""

    def __init__(self, sus):
        self.sus = sus
        self.blocks = []
        off = sus.body_off
        d3 = _shift3(sus)
        for p in range(sus.n_bodies):
            s, e = off[p], off[p + 1]
            pos = sus.pos[s:e]
            Mpp = assemble(pos, sus.a, sus.eta, sus.wall)
            if d3 is not None:
                Mpp[np.diag_indices_from(Mpp)] += d3[3 * s:3 * e]
            Kp = K_dense(pos, np.array([0, e - s]), sus.q[p:p + 1])
            cf = sla.cho_factor(Mpp, lower=True)
            MinvK = sla.cho_solve(cf, Kp)
            Np = np.linalg.inv(Kp.T @ MinvK)
            self.blocks.append((s, e, cf, Kp, MinvK, Np))

    def apply(self, v) -> np.ndarray:
        sus = self.sus
        sv, Fv = split(sus, np.asarray(v, dtype=np.float64))
        lam = np.empty_like(sv)
        U = np.empty_like(Fv)
        for p, (s, e, cf, Kp, MinvK, Np) in enumerate(self.blocks):
            sp_ = sv[s:e].ravel()
            Minvs = sla.cho_solve(cf, sp_)
            # the bottom block row reads -K^T lambda = (given) bottom entry,
            # so the body force is minus the bottom part of v
            Fp = -Fv[p]
            Up = Np @ (Fp - Kp.T @ Minvs)
            lam[s:e] = (Minvs + MinvK @ Up).reshape(-1, 3)
            U[p] = Up
        return np.concatenate([lam.ravel(), U.ravel()])

    def apply_resistance(self, v) -> np.ndarray:
        """M_pp^-1 s per body (preconditioner of the resistance problem)."""
        sv = np.asarray(v, dtype=np.float64).reshape(-1, 3)
        out = np.empty_like(sv)
        for (s, e, cf, Kp, MinvK, Np) in self.blocks:
            out[s:e] = sla.cho_solve(cf, sv[s:e].ravel()).reshape(-1, 3)
        return out.ravel()


class ShapePreconditioner:
    """Block-diagonal preconditioner from one block per reference shape
    (Sec. 2.2.2, after eq:saddle_M_precon: the free-space RPY block of a body
    is its reference configuration's, rotated; Sec. 5.4: the same blocks used
    for a wall problem give the approximate preconditioner that neglects the
    boundary; permeability shifts are left out as well).  Shape k's saddle
    block [M_ref -K_ref; -K_ref^T 0] is formed in free space from its
    body-frame blob positions (tracking point at the origin).  For body p with rotation R_p (from its quaternion), the blob
    velocities, force and torque of the input are rotated into the body
    frame (R_p^T), the shape's block is solved, and lambda, u and omega are
    rotated back (R_p)."""

    def __init__(self, sus, shapes, body_shape, quats):
        from scipy.spatial.transform import Rotation
        self.sus = sus
        self.body_shape = np.asarray(body_shape, dtype=np.int64)
        q = np.asarray(quats, dtype=np.float64).reshape(-1, 4)
        # scipy orders quaternions (x, y, z, w) and normalises them
        self.R = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
        self.blocks = []
        for ref in shapes:
            ref = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
            M = assemble(ref, sus.a, sus.eta, False)
            K = K_dense(ref, np.array([0, len(ref)]), np.zeros((1, 3)))
            self.blocks.append(np.block([[M, -K], [-K.T, np.zeros((6, 6))]]))

    def apply(self, v) -> np.ndarray:
        sus = self.sus
        sv, Fv = split(sus, np.asarray(v, dtype=np.float64))
        lam = np.empty_like(sv)
        U = np.empty_like(Fv)
        off = sus.body_off
        for p in range(sus.n_bodies):
            s, e = off[p], off[p + 1]
            R = self.R[p]
            # row vectors: (R^T x)^T = x^T R
            top = sv[s:e] @ R
            bot = np.concatenate([Fv[p, 0:3] @ R, Fv[p, 3:6] @ R])
            x = np.linalg.solve(self.blocks[self.body_shape[p]], np.concatenate([top.ravel(), bot]))
            lam[s:e] = x[:3 * (e - s)].reshape(-1, 3) @ R.T
            U[p, 0:3] = x[-6:-3] @ R.T
            U[p, 3:6] = x[-3:] @ R.T
        return np.concatenate([lam.ravel(), U.ravel()])

    def apply_resistance(self, v) -> np.ndarray:
        """Per body R_p M_ref^-1 R_p^T s (the shape's mobility block alone)."""
        sus = self.sus
        sv = np.asarray(v, dtype=np.float64).reshape(-1, 3)
        out = np.empty_like(sv)
        off = sus.body_off
        for p in range(sus.n_bodies):
            s, e = off[p], off[p + 1]
            m = 3 * (e - s)
            R = self.R[p]
            x = np.linalg.solve(self.blocks[self.body_shape[p]][:m, :m], (sv[s:e] @ R).ravel())
            out[s:e] = x.reshape(-1, 3) @ R.T
        return out.ravel()


# ----------------------------------------------------------------------------
# GMRES
# ----------------------------------------------------------------------------

def gmres(apply_A, apply_Pinv, b, tol=1e-12, restart=100, maxiter=1000):
    """Right-preconditioned GMRES(restart) from x0 = 0 with modified
    Gram-Schmidt and Givens rotations; stops when the true residual
    ||b - A x|| / ||b|| <= tol.  Returns (x, iterations, residual history)."""
    n = b.shape[0]
    bnorm = np.linalg.norm(b)
    x = np.zeros(n)
    if bnorm == 0.0:
        return x, 0, [0.0]
    hist = []
    it = 0
    while True:
        r = b - apply_A(x) if it > 0 else b.copy()
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta / bnorm <= tol or it >= maxiter:
            return x, it, hist
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for k in range(restart):
            w = apply_A(apply_Pinv(V[k]))
            for i in range(k + 1):
                H[i, k] = w @ V[i]
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0.0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            it += 1
            k_used = k + 1
            hist.append(abs(g[k + 1]) / bnorm)
            if abs(g[k + 1]) / bnorm <= tol or it >= maxiter:
                break
        y = sla.solve_triangular(H[:k_used, :k_used], g[:k_used])
        x = x + apply_Pinv(V[:k_used].T @ y)


def solve_resistance(sus, U, slip=None, tol=1e-12, restart=100, maxiter=1000, precond=None):
    """Resistance problem by right-preconditioned GMRES on M lambda = K U +
    slip with the block-diagonal M_pp^-1 (or `precond`'s apply_resistance),
    then F = K^T lambda.  Returns (F, lambda, info)."""
    t0 = time.perf_counter()
    P = BlockPreconditioner(sus) if precond is None else precond
    b = K_apply(sus.pos, sus.body_off, sus.q, U).ravel()
    if slip is not None:
        b = b + np.asarray(slip, dtype=np.float64).ravel()
    d3 = _shift3(sus)

    def apply_M(x):
        y = matvec(sus.pos, x.reshape(-1, 3), sus.a, sus.eta, sus.wall).ravel()
        return y if d3 is None else y + d3 * x

    lam, it, hist = gmres(apply_M, P.apply_resistance, b, tol, restart, maxiter)
    lam = lam.reshape(-1, 3)
    return KT_apply(sus.pos, sus.body_off, sus.q, lam), lam, {
        "iterations": it, "history": hist, "seconds": time.perf_counter() - t0}


def solve_mobility(sus, FT, slip=None, tol=1e-12, restart=100, maxiter=1000, precond=None):
    """Mobility problem by right-preconditioned GMRES with the block-diagonal
    preconditioner (or `precond`, e.g. a ShapePreconditioner).  Returns
    (U, lambda, info)."""
    t0 = time.perf_counter()
    P = BlockPreconditioner(sus) if precond is None else precond
    b = rhs(sus, FT, slip)
    x, it, hist = gmres(lambda v: saddle_apply(sus, v), P.apply, b, tol, restart, maxiter)
    lam, U = split(sus, x)
    return U.copy(), lam.copy(), {"iterations": it, "history": hist,
                                  "seconds": time.perf_counter() - t0}
