"""Resistance problem on the GPU (rmb_solve_resistance, eq:resistance_problem)
against the oracle: M lambda = K U + slip by preconditioned GMRES with the
blocks M_pp^-1, then F = K^T lambda.

Bar: F against the dense oracle (relative 1e-8 at solve tolerance 1e-10),
the oracle's FP64 residual ||K U + slip - M lambda|| / ||K U + slip|| within
the tolerance, and the GMRES iteration count of the FP64 solve within one of
the oracle's GMRES with the same preconditioner."""
import numpy as np
import pytest

import parity
import suspensions as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(oracle_mod):
    import torch
    import paper_1602_02170_amd as rmb
    ctx = rmb.Context(0)
    yield rmb, torch, ctx, oracle_mod
    ctx.close()


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


_rel = parity.solve_err  # 2-norm and per-row bound (tests/parity.py)


def _residual(O, sus, U, slip, lam):
    b = O.K_apply(sus.pos, sus.body_off, sus.q, U)
    if slip is not None:
        b = b + slip
    r = b - O.matvec(sus.pos, lam, sus.a, sus.eta, sus.wall)
    if getattr(sus, "blob_shift", None) is not None:
        r = r - sus.blob_shift[:, None] * lam
    return np.linalg.norm(r) / np.linalg.norm(b)


def _lattice(nside, spacing=2.6):
    shp = S.sphere_shell(42)
    c = spacing * np.array([[i, j, k] for i in range(nside) for j in range(nside) for k in range(nside)], float)
    pos, off = S.assemble([shp] * len(c), c, np.tile([1.0, 0, 0, 0], (len(c), 1)))
    return S.Suspension(pos, off, c, 0.5 * S.min_spacing(shp), 1.0, False)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_resistance_parity_wall(env, prec):
    rmb, torch, ctx, O = env
    sus = S.boomerangs_wall(n_bodies=60, lateral=50.0, seed=401)
    rng = np.random.default_rng(402)
    U = rng.standard_normal((sus.n_bodies, 6))
    slip = 0.2 * rng.standard_normal((sus.n_blobs, 3))
    Fd, ld = O.resistance_dense(sus, U, slip)
    _, _, io = O.solve_resistance(sus, U, slip, tol=1e-10)
    F, lam, info = rmb.solve_resistance(ctx, rmb.System.from_suspension(sus), _dev(torch, U), _dev(torch, slip),
                                        tol=1e-10, precision=prec)
    F, lam = F.cpu().numpy(), lam.cpu().numpy()
    res = _residual(O, sus, U, slip, lam)
    print(f"[gpu] resistance wall 60 boomerangs {prec}: {info} residual {res:.2e} F err {_rel(F, Fd):.2e} "
          f"oracle iterations {io['iterations']}", flush=True)
    assert info["status"] == 0 and res <= 1.05e-10
    assert _rel(F, Fd) <= 1e-8 and _rel(lam, ld) <= 1e-8
    if prec == "fp64":
        assert abs(info["iterations"] - io["iterations"]) <= 1


def test_resistance_iterations_grow_with_size(env):
    """Lattices of 42-blob shells, 8 and 27 bodies (336 and 1134 blobs, the
    second on the symmetric product): resistance iterations grow, mobility
    iterations barely do (Sec. 4.4); the larger one against the dense
    oracle."""
    rmb, torch, ctx, O = env
    its = {}
    for nside in (2, 3):
        sus = _lattice(nside)
        sysd = rmb.System.from_suspension(sus)
        U = np.random.default_rng(3).standard_normal((sus.n_bodies, 6))
        F, lam, ir = rmb.solve_resistance(ctx, sysd, _dev(torch, U), tol=1e-8)
        FT = np.random.default_rng(4).standard_normal((sus.n_bodies, 6))
        _, _, im = rmb.solve_mobility(ctx, sysd, _dev(torch, FT), tol=1e-8)
        its[nside] = (ir["iterations"], im["iterations"])
        if nside == 3:
            Fd, _ = O.resistance_dense(sus, U)
            assert _rel(F.cpu().numpy(), Fd) <= 1e-6
            assert _residual(O, sus, U, None, lam.cpu().numpy()) <= 1.05e-8
    print(f"[gpu] resistance/mobility iterations: {its}", flush=True)
    assert its[3][0] / its[2][0] > its[3][1] / its[2][1] + 0.2


def test_resistance_large_bodies_and_permeable(env):
    rmb, torch, ctx, O = env
    sus, _ = S.shells_wall(n_bodies=4, lateral=10.0, seed=93)
    U = np.random.default_rng(5).standard_normal((sus.n_bodies, 6))
    for shift in (None, np.random.default_rng(6).uniform(0.2, 3.0, sus.n_blobs)):
        sus.blob_shift = shift
        Fd, _ = O.resistance_dense(sus, U)
        F, lam, info = rmb.solve_resistance(ctx, rmb.System.from_suspension(sus), _dev(torch, U), tol=1e-10)
        print(f"[gpu] resistance shells permeable={shift is not None}: {info} F err "
              f"{_rel(F.cpu().numpy(), Fd):.2e}", flush=True)
        assert info["status"] == 0 and _rel(F.cpu().numpy(), Fd) <= 1e-8


def test_resistance_with_shared_blocks(env):
    rmb, torch, ctx, O = env
    sus = S.boomerangs_wall(n_bodies=40, lateral=40.0, seed=403)
    boo = S.boomerang()
    sysd = rmb.System.from_suspension(sus)
    pc = rmb.Precond.from_shapes(ctx, sysd, [boo - boo.mean(axis=0)], np.zeros(sus.n_bodies, np.int32),
                                 _dev(torch, sus.quat))
    U = np.random.default_rng(7).standard_normal((sus.n_bodies, 6))
    Fd, _ = O.resistance_dense(sus, U)
    Q = O.ShapePreconditioner(sus, [boo - boo.mean(axis=0)], np.zeros(sus.n_bodies, int), sus.quat)
    _, _, io = O.solve_resistance(sus, U, tol=1e-10, precond=Q)
    F, lam, info = rmb.solve_resistance(ctx, sysd, _dev(torch, U), precond=pc, tol=1e-10)
    assert info["status"] == 0 and _rel(F.cpu().numpy(), Fd) <= 1e-8
    assert abs(info["iterations"] - io["iterations"]) <= 1
    pc.close()


def test_mobility_then_resistance_round_trip(env):
    """U from the mobility solve, then F back from the resistance solve."""
    rmb, torch, ctx, O = env
    sus = S.boomerangs_wall(n_bodies=80, lateral=np.sqrt(40 * 80), seed=404)
    sysd = rmb.System.from_suspension(sus)
    U, _, _ = rmb.solve_mobility(ctx, sysd, _dev(torch, sus.FT), tol=1e-12)
    F, _, info = rmb.solve_resistance(ctx, sysd, U, tol=1e-12)
    assert info["status"] == 0 and _rel(F.cpu().numpy(), sus.FT) <= 1e-9


def test_resistance_full_boomerangs(env):
    """1000 x 15-blob boomerangs (15,000 blobs), FP32 pairs with FP64
    refinement to 1e-8, checked by the oracle's FP64 residual."""
    rmb, torch, ctx, O = env
    sus = S.boomerangs_wall()
    U = np.random.default_rng(8).standard_normal((sus.n_bodies, 6))
    print("[gpu] resistance, full boomerangs", flush=True)
    F, lam, info = rmb.solve_resistance(ctx, rmb.System.from_suspension(sus), _dev(torch, U), tol=1e-8,
                                        precision="fp32")
    res = _residual(O, sus, U, None, lam.cpu().numpy())
    print(f"    {info} oracle residual {res:.2e}", flush=True)
    assert info["status"] == 0 and res <= 1.05e-8
    Fo = O.KT_apply(sus.pos, sus.body_off, sus.q, lam.cpu().numpy())
    assert _rel(F.cpu().numpy(), Fo) <= 1e-12


def test_resistance_errors(env):
    rmb, torch, ctx, O = env
    sus = S.boomerangs_wall(n_bodies=5, lateral=10.0)
    sysd = rmb.System.from_suspension(sus)
    with pytest.raises(ValueError):
        rmb.solve_resistance(ctx, sysd, _dev(torch, np.zeros((4, 6))))
    sus.blob_shift = np.full(sus.n_blobs, -1.0)
    with pytest.raises(rmb.RmbError) as e:
        rmb.solve_resistance(ctx, rmb.System.from_suspension(sus), _dev(torch, np.zeros((5, 6))))
    assert e.value.status == rmb.RMB_EINVAL
    # U = 0 and no slip: lambda = 0, F = 0
    sus.blob_shift = None
    F, lam, info = rmb.solve_resistance(ctx, sysd, _dev(torch, np.zeros((5, 6))))
    assert info["status"] == 0 and float(F.abs().max()) == 0.0 and float(lam.abs().max()) == 0.0
