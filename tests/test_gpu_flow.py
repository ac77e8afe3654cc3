"""Parity of the HIP flow-field product (rmb_flow_field) with the CPU FP64
oracle: each blob split into tracer-size blobs at fixed offsets on its
surface, carrying equal shares of its force, and the velocity of the fluid
taken at arbitrary points (appendix on computing flow fields).

Bar: relative 2-norm error <= 1e-12 for FP64 pairs and <= 1e-5 for FP32
pairs with FP64 accumulation, as for the square product.
"""
import numpy as np
import pytest

import parity
import suspensions as S

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _ico():
    u = S.icosahedron()
    return u / np.linalg.norm(u, axis=1, keepdims=True)


@pytest.fixture(scope="module")
def env(oracle_mod):
    import torch
    import paper_1602_02170_amd as rmb
    ctx = rmb.Context(0)
    yield rmb, torch, ctx, oracle_mod
    ctx.close()


def _run(env, sus, lam, offs, ta, targets, prec):
    rmb, torch, ctx, _ = env
    sysd = rmb.System.from_suspension(sus)
    lt = torch.tensor(lam, dtype=torch.float64, device="cuda")
    tt = torch.tensor(targets, dtype=torch.float64, device="cuda").reshape(-1, 3)
    v = rmb.flow_field(ctx, sysd, lt, offs, ta, tt, prec)
    torch.cuda.synchronize()
    return v.cpu().numpy()


_rel = parity.err  # 2-norm and per-row bound (tests/parity.py)


def _plane(z, nx=40, ny=30, half=25.0):
    gx, gy = np.meshgrid(np.linspace(-half, half, nx), np.linspace(-half, half, ny))
    return np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, z)], 1)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("wall", [True, False])
def test_flow_field_plane_parity(env, wall, prec):
    """60 boomerangs (900 blobs) split 12 ways: 10,800 sources in several
    chunks, 1,200 targets on a plane (last target tile ragged)."""
    sus = S.boomerangs_wall(n_bodies=60, lateral=40.0)
    sus.wall = wall
    lam = np.random.default_rng(21).standard_normal((sus.n_blobs, 3))
    T = _plane(3.0)
    print(f"[gpu] flow field plane wall={wall} {prec} ns={sus.n_blobs * 12} nt={len(T)}", flush=True)
    ref = env[3].flow_field(sus.pos, lam, sus.a, _ico(), 0.1 * sus.a, T, sus.eta, sus.wall)
    v = _run(env, sus, lam, _ico(), 0.1 * sus.a, T, prec)
    err = _rel(v, ref)
    print(f"    rel err {err:.3e}", flush=True)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_flow_field_inside_and_near_blobs(env, prec):
    """Targets on the blobs themselves, on sub-blob centres and inside the
    near-field overlap range of the tracer radius."""
    sus = S.boomerangs_wall(n_bodies=7, lateral=10.0)
    rng = np.random.default_rng(22)
    lam = rng.standard_normal((sus.n_blobs, 3))
    u = _ico()
    ta = 0.25 * sus.a
    T = np.concatenate([sus.pos, sus.pos[:5] + sus.a * u[:5],
                        sus.pos[5:40] + rng.uniform(-0.4, 0.4, (35, 3)) * ta])
    T[:, 2] = np.maximum(T[:, 2], 0.05)
    print(f"[gpu] flow field near {prec} nt={len(T)}", flush=True)
    ref = env[3].flow_field(sus.pos, lam, sus.a, u, ta, T, sus.eta, sus.wall)
    v = _run(env, sus, lam, u, ta, T, prec)
    err = _rel(v, ref)
    print(f"    rel err {err:.3e}", flush=True)
    assert err <= TOL[prec]
    assert np.all(np.isfinite(v))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_flow_field_full_monolayer_sampled(env, prec):
    """196,608-blob monolayer split 12 ways (2.36M sources) over a
    128 x 128 plane of targets; 16 sampled targets against the oracle."""
    sus, lam = S.icosahedra_monolayer()
    # blobs sit as low as z = 0.2 < a, so the sub-blobs lie on a sphere of
    # radius 0.4 a to stay above the wall
    offs = 0.4 * _ico()
    lo, hi = sus.pos[:, :2].min(0), sus.pos[:, :2].max(0)
    gx, gy = np.meshgrid(np.linspace(lo[0], hi[0], 128), np.linspace(lo[1], hi[1], 128))
    T = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, 2.5)], 1)
    print(f"[gpu] flow field full monolayer {prec} ns={sus.n_blobs * 12} nt={len(T)}", flush=True)
    v = _run(env, sus, lam, offs, 0.1 * sus.a, T, prec)
    rows = np.concatenate([np.random.default_rng(23).choice(len(T), 14, replace=False), [0, len(T) - 1]])
    ref = env[3].flow_field(sus.pos, lam, sus.a, offs, 0.1 * sus.a, T[rows], sus.eta, sus.wall)
    err = _rel(v[rows], ref)
    print(f"    sampled rel err {err:.3e}", flush=True)
    assert err <= TOL[prec]
    assert np.all(np.isfinite(v))


def test_flow_field_trivial_split_matches_matvec(env):
    """One sub-blob at zero offset with the blob's own radius, evaluated at
    the blob positions, is the mobility product."""
    rmb, torch, ctx, O = env
    sus = S.boomerangs_wall(n_bodies=20, lateral=20.0)
    lam = np.random.default_rng(24).standard_normal((sus.n_blobs, 3))
    v = _run(env, sus, lam, np.zeros((1, 3)), sus.a, sus.pos, "fp64")
    sysd = rmb.System.from_suspension(sus)
    m = rmb.mobility_matvec(ctx, sysd, torch.tensor(lam, dtype=torch.float64, device="cuda"), "fp64")
    assert _rel(v, m.cpu().numpy()) <= 1e-13


def test_flow_field_deterministic_and_edges(env):
    rmb, torch, ctx, O = env
    sus = S.boomerangs_wall(n_bodies=10, lateral=12.0)
    lam = np.random.default_rng(25).standard_normal((sus.n_blobs, 3))
    T = _plane(1.5, 9, 7, 6.0)
    for prec in ("fp64", "fp32"):
        v1 = _run(env, sus, lam, _ico(), 0.1 * sus.a, T, prec)
        v2 = _run(env, sus, lam, _ico(), 0.1 * sus.a, T, prec)
        assert np.array_equal(v1, v2)
    # one target
    v = _run(env, sus, lam, _ico(), 0.1 * sus.a, T[:1], "fp64")
    ref = O.flow_field(sus.pos, lam, sus.a, _ico(), 0.1 * sus.a, T[:1], sus.eta, sus.wall)
    assert _rel(v, ref) <= TOL["fp64"]
    # no targets: nothing to do
    assert _run(env, sus, lam, _ico(), 0.1 * sus.a, np.zeros((0, 3)), "fp64").shape == (0, 3)


def test_flow_field_rejects_bad_input(env):
    rmb, torch, ctx, O = env
    sus = S.boomerangs_wall(n_bodies=4, lateral=8.0)
    lam = np.ones((sus.n_blobs, 3))
    T = _plane(2.0, 4, 4, 3.0)
    # a target at or below the wall
    Tb = T.copy()
    Tb[3, 2] = -0.5
    with pytest.raises(rmb.RmbError) as e:
        _run(env, sus, lam, _ico(), 0.1 * sus.a, Tb, "fp64")
    assert e.value.status == rmb.RMB_EINVAL and "target" in str(e.value)
    # sub-blob offsets that reach through the wall
    with pytest.raises(rmb.RmbError) as e:
        _run(env, sus, lam, 50.0 * _ico(), 0.1 * sus.a, T, "fp64")
    assert e.value.status == rmb.RMB_EINVAL and "z <= 0" in str(e.value)
    # no sub-blobs, bad tracer radius, non-finite offsets
    for offs, ta in [(np.zeros((0, 3)), 0.1), (_ico(), 0.0), (np.full((2, 3), np.nan), 0.1)]:
        with pytest.raises(rmb.RmbError) as e:
            _run(env, sus, lam, offs, ta, T, "fp64")
        assert e.value.status == rmb.RMB_EINVAL
    # the context still works afterwards
    v = _run(env, sus, lam, _ico(), 0.1 * sus.a, T, "fp64")
    ref = O.flow_field(sus.pos, lam, sus.a, _ico(), 0.1 * sus.a, T, sus.eta, sus.wall)
    assert _rel(v, ref) <= TOL["fp64"]
