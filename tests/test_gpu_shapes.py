"""Shared reference-shape preconditioner on the GPU (rmb_precond_factor_shapes,
rmb_precond_set_orientations) against the oracle's ShapePreconditioner
(Sec. 2.2.2 after eq:saddle_M_precon; Sec. 5.4), and solves that use it.

Bar: the apply as for the per-body preconditioner (relative 1e-10 over the
whole output); solves as for the per-body solves (the oracle's FP64
residual within the tolerance, U against the dense solve)."""
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


_rel = parity.err  # 2-norm and per-row bound (tests/parity.py)
_srel = parity.solve_err  # the same for solve results


def _centred(shp):
    return shp - shp.mean(axis=0)


def _by_size(sus, shapes):
    """Shape index of every body, matched by blob count."""
    sizes = {len(s): k for k, s in enumerate(shapes)}
    return np.array([sizes[int(n)] for n in np.diff(sus.body_off)], dtype=np.int32)


def _mixed_large(seed=7):
    """Seven 162-blob shells and nine icosahedra above the wall (both the
    LDS path and the MFMA path, two shapes)."""
    rng = np.random.default_rng(seed)
    shapes = [_centred(S.sphere_shell(162)), _centred(S.icosahedron(1.0))]
    kinds = rng.permutation([0] * 7 + [1] * 9)
    centres = np.stack([np.arange(len(kinds)) * 3.5, rng.uniform(0, 3, len(kinds)),
                        rng.uniform(1.5, 3.0, len(kinds))], axis=1)
    quats = np.stack([S.random_quaternion(rng) for _ in kinds])
    pos, off = S.assemble([shapes[k] for k in kinds], centres, quats)
    sus = S.Suspension(pos, off, centres, 0.1742, 1.0, True, rng.standard_normal((len(kinds), 6)), None, 1e-8,
                       quats)
    return sus, shapes


def _cases():
    out = []
    s = S.boomerangs_wall(n_bodies=60, lateral=50.0)
    out.append(("wall 60 boomerangs", s, [_centred(S.boomerang())]))
    s = S.mixed_wall_request(4, n_bodies=40)
    out.append(("wall 40 mixed", s, [_centred(S.icosahedron(1.0)), _centred(S.boomerang())]))
    s, _ = S.shells_wall(n_bodies=4, lateral=12.0, seed=77)
    out.append(("wall 4 x 162-blob shells", s, [_centred(S.sphere_shell(162))]))
    s, shapes = _mixed_large()
    out.append(("wall shells + icosahedra", s, shapes))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_shared_apply_parity(env, case):
    rmb, torch, ctx, O = env
    name, sus, shapes = CASES[case]
    idx = _by_size(sus, shapes)
    print(f"[gpu] shared precond apply {name}", flush=True)
    rhs = np.random.default_rng(31 + case).standard_normal((3, 3 * sus.n_blobs + 6 * sus.n_bodies))
    Q = O.ShapePreconditioner(sus, shapes, idx, sus.quat)
    ref = np.stack([Q.apply(r) for r in rhs])
    pc = rmb.Precond.from_shapes(ctx, rmb.System.from_suspension(sus), shapes, idx, _dev(torch, sus.quat))
    got = pc.apply(_dev(torch, rhs)).cpu().numpy()
    err = _rel(got, ref)
    print(f"    rel err {err:.2e}", flush=True)
    assert err <= 1e-10
    pc.close()


@pytest.mark.parametrize("which", ["boomerangs", "shells + icosahedra"])
def test_shared_equals_per_body_in_free_space(env, which):
    rmb, torch, ctx, O = env
    if which == "boomerangs":
        sus = S.boomerangs_wall(n_bodies=50, lateral=45.0)
        shapes = [_centred(S.boomerang())]
    else:
        sus, shapes = _mixed_large(seed=9)
    sus.wall = False
    idx = _by_size(sus, shapes)
    sysd = rmb.System.from_suspension(sus)
    rhs = _dev(torch, np.random.default_rng(41).standard_normal((2, 3 * sus.n_blobs + 6 * sus.n_bodies)))
    a = rmb.Precond(ctx, sysd).apply(rhs).cpu().numpy()
    b = rmb.Precond.from_shapes(ctx, sysd, shapes, idx, _dev(torch, sus.quat)).apply(rhs).cpu().numpy()
    err = _rel(b, a)
    print(f"[gpu] shared vs per-body, free space, {which}: rel {err:.2e}", flush=True)
    assert err <= 1e-10


def test_solve_with_shared_blocks_wall(env):
    """80 boomerangs above the wall: the unbounded shared blocks still give
    the exact solution; the iteration count matches the oracle's GMRES with
    the same preconditioner and is at most 1.5x that of the wall blocks."""
    rmb, torch, ctx, O = env
    sus = S.boomerangs_wall(n_bodies=80, lateral=np.sqrt(40 * 80), seed=101)
    shapes = [_centred(S.boomerang())]
    idx = _by_size(sus, shapes)
    sysd = rmb.System.from_suspension(sus)
    pc = rmb.Precond.from_shapes(ctx, sysd, shapes, idx, _dev(torch, sus.quat))
    FT = _dev(torch, sus.FT)
    Ud, _ = O.dense_solve(sus, sus.FT)
    _, _, io = O.solve_mobility(sus, sus.FT, tol=1e-10, precond=O.ShapePreconditioner(sus, shapes, idx, sus.quat))
    for prec in ("fp64", "fp32"):
        U, lam, info = rmb.solve_mobility(ctx, sysd, FT, precond=pc, tol=1e-10, precision=prec)
        U, lam = U.cpu().numpy(), lam.cpu().numpy()
        res = O.relative_residual(sus, sus.FT, None, U, lam)
        _, _, iw = rmb.solve_mobility(ctx, sysd, FT, tol=1e-10, precision=prec)
        # velocities to the 1e-8 bar: the same solve under velocity-error control
        Uv, _, iv = rmb.solve_mobility(ctx, sysd, FT, precond=pc, tol=1e-10, u_tol=1e-9, precision=prec)
        Uv = Uv.cpu().numpy()
        print(f"[gpu] shared-block solve {prec}: {info} oracle residual {res:.2e} U err {_srel(U, Ud):.2e}; "
              f"oracle iterations {io['iterations']}, wall blocks {iw['iterations']}", flush=True)
        assert info["status"] == 0 and res <= 1.05e-10
        assert iv["status"] == 0 and _srel(Uv, Ud) <= 1e-8, (iv, _srel(Uv, Ud))
        if prec == "fp64":
            assert abs(info["iterations"] - io["iterations"]) <= 1
            assert info["iterations"] <= 1.5 * iw["iterations"]
    pc.close()


def test_solve_with_shared_blocks_full_boomerangs(env):
    """1000 x 15-blob boomerangs (15,000 blobs) to 1e-8 with the shared
    unbounded blocks, FP32 pairs with FP64 refinement."""
    rmb, torch, ctx, O = env
    sus = S.boomerangs_wall()
    shapes = [_centred(S.boomerang())]
    sysd = rmb.System.from_suspension(sus)
    pc = rmb.Precond.from_shapes(ctx, sysd, shapes, np.zeros(sus.n_bodies, np.int32), _dev(torch, sus.quat))
    print("[gpu] full boomerangs, shared blocks", flush=True)
    U, lam, info = rmb.solve_mobility(ctx, sysd, _dev(torch, sus.FT), precond=pc, tol=1e-8, precision="fp32")
    res = O.relative_residual(sus, sus.FT, None, U.cpu().numpy(), lam.cpu().numpy())
    print(f"    info {info} oracle residual {res:.2e}", flush=True)
    assert info["status"] == 0 and res <= 1.05e-8
    pc.close()


def test_set_orientations_follows_the_bodies(env):
    """The same bodies turned to new orientations: new quaternions only, no
    refactorisation, and the apply matches the oracle for the new
    configuration."""
    rmb, torch, ctx, O = env
    sus = S.boomerangs_wall(n_bodies=30, lateral=35.0)
    shapes = [_centred(S.boomerang())]
    idx = np.zeros(sus.n_bodies, np.int32)
    pc = rmb.Precond.from_shapes(ctx, rmb.System.from_suspension(sus), shapes, idx, _dev(torch, sus.quat))
    rng = np.random.default_rng(51)
    q2 = np.stack([S.random_quaternion(rng) for _ in range(sus.n_bodies)])
    pos2, off2 = S.assemble([shapes[0]] * sus.n_bodies, sus.q + np.array([0, 0, 3.0]), q2)
    sus2 = S.Suspension(pos2, off2, sus.q + np.array([0, 0, 3.0]), sus.a, 1.0, True, None, None, 1e-8, q2)
    pc.set_orientations(_dev(torch, 0.5 * q2))
    rhs = np.random.default_rng(52).standard_normal((2, 3 * sus.n_blobs + 6 * sus.n_bodies))
    Q = O.ShapePreconditioner(sus2, shapes, idx, q2)
    ref = np.stack([Q.apply(r) for r in rhs])
    got = pc.apply(_dev(torch, rhs)).cpu().numpy()
    assert _rel(got, ref) <= 1e-10
    pc.close()


def test_shared_precond_errors(env):
    rmb, torch, ctx, O = env
    sus = S.mixed_wall_request(6, n_bodies=12)
    shapes = [_centred(S.icosahedron(1.0)), _centred(S.boomerang())]
    idx = _by_size(sus, shapes)
    sysd = rmb.System.from_suspension(sus)
    qd = _dev(torch, sus.quat)
    # a body whose blob count differs from its shape's
    with pytest.raises(rmb.RmbError) as e:
        rmb.Precond.from_shapes(ctx, sysd, shapes, 1 - idx, qd)
    assert e.value.status == rmb.RMB_EINVAL and "blobs" in str(e.value)
    # shape index out of range
    bad = idx.copy()
    bad[3] = 2
    with pytest.raises(rmb.RmbError) as e:
        rmb.Precond.from_shapes(ctx, sysd, shapes, bad, qd)
    assert e.value.status == rmb.RMB_EINVAL
    # a zero quaternion
    q0 = sus.quat.copy()
    q0[5] = 0.0
    with pytest.raises(rmb.RmbError) as e:
        rmb.Precond.from_shapes(ctx, sysd, shapes, idx, _dev(torch, q0))
    assert e.value.status == rmb.RMB_EINVAL and "quaternion" in str(e.value)
    # new orientations only for shared-shape factors
    pc = rmb.Precond(ctx, sysd)
    with pytest.raises(rmb.RmbError) as e:
        pc.set_orientations(qd)
    assert e.value.status == rmb.RMB_EINVAL
    pc.close()
    # and a good build still works afterwards
    pc = rmb.Precond.from_shapes(ctx, sysd, shapes, idx, qd)
    with pytest.raises(rmb.RmbError):
        pc.set_orientations(_dev(torch, q0))
    pc.set_orientations(qd)
    rhs = np.random.default_rng(61).standard_normal((1, 3 * sus.n_blobs + 6 * sus.n_bodies))
    ref = O.ShapePreconditioner(sus, shapes, idx, sus.quat).apply(rhs[0])
    assert _rel(pc.apply(_dev(torch, rhs)).cpu().numpy()[0], ref) <= 1e-10
    pc.close()
