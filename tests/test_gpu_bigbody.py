"""Large bodies (3n x 3n blocks beyond the LDS path): batched MFMA Cholesky,
projection and apply of the block-diagonal preconditioner, against the
oracle's per-body dense solves (eq:saddle_M_precon)."""
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


def _sub(sus, bodies):
    """Suspension of a subset of bodies (block-diagonal preconditioner rows of
    those bodies are independent of the others)."""
    pos, off = [], [0]
    for p in bodies:
        o, e = sus.body_off[p], sus.body_off[p + 1]
        pos.append(sus.pos[o:e])
        off.append(off[-1] + e - o)
    return S.Suspension(np.concatenate(pos), np.array(off), sus.q[bodies], sus.a, sus.eta, sus.wall)


def _rows(sus, bodies, vec):
    """Rows of saddle vectors (k, 3Nb+6N) belonging to `bodies`."""
    nb3 = 3 * sus.n_blobs
    lam = [vec[:, 3 * sus.body_off[p]:3 * sus.body_off[p + 1]] for p in bodies]
    U = [vec[:, nb3 + 6 * p:nb3 + 6 * p + 6] for p in bodies]
    return np.concatenate(lam + U, axis=1)


def _mixed(n_shells=5, shell=162, n_ico=7, seed=3):
    rng = np.random.default_rng(seed)
    shapes = [S.sphere_shell(shell)] * n_shells + [S.icosahedron(1.0)] * n_ico
    order = rng.permutation(len(shapes))
    shapes = [shapes[k] for k in order]
    centres = np.stack([np.arange(len(shapes)) * 3.5, rng.uniform(0, 3, len(shapes)),
                        rng.uniform(1.5, 3.0, len(shapes))], axis=1)
    quats = np.stack([S.random_quaternion(rng) for _ in shapes])
    pos, off = S.assemble(shapes, centres, quats)
    return S.Suspension(pos, off, centres, 0.0871 * 2, 1.0, True, rng.standard_normal((len(shapes), 6)))


@pytest.mark.parametrize("shell,a", [(162, 0.0871), (42, 0.25)])
def test_large_body_precond_apply_parity(env, shell, a):
    rmb, torch, ctx, O = env
    s, rhs = S.shells_wall(n_bodies=4, n_blobs=shell, a=a, lateral=12.0, seed=41 + shell)
    print(f"[gpu] large-body precond {shell}-blob shells m={3 * shell}", flush=True)
    ref = np.stack([O.BlockPreconditioner(s).apply(r) for r in rhs])
    pc = rmb.Precond(ctx, rmb.System.from_suspension(s))
    got = pc.apply(_dev(torch, rhs)).cpu().numpy()
    err = _rel(got, ref)
    print(f"    8 rhs rel err {err:.2e}", flush=True)
    assert err <= 1e-10
    one = pc.apply(_dev(torch, rhs[:1])).cpu().numpy()
    assert np.array_equal(one[0], got[0])  # the apply of a column does not depend on the others
    pc.close()


def test_mixed_small_and_large_bodies(env):
    rmb, torch, ctx, O = env
    s = _mixed()
    rhs = np.random.default_rng(5).standard_normal((3, 3 * s.n_blobs + 6 * s.n_bodies))
    ref = np.stack([O.BlockPreconditioner(s).apply(r) for r in rhs])
    pc = rmb.Precond(ctx, rmb.System.from_suspension(s))
    got = pc.apply(_dev(torch, rhs)).cpu().numpy()
    assert _rel(got, ref) <= 1e-10
    pc.close()
    # and a full solve over the mixture matches the dense oracle
    Ud, _ = O.dense_solve(s, s.FT)
    U, lam, info = rmb.solve_mobility(ctx, rmb.System.from_suspension(s), _dev(torch, s.FT), tol=1e-11,
                                      precision="fp32")
    U = U.cpu().numpy()
    print(f"[gpu] mixed solve info {info} U err {_srel(U, Ud):.2e}", flush=True)
    assert info["status"] == 0 and _srel(U, Ud) <= 1e-8


def test_free_space_42_blob_shells_solve(env):
    rmb, torch, ctx, O = env
    rng = np.random.default_rng(8)
    shp = S.sphere_shell(42)
    centres = np.array([[0, 0, 0], [3.0, 0.5, 0], [0.2, 3.1, 0.4], [3.3, 3.0, -0.5]])
    quats = np.stack([S.random_quaternion(rng) for _ in centres])
    pos, off = S.assemble([shp] * 4, centres, quats)
    s = S.Suspension(pos, off, centres, 0.5 * S.min_spacing(shp), 1.0, False, rng.standard_normal((4, 6)))
    Ud, _ = O.dense_solve(s, s.FT)
    U, lam, info = rmb.solve_mobility(ctx, rmb.System.from_suspension(s), _dev(torch, s.FT), tol=1e-11)
    assert info["status"] == 0 and _srel(U.cpu().numpy(), Ud) <= 1e-8


def test_shell_batch_512x162_factor_and_apply_sampled(env):
    """The full batched factorisation (512 x 162-blob shells, 486 x 486
    blocks) applied to 8 right-hand sides; sampled bodies against the oracle."""
    rmb, torch, ctx, O = env
    s, rhs = S.shells_wall()
    sysd = rmb.System.from_suspension(s)
    print(f"[gpu] 512 x 162-blob shells: factor + apply 8 rhs", flush=True)
    pc = rmb.Precond(ctx, sysd)
    got = pc.apply(_dev(torch, rhs)).cpu().numpy()
    assert np.all(np.isfinite(got))
    bodies = np.sort(np.random.default_rng(9).choice(s.n_bodies, 6, replace=False))
    bodies = np.concatenate([[0], bodies, [s.n_bodies - 1]])
    sub = _sub(s, bodies)
    rsub = _rows(s, bodies, rhs)
    ref = np.stack([O.BlockPreconditioner(sub).apply(r) for r in rsub])
    err = _rel(_rows(s, bodies, got), ref)
    print(f"    sampled bodies rel err {err:.2e}", flush=True)
    assert err <= 1e-10
    pc.close()


def test_body_size_limit(env):
    rmb, torch, ctx, O = env
    shp = S.sphere_shell(642)
    s = S.Suspension(shp + np.array([0, 0, 3.0]), np.array([0, 642]), np.array([[0, 0, 3.0]]), 0.07, 1.0, True)
    with pytest.raises(rmb.RmbError) as e:
        rmb.Precond(ctx, rmb.System.from_suspension(s))
    assert e.value.status == rmb.RMB_EINVAL


def test_large_body_not_spd(env):
    rmb, torch, ctx, O = env
    shp = S.sphere_shell(162)
    pos = shp + np.array([0, 0, 1.0])
    pos[:, 2] = np.maximum(pos[:, 2], 0.01)  # flatten the bottom onto the wall
    s = S.Suspension(pos, np.array([0, 162]), np.array([[0, 0, 1.0]]), 0.3, 1.0, True)
    assert np.linalg.eigvalsh(O.assemble(s.pos, s.a, 1.0, True)).min() < 0
    with pytest.raises(rmb.RmbError) as e:
        rmb.Precond(ctx, rmb.System.from_suspension(s))
    assert e.value.status == rmb.RMB_ENOTSPD


def _padded(n):
    return (3 * n + 6 + 63) // 64 * 64


@pytest.mark.parametrize("shape", range(4))
def test_every_tile_shape(env, shape):
    """Each tile shape of the large-body factorisation, forced on a context
    for both padded sizes of the mixture (162-blob shells: 512; 42-blob
    shells: 192): the factor through rmb_precond_apply, and a full solve whose
    factors and applies go through the engine's per-panel-width tables,
    against the oracle.  (A solve once indexed the engine's two apply tables
    with the shape number, which aborted the process; this pins the mapping
    from shape to panel width.)"""
    rmb, torch, ctx, O = env
    shapes = rmb.tile_shapes()
    assert len(shapes) == 4
    c = rmb.Context(0)
    try:
        for Mp in (_padded(162), _padded(42)):
            c.set_tile_shape(Mp, shape)
        s = _mixed(n_shells=3, seed=11 + shape)
        s42 = _mixed(n_shells=2, shell=42, n_ico=3, seed=21 + shape)
        for sus in (s, s42):
            print(f"[gpu] tile shape {shape} {shapes[shape]} nb={sus.n_blobs}", flush=True)
            rhs = np.random.default_rng(6).standard_normal((2, 3 * sus.n_blobs + 6 * sus.n_bodies))
            ref = np.stack([O.BlockPreconditioner(sus).apply(r) for r in rhs])
            pc = rmb.Precond(c, rmb.System.from_suspension(sus))
            got = pc.apply(_dev(torch, rhs)).cpu().numpy()
            pc.close()
            assert _rel(got, ref) <= 1e-10
            Ud, _ = O.dense_solve(sus, sus.FT)
            U, lam, info = rmb.solve_mobility(c, rmb.System.from_suspension(sus), _dev(torch, sus.FT), tol=1e-11,
                                              precision="fp32")
            err = _srel(U.cpu().numpy(), Ud)
            print(f"    apply err {_rel(got, ref):.2e}, solve {info['iterations']} iterations, U err {err:.2e}",
                  flush=True)
            assert info["status"] == 0 and err <= 1e-8
        with pytest.raises(rmb.RmbError):
            c.set_tile_shape(512, len(shapes))
    finally:
        c.close()
