"""GPU mobility solves against the CPU oracle.

Bar (velocities): ||U - U_oracle|| / ||U_oracle|| <= 1e-8 for solves run to a
residual tight enough that the forward error is below it; every solve's FP64
residual ||b - A x|| / ||b|| is re-evaluated by the oracle on the GPU's
(U, lambda) and must meet the requested tolerance.  lambda is checked through
that residual (it is unique, but only determined to the solve tolerance).
"""
import os

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


def _solve(env, sus, FT=None, slip=None, **opts):
    rmb, torch, ctx, _ = env
    sysd = rmb.System.from_suspension(sus)
    FT = sus.FT if FT is None else FT
    U, lam, info = rmb.solve_mobility(ctx, sysd, _dev(torch, FT), None if slip is None else _dev(torch, slip),
                                      **opts)
    torch.cuda.synchronize()
    return U.cpu().numpy(), lam.cpu().numpy(), info


_rel = parity.solve_err  # 2-norm and per-row bound (tests/parity.py)


def small_wall():
    return S.boomerangs_wall(n_bodies=80, lateral=56.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_free_space_spheres_parity(env, prec):
    O = env[3]
    s = S.spheres_free_space()
    print(f"[gpu] free-space 8 spheres {prec}", flush=True)
    Ud, ld = O.dense_solve(s, s.FT)
    U, lam, info = _solve(env, s, tol=1e-10, precision=prec)
    res = O.relative_residual(s, s.FT, None, U, lam)
    print(f"    info {info}  oracle residual {res:.2e}  U err {_rel(U, Ud):.2e}", flush=True)
    assert info["status"] == 0
    assert info["rel_residual"] <= 1e-10
    assert res <= 1.05e-10
    assert _rel(U, Ud) <= 1e-8
    if prec == "fp32":
        assert info["matvecs_fp32"] > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wall_boomerangs_parity(env, prec):
    O = env[3]
    s = small_wall()
    print(f"[gpu] wall 80 boomerangs {prec}", flush=True)
    Ud, ld = O.dense_solve(s, s.FT)
    U, lam, info = _solve(env, s, tol=1e-8, precision=prec)
    res = O.relative_residual(s, s.FT, None, U, lam)
    print(f"    tol 1e-8: info {info}  oracle residual {res:.2e}  U err {_rel(U, Ud):.2e}", flush=True)
    assert info["status"] == 0 and res <= 1.05e-8
    U, lam, info = _solve(env, s, tol=1e-11, precision=prec)
    res = O.relative_residual(s, s.FT, None, U, lam)
    print(f"    tol 1e-11: info {info}  oracle residual {res:.2e}  U err {_rel(U, Ud):.2e}", flush=True)
    assert info["status"] == 0 and res <= 1.05e-11
    assert _rel(U, Ud) <= 1e-8


def test_wall_slip_parity(env):
    O = env[3]
    s = small_wall()
    slip = np.random.default_rng(21).standard_normal((s.n_blobs, 3)) * 0.2
    FT = np.random.default_rng(22).standard_normal((s.n_bodies, 6))
    Ud, ld = O.dense_solve(s, FT, slip)
    U, lam, info = _solve(env, s, FT=FT, slip=slip, tol=1e-11)
    res = O.relative_residual(s, FT, slip, U, lam)
    print(f"[gpu] slip: info {info}  oracle residual {res:.2e}  U err {_rel(U, Ud):.2e}", flush=True)
    assert info["status"] == 0 and res <= 1.05e-11
    assert _rel(U, Ud) <= 1e-8


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_full_boomerang_suspension_velocities(env):
    """The headline workload, 1000 x 15-blob boomerangs (15,000 blobs),
    solved to a relative residual of 1e-8 with the velocity error bounded by
    1e-8 as well: U matches the oracle's GMRES solution to 1e-12 (stored by
    tests/golden/make_oracle_solutions.py) within 1e-8 for FP64 pairs and for
    FP32 pairs with FP64 refinement, and the oracle's FP64 residual of the
    GPU result meets the tolerance."""
    O = env[3]
    s = S.boomerangs_wall()
    Uo = np.loadtxt(os.path.join(GOLDEN, "boomerangs1000_oracle_U.txt"))
    assert Uo.shape == (s.n_bodies, 6)
    for prec in ("fp32", "fp64", "relaxed"):
        print(f"[gpu] full boomerangs {prec}", flush=True)
        U0, lam0, info0 = _solve(env, s, tol=1e-8, precision=prec)
        U, lam, info = _solve(env, s, tol=1e-8, u_tol=1e-8, precision=prec)
        res = O.relative_residual(s, s.FT, None, U, lam)
        print(f"    residual only: {info0['iterations']} iterations, U err {parity.rel2(U0, Uo):.2e}", flush=True)
        print(f"    velocity bound: {info}  oracle residual {res:.2e}  U err {parity.rel2(U, Uo):.2e} "
              f"(worst body {parity.rowmax(U, Uo):.2e})", flush=True)
        assert info0["status"] == 0 and O.relative_residual(s, s.FT, None, U0, lam0) <= 1.05e-8
        assert info["status"] == 0
        assert res <= 1.05e-8
        assert info["tol_internal"] <= 1e-8 and 0 < info["u_err_est"] <= 1e-8
        assert _rel(U, Uo) <= 1e-8


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_band_product_and_solve(env, prec, monkeypatch):
    """The symmetric product in many bands of tile rows (the path of systems
    above about 210,000 blobs, forced here on 1,200 blobs by a 64 KiB band
    budget: 19 tile rows in about a dozen bands) against the one-band
    product and solve of the default context, and the solve against the
    oracle."""
    rmb, torch, ctx, O = env
    s = small_wall()
    monkeypatch.setenv("RMB_SYM_BAND_BYTES", str(64 << 10))
    cb = rmb.Context(0)
    try:
        print(f"[gpu] multi-band 80 boomerangs {prec}", flush=True)
        sysd = rmb.System.from_suspension(s)
        lam = _dev(torch, np.random.default_rng(61).standard_normal((s.n_blobs, 3)))
        v1 = rmb.mobility_matvec(ctx, sysd, lam, prec).cpu().numpy()
        vb = rmb.mobility_matvec(cb, sysd, lam, prec).cpu().numpy()
        ref = O.matvec(s.pos, lam.cpu().numpy(), s.a, s.eta, s.wall)
        print(f"    product: bands vs one band {parity.rel2(vb, v1):.2e}, vs oracle {parity.err(vb, ref):.2e}",
              flush=True)
        assert parity.err(vb, v1) <= 1e-14  # only the order of the FP64 sums over bands differs
        assert parity.err(vb, ref) <= (1e-12 if prec == "fp64" else 1e-5)
        Ud, _ = O.dense_solve(s, s.FT)
        U1, _, i1 = _solve(env, s, tol=1e-11, precision=prec)
        Ub, lb, ib = rmb.solve_mobility(cb, sysd, _dev(torch, s.FT), tol=1e-11, precision=prec)
        Ub, lb = Ub.cpu().numpy(), lb.cpu().numpy()
        res = O.relative_residual(s, s.FT, None, Ub, lb)
        print(f"    solve: iterations {ib['iterations']} (one band {i1['iterations']}), oracle residual {res:.2e}, "
              f"U err {_rel(Ub, Ud):.2e}, vs one band {_rel(Ub, U1):.2e}", flush=True)
        assert ib["status"] == 0 and res <= 1.05e-11
        assert _rel(Ub, Ud) <= 1e-8
        assert abs(ib["iterations"] - i1["iterations"]) <= 1
    finally:
        cb.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "relaxed"])
def test_velocity_error_control(env, prec):
    """80 wall boomerangs: with u_tol = 1e-8 the velocities match the dense
    solution within 1e-8 whatever the residual tolerance asked, the solver
    tightens its residual target (tol_internal) and its error estimate is
    of the size of the true error."""
    O = env[3]
    s = small_wall()
    Ud, _ = O.dense_solve(s, s.FT)
    U, lam, info = _solve(env, s, tol=1e-8, u_tol=1e-8, precision=prec)
    err = _rel(U, Ud)
    print(f"[gpu] velocity bound {prec}: {info} U err {parity.rel2(U, Ud):.2e}", flush=True)
    assert info["status"] == 0 and err <= 1e-8
    assert info["tol_internal"] <= 1e-8 and info["gamma"] > 0
    assert info["u_err_est"] <= 1e-8
    assert parity.rel2(U, Ud) <= 10 * info["u_err_est"]
    # a loose residual tolerance is tightened to reach the velocity bound
    U, lam, info = _solve(env, s, tol=1e-4, u_tol=1e-8, precision=prec)
    print(f"    tol 1e-4: {info} U err {parity.rel2(U, Ud):.2e}", flush=True)
    assert info["status"] == 0 and _rel(U, Ud) <= 1e-8 and info["tol_internal"] < 1e-8
    # resistance solves refuse it
    rmb, torch = env[0], env[1]
    with pytest.raises(rmb.RmbError) as e:
        rmb.solve_resistance(env[2], rmb.System.from_suspension(s), _dev(torch, np.zeros((s.n_bodies, 6))),
                             u_tol=1e-8)
    assert e.value.status == rmb.RMB_EINVAL


def test_large_system_multi_chunk_krylov(env):
    """3000 x 15-blob boomerangs (45,000 blobs, 153,000 unknowns): more
    unknowns than 256 Krylov workgroups of 512 elements cover, so each
    workgroup takes several chunks.  The oracle's FP64 residual of the GPU
    result meets the tolerance."""
    O = env[3]
    s = S.boomerangs_wall(n_bodies=3000, lateral=200.0 * np.sqrt(3.0))
    assert 3 * s.n_blobs + 6 * 3000 > 256 * 512
    print(f"[gpu] 3000 boomerangs fp32 ({s.n_blobs} blobs)", flush=True)
    U, lam, info = _solve(env, s, tol=1e-8, precision="fp32")
    res = O.relative_residual(s, s.FT, None, U, lam)
    print(f"    info {info}  oracle residual {res:.2e}", flush=True)
    assert info["status"] == 0
    assert res <= 1.05e-8


def test_precond_apply_parity(env):
    rmb, torch, ctx, O = env
    s = small_wall()
    rhs = np.random.default_rng(23).standard_normal((8, 3 * s.n_blobs + 6 * s.n_bodies))
    P = O.BlockPreconditioner(s)
    ref = np.stack([P.apply(r) for r in rhs])
    sysd = rmb.System.from_suspension(s)
    pc = rmb.Precond(ctx, sysd)
    got = pc.apply(_dev(torch, rhs)).cpu().numpy()
    err = _rel(got, ref)
    print(f"[gpu] precond apply 8 rhs rel err {err:.2e}", flush=True)
    assert err <= 1e-10
    # a solve that reuses the factors gives the same result as one that builds them
    FT = _dev(torch, s.FT)
    U1, l1, i1 = rmb.solve_mobility(ctx, sysd, FT, precond=pc, tol=1e-9)
    U2, l2, i2 = rmb.solve_mobility(ctx, sysd, FT, tol=1e-9)
    assert torch.equal(U1, U2) and torch.equal(l1, l2)
    pc.close()


def test_batch_results_equal_alone(env):
    rmb, torch, ctx, O = env
    sus = [S.boomerangs_wall(n_bodies=n, lateral=np.sqrt(40 * n), seed=500 + n) for n in (7, 60, 200)]
    sus.append(S.spheres_free_space())
    systems = [rmb.System.from_suspension(x) for x in sus]
    FTs = [_dev(torch, x.FT) for x in sus]
    for prec in ("fp64", "fp32"):
        alone = [rmb.solve_mobility(ctx, systems[i], FTs[i], tol=1e-9, precision=prec) for i in range(len(sus))]
        mixed = rmb.solve_batch(ctx, systems, FTs, tol=1e-9, precision=prec)
        for (Ua, la, ia), (Um, lm, im) in zip(alone, mixed):
            assert im["status"] == 0
            assert torch.equal(Ua, Um) and torch.equal(la, lm)
            assert ia["iterations"] == im["iterations"]


def test_server_results_equal_alone(env):
    rmb, torch, ctx, O = env
    reqs = [S.mixed_wall_request(i, n_bodies=n) for i, n in enumerate((12, 90, 33, 150, 5))]
    systems = [rmb.System.from_suspension(x) for x in reqs]
    FTs = [_dev(torch, x.FT) for x in reqs]
    alone = [rmb.solve_mobility(ctx, systems[i], FTs[i], tol=1e-8, precision="fp32") for i in range(len(reqs))]
    srv = rmb.Server(ctx, max_active=3)
    got = {}
    pending = list(range(len(reqs)))
    steps = 0
    while len(got) < len(reqs):
        if pending and steps % 3 == 0:  # requests arrive while others run
            i = pending.pop(0)
            srv.submit(i, systems[i], FTs[i], tol=1e-8, precision="fp32")
        srv.step()
        for tag, U, lam, info in srv.poll():
            got[tag] = (U, lam, info)
        steps += 1
        assert steps < 5000
    srv.close()
    for i, (Ua, la, ia) in enumerate(alone):
        Um, lm, im = got[i]
        assert im["status"] == 0
        assert torch.equal(Ua, Um) and torch.equal(la, lm)
        res = O.relative_residual(reqs[i], reqs[i].FT, None, Um.cpu().numpy(), lm.cpu().numpy())
        assert res <= 1.05e-8


def test_largest_small_bodies(env):
    """Bodies of 28 blobs (m = 84, the largest on the small-body path): the
    factor build and apply against the oracle's preconditioner, and a solve
    against the dense solution."""
    rmb, torch, ctx, O = env
    lattice = np.array([[x, y, z] for x in range(3) for y in range(3) for z in range(3)], float)
    shp = np.vstack([lattice, [[1.0, 1.0, 3.0]]])
    rng = np.random.default_rng(31)
    n = 6
    centres = np.column_stack([rng.uniform(0, 20, n), rng.uniform(0, 20, n), rng.uniform(4.0, 6.0, n)])
    quats = rng.standard_normal((n, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    pos, off = S.assemble([shp] * n, centres, quats)
    sus = S.Suspension(pos, off, centres, 0.4, 1.0, True)
    sus.FT = rng.standard_normal((n, 6))
    assert np.all(np.diff(off) == 28) and pos[:, 2].min() > 0.4
    sysd = rmb.System.from_suspension(sus)
    rhs = rng.standard_normal((3, 3 * sus.n_blobs + 6 * n))
    P = O.BlockPreconditioner(sus)
    ref = np.stack([P.apply(r) for r in rhs])
    pc = rmb.Precond(ctx, sysd)
    err = _rel(pc.apply(_dev(torch, rhs)).cpu().numpy(), ref)
    print(f"[gpu] 28-blob bodies: precond apply rel err {err:.2e}", flush=True)
    assert err <= 1e-10
    pc.close()
    Ud, _ = O.dense_solve(sus, sus.FT)
    U, lam, info = _solve(env, sus, tol=1e-10, precision="fp64")
    print(f"    solve {info}  U err {_rel(U, Ud):.2e}", flush=True)
    assert info["status"] == 0 and _rel(U, Ud) <= 1e-8


def test_solve_error_paths(env):
    rmb, torch, ctx, O = env
    # a layer of blobs overlapping the wall: the body's block is not SPD
    a = 0.5
    g = np.arange(5) * 0.6
    X, Y = np.meshgrid(g, g)
    pos = np.stack([X.ravel(), Y.ravel(), np.full(X.size, 0.3 * a)], axis=1)
    s = S.Suspension(pos, np.array([0, 25]), pos.mean(axis=0, keepdims=True), a, 1.0, True,
                     np.ones((1, 6)))
    with pytest.raises(rmb.RmbError) as e:
        _solve(env, s)
    assert e.value.status == rmb.RMB_ENOTSPD
    # iteration limit: status ENOCONV, residual reported
    s = small_wall()
    U, lam, info = _solve(env, s, tol=1e-12, max_iters=2)
    assert info["status"] == rmb.RMB_ENOCONV and 0 < info["rel_residual"] < 1
    res = O.relative_residual(s, s.FT, None, U, lam)
    assert abs(res - info["rel_residual"]) <= 1e-6 * res
    # a blob below the wall
    pos = s.pos.copy()
    pos[3, 2] = -0.1
    bad = S.Suspension(pos, s.body_off, s.q, s.a, 1.0, True, s.FT)
    with pytest.raises(rmb.RmbError) as e:
        _solve(env, bad)
    assert e.value.status == rmb.RMB_EINVAL
    # zero load: zero velocities without iterating
    U, lam, info = _solve(env, s, FT=np.zeros_like(s.FT))
    assert info["status"] == 0 and not U.any() and not lam.any()
