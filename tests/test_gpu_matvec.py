"""Parity of the HIP blob mobility product with the CPU FP64 oracle.

Bar: relative 2-norm error over the whole (Nb, 3) result, and the largest
error of any one blob relative to the rms blob velocity, both <= 1e-12 for
FP64 pairs and <= 1e-5 for FP32 pairs with FP64 accumulation.  Every block
size of the symmetric product (64, 128, 256 blobs), products taken in
several bands of tile rows, and the one-sided
kernel are covered.
"""
import numpy as np
import pytest

import parity
import suspensions as S

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def env(oracle_mod):
    import torch
    import paper_1602_02170_amd as rmb
    ctx = rmb.Context(0)
    yield rmb, torch, ctx, oracle_mod
    ctx.close()


def _run(env, sus, lam, prec):
    rmb, torch, ctx, _ = env
    sysd = rmb.System.from_suspension(sus) if sus.body_off is not None else None
    lt = torch.tensor(lam, dtype=torch.float64, device="cuda")
    v = rmb.mobility_matvec(ctx, sysd, lt, prec)
    torch.cuda.synchronize()
    return v.cpu().numpy()


_rel = parity.err  # 2-norm and per-row bound (tests/parity.py)


def _cases():
    out = []
    s1 = S.spheres_free_space()
    out.append(("free 8x12 icosahedra", s1, np.random.default_rng(11).standard_normal((96, 3))))
    s2 = S.boomerangs_wall(n_bodies=203, lateral=90.0)  # 3045 blobs: ragged last tile
    out.append(("wall 203 boomerangs", s2, np.random.default_rng(12).standard_normal((s2.n_blobs, 3))))
    s3, l3 = S.icosahedra_monolayer(n_bodies=1100)  # 13200 blobs
    out.append(("wall monolayer 1100 icosahedra", s3, l3))
    # 11655 blobs: 183 blocks of 64, the last one holding 7; and a
    # free-space system of 12000 blobs (both over 16,000 tiles)
    s4 = S.boomerangs_wall(n_bodies=777, lateral=np.sqrt(40 * 777), seed=21)
    out.append(("wall 777 boomerangs ragged", s4, np.random.default_rng(22).standard_normal((s4.n_blobs, 3))))
    s5 = S.boomerangs_wall(n_bodies=800, lateral=np.sqrt(40 * 800), seed=23)
    s5.wall = False
    out.append(("free 800 boomerangs", s5, np.random.default_rng(24).standard_normal((s5.n_blobs, 3))))
    return out


CASES = _cases()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_matvec_parity(env, case, prec):
    name, sus, lam = CASES[case]
    print(f"[gpu] matvec parity {name} {prec} nb={sus.n_blobs}", flush=True)
    ref = env[3].matvec(sus.pos, lam, sus.a, sus.eta, sus.wall)
    v = _run(env, sus, lam, prec)
    err = _rel(v, ref)
    print(f"    rel err {err:.3e}", flush=True)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_matvec_full_monolayer_sampled_rows(env, prec):
    """Full 16384 x 12 = 196,608-blob monolayer: sampled target rows against
    the oracle's per-row sums."""
    sus, lam = S.icosahedra_monolayer()
    print(f"[gpu] full monolayer {prec} nb={sus.n_blobs}", flush=True)
    v = _run(env, sus, lam, prec)
    rows = np.random.default_rng(13).choice(sus.n_blobs, 96, replace=False)
    rows = np.concatenate([rows, [0, sus.n_blobs - 1]])
    ref = env[3].matvec_rows(sus.pos, lam, rows, sus.a, sus.eta, sus.wall)
    err = _rel(v[rows], ref)
    print(f"    sampled rel err {err:.3e}", flush=True)
    assert err <= TOL[prec]
    assert np.all(np.isfinite(v))


_B128 = {}


def _b128_case(env):
    """4096 icosahedra of the monolayer (49,152 blobs): the symmetric product
    with 128-blob blocks (384 blocks); the oracle's full product is computed
    once for both precisions."""
    if not _B128:
        sus, lam = S.icosahedra_monolayer(n_bodies=4096)
        _B128["sus"], _B128["lam"] = sus, lam
        _B128["ref"] = env[3].matvec(sus.pos, lam, sus.a, sus.eta, sus.wall)
    return _B128["sus"], _B128["lam"], _B128["ref"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_matvec_block128_full_parity(env, prec):
    rmb = env[0]
    sus, lam, ref = _b128_case(env)
    assert rmb.pair_plan(sus.n_blobs) == (True, 128)
    print(f"[gpu] 128-blob blocks {prec} nb={sus.n_blobs}", flush=True)
    v = _run(env, sus, lam, prec)
    err = _rel(v, ref)
    print(f"    rel err {parity.rel2(v, ref):.3e}, worst blob {parity.rowmax(v, ref):.3e}", flush=True)
    assert err <= TOL[prec]


_MILLION = {}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_matvec_million_blobs_sampled_rows(env, prec):
    """A 289 x 289 monolayer lattice (83,521 icosahedra, 1,002,252 blobs) in
    the default 16 GiB budget: the symmetric product's partial sums (94 GB
    for FP64 pairs in one pass) are taken in bands of tile rows, so its
    workspace stays bounded; sampled rows (the first and last blob among
    them) against the oracle's per-row sums."""
    rmb = env[0]
    if not _MILLION:
        _MILLION["case"] = S.icosahedra_monolayer(n_side=289)
    sus, lam = _MILLION["case"]
    assert sus.n_blobs > 10 ** 6 and rmb.pair_plan(sus.n_blobs) == (True, 256)
    print(f"[gpu] million-blob product {prec} nb={sus.n_blobs}", flush=True)
    v = _run(env, sus, lam, prec)
    rows = np.random.default_rng(17).choice(sus.n_blobs, 126, replace=False)
    rows = np.concatenate([rows, [0, sus.n_blobs - 1]])
    ref = env[3].matvec_rows(sus.pos, lam, rows, sus.a, sus.eta, sus.wall)
    err = _rel(v[rows], ref)
    print(f"    sampled rel err {parity.rel2(v[rows], ref):.3e}, worst blob {parity.rowmax(v[rows], ref):.3e}",
          flush=True)
    assert err <= TOL[prec]
    assert np.all(np.isfinite(v))


@pytest.mark.parametrize("case", [0, 1, 3], ids=[CASES[c][0] for c in (0, 1, 3)])
def test_matvec_float32_data(env, case):
    """rmb_mobility_matvec_f32 (float32 forces in, float32 velocities out):
    bitwise the FP32-pair product of the forces widened to float64, rounded
    to float32 once; and the oracle's FP64 product of those forces within
    the FP32 bar.  One-sided (96 blobs) and symmetric sizes, the last with a
    ragged block."""
    rmb, torch, ctx, orc = env
    name, sus, lam = CASES[case]
    print(f"[gpu] float32 data {name} nb={sus.n_blobs}", flush=True)
    sysd = rmb.System.from_suspension(sus)
    l32 = torch.tensor(lam.astype(np.float32), device="cuda")
    v32 = rmb.mobility_matvec_f32(ctx, sysd, l32)
    v64 = rmb.mobility_matvec(ctx, sysd, l32.double(), "fp32")
    torch.cuda.synchronize()
    assert v32.dtype == torch.float32
    assert torch.equal(v32, v64.float())
    ref = orc.matvec(sus.pos, lam.astype(np.float32).astype(np.float64), sus.a, sus.eta, sus.wall)
    err = _rel(v32.cpu().numpy().astype(np.float64), ref)
    print(f"    rel err {err:.3e}", flush=True)
    assert err <= TOL["fp32"]
    with pytest.raises(TypeError):
        rmb.mobility_matvec_f32(ctx, sysd, l32.double())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("wall", [True, False], ids=["wall", "free"])
@pytest.mark.parametrize("a", [0.002, 30.0])
def test_matvec_extreme_blob_radius(env, a, wall, prec):
    """The kernels take lengths in units of the blob radius.  The 203
    boomerangs, over the wall and in free space, with a = 0.002 (positions
    up to ~1e5 radii, every pair far apart) and a = 30 (nearly every pair
    overlapping, the contact branch throughout; heights lifted above a):
    the oracle's product within the bar of each precision, symmetric (3045
    blobs) and one-sided (the first 60 bodies, 900 blobs) paths."""
    import copy
    rmb, torch, ctx, orc = env
    base = CASES[1][1]
    sus = copy.deepcopy(base)
    sus.a = a
    sus.wall = wall
    if a > 1.0:
        sus.pos = sus.pos.copy()
        sus.pos[:, 2] += a
    lam = np.random.default_rng(31).standard_normal((sus.n_blobs, 3))
    for nb_bodies in (sus.n_bodies, 60):
        part = copy.deepcopy(sus)
        if nb_bodies < sus.n_bodies:
            nbl = int(sus.body_off[nb_bodies])
            part.pos = sus.pos[:nbl].copy()
            part.body_off = sus.body_off[:nb_bodies + 1].copy()
            part.q = sus.q[:nb_bodies].copy()
            part.FT = None if sus.FT is None else sus.FT[:nb_bodies].copy()
            part.quat = None if getattr(sus, "quat", None) is None else sus.quat[:nb_bodies].copy()
        l = lam[:part.n_blobs]
        print(f"[gpu] extreme radius a={a} {prec} nb={part.n_blobs}", flush=True)
        ref = orc.matvec(part.pos, l, part.a, part.eta, part.wall)
        v = _run(env, part, l, prec)
        err = _rel(v, ref)
        print(f"    rel err {err:.3e}", flush=True)
        assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_matvec_edge_cases(env, prec):
    rmb, torch, ctx, O = env
    a = 0.5
    # one blob: the self block alone, above the wall
    for pos, wall in [(np.array([[0.3, -0.2, 1.7]]), True), (np.array([[0.0, 0.0, 0.0]]), False)]:
        sus = S.Suspension(pos, np.array([0, 1]), pos.copy(), a, 1.0, wall)
        lam = np.array([[1.0, -2.0, 0.5]])
        v = _run(env, sus, lam, prec)
        ref = O.matvec(pos, lam, a, 1.0, wall)
        assert _rel(v, ref) <= TOL[prec]
    # coincident blobs, a pair exactly at 2a, overlapping pairs, and 65 blobs
    # (one full wave plus a ragged lane)
    rng = np.random.default_rng(14)
    pos = rng.uniform(0, 2.0, (65, 3))
    pos[:, 2] += 0.6
    pos[1] = pos[0]
    pos[2] = pos[0] + np.array([2 * a, 0, 0])
    sus = S.Suspension(pos, np.array([0, 65]), pos[:1].copy(), a, 1.0, True)
    lam = rng.standard_normal((65, 3))
    for wall in (True, False):
        sus.wall = wall
        v = _run(env, sus, lam, prec)
        ref = O.matvec(pos, lam, a, 1.0, wall)
        assert _rel(v, ref) <= TOL[prec]


def test_matvec_deterministic_and_permutation_covariant(env):
    rmb, torch, ctx, O = env
    sus = S.boomerangs_wall(n_bodies=150, lateral=70.0)
    lam = np.random.default_rng(15).standard_normal((sus.n_blobs, 3))
    for prec in ("fp64", "fp32"):
        v1 = _run(env, sus, lam, prec)
        v2 = _run(env, sus, lam, prec)
        assert np.array_equal(v1, v2)
        perm = np.random.default_rng(16).permutation(sus.n_blobs)
        sp = S.Suspension(sus.pos[perm], np.array([0, sus.n_blobs]), sus.q[:1], sus.a, 1.0, True)
        vp = _run(env, sp, lam[perm], prec)
        assert _rel(vp, v1[perm]) <= TOL[prec]


def test_matvec_rejects_bad_input(env):
    rmb, torch, ctx, O = env
    pos = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, -0.1]])
    lam = np.ones((2, 3))
    sus = S.Suspension(pos, np.array([0, 2]), pos[:1].copy(), 0.3, 1.0, True)
    with pytest.raises(rmb.RmbError) as e:
        _run(env, sus, lam, "fp64")
    assert e.value.status == rmb.RMB_EINVAL and "z <= 0" in str(e.value)
    pos[1, 2] = np.nan
    sus.wall = False
    with pytest.raises(rmb.RmbError) as e:
        _run(env, sus, lam, "fp64")
    assert e.value.status == rmb.RMB_EINVAL
    sus = S.Suspension(np.array([[0.0, 0, 1]]), np.array([0, 1]), np.zeros((1, 3)), -1.0, 1.0, False)
    with pytest.raises(rmb.RmbError) as e:
        _run(env, sus, np.ones((1, 3)), "fp64")
    assert e.value.status == rmb.RMB_EINVAL
