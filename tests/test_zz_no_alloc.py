"""The no-allocation product entry point (rmb_mobility_matvec_noalloc)
against rmb_mobility_matvec and the oracle.

Two calls in a row through the C ABI, the second on a smaller system, so
that the shared static workspace is reused with a different layout: a
49,152-blob monolayer (the symmetric product in several bands of tile rows
within the 128 MiB workspace) then a 3,045-blob suspension (one band), plus
the one-sided kernel (96 blobs), the asynchronous form without validation,
and the refusal of a system too large for the workspace.  Bar: 1e-12 (FP64
pairs) and 1e-5 (FP32 pairs) relative, also per blob, against the allocating
entry point and, for the large system, against the oracle.
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


def _pair(env, sus, lam, prec, validate=True):
    rmb, torch, ctx, _ = env
    sysd = rmb.System.from_suspension(sus)
    lt = torch.tensor(lam, dtype=torch.float64, device="cuda")
    ref = rmb.mobility_matvec(ctx, sysd, lt, prec)
    out = torch.full((sus.n_blobs, 3), float("nan"), dtype=torch.float64, device="cuda")
    rmb.mobility_matvec_noalloc(ctx, sysd, lt, out, prec, validate=validate)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_the_allocating_product(env, prec):
    rmb, torch, ctx, O = env
    big, lam_big = S.icosahedra_monolayer(n_bodies=4096)
    small = S.boomerangs_wall(n_bodies=203, lateral=90.0)
    lam_small = np.random.default_rng(12).standard_normal((small.n_blobs, 3))
    print(f"[gpu] no-alloc {prec}: {big.n_blobs} then {small.n_blobs} blobs", flush=True)
    v, ref = _pair(env, big, lam_big, prec)
    orc = O.matvec(big.pos, lam_big, big.a, big.eta, big.wall)
    print(f"    large: vs matvec {parity.err(v, ref):.2e}, vs oracle {parity.err(v, orc):.2e}", flush=True)
    assert parity.err(v, ref) <= TOL[prec] and parity.err(v, orc) <= TOL[prec]
    v, ref = _pair(env, small, lam_small, prec)
    print(f"    small: vs matvec {parity.err(v, ref):.2e}", flush=True)
    assert parity.err(v, ref) <= TOL[prec]
    # one band: the same sums as the allocating entry point, bit for bit
    assert np.array_equal(v, ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_one_sided_and_unvalidated(env, prec):
    s1 = S.spheres_free_space()
    lam = np.random.default_rng(11).standard_normal((s1.n_blobs, 3))
    v, ref = _pair(env, s1, lam, prec)
    assert parity.err(v, ref) <= TOL[prec]
    s2 = S.boomerangs_wall(n_bodies=150, lateral=70.0)
    lam2 = np.random.default_rng(15).standard_normal((s2.n_blobs, 3))
    v, ref = _pair(env, s2, lam2, prec, validate=False)
    assert np.array_equal(v, ref)


def test_noalloc_refusals(env):
    rmb, torch, ctx, O = env
    assert rmb.noalloc_workspace_bytes() == 128 << 20
    # a system too large for the workspace is refused before any GPU work
    n = 3_000_000
    pos = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    pos[:, 2] = 1.0
    sysd = rmb.System(pos, 0.5, wall=True)
    lam = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    out = torch.empty_like(lam)
    with pytest.raises(rmb.RmbError) as e:
        rmb.mobility_matvec_noalloc(ctx, sysd, lam, out)
    assert e.value.status == rmb.RMB_EINVAL and "workspace" in str(e.value)
    # validation still reports bad positions
    p = torch.tensor([[0.0, 0.0, 1.0], [1.0, 0.0, -0.1]], dtype=torch.float64, device="cuda")
    sysd = rmb.System(p, 0.3, wall=True)
    l2 = torch.ones((2, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(rmb.RmbError) as e:
        rmb.mobility_matvec_noalloc(ctx, sysd, l2, torch.empty_like(l2))
    assert e.value.status == rmb.RMB_EINVAL and "z <= 0" in str(e.value)
