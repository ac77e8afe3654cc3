"""Pins of the oracle's flow field (appendix on computing flow fields).

The field of one blob split into tracer blobs is checked against a closed
form that does not use the oracle's pair blocks: averaging the Oseen tensor
O over a sphere of radius a gives (1 + a^2/6 lap) O exactly (O is
biharmonic), and the tracer-to-tracer RPY far field is (1 + (2 a'^2)/6 lap) O,
so far from the blob the field is [O + (a^2 + 2 a'^2)/6 lap O] F with
lap O = 2 (I - 3 e e^T) / (8 pi eta r^3).  The 12 icosahedron vertices form
a spherical 5-design, so the discrete average matches the sphere average up
to terms of relative order (a/r)^6.  A second check: with one sub-blob at
zero offset and the tracer radius equal to a, the field at the blob
positions is the mobility product itself.
"""
import numpy as np

import suspensions as S


def _stokeslet_faxen(r_vec, F, a2_eff, eta=1.0):
    r = np.linalg.norm(r_vec)
    e = r_vec / r
    I = np.eye(3)
    O = (I + np.outer(e, e)) / (8 * np.pi * eta * r)
    lapO = 2.0 * (I - 3.0 * np.outer(e, e)) / (8 * np.pi * eta * r ** 3)
    return (O + a2_eff / 6.0 * lapO) @ F


def test_single_blob_far_field_closed_form(oracle_mod):
    O = oracle_mod
    a, at = 0.5, 0.05
    u = S.icosahedron()
    u = u / np.linalg.norm(u, axis=1, keepdims=True)
    F = np.array([0.3, -1.1, 0.7])
    rng = np.random.default_rng(5)
    errs = []
    for dist in (6.0, 12.0):
        d = rng.standard_normal((4, 3))
        d *= dist * a / np.linalg.norm(d, axis=1, keepdims=True)
        v = O.flow_field(np.zeros((1, 3)), F[None, :], a, u, at, d)
        ref = np.array([_stokeslet_faxen(x, F, a * a + 2 * at * at) for x in d])
        errs.append(np.abs(v - ref).max() / np.abs(ref).max())
    # relative error O((a/r)^6): ~2e-5 at 6a, ~3e-7 at 12a
    assert errs[0] < 1e-4, errs
    assert errs[1] < 2e-6, errs
    assert errs[1] < errs[0] / 10, errs


def test_trivial_split_is_the_mobility_product(oracle_mod):
    O = oracle_mod
    sus = S.boomerangs_wall(n_bodies=6, lateral=12.0)
    lam = np.random.default_rng(3).standard_normal((sus.n_blobs, 3))
    v = O.flow_field(sus.pos, lam, sus.a, np.zeros((1, 3)), sus.a, sus.pos, sus.eta, sus.wall)
    ref = O.matvec(sus.pos, lam, sus.a, sus.eta, sus.wall)
    assert np.abs(v - ref).max() <= 1e-14 * np.abs(ref).max()
