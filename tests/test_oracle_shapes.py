"""Pins of the oracle's shared reference-shape preconditioner (Sec. 2.2.2,
after eq:saddle_M_precon; Sec. 5.4).

In free space the RPY tensor and the rigid kinematics are rotation- and
translation-covariant, so for bodies placed exactly at q_p + R_p ref the
shared preconditioner must equal the per-body one (which the other pins tie
to the paper's definitions) to rounding.  That check fails for a transposed
rotation, a wrong quaternion order or a forgotten torque rotation.  In wall
geometry the shared blocks are only an approximation: GMRES must still reach
the exact (dense) solution, with at most 50% more iterations than with the
wall-corrected blocks, as the paper reports for rods near a wall.
"""
import numpy as np
import pytest

import suspensions as S


def _shapes_of(sus):
    """Reference shapes (centred) and the shape index of every body of a
    generated suspension: 12 blobs -> icosahedron, 15 -> boomerang."""
    ico = S.icosahedron(1.0)
    boo = S.boomerang()
    shapes = [ico - ico.mean(0), boo - boo.mean(0)]
    nb = np.diff(sus.body_off)
    idx = np.where(nb == 12, 0, 1)
    assert set(nb.tolist()) <= {12, 15}
    return shapes, idx


def _vec(sus, seed):
    return np.random.default_rng(seed).standard_normal(3 * sus.n_blobs + 6 * sus.n_bodies)


@pytest.mark.parametrize("which", ["boomerangs", "mixed"])
def test_shared_equals_per_body_in_free_space(oracle_mod, which):
    O = oracle_mod
    sus = S.boomerangs_wall(n_bodies=30, lateral=35.0) if which == "boomerangs" else \
        S.mixed_wall_request(3, n_bodies=30)
    sus.wall = False
    shapes, idx = _shapes_of(sus)
    P = O.BlockPreconditioner(sus)
    Q = O.ShapePreconditioner(sus, shapes, idx, sus.quat)
    for seed in (1, 2):
        v = _vec(sus, seed)
        a, b = P.apply(v), Q.apply(v)
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)
    # quaternions are normalised: a scaled copy gives the same operator
    Q2 = O.ShapePreconditioner(sus, shapes, idx, -2.5 * sus.quat)
    v = _vec(sus, 3)
    assert np.linalg.norm(Q2.apply(v) - Q.apply(v)) <= 1e-13 * np.linalg.norm(Q.apply(v))


def test_rotation_mistakes_are_caught(oracle_mod):
    O = oracle_mod
    sus = S.boomerangs_wall(n_bodies=10, lateral=20.0)
    sus.wall = False
    shapes, idx = _shapes_of(sus)
    v = _vec(sus, 4)
    ref = O.BlockPreconditioner(sus).apply(v)
    bad = O.ShapePreconditioner(sus, shapes, idx, sus.quat)
    bad.R = bad.R.transpose(0, 2, 1)
    assert np.linalg.norm(bad.apply(v) - ref) > 1e-2 * np.linalg.norm(ref)
    # quaternion read as (x, y, z, w) instead of (w, x, y, z)
    bad = O.ShapePreconditioner(sus, shapes, idx, sus.quat[:, [1, 2, 3, 0]])
    assert np.linalg.norm(bad.apply(v) - ref) > 1e-2 * np.linalg.norm(ref)


def test_unbounded_blocks_for_a_wall_problem(oracle_mod):
    O = oracle_mod
    sus = S.boomerangs_wall(n_bodies=40, lateral=40.0)
    shapes, idx = _shapes_of(sus)
    Q = O.ShapePreconditioner(sus, shapes, idx, sus.quat)
    v = _vec(sus, 5)
    # an approximation here: the wall changes every block
    assert np.linalg.norm(Q.apply(v) - O.BlockPreconditioner(sus).apply(v)) > 1e-3 * np.linalg.norm(v)
    U0, l0 = O.dense_solve(sus, sus.FT)
    U1, l1, i1 = O.solve_mobility(sus, sus.FT, tol=1e-10)
    U2, l2, i2 = O.solve_mobility(sus, sus.FT, tol=1e-10, precond=Q)
    assert np.abs(U2 - U0).max() <= 1e-8 * np.abs(U0).max()
    assert O.relative_residual(sus, sus.FT, None, U2, l2) <= 1e-10
    assert i1["iterations"] <= i2["iterations"] <= 1.5 * i1["iterations"]
