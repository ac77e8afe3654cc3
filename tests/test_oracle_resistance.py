"""Pins of the oracle's resistance problem (eq:resistance_problem):
M lambda = K U + slip, F = K^T lambda.

- Duality with the mobility problem (eq:saddle_M): the velocities that the
  mobility solve returns for (F, slip) give back F through the resistance
  problem, with the same lambda (free space and wall).
- Table 1 (left): a shell translated with velocity U feels the force
  6 pi eta R_h U, and rotated with Omega the torque 8 pi eta R_tau^3 Omega,
  with the printed radii (4 decimals).
- GMRES with the blocks M_pp^-1 reaches the dense answer, and its iteration
  count grows with the size of a lattice of spheres much faster than the
  mobility solve's (Sec. 4.4).
"""
import os

import numpy as np
import pytest

import suspensions as S

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("wall", [False, True])
def test_duality_with_the_mobility_problem(oracle_mod, wall):
    O = oracle_mod
    sus = S.boomerangs_wall(n_bodies=12, lateral=18.0)
    sus.wall = wall
    slip = 0.1 * np.random.default_rng(1).standard_normal((sus.n_blobs, 3))
    U, lam = O.dense_solve(sus, sus.FT, slip)
    F, lam2 = O.resistance_dense(sus, U, slip)
    assert np.abs(F - sus.FT).max() <= 1e-12 * np.abs(sus.FT).max()
    assert np.abs(lam - lam2).max() <= 1e-12 * np.abs(lam).max()


def _table1():
    rows = [l.split() for l in open(os.path.join(GOLD, "table1_effective_radii.txt"))
            if l.strip() and not l.startswith("#")]
    return [(int(r[0]), float(r[1]), float(r[2]), float(r[3])) for r in rows]


@pytest.mark.parametrize("n_blobs,ratio,Rh,Rt", [r for r in _table1() if r[0] <= 162])
def test_table1_radii_from_the_resistance_problem(oracle_mod, n_blobs, ratio, Rh, Rt):
    O = oracle_mod
    shp = S.sphere_shell(n_blobs)
    sus = S.Suspension(shp.copy(), np.array([0, n_blobs]), np.zeros((1, 3)), ratio * S.min_spacing(shp), 1.0,
                       False)
    U = np.array([[1.0, 0, 0, 0, 0, 0]])
    F, _ = O.resistance_dense(sus, U)
    assert abs(F[0, 0] / (6 * np.pi) - Rh) <= 6e-5
    W = np.array([[0, 0, 0, 0, 0, 1.0]])
    F, _ = O.resistance_dense(sus, W)
    assert abs((F[0, 5] / (8 * np.pi)) ** (1 / 3) - Rt) <= 6e-5


def test_gmres_resistance_and_iteration_growth(oracle_mod):
    O = oracle_mod
    sus = S.boomerangs_wall(n_bodies=12, lateral=18.0)
    U = np.random.default_rng(2).standard_normal((sus.n_bodies, 6))
    Fd, ld = O.resistance_dense(sus, U)
    F, lam, info = O.solve_resistance(sus, U, tol=1e-12)
    assert np.abs(F - Fd).max() <= 1e-9 * np.abs(Fd).max()
    # lattices of 42-blob shells (2x2x2 and 3x3x3, spacing 2.6 radii)
    shp = S.sphere_shell(42)
    a = 0.5 * S.min_spacing(shp)
    its = {}
    for nside in (2, 3):
        c = 2.6 * np.array([[i, j, k] for i in range(nside) for j in range(nside) for k in range(nside)], float)
        pos, off = S.assemble([shp] * len(c), c, np.tile([1.0, 0, 0, 0], (len(c), 1)))
        s = S.Suspension(pos, off, c, a, 1.0, False)
        _, _, ir = O.solve_resistance(s, np.random.default_rng(3).standard_normal((len(c), 6)), tol=1e-8)
        _, _, im = O.solve_mobility(s, np.random.default_rng(4).standard_normal((len(c), 6)), tol=1e-8)
        its[nside] = (ir["iterations"], im["iterations"])
    grow_r = its[3][0] / its[2][0]
    grow_m = its[3][1] / its[2][1]
    assert its[2][0] > its[2][1] and its[3][0] > its[3][1]
    assert grow_r > grow_m + 0.2, its
