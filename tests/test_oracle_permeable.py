"""Pins of the oracle's permeable bodies (appendix on permeable bodies,
eq:permeable_slip): blob i of body p carries the slip -d_i lambda_i with
d_i = kappa_p / (eta dV_i), so M gains d_i on its diagonal.

- The permeable solution solves the rigid problem with the slip of
  eq:permeable_slip evaluated at its own lambda (sign and placement of d).
- Free-draining limit, from the Neumann series of (M + d I)^-1: the body
  mobility is d (K^T K)^-1 + (K^T K)^-1 K^T M K (K^T K)^-1 + O(1/d), so the
  two-term form is off by a relative O(1/d^2) and the one-term form by
  O(1/d).  A shift scaled or placed wrongly breaks either rate.
- The system is no longer a saddle point for d > 0: GMRES needs no more
  iterations than for rigid bodies, and reaches the dense solution.
"""
import numpy as np

import suspensions as S


def test_permeable_solution_is_the_rigid_one_with_its_own_slip(oracle_mod):
    O = oracle_mod
    sus = S.boomerangs_wall(n_bodies=10, lateral=15.0)
    d = np.random.default_rng(3).uniform(0.1, 2.0, sus.n_blobs)
    sus.blob_shift = d
    U1, l1 = O.dense_solve(sus, sus.FT)
    sus.blob_shift = None
    U2, l2 = O.dense_solve(sus, sus.FT, slip=-d[:, None] * l1)
    assert np.abs(U1 - U2).max() <= 1e-12 * np.abs(U1).max()
    assert np.abs(l1 - l2).max() <= 1e-12 * np.abs(l1).max()
    # and it differs from the rigid answer
    U0, _ = O.dense_solve(sus, sus.FT)
    assert np.abs(U1 - U0).max() > 1e-2 * np.abs(U0).max()


def test_free_draining_limit(oracle_mod):
    O = oracle_mod
    sus = S.spheres_free_space(n_bodies=3)
    K = O.K_dense(sus.pos, sus.body_off, sus.q)
    M = O.assemble(sus.pos, sus.a, sus.eta, sus.wall)
    iK = np.linalg.inv(K.T @ K)
    e1, e2 = [], []
    for d in (1e2, 1e3):
        sus.blob_shift = np.full(sus.n_blobs, d)
        N = O.body_mobility(sus)
        e1.append(np.abs(N - d * iK).max() / np.abs(N).max())
        e2.append(np.abs(N - d * iK - iK @ K.T @ M @ K @ iK).max() / np.abs(N).max())
    assert 5 < e1[0] / e1[1] < 20        # O(1/d)
    assert 50 < e2[0] / e2[1] < 200      # O(1/d^2)
    assert e2[1] < 1e-8


def test_gmres_with_permeable_bodies(oracle_mod):
    O = oracle_mod
    sus = S.boomerangs_wall(n_bodies=10, lateral=15.0)
    _, _, rigid = O.solve_mobility(sus, sus.FT, tol=1e-12)
    sus.blob_shift = np.random.default_rng(4).uniform(0.1, 2.0, sus.n_blobs)
    Ud, ld = O.dense_solve(sus, sus.FT)
    U, lam, info = O.solve_mobility(sus, sus.FT, tol=1e-12)
    assert np.abs(U - Ud).max() <= 1e-10 * np.abs(Ud).max()
    assert O.relative_residual(sus, sus.FT, None, U, lam) <= 1e-12
    assert info["iterations"] <= rigid["iterations"]
