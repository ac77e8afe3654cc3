"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: each compares the oracle with an
independent route (a symbolic derivation from the Green's function, a Monte
Carlo surface average, the paper's printed tables, closed-form limits, or
structural invariants).
"""
import os

import numpy as np
import pytest

import suspensions as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rng(k=0):
    return np.random.default_rng(1234 + k)


# ---------------------------------------------------------------------------
# free-space RPY (eq:RPYTensor)
# ---------------------------------------------------------------------------

def test_rpy_far_branch_is_double_faxen_of_oseen(oracle_mod):
    """For r > 2a the RPY block is the Faxen operator applied on both sides of
    the Oseen tensor (eq:MobilityFaxen with eq:OseenTensor)."""
    import sympy as sp
    x = sp.symbols("x1 x2 x3", real=True)
    a = sp.symbols("a", positive=True)
    X = sp.Matrix(x)
    r = sp.sqrt(X.dot(X))
    G = (sp.eye(3) / r + X * X.T / r ** 3) / (8 * sp.pi)
    lap = lambda M: M.applyfunc(lambda e: sum(sp.diff(e, v, 2) for v in x))
    # the Faxen operators in r' and r'' act on G(r' - r''): each Laplacian is
    # the same second derivative in the difference variable
    G1 = G + a ** 2 / 6 * lap(G)
    M = G1 + a ** 2 / 6 * lap(G1)
    f = sp.lambdify((*x, a), M, "numpy")
    rng = _rng(1)
    for _ in range(20):
        aa = rng.uniform(0.1, 1.0)
        d = rng.standard_normal(3)
        d *= rng.uniform(2.05 * aa, 20 * aa) / np.linalg.norm(d)
        ri = rng.uniform(-5, 5, 3)
        ref = np.array(f(*d, aa), dtype=float)  # eta = 1
        got = oracle_mod.pair_block(ri, ri - d, aa, 1.0, wall=False)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_rpy_is_surface_average_of_oseen_including_overlap(oracle_mod):
    """The RPY tensor (both branches) equals the Oseen tensor averaged over
    the surfaces of the two blob spheres, the integral form that extends it to
    overlapping blobs.  Monte Carlo over sphere surfaces."""
    rng = _rng(2)
    a = 0.7
    n = 1_500_000
    for dist in (0.35 * a, 1.0 * a, 1.6 * a, 2.5 * a):
        u = rng.standard_normal((n, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        v = rng.standard_normal((n, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        d = np.array([dist, 0.0, 0.0]) + a * (u - v)
        rr = np.linalg.norm(d, axis=1)
        iso = np.mean(1.0 / rr) / (8 * np.pi)
        xx = np.mean(d[:, 0] ** 2 / rr ** 3) / (8 * np.pi)
        yy = np.mean(d[:, 1] ** 2 / rr ** 3) / (8 * np.pi)
        mc = np.array([iso + xx, iso + yy])  # parallel and transverse
        got = oracle_mod.pair_block([dist, 0, 0], [0, 0, 0], a, 1.0, wall=False)
        ref = np.array([got[0, 0], got[1, 1]])
        assert np.allclose(mc, ref, rtol=6e-3), (dist, mc, ref)


def test_rpy_self_continuity_and_far_field(oracle_mod):
    a, eta = 0.4, 1.3
    mu0 = 1.0 / (6 * np.pi * eta * a)
    r0 = np.array([1.0, -2.0, 0.5])
    assert np.allclose(oracle_mod.pair_block(r0, r0, a, eta), mu0 * np.eye(3), rtol=0, atol=1e-15)
    e = np.array([0.36, 0.48, 0.8])
    lo = oracle_mod.pair_block(r0 + (2 * a - 1e-12) * e, r0, a, eta)
    hi = oracle_mod.pair_block(r0 + (2 * a + 1e-12) * e, r0, a, eta)
    assert np.abs(lo - hi).max() < 1e-10 * mu0
    # far field: the Oseen tensor 1/(8 pi eta r) (I + e e^T)
    r = 1e4
    far = oracle_mod.pair_block(r0 + r * e, r0, a, eta)
    oseen = (np.eye(3) + np.outer(e, e)) / (8 * np.pi * eta * r)
    assert np.abs(far - oseen).max() < 1e-7 * np.abs(oseen).max()


# ---------------------------------------------------------------------------
# wall-corrected RPY
# ---------------------------------------------------------------------------

def _blake_symbolic():
    """Blake's Green's function of a point force above a no-slip plane z = 0
    (Stokeslet, image Stokeslet, source dipole and Stokeslet doublet images),
    unit viscosity, as a sympy matrix in target x and source y."""
    import sympy as sp
    xs = sp.symbols("x1 x2 x3", real=True)
    ys = sp.symbols("y1 y2 y3", real=True)
    X, Y = sp.Matrix(xs), sp.Matrix(ys)

    def oseen(rv):
        rn = sp.sqrt(rv.dot(rv))
        return (sp.eye(3) / rn + rv * rv.T / rn ** 3) / (8 * sp.pi)

    h = ys[2]
    R = X - sp.Matrix([ys[0], ys[1], -ys[2]])
    Rs = sp.symbols("R1 R2 R3", real=True)
    Rv = sp.Matrix(Rs)
    Rl = sp.sqrt(Rv.dot(Rv))
    inner = [h * Rv[i] / Rl ** 3 - ((1 if i == 2 else 0) / Rl + Rv[i] * Rv[2] / Rl ** 3)
             for i in range(3)]
    refl = [1, 1, -1]
    D = sp.zeros(3, 3)
    for i in range(3):
        for j in range(3):
            D[i, j] = 2 * h * refl[j] * sp.diff(inner[i], Rs[j]) / (8 * sp.pi)
    D = D.subs({Rs[0]: R[0], Rs[1]: R[1], Rs[2]: R[2]})
    GB = oseen(X - Y) - oseen(R) + D
    return sp, xs, ys, GB, oseen(X - Y)


@pytest.fixture(scope="module")
def blake():
    return _blake_symbolic()


def test_blake_image_system_invariants(blake):
    """The image system used for the wall correction is the half-space Stokes
    Green's function: zero velocity on z = 0, divergence free, reciprocal."""
    sp, xs, ys, GB, _ = blake
    f = sp.lambdify((*xs, *ys), GB, "numpy")
    div = sp.Matrix([sum(sp.diff(GB[i, j], xs[i]) for i in range(3)) for j in range(3)])
    fd = sp.lambdify((*xs, *ys), div, "numpy")
    rng = _rng(3)
    for _ in range(10):
        y = np.array([*rng.uniform(-2, 2, 2), rng.uniform(0.3, 3)])
        xw = np.array([*rng.uniform(-2, 2, 2), 0.0])
        assert np.abs(np.array(f(*xw, *y), dtype=float)).max() < 1e-15
        x = np.array([*rng.uniform(-2, 2, 2), rng.uniform(0.3, 3)])
        gxy = np.array(f(*x, *y), dtype=float)
        gyx = np.array(f(*y, *x), dtype=float)
        assert np.abs(gxy - gyx.T).max() < 1e-14
        assert np.abs(np.array(fd(*x, *y), dtype=float)).max() < 1e-14


@pytest.mark.slow
def test_wall_correction_is_double_faxen_of_blake_image(oracle_mod, blake):
    """The oracle's wall correction equals the Faxen operators in target and
    source applied to the image part of Blake's Green's function."""
    sp, xs, ys, GB, G0 = blake
    a = sp.symbols("a", positive=True)
    Wim = GB - G0
    lapx = lambda M: M.applyfunc(lambda e: sum(sp.diff(e, v, 2) for v in xs))
    lapy = lambda M: M.applyfunc(lambda e: sum(sp.diff(e, v, 2) for v in ys))
    A1 = Wim + a ** 2 / 6 * lapx(Wim)
    W = A1 + a ** 2 / 6 * lapy(A1)
    f = sp.lambdify((*xs, *ys, a), W, "numpy")
    rng = _rng(4)
    for _ in range(12):
        aa = rng.uniform(0.1, 0.6)
        xi = np.array([*rng.uniform(-3, 3, 2), rng.uniform(aa, 4)])
        xj = np.array([*rng.uniform(-3, 3, 2), rng.uniform(aa, 4)])
        if rng.uniform() < 0.25:
            xj = xi.copy()  # self block
        ref = np.array(f(*xi, *xj, aa), dtype=float)  # eta = 1
        got = oracle_mod.wall_block(xi, xj, aa, 1.0)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), (xi, xj)


def test_wall_self_mobility_leading_orders(oracle_mod):
    """Self block above the wall, expanded in a/h: the parallel correction
    starts at -9/16 a/h (the leading coefficient the Appendix D fit imposes on
    the parallel translational mobility) and the perpendicular one at
    -9/8 a/h (Lorentz)."""
    a = 0.3
    for h in (300.0, 3000.0):
        r = np.array([0.0, 0.0, h])
        W = oracle_mod.wall_block(r, r, a, 1.0) * (6 * np.pi * a)
        eps = a / h
        assert abs(W[0, 0] / eps + 9 / 16) < 2 * eps ** 2
        assert abs(W[1, 1] / eps + 9 / 16) < 2 * eps ** 2
        assert abs(W[2, 2] / eps + 9 / 8) < 2 * eps ** 2
        assert abs(W[0, 1]) + abs(W[0, 2]) + abs(W[1, 2]) < 1e-15


def test_wall_correction_decays_with_height(oracle_mod):
    """Far from the wall the wall-corrected tensor tends to free-space RPY:
    the image flow of a source at height H is that of a Stokeslet at distance
    about 2H, so the relative correction for a pair at separation d falls off
    like d/H."""
    a = 0.4
    d = np.array([1.1, -0.6, 0.3])
    prev = None
    for H in (5.0, 50.0, 500.0):
        ri = np.array([0.0, 0.0, H]) + d
        rj = np.array([0.0, 0.0, H])
        Mw = oracle_mod.pair_block(ri, rj, a, 1.0, wall=True)
        Mf = oracle_mod.pair_block(ri, rj, a, 1.0, wall=False)
        rel = np.abs(Mw - Mf).max() / np.abs(Mf).max()
        assert rel < 1.5 * np.linalg.norm(d) / H
        if prev is not None:
            assert 8.0 < prev / rel < 12.0
        prev = rel


def test_mobility_matrix_symmetric_and_spd(oracle_mod):
    """M is symmetric and positive definite in free space (overlapping blobs
    included) and above the wall when every blob has z >= a."""
    rng = _rng(5)
    a = 0.5
    pos = rng.uniform(0, 3, (40, 3))
    M = oracle_mod.assemble(pos, a, 1.0, wall=False)
    assert np.abs(M - M.T).max() < 1e-15
    assert np.linalg.eigvalsh(M).min() > 0
    pos[:, 2] += a
    M = oracle_mod.assemble(pos, a, 1.0, wall=True)
    assert np.abs(M - M.T).max() < 1e-15
    assert np.linalg.eigvalsh(M).min() > 0


def test_wall_overlap_loses_positive_definiteness(oracle_mod):
    """The wall correction is not guaranteed SPD when blobs overlap the wall
    (Sec. 2.1.1, Conclusions): a dense layer of blobs at z = 0.3 a."""
    a = 0.5
    g = np.arange(5) * 0.6
    X, Y = np.meshgrid(g, g)
    pos = np.stack([X.ravel(), Y.ravel(), np.full(X.size, 0.3 * a)], axis=1)
    M = oracle_mod.assemble(pos, a, 1.0, wall=True)
    assert np.linalg.eigvalsh(M).min() < 0


def test_matvec_equals_dense_assembly_and_rows(oracle_mod):
    s, lam = S.icosahedra_monolayer(n_side=4, n_bodies=7)
    v = oracle_mod.matvec(s.pos, lam, s.a, 1.0, True)
    M = oracle_mod.assemble(s.pos, s.a, 1.0, True)
    ref = (M @ lam.ravel()).reshape(-1, 3)
    assert np.abs(v - ref).max() < 1e-13 * np.abs(ref).max()
    rows = np.array([0, 5, 17, 40])
    assert np.array_equal(oracle_mod.matvec_rows(s.pos, lam, rows, s.a, 1.0, True), v[rows])


# ---------------------------------------------------------------------------
# kinematics and body-level solves
# ---------------------------------------------------------------------------

def test_K_transpose_is_adjoint_and_rigid(oracle_mod):
    """K^T is the adjoint of K (<K^T lambda, U> = <lambda, K U>), and K U of a
    pure rotation is perpendicular to the lever arm."""
    s = S.boomerangs_wall(n_bodies=5)
    rng = _rng(6)
    U = rng.standard_normal((5, 6))
    lam = rng.standard_normal((s.n_blobs, 3))
    KU = oracle_mod.K_apply(s.pos, s.body_off, s.q, U)
    KTl = oracle_mod.KT_apply(s.pos, s.body_off, s.q, lam)
    assert abs(np.sum(KTl * U) - np.sum(lam * KU)) < 1e-12 * np.abs(KU).sum()
    U[:, :3] = 0
    KU = oracle_mod.K_apply(s.pos, s.body_off, s.q, U)
    for p in range(5):
        o, e = s.body_off[p], s.body_off[p + 1]
        arm = s.pos[o:e] - s.q[p]
        assert np.abs(np.sum(KU[o:e] * arm, axis=1)).max() < 1e-13


def _table1():
    rows = [l.split() for l in open(os.path.join(GOLD, "table1_effective_radii.txt"))
            if l.strip() and not l.startswith("#")]
    return [(int(r[0]), float(r[1]), float(r[2]), float(r[3]), float(r[4])) for r in rows]


@pytest.mark.parametrize("n_blobs,ratio,Rh,Rt,Rs",
                         [r for r in _table1() if r[0] <= 642])
def test_table1_effective_radii(oracle_mod, n_blobs, ratio, Rh, Rt, Rs):
    """Effective translational, rotational and stresslet radii of sphere
    shells (Sec. 4.1, Table 1 left) to the printed 4 decimals."""
    shp = S.sphere_shell(n_blobs)
    a = ratio * S.min_spacing(shp)
    sus = S.Suspension(shp.copy(), np.array([0, n_blobs]), np.zeros((1, 3)), a, 1.0, False)
    N = oracle_mod.body_mobility(sus)
    assert abs(1.0 / (6 * np.pi * N[0, 0]) - Rh) <= 6e-5
    assert abs((1.0 / (8 * np.pi * N[3, 3])) ** (1 / 3) - Rt) <= 6e-5
    # isotropy of the shells (Sec. 4.1): translational block is a multiple of I
    assert np.abs(N[:3, :3] - N[0, 0] * np.eye(3)).max() < 1e-12 * N[0, 0]
    if n_blobs <= 42:
        # stresslet radius from the slip -gamma (x, -y, 0) with zero force.
        # The stresslet of the finer shells depends on how the shell is
        # oriented relative to the shear axes at the 1e-4 level, which the
        # paper does not state, so only the 12- and 42-blob shells are pinned.
        g = 1.0
        slip = -g * np.stack([shp[:, 0], -shp[:, 1], np.zeros(n_blobs)], axis=1)
        U, lam = oracle_mod.dense_solve(sus, np.zeros((1, 6)), slip)
        Sm = (lam[:, :, None] * shp[:, None, :]).sum(axis=0)
        Sm = 0.5 * (Sm + Sm.T) - np.trace(Sm) / 3 * np.eye(3)
        assert abs((-3 * Sm[0, 0] / (20 * np.pi * g)) ** (1 / 3) - Rs) <= 6e-5


def _fits():
    out = {}
    for l in open(os.path.join(GOLD, "appendixD_wall_fits.txt")):
        if l.strip() and not l.startswith("#"):
            t = l.split()
            out[t[0]] = [float(v) for v in t[1:]]
    return out


@pytest.mark.slow
def test_appendixD_sphere_near_wall_fits(oracle_mod):
    """642-blob shell (a/s = 1/2) above the wall, mobility averaged over
    random orientations, against the rational fits of Appendix D within
    their printed maximum relative error."""
    fits = _fits()

    def fit(k, x):
        d, al, n2, n1, n0, d1, d0, _ = fits[k]
        return d + (1 / x) ** al * (n2 * x * x + n1 * x + n0) / (x * x + d1 * x + d0)

    shp = S.sphere_shell(642)
    a = 0.5 * S.min_spacing(shp)
    free = S.Suspension(shp.copy(), np.array([0, 642]), np.zeros((1, 3)), a, 1.0, False)
    N0 = oracle_mod.body_mobility(free)
    Rh = 1 / (6 * np.pi * N0[0, 0])
    Rt = (1 / (8 * np.pi * N0[3, 3])) ** (1 / 3)
    rng = _rng(7)
    for x in (1.5, 3.0, 6.0):
        H = x * Rh
        vals = {k: [] for k in fits}
        for _ in range(2):
            qt = S.random_quaternion(rng)
            pos = shp @ S.rotation_matrix(qt).T + np.array([0, 0, H])
            N = oracle_mod.body_mobility(
                S.Suspension(pos, np.array([0, 642]), np.array([[0, 0, H]]), a, 1.0, True))
            vals["tt_par"].append(0.5 * (N[0, 0] + N[1, 1]) * 6 * np.pi * Rh)
            vals["rr_par"].append(0.5 * (N[3, 3] + N[4, 4]) * 8 * np.pi * Rt ** 3)
            vals["rr_perp"].append(N[5, 5] * 8 * np.pi * Rt ** 3)
            vals["rt_par"].append(0.5 * (N[4, 0] - N[3, 1]) * 6 * np.pi * Rh ** 2)
        for k, v in vals.items():
            ref = fit(k, x)
            assert abs(np.mean(v) / ref - 1) <= fits[k][-1], (k, x, np.mean(v), ref)


def test_dense_solve_equals_gmres_free_space(oracle_mod):
    s = S.spheres_free_space()
    Ud, ld = oracle_mod.dense_solve(s, s.FT)
    Ug, lg, info = oracle_mod.solve_mobility(s, s.FT, tol=1e-13)
    assert np.linalg.norm(Ug - Ud) <= 1e-10 * np.linalg.norm(Ud)
    assert np.linalg.norm(lg - ld) <= 1e-9 * np.linalg.norm(ld)
    assert oracle_mod.relative_residual(s, s.FT, None, Ud, ld) < 1e-12
    assert info["iterations"] < 40


def test_dense_solve_equals_gmres_wall_with_slip(oracle_mod):
    s = S.boomerangs_wall(n_bodies=12, lateral=12.0)
    slip = _rng(8).standard_normal((s.n_blobs, 3)) * 0.1
    Ud, ld = oracle_mod.dense_solve(s, s.FT, slip)
    Ug, lg, info = oracle_mod.solve_mobility(s, s.FT, slip, tol=1e-13)
    assert np.linalg.norm(Ug - Ud) <= 1e-10 * np.linalg.norm(Ud)
    assert oracle_mod.relative_residual(s, s.FT, slip, Ud, ld) < 1e-12


def test_block_preconditioner_exact_for_one_body(oracle_mod):
    """With a single body the block-diagonal preconditioner is the system
    itself, so GMRES converges in one iteration."""
    shp = S.boomerang()
    s = S.Suspension(shp + np.array([0, 0, 3.0]), np.array([0, 15]), np.array([[0, 0, 3.0]]),
                     0.3, 1.0, True)
    FT = _rng(9).standard_normal((1, 6))
    U, lam, info = oracle_mod.solve_mobility(s, FT, tol=1e-12)
    assert info["iterations"] == 1
    Ud, _ = oracle_mod.dense_solve(s, FT)
    assert np.allclose(U, Ud, rtol=1e-11, atol=1e-14)


def test_triangle_body_pulled_normal_to_its_plane(oracle_mod):
    """Smallest non-degenerate body: three blobs on an equilateral triangle
    pulled normal to their plane share the force equally by symmetry and
    translate without rotating, with (M_11 + 2 M_12) per unit blob force."""
    a, side = 0.2, 1.0
    ang = np.arange(3) * 2 * np.pi / 3
    pos = np.stack([np.cos(ang), np.sin(ang), np.zeros(3)], axis=1) * side / np.sqrt(3)
    s = S.Suspension(pos, np.array([0, 3]), np.zeros((1, 3)), a, 1.0, False)
    F = np.array([[0, 0, 3.0, 0, 0, 0]])
    U, lam = oracle_mod.dense_solve(s, F)
    assert np.allclose(lam, [[0, 0, 1]] * 3, atol=1e-13)
    assert np.abs(U[0, 3:]).max() < 1e-13 and np.abs(U[0, :2]).max() < 1e-13
    mu0 = 1 / (6 * np.pi * a)
    C1 = 3 * a / (4 * side) + a ** 3 / (2 * side ** 3)  # r_12 is normal to z
    assert abs(U[0, 2] - mu0 * (1 + 2 * C1)) < 1e-13
