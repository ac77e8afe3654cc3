"""The oracle's pins catch plausible mistakes.

Each mutant is the oracle's C source with one plausible error planted (a
wrong coefficient, a flipped sign, a transposed operand, a wrong image
point, a dropped term, a wrong branch threshold).  It is compiled on the CPU
and must fail at least one of the independent checks the pin tests use:
the symbolic double-Faxen derivations (Oseen and Blake image), the surface
average of the Oseen tensor over overlapping blobs, continuity at
r = 2a, the self limits, and reciprocity of the assembled wall mobility.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rmb_oracle.c")

MUTANTS = {
    "near-branch coefficient": ("9.0 * d / (32.0 * a)", "9.0 * d / (16.0 * a)"),
    "sign of C2": ("crr = 3.0 * a / (4.0 * d) - 3.0 * a * a * a", "crr = 3.0 * a / (4.0 * d) + 3.0 * a * a * a"),
    "image point": ("ri[2] + rj[2]", "ri[2] - rj[2] + 2.0 * rj[2] * 0.999"),
    "transposed operand": ("c3 * e[p] * zh[q]", "c3 * zh[p] * e[q]"),
    "height of the wrong blob": ("double hh = rj[2] / L;", "double hh = ri[2] / L;"),
    "dropped xi^4 term": ("+ 2.0 * xi4 * (1.0 - 5.0 * ez2));", ");"),
    "branch threshold": ("if (d > 2.0 * a)", "if (d > a)"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, name
    path = tmp_path / f"mut_{abs(hash(name))}.c"
    path.write_text(src.replace(old, new, 1))
    lib = tmp_path / f"mut_{abs(hash(name))}.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-o", str(lib), str(path), "-lm"])
    L = ctypes.CDLL(str(lib))
    dp = ctypes.POINTER(ctypes.c_double)
    L.oracle_pair_block.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
    L.oracle_wall_block.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp]
    return L


def _block(L, fn, ri, rj, a, wall=None):
    ri = np.ascontiguousarray(ri, dtype=np.float64)
    rj = np.ascontiguousarray(rj, dtype=np.float64)
    out = np.empty(9)
    p = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if fn == "pair":
        L.oracle_pair_block(p(ri), p(rj), a, 1.0, int(bool(wall)), p(out))
    else:
        L.oracle_wall_block(p(ri), p(rj), a, 1.0, p(out))
    return out.reshape(3, 3)


@pytest.fixture(scope="module")
def references():
    """Independent references: symbolic double-Faxen of Oseen and of Blake's
    image system (the same derivations as the pin tests)."""
    import sympy as sp
    from test_oracle_pins import _blake_symbolic
    x = sp.symbols("x1 x2 x3", real=True)
    a = sp.symbols("a", positive=True)
    X = sp.Matrix(x)
    r = sp.sqrt(X.dot(X))
    G = (sp.eye(3) / r + X * X.T / r ** 3) / (8 * sp.pi)
    lap = lambda M: M.applyfunc(lambda e: sum(sp.diff(e, v, 2) for v in x))
    G1 = G + a ** 2 / 6 * lap(G)
    rpy = sp.lambdify((*x, a), G1 + a ** 2 / 6 * lap(G1), "numpy")
    sp_, xs, ys, GB, G0 = _blake_symbolic()
    Wim = GB - G0
    lapx = lambda M: M.applyfunc(lambda e: sum(sp.diff(e, v, 2) for v in xs))
    lapy = lambda M: M.applyfunc(lambda e: sum(sp.diff(e, v, 2) for v in ys))
    A1 = Wim + a ** 2 / 6 * lapx(Wim)
    wall = sp.lambdify((*xs, *ys, a), A1 + a ** 2 / 6 * lapy(A1), "numpy")
    return rpy, wall


def _pins_hold(L, references):
    rpy, wall = references
    rng = np.random.default_rng(77)
    a = 0.4
    # far-branch RPY against the derivation
    for _ in range(5):
        d = rng.standard_normal(3)
        d *= rng.uniform(2.1 * a, 10 * a) / np.linalg.norm(d)
        ref = np.array(rpy(*d, a), dtype=float)
        if np.abs(_block(L, "pair", d, np.zeros(3), a) - ref).max() > 1e-12 * np.abs(ref).max():
            return False
    # continuity at 2a and the self block
    e = np.array([0.6, 0.0, 0.8])
    lo = _block(L, "pair", (2 * a - 1e-10) * e, np.zeros(3), a)
    hi = _block(L, "pair", (2 * a + 1e-10) * e, np.zeros(3), a)
    if np.abs(lo - hi).max() > 1e-8:
        return False
    if np.abs(_block(L, "pair", np.ones(3), np.ones(3), a) - np.eye(3) / (6 * np.pi * a)).max() > 1e-15:
        return False
    # overlap branch: linear in d between the self value and the value at 2a
    half = _block(L, "pair", a * e, np.zeros(3), a)
    mid = 0.5 * (_block(L, "pair", 1e-9 * e, np.zeros(3), a) + lo)
    if np.abs(half - mid).max() > 1e-8:
        return False
    # overlap branch against the Oseen tensor averaged over both blob surfaces
    n = 400_000
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    dist = 1.5 * a
    dd = np.array([dist, 0.0, 0.0]) + a * (u - v)
    rr = np.linalg.norm(dd, axis=1)
    mc_par = (np.mean(1.0 / rr) + np.mean(dd[:, 0] ** 2 / rr ** 3)) / (8 * np.pi)
    if abs(_block(L, "pair", [dist, 0, 0], np.zeros(3), a)[0, 0] / mc_par - 1) > 1e-2:
        return False
    # wall correction against the derivation
    for _ in range(5):
        xi = np.array([*rng.uniform(-2, 2, 2), rng.uniform(a, 3)])
        xj = np.array([*rng.uniform(-2, 2, 2), rng.uniform(a, 3)])
        ref = np.array(wall(*xi, *xj, a), dtype=float)
        if np.abs(_block(L, "wall", xi, xj, a) - ref).max() > 1e-12 * np.abs(ref).max():
            return False
    # reciprocity of the full wall block
    xi, xj = np.array([0.3, -0.2, 1.1]), np.array([-0.5, 0.4, 0.7])
    if np.abs(_block(L, "pair", xi, xj, a, True) - _block(L, "pair", xj, xi, a, True).T).max() > 1e-15:
        return False
    return True


@pytest.mark.slow
def test_unmutated_oracle_passes_the_checks(tmp_path, references):
    L = _build(tmp_path, "none", "#include <math.h>", "#include <math.h>")
    assert _pins_hold(L, references)


@pytest.mark.slow
@pytest.mark.parametrize("name", list(MUTANTS))
def test_mutant_is_caught(tmp_path, references, name):
    old, new = MUTANTS[name]
    L = _build(tmp_path, name, old, new)
    assert not _pins_hold(L, references), f"mutant '{name}' passed every pin"
