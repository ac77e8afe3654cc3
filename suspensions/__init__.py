"""Seeded synthetic suspensions of rigid multiblobs (inputs only).

This module builds the inputs that both the CPU oracle and the GPU library
consume: blob positions, body offsets, tracking points, applied forces and
torques, and blob force vectors for bare mobility products.  It holds none of
the method's arithmetic (no mobility tensor, no kinematic matrix, no solver):
only body shapes, placement, orientations and random loads.

Body models follow the paper:
  * sphere shells: an icosahedron refined by edge-midpoint subdivision with
    projection back onto the sphere, giving 12, 42, 162, 642 blobs
    (Sec. 4, construction of the shell models);
  * a 15-blob boomerang: a corner blob and two perpendicular arms of 7 blobs
    each, spacing 0.525 (bent-rod model of Sec. 5.3, geometry as specified
    for the single-wall benchmark workload).

The tracking point of every body is the centroid of its blobs.  Orientations
are uniform random unit quaternions (normalised 4-D Gaussians).

Every generator is deterministic given its seed: numpy's PCG64 with
seed = 160202170 + 1000 * workload_id + request_id.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_BASE = 160202170


def seed_for(workload: int, request: int = 0) -> int:
    return SEED_BASE + 1000 * workload + request


# ----------------------------------------------------------------------------
# body shapes (reference configurations, centred on the blob centroid)
# ----------------------------------------------------------------------------

def icosahedron(radius: float = 1.0) -> np.ndarray:
    """12 vertices of a regular icosahedron on a sphere of the given radius."""
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v.append((0.0, s1, s2 * phi))
            v.append((s1, s2 * phi, 0.0))
            v.append((s2 * phi, 0.0, s1))
    v = np.asarray(v, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return radius * v


def _icosahedron_faces(v: np.ndarray) -> List[tuple]:
    """Triangular faces of the icosahedron: triples of mutually nearest vertices."""
    n = len(v)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    edge = np.min(d[d > 1e-12])
    adj = np.abs(d - edge) < 1e-9 * max(edge, 1.0)
    faces = []
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    assert len(faces) == 20
    return faces


def sphere_shell(n_blobs: int, radius: float = 1.0) -> np.ndarray:
    """Shell of 12, 42, 162, 642 or 2562 blobs: recursive midpoint subdivision
    of the icosahedron with every new vertex projected onto the sphere."""
    levels = {12: 0, 42: 1, 162: 2, 642: 3, 2562: 4}
    if n_blobs not in levels:
        raise ValueError("shell sizes are 12, 42, 162, 642, 2562")
    verts = [tuple(p) for p in icosahedron(1.0)]
    faces = _icosahedron_faces(np.asarray(verts))
    for _ in range(levels[n_blobs]):
        cache = {}
        new_faces = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = (np.asarray(verts[i]) + np.asarray(verts[j])) / 2.0
                m /= np.linalg.norm(m)
                verts.append(tuple(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for (i, j, k) in faces:
            ij, jk, ki = mid(i, j), mid(j, k), mid(k, i)
            new_faces += [(i, ij, ki), (j, jk, ij), (k, ki, jk), (ij, jk, ki)]
        faces = new_faces
    out = radius * np.asarray(verts, dtype=np.float64)
    assert out.shape == (n_blobs, 3)
    return out


def boomerang(spacing: float = 0.525, arm: int = 7) -> np.ndarray:
    """Corner blob plus two perpendicular arms of `arm` blobs, centred on the
    blob centroid (15 blobs for arm=7)."""
    pts = [(0.0, 0.0, 0.0)]
    for k in range(1, arm + 1):
        pts.append((spacing * k, 0.0, 0.0))
    for k in range(1, arm + 1):
        pts.append((0.0, spacing * k, 0.0))
    pts = np.asarray(pts, dtype=np.float64)
    return pts - pts.mean(axis=0)


def min_spacing(shape: np.ndarray) -> float:
    d = np.linalg.norm(shape[:, None, :] - shape[None, :, :], axis=2)
    return float(np.min(d[d > 1e-12]))


# ----------------------------------------------------------------------------
# orientations
# ----------------------------------------------------------------------------

def random_quaternion(rng: np.random.Generator) -> np.ndarray:
    q = rng.standard_normal(4)
    return q / np.linalg.norm(q)


def rotation_matrix(q: np.ndarray) -> np.ndarray:
    """Rotation matrix of a unit quaternion (w, x, y, z)."""
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


# ----------------------------------------------------------------------------
# a suspension
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Suspension:
    """Lab-frame description of one mobility problem.

    pos      (Nb, 3) float64  blob positions
    body_off (N+1,)  int64    blobs of body p are pos[body_off[p]:body_off[p+1]]
    q        (N, 3)  float64  tracking points (blob centroids)
    a, eta                    blob radius, viscosity
    wall                      True: no-slip wall at z = 0, fluid in z > 0
    FT       (N, 6)  float64  applied force then torque per body (or None)
    slip     (Nb, 3) float64  active slip (or None for passive bodies)
    tol                       requested relative residual of the solve
    quat     (N, 4)           orientations used to place the bodies
    blob_shift (Nb,)          permeable bodies: kappa_p / (eta dV_i) per blob
                              (or None for impermeable bodies)
    """
    pos: np.ndarray
    body_off: np.ndarray
    q: np.ndarray
    a: float
    eta: float
    wall: bool
    FT: Optional[np.ndarray] = None
    slip: Optional[np.ndarray] = None
    tol: float = 1e-8
    quat: Optional[np.ndarray] = None
    name: str = ""
    blob_shift: Optional[np.ndarray] = None

    @property
    def n_blobs(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_bodies(self) -> int:
        return int(self.q.shape[0])


def assemble(shapes: List[np.ndarray], centres: np.ndarray, quats: np.ndarray):
    """Blob positions of bodies with reference shapes `shapes` placed so that
    their blob centroids sit at `centres` with orientations `quats`."""
    pos, off = [], [0]
    for shp, c, qt in zip(shapes, centres, quats):
        ref = shp - shp.mean(axis=0)
        pos.append(ref @ rotation_matrix(qt).T + c)
        off.append(off[-1] + len(shp))
    return np.concatenate(pos, axis=0), np.asarray(off, dtype=np.int64)


def _orient_above(rng, shape, centre_xy, h, zmin, max_tries=10000):
    """Draw orientations until every blob of `shape` centred at height h has
    z >= zmin.  Returns (quat, positions) or None."""
    ref = shape - shape.mean(axis=0)
    for _ in range(max_tries):
        qt = random_quaternion(rng)
        p = ref @ rotation_matrix(qt).T
        if h + p[:, 2].min() >= zmin:
            return qt
    return None


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def spheres_free_space(n_bodies: int = 8, box: float = 20.0, min_dist: float = 3.0,
                       radius: float = 1.0, a: float = 0.416, seed: Optional[int] = None,
                       tol: float = 1e-10) -> Suspension:
    """Icosahedral 12-blob spheres in unbounded flow: centres by random
    sequential addition in [0, box)^3 with a minimum centre distance, random
    orientations, forces and torques N(0, 1) per component."""
    rng = np.random.default_rng(seed_for(1) if seed is None else seed)
    centres = []
    while len(centres) < n_bodies:
        c = rng.uniform(0.0, box, 3)
        if all(np.linalg.norm(c - o) >= min_dist for o in centres):
            centres.append(c)
    centres = np.asarray(centres)
    quats = np.asarray([random_quaternion(rng) for _ in range(n_bodies)])
    shp = icosahedron(radius)
    pos, off = assemble([shp] * n_bodies, centres, quats)
    FT = rng.standard_normal((n_bodies, 6))
    return Suspension(pos, off, centres.copy(), a, 1.0, False, FT, None, tol, quats,
                      name=f"free-space {n_bodies} x 12-blob icosahedra")


def boomerangs_wall(n_bodies: int = 1000, lateral: float = 200.0, hmin: float = 1.5,
                    hmax: float = 6.0, a: float = 0.3, seed: Optional[int] = None,
                    tol: float = 1e-8) -> Suspension:
    """15-blob boomerangs above a no-slip wall: centroids uniform in
    [0, lateral)^2 laterally, heights uniform in [hmin, hmax]; the orientation
    is redrawn (same height) until every blob has z >= a.  Each body carries
    gravity -1 along z plus N(0, 0.1^2) noise per force component, zero
    torque."""
    rng = np.random.default_rng(seed_for(2) if seed is None else seed)
    shp = boomerang()
    centres, quats = [], []
    for _ in range(n_bodies):
        xy = rng.uniform(0.0, lateral, 2)
        h = rng.uniform(hmin, hmax)
        qt = _orient_above(rng, shp, xy, h, a)
        assert qt is not None
        centres.append([xy[0], xy[1], h])
        quats.append(qt)
    centres = np.asarray(centres)
    quats = np.asarray(quats)
    pos, off = assemble([shp] * n_bodies, centres, quats)
    FT = np.zeros((n_bodies, 6))
    FT[:, 0:3] = rng.normal(0.0, 0.1, (n_bodies, 3))
    FT[:, 2] -= 1.0
    return Suspension(pos, off, centres.copy(), a, 1.0, True, FT, None, tol, quats,
                      name=f"wall {n_bodies} x 15-blob boomerangs")


def icosahedra_monolayer(n_side: int = 128, n_bodies: Optional[int] = None,
                         spacing: float = 3.0, jitter: float = 0.25, hmin: float = 1.2,
                         hmax: float = 3.0, radius: float = 1.0, a: float = 0.416,
                         seed: Optional[int] = None):
    """Sedimented monolayer of 12-blob icosahedra over a wall: a jittered
    n_side x n_side square lattice (spacing 3, jitter U(-0.25, 0.25) per
    lateral axis), heights U[1.2, 3], random orientations.  `n_bodies` takes a
    prefix (row-major) of the lattice.  Returns (Suspension, blob_forces) with
    blob forces N(0, 1) per component in float64 (their float32 rounding is
    the single-precision input)."""
    rng = np.random.default_rng(seed_for(3) if seed is None else seed)
    nb_all = n_side * n_side
    ii, jj = np.meshgrid(np.arange(n_side), np.arange(n_side), indexing="ij")
    xy = np.stack([ii.ravel(), jj.ravel()], axis=1) * spacing
    xy = xy + rng.uniform(-jitter, jitter, (nb_all, 2))
    h = rng.uniform(hmin, hmax, nb_all)
    quats = np.asarray([random_quaternion(rng) for _ in range(nb_all)])
    lam = rng.standard_normal((nb_all * 12, 3))
    n = nb_all if n_bodies is None else int(n_bodies)
    centres = np.concatenate([xy[:n], h[:n, None]], axis=1)
    shp = icosahedron(radius)
    pos, off = assemble([shp] * n, centres, quats[:n])
    s = Suspension(pos, off, centres.copy(), a, 1.0, True, None, None, 1e-8, quats[:n],
                   name=f"wall monolayer {n} x 12-blob icosahedra")
    return s, lam[: n * 12].copy()


def shells_wall(n_bodies: int = 512, n_blobs: int = 162, radius: float = 1.0,
                a: float = 0.0871, lateral: float = 100.0, hmin: float = 1.2,
                hmax: float = 4.0, n_rhs: int = 8, seed: Optional[int] = None):
    """Shell spheres above a wall: centres uniform in [0, lateral)^2 laterally,
    heights U[hmin, hmax], random orientations.  Returns (Suspension, rhs)
    with `n_rhs` right-hand sides of length 3 Nb + 6 N, entries N(0, 1)."""
    rng = np.random.default_rng(seed_for(4) if seed is None else seed)
    shp = sphere_shell(n_blobs, radius)
    xy = rng.uniform(0.0, lateral, (n_bodies, 2))
    h = rng.uniform(hmin, hmax, n_bodies)
    quats = np.asarray([random_quaternion(rng) for _ in range(n_bodies)])
    centres = np.concatenate([xy, h[:, None]], axis=1)
    pos, off = assemble([shp] * n_bodies, centres, quats)
    s = Suspension(pos, off, centres.copy(), a, 1.0, True, None, None, 1e-8, quats,
                   name=f"wall {n_bodies} x {n_blobs}-blob shells")
    rhs = rng.standard_normal((n_rhs, 3 * s.n_blobs + 6 * n_bodies))
    return s, rhs


def mixed_wall_request(request_id: int, n_bodies: Optional[int] = None,
                       nmin: int = 10, nmax: int = 4000, a: float = 0.3,
                       area_per_body: float = 40.0, tol: float = 1e-8) -> Suspension:
    """One wall-bounded suspension of a request stream: the body count is
    log-uniform in [nmin, nmax]; each body is a 12-blob icosahedron (radius 1,
    height U[1.2, 3], redrawn until every blob has z >= a) or a 15-blob
    boomerang (height U[1.5, 6], orientation redrawn until every blob has
    z >= a) with equal probability; one blob radius per request.  The lateral
    box keeps the boomerang benchmark's area per body.  Loads are gravity -1
    along z plus N(0, 0.1^2) noise per force component, zero torque."""
    rng = np.random.default_rng(seed_for(5, request_id))
    if n_bodies is None:
        n_bodies = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    lateral = math.sqrt(area_per_body * n_bodies)
    ico, boo = icosahedron(1.0), boomerang()
    shapes, centres, quats = [], [], []
    for _ in range(n_bodies):
        xy = rng.uniform(0.0, lateral, 2)
        if rng.uniform() < 0.5:
            while True:
                h = rng.uniform(1.2, 3.0)
                qt = _orient_above(rng, ico, xy, h, a, max_tries=1)
                if qt is not None:
                    break
            shapes.append(ico)
        else:
            h = rng.uniform(1.5, 6.0)
            qt = _orient_above(rng, boo, xy, h, a)
            assert qt is not None
            shapes.append(boo)
        centres.append([xy[0], xy[1], h])
        quats.append(qt)
    centres = np.asarray(centres)
    quats = np.asarray(quats)
    pos, off = assemble(shapes, centres, quats)
    FT = np.zeros((n_bodies, 6))
    FT[:, 0:3] = rng.normal(0.0, 0.1, (n_bodies, 3))
    FT[:, 2] -= 1.0
    return Suspension(pos, off, centres.copy(), a, 1.0, True, FT, None, tol, quats,
                      name=f"request {request_id}: wall {n_bodies} mixed bodies")


def poisson_arrivals(n_requests: int = 256, rate: float = 50.0, seed: Optional[int] = None):
    """Arrival times (s) of a Poisson stream."""
    rng = np.random.default_rng(seed_for(5, 999) if seed is None else seed)
    return np.cumsum(rng.exponential(1.0 / rate, n_requests))


def random_blob_forces(n_blobs: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((n_blobs, 3))


# Table 1 (left) of the paper: hydrodynamic radius R_h / R_g of the shells at
# blob radius a = s/2 (s: the shell's minimal blob spacing).  The lattice
# workload states its volume fractions in terms of R_h, so the spacing needs
# it; this is a printed input of the geometry, not a computed quantity.
SHELL_RH_HALF_SPACING = {12: 1.2625, 42: 1.1220, 162: 1.0530, 642: 1.0239}
LATTICE_PHI = (1.4e-3, 0.011, 0.09, 0.18, 0.36)


def sphere_lattice(n_side: int, n_blobs: int, phi: float, seed: Optional[int] = None,
                   tol: float = 1e-8) -> Suspension:
    """Finite simple cubic lattice of n_side^3 sphere shells (radius 1, blob
    radius a = s/2) in unbounded flow (Sec. 4.4, Table 1 right).  The volume
    fraction is phi = (4 pi / 3) R_h^3 / d^3 with d the centre-to-centre
    spacing and R_h the shell's hydrodynamic radius (the paper pairs a spacing
    of 4 R_g ~ 3.6 R_h with phi ~ 0.09).  Every shell has the reference
    orientation.  Forces and torques are N(0, 1) per component; per-blob
    slips are N(0, 1) per component in units of the velocity a unit force
    gives an isolated shell, 1 / (6 pi eta R_h), so that the three random
    loads move the bodies comparably.  The seed defaults to one per
    (n_blobs, phi index)."""
    shp = sphere_shell(n_blobs, 1.0)
    a = 0.5 * min_spacing(shp)
    rh = SHELL_RH_HALF_SPACING[n_blobs]
    d = rh * (4.0 * math.pi / (3.0 * phi)) ** (1.0 / 3.0)
    if seed is None:
        k = min(range(len(LATTICE_PHI)), key=lambda i: abs(math.log(LATTICE_PHI[i] / phi)))
        seed = seed_for(6 if n_blobs == 12 else 7, k)
    rng = np.random.default_rng(seed)
    n = n_side ** 3
    ii, jj, kk = np.meshgrid(np.arange(n_side), np.arange(n_side), np.arange(n_side), indexing="ij")
    centres = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.float64) * d
    quats = np.tile(np.array([1.0, 0.0, 0.0, 0.0]), (n, 1))
    pos, off = assemble([shp] * n, centres, quats)
    FT = rng.standard_normal((n, 6))
    slip = rng.standard_normal((pos.shape[0], 3)) / (6.0 * math.pi * rh)
    return Suspension(pos, off, centres.copy(), a, 1.0, False, FT, slip, tol, quats,
                      name=f"free-space {n_side}^3 lattice of {n_blobs}-blob shells, phi {phi:g}")
