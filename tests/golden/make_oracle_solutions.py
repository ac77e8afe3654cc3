"""Writes the oracle's reference solutions used by the GPU parity tests.

Calls only `oracle/` (and the seeded input generators in `suspensions/`):
  boomerangs1000_oracle_U.txt
      U of the 1000-boomerang wall suspension (15,000 blobs, the headline
      workload) solved by the oracle's right-preconditioned GMRES to a
      relative residual of 1e-12.
  table1_right_oracle.txt
      Iterations of the oracle's GMRES (no restarts, tolerance 1e-8) on the
      simple cubic lattices of Sec. 4.4, Table 1 (right): 16^3 = 4096
      12-blob shells and 8^3 = 512 42-blob shells at the five volume
      fractions, with the paper's printed counts beside them.
  lattice42_phi0.0014_oracle_U.txt, lattice12_phi0.0014_oracle_U_sampled.txt
      U of the sparsest lattice of each kind solved to 1e-12 (every body of
      the 512-shell lattice; 64 sampled bodies of the 4096-shell lattice).

Run from the repository root:  python tests/golden/make_oracle_solutions.py [which...]
with `which` among boomerangs, table1, lattice_u (default: all).  The oracle
uses every host core (OpenMP); the 49,152-blob lattice takes tens of minutes.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import suspensions as S  # noqa: E402

PAPER_ITERS = {12: (4, 5, 9, 13, 20), 42: (4, 6, 10, 13, 23)}
LATTICES = {12: 16, 42: 8}
SAMPLE_BODIES = 64


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def boomerangs():
    s = S.boomerangs_wall()
    U, lam, info = oracle.solve_mobility(s, s.FT, tol=1e-12)
    res = oracle.relative_residual(s, s.FT, None, U, lam)
    log(f"boomerangs: {info['iterations']} iterations, residual {res:.2e}")
    with open(os.path.join(HERE, "boomerangs1000_oracle_U.txt"), "w") as f:
        f.write("# U (u_x u_y u_z w_x w_y w_z per body) of the 1000 x 15-blob boomerang wall suspension\n")
        f.write("# (suspensions.boomerangs_wall() defaults), oracle GMRES to relative residual 1e-12;\n")
        f.write(f"# {info['iterations']} iterations, final oracle residual {res:.3e}.  Written by make_oracle_solutions.py.\n")
        np.savetxt(f, U, fmt="%.17e")


def table1():
    rows = []
    for nb, ns in LATTICES.items():
        for k, phi in enumerate(S.LATTICE_PHI):
            s = S.sphere_lattice(ns, nb, phi)
            t0 = time.time()
            U, lam, info = oracle.solve_mobility(s, s.FT, s.slip, tol=1e-8, restart=200)
            res = oracle.relative_residual(s, s.FT, s.slip, U, lam)
            log(f"lattice {nb} blobs phi {phi}: {info['iterations']} iterations (paper {PAPER_ITERS[nb][k]}), "
                f"residual {res:.2e}, {time.time() - t0:.0f} s")
            rows.append((nb, ns ** 3, phi, PAPER_ITERS[nb][k], info["iterations"], res))
    with open(os.path.join(HERE, "table1_right_oracle.txt"), "w") as f:
        f.write("# Sec. 4.4, Table 1 (right): GMRES iterations to a relative residual of 1e-8 for simple cubic\n")
        f.write("# lattices of sphere shells in unbounded flow (suspensions.sphere_lattice: a = s/2, spacing from\n")
        f.write("# phi with the shell's R_h, random forces, torques and slips), right preconditioning with the\n")
        f.write("# block-diagonal preconditioner, x0 = 0, no restarts.  paper_iters: the printed counts;\n")
        f.write("# oracle_iters: the oracle's GMRES.  Written by make_oracle_solutions.py.\n")
        f.write("# n_blobs n_bodies phi paper_iters oracle_iters oracle_residual\n")
        for r in rows:
            f.write(f"{r[0]} {r[1]} {r[2]:g} {r[3]} {r[4]} {r[5]:.3e}\n")


def lattice_u():
    phi = S.LATTICE_PHI[0]
    for nb, ns in ((42, 8), (12, 16)):
        s = S.sphere_lattice(ns, nb, phi)
        U, lam, info = oracle.solve_mobility(s, s.FT, s.slip, tol=1e-12, restart=200)
        res = oracle.relative_residual(s, s.FT, s.slip, U, lam)
        log(f"lattice {nb} U: {info['iterations']} iterations, residual {res:.2e}")
        if nb == 42:
            name, rows, body_ids = f"lattice42_phi{phi:g}_oracle_U.txt", U, np.arange(s.n_bodies)
        else:
            body_ids = np.sort(np.random.default_rng(S.seed_for(6, 99)).choice(s.n_bodies, SAMPLE_BODIES,
                                                                                replace=False))
            name, rows = f"lattice12_phi{phi:g}_oracle_U_sampled.txt", U[body_ids]
        with open(os.path.join(HERE, name), "w") as f:
            f.write(f"# U of the {ns}^3 lattice of {nb}-blob shells at phi = {phi:g} (suspensions.sphere_lattice),\n")
            f.write(f"# oracle GMRES to relative residual 1e-12 ({info['iterations']} iterations, residual {res:.3e}).\n")
            f.write("# columns: body index, u_x u_y u_z w_x w_y w_z.  Written by make_oracle_solutions.py.\n")
            np.savetxt(f, np.concatenate([body_ids[:, None], rows], axis=1), fmt=["%d"] + ["%.17e"] * 6)


if __name__ == "__main__":
    which = sys.argv[1:] or ["boomerangs", "table1", "lattice_u"]
    for w in which:
        log(f"start {w} ({oracle.num_threads()} threads)")
        globals()[w]()
