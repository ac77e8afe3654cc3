"""Error measures of the GPU parity tests.

err(a, b) is the larger of
  * the relative 2-norm error ||a - b|| / ||b|| over the whole array, and
  * the largest per-row error max_r ||a_r - b_r|| divided by the rms row norm
    of the reference (rows: blobs of an (Nb, 3) array, bodies of an (N, 6)
    array, elements of a 1-D array), scaled down by `row_factor`,
so one bar bounds both the global error and the error of any single blob or
body: a defect confined to a few rows fails it even where it would hardly
move the 2-norm.  Products use row_factor 1 (their per-row errors sit far
below the bar); solves use 10, since their velocity errors near the bar are
spread unevenly over the bodies.
"""
import numpy as np


def rel2(a, b) -> float:
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rowmax(a, b) -> float:
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    a2 = a.reshape(a.shape[0], -1) if a.ndim > 1 else a.reshape(-1, 1)
    b2 = b.reshape(a2.shape)
    rms = np.sqrt(np.mean(np.sum(b2 * b2, axis=1)))
    return float(np.max(np.linalg.norm(a2 - b2, axis=1)) / rms)


def err(a, b, row_factor: float = 1.0) -> float:
    return max(rel2(a, b), rowmax(a, b) / row_factor)


def solve_err(a, b) -> float:
    return err(a, b, 10.0)
