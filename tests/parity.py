"""Comparison helpers for GPU-vs-oracle parity tests.

Roots of one phase form a set; labels may differ between two solvers after
a cold start, so rows are compared as point sets (nearest-neighbour pairing
that must be one-to-one).

Tolerance (FP64 roots).  The paper's cutoffs (Sec. 3.2 footnote) flag a root
when its last step is below 1e-9 or when the App. C bound
|F|(|F| + 2|1-kappa_s|) < 1e-9 holds, i.e. |F| < ~1e-9 / (2|1-kappa_s|).  A
root flagged by the second test can sit |F|/|F'| from the exact zero, so the
gate is conditioning-aware, using only the reference root:
    |z_gpu - z_ref| <= tol + tol / (|1 - kappa_s| |F'(z_ref)|).
Caustics: on the critical curve |dw/dz| = |dw/dzbar| = |1 - kappa_s|, so
|w_gpu - w_ref| <= 2 |1 - kappa_s| (root bound) + 1e-11 (1 + |w|).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def pair(a, b):
    """perm with b[perm[k]] nearest a[k]; asserts the pairing is one-to-one."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    tree = cKDTree(np.stack([b.real, b.imag], axis=1))
    d, idx = tree.query(np.stack([a.real, a.imag], axis=1))
    assert np.unique(idx).shape[0] == a.shape[0], "pairing is not one-to-one"
    return idx, d


def root_bound(field, Fp_ref, tol=1e-9):
    a = abs(1.0 - field.kappa_s)
    return tol + tol / (a * np.abs(Fp_ref))


def compare_row_sets(gpu_rows, ref_rows, bound_rows=None):
    """Max paired distance per row and, if bounds are given, the max ratio
    distance / bound (must be <= 1)."""
    worst = 0.0
    worst_ratio = 0.0
    for j in range(ref_rows.shape[0]):
        idx, d = pair(ref_rows[j], gpu_rows[j])
        worst = max(worst, float(d.max()))
        if bound_rows is not None:
            worst_ratio = max(worst_ratio, float((d / bound_rows[j]).max()))
    return worst, worst_ratio
