"""Shared test helpers: tolerance checks and small mesh builders."""
import numpy as np

#: per-row max-norm relative tolerance for FP64 values (from the target spec)
RTOL_ROW = 1e-13


def row_rel_err(row_ptr, got, ref, dof_rows=None):
    """max over rows of  max_j |got_ij - ref_ij| / max_j |ref_ij|."""
    row_ptr = np.asarray(row_ptr)
    n = row_ptr.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    err = np.zeros(n)
    scale = np.zeros(n)
    np.maximum.at(err, rows, np.abs(np.asarray(got) - np.asarray(ref)))
    np.maximum.at(scale, rows, np.abs(np.asarray(ref)))
    nz = scale > 0
    assert np.all(err[~nz] == 0)
    return float(np.max(err[nz] / scale[nz])) if nz.any() else 0.0


def fan_mesh(n_fan: int, extra: int = 0, seed: int = 0):
    """A wheel around vertex 0 with n_fan triangles (valence n_fan), plus
    `extra` isolated vertices that no triangle uses."""
    ang = 2 * np.pi * np.arange(n_fan) / n_fan
    rng = np.random.default_rng(seed)
    r = 1.0 + 0.1 * rng.uniform(-1, 1, size=n_fan)
    q = np.vstack([[0.0, 0.0], np.column_stack([r * np.cos(ang), r * np.sin(ang)]),
                   rng.uniform(2, 3, size=(extra, 2))])
    me = np.array([[0, 1 + t, 1 + (t + 1) % n_fan] for t in range(n_fan)], dtype=np.int32)
    perm = rng.permutation(q.shape[0])
    q2 = np.empty_like(q)
    q2[perm] = q
    return q2, perm[me].astype(np.int32)
