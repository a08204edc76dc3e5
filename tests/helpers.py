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


def row_rel_err_fast(row_ptr, got, ref):
    """row_rel_err for large patterns (segment maxima with reduceat); rows
    must not be empty unless their whole segment is."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    got = np.asarray(got)
    ref = np.asarray(ref)
    if ref.size == 0:
        return 0.0
    starts = row_ptr[:-1]
    nonempty = row_ptr[1:] > starts
    s = starts[nonempty]
    err = np.maximum.reduceat(np.abs(got - ref), s)
    scale = np.maximum.reduceat(np.abs(ref), s)
    assert np.all(err[scale == 0] == 0)
    nz = scale > 0
    return float(np.max(err[nz] / scale[nz])) if nz.any() else 0.0


def check_fan_codes(fan, row_ptr, col_idx, me):
    """Every nonzero fan code must describe a walk around its row's vertex
    over triangles of the mesh, each in its own vertex order, covering every
    off-diagonal slot once, with the diagonal slot named.  Returns the number
    of rows with a code."""
    fan = np.asarray(fan).view(np.uint64)
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx)
    me = np.asarray(me)
    tris = set()
    for a, b, c in me.tolist():
        tris.add((a, b, c))
        tris.add((b, c, a))
        tris.add((c, a, b))
    coded = np.nonzero(fan & np.uint64(15))[0]
    for i in coded.tolist():
        code = int(fan[i])
        n = code & 15
        closed = (code >> 4) & 1
        pd = (code >> 5) & 15
        slots = [(code >> (9 + 4 * j)) & 15 for j in range(n)]
        rs, re = int(row_ptr[i]), int(row_ptr[i + 1])
        assert re - rs == n + 1, i
        assert col_idx[rs + pd] == i, i
        assert sorted(slots + [pd]) == list(range(n + 1)), i
        d = n if closed else n - 1
        for j in range(d):
            s1, s2 = slots[j], slots[(j + 1) % n]
            assert (i, int(col_idx[rs + s1]), int(col_idx[rs + s2])) in tris, (i, j)
    return int(coded.size)


def check_fan_codes_vec(fan, row_ptr, col_idx, me, nq):
    """check_fan_codes, vectorised for full-size meshes whose every oriented
    edge (v, next) belongs to one triangle (consistently oriented manifold
    meshes, such as the benchmark meshes).  Returns the number of coded rows."""
    fan = np.asarray(fan).view(np.uint64).astype(np.uint64)
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    me = np.asarray(me, dtype=np.int64)
    # oriented edges (v, next) -> previous vertex of the same triangle
    v = me.reshape(-1)
    nxt = me[:, [1, 2, 0]].reshape(-1)
    prv = me[:, [2, 0, 1]].reshape(-1)
    key = v * nq + nxt
    order = np.argsort(key, kind="stable")
    key, prv = key[order], prv[order]
    assert np.all(np.diff(key) > 0), "an oriented edge belongs to two triangles"
    rows = np.nonzero(fan & np.uint64(15))[0]
    code = fan[rows]
    n = (code & np.uint64(15)).astype(np.int64)
    closed = ((code >> np.uint64(4)) & np.uint64(1)).astype(bool)
    pd = ((code >> np.uint64(5)) & np.uint64(15)).astype(np.int64)
    rs = row_ptr[rows]
    L = row_ptr[rows + 1] - rs
    assert np.all(L == n + 1)
    assert np.all(col_idx[rs + pd] == rows)
    seen = np.zeros(rows.size, np.int64)
    seen |= np.int64(1) << pd
    nmax = int(n.max()) if rows.size else 0
    slots = [((code >> np.uint64(9 + 4 * j)) & np.uint64(15)).astype(np.int64) for j in range(nmax + 1)]
    for j in range(nmax):
        on = j < n
        seen[on] |= np.int64(1) << slots[j][on]
        # step j: the triangle (i, s_j, s_{j+1 mod n}); an open fan has n - 1 steps
        step = on & (closed | (j < n - 1))
        jn = np.where(j + 1 < n, slots[min(j + 1, nmax)], slots[0])
        a = col_idx[rs[step] + slots[j][step]]
        b = col_idx[rs[step] + jn[step]]
        k = rows[step] * nq + a
        at = np.searchsorted(key, k)
        assert np.all(at < key.size) and np.all(key[np.minimum(at, key.size - 1)] == k)
        assert np.all(prv[at] == b)
    assert np.all(seen == (np.int64(1) << (n + 1)) - 1)
    return int(rows.size)
