"""GPU sparse(I, J, V, m, n) against the oracle's, through the C ABI.

The pattern must match bit for bit; every value is the left-to-right sum of
its triplets in ascending t on both sides, so values match bitwise too."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1305_3122_amd import meshgen as mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1305_3122_amd as fem  # noqa: E402
from paper_1305_3122_amd import _lib  # noqa: E402

DEV = torch.device("cuda:0")


def _up(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _np(t):
    return t.detach().cpu().numpy()


def optv2_triplets(me):
    """Ig, Jg of the OptV2 assembly, local entry r = 3b + a of triangle k at
    t = r nme + k: row me[k][a], column me[k][b]."""
    a = np.tile(np.arange(3), 3)
    b = np.repeat(np.arange(3), 3)
    Ig = me[:, a].T.reshape(-1)
    Jg = me[:, b].T.reshape(-1)
    return Ig.astype(np.int32), Jg.astype(np.int32)


def _check(I, J, V, m, n, contrib=True):
    A = fem.fem_sparse(_up(I), _up(J), None if V is None else _up(V), m, n, contrib=contrib)
    torch.cuda.synchronize()
    rp, ci, pos = oracle.sparse_positions(I, J, m, n)
    assert A.nnz == ci.shape[0]
    np.testing.assert_array_equal(_np(A.row_ptr), rp)
    np.testing.assert_array_equal(_np(A.col_idx), ci)
    if V is not None:
        _, _, vals = oracle.sparse(I, J, V, m, n)
        np.testing.assert_array_equal(_np(A.vals), vals)
    if contrib:
        order = np.argsort(pos, kind="stable")          # triplets by entry, ascending t
        cptr = np.concatenate([[0], np.cumsum(np.bincount(pos, minlength=A.nnz))])
        np.testing.assert_array_equal(_np(A.contrib), order)
        np.testing.assert_array_equal(_np(A.contrib_ptr), cptr)
    return A


def _cases():
    rng = np.random.default_rng(1305)
    out = []
    for name, m in (("cfg1", mg.config_mesh(1)), ("disk24", mg.unit_disk(24, seed=3)),
                    ("square40", mg.unit_square(40, seed=4))):
        I, J = optv2_triplets(m.me)
        out.append((f"optv2_{name}", I, J, rng.standard_normal(I.shape[0]), m.nq, m.nq))
    # heavy duplicates, empty rows, rectangular
    I = rng.integers(0, 300, 20000).astype(np.int32) * 3
    J = rng.integers(0, 40, 20000).astype(np.int32)
    out.append(("dup_rect", I, J, rng.standard_normal(20000), 1000, 41))
    # one long row sorted in LDS (2000 triplets) among short ones
    I = np.concatenate([np.full(2000, 7), rng.integers(0, 64, 500)]).astype(np.int32)
    J = rng.integers(0, 5000, 2500).astype(np.int32)
    out.append(("long_row", I, J, rng.standard_normal(2500), 64, 5000))
    # a row whose bucket does not fit in LDS (global path), values that cancel
    I = np.concatenate([np.full(9000, 2), rng.integers(0, 5, 300)]).astype(np.int32)
    J = rng.integers(0, 3000, 9300).astype(np.int32)
    V = rng.standard_normal(9300)
    V[::2] = 1e16
    V[1::2] = -1e16
    out.append(("big_bucket", rng.permutation(I), J, V, 5, 3000))
    # all triplets on one entry
    out.append(("one_entry", np.zeros(777, np.int32), np.full(777, 3, np.int32),
                rng.standard_normal(777), 1, 4))
    # uneven density over many coarse buckets: dense rows (40 triplets), then
    # sparse ones (2), then empty ones, so that the coarse buckets choose
    # different fine sizes and leave slots empty
    m = 300_000
    dense = np.repeat(np.arange(50_000), 40)
    sparse_rows = np.repeat(np.arange(50_000, 250_000), 2)
    I = rng.permutation(np.concatenate([dense, sparse_rows])).astype(np.int32)
    J = rng.integers(0, 60_000, I.shape[0]).astype(np.int32)
    out.append(("uneven_density", I, J, rng.standard_normal(I.shape[0]), m, 60_000))
    return out


CASES = _cases()


@pytest.mark.parametrize("name,I,J,V,m,n", CASES, ids=[c[0] for c in CASES])
def test_sparse_matches_oracle(name, I, J, V, m, n):
    print(f"[case] sparse {name} m={m} n={n} nt={I.shape[0]}", flush=True)
    _check(I, J, V, m, n)


def test_sparse_pattern_only_and_empty():
    rng = np.random.default_rng(2)
    I = rng.integers(0, 50, 400).astype(np.int32)
    J = rng.integers(0, 50, 400).astype(np.int32)
    A = _check(I, J, None, 50, 50, contrib=False)
    assert A.vals is None
    A = fem.fem_sparse(torch.zeros(0, dtype=torch.int32, device=DEV),
                       torch.zeros(0, dtype=torch.int32, device=DEV),
                       torch.zeros(0, dtype=torch.float64, device=DEV), 6, 3, contrib=True)
    torch.cuda.synchronize()
    assert A.nnz == 0
    np.testing.assert_array_equal(_np(A.row_ptr), np.zeros(7, np.int32))
    np.testing.assert_array_equal(_np(A.contrib_ptr), [0])


def test_sparse_values_resum_bitwise():
    m = mg.unit_square(30, seed=8)
    I, J = optv2_triplets(m.me)
    rng = np.random.default_rng(3)
    V1, V2 = rng.standard_normal(I.shape[0]), rng.standard_normal(I.shape[0])
    A = fem.fem_sparse(_up(I), _up(J), _up(V1), m.nq, m.nq, contrib=True)
    v2 = fem.fem_sparse_values(A, _up(V2))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(v2), oracle.sparse(I, J, V2, m.nq, m.nq)[2])
    v1 = fem.fem_sparse_values(A, _up(V1))
    assert torch.equal(v1, A.vals)
    fem.fem_sparse_values(A, _up(V2), out=v1, flags=fem.FEM_ACCUMULATE)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(v1), _np(A.vals) + _np(v2))


def test_sparse_errors():
    with pytest.raises(fem.FemError) as e:
        fem.fem_sparse(_up(np.array([0, 3], np.int32)), _up(np.array([0, 0], np.int32)), None, 3, 3)
    assert e.value.status == _lib.FEM_ERANGE
    with pytest.raises(fem.FemError) as e:
        fem.fem_sparse(_up(np.array([0, 1], np.int32)), _up(np.array([0, -1], np.int32)), None, 3, 3)
    assert e.value.status == _lib.FEM_ERANGE
    # col_cap below nnz
    lib = _lib.load()
    I = _up(np.array([0, 1, 2], np.int32))
    ws = C.c_size_t(0)
    _lib.check(lib.fem_sparse_workspace(3, 3, 3, C.byref(ws)))
    work = torch.empty(int(ws.value), dtype=torch.uint8, device=DEV)
    rp = torch.empty(4, dtype=torch.int32, device=DEV)
    col = torch.full((8,), -5, dtype=torch.int32, device=DEV)
    nnz = C.c_int64(0)
    st = lib.fem_sparse(3, 3, 3, I.data_ptr(), I.data_ptr(), None, rp.data_ptr(), col.data_ptr(),
                        None, 2, None, None, work.data_ptr(), int(ws.value), C.byref(nnz),
                        torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == _lib.FEM_ENOSPC
    assert bool((col[2:] == -5).all())
    # and the library keeps working
    _check(np.array([2, 0, 2], np.int32), np.array([1, 1, 1], np.int32), np.ones(3), 3, 3)


def test_sparse_full_size_optv2_triplets():
    # the 75.5M triplets of the 2048 x 2048 square: pattern equal to
    # fem_pattern's, sampled rows equal to a sequential sum in ascending t
    m = mg.config_mesh(2)
    I, J = optv2_triplets(m.me)
    V = mg.normal_seed(I.shape[0], seed=mg.BASE_SEED + 202)
    print(f"[case] sparse optv2 cfg2 nt={I.shape[0]}", flush=True)
    Id, Jd = _up(I), _up(J)
    A = fem.fem_sparse(Id, Jd, _up(V), m.nq, m.nq)
    pat = fem.fem_pattern(_up(m.me), m.nq)
    torch.cuda.synchronize()
    assert A.nnz == pat.nnz == m.nq + 2 * (m.nq + m.nme - 1)
    assert torch.equal(A.row_ptr, pat.row_ptr) and torch.equal(A.col_idx, pat.col_idx)
    rng = np.random.default_rng(11)
    rows = np.unique(rng.choice(m.nq, 300, replace=False))
    sel = np.nonzero(np.isin(I, rows))[0]            # ascending t
    rp, ci, vals = _np(A.row_ptr), _np(A.col_idx), _np(A.vals)
    for r in rows[:100]:
        t = sel[I[sel] == r]
        cols = ci[rp[r]:rp[r + 1]]
        want = np.zeros(cols.shape[0])
        k = np.searchsorted(cols, J[t])
        for kk, tt in zip(k, t):                     # left to right, ascending t
            want[kk] += V[tt]
        np.testing.assert_array_equal(vals[rp[r]:rp[r + 1]], want)
