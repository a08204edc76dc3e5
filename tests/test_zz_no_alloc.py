"""fem_assemble_noalloc (the entry point that allocates nothing) against
fem_assemble, through the C ABI: the same kernels, so the same bits, on two
calls in a row (the second on a smaller mesh, over the scratch the first one
left), with the weighted mass (packed records in the scratch) and
FEM_CHECK_AREA (its flag in the scratch)."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1305_3122_amd import meshgen as mg
from tests.helpers import RTOL_ROW, row_rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1305_3122_amd as fem  # noqa: E402
from paper_1305_3122_amd import _lib  # noqa: E402

DEV = torch.device("cuda:0")
MAX_NQ = 1048576   # FEM_NOALLOC_MAX_NQ


def _up(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _call(noalloc, pat, q, w, flags, lam=1.0, mu=0.5):
    lib = _lib.load()
    out = {k: torch.full((n * pat.nnz,), np.nan, dtype=torch.float64, device=DEV)
           for k, n in (("M", 1), ("Mw", 1), ("S", 1), ("K", 4))}
    s = torch.cuda.current_stream().cuda_stream
    head = (15, pat.nq, pat.nme, pat.nnz, q.data_ptr(), w.data_ptr(), pat.me.data_ptr(),
            *pat.args(), float(lam), float(mu), out["M"].data_ptr(), out["Mw"].data_ptr(),
            out["S"].data_ptr(), out["K"].data_ptr())
    if noalloc:
        st = lib.fem_assemble_noalloc(*head, None, flags, s)
    else:
        ws = C.c_size_t(0)
        _lib.check(lib.fem_assemble_workspace(pat.nq, 15, C.byref(ws)))
        work = torch.empty(int(ws.value), dtype=torch.uint8, device=DEV)
        st = lib.fem_assemble(*head, work.data_ptr(), int(ws.value), None, flags, s)
    torch.cuda.synchronize()
    return st, out


@pytest.mark.parametrize("flags", [0, _lib.FEM_CHECK_AREA])
def test_noalloc_matches_fem_assemble(flags):
    for n, seed in ((96, 5), (24, 6)):          # the second call on a smaller mesh
        m = mg.unit_square(n, seed=seed)
        print(f"[case] noalloc square{n} nq={m.nq} flags={flags}", flush=True)
        w = mg.weight_quadratic(m.q)
        pat = fem.fem_pattern(_up(m.me), m.nq)
        q, wd = _up(m.q), _up(w)
        st0, ref = _call(False, pat, q, wd, flags)
        st1, got = _call(True, pat, q, wd, flags)
        assert st0 == _lib.FEM_OK and st1 == _lib.FEM_OK, _lib.load().fem_last_error()
        for k in ref:
            assert torch.equal(got[k], ref[k]), (n, k)
        P = oracle.pattern(m.nq, m.me)
        assert row_rel_err(P.row_ptr, got["Mw"].cpu().numpy(),
                           oracle.assemble("wmass", m.q, m.me, P.slot, P.nnz, w=w)) <= RTOL_ROW


def test_noalloc_area_flag_is_cleared_between_calls():
    # a mesh with a zero-area triangle reports FEM_EDEGEN; the next call on a
    # valid mesh must not see that call's flag
    q = np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0], [0.0, 1.0]])
    me = np.array([[0, 1, 3], [0, 1, 2]], np.int32)
    pat = fem.fem_pattern(_up(me), 4)
    st, _ = _call(True, pat, _up(q), _up(np.ones(4)), _lib.FEM_CHECK_AREA)
    assert st == _lib.FEM_EDEGEN
    m = mg.unit_square(8, seed=2)
    pat = fem.fem_pattern(_up(m.me), m.nq)
    st, got = _call(True, pat, _up(m.q), _up(np.ones(m.nq)), _lib.FEM_CHECK_AREA)
    assert st == _lib.FEM_OK
    assert bool(torch.isfinite(got["S"]).all())


def test_noalloc_limits_are_checked_on_the_host():
    lib = _lib.load()
    fake = C.c_void_p(0x1000)   # never dereferenced: the checks fail first
    # q, w, me, row_ptr, col_idx, inc_ptr, inc_pos, fan; slot, lambda, mu; the four outputs; tune
    args = [fake] * 8 + [None, 1.0, 0.5, fake, fake, fake, fake, None]
    st = lib.fem_assemble_noalloc(fem.FEM_OP_WMASS, MAX_NQ + 1, 2, 10, *args, 0, None)
    assert st == _lib.FEM_ENOSPC and b"noalloc" in lib.fem_last_error()
    st = lib.fem_assemble_noalloc(fem.FEM_OP_WMASS, 16, 2, 10, *args, _lib.FEM_PACKED_QW, None)
    assert st == _lib.FEM_EINVAL
