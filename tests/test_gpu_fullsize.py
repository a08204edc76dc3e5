"""Full-size parity on the benchmark workloads, against the oracle.

The 2048 x 2048-cell square (8.4M triangles), the 1024-ring disk (6.3M) and
the batch of 512 squares (31.8M triangles, one block-diagonal pattern): every
integer output of the symbolic phase bit for bit (row_ptr, col_idx, inc_ptr,
inc, slot, the elasticity pattern; inc_pos and the fan codes by what they
must index), and every row of every operator within 1e-13 (per-row max norm)
of the oracle's CSR values -- the storage of Section 4 filled with the sums
sparse() forms in Section 6.
"""
import numpy as np
import pytest

import oracle
from paper_1305_3122_amd import meshgen as mg
from tests.helpers import RTOL_ROW, check_fan_codes_vec, row_rel_err_fast

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1305_3122_amd as fem  # noqa: E402

DEV = torch.device("cuda:0")


def _up(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _np(t):
    return t.detach().cpu().numpy()


def _check_inc_pos(pat, P, me):
    """inc_pos names, inside row v, the next and previous vertex of each of
    v's triangles (vectorised)."""
    pos = _np(pat.inc_pos).view(np.uint32)
    p1 = (pos & 0xFFFF).astype(np.int64)
    p2 = (pos >> 16).astype(np.int64)
    v = np.repeat(np.arange(P.nq), np.diff(P.inc_ptr))
    k, a = P.inc // 3, P.inc % 3
    rs = P.row_ptr[v].astype(np.int64)
    np.testing.assert_array_equal(P.col_idx[rs + p1], me[k, (a + 1) % 3])
    np.testing.assert_array_equal(P.col_idx[rs + p2], me[k, (a + 2) % 3])


def _check_full_mesh(m, lam, mu, w):
    print(f"[case] {m.name} nq={m.nq} nme={m.nme}", flush=True)
    P = oracle.pattern(m.nq, m.me)
    pat = fem.fem_pattern(_up(m.me), m.nq, slot=True)
    torch.cuda.synchronize()
    # ---- symbolic phase, bit for bit
    assert pat.nnz == P.nnz == m.nq + 2 * (m.nq + m.nme - 1)   # Euler, simply connected
    np.testing.assert_array_equal(_np(pat.row_ptr), P.row_ptr)
    np.testing.assert_array_equal(_np(pat.col_idx), P.col_idx)
    np.testing.assert_array_equal(_np(pat.inc_ptr), P.inc_ptr)
    np.testing.assert_array_equal(_np(pat.inc), P.inc)
    np.testing.assert_array_equal(_np(pat.slot), P.slot)
    _check_inc_pos(pat, P, m.me)
    # every row of these consistently oriented meshes has a fan code
    assert check_fan_codes_vec(_np(pat.fan), P.row_ptr, P.col_idx, m.me, m.nq) == m.nq
    rpe, cie, se = oracle.pattern_elas(m.nq, m.me)
    grpe, gcie = fem.fem_elas_pattern(pat)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(grpe), rpe)
    np.testing.assert_array_equal(_np(gcie), cie)
    del grpe, gcie, cie
    # ---- numeric phase: every row of every operator
    qd, wd = _up(m.q), _up(w)
    allv = fem.fem_assemble(pat, qd, 15, w=wd, lam=lam, mu=mu)
    single = {"M": fem.fem_assemble_mass(pat, qd), "Mw": fem.fem_assemble_wmass(pat, qd, wd),
              "S": fem.fem_assemble_stiff(pat, qd), "K": fem.fem_assemble_elas(pat, qd, lam, mu)}
    S2, M2 = fem.fem_assemble_stiff_mass(pat, qd)
    torch.cuda.synchronize()
    for k in single:
        assert torch.equal(allv[k], single[k]), k      # fused = single-operator calls
    assert torch.equal(S2, single["S"]) and torch.equal(M2, single["M"])
    del single, S2, M2
    got = {k: _np(v) for k, v in allv.items()}
    del allv
    ref = {"M": oracle.assemble("mass", m.q, m.me, P.slot, P.nnz),
           "Mw": oracle.assemble("wmass", m.q, m.me, P.slot, P.nnz, w=w),
           "S": oracle.assemble("stiff", m.q, m.me, P.slot, P.nnz)}
    for k in ref:
        err = row_rel_err_fast(P.row_ptr, got[k], ref[k])
        print(f"   {k}: max row error {err:.2e}", flush=True)
        assert err <= RTOL_ROW, k
    Kref = oracle.assemble("elas", m.q, m.me, se, int(rpe[-1]), lam=lam, mu=mu)
    err = row_rel_err_fast(rpe, got["K"], Kref)
    print(f"   K: max row error {err:.2e}", flush=True)
    assert err <= RTOL_ROW
    # ---- the ascending-order path (no fan codes) meets the same bar
    pat0 = fem.Pattern(**{**pat.__dict__, "fan": None})
    S0, M0 = fem.fem_assemble_stiff_mass(pat0, qd)
    torch.cuda.synchronize()
    assert row_rel_err_fast(P.row_ptr, _np(S0), ref["S"]) <= RTOL_ROW
    assert row_rel_err_fast(P.row_ptr, _np(M0), ref["M"]) <= RTOL_ROW
    # ---- the atomic scheme through the slot map
    Sa, Ma = fem.fem_assemble_stiff_mass(pat, qd, flags=fem.FEM_ATOMIC)
    torch.cuda.synchronize()
    assert row_rel_err_fast(P.row_ptr, _np(Sa), ref["S"]) <= RTOL_ROW
    assert row_rel_err_fast(P.row_ptr, _np(Ma), ref["M"]) <= RTOL_ROW


@pytest.mark.timeout(900)
def test_square2048_full_parity():
    m = mg.config_mesh(2)
    _check_full_mesh(m, 1.0, 0.5, mg.weight_quadratic(m.q))


@pytest.mark.timeout(900)
def test_disk1024_full_parity():
    m = mg.config_mesh(3)
    _check_full_mesh(m, 2.0, 1.0, mg.weight_quadratic(m.q))


@pytest.mark.timeout(900)
def test_batch512_full_parity():
    # 512 squares of log-uniform size, globalised on the GPU, one pattern and
    # one batched S + M launch over all blocks (default and autotuned launch
    # shapes, and replayed from a HIP graph), against the oracle on the
    # global connectivity
    b = mg.config_mesh(4)
    nq = int(b.vtx_off[-1])
    print(f"[case] batch512 nb={b.nb} nq={nq} nme={b.me.shape[0]}", flush=True)
    me_g = fem.fem_batch_globalize(_up(b.me_local), _up(b.vtx_off), _up(b.elem_off))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(me_g), b.me)
    pat = fem.fem_pattern(me_g, nq)
    torch.cuda.synchronize()
    P = oracle.pattern(nq, b.me)
    assert pat.nnz == P.nnz
    np.testing.assert_array_equal(_np(pat.row_ptr), P.row_ptr)
    np.testing.assert_array_equal(_np(pat.col_idx), P.col_idx)
    np.testing.assert_array_equal(_np(pat.inc_ptr), P.inc_ptr)
    np.testing.assert_array_equal(_np(pat.inc), P.inc)
    _check_inc_pos(pat, P, b.me)
    # block-diagonal: no entry leaves its mesh's vertex range
    rows = np.repeat(np.arange(nq), np.diff(P.row_ptr))
    blk = np.searchsorted(b.vtx_off, rows, side="right") - 1
    assert np.all((P.col_idx >= b.vtx_off[blk]) & (P.col_idx < b.vtx_off[blk + 1]))
    del rows, blk
    assert check_fan_codes_vec(_np(pat.fan), P.row_ptr, P.col_idx, b.me, nq) == nq
    q = _up(b.q)
    S, M = fem.fem_assemble_stiff_mass_batched(pat, q, b.nb)
    from paper_1305_3122_amd import autotune
    tune, _ = autotune.tune_batched(fem, torch, pat, q, b.nb, reps=1, use_cache=False)
    St, Mt = fem.fem_assemble_stiff_mass_batched(pat, q, b.nb, tune=tune)
    side = torch.cuda.Stream()
    Sg = torch.full_like(S, np.nan)
    Mg = torch.full_like(M, np.nan)
    torch.cuda.synchronize()
    g = fem.Graph(side)
    with torch.cuda.stream(side):
        with g.capture():
            fem.fem_assemble_stiff_mass_batched(pat, q, b.nb, tune=tune, out_S=Sg, out_M=Mg,
                                                stream=side)
    for rep in range(2):
        Sg.fill_(-1.0)
        Mg.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay(side)
        side.synchronize()
        assert torch.equal(Sg, S) and torch.equal(Mg, M), rep
    assert torch.equal(St, S) and torch.equal(Mt, M)
    Sh, Mh = _np(S), _np(M)
    del S, M, St, Mt, Sg, Mg
    for name, got in (("stiff", Sh), ("mass", Mh)):
        ref = oracle.assemble(name, b.q, b.me, P.slot, P.nnz)
        err = row_rel_err_fast(P.row_ptr, got, ref)
        print(f"   {name}: max row error {err:.2e}", flush=True)
        assert err <= RTOL_ROW, name
