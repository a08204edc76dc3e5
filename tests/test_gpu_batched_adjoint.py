"""GPU tests of the batched (block-diagonal) path, HIP graph replay and the
hand-written adjoint, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1305_3122_amd import meshgen as mg
from tests.helpers import RTOL_ROW, fan_mesh, row_rel_err

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


@pytest.fixture(scope="module")
def batch():
    b = mg.batch_of_squares(48, 4, 40, seed=77)
    me_g = fem.fem_batch_globalize(_up(b.me_local), _up(b.vtx_off), _up(b.elem_off))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(me_g), b.me)
    pat = fem.fem_pattern(me_g, int(b.vtx_off[-1]))
    return b, pat


def test_batched_blocks_equal_single_mesh(batch):
    b, pat = batch
    q = _up(b.q)
    S, M = fem.fem_assemble_stiff_mass_batched(pat, q, b.nb)
    torch.cuda.synchronize()
    rp, ci, Sh, Mh = _np(pat.row_ptr), _np(pat.col_idx), _np(S), _np(M)
    for i in range(b.nb):
        m = b.mesh(i)
        v0, v1 = int(b.vtx_off[i]), int(b.vtx_off[i + 1])
        pm = fem.fem_pattern(_up(m.me), m.nq)
        Sm, Mm = fem.fem_assemble_stiff_mass(pm, _up(m.q))
        torch.cuda.synchronize()
        e0, e1 = rp[v0], rp[v1]
        # block i of the batched pattern == pattern of mesh i, shifted
        np.testing.assert_array_equal(rp[v0:v1 + 1] - e0, _np(pm.row_ptr))
        np.testing.assert_array_equal(ci[e0:e1] - v0, _np(pm.col_idx))
        # same kernel, same order of additions: bitwise equal values
        np.testing.assert_array_equal(Sh[e0:e1], _np(Sm))
        np.testing.assert_array_equal(Mh[e0:e1], _np(Mm))
        if i % 12 == 0:
            P = oracle.pattern(m.nq, m.me)
            assert row_rel_err(P.row_ptr, _np(Sm), oracle.assemble("stiff", m.q, m.me, P.slot, P.nnz)) <= RTOL_ROW
            assert row_rel_err(P.row_ptr, _np(Mm), oracle.assemble("mass", m.q, m.me, P.slot, P.nnz)) <= RTOL_ROW


# every compiled tile size (LDS entries 256, 448, 512, 640, 768, 1024 -> 4, 7,
# 8, 10, 12, 16 per lane), persistent and not
TUNES = [(256, 0), (448, 64), (512, 0), (512, 256), (640, 0), (640, 512), (768, 1024),
         (1024, 37), (384, 64)]


@pytest.mark.parametrize("tune", TUNES)
def test_batched_tunings_agree(batch, tune):
    b, pat = batch
    q = _up(b.q)
    S0, M0 = fem.fem_assemble_stiff_mass(pat, q)
    S1, M1 = fem.fem_assemble_stiff_mass_batched(pat, q, b.nb, tune=fem.fem_tune(*tune))
    assert torch.equal(S0, S1) and torch.equal(M0, M1)
    # without fan codes the register kernel sums in ascending triangle order,
    # the same bits for every launch shape
    pat0 = fem.Pattern(**{**pat.__dict__, "fan": None})
    S2, M2 = fem.fem_assemble_stiff_mass(pat0, q)
    S3, M3 = fem.fem_assemble_stiff_mass_batched(pat0, q, b.nb, tune=fem.fem_tune(*tune))
    assert torch.equal(S2, S3) and torch.equal(M2, M3)


@pytest.mark.parametrize("tune", [(512, 0), (256, 64), (1024, 0)])
def test_lds_accumulator_variant(batch, tune):
    # variant 1 keeps the row accumulators in LDS and sums in ascending
    # triangle order: the same bits as the register kernel without fan codes,
    # and the oracle's values within the tolerance
    b, pat = batch
    q = _up(b.q)
    pat0 = fem.Pattern(**{**pat.__dict__, "fan": None})
    S0, M0 = fem.fem_assemble_stiff_mass(pat0, q)
    S1, M1 = fem.fem_assemble_stiff_mass_batched(pat, q, b.nb, tune=fem.fem_tune(*tune, 1))
    w = _up(mg.weight_quadratic(b.q))
    a = fem.fem_assemble(pat0, q, 15, w=w, lam=1.0, mu=0.5)
    c = fem.fem_assemble(pat, q, 15, w=w, lam=1.0, mu=0.5, tune=fem.fem_tune(*tune, 1))
    torch.cuda.synchronize()
    assert torch.equal(S0, S1) and torch.equal(M0, M1)
    for k in a:
        assert torch.equal(a[k], c[k]), k
    P = oracle.pattern(int(b.vtx_off[-1]), b.me)
    assert row_rel_err(P.row_ptr, _np(S1), oracle.assemble("stiff", b.q, b.me, P.slot, P.nnz)) <= RTOL_ROW
    assert row_rel_err(P.row_ptr, _np(M1), oracle.assemble("mass", b.q, b.me, P.slot, P.nnz)) <= RTOL_ROW


def test_autotuner_pick(batch):
    # the autotuner times its candidates on the pattern and returns one of
    # them; the pick gives the default launch's bits
    from paper_1305_3122_amd import autotune
    b, pat = batch
    q = _up(b.q)
    tune, table = autotune.tune_batched(fem, torch, pat, q, b.nb, reps=1, use_cache=False)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    assert len(table) == len(autotune.LDS_ENTRIES) * len(autotune.GRID_PER_CU)
    assert tune.lds_entries in autotune.LDS_ENTRIES
    assert tune.grid_blocks in [g * n_cu for g in autotune.GRID_PER_CU]
    assert f"{tune.lds_entries}/{tune.grid_blocks}" in table
    S0, M0 = fem.fem_assemble_stiff_mass(pat, q)
    S1, M1 = fem.fem_assemble_stiff_mass_batched(pat, q, b.nb, tune=tune)
    assert torch.equal(S0, S1) and torch.equal(M0, M1)


def test_graph_replay_matches_eager(batch):
    b, pat = batch
    q = _up(b.q)
    S_ref, M_ref = fem.fem_assemble_stiff_mass_batched(pat, q, b.nb)
    side = torch.cuda.Stream()
    S = torch.full_like(S_ref, np.nan)
    M = torch.full_like(M_ref, np.nan)
    torch.cuda.synchronize()
    g = fem.Graph(side)
    with torch.cuda.stream(side):
        with g.capture():
            fem.fem_assemble_stiff_mass_batched(pat, q, b.nb, out_S=S, out_M=M, stream=side)
    side.synchronize()
    for rep in range(4):
        S.zero_()
        M.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay(side)
        side.synchronize()
        assert torch.equal(S, S_ref), rep
        assert torch.equal(M, M_ref), rep
        # eager work between replays
        fem.fem_assemble_stiff(pat, q)
        torch.cuda.synchronize()


def test_graph_replay_of_atomic_path_clears_values():
    m = mg.unit_square(24, seed=4)
    pat = fem.fem_pattern(_up(m.me), m.nq, slot=True)
    q = _up(m.q)
    S_ref = fem.fem_assemble_stiff(pat, q, flags=fem.FEM_ATOMIC)
    side = torch.cuda.Stream()
    S = torch.full_like(S_ref, 123.0)
    torch.cuda.synchronize()
    g = fem.Graph(side)
    with torch.cuda.stream(side):
        with g.capture():
            fem.fem_assemble_stiff(pat, q, out=S, flags=fem.FEM_ATOMIC, stream=side)
    for rep in range(3):
        S.fill_(7.0)
        torch.cuda.synchronize()
        g.replay(side)
        side.synchronize()
        assert float((S - S_ref).abs().max()) <= 1e-13 * float(S_ref.abs().max()), rep


# ------------------------------------------------------------------ adjoint

@pytest.fixture(scope="module")
def cfg5():
    m = mg.config_mesh(5)
    w = mg.weight_uniform(m.nq, 0.5, 2.0, seed=mg.BASE_SEED + 5)
    P = oracle.pattern(m.nq, m.me)
    G = mg.normal_seed(P.nnz, seed=mg.BASE_SEED + 55)
    pat = fem.fem_pattern(_up(m.me), m.nq)
    return m, w, P, G, pat


def test_adjoint_matches_oracle(cfg5):
    m, w, P, G, pat = cfg5
    print(f"[case] adjoint cfg5 nnz={P.nnz}", flush=True)
    q, wd, Gd = _up(m.q), _up(w), _up(G)
    rdq, rdw = oracle.adjoint_stiff_wmass(m.q, m.me, w, P.slot, G, G)
    for tp in (None, "map"):
        if tp == "map":
            fem.fem_transpose_map(pat)
        dq, dw = fem.fem_adjoint_stiff_wmass(pat, q, wd, Gd, Gd)
        torch.cuda.synchronize()
        assert np.max(np.abs(_np(dq) - rdq)) <= 1e-13 * np.max(np.abs(rdq))
        assert np.max(np.abs(_np(dw) - rdw)) <= 1e-13 * np.max(np.abs(rdw))
    # single terms
    dqS, _ = fem.fem_adjoint_stiff_wmass(pat, q, None, Gd, None)
    rS, _ = oracle.adjoint_stiff_wmass(m.q, m.me, w, P.slot, G, None)
    torch.cuda.synchronize()
    assert np.max(np.abs(_np(dqS) - rS)) <= 1e-13 * np.max(np.abs(rS))
    pat.tpos = None


@pytest.mark.parametrize("n_fan", [12, 40])
def test_adjoint_long_rows(n_fan):
    # the hub of a fan has a row longer than the register path: pass 1 sums
    # it in memory, at the transposed places when the transpose map is given;
    # both variants against the oracle and bitwise against each other
    q0, me = fan_mesh(n_fan, 2, seed=n_fan)
    nq = q0.shape[0]
    w = mg.weight_uniform(nq, 0.5, 2.0, seed=mg.BASE_SEED + n_fan)
    P = oracle.pattern(nq, me)
    G = mg.normal_seed(P.nnz, seed=mg.BASE_SEED + 60 + n_fan)
    rdq, rdw = oracle.adjoint_stiff_wmass(q0, me, w, P.slot, G, G)
    pat = fem.fem_pattern(_up(me), nq)
    q, wd, Gd = _up(q0), _up(w), _up(G)
    dq_s, dw_s = fem.fem_adjoint_stiff_wmass(pat, q, wd, Gd, Gd)
    fem.fem_transpose_map(pat)
    dq_t, dw_t = fem.fem_adjoint_stiff_wmass(pat, q, wd, Gd, Gd)
    torch.cuda.synchronize()
    assert np.max(np.abs(_np(dq_t) - rdq)) <= 1e-13 * np.max(np.abs(rdq))
    assert np.max(np.abs(_np(dw_t) - rdw)) <= 1e-13 * np.max(np.abs(rdw))
    assert torch.equal(dq_t, dq_s) and torch.equal(dw_t, dw_s)


def test_adjoint_variants_bitwise_equal(cfg5):
    # tpos or search, packed records from the forward or packed here, fresh or
    # reused workspace: the same sums in the same order
    m, w, P, G, pat = cfg5
    q, wd, Gd = _up(m.q), _up(w), _up(G)
    pat.tpos = None
    ref = fem.fem_adjoint_stiff_wmass(pat, q, wd, Gd, Gd)
    fem.fem_transpose_map(pat)
    work = fem.fem_adjoint_workspace(pat)
    fem.fem_assemble(pat, q, fem.FEM_OP_STIFF | fem.FEM_OP_WMASS, w=wd, work=work)
    for packed in (True, False, True):
        got = fem.fem_adjoint_stiff_wmass(pat, q, wd, Gd, Gd, work=work, packed=packed)
        torch.cuda.synchronize()
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), packed
    # accumulate adds into the outputs
    dq, dw = ref[0].clone(), ref[1].clone()
    fem.fem_adjoint_stiff_wmass(pat, q, wd, Gd, Gd, dq=dq, dw=dw, flags=fem.FEM_ACCUMULATE)
    assert torch.equal(dq, 2 * ref[0]) and torch.equal(dw, 2 * ref[1])
    pat.tpos = None


def test_adjoint_central_differences(cfg5):
    # central differences of L on 64 random coordinates (h = 1e-6 for q); L restricted
    # to the rows the perturbed vertex touches (the other values are computed
    # from unchanged inputs in a fixed order, so they cancel exactly)
    m, w, P, G, pat = cfg5
    q0 = _up(m.q)
    wd, Gd = _up(w), _up(G)
    dq, dw = fem.fem_adjoint_stiff_wmass(pat, q0, wd, Gd, Gd)
    dq, dw = _np(dq), _np(dw)
    rp, ci = P.row_ptr, P.col_idx
    rng = np.random.default_rng(64)
    h = 1e-6
    verts = rng.choice(m.nq, size=64, replace=False)
    comps = rng.integers(0, 3, size=64)
    for v, c in zip(verts, comps):
        rows = ci[rp[v]:rp[v + 1]]          # v and its neighbours
        sel = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
        seld = torch.from_numpy(sel).to(DEV)

        def L(qa, wa, only_w=False):
            S, Mw = fem.fem_assemble_stiff_wmass(pat, qa, wa)
            if only_w:
                # S does not depend on w; leaving it out keeps the O(1)
                # stiffness terms from rounding away the w-part of L
                return float((Gd[seld] * Mw[seld]).sum())
            return float((Gd[seld] * (S[seld] + Mw[seld])).sum())

        if c < 2:
            def fd(step):
                qp, qm = m.q.copy(), m.q.copy()
                qp[v, c] += step
                qm[v, c] -= step
                return (L(_up(qp), wd) - L(_up(qm), wd)) / (2 * step)

            f1 = fd(h)
            assert dq[v, c] == pytest.approx(f1, rel=1e-6, abs=1e-6 * np.abs(dq).max()), (v, c)
            # one Richardson step removes the h^2 term of the central difference
            fr = (4 * fd(h / 2) - f1) / 3
            assert dq[v, c] == pytest.approx(fr, rel=1e-6, abs=1e-9 * np.abs(dq).max()), (v, c)
        else:
            # L is linear in w: a unit step is exact up to rounding
            wp, wm = w.copy(), w.copy()
            wp[v] += 1.0
            wm[v] -= 1.0
            fd = (L(q0, _up(wp), True) - L(q0, _up(wm), True)) / 2.0
            assert dw[v] == pytest.approx(fd, rel=1e-8, abs=1e-12 * np.abs(dw).max()), v


def test_autograd_function(cfg5):
    m, w, P, G, pat = cfg5
    q = _up(m.q).requires_grad_(True)
    wd = _up(w).requires_grad_(True)
    Gd = _up(G)
    S, Mw = fem.AssembleStiffWMass.apply(q, wd, pat)
    Lv = (Gd * S).sum() + (Gd * Mw).sum()
    gq, gw = torch.autograd.grad(Lv, (q, wd))
    dq, dw = fem.fem_adjoint_stiff_wmass(pat, q.detach(), wd.detach(), Gd, Gd)
    assert torch.equal(gq, dq) and torch.equal(gw, dw)
    # invariants of the exact gradient: translation and rotation
    gqh = _np(gq)
    scale = np.abs(gqh).max()
    assert np.abs(gqh.sum(axis=0)).max() <= 1e-9 * scale
    assert abs(np.sum(m.q[:, 0] * gqh[:, 1] - m.q[:, 1] * gqh[:, 0])) <= 1e-9 * scale
