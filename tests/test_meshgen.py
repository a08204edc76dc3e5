"""Invariants of the seeded synthetic meshes (inputs only)."""
import numpy as np
import pytest

from paper_1305_3122_amd import meshgen as mg


def _signed_areas(q, me):
    a, b, c = q[me[:, 0]], q[me[:, 1]], q[me[:, 2]]
    return 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1]))


@pytest.mark.parametrize("n", [1, 2, 7, 32])
def test_unit_square_counts_orientation_area(n):
    m = mg.unit_square(n, seed=n)
    assert m.nq == (n + 1) ** 2 and m.nme == 2 * n * n
    A = _signed_areas(m.q, m.me)
    assert np.all(A > 0.2 * 0.5 / n ** 2 * 0.5)  # counter-clockwise, never inverted
    assert A.sum() == pytest.approx(1.0, rel=1e-13)
    assert m.q.min() == 0.0 and m.q.max() == 1.0
    assert m.me.dtype == np.int32 and m.q.dtype == np.float64


def test_unit_square_permutation_round_trip():
    a = mg.unit_square(9, seed=5, permute=False)
    b = mg.unit_square(9, seed=5, permute=True)
    # same triangles up to the relabelling: match coordinates
    key = {tuple(p): i for i, p in enumerate(a.q)}
    pi = np.array([key[tuple(p)] for p in b.q])
    np.testing.assert_array_equal(pi[b.me], a.me)
    assert not np.array_equal(a.me, b.me)


@pytest.mark.parametrize("K", [1, 2, 8, 64])
def test_unit_disk_counts_area(K):
    m = mg.unit_disk(K, seed=K)
    assert m.nq == 1 + 3 * K * (K + 1) and m.nme == 6 * K * K
    A = _signed_areas(m.q, m.me)
    assert np.all(A > 0)
    N = 6 * K
    assert A.sum() == pytest.approx(N / 2 * np.sin(2 * np.pi / N), rel=1e-12)
    # every vertex used, valence of interior vertices 5..7
    deg = np.bincount(m.me.reshape(-1), minlength=m.nq)
    assert deg.min() >= 1


def test_batch_offsets():
    b = mg.batch_of_squares(6, 8, 20, seed=3)
    assert b.nb == 6 and b.vtx_off[-1] == b.q.shape[0] and b.elem_off[-1] == b.me.shape[0]
    for i in range(b.nb):
        e0, e1 = b.elem_off[i], b.elem_off[i + 1]
        assert np.all(b.me[e0:e1] >= b.vtx_off[i]) and np.all(b.me[e0:e1] < b.vtx_off[i + 1])
        np.testing.assert_array_equal(b.me[e0:e1] - b.vtx_off[i], b.me_local[e0:e1])
        assert e1 - e0 == 2 * b.sizes[i] ** 2


def test_seeded_reproducible():
    a = mg.config_mesh(1)
    b = mg.config_mesh(1)
    np.testing.assert_array_equal(a.q, b.q)
    np.testing.assert_array_equal(a.me, b.me)
    assert (a.nq, a.nme) == (1089, 2048)
