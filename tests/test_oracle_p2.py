"""Pins of the oracle's P2 (quadratic Lagrange) triangle assembly (no GPU).

Each check ties the oracle to something other than its own barycentric
integration:
- the textbook element matrices of the reference right triangle;
- a Lagrange basis built by a different route: monomials in x, y with a
  Vandermonde solve at the vertices and the edge midpoints, integrated by a
  collapsed Gauss-Legendre rule that is exact for these degrees;
- the exactness of P2 for quadratic fields: u^T M u is the integral of u^2 and
  u^T S u the integral of |grad u|^2 over the unit square;
- Euler's count of the edges and a closed form for nnz;
- a dense brute-force assembly on tiny meshes."""
import numpy as np
import pytest

import oracle
from paper_1305_3122_amd import meshgen as mg

REF = [np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.0, 1.0])]

# The quadratic triangle on (0,0), (1,0), (0,1), local order: the vertices,
# then the midpoint of the edge opposite vertex 0, 1, 2 (the standard tables
# of the P2 Lagrange element, rearranged to that order).
REF_MASS_360 = np.array([[6, -1, -1, -4, 0, 0],
                         [-1, 6, -1, 0, -4, 0],
                         [-1, -1, 6, 0, 0, -4],
                         [-4, 0, 0, 32, 16, 16],
                         [0, -4, 0, 16, 32, 16],
                         [0, 0, -4, 16, 16, 32]], float)
REF_STIFF_6 = np.array([[6, 1, 1, 0, -4, -4],
                        [1, 3, 0, 0, 0, -4],
                        [1, 0, 3, 0, -4, 0],
                        [0, 0, 0, 16, -8, -8],
                        [-4, 0, -4, -8, 16, 0],
                        [-4, -4, 0, -8, 0, 16]], float)


def test_reference_triangle_matrices():
    np.testing.assert_allclose(oracle.elem_p2_mass(0.5) * 360, REF_MASS_360, atol=1e-13)
    np.testing.assert_allclose(oracle.elem_p2_stiff(*REF) * 6, REF_STIFF_6, atol=1e-13)


# ---- an independent construction of the element matrices ------------------

def _nodes(x):
    x0, x1, x2 = x
    return [x0, x1, x2, (x1 + x2) / 2, (x2 + x0) / 2, (x0 + x1) / 2]


def _mono(p):
    x, y = p
    return np.array([1.0, x, y, x * x, x * y, y * y])


def _mono_grad(p):
    x, y = p
    return np.array([[0.0, 1.0, 0.0, 2 * x, y, 0.0], [0.0, 0.0, 1.0, 0.0, x, 2 * y]])


def _quad_rule(x, n=5):
    """Points and weights of a collapsed (Duffy) Gauss-Legendre rule on the
    triangle x: exact for polynomials of degree <= 2n - 2."""
    g, w = np.polynomial.legendre.leggauss(n)
    s, ws = (g + 1) / 2, w / 2
    x0, x1, x2 = x
    detB = abs((x1[0] - x0[0]) * (x2[1] - x0[1]) - (x2[0] - x0[0]) * (x1[1] - x0[1]))
    pts, wts = [], []
    for si, wi in zip(s, ws):
        for ti, wj in zip(s, ws):
            xi, eta = si, ti * (1 - si)
            pts.append(x0 + xi * (x1 - x0) + eta * (x2 - x0))
            wts.append(wi * wj * (1 - si) * detB)
    return pts, wts


def _elem_by_quadrature(x):
    V = np.stack([_mono(p) for p in _nodes(x)])     # V[i, m] = mono_m(node_i)
    C = np.linalg.inv(V)                            # phi_j = sum_m mono_m C[m, j]
    M = np.zeros((6, 6))
    S = np.zeros((6, 6))
    for p, wt in zip(*_quad_rule(x)):
        phi = _mono(p) @ C
        dphi = _mono_grad(p) @ C                    # [2, 6]
        M += wt * np.outer(phi, phi)
        S += wt * dphi.T @ dphi
    return M, S


def _random_triangle(rng):
    while True:
        x = [rng.uniform(-1, 1, 2) for _ in range(3)]
        if abs(oracle.det(*x)) > 0.1:
            return x


def test_lagrange_basis_is_nodal():
    # the construction above interpolates: phi_j(node_i) = delta_ij
    x = _random_triangle(np.random.default_rng(3))
    C = np.linalg.inv(np.stack([_mono(p) for p in _nodes(x)]))
    np.testing.assert_allclose(np.stack([_mono(p) @ C for p in _nodes(x)]), np.eye(6), atol=1e-12)


def test_element_matrices_match_quadrature():
    rng = np.random.default_rng(11)
    for _ in range(20):
        x = _random_triangle(rng)
        M, S = _elem_by_quadrature(x)
        area = abs(oracle.det(*x)) / 2
        np.testing.assert_allclose(oracle.elem_p2_mass(area), M, rtol=0, atol=1e-13 * np.abs(M).max())
        np.testing.assert_allclose(oracle.elem_p2_stiff(*x), S, rtol=0, atol=1e-12 * np.abs(S).max())
        # the orientation of the triangle does not matter
        Sf = oracle.elem_p2_stiff(x[0], x[2], x[1])
        perm = [0, 2, 1, 3, 5, 4]
        np.testing.assert_allclose(Sf, S[np.ix_(perm, perm)], rtol=0, atol=1e-12 * np.abs(S).max())


# ---- the degrees of freedom ----------------------------------------------------

def _meshes():
    rng = np.random.default_rng(5)
    return [mg.unit_square(1, seed=1), mg.unit_square(6, seed=2), mg.unit_disk(4, seed=3),
            mg.random_tiny_mesh(rng), mg.random_tiny_mesh(rng)]


@pytest.mark.parametrize("mi", range(5))
def test_edge_numbering(mi):
    m = _meshes()[mi]
    dofs, edges = oracle.p2_dofs(m.nq, m.me)
    np.testing.assert_array_equal(dofs[:, :3], m.me)
    assert np.all(edges[:, 0] < edges[:, 1])
    key = edges[:, 0].astype(np.int64) * m.nq + edges[:, 1]
    assert np.all(np.diff(key) > 0)                 # lexicographic, distinct
    sides = set()
    for k in range(m.nme):
        for a in range(3):
            u, v = sorted((m.me[k, (a + 1) % 3], m.me[k, (a + 2) % 3]))
            e = dofs[k, 3 + a] - m.nq
            assert (edges[e, 0], edges[e, 1]) == (u, v)
            sides.add((u, v))
    assert len(sides) == edges.shape[0]             # every edge is a side
    if mi < 3:                                      # simply connected: Euler
        assert edges.shape[0] == m.nq + m.nme - 1


def _poly_mul(a, b):
    out = {}
    for (i1, j1), c1 in a.items():
        for (i2, j2), c2 in b.items():
            out[(i1 + i2, j1 + j2)] = out.get((i1 + i2, j1 + j2), 0.0) + c1 * c2
    return out


def _int_square(p):
    return sum(c / ((i + 1) * (j + 1)) for (i, j), c in p.items())


def _poly_eval(p, x, y):
    return sum(c * x ** i * y ** j for (i, j), c in p.items())


def _dof_points(q, edges):
    return np.concatenate([q, (q[edges[:, 0]] + q[edges[:, 1]]) / 2])


def _dense(rp, ci, v, n):
    A = np.zeros((n, n))
    A[np.repeat(np.arange(n), np.diff(rp)), ci] = v
    return A


def test_quadratic_fields_are_exact_on_the_square():
    m = mg.unit_square(6, seed=7)
    rpM, ciM, M, dofs, edges = oracle.assemble_p2("mass", m.q, m.me)
    rpS, ciS, S, _, _ = oracle.assemble_p2("stiff", m.q, m.me)
    n = m.nq + edges.shape[0]
    np.testing.assert_array_equal(rpM, rpS)
    np.testing.assert_array_equal(ciM, ciS)
    Md, Sd = _dense(rpM, ciM, M, n), _dense(rpS, ciS, S, n)
    assert M.sum() == pytest.approx(1.0, rel=1e-13)
    np.testing.assert_allclose(Md, Md.T, atol=1e-15)
    np.testing.assert_allclose(Sd, Sd.T, atol=1e-13)
    np.testing.assert_allclose(Sd.sum(axis=1), 0.0, atol=1e-12)
    pts = _dof_points(m.q, edges)
    rng = np.random.default_rng(8)
    for _ in range(3):
        c = rng.standard_normal(6)
        u = {(0, 0): c[0], (1, 0): c[1], (0, 1): c[2], (2, 0): c[3], (1, 1): c[4], (0, 2): c[5]}
        ux = {(0, 0): c[1], (1, 0): 2 * c[3], (0, 1): c[4]}
        uy = {(0, 0): c[2], (1, 0): c[4], (0, 1): 2 * c[5]}
        U = _poly_eval(u, pts[:, 0], pts[:, 1])
        assert U @ Md @ U == pytest.approx(_int_square(_poly_mul(u, u)), rel=1e-12)
        grad2 = _int_square(_poly_mul(ux, ux)) + _int_square(_poly_mul(uy, uy))
        assert U @ Sd @ U == pytest.approx(grad2, rel=1e-11)


def test_disk_area_and_null_space():
    m = mg.unit_disk(4, seed=9)
    rp, ci, M, dofs, edges = oracle.assemble_p2("mass", m.q, m.me)
    _, _, S, _, _ = oracle.assemble_p2("stiff", m.q, m.me)
    N = 6 * 4
    assert M.sum() == pytest.approx(N / 2 * np.sin(2 * np.pi / N), rel=1e-13)
    n = m.nq + edges.shape[0]
    rows = np.repeat(np.arange(n), np.diff(rp))
    rs = np.bincount(rows, weights=S, minlength=n)
    assert np.abs(rs).max() <= 1e-12 * np.abs(S).max()
    # the P2 vertex functions integrate to zero, the edge functions to |T| / 3
    rsM = np.bincount(rows, weights=M, minlength=n)
    assert np.abs(rsM[:m.nq]).max() <= 1e-15
    tri_area = np.zeros(edges.shape[0])
    for k in range(m.nme):
        a = abs(oracle.det(*m.q[m.me[k]])) / 2
        tri_area[dofs[k, 3:] - m.nq] += a / 3
    np.testing.assert_allclose(rsM[m.nq:], tri_area, rtol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_nnz_closed_form(n):
    # pairs of DOFs sharing a triangle: 15 per triangle, minus the 3 pairs on
    # each interior edge (counted by both of its triangles)
    m = mg.unit_square(n, seed=n)
    rp, ci, _, _, edges = oracle.assemble_p2("mass", m.q, m.me)
    ne = edges.shape[0]
    assert ne == 3 * n * n + 2 * n
    e_int = ne - 4 * n
    assert ci.shape[0] == m.nq + ne + 2 * (15 * m.nme - 3 * e_int)


def test_brute_force_dense_assembly():
    rng = np.random.default_rng(21)
    for _ in range(4):
        m = mg.random_tiny_mesh(rng)
        for op in ("mass", "stiff"):
            rp, ci, v, dofs, edges = oracle.assemble_p2(op, m.q, m.me)
            n = m.nq + edges.shape[0]
            D = np.zeros((n, n))
            touched = np.zeros((n, n), bool)
            for k in range(m.nme):
                x = m.q[m.me[k]]
                E = oracle.elem_p2_mass(abs(oracle.det(*x)) / 2) if op == "mass" else oracle.elem_p2_stiff(*x)
                d = dofs[k]
                D[np.ix_(d, d)] += E
                touched[np.ix_(d, d)] = True
            A = _dense(rp, ci, v, n)
            np.testing.assert_array_equal(_dense(rp, ci, np.ones_like(v), n) > 0, touched)
            np.testing.assert_allclose(A, D, rtol=0, atol=1e-14 * np.abs(D).max())


def test_invalid_meshes_are_rejected():
    q = np.zeros((4, 2))
    with pytest.raises(oracle.OracleError):
        oracle.assemble_p2("mass", q, np.array([[0, 1, 4]], np.int32))
    with pytest.raises(oracle.OracleError):
        oracle.assemble_p2("mass", q, np.array([[0, 1, 1]], np.int32))


def test_p2_incidence_brute_force():
    # the transpose of dofs against a per-DOF scan of every (k, a); on the
    # square and the disk (manifold meshes) each interior edge lies in two
    # triangles and a boundary edge in one
    rng = np.random.default_rng(13)
    for m in (mg.unit_square(3, seed=5), mg.random_tiny_mesh(rng, 25), mg.unit_disk(3, seed=6)):
        dofs, edges = oracle.p2_dofs(m.nq, m.me)
        ndof = m.nq + edges.shape[0]
        inc_ptr, inc = oracle.p2_incidence(ndof, dofs)
        assert inc_ptr[0] == 0 and inc_ptr[-1] == 6 * m.nme
        for i in range(ndof):
            want = [6 * k + a for k in range(m.nme) for a in range(6) if dofs[k, a] == i]
            np.testing.assert_array_equal(inc[inc_ptr[i]:inc_ptr[i + 1]], want)
        if m.name != "tiny":
            deg_edges = np.diff(inc_ptr)[m.nq:]
            assert set(deg_edges.tolist()) == {1, 2}
