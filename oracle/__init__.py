"""CPU oracle for P1 assembly -- TEST INFRASTRUCTURE.

A thin numpy/ctypes wrapper over ``fem_oracle.c`` (plain per-triangle loop,
triplet accumulation, Matlab ``sparse`` semantics).  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import this package; the
GPU library never does, and this package never imports the GPU library.

``build()`` compiles the C file with ``gcc -O2 -ffp-contract=off``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fem_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OP_MASS, OP_WMASS, OP_STIFF, OP_ELAS = 0, 1, 2, 3
OPS = {"mass": OP_MASS, "wmass": OP_WMASS, "stiff": OP_STIFF, "elas": OP_ELAS}

_lib = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


class OracleError(RuntimeError):
    pass


def sanitize_flags() -> list:
    """With FEM_ORACLE_SANITIZE=1 the oracle is built with AddressSanitizer and
    UndefinedBehaviorSanitizer (then run Python with libasan preloaded; see
    the sanitizer command in the repository's design notes)."""
    if os.environ.get("FEM_ORACLE_SANITIZE") == "1":
        return ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                "-fno-omit-frame-pointer", "-g"]
    return []


def build() -> str:
    """Compile liboracle.so (always), and the CPU-baseline library beside it."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-Wall", "-fPIC", *sanitize_flags(),
                    "-shared", "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    from . import cpu_baseline
    cpu_baseline.build()
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = C.CDLL(LIB)
    vp = C.c_void_p
    lib.oracle_det.restype = C.c_double
    lib.oracle_det.argtypes = [_f64p, _f64p, _f64p]
    lib.oracle_area.restype = C.c_double
    lib.oracle_area.argtypes = [_f64p, _f64p, _f64p]
    lib.oracle_elem_mass.argtypes = [C.c_double, _f64p]
    lib.oracle_elem_wmass.argtypes = [C.c_double, _f64p, _f64p]
    lib.oracle_elem_stiff.argtypes = [_f64p, _f64p, _f64p, _f64p]
    lib.oracle_elem_elas.argtypes = [_f64p, _f64p, _f64p, C.c_double, C.c_double, _f64p]
    lib.oracle_csr_pattern.restype = C.c_int64
    lib.oracle_csr_pattern.argtypes = [C.c_int32, C.c_int32, C.c_int64, _i32p, _i32p,
                                       _i32p, _i32p, _i64p]
    lib.oracle_sparse.restype = C.c_int64
    lib.oracle_sparse.argtypes = [C.c_int32, C.c_int32, C.c_int64, _i32p, _i32p, _f64p,
                                  _i32p, _i32p, _f64p]
    lib.oracle_validate.restype = C.c_int
    lib.oracle_validate.argtypes = [C.c_int32, C.c_int32, _i32p]
    lib.oracle_adjoint_elas.argtypes = [C.c_int32, C.c_int32, _f64p, _i32p, _i32p, _f64p, C.c_double,
                                        C.c_double, _f64p, _f64p]
    lib.oracle_tet_det.restype = C.c_double
    lib.oracle_tet_det.argtypes = [_f64p, _f64p, _f64p, _f64p]
    lib.oracle_elem_tet_mass.argtypes = [C.c_double, _f64p]
    lib.oracle_elem_tet_stiff.argtypes = [_f64p, _f64p, _f64p, _f64p, _f64p]
    lib.oracle_assemble_tet.restype = C.c_int64
    lib.oracle_assemble_tet.argtypes = [C.c_int, C.c_int32, C.c_int32, _f64p, _i32p, _i32p, _i32p,
                                        _f64p]
    lib.oracle_elem_p2_mass.argtypes = [C.c_double, _f64p]
    lib.oracle_elem_p2_stiff.argtypes = [_f64p, _f64p, _f64p, _f64p]
    lib.oracle_p2_dofs.restype = C.c_int64
    lib.oracle_p2_dofs.argtypes = [C.c_int32, C.c_int32, _i32p, _i32p, _i32p]
    lib.oracle_assemble_p2.restype = C.c_int64
    lib.oracle_assemble_p2.argtypes = [C.c_int, C.c_int32, C.c_int32, _f64p, _i32p, _i32p, _i32p,
                                       _i32p, _f64p]
    lib.oracle_pattern.restype = C.c_int64
    lib.oracle_pattern.argtypes = [C.c_int32, C.c_int32, _i32p, _i32p, _i32p, vp, vp, vp]
    lib.oracle_pattern_elas.restype = C.c_int64
    lib.oracle_pattern_elas.argtypes = [C.c_int32, C.c_int32, _i32p, _i32p, _i32p, vp]
    lib.oracle_assemble.restype = C.c_int
    lib.oracle_assemble.argtypes = [C.c_int, C.c_int32, C.c_int32, _f64p, _i32p, vp,
                                    C.c_double, C.c_double, _i32p, C.c_int64, _f64p]
    lib.oracle_rows.restype = C.c_int64
    lib.oracle_rows.argtypes = [C.c_int, C.c_int32, C.c_int32, _f64p, _i32p, vp,
                                C.c_double, C.c_double, C.c_int32, _i32p, _i32p, _i32p,
                                _f64p, C.c_int64]
    lib.oracle_adjoint_stiff_wmass.restype = C.c_int
    lib.oracle_adjoint_stiff_wmass.argtypes = [C.c_int32, C.c_int32, _f64p, _i32p, vp,
                                               _i32p, vp, vp, _f64p, _f64p]
    _lib = lib
    return lib


def _check(st):
    if st < 0:
        raise OracleError(f"oracle status {st}")
    return st


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---- element matrices (3x3 / 6x6 numpy arrays, E[a, b]) ------------------

def det(q1, q2, q3) -> float:
    return _load().oracle_det(_f64(q1), _f64(q2), _f64(q3))


def area(q1, q2, q3) -> float:
    return _load().oracle_area(_f64(q1), _f64(q2), _f64(q3))


def elem_mass(area_: float) -> np.ndarray:
    E = np.zeros(9)
    _load().oracle_elem_mass(float(area_), E)
    return E.reshape(3, 3).T.copy()


def elem_wmass(area_: float, w) -> np.ndarray:
    E = np.zeros(9)
    _load().oracle_elem_wmass(float(area_), _f64(w), E)
    return E.reshape(3, 3).T.copy()


def elem_stiff(q1, q2, q3) -> np.ndarray:
    E = np.zeros(9)
    _load().oracle_elem_stiff(_f64(q1), _f64(q2), _f64(q3), E)
    return E.reshape(3, 3).T.copy()


def elem_elas(q1, q2, q3, lam: float, mu: float) -> np.ndarray:
    E = np.zeros(36)
    _load().oracle_elem_elas(_f64(q1), _f64(q2), _f64(q3), float(lam), float(mu), E)
    return E.reshape(6, 6).T.copy()


# ---- sparse(I, J, V) ----------------------------------------------------------

def sparse(I, J, V, nrows: int, ncols: int):
    """Matlab sparse(I, J, V, nrows, ncols) with 0-based indices, as CSR
    (row_ptr, col_idx, values); duplicates summed, structural zeros kept."""
    I, J, V = _i32(I), _i32(J), _f64(V)
    n = I.shape[0]
    row_ptr = np.zeros(nrows + 1, np.int32)
    col_idx = np.zeros(max(n, 1), np.int32)
    vals = np.zeros(max(n, 1), np.float64)
    nnz = _check(_load().oracle_sparse(nrows, ncols, n, I, J, V, row_ptr, col_idx, vals))
    return row_ptr, col_idx[:nnz].copy(), vals[:nnz].copy()


def adjoint_elas(q, me, slot_e, G, lam: float, mu: float):
    """(dq [nq][2], dL/dlambda, dL/dmu) of L = <G, K(q; lambda, mu)> on the
    elasticity pattern whose slot map slot_e [36][nme] is given."""
    q, me, slot_e, G = _f64(q), _i32(me), _i32(slot_e), _f64(G)
    nq = q.shape[0]
    dq = np.zeros(2 * nq)
    dlm = np.zeros(2)
    _check(_load().oracle_adjoint_elas(nq, me.shape[0], q.reshape(-1), me.reshape(-1),
                                       slot_e.reshape(-1), G, float(lam), float(mu), dq, dlm))
    return dq.reshape(nq, 2), float(dlm[0]), float(dlm[1])


def tet_det(x0, x1, x2, x3) -> float:
    """det [x1 - x0 | x2 - x0 | x3 - x0] (six times the signed volume)."""
    return _load().oracle_tet_det(_f64(x0), _f64(x1), _f64(x2), _f64(x3))


def elem_tet_mass(vol: float):
    E = np.zeros(16)
    _load().oracle_elem_tet_mass(float(vol), E)
    return E.reshape(4, 4).T.copy()     # [a][b]


def elem_tet_stiff(x0, x1, x2, x3):
    E = np.zeros(16)
    _load().oracle_elem_tet_stiff(_f64(x0), _f64(x1), _f64(x2), _f64(x3), E)
    return E.reshape(4, 4).T.copy()


def assemble_tet(op: str, q, me):
    """Global P1 tetrahedron mass ("mass") or stiffness ("stiff") as CSR
    (row_ptr, col_idx, values): OptV2 triplets t = r nme + k, then sparse()."""
    q, me = _f64(q), _i32(me)
    nq, nme = q.shape[0], me.shape[0]
    row_ptr = np.zeros(nq + 1, np.int32)
    col_idx = np.zeros(max(16 * nme, 1), np.int32)
    vals = np.zeros(max(16 * nme, 1), np.float64)
    nnz = _check(_load().oracle_assemble_tet({"mass": 0, "stiff": 1}[op], nq, nme, q.reshape(-1),
                                             me.reshape(-1), row_ptr, col_idx, vals))
    return row_ptr, col_idx[:nnz].copy(), vals[:nnz].copy()


def tet_incidence(nq: int, me):
    """The tetrahedra of every vertex (the transpose of me): vertex v's are
    the ids 4 k + a with me[k][a] == v, ascending, at inc[inc_ptr[v] ..
    inc_ptr[v+1]).  Returns (inc_ptr [nq+1], inc [4 nme]) int32."""
    me = _i32(me)
    v = me.reshape(-1).astype(np.int64)          # entry 4 k + a of the flat array
    inc = np.argsort(v, kind="stable").astype(np.int32)
    inc_ptr = np.zeros(nq + 1, np.int32)
    inc_ptr[1:] = np.cumsum(np.bincount(v, minlength=nq))
    return inc_ptr, inc


def p2_incidence(ndof: int, dofs):
    """The triangles of every P2 DOF (the transpose of dofs): DOF i's are the
    ids 6 k + a with dofs[k][a] == i, ascending, at inc[inc_ptr[i] ..
    inc_ptr[i+1]).  Returns (inc_ptr [ndof+1], inc [6 nme]) int32."""
    dofs = _i32(dofs)
    v = dofs.reshape(-1).astype(np.int64)        # entry 6 k + a of the flat array
    inc = np.argsort(v, kind="stable").astype(np.int32)
    inc_ptr = np.zeros(ndof + 1, np.int32)
    inc_ptr[1:] = np.cumsum(np.bincount(v, minlength=ndof))
    return inc_ptr, inc


def elem_p2_mass(area_: float):
    """6x6 P2 mass matrix [a][b] (vertices 0..2, then the edge opposite each)."""
    E = np.zeros(36)
    _load().oracle_elem_p2_mass(float(area_), E)
    return E.reshape(6, 6).T.copy()


def elem_p2_stiff(x0, x1, x2):
    E = np.zeros(36)
    _load().oracle_elem_p2_stiff(_f64(x0), _f64(x1), _f64(x2), E)
    return E.reshape(6, 6).T.copy()


def p2_dofs(nq: int, me):
    """(dofs [nme][6], edges [ne][2]): P2 degrees of freedom, vertices first,
    then nq + e for the edge opposite each local vertex; edges numbered in
    lexicographic order of (lower, higher) vertex."""
    me = _i32(me)
    nme = me.shape[0]
    dofs = np.zeros((nme, 6), np.int32)
    edges = np.zeros((max(3 * nme, 1), 2), np.int32)
    ne = _check(_load().oracle_p2_dofs(nq, nme, me.reshape(-1), dofs.reshape(-1), edges.reshape(-1)))
    return dofs, edges[:ne].copy()


def assemble_p2(op: str, q, me):
    """Global P2 mass ("mass") or stiffness ("stiff") as CSR over nq + ne
    DOFs: (row_ptr, col_idx, values, dofs, edges); OptV2 triplets
    t = r nme + k (r = 6 b + a), then sparse()."""
    q, me = _f64(q), _i32(me)
    nq, nme = q.shape[0], me.shape[0]
    dofs, edges = p2_dofs(nq, me)
    ndof = nq + edges.shape[0]
    row_ptr = np.zeros(ndof + 1, np.int32)
    col_idx = np.zeros(max(36 * nme, 1), np.int32)
    vals = np.zeros(max(36 * nme, 1), np.float64)
    nnz = _check(_load().oracle_assemble_p2({"mass": 0, "stiff": 1}[op], ndof, nme, q.reshape(-1),
                                            me.reshape(-1), dofs.reshape(-1), row_ptr, col_idx, vals))
    return row_ptr, col_idx[:nnz].copy(), vals[:nnz].copy(), dofs, edges


def sparse_positions(I, J, nrows: int, ncols: int):
    """(row_ptr, col_idx, pos) of sparse(I, J, ., nrows, ncols): pos[t] is the
    CSR position triplet t is summed into."""
    I, J = _i32(I), _i32(J)
    n = I.shape[0]
    row_ptr = np.zeros(nrows + 1, np.int32)
    col_idx = np.zeros(max(n, 1), np.int32)
    pos = np.zeros(max(n, 1), np.int64)
    nnz = _check(_load().oracle_csr_pattern(nrows, ncols, n, I, J, row_ptr, col_idx, pos))
    return row_ptr, col_idx[:nnz].copy(), pos[:n].copy()


# ---- mesh-level entry points ----------------------------------------------------

class Pattern:
    """Oracle CSR pattern of a P1 mesh (scalar operators)."""

    def __init__(self, nq, nme, row_ptr, col_idx, slot, inc_ptr, inc):
        self.nq, self.nme = nq, nme
        self.row_ptr, self.col_idx, self.slot = row_ptr, col_idx, slot
        self.inc_ptr, self.inc = inc_ptr, inc

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def validate(nq: int, me) -> int:
    me = _i32(me)
    return _load().oracle_validate(nq, me.shape[0], me.reshape(-1))


def pattern(nq: int, me) -> Pattern:
    me = _i32(me)
    nme = me.shape[0]
    row_ptr = np.zeros(nq + 1, np.int32)
    col_idx = np.zeros(max(9 * nme, 1), np.int32)
    slot = np.zeros(max(9 * nme, 1), np.int32)
    inc_ptr = np.zeros(nq + 1, np.int32)
    inc = np.zeros(max(3 * nme, 1), np.int32)
    nnz = _check(_load().oracle_pattern(nq, nme, me.reshape(-1), row_ptr, col_idx,
                                        _ptr(slot), _ptr(inc_ptr), _ptr(inc)))
    return Pattern(nq, nme, row_ptr, col_idx[:nnz].copy(), slot[:9 * nme].reshape(9, nme),
                   inc_ptr, inc[:3 * nme].copy())


def pattern_elas(nq: int, me):
    """(row_ptr_e, col_idx_e, slot_e [36][nme]) over 2 nq interleaved dofs."""
    me = _i32(me)
    nme = me.shape[0]
    row_ptr = np.zeros(2 * nq + 1, np.int32)
    col_idx = np.zeros(max(36 * nme, 1), np.int32)
    slot = np.zeros(max(36 * nme, 1), np.int32)
    nnz = _check(_load().oracle_pattern_elas(nq, nme, me.reshape(-1), row_ptr, col_idx,
                                             _ptr(slot)))
    return row_ptr, col_idx[:nnz].copy(), slot[:36 * nme].reshape(36, nme)


def assemble(op: str, q, me, slot, nnz: int, w=None, lam: float = 0.0, mu: float = 0.0):
    """Values of operator op ('mass', 'wmass', 'stiff', 'elas') on the pattern
    whose slot map is given (9 x nme, or 36 x nme for 'elas')."""
    q, me, slot = _f64(q), _i32(me), _i32(slot)
    w = None if w is None else _f64(w)
    vals = np.zeros(max(nnz, 1), np.float64)
    _check(_load().oracle_assemble(OPS[op], q.shape[0], me.shape[0], q.reshape(-1),
                                   me.reshape(-1), _ptr(w), float(lam), float(mu),
                                   slot.reshape(-1), nnz, vals))
    return vals[:nnz].copy()


def rows(op: str, q, me, rows_, w=None, lam: float = 0.0, mu: float = 0.0):
    """Selected rows computed one by one: (ptr, cols, vals) per requested row."""
    q, me, rows_ = _f64(q), _i32(me), _i32(rows_)
    w = None if w is None else _f64(w)
    nr = rows_.shape[0]
    deg = np.bincount(me.reshape(-1), minlength=q.shape[0])
    dofs = 2 if op == "elas" else 1
    cap = int(np.sum(dofs * (1 + 2 * deg[rows_ // dofs]))) + 1
    ptr = np.zeros(nr + 1, np.int32)
    cols = np.zeros(cap, np.int32)
    vals = np.zeros(cap, np.float64)
    tot = _check(_load().oracle_rows(OPS[op], q.shape[0], me.shape[0], q.reshape(-1),
                                     me.reshape(-1), _ptr(w), float(lam), float(mu), nr,
                                     rows_, ptr, cols, vals, cap))
    return ptr, cols[:tot].copy(), vals[:tot].copy()


def adjoint_stiff_wmass(q, me, w, slot, GS=None, GM=None):
    """(dq [nq][2], dw [nq]) of L = <GS, S(q)> + <GM, Mw(q, w)>."""
    q, me, slot = _f64(q), _i32(me), _i32(slot)
    w = None if w is None else _f64(w)
    GS = None if GS is None else _f64(GS)
    GM = None if GM is None else _f64(GM)
    nq = q.shape[0]
    dq = np.zeros(2 * nq)
    dw = np.zeros(nq)
    _check(_load().oracle_adjoint_stiff_wmass(nq, me.shape[0], q.reshape(-1), me.reshape(-1),
                                              _ptr(w), slot.reshape(-1), _ptr(GS), _ptr(GM),
                                              dq, dw))
    return dq.reshape(nq, 2), dw
