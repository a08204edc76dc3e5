"""MI355X (gfx950) P1 finite element assembly.

Python binding of ``libfem_p1.so`` (C ABI in ``include/fem_p1.h``).  Every
function keeps the name of its C entry point and only marshals arguments:
PyTorch provides device memory and the current HIP stream; every step of the
assembly runs in the library's HIP kernels.  There is no CPU fallback: calls
raise if the library is not built or no GPU is visible.

Typical use::

    import torch, paper_1305_3122_amd as fem
    pat = fem.fem_pattern(me_dev, nq)                 # symbolic phase, once per mesh
    S, M = fem.fem_assemble_stiff_mass(pat, q_dev)    # numeric phase
    A = pat.csr(S)                                    # torch.sparse_csr_tensor view
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

from . import _lib
from ._lib import (FEM_ACCUMULATE, FEM_ATOMIC, FEM_CHECK_AREA, FEM_DETERMINISTIC, FEM_OP_ELAS,  # noqa: F401
                   FEM_OP_MASS, FEM_OP_STIFF, FEM_OP_WMASS, FEM_PACKED_QW, FEM_PATTERN_ATOMIC,
                   FEM_PATTERN_AUTO, FEM_PATTERN_COARSE, FemError, fem_tune)

__all__ = [
    "Pattern", "FemError", "FEM_ATOMIC", "FEM_DETERMINISTIC", "FEM_ACCUMULATE", "FEM_CHECK_AREA",
    "FEM_PACKED_QW", "fem_tune",
    "FEM_OP_MASS", "FEM_OP_WMASS", "FEM_OP_STIFF", "FEM_OP_ELAS",
    "FEM_PATTERN_AUTO", "FEM_PATTERN_COARSE", "FEM_PATTERN_ATOMIC", "fem_pattern_set_path",
    "fem_pattern", "fem_fan_plan", "fem_transpose_map", "fem_elas_pattern", "fem_assemble", "fem_assemble_mass",
    "fem_assemble_wmass", "fem_assemble_stiff", "fem_assemble_stiff_mass",
    "fem_assemble_stiff_wmass", "fem_assemble_elas", "fem_batch_globalize",
    "fem_assemble_stiff_mass_batched", "Graph", "SparseCSR", "fem_sparse", "fem_sparse_values",
    "TetPattern", "fem_tet_pattern", "fem_tet_pattern_set_path", "fem_tet_assemble", "P2Pattern", "fem_p2_pattern", "fem_p2_assemble",
    "fem_adjoint_workspace", "fem_adjoint_stiff_wmass", "fem_adjoint_elas",
    "AssembleStiffWMass", "AssembleElas",
    "library_path",
]


def library_path() -> str:
    return _lib.LIB_PATH


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev(t, dtype, name, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    return t


@dataclasses.dataclass
class Pattern:
    """Result of fem_pattern: CSR pattern and triangle lists (device tensors)."""
    nq: int
    nme: int
    nnz: int
    me: object            # [nme][3] int32
    row_ptr: object       # [nq+1]   int32
    col_idx: object       # [nnz]    int32 (a view of the capacity buffer)
    inc_ptr: object       # [nq+1]   int32
    inc: object           # [3 nme]  int32  (3k + a)
    inc_pos: object       # [3 nme]  uint32 stored as int32 (p1 | p2 << 16)
    slot: object = None   # [9][nme] int32 or None
    tpos: object = None   # [nnz]    int32 or None (fem_transpose_map)
    fan: object = None    # [nq]     int64 (uint64 fan codes of fem_fan_plan) or None

    def csr(self, values):
        """torch.sparse_csr_tensor sharing row_ptr / col_idx / values."""
        torch = _torch()
        return torch.sparse_csr_tensor(self.row_ptr, self.col_idx, values, (self.nq, self.nq))

    def args(self):
        return (_ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.inc_ptr), _ptr(self.inc_pos),
                _ptr(self.fan), _ptr(self.slot))


def fem_pattern(me, nq: int, *, slot: bool = False, fan: bool = True, stream=None) -> Pattern:
    """Symbolic phase (C: fem_pattern), with the fan codes unless fan=False.
    me: [nme][3] int32 on the GPU."""
    torch = _torch()
    lib = _lib.load()
    _dev(me, torch.int32, "me")
    if me.dim() != 2 or me.shape[1] != 3:
        raise ValueError("me must have shape [nme, 3]")
    nme = int(me.shape[0])
    dev = me.device
    ws = C.c_size_t(0)
    _lib.check(lib.fem_pattern_workspace(int(nq), nme, C.byref(ws)))
    cap = int(lib.fem_nnz_bound(int(nq), nme))
    i32 = dict(dtype=torch.int32, device=dev)
    row_ptr = torch.empty(nq + 1, **i32)
    col_buf = torch.empty(max(cap, 1), **i32)
    inc_ptr = torch.empty(nq + 1, **i32)
    inc = torch.empty(max(3 * nme, 1), **i32)
    inc_pos = torch.empty(max(3 * nme, 1), **i32)
    sl = torch.empty(max(9 * nme, 1), **i32) if slot else None
    fn = torch.empty(nq, dtype=torch.int64, device=dev) if fan else None
    work = torch.empty(max(int(ws.value), 1), dtype=torch.uint8, device=dev)
    nnz = C.c_int64(0)
    _lib.check(lib.fem_pattern(int(nq), nme, _ptr(me), _ptr(row_ptr), _ptr(col_buf), cap,
                               _ptr(inc_ptr), _ptr(inc), _ptr(inc_pos), _ptr(fn), _ptr(sl), _ptr(work),
                               int(ws.value), C.byref(nnz), _stream(stream)))
    n = int(nnz.value)
    return Pattern(int(nq), nme, n, me, row_ptr, col_buf[:n], inc_ptr, inc[:3 * nme],
                   inc_pos[:3 * nme], None if sl is None else sl[:9 * nme].view(9, nme), fan=fn)


def fem_fan_plan(pat: Pattern, *, stream=None):
    """Fan codes of every row (C: fem_fan_plan), kept on the pattern; the
    numeric calls then walk each row's triangles around its vertex."""
    torch = _torch()
    fan = torch.empty(pat.nq, dtype=torch.int64, device=pat.row_ptr.device)
    _lib.check(_lib.load().fem_fan_plan(pat.nq, pat.nme, _ptr(pat.row_ptr), _ptr(pat.inc_ptr),
                                        _ptr(pat.inc_pos), _ptr(fan), _stream(stream)))
    pat.fan = fan
    return fan


def fem_pattern_set_path(path: int) -> None:
    """Process-wide choice of the symbolic algorithm (C: fem_pattern_set_path)."""
    _lib.check(_lib.load().fem_pattern_set_path(int(path)))


def fem_transpose_map(pat: Pattern, *, stream=None):
    torch = _torch()
    tpos = torch.empty(max(pat.nnz, 1), dtype=torch.int32, device=pat.row_ptr.device)
    _lib.check(_lib.load().fem_transpose_map(pat.nq, pat.nnz, _ptr(pat.row_ptr), _ptr(pat.col_idx),
                                             _ptr(tpos), _stream(stream)))
    pat.tpos = tpos[:pat.nnz]
    return pat.tpos


def fem_elas_pattern(pat: Pattern, *, stream=None):
    """(row_ptr_e [2nq+1], col_idx_e [4nnz]) of the interleaved elasticity matrix."""
    torch = _torch()
    dev = pat.row_ptr.device
    rpe = torch.empty(2 * pat.nq + 1, dtype=torch.int32, device=dev)
    cie = torch.empty(max(4 * pat.nnz, 1), dtype=torch.int32, device=dev)
    _lib.check(_lib.load().fem_elas_pattern(pat.nq, pat.nnz, _ptr(pat.row_ptr), _ptr(pat.col_idx),
                                            _ptr(rpe), _ptr(cie), _stream(stream)))
    return rpe, cie[:4 * pat.nnz]


def _q(pat, q):
    torch = _torch()
    return _dev(q, torch.float64, "q", (pat.nq, 2))


def _out(pat, out, n, name):
    torch = _torch()
    if out is None:
        return torch.empty(max(n, 1), dtype=torch.float64, device=pat.row_ptr.device)[:n]
    return _dev(out, torch.float64, name, (n,))


def _head(pat, q):
    return (pat.nq, pat.nme, pat.nnz, _ptr(_q(pat, q)), _ptr(pat.me))


def fem_assemble(pat: Pattern, q, ops: int, *, w=None, lam: float = 0.0, mu: float = 0.0,
                 out: Optional[dict] = None, work=None, tune: Optional[fem_tune] = None,
                 flags: int = 0, stream=None) -> dict:
    """Any subset of {M, Mw, S, K} in one pass (C: fem_assemble).  Returns a
    dict with keys "M", "Mw", "S", "K" for the requested operators; `out` may
    supply preallocated tensors under the same keys.  A packing workspace for
    the weighted mass is allocated here unless `work` is given; with
    FEM_PACKED_QW in `flags`, `work` is the one a previous call with the same
    q and w filled, and the packing pass is skipped."""
    torch = _torch()
    lib = _lib.load()
    out = dict(out or {})
    names = (("M", FEM_OP_MASS, 1), ("Mw", FEM_OP_WMASS, 1), ("S", FEM_OP_STIFF, 1),
             ("K", FEM_OP_ELAS, 4))
    for key, bit, mult in names:
        if ops & bit:
            out[key] = _out(pat, out.get(key), mult * pat.nnz, key)
    if ops & FEM_OP_WMASS:
        _dev(w, torch.float64, "w", (pat.nq,))
    ws = C.c_size_t(0)
    _lib.check(lib.fem_assemble_workspace(pat.nq, int(ops), C.byref(ws)))
    if work is None and ws.value > 0:
        work = torch.empty(int(ws.value), dtype=torch.uint8, device=pat.row_ptr.device)
    t = C.byref(tune) if tune is not None else None
    _lib.check(lib.fem_assemble(int(ops), pat.nq, pat.nme, pat.nnz, _ptr(_q(pat, q)), _ptr(w),
                                _ptr(pat.me), *pat.args(), float(lam), float(mu),
                                _ptr(out.get("M")), _ptr(out.get("Mw")), _ptr(out.get("S")),
                                _ptr(out.get("K")), _ptr(work),
                                0 if work is None else work.numel() * work.element_size(), t,
                                flags, _stream(stream)))
    return {k: out[k] for k, bit, _ in names if ops & bit}


def fem_assemble_mass(pat: Pattern, q, *, out=None, flags: int = 0, stream=None):
    v = _out(pat, out, pat.nnz, "out")
    _lib.check(_lib.load().fem_assemble_mass(*_head(pat, q), *pat.args(), _ptr(v), flags,
                                             _stream(stream)))
    return v


def fem_assemble_wmass(pat: Pattern, q, w, *, out=None, flags: int = 0, stream=None):
    torch = _torch()
    _dev(w, torch.float64, "w", (pat.nq,))
    v = _out(pat, out, pat.nnz, "out")
    _lib.check(_lib.load().fem_assemble_wmass(*_head(pat, q), *pat.args(), _ptr(w), _ptr(v), flags,
                                              _stream(stream)))
    return v


def fem_assemble_stiff(pat: Pattern, q, *, out=None, flags: int = 0, stream=None):
    v = _out(pat, out, pat.nnz, "out")
    _lib.check(_lib.load().fem_assemble_stiff(*_head(pat, q), *pat.args(), _ptr(v), flags,
                                              _stream(stream)))
    return v


def fem_assemble_stiff_mass(pat: Pattern, q, *, out_S=None, out_M=None, flags: int = 0,
                            stream=None):
    S = _out(pat, out_S, pat.nnz, "out_S")
    M = _out(pat, out_M, pat.nnz, "out_M")
    _lib.check(_lib.load().fem_assemble_stiff_mass(*_head(pat, q), *pat.args(), _ptr(S), _ptr(M),
                                                   flags, _stream(stream)))
    return S, M


def fem_assemble_stiff_wmass(pat: Pattern, q, w, *, out_S=None, out_M=None, flags: int = 0,
                             stream=None):
    torch = _torch()
    _dev(w, torch.float64, "w", (pat.nq,))
    S = _out(pat, out_S, pat.nnz, "out_S")
    M = _out(pat, out_M, pat.nnz, "out_M")
    _lib.check(_lib.load().fem_assemble_stiff_wmass(*_head(pat, q), *pat.args(), _ptr(w), _ptr(S),
                                                    _ptr(M), flags, _stream(stream)))
    return S, M


def fem_assemble_elas(pat: Pattern, q, lam: float, mu: float, *, out=None, flags: int = 0,
                      stream=None):
    v = _out(pat, out, 4 * pat.nnz, "out")
    _lib.check(_lib.load().fem_assemble_elas(*_head(pat, q), *pat.args(), float(lam), float(mu),
                                             _ptr(v), flags, _stream(stream)))
    return v


def fem_batch_globalize(me_local, vtx_off, elem_off, *, stream=None):
    """Connectivity of a batch with global vertex ids (C: fem_batch_globalize).
    vtx_off / elem_off: [nb+1] int64 GPU tensors."""
    torch = _torch()
    _dev(me_local, torch.int32, "me_local")
    _dev(vtx_off, torch.int64, "vtx_off")
    _dev(elem_off, torch.int64, "elem_off", (vtx_off.shape[0],))
    nb = int(vtx_off.shape[0]) - 1
    out = torch.empty_like(me_local)
    _lib.check(_lib.load().fem_batch_globalize(nb, int(me_local.shape[0]), _ptr(vtx_off),
                                               _ptr(elem_off), _ptr(me_local), _ptr(out),
                                               _stream(stream)))
    return out


def fem_assemble_stiff_mass_batched(pat: Pattern, q, nb: int, *, tune: Optional[fem_tune] = None,
                                    out_S=None, out_M=None, flags: int = 0, stream=None):
    S = _out(pat, out_S, pat.nnz, "out_S")
    M = _out(pat, out_M, pat.nnz, "out_M")
    t = C.byref(tune) if tune is not None else None
    _lib.check(_lib.load().fem_assemble_stiff_mass_batched(
        int(nb), pat.nq, pat.nnz, _ptr(_q(pat, q)), _ptr(pat.row_ptr), _ptr(pat.col_idx),
        _ptr(pat.inc_ptr), _ptr(pat.inc_pos), _ptr(pat.fan), _ptr(S), _ptr(M), t, flags,
        _stream(stream)))
    return S, M


class Graph:
    """HIP graph of library calls (C: fem_graph_begin / end / launch / destroy).

        g = Graph(stream)
        with g.capture():
            fem_assemble_stiff_mass(pat, q, out_S=S, out_M=M, stream=stream)
        g.replay()
    """

    def __init__(self, stream):
        self.stream = stream
        self.handle = None

    def capture(self):
        g = self

        class _Ctx:
            def __enter__(self_):
                _lib.check(_lib.load().fem_graph_begin(_stream(g.stream)))
                return g

            def __exit__(self_, et, ev, tb):
                h = C.c_void_p()
                st = _lib.load().fem_graph_end(_stream(g.stream), C.byref(h))
                if et is None:
                    _lib.check(st)
                    g.handle = h.value
                return False

        return _Ctx()

    def replay(self, stream=None):
        _lib.check(_lib.load().fem_graph_launch(self.handle, _stream(stream or self.stream)))

    def __del__(self):
        if self.handle is not None and _lib._lib is not None:
            _lib._lib.fem_graph_destroy(self.handle)
            self.handle = None


@dataclasses.dataclass
class SparseCSR:
    """Result of fem_sparse (device tensors)."""
    m: int
    n: int
    nnz: int
    row_ptr: object          # [m+1] int32
    col_idx: object          # [nnz] int32
    vals: object = None      # [nnz] float64 or None
    contrib_ptr: object = None   # [nnz+1] int32 or None
    contrib: object = None       # [nt] int32 or None

    def csr(self):
        torch = _torch()
        return torch.sparse_csr_tensor(self.row_ptr, self.col_idx, self.vals, (self.m, self.n))


def fem_sparse(I, J, V, m: int, n: int, *, contrib: bool = False, stream=None) -> SparseCSR:
    """sparse(I, J, V, m, n) into CSR (C: fem_sparse).  I, J: [nt] int32 and V:
    [nt] float64 (or None for the pattern only) on the GPU."""
    torch = _torch()
    lib = _lib.load()
    _dev(I, torch.int32, "I")
    nt = int(I.shape[0])
    _dev(J, torch.int32, "J", (nt,))
    if V is not None:
        _dev(V, torch.float64, "V", (nt,))
    dev = I.device
    ws = C.c_size_t(0)
    _lib.check(lib.fem_sparse_workspace(int(m), int(n), nt, C.byref(ws)))
    work = torch.empty(max(int(ws.value), 1), dtype=torch.uint8, device=dev)
    cap = nt
    i32 = dict(dtype=torch.int32, device=dev)
    row_ptr = torch.empty(int(m) + 1, **i32)
    col = torch.empty(max(cap, 1), **i32)
    vals = torch.empty(max(cap, 1), dtype=torch.float64, device=dev) if V is not None else None
    cptr = torch.empty(cap + 1, **i32) if contrib else None
    ctb = torch.empty(max(nt, 1), **i32) if contrib else None
    nnz = C.c_int64(0)
    _lib.check(lib.fem_sparse(int(m), int(n), nt, _ptr(I), _ptr(J), _ptr(V), _ptr(row_ptr),
                              _ptr(col), _ptr(vals), cap, _ptr(cptr), _ptr(ctb), _ptr(work),
                              int(ws.value), C.byref(nnz), _stream(stream)))
    k = int(nnz.value)
    return SparseCSR(int(m), int(n), k, row_ptr, col[:k], None if vals is None else vals[:k],
                     None if cptr is None else cptr[:k + 1], None if ctb is None else ctb[:nt])


def fem_sparse_values(A: SparseCSR, V, *, out=None, flags: int = 0, stream=None):
    """New values on the triplets of a fem_sparse result built with contrib=True
    (C: fem_sparse_values)."""
    torch = _torch()
    if A.contrib is None:
        raise ValueError("fem_sparse_values needs a fem_sparse result with contrib=True")
    _dev(V, torch.float64, "V", (int(A.contrib.shape[0]),))
    out = torch.empty(max(A.nnz, 1), dtype=torch.float64, device=V.device)[:A.nnz] if out is None else out
    _lib.check(_lib.load().fem_sparse_values(A.nnz, _ptr(A.contrib_ptr), _ptr(A.contrib), _ptr(V),
                                             _ptr(out), flags, _stream(stream)))
    return out


@dataclasses.dataclass
class TetPattern:
    """Result of fem_tet_pattern (device tensors)."""
    nq: int
    nme: int
    nnz: int
    me: object               # [nme][4] int32
    row_ptr: object          # [nq+1] int32
    col_idx: object          # [nnz] int32
    inc_ptr: object          # [nq+1] int32
    inc: object              # [4 nme] int32: 4 k + a, ascending per vertex
    inc_pos: object          # [4 nme] int32 (uint32 bits): three 10-bit row slots

    def csr(self, values):
        torch = _torch()
        return torch.sparse_csr_tensor(self.row_ptr, self.col_idx, values, (self.nq, self.nq))


def fem_tet_pattern_set_path(path: int) -> None:
    """FEM_PATTERN_AUTO or FEM_PATTERN_COARSE (the general path), for tests."""
    _lib.check(_lib.load().fem_tet_pattern_set_path(int(path)))


def fem_tet_pattern(me, nq: int, *, stream=None) -> TetPattern:
    """P1 tetrahedron pattern (C: fem_tet_pattern).  me: [nme][4] int32 on the GPU."""
    torch = _torch()
    lib = _lib.load()
    _dev(me, torch.int32, "me")
    if me.dim() != 2 or me.shape[1] != 4:
        raise ValueError("me must have shape [nme, 4]")
    nme = int(me.shape[0])
    dev = me.device
    ws = C.c_size_t(0)
    _lib.check(lib.fem_tet_pattern_workspace(int(nq), nme, C.byref(ws)))
    work = torch.empty(max(int(ws.value), 1), dtype=torch.uint8, device=dev)
    cap = int(lib.fem_tet_nnz_bound(int(nq), nme))
    i32 = dict(dtype=torch.int32, device=dev)
    row_ptr = torch.empty(int(nq) + 1, **i32)
    inc_ptr = torch.empty(int(nq) + 1, **i32)
    col = torch.empty(max(cap, 1), **i32)
    inc = torch.empty(max(4 * nme, 1), **i32)
    inc_pos = torch.empty(max(4 * nme, 1), **i32)
    nnz = C.c_int64(0)
    _lib.check(lib.fem_tet_pattern(int(nq), nme, _ptr(me), _ptr(row_ptr), _ptr(col), cap,
                                   _ptr(inc_ptr), _ptr(inc), _ptr(inc_pos), _ptr(work),
                                   int(ws.value), C.byref(nnz), _stream(stream)))
    k = int(nnz.value)
    return TetPattern(int(nq), nme, k, me, row_ptr, col[:k], inc_ptr, inc[:4 * nme],
                      inc_pos[:4 * nme])


def fem_tet_assemble(pat: TetPattern, q, ops: int = FEM_OP_MASS | FEM_OP_STIFF, *, out=None,
                     flags: int = 0, stream=None):
    """P1 tetrahedron mass / stiffness values on `pat` (C: fem_tet_assemble).
    q: [nq][3] float64 on the GPU.  Returns {"M": ..., "S": ...} for the
    requested operators."""
    torch = _torch()
    lib = _lib.load()
    _dev(q, torch.float64, "q", (pat.nq, 3))
    dev = q.device
    out = {} if out is None else dict(out)
    f64 = dict(dtype=torch.float64, device=dev)
    for key, bit in (("M", FEM_OP_MASS), ("S", FEM_OP_STIFF)):
        if ops & bit and key not in out:
            out[key] = torch.empty(max(pat.nnz, 1), **f64)[:pat.nnz]
    _lib.check(lib.fem_tet_assemble(int(ops), pat.nq, pat.nme, pat.nnz, _ptr(q), _ptr(pat.row_ptr),
                                    _ptr(pat.col_idx), _ptr(pat.inc_ptr), _ptr(pat.inc_pos),
                                    _ptr(out.get("M")), _ptr(out.get("S")), flags,
                                    _stream(stream)))
    return out


@dataclasses.dataclass
class P2Pattern:
    """Result of fem_p2_pattern (device tensors): P2 DOFs (vertices, then
    nq + edge) and the CSR pattern over them."""
    nq: int
    ne: int
    nme: int
    nnz: int
    me: object               # [nme][3] int32
    dofs: object             # [nme][6] int32
    edges: object            # [ne][2] int32
    row_ptr: object          # [ndof+1] int32
    col_idx: object          # [nnz] int32
    inc_ptr: object          # [ndof+1] int32
    inc: object              # [6 nme] int32: 6 k + a, ascending per DOF
    inc_pos: object          # [6 nme] int64 (uint64 bits): six 10-bit row slots, a in bits 60-62

    @property
    def ndof(self) -> int:
        return self.nq + self.ne

    def csr(self, values):
        torch = _torch()
        return torch.sparse_csr_tensor(self.row_ptr, self.col_idx, values, (self.ndof, self.ndof))


def fem_p2_pattern(me, nq: int, *, stream=None) -> P2Pattern:
    """P2 triangle DOFs and pattern (C: fem_p2_dofs, then fem_p2_pattern).
    me: [nme][3] int32 on the GPU."""
    torch = _torch()
    lib = _lib.load()
    _dev(me, torch.int32, "me")
    if me.dim() != 2 or me.shape[1] != 3:
        raise ValueError("me must have shape [nme, 3]")
    nme = int(me.shape[0])
    dev = me.device
    i32 = dict(dtype=torch.int32, device=dev)
    ws = C.c_size_t(0)
    _lib.check(lib.fem_p2_dofs_workspace(int(nq), nme, C.byref(ws)))
    work = torch.empty(max(int(ws.value), 1), dtype=torch.uint8, device=dev)
    dofs = torch.empty((max(nme, 1), 6), **i32)[:nme]
    ecap = 3 * nme
    edges = torch.empty((max(ecap, 1), 2), **i32)
    ne = C.c_int64(0)
    _lib.check(lib.fem_p2_dofs(int(nq), nme, _ptr(me), _ptr(dofs), _ptr(edges), ecap, _ptr(work),
                               int(ws.value), C.byref(ne), _stream(stream)))
    ne = int(ne.value)
    del work
    ndof = int(nq) + ne
    _lib.check(lib.fem_p2_pattern_workspace(ndof, nme, C.byref(ws)))
    work = torch.empty(max(int(ws.value), 1), dtype=torch.uint8, device=dev)
    cap = min(36 * nme, ndof + 30 * nme)
    row_ptr = torch.empty(ndof + 1, **i32)
    col = torch.empty(max(cap, 1), **i32)
    inc_ptr = torch.empty(ndof + 1, **i32)
    inc = torch.empty(max(6 * nme, 1), **i32)
    inc_pos = torch.empty(max(6 * nme, 1), dtype=torch.int64, device=dev)
    nnz = C.c_int64(0)
    _lib.check(lib.fem_p2_pattern(ndof, nme, _ptr(dofs), _ptr(row_ptr), _ptr(col), cap, _ptr(inc_ptr),
                                  _ptr(inc), _ptr(inc_pos), _ptr(work), int(ws.value), C.byref(nnz),
                                  _stream(stream)))
    k = int(nnz.value)
    return P2Pattern(int(nq), ne, nme, k, me, dofs, edges[:ne], row_ptr, col[:k], inc_ptr,
                     inc[:6 * nme], inc_pos[:6 * nme])


def fem_p2_assemble(pat: P2Pattern, q, ops: int = FEM_OP_MASS | FEM_OP_STIFF, *, out=None,
                    work=None, flags: int = 0, stream=None):
    """P2 triangle mass / stiffness values on `pat` (C: fem_p2_assemble).
    q: [nq][2] float64 on the GPU.  Returns {"M": ..., "S": ...} for the
    requested operators."""
    torch = _torch()
    lib = _lib.load()
    _dev(q, torch.float64, "q", (pat.nq, 2))
    dev = q.device
    out = {} if out is None else dict(out)
    f64 = dict(dtype=torch.float64, device=dev)
    for key, bit in (("M", FEM_OP_MASS), ("S", FEM_OP_STIFF)):
        if ops & bit and key not in out:
            out[key] = torch.empty(max(pat.nnz, 1), **f64)[:pat.nnz]
    if work is None:
        ws = C.c_size_t(0)
        _lib.check(lib.fem_p2_assemble_workspace(pat.nme, C.byref(ws)))
        work = torch.empty(max(int(ws.value), 32), dtype=torch.uint8, device=dev)
    _lib.check(lib.fem_p2_assemble(int(ops), pat.nq, pat.nme, pat.ndof, pat.nnz, _ptr(q), _ptr(pat.me),
                                   _ptr(pat.row_ptr), _ptr(pat.inc_ptr), _ptr(pat.inc), _ptr(pat.inc_pos),
                                   _ptr(out.get("M")), _ptr(out.get("S")), _ptr(work),
                                   work.numel() * work.element_size(), flags, _stream(stream)))
    return out


def fem_adjoint_workspace(pat: Pattern):
    """A device workspace for fem_adjoint_stiff_wmass (also usable as the
    packing workspace of fem_assemble, see FEM_PACKED_QW)."""
    torch = _torch()
    ws = C.c_size_t(0)
    _lib.check(_lib.load().fem_adjoint_workspace(pat.nq, pat.nnz, C.byref(ws)))
    return torch.empty(max(int(ws.value), 1), dtype=torch.uint8, device=pat.row_ptr.device)


def fem_adjoint_stiff_wmass(pat: Pattern, q, w, GS, GM, *, dq=None, dw=None, flags: int = 0,
                            work=None, packed: bool = False, stream=None):
    """(dq [nq][2], dw [nq]) of L = <GS, S(q)> + <GM, Mw(q, w)>.

    packed=True: `work` is the workspace fem_assemble packed the (x, y, w)
    records of these q and w into (C flag FEM_PACKED_QW)."""
    torch = _torch()
    lib = _lib.load()
    dev = pat.row_ptr.device
    _q(pat, q)
    if GS is not None:
        _dev(GS, torch.float64, "GS", (pat.nnz,))
    if GM is not None:
        _dev(GM, torch.float64, "GM", (pat.nnz,))
        _dev(w, torch.float64, "w", (pat.nq,))
    dq = torch.empty((pat.nq, 2), dtype=torch.float64, device=dev) if dq is None else dq
    dw = torch.empty(pat.nq, dtype=torch.float64, device=dev) if dw is None else dw
    if packed and work is None:
        raise ValueError("packed=True needs the workspace fem_assemble packed into")
    if work is None:
        work = fem_adjoint_workspace(pat)
    if packed:
        flags |= _lib.FEM_PACKED_QW
    _lib.check(lib.fem_adjoint_stiff_wmass(pat.nq, pat.nme, pat.nnz, _ptr(q), _ptr(w),
                                           _ptr(pat.row_ptr), _ptr(pat.col_idx), _ptr(pat.inc_ptr),
                                           _ptr(pat.inc_pos), _ptr(pat.fan), _ptr(pat.tpos),
                                           _ptr(GS), _ptr(GM),
                                           _ptr(dq), _ptr(dw), _ptr(work),
                                           work.numel() * work.element_size(), flags,
                                           _stream(stream)))
    return dq, dw


def fem_adjoint_elas(pat: Pattern, q, lam: float, mu: float, G, *, dq=None, dlm=None,
                     flags: int = 0, stream=None):
    """(dq [nq][2], dlm [2] = (dL/dlambda, dL/dmu)) of L = <G, K(q; lambda, mu)>,
    G [4 nnz] in the elasticity layout (C: fem_adjoint_elas)."""
    torch = _torch()
    lib = _lib.load()
    dev = pat.row_ptr.device
    _q(pat, q)
    _dev(G, torch.float64, "G", (4 * pat.nnz,))
    dq = torch.empty((pat.nq, 2), dtype=torch.float64, device=dev) if dq is None else dq
    dlm = torch.empty(2, dtype=torch.float64, device=dev) if dlm is None else dlm
    ws = C.c_size_t(0)
    _lib.check(lib.fem_adjoint_elas_workspace(pat.nq, pat.nnz, C.byref(ws)))
    work = torch.empty(max(int(ws.value), 1), dtype=torch.uint8, device=dev)
    _lib.check(lib.fem_adjoint_elas(pat.nq, pat.nme, pat.nnz, _ptr(q), _ptr(pat.row_ptr),
                                    _ptr(pat.col_idx), _ptr(pat.inc_ptr), _ptr(pat.inc_pos),
                                    _ptr(pat.fan), _ptr(pat.tpos), float(lam), float(mu), _ptr(G),
                                    _ptr(dq),
                                    _ptr(dlm), _ptr(work), int(ws.value), flags, _stream(stream)))
    return dq, dlm


def _autograd_function():
    torch = _torch()

    class AssembleStiffWMass(torch.autograd.Function):
        """(S values, Mw values) = F(q, w) on a fixed pattern; backward runs the
        hand-written adjoint kernels (fem_adjoint_stiff_wmass), with the
        pattern's transpose map (built on the first backward if missing)."""

        @staticmethod
        def forward(ctx, q, w, pat):
            # the adjoint's workspace doubles as the forward's packing
            # workspace, so the backward reuses the packed (x, y, w) records
            work = fem_adjoint_workspace(pat)
            r = fem_assemble(pat, q.contiguous(), FEM_OP_STIFF | FEM_OP_WMASS, w=w.contiguous(),
                             work=work)
            S, M = r["S"], r["Mw"]
            ctx.pat = pat
            ctx.work = work
            ctx.save_for_backward(q, w)
            return S, M

        @staticmethod
        def backward(ctx, gS, gM):
            q, w = ctx.saved_tensors   # version-checked: q, w unchanged since forward
            gS = None if gS is None else gS.contiguous()
            gM = None if gM is None else gM.contiguous()
            if ctx.pat.tpos is None and ctx.pat.nnz > 0:
                # the transpose map, built once and kept on the pattern: the
                # second pass then reads rows in place instead of searching
                fem_transpose_map(ctx.pat)
            dq, dw = fem_adjoint_stiff_wmass(ctx.pat, q.contiguous(), w.contiguous(), gS, gM,
                                             work=ctx.work, packed=q.is_contiguous() and
                                             w.is_contiguous())
            # ctx.work is kept: a second backward through the same graph
            # (retain_graph=True) reads the packed records again
            return dq, (dw if gM is not None else None), None

    class AssembleElas(torch.autograd.Function):
        """Elasticity values K(q; lambda, mu) [4 nnz] on a fixed pattern, with
        lambda and mu as 0-dim tensors; backward runs fem_adjoint_elas."""

        @staticmethod
        def forward(ctx, q, lam, mu, pat):
            K = fem_assemble_elas(pat, q.contiguous(), float(lam), float(mu))
            ctx.pat = pat
            ctx.save_for_backward(q, lam, mu)
            return K

        @staticmethod
        def backward(ctx, gK):
            q, lam, mu = ctx.saved_tensors
            if ctx.pat.tpos is None and ctx.pat.nnz > 0:
                fem_transpose_map(ctx.pat)   # once per pattern, as above
            dq, dlm = fem_adjoint_elas(ctx.pat, q.contiguous(), float(lam), float(mu), gK.contiguous())
            return dq, dlm[0].to(lam.dtype), dlm[1].to(mu.dtype), None

    return AssembleStiffWMass, AssembleElas


class _Lazy:
    _fns = None

    def __init__(self, which):
        self.which = which

    def apply(self, *args):
        if _Lazy._fns is None:
            _Lazy._fns = _autograd_function()
        return _Lazy._fns[self.which].apply(*args)


AssembleStiffWMass = _Lazy(0)
AssembleElas = _Lazy(1)
