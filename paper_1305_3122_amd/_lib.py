"""ctypes declarations of the C ABI in include/fem_p1.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfem_p1.so")

FEM_OK = 0
FEM_EINVAL = -1
FEM_ERANGE = -2
FEM_EDEGEN = -3
FEM_ENOSPC = -4
FEM_EOVERFLOW = -5
FEM_EHIP = -6
FEM_EUNSUPPORTED = -8

FEM_DETERMINISTIC = 0
FEM_ATOMIC = 1
FEM_ACCUMULATE = 2
FEM_PACKED_QW = 4
FEM_CHECK_AREA = 8

FEM_PATTERN_AUTO = 0
FEM_PATTERN_COARSE = 1
FEM_PATTERN_ATOMIC = 2

FEM_OP_MASS = 1
FEM_OP_WMASS = 2
FEM_OP_STIFF = 4
FEM_OP_ELAS = 8

STATUS_NAMES = {0: "FEM_OK", -1: "FEM_EINVAL", -2: "FEM_ERANGE", -3: "FEM_EDEGEN",
                -4: "FEM_ENOSPC", -5: "FEM_EOVERFLOW", -6: "FEM_EHIP", -8: "FEM_EUNSUPPORTED"}


class FemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class fem_tune(C.Structure):
    _fields_ = [("lds_entries", C.c_int32), ("grid_blocks", C.c_int32), ("variant", C.c_int32)]


_vp = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_int = C.c_int
_dbl = C.c_double
_szp = C.POINTER(C.c_size_t)

_PAT = [_vp, _vp, _vp, _vp, _vp, _vp]  # row_ptr, col_idx, inc_ptr, inc_pos, fan, slot
_NUM_HEAD = [_i32, _i32, _i64, _vp, _vp]  # nq, nme, nnz, q, me

SIGNATURES = {
    "fem_last_error": (C.c_char_p, []),
    "fem_version": (_int, []),
    "fem_pattern_workspace": (_int, [_i32, _i32, _szp]),
    "fem_nnz_bound": (_i64, [_i32, _i32]),
    "fem_pattern": (_int, [_i32, _i32, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp,
                           C.c_size_t, C.POINTER(_i64), _vp]),
    "fem_pattern_set_path": (_int, [_int]),
    "fem_transpose_map": (_int, [_i32, _i64, _vp, _vp, _vp, _vp]),
    "fem_fan_plan": (_int, [_i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "fem_elas_pattern": (_int, [_i32, _i64, _vp, _vp, _vp, _vp, _vp]),
    "fem_assemble_workspace": (_int, [_i32, _int, _szp]),
    "fem_assemble": (_int, [_int, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                            _dbl, _dbl, _vp, _vp, _vp, _vp, _vp, C.c_size_t, C.POINTER(fem_tune),
                            _int, _vp]),
    "fem_assemble_noalloc": (_int, [_int, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                    _vp, _dbl, _dbl, _vp, _vp, _vp, _vp, C.POINTER(fem_tune), _int,
                                    _vp]),
    "fem_gather_probe_threads": (_int, []),
    "fem_gather_probe": (_int, [_i64, _i32, _vp, _vp, _int, _vp, _vp]),
    "fem_assemble_mass": (_int, _NUM_HEAD + _PAT + [_vp, _int, _vp]),
    "fem_assemble_wmass": (_int, _NUM_HEAD + _PAT + [_vp, _vp, _int, _vp]),
    "fem_assemble_stiff": (_int, _NUM_HEAD + _PAT + [_vp, _int, _vp]),
    "fem_assemble_stiff_mass": (_int, _NUM_HEAD + _PAT + [_vp, _vp, _int, _vp]),
    "fem_assemble_stiff_wmass": (_int, _NUM_HEAD + _PAT + [_vp, _vp, _vp, _int, _vp]),
    "fem_assemble_elas": (_int, _NUM_HEAD + _PAT + [_dbl, _dbl, _vp, _int, _vp]),
    "fem_batch_globalize": (_int, [_i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "fem_assemble_stiff_mass_batched": (_int, [_i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                               _vp, C.POINTER(fem_tune), _int, _vp]),
    "fem_graph_begin": (_int, [_vp]),
    "fem_graph_end": (_int, [_vp, C.POINTER(_vp)]),
    "fem_graph_launch": (_int, [_vp, _vp]),
    "fem_graph_destroy": (_int, [_vp]),
    "fem_sparse_workspace": (_int, [_i32, _i32, _i64, _szp]),
    "fem_sparse": (_int, [_i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp,
                          C.c_size_t, C.POINTER(_i64), _vp]),
    "fem_sparse_values": (_int, [_i64, _vp, _vp, _vp, _vp, _int, _vp]),
    "fem_tet_pattern_workspace": (_int, [_i32, _i32, _szp]),
    "fem_tet_nnz_bound": (_i64, [_i32, _i32]),
    "fem_tet_pattern": (_int, [_i32, _i32, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, C.c_size_t,
                               C.POINTER(_i64), _vp]),
    "fem_tet_pattern_set_path": (_int, [_int]),
    "fem_tet_assemble": (_int, [_int, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _int,
                                _vp]),
    "fem_p2_dofs_workspace": (_int, [_i32, _i32, _szp]),
    "fem_p2_dofs": (_int, [_i32, _i32, _vp, _vp, _vp, _i64, _vp, C.c_size_t, C.POINTER(_i64), _vp]),
    "fem_p2_pattern_workspace": (_int, [_i32, _i32, _szp]),
    "fem_p2_pattern": (_int, [_i32, _i32, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, C.c_size_t,
                              C.POINTER(_i64), _vp]),
    "fem_p2_assemble_workspace": (_int, [_i32, _szp]),
    "fem_p2_assemble": (_int, [_int, _i32, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                               _vp, C.c_size_t, _int, _vp]),
    "fem_adjoint_elas_workspace": (_int, [_i32, _i64, _szp]),
    "fem_adjoint_elas": (_int, [_i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _dbl, _dbl, _vp,
                                _vp, _vp, _vp, C.c_size_t, _int, _vp]),
    "fem_adjoint_workspace": (_int, [_i32, _i64, _szp]),
    "fem_adjoint_stiff_wmass": (_int, [_i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                       _vp, _vp, _vp, _vp, _vp, C.c_size_t, _int, _vp]),
}

_lib = None


def load():
    """Load libfem_p1.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1305_3122_amd.build` (or __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> int:
    if status != FEM_OK:
        msg = load().fem_last_error().decode(errors="replace")
        raise FemError(status, msg)
    return status
