"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/fem_p1.h, and rejects bad arguments on the host before
touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_1305_3122_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fem_p1.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1305_3122_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares a signature for each of them
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_version_and_bounds(lib):
    assert lib.fem_version() == 200
    assert lib.fem_nnz_bound(10, 7) == 10 + 42
    sz = C.c_size_t(0)
    assert lib.fem_pattern_workspace(1089, 2048, C.byref(sz)) == 0
    assert sz.value > 4 * (6 * 2048 + 1089)
    assert lib.fem_pattern_workspace(0, 5, C.byref(sz)) == _lib.FEM_EINVAL
    assert lib.fem_adjoint_workspace(10, 100, C.byref(sz)) == 0 and sz.value == 512 + 3200


def test_host_validation_before_any_launch(lib):
    nnz = C.c_int64(0)
    fake = C.c_void_p(0x1000)  # never dereferenced: the checks fail first
    # nq < 1
    st = lib.fem_pattern(0, 1, fake, fake, fake, 10, fake, fake, fake, None, None, fake, 1 << 20,
                         C.byref(nnz), None)
    assert st == _lib.FEM_EINVAL
    assert b"nq" in lib.fem_last_error()
    # nq + 6 nme beyond int32
    st = lib.fem_pattern(10, 400_000_000, fake, fake, fake, 10, fake, fake, fake, None, None, fake,
                         1 << 20, C.byref(nnz), None)
    assert st == _lib.FEM_EOVERFLOW
    # workspace too small
    st = lib.fem_pattern(10, 4, fake, fake, fake, 100, fake, fake, fake, None, None, fake, 16,
                         C.byref(nnz), None)
    assert st == _lib.FEM_ENOSPC
    # elasticity: lambda + mu must be positive (elasticity section)
    st = lib.fem_assemble_elas(4, 2, 10, fake, fake, fake, fake, fake, fake, None, None, -1.0, 0.5,
                               fake, 0, None)
    assert st == _lib.FEM_EINVAL and b"lambda" in lib.fem_last_error()
    # FEM_ATOMIC needs the slot map
    st = lib.fem_assemble_stiff(4, 2, 10, fake, fake, fake, fake, fake, fake, None, None, fake,
                                _lib.FEM_ATOMIC, None)
    assert st == _lib.FEM_EINVAL
    # FEM_CHECK_AREA needs a workspace for its flag (the single-operator calls have none)
    st = lib.fem_assemble_stiff(4, 2, 10, fake, fake, fake, fake, fake, fake, None, None, fake,
                                _lib.FEM_CHECK_AREA, None)
    assert st == _lib.FEM_ENOSPC and b"FEM_CHECK_AREA" in lib.fem_last_error()
    ws = C.c_size_t(0)
    assert lib.fem_assemble_workspace(4, _lib.FEM_OP_WMASS, C.byref(ws)) == _lib.FEM_OK
    assert ws.value == 256 + 256
    # FEM_PACKED_QW: only with the weighted mass in the row-owner scheme, and
    # only with the workspace that holds the packed records
    args = (4, 2, 10, fake, fake, fake, fake, fake, fake, fake, None, None, 0.0, 0.0, fake, fake,
            fake, fake)
    st = lib.fem_assemble(_lib.FEM_OP_STIFF, *args, fake, 4096, None, _lib.FEM_PACKED_QW, None)
    assert st == _lib.FEM_EINVAL and b"FEM_PACKED_QW" in lib.fem_last_error()
    st = lib.fem_assemble(_lib.FEM_OP_WMASS, *args, fake, 4096, None,
                          _lib.FEM_PACKED_QW | _lib.FEM_ATOMIC, None)
    assert st == _lib.FEM_EINVAL
    st = lib.fem_assemble(_lib.FEM_OP_WMASS, *args, None, 0, None, _lib.FEM_PACKED_QW, None)
    assert st == _lib.FEM_ENOSPC and b"FEM_PACKED_QW" in lib.fem_last_error()
    st = lib.fem_assemble(_lib.FEM_OP_WMASS, *args, fake, 32 * 4 - 8, None, _lib.FEM_PACKED_QW, None)
    assert st == _lib.FEM_ENOSPC
    # unknown flag bits
    st = lib.fem_assemble_mass(4, 2, 10, fake, fake, fake, fake, fake, fake, None, None, fake, 64,
                               None)
    assert st == _lib.FEM_EINVAL
    # the weighted mass needs w
    st = lib.fem_assemble_wmass(4, 2, 10, fake, fake, fake, fake, fake, fake, None, None, None, fake,
                                0, None)
    assert st == _lib.FEM_EINVAL
    # graphs cannot capture the NULL stream
    assert lib.fem_graph_begin(None) == _lib.FEM_EINVAL
    assert lib.fem_graph_destroy(None) == 0
    # adjoint: the GM term needs w and dw
    st = lib.fem_adjoint_stiff_wmass(4, 2, 10, fake, None, fake, fake, fake, fake, None, None, None,
                                     fake, fake, None, fake, 1000, 0, None)
    assert st == _lib.FEM_EINVAL


def test_extension_size_limits_before_any_launch(lib):
    # the triplet counts of the extensions must fit int32: refused on the
    # host with FEM_EOVERFLOW, nothing enqueued
    fake = C.c_void_p(0x1000)   # never dereferenced
    out = C.c_int64(0)
    ws = C.c_size_t(0)
    big_p2 = 60_000_000         # 36 nme > 2^31 - 1
    assert lib.fem_p2_dofs_workspace(10, big_p2, C.byref(ws)) == _lib.FEM_EOVERFLOW
    assert lib.fem_p2_dofs(10, big_p2, fake, fake, None, 0, fake, 1 << 20, C.byref(out),
                           None) == _lib.FEM_EOVERFLOW
    assert lib.fem_p2_pattern(10, big_p2, fake, fake, fake, 0, fake, fake, fake, fake, 1 << 20,
                              C.byref(out), None) == _lib.FEM_EOVERFLOW
    assert lib.fem_p2_assemble(5, 10, big_p2, 20, 10, fake, fake, fake, fake, fake, fake, fake, fake, fake,
                               1 << 20, 0, None) == _lib.FEM_EOVERFLOW
    big_tet = 140_000_000       # 16 nme > 2^31 - 1
    assert lib.fem_tet_pattern_workspace(10, big_tet, C.byref(ws)) == _lib.FEM_EOVERFLOW
    assert lib.fem_tet_pattern(10, big_tet, fake, fake, fake, 0, fake, fake, fake, fake, 1 << 20,
                               C.byref(out), None) == _lib.FEM_EOVERFLOW
    assert lib.fem_sparse_workspace(10, 10, 1 << 31, C.byref(ws)) == _lib.FEM_EOVERFLOW
    assert lib.fem_sparse(10, 10, 1 << 31, fake, fake, None, fake, fake, None, 0, None, None, fake,
                          1 << 20, C.byref(out), None) == _lib.FEM_EOVERFLOW
    # and the workspace queries at sizes that fit answer
    assert lib.fem_p2_dofs_workspace(10, 1000, C.byref(ws)) == _lib.FEM_OK and ws.value > 0
    assert lib.fem_tet_pattern_workspace(1000, 5000, C.byref(ws)) == _lib.FEM_OK
    assert ws.value >= 4 * 16 * 5000
    assert lib.fem_tet_nnz_bound(1000, 5000) == 1000 + 12 * 5000
    # the tetrahedron values refuse bad operator sets and flags on the host
    assert lib.fem_tet_assemble(2, 10, 5, 10, fake, fake, fake, fake, fake, fake, fake, 0,
                                None) == _lib.FEM_EINVAL
    assert lib.fem_tet_assemble(5, 10, 5, 10, fake, fake, fake, fake, fake, fake, fake,
                                _lib.FEM_ATOMIC, None) == _lib.FEM_EINVAL
    assert lib.fem_tet_pattern_set_path(_lib.FEM_PATTERN_ATOMIC) == _lib.FEM_EINVAL


def test_python_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    import paper_1305_3122_amd as fem
    me = torch.zeros((1, 3), dtype=torch.int32)
    with pytest.raises(ValueError, match="GPU"):
        fem.fem_pattern(me, 3)
