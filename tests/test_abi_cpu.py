"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every function include/mhsk.h declares, workspace sizing, and the
argument / instance validation that runs before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

import mhsgen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mhsk.h")


def _lib():
    from paper_2109_06042_amd import _lib
    return _lib


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mhs_[a-z_]+)\s*\(", src)))


def test_header_matches_binding_list():
    assert _declared() == sorted(_lib().EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib().load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.mhs_version()


def test_library_built_from_this_tree():
    """mhs_version() carries the hash of the sources the library was built
    from; it must be the hash of the sources in the tree."""
    from paper_2109_06042_amd import build
    lib = _lib().load()
    assert _lib().library_sha(lib) == build.source_sha()


def test_workspace_sizes_monotone():
    lib = _lib().load()
    a = lib.mhs_workspace_bytes(200, 1000, 5000, 0)
    b = lib.mhs_workspace_bytes(400, 1000, 5000, 0)
    c = lib.mhs_workspace_bytes(200, 2000, 5000, 0)
    d = lib.mhs_workspace_bytes(200, 1000, 9000, 0)
    assert 0 < a < b and a < c and a < d
    # device inputs need no staging copy
    assert lib.mhs_workspace_bytes(200, 1000, 5000, _lib().MHS_INPUT_DEVICE) < a
    assert lib.mhs_workspace_bytes(-1, 5, 5, 0) == 0
    # the dense operand window is at most rows x K, both orientations
    big = lib.mhs_workspace_bytes(20000, 200000, 1_200_000, 0)
    assert 4.0e9 < big < 4.3e9


def _run_host(inst, flags=0):
    L = _lib()
    lib = L.load()
    ptr = np.ascontiguousarray(inst.edge_ptr, np.int64)
    vtx = np.ascontiguousarray(inst.edge_vtx if inst.edge_vtx.size else np.zeros(1), np.int32)
    dem = np.ascontiguousarray(inst.demand if inst.demand.size else np.zeros(1), np.int32)
    st = L.MhsInstance(inst.n, inst.m, ptr.ctypes.data, vtx.ctypes.data, dem.ctypes.data, inst.k)
    out = ctypes.c_void_p()
    # no workspace: every check below must fail before the device is touched
    rc = lib.mhs_run(ctypes.byref(st), flags, None, 0, None, ctypes.byref(out))
    return rc, lib.mhs_last_error().decode()


@pytest.mark.parametrize("case,edges,dem,n", [
    ("range", [[0, 3]], [1], 3),
    ("demand_high", [[0, 1]], [3], 3),
    ("demand_zero", [[0, 1]], [0], 3),
    ("empty_edge", [[]], [1], 3),
])
def test_invalid_instances_rejected_like_oracle(case, edges, dem, n):
    inst = mhsgen.from_edges(n, edges, dem)
    assert oracle.validate(inst) != 0
    rc, msg = _run_host(inst)
    assert rc == _lib().MHS_EINVAL, (case, msg)


def test_unsorted_and_duplicate_members_rejected():
    for vtx in ([2, 1], [1, 1]):
        inst = mhsgen.Instance(n=3, m=1, edge_ptr=np.array([0, 2], np.int64),
                               edge_vtx=np.array(vtx, np.int32), demand=np.array([1], np.int32))
        assert oracle.validate(inst) == -3
        rc, msg = _run_host(inst)
        assert rc == _lib().MHS_EINVAL and "strictly increasing" in msg


def test_bad_edge_ptr_rejected():
    inst = mhsgen.Instance(n=3, m=2, edge_ptr=np.array([0, 2, 1], np.int64),
                           edge_vtx=np.array([0, 1], np.int32), demand=np.array([1, 1], np.int32))
    rc, _ = _run_host(inst)
    assert rc == _lib().MHS_EINVAL


def test_unknown_flags_rejected():
    inst = mhsgen.plain(seed=0)
    for f in (1 << 30, 7, _lib().MHS_GRID_LOG2(7)):
        rc, msg = _run_host(inst, f)
        assert rc == _lib().MHS_EINVAL and "workspace" not in msg, msg
    # the rule flags and the trace flag are accepted (the call then stops at
    # the missing workspace)
    for f in (_lib().MHS_RULE_SE, _lib().MHS_RULE_FE, _lib().MHS_RULE_SE | _lib().MHS_RULE_FE,
              _lib().MHS_TRACE_ROUNDS):
        rc, msg = _run_host(inst, f)
        assert rc == _lib().MHS_EINVAL and "workspace" in msg, msg


def test_valid_instance_needs_workspace():
    rc, msg = _run_host(mhsgen.plain(seed=0))
    assert rc == _lib().MHS_EINVAL and "workspace" in msg


def test_result_accessors_reject_null():
    lib = _lib().load()
    s = _lib().MhsSummary()
    assert lib.mhs_result_summary(None, ctypes.byref(s)) == _lib().MHS_EINVAL
    assert lib.mhs_result_round(None, 1, None, None, None, None) == _lib().MHS_EINVAL
    # the batch export writes and frees nothing when a result is missing
    outs = (ctypes.c_void_p * 2)()
    assert lib.mhs_results_take(outs, 2, None, None, None, None, None, None) == _lib().MHS_EINVAL
    assert "NULL result 0" in lib.mhs_last_error().decode()
    assert lib.mhs_results_take(outs, 0, None, None, None, None, None, None) == _lib().MHS_OK
