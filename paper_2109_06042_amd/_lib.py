"""ctypes declarations of the C ABI in include/mhsk.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhsk.so")

MHS_OK = 0
MHS_EINVAL = -1
MHS_ENOSPC = -2
MHS_EDEVICE = -3
MHS_EAGAIN = -4
MHS_EREJECT = -5

MHS_VARIANT_AUTO = 0
MHS_VARIANT_INT8 = 1
MHS_VARIANT_BITSET = 2
MHS_VARIANT_SPARSE = 3
MHS_VARIANT_HYBRID = 4
MHS_TRACE_ROUNDS = 1 << 8
MHS_INPUT_DEVICE = 1 << 12
MHS_NO_GRAPH = 1 << 9
MHS_GRAPH = 1 << 11
MHS_PROFILE = 1 << 10
MHS_RULE_SE = 1 << 16
MHS_GRID_MASK = 0xF << 24
MHS_STATIC_SCRATCH_BYTES = 64 << 20


def MHS_GRID_LOG2(k: int) -> int:
    return (k + 1) << 24


def MHS_GEMM_SCHED(k: int) -> int:
    return (k + 1) << 20


MHS_GEMM_SCHED_MASK = 0x3 << 20
MHS_RULE_FE = 1 << 17

# every symbol include/mhsk.h declares
EXPORTS = [
    "mhs_workspace_bytes", "mhs_run", "mhs_batch_workspace_bytes", "mhs_run_batch",
    "mhs_result_summary", "mhs_result_stats", "mhs_result_copy", "mhs_result_deaths",
    "mhs_result_demands", "mhs_result_forced",
    "mhs_result_round", "mhs_result_free", "mhs_results_take", "mhs_server_create", "mhs_server_submit",
    "mhs_server_poll", "mhs_server_pending", "mhs_server_arena_used", "mhs_server_destroy",
    "mhs_last_error", "mhs_version", "mhs_tune", "mhs_tune_reset", "mhs_result_status", "mhs_server_drain",
    "mhs_run_static", "mhs_run_batch_into",
]


class MhsInstance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("edge_ptr", ctypes.c_void_p), ("edge_vtx", ctypes.c_void_p),
                ("demand", ctypes.c_void_p), ("k", ctypes.c_int64), ("nnz", ctypes.c_int64)]


class MhsSummary(ctypes.Structure):
    _fields_ = [("n_kept", ctypes.c_int32), ("m_kept", ctypes.c_int32),
                ("n_forced", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("k_out", ctypes.c_int64)]


class MhsStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("gemm_launches", ctypes.c_int32),
                ("gemm_ms", ctypes.c_double), ("edge_gemm_ms", ctypes.c_double),
                ("vertex_gemm_ms", ctypes.c_double), ("rows_ms", ctypes.c_double),
                ("compact_ms", ctypes.c_double),
                ("round_end_ms", ctypes.c_double), ("issued_ops", ctypes.c_double),
                ("edge_issued_ops", ctypes.c_double), ("vertex_issued_ops", ctypes.c_double),
                ("blob_bytes", ctypes.c_double), ("encode_bytes", ctypes.c_double),
                ("terms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("sparse_ms", ctypes.c_double),
                ("edge_sparse_ms", ctypes.c_double), ("vertex_sparse_ms", ctypes.c_double)]


class MhsTuneReport(ctypes.Structure):
    _fields_ = [("best_flags", ctypes.c_uint32), ("candidates", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]


class MhsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mhsk error {code}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree HIP library.  There is no fallback: a missing library
    is an error."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    # torch first: its HIP runtime (same soname) then serves this library too,
    # so torch's streams and allocations are valid here.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, u64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                 ctypes.c_uint64, ctypes.c_size_t)
    PI = ctypes.POINTER(MhsInstance)
    lib.mhs_workspace_bytes.argtypes = [i32, i32, i64, u32]
    lib.mhs_workspace_bytes.restype = sz
    lib.mhs_run.argtypes = [PI, u32, P, sz, P, ctypes.POINTER(P)]
    lib.mhs_run.restype = ctypes.c_int
    lib.mhs_batch_workspace_bytes.argtypes = [PI, i32, u32]
    lib.mhs_batch_workspace_bytes.restype = sz
    lib.mhs_run_batch.argtypes = [PI, i32, u32, P, sz, P, ctypes.POINTER(P)]
    lib.mhs_run_batch.restype = ctypes.c_int
    lib.mhs_result_summary.argtypes = [P, ctypes.POINTER(MhsSummary)]
    lib.mhs_result_stats.argtypes = [P, ctypes.POINTER(MhsStats)]
    lib.mhs_result_copy.argtypes = [P, P, P, P]
    lib.mhs_result_deaths.argtypes = [P, P, P]
    lib.mhs_result_demands.argtypes = [P, P]
    lib.mhs_result_forced.argtypes = [P, P]
    lib.mhs_result_round.argtypes = [P, i32, P, P, P, P]
    lib.mhs_result_free.argtypes = [P]
    lib.mhs_result_free.restype = None
    lib.mhs_results_take.argtypes = [ctypes.POINTER(P), i32, ctypes.POINTER(MhsSummary), ctypes.POINTER(MhsStats),
                                     P, P, P, P]
    lib.mhs_server_create.argtypes = [P, sz, i32, u32, P, ctypes.POINTER(P)]
    lib.mhs_server_submit.argtypes = [P, PI, u64]
    lib.mhs_server_poll.argtypes = [P, i32, ctypes.POINTER(u64), ctypes.POINTER(P), ctypes.POINTER(i32)]
    lib.mhs_server_pending.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.mhs_server_arena_used.argtypes = [P, ctypes.POINTER(sz)]
    lib.mhs_server_destroy.argtypes = [P]
    lib.mhs_server_destroy.restype = None
    lib.mhs_tune.argtypes = [PI, i32, u32, P, sz, P, ctypes.POINTER(MhsTuneReport)]
    lib.mhs_tune_reset.argtypes = []
    lib.mhs_tune_reset.restype = None
    lib.mhs_last_error.restype = ctypes.c_char_p
    lib.mhs_version.restype = ctypes.c_char_p
    lib.mhs_run_batch_into.argtypes = [PI, i32, u32, P, sz, P, ctypes.POINTER(MhsSummary), ctypes.POINTER(MhsStats),
                                       P, P, P, P]
    lib.mhs_result_status.argtypes = [P]
    lib.mhs_server_drain.argtypes = [P]
    lib.mhs_run_static.argtypes = [PI, u32, P, ctypes.POINTER(MhsSummary), P, P]
    verify_build(lib)
    _lib = lib
    return lib


def library_sha(lib) -> str:
    """Source hash the loaded library was built from (mhs_version's src=)."""
    v = lib.mhs_version().decode()
    return v.rsplit("src=", 1)[-1] if "src=" in v else ""


def verify_build(lib):
    """Refuse a library built from other sources than the ones in this tree."""
    from .build import source_sha
    want, got = source_sha(), library_sha(lib)
    if want != got:
        raise ImportError(f"{LIB_PATH} was built from sources {got or 'of unknown hash'}, the tree holds "
                          f"{want}: rebuild it (__graft_entry__.build())")


def check(rc: int):
    if rc != MHS_OK:
        raise MhsError(rc, load().mhs_last_error().decode())
