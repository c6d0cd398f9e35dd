"""Multiple Hitting Set kernelization (DP + MD, Algorithm 3) on MI355X.

Thin Python binding over the C ABI of ``libmhsk.so`` (include/mhsk.h).  The
binding only marshals arguments: every step of the reduction runs in the HIP
kernels of the library.  PyTorch provides device memory (the workspace) and
the stream.  Importing this package does not load the library; the first call
does, and fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes
from collections.abc import Sequence
from dataclasses import dataclass, field

import numpy as np

from . import _lib
from ._lib import (MHS_RULE_FE, MHS_RULE_SE, MHS_INPUT_DEVICE, MHS_GRAPH, MHS_NO_GRAPH, MHS_PROFILE, MHS_VARIANT_AUTO,
                   MHS_VARIANT_BITSET, MHS_VARIANT_HYBRID, MHS_VARIANT_INT8, MHS_VARIANT_SPARSE, MhsError)

__all__ = ["reduce", "reduce_static", "reduce_batch", "tune", "tune_reset", "Result", "Server", "DeviceInstance", "workspace_bytes",
           "MhsError", "MHS_INPUT_DEVICE", "MHS_GRAPH", "MHS_NO_GRAPH", "MHS_PROFILE", "MHS_VARIANT_INT8",
           "MHS_VARIANT_AUTO", "MHS_VARIANT_BITSET",
           "MHS_VARIANT_SPARSE", "MHS_VARIANT_HYBRID", "MHS_RULE_SE", "MHS_RULE_FE"]


@dataclass
class Result:
    """Result of one reduction (original ids)."""

    rounds: int
    death_e: np.ndarray   # int32[m]: productive round of deletion, 0 = kept
    death_v: np.ndarray   # int32[n]
    k_out: int = 0
    stats: dict = field(default_factory=dict)
    forced_v: np.ndarray = None    # bool[n]: forced into the solution (MHS_RULE_FE)
    demand_out: np.ndarray = None  # int32[m]: demands at the end (0 if deleted)
    n_forced: int = 0

    @property
    def forced(self):
        return np.nonzero(self.forced_v)[0].astype(np.int32)

    @property
    def kept_e(self):
        return np.nonzero(self.death_e == 0)[0].astype(np.int32)

    @property
    def kept_v(self):
        return np.nonzero(self.death_v == 0)[0].astype(np.int32)

    def round_deletions(self, r: int):
        return (np.nonzero(self.death_e == r)[0].astype(np.int32),
                np.nonzero(self.death_v == r)[0].astype(np.int32))


def _torch():
    import torch
    return torch


def _host_struct(inst):
    """mhs_instance over host numpy arrays (kept alive by the returned tuple)."""
    ptr = np.ascontiguousarray(inst.edge_ptr, dtype=np.int64)
    vtx = np.ascontiguousarray(inst.edge_vtx, dtype=np.int32)
    dem = np.ascontiguousarray(inst.demand, dtype=np.int32)
    s = _lib.MhsInstance(int(inst.n), int(inst.m),
                         ptr.ctypes.data if ptr.size else None,
                         vtx.ctypes.data if vtx.size else None,
                         dem.ctypes.data if dem.size else None, int(inst.k),
                         int(ptr[-1]) if inst.m else 0)
    return s, (ptr, vtx, dem)


class DeviceInstance:
    """An instance whose CSR already lives in device memory (torch tensors)."""

    def __init__(self, inst, device="cuda"):
        torch = _torch()
        self.n, self.m, self.k = int(inst.n), int(inst.m), int(inst.k)
        self.nnz = int(inst.edge_ptr[-1]) if inst.m else 0
        self.size_nnz = self.nnz          # for workspace sizing
        self.edge_ptr = torch.as_tensor(np.ascontiguousarray(inst.edge_ptr, np.int64)).to(device)
        self.edge_vtx = torch.as_tensor(np.ascontiguousarray(inst.edge_vtx, np.int32)).to(device)
        self.demand = torch.as_tensor(np.ascontiguousarray(inst.demand, np.int32)).to(device)
        self._struct, self._key = None, None

    def struct(self):
        # rebuilt when a field was reassigned since (tests change nnz hints)
        key = (self.n, self.m, self.k, self.nnz, id(self.edge_ptr), id(self.edge_vtx), id(self.demand))
        if self._struct is None or self._key != key:
            self._key = key
            self._struct = _lib.MhsInstance(self.n, self.m,
                                            self.edge_ptr.data_ptr() if self.edge_ptr.numel() else None,
                                            self.edge_vtx.data_ptr() if self.edge_vtx.numel() else None,
                                            self.demand.data_ptr() if self.demand.numel() else None, self.k,
                                            self.nnz)
        return self._struct


def workspace_bytes(n: int, m: int, nnz: int, flags: int = 0) -> int:
    return int(_lib.load().mhs_workspace_bytes(n, m, nnz, flags))


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _alloc(nbytes: int, device="cuda"):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _result_from_handle(lib, handle, n: int, m: int) -> Result:
    try:
        s = _lib.MhsSummary()
        _lib.check(lib.mhs_result_summary(handle, ctypes.byref(s)))
        st = _lib.MhsStats()
        _lib.check(lib.mhs_result_stats(handle, ctypes.byref(st)))
        # filled completely by the library (one spare element keeps empty
        # instances' pointers valid); the results are views of them
        de = np.empty(max(m, 1), np.int32)
        dv = np.empty(max(n, 1), np.int32)
        fo = np.empty(max(m, 1), np.int32)
        fv = np.empty(max(n, 1), np.uint8)
        _lib.check(lib.mhs_result_deaths(handle, de.ctypes.data, dv.ctypes.data))
        _lib.check(lib.mhs_result_demands(handle, fo.ctypes.data))
        _lib.check(lib.mhs_result_forced(handle, fv.ctypes.data))
        stats = {f: getattr(st, f) for f, _ in _lib.MhsStats._fields_}
        return Result(int(s.rounds), de[:m], dv[:n], int(s.k_out), stats,
                      fv[:n].view(np.bool_), fo[:m], int(s.n_forced))
    finally:
        lib.mhs_result_free(handle)


def reduce(inst, flags: int = 0, workspace=None, stream=None) -> Result:
    """Reduce one instance to the fixpoint of Algorithm 3 on the current GPU.

    ``inst`` is an ``mhsgen.Instance`` (host arrays) or a ``DeviceInstance``
    (then MHS_INPUT_DEVICE is implied).  ``workspace`` is an optional uint8
    CUDA tensor of at least ``workspace_bytes`` bytes."""
    lib = _lib.load()
    if isinstance(inst, DeviceInstance):
        flags |= MHS_INPUT_DEVICE
        st = inst.struct()
        keep = None
        n, m, nnz = inst.n, inst.m, max(inst.nnz, inst.size_nnz)
    else:
        st, keep = _host_struct(inst)
        n, m, nnz = int(inst.n), int(inst.m), int(inst.edge_ptr[-1]) if inst.m else 0
    need = int(lib.mhs_workspace_bytes(n, m, nnz, flags))
    ws = workspace if workspace is not None and workspace.numel() >= need else _alloc(need)
    h = ctypes.c_void_p()
    rc = lib.mhs_run(ctypes.byref(st), flags, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                     _stream_ptr(stream), ctypes.byref(h))
    del keep
    _lib.check(rc)
    return _result_from_handle(lib, h, n, m)


def reduce_static(inst, flags: int = 0, stream=None) -> Result:
    """Reduce one instance with the library's static device scratch
    (mhs_run_static: nothing is allocated on the device); the instance's
    workspace must fit MHS_STATIC_SCRATCH_BYTES."""
    lib = _lib.load()
    if isinstance(inst, DeviceInstance):
        flags |= MHS_INPUT_DEVICE
        st, keep = inst.struct(), None
    else:
        st, keep = _host_struct(inst)
    n, m = int(inst.n), int(inst.m)
    de = np.empty(max(m, 1), np.int32)
    dv = np.empty(max(n, 1), np.int32)
    s = _lib.MhsSummary()
    rc = lib.mhs_run_static(ctypes.byref(st), flags, _stream_ptr(stream), ctypes.byref(s), de.ctypes.data,
                            dv.ctypes.data)
    del keep
    _lib.check(rc)
    return Result(int(s.rounds), de[:m], dv[:n], int(s.k_out), {}, None, None, int(s.n_forced))


def _batch_structs(insts, flags):
    """mhs_instance array of a batch: host instances, or DeviceInstances
    (then MHS_INPUT_DEVICE is implied; all members must be of one kind)."""
    dev = [isinstance(i, DeviceInstance) for i in insts]
    if any(dev) and not all(dev):
        raise ValueError("a batch holds host instances or device instances, not both")
    if insts and all(dev):
        flags |= MHS_INPUT_DEVICE
    arr = (_lib.MhsInstance * max(len(insts), 1))()
    keep = []
    for i, inst in enumerate(insts):
        if dev[i]:
            arr[i] = inst.struct()
        else:
            s, k = _host_struct(inst)
            arr[i] = s
            keep.append(k)
    return arr, keep, flags


def batch_workspace_bytes(insts, flags: int = 0) -> int:
    lib = _lib.load()
    arr, keep, flags = _batch_structs(insts, flags)
    return int(lib.mhs_batch_workspace_bytes(arr, len(insts), flags))


def reduce_batch(insts, flags: int = 0, workspace=None, stream=None):
    """Reduce many instances together (shared launches per phase): host
    instances, or DeviceInstances whose arrays already live in HBM.  Returns
    a BatchResults, one Result per instance in order."""
    lib = _lib.load()
    cnt = len(insts)
    arr, keep, flags = _batch_structs(insts, flags)
    need = int(lib.mhs_batch_workspace_bytes(arr, cnt, flags))
    ws = workspace if workspace is not None and workspace.numel() >= need else _alloc(need)
    # results written by the library straight into the arrays the Results view
    ns, ms = [int(i.n) for i in insts], [int(i.m) for i in insts]
    moff = np.concatenate([[0], np.cumsum(ms, dtype=np.int64)])
    noff = np.concatenate([[0], np.cumsum(ns, dtype=np.int64)])
    M, N = int(moff[-1]), int(noff[-1])
    sums = (_lib.MhsSummary * max(cnt, 1))()
    stats = (_lib.MhsStats * max(cnt, 1))()
    de = np.empty(max(M, 1), np.int32)
    fo = np.empty(max(M, 1), np.int32)
    dv = np.empty(max(N, 1), np.int32)
    fv = np.empty(max(N, 1), np.uint8)
    rc = lib.mhs_run_batch_into(arr, cnt, flags, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream),
                                sums, stats, de.ctypes.data, dv.ctypes.data, fo.ctypes.data, fv.ctypes.data)
    _lib.check(rc)
    return _batch_results(cnt, moff, noff, sums, stats, de, dv, fo, fv)


class BatchResults(Sequence):
    """Results of a batch: a sequence of Result, each a view of four arrays
    shared by the whole batch (death_e, death_v, demand_out, forced_v, in
    instance order) and built when first asked for."""

    def __init__(self, cnt, moff, noff, sums, stats, de, dv, fo, fv):
        self._cnt = cnt
        self._moff, self._noff = moff, noff
        self._sums, self._stats = sums, stats
        self.death_e, self.death_v, self.demand_out = de[:int(moff[-1])], dv[:int(noff[-1])], fo[:int(moff[-1])]
        self.forced_v = fv[:int(noff[-1])].view(np.bool_)
        self._items = [None] * cnt

    def __len__(self):
        return self._cnt

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[k] for k in range(*i.indices(self._cnt))]
        i = int(i)
        if i < 0:
            i += self._cnt
        if not 0 <= i < self._cnt:
            raise IndexError("batch result index out of range")
        r = self._items[i]
        if r is None:
            s, st = self._sums[i], self._stats[i]
            a, b, c, d = self._moff[i], self._moff[i + 1], self._noff[i], self._noff[i + 1]
            stats = {f: getattr(st, f) for f, _ in _lib.MhsStats._fields_}
            r = Result(int(s.rounds), self.death_e[a:b], self.death_v[c:d], int(s.k_out), stats,
                       self.forced_v[c:d], self.demand_out[a:b], int(s.n_forced))
            self._items[i] = r
        return r


def _batch_results(cnt, moff, noff, sums, stats, de, dv, fo, fv) -> BatchResults:
    return BatchResults(cnt, moff, noff, sums, stats, de, dv, fo, fv)


def _results_take(lib, outs, ns, ms) -> BatchResults:
    """Results of a batch, exported with one library call (mhs_results_take);
    each result's arrays are views of four arrays shared by the batch."""
    cnt = len(ns)
    moff = np.concatenate([[0], np.cumsum(ms, dtype=np.int64)])
    noff = np.concatenate([[0], np.cumsum(ns, dtype=np.int64)])
    M, N = int(moff[-1]), int(noff[-1])
    sums = (_lib.MhsSummary * max(cnt, 1))()
    stats = (_lib.MhsStats * max(cnt, 1))()
    de = np.empty(max(M, 1), np.int32)
    fo = np.empty(max(M, 1), np.int32)
    dv = np.empty(max(N, 1), np.int32)
    fv = np.empty(max(N, 1), np.uint8)
    try:
        _lib.check(lib.mhs_results_take(outs, cnt, sums, stats, de.ctypes.data, dv.ctypes.data,
                                        fo.ctypes.data, fv.ctypes.data))
    except Exception:
        for i in range(cnt):
            if outs[i]:
                lib.mhs_result_free(ctypes.c_void_p(outs[i]))
        raise
    return _batch_results(cnt, moff, noff, sums, stats, de, dv, fo, fv)


def tune(sample, flags: int = 0, workspace=None, stream=None) -> dict:
    """Run the schedule autotuner on sample instances (see mhs_tune): host
    instances, or DeviceInstances whose arrays already live in HBM (then the
    timings leave out the host-to-device copies)."""
    lib = _lib.load()
    cnt = len(sample)
    arr, keep, flags = _batch_structs(sample, flags)
    need = int(lib.mhs_batch_workspace_bytes(arr, cnt, flags))
    ws = workspace if workspace is not None and workspace.numel() >= need else _alloc(need)
    rep = _lib.MhsTuneReport()
    _lib.check(lib.mhs_tune(arr, cnt, flags, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                            _stream_ptr(stream), ctypes.byref(rep)))
    return {"best_flags": int(rep.best_flags), "candidates": int(rep.candidates),
            "best_ms": rep.best_ms, "default_ms": rep.default_ms}


def tune_reset():
    _lib.load().mhs_tune_reset()


class Server:
    """Continuous-batching server over a device arena (see mhs_server_* in include/mhsk.h)."""

    def __init__(self, arena_bytes: int, max_slots: int = 256, flags: int = 0, stream=None):
        self._lib = _lib.load()
        self.arena = _alloc(arena_bytes)
        self._h = ctypes.c_void_p()
        self._sizes = {}
        _lib.check(self._lib.mhs_server_create(ctypes.c_void_p(self.arena.data_ptr()), self.arena.numel(),
                                               max_slots, flags, _stream_ptr(stream), ctypes.byref(self._h)))

    def submit(self, inst, request_id: int):
        st, keep = _host_struct(inst)
        rc = self._lib.mhs_server_submit(self._h, ctypes.byref(st), ctypes.c_uint64(request_id))
        del keep
        _lib.check(rc)
        self._sizes[int(request_id)] = (int(inst.n), int(inst.m))

    def poll(self, cap: int = 1024):
        """Finished requests as (request id, Result); a request the device
        could not reduce comes back as (request id, MhsError).  Never waits."""
        ids = (ctypes.c_uint64 * cap)()
        res = (ctypes.c_void_p * cap)()
        nd = ctypes.c_int32(0)
        rc = self._lib.mhs_server_poll(self._h, cap, ids, res, ctypes.byref(nd))
        if rc == _lib.MHS_EAGAIN:      # nothing finished yet (or idle)
            return []
        _lib.check(rc)
        out, good = [], []
        for i in range(nd.value):
            rid = int(ids[i])
            st = self._lib.mhs_result_status(ctypes.c_void_p(res[i]))
            if st != _lib.MHS_OK:
                err = MhsError(st, self._lib.mhs_last_error().decode())
                self._lib.mhs_result_free(ctypes.c_void_p(res[i]))
                self._sizes.pop(rid, None)
                out.append((rid, err))
            else:
                good.append((rid, res[i]))
        if good:
            arr = (ctypes.c_void_p * len(good))(*[h for _, h in good])
            shapes = [self._sizes.pop(rid) for rid, _ in good]
            out += list(zip([rid for rid, _ in good],
                            _results_take(self._lib, arr, [n for n, _ in shapes], [m for _, m in shapes])))
        return out

    def drain(self):
        """Run everything queued or resident to its fixpoint (blocking); the
        results are then returned by poll."""
        _lib.check(self._lib.mhs_server_drain(self._h))

    def pending(self):
        q, r = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(self._lib.mhs_server_pending(self._h, ctypes.byref(q), ctypes.byref(r)))
        return q.value, r.value

    def arena_used(self) -> int:
        u = ctypes.c_size_t()
        _lib.check(self._lib.mhs_server_arena_used(self._h, ctypes.byref(u)))
        return u.value

    def close(self):
        if self._h:
            self._lib.mhs_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
