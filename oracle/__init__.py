"""CPU oracle for the round-synchronous DP + MD reduction (Algorithms 1-3).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_2109_06042_amd``) never imports it, and the two share no
code: the oracle is plain C written from the set definitions of supersedence
and domination (Section 3.1) and the steps of Algorithms 1, 2 and 3
(Section 4.1), see ``mhs_oracle.c``.

Every function here is pinned by ``-m "not gpu"`` tests against values the
paper fixes (the Appendix A counterexample, the tightness example after
Theorem 3.4), hand-derived fixtures under ``tests/golden/``, brute-force
optimum hitting sets on tiny inputs (the ILP of Section 5.1 solved by
enumeration), the lemma invariants (safety, exhaustiveness, transitivity) and
the f = 1 special case (Weihe's rules W1/W2), and a second implementation:
``kernelcpu`` runs the paper's sequential reduction (Algorithms 4-6, Section
4.2, ``mhs_kernelcpu.c``) on incrementally updated intersection counts, with
no code in common with the set-based oracle, and must delete the same
hyperedges and vertices in every iteration.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mhs_oracle.c")
_SRC_KCPU = os.path.join(_HERE, "mhs_kernelcpu.c")
_LIB = os.path.join(_HERE, "libmhs_oracle.so")

ALLPAIRS = 0
PRUNED = 1
RULE_DP = 0
RULE_SE = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (plain C99, single threaded)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, _SRC, _SRC_KCPU])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.mhs_oracle_validate.argtypes = [i32, i32, P, P, P]
        lib.mhs_oracle_validate.restype = ctypes.c_int
        for fn in (lib.mhs_oracle_dp_pass, lib.mhs_oracle_md_pass):
            fn.argtypes = [i32, i32, P, P, P, P, P, P, ctypes.c_int]
            fn.restype = i64
        lib.mhs_oracle_run.argtypes = [i32, i32, P, P, P, ctypes.c_int, i32, P, P, P]
        lib.mhs_oracle_run.restype = ctypes.c_int
        lib.mhs_oracle_run_fe.argtypes = [i32, i32, P, P, P, ctypes.c_int, i32, P, P, P, P, P, P]
        lib.mhs_oracle_run_fe.restype = ctypes.c_int
        lib.mhs_oracle_fe_pass.argtypes = [i32, i32, P, P, P, P, P, P, P]
        lib.mhs_oracle_fe_pass.restype = i64
        lib.mhs_kernelcpu_run.argtypes = [i32, i32, P, P, P, P, P, P]
        lib.mhs_kernelcpu_run.restype = ctypes.c_int
        lib.mhs_oracle_set_edge_rule.argtypes = [ctypes.c_int]
        lib.mhs_oracle_set_edge_rule.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(inst):
    ptr = np.ascontiguousarray(inst.edge_ptr, dtype=np.int64)
    if ptr.size == 0:
        ptr = np.zeros(1, np.int64)
    vtx = np.ascontiguousarray(inst.edge_vtx, dtype=np.int32)
    if vtx.size == 0:
        vtx = np.zeros(1, np.int32)
    dem = np.ascontiguousarray(inst.demand, dtype=np.int32)
    if dem.size == 0:
        dem = np.zeros(1, np.int32)
    return ptr, vtx, dem


@dataclass
class OracleResult:
    rounds: int
    death_e: np.ndarray   # int32[m]: round of deletion, 0 = survives
    death_v: np.ndarray   # int32[n]
    forced_v: np.ndarray = None   # bool[n]: forced into the solution (FE runs only)
    demand_out: np.ndarray = None  # int32[m]: demands at the end (FE runs only)
    n_forced: int = 0

    @property
    def forced(self):
        return (np.nonzero(self.forced_v)[0].astype(np.int32) if self.forced_v is not None
                else np.zeros(0, np.int32))

    @property
    def kept_e(self):
        return np.nonzero(self.death_e == 0)[0].astype(np.int32)

    @property
    def kept_v(self):
        return np.nonzero(self.death_v == 0)[0].astype(np.int32)

    def round_deletions(self, r: int):
        """(deleted hyperedges, deleted vertices) of productive round r >= 1."""
        return (np.nonzero(self.death_e == r)[0].astype(np.int32),
                np.nonzero(self.death_v == r)[0].astype(np.int32))


def validate(inst) -> int:
    ptr, vtx, dem = _csr(inst)
    return int(_load().mhs_oracle_validate(inst.n, inst.m, _ptr(ptr), _ptr(vtx), _ptr(dem)))


def run(inst, mode: int = PRUNED, max_rounds: int = -1, rule: int = RULE_DP) -> OracleResult:
    """Algorithm 3 to its fixpoint (or ``max_rounds`` productive rounds).

    ``rule`` selects the edge phase: RULE_DP (Algorithm 1, demand pushing)
    or RULE_SE (the superedge rule of Section 3.1 in its place)."""
    lib = _load()
    old = lib.mhs_oracle_set_edge_rule(rule)
    try:
        return _run(lib, inst, mode, max_rounds)
    finally:
        lib.mhs_oracle_set_edge_rule(old)


def _run(lib, inst, mode, max_rounds):
    ptr, vtx, dem = _csr(inst)
    de = np.zeros(max(inst.m, 1), np.int32)
    dv = np.zeros(max(inst.n, 1), np.int32)
    rounds = np.zeros(1, np.int32)
    rc = lib.mhs_oracle_run(inst.n, inst.m, _ptr(ptr), _ptr(vtx), _ptr(dem), mode,
                            max_rounds, _ptr(de), _ptr(dv), _ptr(rounds))
    if rc != 0:
        raise ValueError(f"oracle rejected instance (code {rc})")
    return OracleResult(int(rounds[0]), de[:inst.m].copy(), dv[:inst.n].copy())


def _pass(fn, inst, alive_v, alive_e, mode):
    ptr, vtx, dem = _csr(inst)
    av = np.ascontiguousarray(alive_v, dtype=np.uint8)
    ae = np.ascontiguousarray(alive_e, dtype=np.uint8)
    if av.size == 0:
        av = np.zeros(1, np.uint8)
    if ae.size == 0:
        ae = np.zeros(1, np.uint8)
    size = inst.m if fn == "dp" else inst.n
    kill = np.zeros(max(size, 1), np.uint8)
    f = _load().mhs_oracle_dp_pass if fn == "dp" else _load().mhs_oracle_md_pass
    rc = f(inst.n, inst.m, _ptr(ptr), _ptr(vtx), _ptr(dem), _ptr(av), _ptr(ae), _ptr(kill), mode)
    if rc < 0:
        raise MemoryError("oracle pass failed")
    return kill[:size].astype(bool)


def dp_pass(inst, alive_v, alive_e, mode: int = PRUNED, rule: int = RULE_DP) -> np.ndarray:
    """One Algorithm 1 pass (edge rule ``rule``): mask of alive hyperedges it deletes."""
    lib = _load()
    old = lib.mhs_oracle_set_edge_rule(rule)
    try:
        return _pass("dp", inst, alive_v, alive_e, mode)
    finally:
        lib.mhs_oracle_set_edge_rule(old)


def md_pass(inst, alive_v, alive_e, mode: int = PRUNED) -> np.ndarray:
    """One Algorithm 2 pass: boolean mask of alive vertices it deletes."""
    return _pass("md", inst, alive_v, alive_e, mode)


def run_fe(inst, mode: int = PRUNED, max_rounds: int = -1, rule: int = RULE_DP) -> OracleResult:
    """KernelGPU-FE: DP (or SE) + MD rounds with an FE pass (Section 3.1) in
    every iteration that DP and MD leave unchanged, to the common fixpoint."""
    lib = _load()
    old = lib.mhs_oracle_set_edge_rule(rule)
    try:
        ptr, vtx, dem = _csr(inst)
        de = np.zeros(max(inst.m, 1), np.int32)
        dv = np.zeros(max(inst.n, 1), np.int32)
        fv = np.zeros(max(inst.n, 1), np.uint8)
        fo = np.zeros(max(inst.m, 1), np.int32)
        rounds = np.zeros(1, np.int32)
        nf = np.zeros(1, np.int64)
        rc = lib.mhs_oracle_run_fe(inst.n, inst.m, _ptr(ptr), _ptr(vtx), _ptr(dem), mode, max_rounds,
                                   _ptr(de), _ptr(dv), _ptr(fv), _ptr(fo), _ptr(rounds), _ptr(nf))
    finally:
        lib.mhs_oracle_set_edge_rule(old)
    if rc != 0:
        raise ValueError(f"oracle rejected instance (code {rc})")
    return OracleResult(int(rounds[0]), de[:inst.m].copy(), dv[:inst.n].copy(),
                        fv[:inst.n].astype(bool), fo[:inst.m].copy(), int(nf[0]))


def kernelcpu(inst) -> OracleResult:
    """KernelCPU (Algorithms 4-6): the sequential exhaustive DP + MD reduction.

    Each iteration of its loop deletes what one round of Algorithm 3 deletes,
    so the result, including the per-iteration deletion trace, equals
    ``run(inst)``.  Memory grows with the nonzero intersection counts
    (sum of |E(v)|^2 plus sum of |e|^2 entries)."""
    rc = validate(inst)
    if rc != 0:
        raise ValueError(f"oracle rejected instance (code {rc})")
    ptr, vtx, dem = _csr(inst)
    de = np.zeros(max(inst.m, 1), np.int32)
    dv = np.zeros(max(inst.n, 1), np.int32)
    rounds = np.zeros(1, np.int32)
    rc = _load().mhs_kernelcpu_run(inst.n, inst.m, _ptr(ptr), _ptr(vtx), _ptr(dem),
                                   _ptr(de), _ptr(dv), _ptr(rounds))
    if rc != 0:
        raise MemoryError("KernelCPU ran out of memory")
    return OracleResult(int(rounds[0]), de[:inst.m].copy(), dv[:inst.n].copy())
