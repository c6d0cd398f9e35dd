"""Mutation check of the oracle's pins.

Each case plants one plausible mistake in a copy of the oracle source (a
flipped tie break, a strict inequality, a transposed set difference, a wrong
empty-set convention, a miscounted round, ...), compiles the copy on the CPU,
and asserts that the pins used in test_oracle.py (golden fixtures, optimum
preservation by brute force, exhaustiveness at the fixpoint) reject it.  A
mutant that passed every pin would mean the pins cannot tell that mistake
from the paper's method.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import brute
import golden_io
import mhsgen

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "mhs_oracle.c")

MUTANTS = {
    "dp_tiebreak_flipped": [("if (supersedes(&A, demand, i, j) && (!supersedes(&A, demand, j, i) || i < j))\n                    kill_e[j] = 1;",
                             "if (supersedes(&A, demand, i, j) && (!supersedes(&A, demand, j, i) || i > j))\n                    kill_e[j] = 1;"),
                            ("if (supersedes(&A, demand, i, j) && (!supersedes(&A, demand, j, i) || i < j)) {",
                             "if (supersedes(&A, demand, i, j) && (!supersedes(&A, demand, j, i) || i > j)) {")],
    "dp_no_tiebreak": [("if (supersedes(&A, demand, i, j) && (!supersedes(&A, demand, j, i) || i < j))\n                    kill_e[j] = 1;",
                        "if (supersedes(&A, demand, i, j))\n                    kill_e[j] = 1;"),
                       ("if (supersedes(&A, demand, i, j) && (!supersedes(&A, demand, j, i) || i < j)) {",
                        "if (supersedes(&A, demand, i, j)) {")],
    "dp_strict_inequality": [("return (int64_t)demand[i] - d >= (int64_t)demand[j];",
                              "return (int64_t)demand[i] - d > (int64_t)demand[j];")],
    "dp_weak_by_one": [("return (int64_t)demand[i] - d >= (int64_t)demand[j];",
                        "return (int64_t)demand[i] - d + 1 >= (int64_t)demand[j];")],
    "dp_transposed_difference": [("int64_t d = set_minus_size(A->cvtx + A->cptr[i], A->cptr[i + 1] - A->cptr[i],\n                               A->cvtx + A->cptr[j], A->cptr[j + 1] - A->cptr[j]);",
                                  "int64_t d = set_minus_size(A->cvtx + A->cptr[j], A->cptr[j + 1] - A->cptr[j],\n                               A->cvtx + A->cptr[i], A->cptr[i + 1] - A->cptr[i]);")],
    "dp_demand_terms_swapped": [("return (int64_t)demand[i] - d >= (int64_t)demand[j];",
                                 "return (int64_t)demand[j] - d >= (int64_t)demand[i];")],
    "md_count_twins_both_ways": [("if (dominates(&A, i, j) && (!dominates(&A, j, i) || i < j)) c++;\n            }\n            kill_v[j] = c >= maxf;\n        } else {",
                                  "if (dominates(&A, i, j)) c++;\n            }\n            kill_v[j] = c >= maxf;\n        } else {"),
                                 ("if (dominates(&A, i, j) && (!dominates(&A, j, i) || i < j)) c++;\n            }\n            kill_v[j] = c >= maxf;\n        }\n",
                                  "if (dominates(&A, i, j)) c++;\n            }\n            kill_v[j] = c >= maxf;\n        }\n")],
    "md_transposed_domination": [("return is_subset(A->iedg + A->iptr[j], A->iptr[j + 1] - A->iptr[j],\n                     A->iedg + A->iptr[i], A->iptr[i + 1] - A->iptr[i]);",
                                  "return is_subset(A->iedg + A->iptr[i], A->iptr[i + 1] - A->iptr[i],\n                     A->iedg + A->iptr[j], A->iptr[j + 1] - A->iptr[j]);")],
    "md_keeps_isolated": [("int32_t maxf = 0;                       /* max over the empty set: 0 */",
                           "int32_t maxf = 1;")],
    "md_min_demand": [("if (demand[A.iedg[q]] > maxf) maxf = demand[A.iedg[q]];",
                       "if (maxf == 0 || demand[A.iedg[q]] < maxf) maxf = demand[A.iedg[q]];")],
    "md_off_by_one": [("kill_v[j] = c >= maxf;\n        } else {", "kill_v[j] = c > maxf;\n        } else {"),
                      ("kill_v[j] = c >= maxf;\n        }\n", "kill_v[j] = c > maxf;\n        }\n")],
    "rounds_count_last_iteration": [("if (ke == 0 && kv == 0) break;\n        r++;",
                                     "r++;\n        if (ke == 0 && kv == 0) break;")],
    "single_round_only": [("if (ke == 0 && kv == 0) break;\n        r++;",
                           "r++;\n        break;")],
    "md_before_dp_same_round": [("int64_t ke = mhs_oracle_dp_pass(n, m, edge_ptr, edge_vtx, demand,\n                                        alive_v, alive_e, kill_e, mode);",
                                 "int64_t ke0 = mhs_oracle_md_pass(n, m, edge_ptr, edge_vtx, demand,\n                                        alive_v, alive_e, kill_v, mode);\n        for (int32_t v = 0; v < n; v++) if (kill_v[v]) { alive_v[v] = 0; death_v[v] = r + 1; }\n        int64_t ke = mhs_oracle_dp_pass(n, m, edge_ptr, edge_vtx, demand,\n                                        alive_v, alive_e, kill_e, mode);\n        ke += ke0 * 0;\n        if (ke0 > 0 && ke == 0) ke = 0;")],
}


def _build(name, tmp_path):
    src = open(SRC).read()
    for old, new in MUTANTS[name]:
        assert old in src, f"mutation anchor for {name} not found"
        src = src.replace(old, new)
    cpath = os.path.join(tmp_path, name + ".c")
    lpath = os.path.join(tmp_path, name + ".so")
    with open(cpath, "w") as fh:
        fh.write(src)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-w", "-o", lpath, cpath])
    lib = ctypes.CDLL(lpath)
    P, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.mhs_oracle_run.argtypes = [i32, i32, P, P, P, ctypes.c_int, i32, P, P, P]
    lib.mhs_oracle_run.restype = ctypes.c_int
    lib.mhs_oracle_set_edge_rule.argtypes = [ctypes.c_int]
    lib.mhs_oracle_set_edge_rule.restype = ctypes.c_int
    return lib


def _run(lib, inst, mode):
    ptr = np.ascontiguousarray(inst.edge_ptr, np.int64)
    vtx = np.ascontiguousarray(inst.edge_vtx if inst.edge_vtx.size else np.zeros(1), np.int32)
    dem = np.ascontiguousarray(inst.demand if inst.demand.size else np.zeros(1), np.int32)
    de = np.zeros(max(inst.m, 1), np.int32)
    dv = np.zeros(max(inst.n, 1), np.int32)
    rounds = np.zeros(1, np.int32)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = lib.mhs_oracle_run(inst.n, inst.m, p(ptr), p(vtx), p(dem), mode, 64, p(de), p(dv), p(rounds))
    assert rc == 0
    return int(rounds[0]), de[:inst.m], dv[:inst.n]


def _pins_reject(lib) -> str:
    for mode in (0, 1):
        for fx in golden_io.all_fixtures():
            inst, exp = golden_io.load(fx)
            if exp.get("rule") == "fe":
                continue          # the FE driver has pins of its own
            lib.mhs_oracle_set_edge_rule(1 if exp.get("rule") == "se" else 0)
            r, de, dv = _run(lib, inst, mode)
            lib.mhs_oracle_set_edge_rule(0)
            if r != exp["rounds"] or de.tolist() != exp["death_e"] or dv.tolist() != exp["death_v"]:
                return f"golden {fx} (mode {mode})"
        for i in range(80):
            inst = mhsgen.tiny(seed=0, idx=i)
            r, de, dv = _run(lib, inst, mode)
            kept_v = np.nonzero(dv == 0)[0].tolist()
            kept_e = np.nonzero(de == 0)[0].tolist()
            ek, dk = brute.reduced(inst, kept_v, kept_e)
            if brute.opt(inst.n, ek, dk, allowed=kept_v) != brute.opt(inst.n, inst.edges(), inst.demand.tolist()):
                return f"optimum changed on {inst.name} (mode {mode})"
            if brute.dp_applicable(ek, dk) or brute.md_applicable(kept_v, ek, dk):
                return f"rule still applies on {inst.name} (mode {mode})"
    return ""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_rejected(name, tmp_path):
    lib = _build(name, str(tmp_path))
    assert _pins_reject(lib) != "", f"mutant {name} passed every pin"
