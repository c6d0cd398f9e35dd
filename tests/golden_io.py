"""Reader for the hand-checked fixtures under tests/golden/ (plain text).

Format, one item per line, ``#`` starts a comment:
    n <int>            number of vertices
    k <int>            budget (passed through untouched by DP/MD)
    e <f> : <v> <v>..  one hyperedge: its demand, then its vertices (0-based)
    rounds <int>       expected number of productive rounds of Algorithm 3
    death_e <r>..      expected deletion round per hyperedge (0 = survives)
    death_v <r>..      expected deletion round per vertex (0 = survives)
    opt <int>          optimum multiple hitting set size of the input
    rule se            the fixture reduces with the superedge rule SE in place of DP
    rule fe            the fixture reduces with FE alternated with DP + MD
    forced <v>..       expected vertices forced into the solution (FE)
    k_out <int>        expected budget after the reduction (FE)
"""
from __future__ import annotations

import os

import mhsgen

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name: str):
    n = k = None
    edges, dem = [], []
    expect = {}
    with open(os.path.join(GOLDEN_DIR, name)) as fh:
        for raw in fh:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            key, _, rest = line.partition(" ")
            if key == "n":
                n = int(rest)
            elif key == "k":
                k = int(rest)
            elif key == "e":
                f, _, vs = rest.partition(":")
                dem.append(int(f))
                edges.append([int(v) for v in vs.split()])
            elif key in ("death_e", "death_v", "forced"):
                expect[key] = [int(x) for x in rest.split()]
            elif key == "rule":
                expect["rule"] = rest.strip()
            else:
                expect[key] = int(rest)
    inst = mhsgen.from_edges(n, edges, dem, k=k or 0, name=name)
    return inst, expect


def all_fixtures():
    return sorted(f for f in os.listdir(GOLDEN_DIR) if f.endswith(".txt"))
