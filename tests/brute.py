"""Brute-force checks on tiny hypergraphs (n <= 12), independent of the oracle.

These helpers pin the oracle to facts the paper and the mathematics fix:

* ``opt``: the minimum multiple hitting set, i.e. the ILP of Section 5.1
  (minimise |S| subject to |e & S| >= f(e) for every hyperedge) solved by
  enumerating every vertex subset.
* ``supersedes`` / ``dominators``: the set definitions of Section 3.1, used to
  check that no rule applies at a fixpoint (exhaustiveness, Lemmas 4.2(iii)
  and 4.3(iii)).
* ``dilworth``: the Dilworth number of the incidence graph (Section 2.2) as a
  largest antichain of the vicinal preorder, via Dilworth/Fulkerson (minimum
  chain cover = elements minus a maximum matching of the strict order).
"""
from __future__ import annotations

from itertools import combinations


def masks(edges):
    out = []
    for e in edges:
        b = 0
        for v in e:
            b |= 1 << v
        out.append(b)
    return out


def is_hitting_set(S: int, emasks, demand) -> bool:
    return all(bin(em & S).count("1") >= f for em, f in zip(emasks, demand))


def opt(n: int, edges, demand, allowed=None) -> int:
    """Minimum |S| over S subset of ``allowed`` (default all vertices) hitting every edge f times."""
    verts = list(range(n)) if allowed is None else sorted(allowed)
    em = masks(edges)
    for size in range(len(verts) + 1):
        for comb in combinations(verts, size):
            S = 0
            for v in comb:
                S |= 1 << v
            if is_hitting_set(S, em, demand):
                return size
    return -1  # infeasible


def all_hitting_sets(n: int, edges, demand, allowed):
    verts = sorted(allowed)
    em = masks(edges)
    out = []
    for size in range(len(verts) + 1):
        for comb in combinations(verts, size):
            S = 0
            for v in comb:
                S |= 1 << v
            if is_hitting_set(S, em, demand):
                out.append(S)
    return out


def supersedes(ei: set, fi: int, ej: set, fj: int) -> bool:
    """e_i supersedes e_j: f(e_i) - |e_i minus e_j| >= f(e_j)."""
    return fi - len(ei - ej) >= fj


def dominators(j: int, inc: dict) -> list:
    """All vertices i != j with E(v_j) a subset of E(v_i)."""
    return [i for i in inc if i != j and inc[j] <= inc[i]]


def reduced(inst, kept_v, kept_e):
    """The reduced hypergraph: kept hyperedges restricted to kept vertices."""
    kv = set(int(v) for v in kept_v)
    edges = inst.edges()
    out_edges = [sorted(set(edges[e]) & kv) for e in kept_e]
    out_dem = [int(inst.demand[e]) for e in kept_e]
    return out_edges, out_dem


def incidence(kept_v, edges_kept):
    inc = {int(v): set() for v in kept_v}
    for idx, e in enumerate(edges_kept):
        for v in e:
            inc[v].add(idx)
    return inc


def dp_applicable(edges_kept, dem_kept) -> bool:
    sets = [set(e) for e in edges_kept]
    for i in range(len(sets)):
        for j in range(len(sets)):
            if i != j and supersedes(sets[i], dem_kept[i], sets[j], dem_kept[j]):
                return True
    return False


def md_applicable(kept_v, edges_kept, dem_kept) -> bool:
    inc = incidence(kept_v, edges_kept)
    for j in inc:
        maxf = max((dem_kept[e] for e in inc[j]), default=0)
        if len(dominators(j, inc)) >= maxf:
            return True
    return False


def _max_matching(nl: int, adj) -> int:
    match_r = {}

    def aug(u, seen):
        for w in adj[u]:
            if w in seen:
                continue
            seen.add(w)
            if w not in match_r or aug(match_r[w], seen):
                match_r[w] = u
                return True
        return False

    return sum(1 for u in range(nl) if aug(u, set()))


def dilworth_incidence(n: int, edges) -> int:
    """Dilworth number of the incidence graph of (V, E).

    Graph vertices: 0..n-1 are hypergraph vertices, n+i is hyperedge i.
    Vicinal preorder: u below w iff N(u) is a subset of N[w]."""
    N = [set() for _ in range(n + len(edges))]
    for i, e in enumerate(edges):
        for v in e:
            N[v].add(n + i)
            N[n + i].add(v)
    tot = len(N)
    le = [[N[u] <= (N[w] | {w}) for w in range(tot)] for u in range(tot)]
    # collapse equivalence classes (u below w and w below u)
    rep = list(range(tot))
    for u in range(tot):
        for w in range(u):
            if le[u][w] and le[w][u]:
                rep[u] = rep[w]
                break
    reps = sorted(set(rep))
    idx = {r: k for k, r in enumerate(reps)}
    adj = [[] for _ in reps]
    for a in reps:
        for b in reps:
            if a != b and le[a][b]:
                adj[idx[a]].append(idx[b])
    return len(reps) - _max_matching(len(reps), adj)
