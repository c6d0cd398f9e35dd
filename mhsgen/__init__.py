"""Seeded synthetic Multiple Hitting Set instances.

This module only draws random hypergraphs in CSR form.  It contains none of
the reduction arithmetic (no intersection counts, no supersedence or
domination tests), so both the CPU oracle and the GPU path may import it.

An instance is a hypergraph H = (V, E) with vertices 0..n-1, hyperedges
0..m-1, a demand f(e) in {1, .., |e|} per hyperedge and a budget k
(problem definition, Section 1).  Hyperedges are stored in CSR:
``edge_ptr`` (int64, m+1 entries) and ``edge_vtx`` (int32, strictly
increasing within each hyperedge).

Workload families (sizes follow the measured configurations; the paper's own
data sets, NCI60 and the GIRG transport instances of Section 5, are not
available, so these stand in for them):

* ``plain``     n=200, m=1000, |e| ~ U{2..8} members drawn uniformly without
                replacement, f = 1, k = 50.
* ``transport`` n=8000 vertices on a line, m=60000 hyperedges, each a random
                contiguous interval of length U{5..40} whose members are kept
                independently with p=0.8 (empty draws are redrawn), f = 1.
* ``multidemand`` n=20000, m=200000, |e| from the discrete power law
                P(s) ~ s^-2.2 on {2..200}, members uniform without replacement,
                f ~ U{1,2,3} capped at |e|.
* ``batch``     one of 512 instances: n ~ U{100..4000}, m = round(n*U(5,10)),
                interval style (as ``transport``) or uniform style (as
                ``plain``) with probability 1/2 each, f ~ U{1,2} capped.
* ``serve``     one request: u ~ U(0,1), n = round(100*300^u),
                m = round(500*600^u), style as ``batch``, f ~ U{1,2,3} capped.
* ``nci60_shaped`` n=7124, m=152 (the paper's NCI60 shape, vertices far
                outnumber hyperedges), nested memberships, f = min(alpha, |e|).
* ``girg_shaped`` n=15015, m=1903, interval hyperedges of mean size 8 (the
                paper's GIRG transport shape), f = min(alpha, |e|).
* ``tiny``      n <= 12, m <= 14 random hypergraphs with planted twin
                hyperedges, nested hyperedges and twin vertices, f <= 3.

Every draw uses ``numpy.random.default_rng(SeedSequence([family_id, idx,
seed]))`` so an instance is a pure function of (family, idx, seed).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

FAMILY_IDS = {
    "plain": 1,
    "transport": 2,
    "multidemand": 3,
    "batch": 4,
    "serve": 5,
    "tiny": 10,
    "tiny_dense": 11,
    "nci60_shaped": 20,
    "girg_shaped": 21,
}


@dataclass
class Instance:
    """A Multiple Hitting Set instance in CSR form (host memory)."""

    n: int
    m: int
    edge_ptr: np.ndarray  # int64[m+1]
    edge_vtx: np.ndarray  # int32[nnz], strictly increasing within each edge
    demand: np.ndarray    # int32[m], 1 <= demand[e] <= |e|
    k: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.edge_ptr[-1]) if self.m > 0 else 0

    def edges(self):
        """List of hyperedges as Python lists (small instances only)."""
        p = self.edge_ptr
        return [self.edge_vtx[p[i]:p[i + 1]].tolist() for i in range(self.m)]


def _rng(family: str, idx: int, seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([FAMILY_IDS[family], idx, seed]))


def from_edges(n: int, edges, demand=None, k: int = 0, name: str = "") -> Instance:
    """Build an Instance from a list of vertex lists (sorted here)."""
    m = len(edges)
    sizes = np.array([len(e) for e in edges], dtype=np.int64)
    ptr = np.zeros(m + 1, dtype=np.int64)
    if m:
        ptr[1:] = np.cumsum(sizes)
    vtx = np.array([v for e in edges for v in sorted(e)], dtype=np.int32)
    if demand is None:
        dem = np.ones(m, dtype=np.int32)
    else:
        dem = np.asarray(demand, dtype=np.int32).reshape(m)
    return Instance(n=n, m=m, edge_ptr=ptr, edge_vtx=vtx, demand=dem, k=k, name=name)


def _csr(n, sizes, vtx, demand, k, name, meta=None) -> Instance:
    m = len(sizes)
    ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(sizes, out=ptr[1:])
    return Instance(n=n, m=m, edge_ptr=ptr, edge_vtx=np.asarray(vtx, dtype=np.int32),
                    demand=np.asarray(demand, dtype=np.int32), k=k, name=name,
                    meta=dict(meta or {}))


def _uniform_members(rng, n: int, sizes: np.ndarray):
    """Flat CSR members: for each requested size s, s distinct vertices of
    0..n-1 drawn uniformly, sorted.  Rows of equal size are drawn together;
    rows with a repeated vertex are redrawn (rejection keeps the draw
    uniform)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    m = len(sizes)
    ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(sizes, out=ptr[1:])
    vtx = np.zeros(int(ptr[-1]), dtype=np.int32)
    for s in np.unique(sizes):
        s = int(s)
        if s > n:
            raise ValueError("hyperedge size exceeds n")
        todo = np.nonzero(sizes == s)[0]
        while len(todo):
            if 2 * s * s > n:
                # a repeat-free draw would be unlikely (birthday bound): take
                # the first s of a random permutation per row instead
                draw = np.argsort(rng.random((len(todo), n)), axis=1)[:, :s]
                draw.sort(axis=1)
                bad = np.zeros(len(todo), dtype=bool)
            else:
                draw = rng.integers(0, n, size=(len(todo), s))
                draw.sort(axis=1)
                bad = (np.diff(draw, axis=1) == 0).any(axis=1) if s > 1 else np.zeros(len(todo), bool)
            ok = todo[~bad]
            pos = ptr[ok][:, None] + np.arange(s)[None, :]
            vtx[pos] = draw[~bad]
            todo = todo[bad]
    return sizes, vtx


def _interval_members(rng, n: int, m: int, lmin=5, lmax=40, p=0.8):
    """Flat CSR members of m hyperedges, each the kept members (probability p
    each) of a random contiguous interval of length U{lmin..lmax} (clamped to
    n); empty draws are redrawn."""
    lmax_eff = min(lmax, n)
    lmin_eff = min(lmin, lmax_eff)
    L = np.zeros(m, dtype=np.int64)
    start = np.zeros(m, dtype=np.int64)
    keep = np.zeros((m, lmax_eff), dtype=bool)
    todo = np.arange(m)
    while len(todo):
        Lt = rng.integers(lmin_eff, lmax_eff + 1, size=len(todo))
        st = rng.integers(0, n - Lt + 1)
        kp = rng.random((len(todo), lmax_eff)) < p
        kp &= np.arange(lmax_eff)[None, :] < Lt[:, None]
        L[todo], start[todo], keep[todo] = Lt, st, kp
        todo = todo[kp.sum(axis=1) == 0]
    sizes = keep.sum(axis=1).astype(np.int64)
    vtx = (start[:, None] + np.arange(lmax_eff)[None, :])[keep]
    return sizes, vtx


def _powerlaw_sizes(rng, m: int, expo=2.2, smin=2, smax=200):
    s = np.arange(smin, smax + 1)
    pr = s.astype(np.float64) ** (-expo)
    pr /= pr.sum()
    return rng.choice(s, size=m, p=pr)


def _capped_demand(rng, sizes, fmax: int):
    f = rng.integers(1, fmax + 1, size=len(sizes))
    return np.minimum(f, sizes).astype(np.int32)


def plain(seed: int = 0, idx: int = 0, n: int = 200, m: int = 1000) -> Instance:
    rng = _rng("plain", idx, seed)
    sizes, vtx = _uniform_members(rng, n, rng.integers(2, 9, size=m))
    return _csr(n, sizes, vtx, np.ones(m, np.int32), 50, f"plain(n={n},m={m},seed={seed})")


def transport(seed: int = 0, idx: int = 0, n: int = 8000, m: int = 60000) -> Instance:
    rng = _rng("transport", idx, seed)
    sizes, vtx = _interval_members(rng, n, m)
    return _csr(n, sizes, vtx, np.ones(m, np.int32), n, f"transport(n={n},m={m},seed={seed})")


def multidemand(seed: int = 0, idx: int = 0, n: int = 20000, m: int = 200000) -> Instance:
    rng = _rng("multidemand", idx, seed)
    sizes = np.minimum(_powerlaw_sizes(rng, m), n)
    sizes, vtx = _uniform_members(rng, n, sizes)
    dem = _capped_demand(rng, sizes, 3)
    return _csr(n, sizes, vtx, dem, n, f"multidemand(n={n},m={m},seed={seed})")


def _styled(rng, n, m, fmax, name, style=None):
    if style is None:
        style = "interval" if rng.random() < 0.5 else "uniform"
    if style == "interval":
        sizes, vtx = _interval_members(rng, n, m)
    else:
        sizes, vtx = _uniform_members(rng, n, np.minimum(rng.integers(2, 9, size=m), n))
    dem = _capped_demand(rng, sizes, fmax)
    return _csr(n, sizes, vtx, dem, n, name, {"style": style})


def batch_member(seed: int = 0, idx: int = 0, nmin: int = 100, nmax: int = 4000) -> Instance:
    rng = _rng("batch", idx, seed)
    n = int(rng.integers(nmin, nmax + 1))
    m = int(round(n * rng.uniform(5.0, 10.0)))
    return _styled(rng, n, m, 2, f"batch[{idx}](seed={seed})")


def batch(count: int = 512, seed: int = 0, nmin: int = 100, nmax: int = 4000):
    return [batch_member(seed, i, nmin, nmax) for i in range(count)]


def serve_request(seed: int = 0, idx: int = 0, scale_max: float = 1.0, u: float | None = None,
                  style: str | None = None) -> Instance:
    """One serving request; ``scale_max`` < 1 truncates the log-uniform range.
    ``u`` fixes the size parameter (1.0: the largest request, n=30000,
    m=300000) and ``style`` the hyperedge style instead of drawing them."""
    rng = _rng("serve", idx, seed)
    draw = rng.uniform(0.0, 1.0) * scale_max
    u = draw if u is None else float(u)
    n = int(round(100 * 300 ** u))
    m = int(round(500 * 600 ** u))
    name = f"serve[{idx}](seed={seed})" if u == draw and style is None else \
        f"serve[{idx}](seed={seed},u={u:g},style={style})"
    return _styled(rng, n, m, 3, name, style)


def nci60_shaped(seed: int = 0, idx: int = 0, alpha: int = 1, n: int = 7124, m: int = 152,
                 mean_degree: float = 5.0) -> Instance:
    """Stand-in with the shape of the paper's NCI60 instances (Section 5.2):
    n = 7124 vertices, m = 152 hyperedges, f(e) = min(alpha, |e|), many more
    vertices than hyperedges.  The paper prints no hyperedge sizes; the
    membership recipe is an assumption: every vertex v has degree
    d_v = 1 + Poisson(mean_degree - 1) (at most m) and picks its d_v
    hyperedges without replacement with probability proportional to a
    Zipf weight 1/rank of the hyperedge (ranks a random permutation), so a
    few hyperedges are large and vertex neighbourhoods nest often.  A
    hyperedge left empty receives one uniformly drawn vertex."""
    rng = _rng("nci60_shaped", idx, seed)
    w = 1.0 / (1.0 + rng.permutation(m))
    deg = np.minimum(1 + rng.poisson(mean_degree - 1.0, size=n), m)
    # weighted sampling without replacement: the d_v largest Gumbel-perturbed
    # log weights of each row
    key = np.log(w)[None, :] + rng.gumbel(size=(n, m))
    rank = np.argsort(-key, axis=1)
    member = np.zeros((n, m), dtype=bool)
    take = np.arange(m)[None, :] < deg[:, None]
    member[np.repeat(np.arange(n), m).reshape(n, m)[take], rank[take]] = True
    for e in np.nonzero(~member.any(axis=0))[0]:
        member[int(rng.integers(0, n)), e] = True
    cols = member.T                      # hyperedge-major
    sizes = cols.sum(axis=1).astype(np.int64)
    vtx = np.nonzero(cols)[1].astype(np.int32)   # row-major: ascending within each hyperedge
    dem = np.minimum(alpha, sizes).astype(np.int32)
    return _csr(n, sizes, vtx, dem, n, f"nci60_shaped(alpha={alpha},seed={seed},idx={idx})",
                {"alpha": alpha})


def girg_shaped(seed: int = 0, idx: int = 0, alpha: int = 1, n: int = 15015, m: int = 1903) -> Instance:
    """Stand-in with the shape of the paper's GIRG transport instances
    (Section 5.3 averages: about 15015 vertices, 1903 hyperedges, mean
    |e| about 8): interval hyperedges on a line of n vertices, length
    U{2..18} with members kept with p = 0.8 (empty draws redrawn), f(e) =
    min(alpha, |e|).  Vertices in no hyperedge stay (the reduction deletes
    them in its first round)."""
    rng = _rng("girg_shaped", idx, seed)
    sizes, vtx = _interval_members(rng, n, m, lmin=2, lmax=18, p=0.8)
    dem = np.minimum(alpha, sizes).astype(np.int32)
    return _csr(n, sizes, vtx, dem, n, f"girg_shaped(alpha={alpha},seed={seed},idx={idx})", {"alpha": alpha})


def tiny(seed: int = 0, idx: int = 0, nmax: int = 12, mmax: int = 14, fmax: int = 3) -> Instance:
    """Tiny random instance with planted structure for brute-force checks."""
    rng = _rng("tiny", idx, seed)
    n = int(rng.integers(1, nmax + 1))
    m = int(rng.integers(0, mmax + 1))
    edges = []
    for _ in range(m):
        r = rng.random()
        if edges and r < 0.15:
            edges.append(list(edges[int(rng.integers(len(edges)))]))  # twin hyperedge
        elif edges and r < 0.35:
            base = edges[int(rng.integers(len(edges)))]
            extra = [int(v) for v in rng.integers(0, n, size=int(rng.integers(1, 3)))]
            edges.append(sorted(set(base) | set(extra)))  # nested (superset)
        else:
            s = int(rng.integers(1, min(n, 5) + 1))
            edges.append(sorted(int(v) for v in rng.choice(n, size=s, replace=False)))
    if n >= 2 and rng.random() < 0.5:
        # twin vertices: make vertex b a copy of vertex a's memberships
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        new = []
        for e in edges:
            s = set(e)
            s.discard(b)
            if a in s:
                s.add(b)
            new.append(sorted(s) if s else [a])
        edges = new
    dem = [int(rng.integers(1, min(fmax, len(e)) + 1)) for e in edges]
    return from_edges(n, edges, dem, k=n, name=f"tiny[{idx}](seed={seed})")


def tiny_dense(seed: int = 0, idx: int = 0, n: int = 64, m: int = 96, fmax: int = 3) -> Instance:
    """Small instances with many overlaps (several GPU tiles, ragged tails)."""
    rng = _rng("tiny_dense", idx, seed)
    edges = []
    for _ in range(m):
        r = rng.random()
        if edges and r < 0.1:
            edges.append(list(edges[int(rng.integers(len(edges)))]))
        elif edges and r < 0.3:
            base = edges[int(rng.integers(len(edges)))]
            extra = [int(v) for v in rng.integers(0, n, size=int(rng.integers(1, 4)))]
            edges.append(sorted(set(base) | set(extra)))
        else:
            s = int(rng.integers(1, min(n, 9) + 1))
            edges.append(sorted(int(v) for v in rng.choice(n, size=s, replace=False)))
    dem = [int(rng.integers(1, min(fmax, len(e)) + 1)) for e in edges]
    return from_edges(n, edges, dem, k=n, name=f"tiny_dense[{idx}](seed={seed},n={n},m={m})")


def make(family: str, seed: int = 0, idx: int = 0, **kw) -> Instance:
    fn = {
        "plain": plain,
        "transport": transport,
        "multidemand": multidemand,
        "batch": batch_member,
        "serve": serve_request,
        "tiny": tiny,
        "tiny_dense": tiny_dense,
        "nci60_shaped": nci60_shaped,
        "girg_shaped": girg_shaped,
    }[family]
    return fn(seed=seed, idx=idx, **kw)


def relabel(inst: Instance, vperm: np.ndarray, eperm: np.ndarray) -> Instance:
    """Rename vertex v to vperm[v] and hyperedge e to eperm[e].

    A pure relabelling (used by metamorphic tests): the hypergraph is the same
    up to names."""
    edges = inst.edges()
    new_edges = [None] * inst.m
    new_dem = np.zeros(inst.m, np.int32)
    for e, vs in enumerate(edges):
        new_edges[int(eperm[e])] = sorted(int(vperm[v]) for v in vs)
        new_dem[int(eperm[e])] = inst.demand[e]
    return from_edges(inst.n, new_edges, new_dem, k=inst.k, name=inst.name + "+relabel")
