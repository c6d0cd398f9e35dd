"""Pins of the CPU oracle against what the paper and the mathematics fix.

* golden fixtures (tests/golden/): the Appendix A counterexample, the
  tightness example after Theorem 3.4, and hand-derived trajectories of
  Algorithms 1-3;
* brute force on tiny instances: the optimum of the ILP of Section 5.1 is
  unchanged by the reduction, every multiple hitting set of the kernel is one
  of the input (Lemmas 4.2(ii), 4.3(ii)), no rule applies at the fixpoint,
  each phase is exhaustive on its own (Lemmas 4.2(iii), 4.3(iii)), the kernel
  bound of Theorem 3.4 / Theorem 4.1(i), f' = f, every surviving hyperedge
  keeps at least f(e) surviving vertices;
* f = 1 reduces DP and MD to Weihe's rules W2 and W1 (Section 1);
* relabelling equivariance (only tie breaks depend on ids, and they choose
  among interchangeable twins);
* the pruned candidate mode equals the all-pairs mode.
"""
import numpy as np
import pytest

import mhsgen
import oracle
import brute
import golden_io


def fixture_rule(exp):
    return oracle.RULE_SE if exp.get("rule") == "se" else oracle.RULE_DP


@pytest.mark.parametrize("name", golden_io.all_fixtures())
@pytest.mark.parametrize("mode", [oracle.ALLPAIRS, oracle.PRUNED])
def test_golden_fixture(name, mode):
    inst, exp = golden_io.load(name)
    if exp.get("rule") == "fe":
        res = oracle.run_fe(inst, mode)
        assert res.forced.tolist() == exp["forced"]
        assert inst.k - res.n_forced == exp["k_out"]
    else:
        res = oracle.run(inst, mode, rule=fixture_rule(exp))
    assert res.rounds == exp["rounds"]
    assert res.death_e.tolist() == exp["death_e"]
    assert res.death_v.tolist() == exp["death_v"]
    assert brute.opt(inst.n, inst.edges(), inst.demand.tolist()) == exp["opt"]
    ek, dk = brute.reduced(inst, res.kept_v, res.kept_e)
    if exp.get("rule") == "fe":
        dk = [int(res.demand_out[e]) for e in res.kept_e]
        assert res.n_forced + brute.opt(inst.n, ek, dk, allowed=res.kept_v.tolist()) == exp["opt"]
    else:
        assert brute.opt(inst.n, ek, dk, allowed=res.kept_v.tolist()) == exp["opt"]


def test_appendix_a_faulty_rule_changes_optimum():
    """Appendix A: deleting v3 (0-based 2) because v2 dominates it raises the
    optimum from 3 to 4; MD keeps v3 since it has one dominator and needs 2."""
    inst, exp = golden_io.load("appendix_a_counterexample.txt")
    edges = inst.edges()
    dem = inst.demand.tolist()
    assert brute.opt(inst.n, edges, dem) == 3
    assert brute.opt(inst.n, edges, dem, allowed=[0, 1, 3, 4]) == 4
    # the printed solution {v1,v2,v3} hits every hyperedge twice
    assert brute.is_hitting_set(0b00111, brute.masks(edges), dem)
    res = oracle.run(inst)
    assert res.death_v[2] == 0


def _tiny_cases(count=300):
    return [mhsgen.tiny(seed=0, idx=i) for i in range(count)]


@pytest.mark.parametrize("chunk", range(6))
def test_bruteforce_tiny(chunk):
    for inst in _tiny_cases(300)[chunk::6]:
        res = oracle.run(inst, oracle.ALLPAIRS)
        edges = inst.edges()
        dem = inst.demand.tolist()
        kept_v = res.kept_v.tolist()
        kept_e = res.kept_e.tolist()
        ek, dk = brute.reduced(inst, kept_v, kept_e)
        # optimum preserved (Lemmas 4.2(i)(ii), 4.3(i)(ii))
        o = brute.opt(inst.n, edges, dem)
        assert brute.opt(inst.n, ek, dk, allowed=kept_v) == o, inst.name
        # every multiple hitting set of the kernel is one of the input
        em = brute.masks(edges)
        for S in brute.all_hitting_sets(inst.n, ek, dk, kept_v):
            assert brute.is_hitting_set(S, em, dem), inst.name
        # invariant: every surviving hyperedge keeps >= f(e) surviving vertices
        for e, f in zip(ek, dk):
            assert len(e) >= f
        # no rule applies at the fixpoint (full Dom count for MD)
        assert not brute.dp_applicable(ek, dk), inst.name
        assert not brute.md_applicable(kept_v, ek, dk), inst.name
        # f' = f: the kernel's demands are the input's demands
        assert dk == [dem[e] for e in kept_e]
        # derived round bound: every round after the first deletes a
        # hyperedge, and the round before it deleted a vertex
        ne = int((res.death_e > 0).sum())
        nv = int((res.death_v > 0).sum())
        assert res.rounds <= 1 + min(ne, nv) or res.rounds <= 1
        for r in range(2, res.rounds + 1):
            de, _ = res.round_deletions(r)
            _, dv_prev = res.round_deletions(r - 1)
            assert len(de) >= 1 and len(dv_prev) >= 1


@pytest.mark.parametrize("chunk", range(3))
def test_kernel_size_bound(chunk):
    """Theorem 3.4 / 4.1(i): |V'| + |E'| <= 2 * alpha * Dilworth(incidence graph)."""
    for inst in _tiny_cases(120)[chunk::3]:
        if inst.m == 0:
            continue
        res = oracle.run(inst)
        alpha = int(inst.demand.max())
        dn = brute.dilworth_incidence(inst.n, inst.edges())
        assert len(res.kept_v) + len(res.kept_e) <= 2 * alpha * dn, inst.name


def test_dilworth_of_tightness_example():
    # n disjoint copies of K2: Dilworth number n (Section 3.2)
    assert brute.dilworth_incidence(5, [[i] for i in range(5)]) == 5


@pytest.mark.parametrize("mode", [oracle.ALLPAIRS, oracle.PRUNED])
def test_phase_exhaustive(mode):
    """One Algorithm 1 pass leaves nothing for DP; one Algorithm 2 pass
    leaves nothing for MD (Lemmas 4.2(iii), 4.3(iii)), from any state."""
    for inst in _tiny_cases(150) + [mhsgen.tiny_dense(seed=0, idx=i) for i in range(4)]:
        res = oracle.run(inst, mode, max_rounds=1)
        av = res.death_v == 0
        ae = res.death_e == 0
        ke = oracle.dp_pass(inst, av, ae, mode)
        ae2 = ae & ~ke
        assert not oracle.dp_pass(inst, av, ae2, mode).any(), inst.name
        kv = oracle.md_pass(inst, av, ae2, mode)
        av2 = av & ~kv
        assert not oracle.md_pass(inst, av2, ae2, mode).any(), inst.name


def test_unit_demand_is_weihe():
    """f = 1: DP is W2 (delete a superset of another hyperedge, the lower
    index surviving among equal ones) and MD is W1 (delete a vertex that some
    other vertex dominates, the lower index surviving among twins)."""
    for i in range(200):
        inst = mhsgen.tiny(seed=1, idx=i, fmax=1)
        if inst.m == 0:
            continue
        av = np.ones(inst.n, bool)
        ae = np.ones(inst.m, bool)
        sets = [set(e) for e in inst.edges()]
        w2 = np.array([any(j != i2 and sets[i2] <= sets[j] and (sets[j] != sets[i2] or i2 < j)
                           for i2 in range(inst.m)) for j in range(inst.m)])
        assert (oracle.dp_pass(inst, av, ae, oracle.ALLPAIRS) == w2).all()
        ae2 = ae & ~w2
        inc = {v: {e for e in range(inst.m) if ae2[e] and v in sets[e]} for v in range(inst.n)}
        w1 = np.array([len(inc[j]) == 0 or any(i2 != j and inc[j] <= inc[i2] and (inc[i2] != inc[j] or i2 < j)
                                               for i2 in range(inst.n)) for j in range(inst.n)])
        assert (oracle.md_pass(inst, av, ae2, oracle.ALLPAIRS) == w1).all()


def _signature(inst, res):
    """Relabelling-invariant description of a trajectory and its kernel."""
    per_round = [tuple(len(x) for x in res.round_deletions(r)) for r in range(1, res.rounds + 1)]
    ek, dk = brute.reduced(inst, res.kept_v, res.kept_e)
    sizes = sorted((len(e), f) for e, f in zip(ek, dk))
    deg = {}
    for e in ek:
        for v in e:
            deg[v] = deg.get(v, 0) + 1
    degs = sorted(deg.get(int(v), 0) for v in res.kept_v)
    return res.rounds, per_round, sizes, degs


def test_relabel_equivariance():
    rng = np.random.default_rng(7)
    for i in range(120):
        inst = mhsgen.tiny(seed=2, idx=i)
        vperm = rng.permutation(inst.n)
        eperm = rng.permutation(inst.m)
        r1 = oracle.run(inst)
        inst2 = mhsgen.relabel(inst, vperm, eperm)
        r2 = oracle.run(inst2)
        assert _signature(inst, r1) == _signature(inst2, r2), inst.name


def test_fixpoint_idempotent():
    """Reducing the kernel again changes nothing (rounds = 0)."""
    for i in range(100):
        inst = mhsgen.tiny(seed=3, idx=i)
        res = oracle.run(inst)
        ek, dk = brute.reduced(inst, res.kept_v, res.kept_e)
        again = mhsgen.from_edges(inst.n, ek, dk)
        r2 = oracle.run(again)
        kept = set(res.kept_v.tolist())
        # vertices outside the kernel are isolated in `again` and go in round 1
        if len(kept) == inst.n:
            assert r2.rounds == 0
        assert (r2.death_e == 0).all()
        assert set(r2.kept_v.tolist()) == kept


@pytest.mark.parametrize("family,count", [("tiny", 200), ("tiny_dense", 12)])
def test_pruned_equals_allpairs(family, count):
    for i in range(count):
        inst = mhsgen.make(family, seed=4, idx=i)
        a = oracle.run(inst, oracle.ALLPAIRS)
        b = oracle.run(inst, oracle.PRUNED)
        assert a.rounds == b.rounds
        assert (a.death_e == b.death_e).all() and (a.death_v == b.death_v).all()


def test_pruned_equals_allpairs_plain_workload():
    inst = mhsgen.plain(seed=0)
    a = oracle.run(inst, oracle.ALLPAIRS)
    b = oracle.run(inst, oracle.PRUNED)
    assert (a.death_e == b.death_e).all() and (a.death_v == b.death_v).all()


def test_pruned_equals_allpairs_small_interval_and_multidemand():
    for inst in (mhsgen.transport(seed=1, n=300, m=2000), mhsgen.multidemand(seed=1, n=300, m=2500),
                 mhsgen.batch_member(seed=5, idx=3, nmax=300)):
        a = oracle.run(inst, oracle.ALLPAIRS)
        b = oracle.run(inst, oracle.PRUNED)
        assert a.rounds == b.rounds
        assert (a.death_e == b.death_e).all() and (a.death_v == b.death_v).all()


def test_validation_codes():
    ok = mhsgen.from_edges(3, [[0, 1], [1, 2]], [1, 2])
    assert oracle.validate(ok) == 0
    bad_range = mhsgen.from_edges(3, [[0, 3]], [1])
    assert oracle.validate(bad_range) == -2
    bad_dem = mhsgen.from_edges(3, [[0, 1]], [3])
    assert oracle.validate(bad_dem) == -5
    bad_zero = mhsgen.from_edges(3, [[0, 1]], [0])
    assert oracle.validate(bad_zero) == -5
    empty_edge = mhsgen.from_edges(3, [[]], [1])
    assert oracle.validate(empty_edge) == -4
    dup = mhsgen.Instance(n=3, m=1, edge_ptr=np.array([0, 2], np.int64),
                          edge_vtx=np.array([1, 1], np.int32), demand=np.array([1], np.int32))
    assert oracle.validate(dup) == -3
    with pytest.raises(ValueError):
        oracle.run(dup)


def test_degenerate_sizes():
    empty = mhsgen.from_edges(0, [], [])
    r = oracle.run(empty)
    assert r.rounds == 0
    no_edges = mhsgen.from_edges(4, [], [])
    r = oracle.run(no_edges)
    assert r.rounds == 1 and (r.death_v == 1).all()


# ------------------------------------------------ superedge rule SE (Section 3.1)

def se_applicable(edges_kept, dem_kept) -> bool:
    sets = [set(e) for e in edges_kept]
    return any(i != j and sets[i] <= sets[j] and dem_kept[i] >= dem_kept[j]
               for i in range(len(sets)) for j in range(len(sets)))


@pytest.mark.parametrize("chunk", range(3))
def test_superedge_bruteforce(chunk):
    """SE in place of DP: the optimum is preserved, neither SE nor MD applies
    at the fixpoint, and the kernel bound of Theorem 3.4 (proved for SE then
    MD) holds."""
    for inst in _tiny_cases(180)[chunk::3]:
        res = oracle.run(inst, oracle.ALLPAIRS, rule=oracle.RULE_SE)
        edges, dem = inst.edges(), inst.demand.tolist()
        kept_v, kept_e = res.kept_v.tolist(), res.kept_e.tolist()
        ek, dk = brute.reduced(inst, kept_v, kept_e)
        assert brute.opt(inst.n, ek, dk, allowed=kept_v) == brute.opt(inst.n, edges, dem), inst.name
        assert not se_applicable(ek, dk), inst.name
        assert not brute.md_applicable(kept_v, ek, dk), inst.name
        if inst.m:
            dn = brute.dilworth_incidence(inst.n, edges)
            assert len(kept_v) + len(kept_e) <= 2 * int(inst.demand.max()) * dn


def test_superedge_equals_dp_for_unit_demands():
    """With f = 1 both rules are Weihe's W2: identical trajectories."""
    for i in range(150):
        inst = mhsgen.tiny(seed=21, idx=i, fmax=1)
        a = oracle.run(inst, rule=oracle.RULE_SE)
        b = oracle.run(inst, rule=oracle.RULE_DP)
        assert a.rounds == b.rounds
        assert (a.death_e == b.death_e).all() and (a.death_v == b.death_v).all()


def test_superedge_pruned_equals_allpairs():
    for i in range(150):
        inst = mhsgen.tiny(seed=22, idx=i)
        a = oracle.run(inst, oracle.ALLPAIRS, rule=oracle.RULE_SE)
        b = oracle.run(inst, oracle.PRUNED, rule=oracle.RULE_SE)
        assert (a.death_e == b.death_e).all() and (a.death_v == b.death_v).all()


def test_superedge_pass_exhaustive():
    for i in range(150):
        inst = mhsgen.tiny(seed=23, idx=i)
        av = np.ones(inst.n, bool)
        ae = np.ones(inst.m, bool)
        ke = oracle.dp_pass(inst, av, ae, oracle.ALLPAIRS, rule=oracle.RULE_SE)
        assert not oracle.dp_pass(inst, av, ae & ~ke, oracle.ALLPAIRS, rule=oracle.RULE_SE).any()


# ------------------------------------------- full-edge rule FE (KernelGPU-FE)

@pytest.mark.parametrize("chunk", range(3))
def test_full_edge_bruteforce(chunk):
    """FE alternated with DP + MD: every solution contains the forced set F,
    OPT(H) = |F| + OPT(H') with the reduced demands, every solution of H'
    plus F solves H, and at the fixpoint no hyperedge is full and neither DP
    nor MD applies."""
    for inst in _tiny_cases(180)[chunk::3]:
        res = oracle.run_fe(inst, oracle.ALLPAIRS)
        edges, dem = inst.edges(), inst.demand.tolist()
        kept_v, kept_e = res.kept_v.tolist(), res.kept_e.tolist()
        ek, _ = brute.reduced(inst, kept_v, kept_e)
        dk = [int(res.demand_out[e]) for e in kept_e]
        assert all(f >= 1 for f in dk)
        F = 0
        for v in res.forced.tolist():
            F |= 1 << v
        assert res.n_forced + brute.opt(inst.n, ek, dk, allowed=kept_v) == brute.opt(inst.n, edges, dem), inst.name
        em = brute.masks(edges)
        for S in brute.all_hitting_sets(inst.n, ek, dk, kept_v):
            assert brute.is_hitting_set(S | F, em, dem), inst.name
        assert not any(len(e) == f for e, f in zip(ek, dk)), inst.name
        assert not brute.dp_applicable(ek, dk), inst.name
        assert not brute.md_applicable(kept_v, ek, dk), inst.name
        # forced vertices are deleted in the round that forced them
        assert all(res.death_v[v] > 0 for v in res.forced.tolist())


def test_full_edge_pruned_equals_allpairs():
    for i in range(150):
        inst = mhsgen.tiny(seed=25, idx=i)
        a = oracle.run_fe(inst, oracle.ALLPAIRS)
        b = oracle.run_fe(inst, oracle.PRUNED)
        assert a.rounds == b.rounds and (a.death_e == b.death_e).all() and (a.death_v == b.death_v).all()
        assert (a.forced_v == b.forced_v).all() and (a.demand_out == b.demand_out).all()


def test_full_edge_without_full_edges_equals_plain_run():
    """If no hyperedge is ever full, FE never fires: same trajectory as DP + MD."""
    for i in range(100):
        inst = mhsgen.tiny(seed=26, idx=i)
        a = oracle.run_fe(inst)
        b = oracle.run(inst)
        if a.n_forced == 0 and a.rounds == b.rounds:
            assert (a.death_e == b.death_e).all() and (a.death_v == b.death_v).all()
        # the plain fixpoint is a prefix of the FE trajectory
        assert (b.death_e[b.death_e > 0] == a.death_e[b.death_e > 0]).all()
        assert (b.death_v[b.death_v > 0] == a.death_v[b.death_v > 0]).all()
