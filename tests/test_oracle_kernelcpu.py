"""Second CPU implementation: KernelCPU (Algorithms 4-6, Section 4.2).

KernelCPU reaches the DP + MD fixpoint by a different route from the
round-synchronous oracle: it keeps the intersection-count matrices I^E and
I^V up to date under deletions and narrows each pass to candidate lists
(superseders P^E, victims P^V), where the oracle re-tests sorted sets from
scratch every round.  The correctness proofs of Algorithms 4 and 5 show that
each iteration of Algorithm 6 deletes what one round of Algorithm 3 deletes,
so the two implementations must agree on every deletion round, and a slip in
either (a dropped term in the supersedence test, a wrong tie break, a missed
candidate) shows up as a disagreement here.

KernelCPU is pinned on its own by the hand-derived fixtures, before it is
used as a cross-check.
"""
import numpy as np
import pytest

import golden_io
import mhsgen
import oracle


def same(a, b):
    return (a.rounds == b.rounds and np.array_equal(a.death_e, b.death_e)
            and np.array_equal(a.death_v, b.death_v))


@pytest.mark.parametrize("name", [f for f in golden_io.all_fixtures()])
def test_fixture(name):
    inst, exp = golden_io.load(name)
    if exp.get("rule") in ("se", "fe"):
        pytest.skip("KernelCPU applies DP + MD only")
    res = oracle.kernelcpu(inst)
    assert res.rounds == exp["rounds"]
    assert res.death_e.tolist() == exp["death_e"]
    assert res.death_v.tolist() == exp["death_v"]


def test_tiny_random_match_round_by_round():
    bad = []
    for seed in range(400):
        inst = mhsgen.tiny(seed=seed)
        if not same(oracle.kernelcpu(inst), oracle.run(inst, oracle.ALLPAIRS)):
            bad.append(seed)
    assert not bad, f"KernelCPU and Algorithm 3 differ on tiny seeds {bad[:10]}"


@pytest.mark.parametrize("seed", range(8))
def test_tiny_dense_match(seed):
    inst = mhsgen.tiny_dense(seed=seed)
    assert same(oracle.kernelcpu(inst), oracle.run(inst))


@pytest.mark.parametrize("family,kw", [
    ("plain", {}),
    ("transport", {"n": 600, "m": 4500}),
    ("multidemand", {"n": 800, "m": 6000}),
])
@pytest.mark.parametrize("seed", [0, 1])
def test_medium_families_match(family, kw, seed):
    inst = mhsgen.make(family, seed=seed, **kw)
    a = oracle.kernelcpu(inst)
    b = oracle.run(inst)
    assert same(a, b)


@pytest.mark.parametrize("idx", range(3))
def test_batch_members_match(idx):
    inst = mhsgen.batch_member(seed=0, idx=idx, nmax=600)
    assert same(oracle.kernelcpu(inst), oracle.run(inst))


def test_twins_and_isolated_vertices():
    # duplicated hyperedges (twins: the lower id survives), identical vertex
    # columns (twin vertices) and isolated vertices (deleted in round 1)
    edges = [[0, 1, 2], [0, 1, 2], [2, 3], [3, 4, 5], [3, 4, 5], [6]]
    inst = mhsgen.from_edges(9, edges, [2, 2, 1, 1, 2, 1])
    a = oracle.kernelcpu(inst)
    assert same(a, oracle.run(inst, oracle.ALLPAIRS))
    assert a.death_v[7] == 1 and a.death_v[8] == 1


def test_degenerate():
    empty = mhsgen.from_edges(0, [], [])
    r = oracle.kernelcpu(empty)
    assert r.rounds == 0
    no_edges = mhsgen.from_edges(5, [], [])
    r = oracle.kernelcpu(no_edges)
    assert r.rounds == 1 and r.death_v.tolist() == [1] * 5
    singletons = mhsgen.from_edges(4, [[0], [1], [2], [3]], [1, 1, 1, 1])
    r = oracle.kernelcpu(singletons)
    assert r.rounds == 0 and not r.death_e.any() and not r.death_v.any()


def test_rejects_invalid():
    bad = mhsgen.from_edges(3, [[0, 1]], [3])
    with pytest.raises(ValueError):
        oracle.kernelcpu(bad)
