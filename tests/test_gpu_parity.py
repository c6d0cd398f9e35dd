"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
bit-exact, round by round (every deletion round of every hyperedge and
vertex), on fixtures, tiny and tile-spanning instances, the measured
workloads at full size, and the degenerate cases."""
import numpy as np
import pytest

import mhsgen
import oracle
import golden_io
from gpu_common import say, assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2109_06042_amd as mh
    mh._lib.load()
    return mh


@pytest.mark.parametrize("name", golden_io.all_fixtures())
def test_golden(mh, name):
    say("golden", name)
    inst, exp = golden_io.load(name)
    rule = {"se": mh.MHS_RULE_SE, "fe": mh.MHS_RULE_FE}.get(exp.get("rule"), 0)
    r = mh.reduce(inst, flags=rule)
    if exp.get("rule") == "fe":
        assert r.forced.tolist() == exp["forced"]
        assert r.k_out == exp["k_out"]
    assert r.rounds == exp["rounds"]
    assert r.death_e.tolist() == exp["death_e"]
    assert r.death_v.tolist() == exp["death_v"]


def test_tiny_single(mh):
    for i in range(60):
        inst = mhsgen.tiny(seed=11, idx=i)
        say("tiny single", inst.name)
        assert_same(mh.reduce(inst), oracle.run(inst), inst.name)


def test_tiny_batched(mh):
    insts = [mhsgen.tiny(seed=12, idx=i) for i in range(400)]
    say("tiny batch of", len(insts))
    res = mh.reduce_batch(insts)
    for inst, r in zip(insts, res):
        assert_same(r, oracle.run(inst), inst.name)


@pytest.mark.parametrize("variant", ["INT8", "BITSET", "SPARSE", "AUTO", "HYBRID"])
@pytest.mark.parametrize("n,m", [(64, 96), (130, 300), (257, 700), (300, 1500), (520, 2100)])
def test_tile_spanning(mh, n, m, variant):
    """Several 128-row tiles and 64-wide K chunks with ragged tails, every
    contraction variant."""
    flags = getattr(mh, "MHS_VARIANT_" + variant)
    for i in range(3):
        inst = mhsgen.tiny_dense(seed=13, idx=i, n=n, m=m)
        say("tile-spanning", variant, inst.name)
        assert_same(mh.reduce(inst, flags=flags), oracle.run(inst), inst.name)


def test_plain_workload(mh):
    inst = mhsgen.plain(seed=0)
    say("plain", inst.name)
    assert_same(mh.reduce(inst), oracle.run(inst), inst.name)


def test_plain_workload_seeds(mh):
    insts = [mhsgen.plain(seed=s) for s in range(1, 9)]
    say("plain seeds batch")
    for inst, r in zip(insts, mh.reduce_batch(insts)):
        assert_same(r, oracle.run(inst), inst.name)


def test_transport_workload_full(mh):
    inst = mhsgen.transport(seed=0)
    say("transport full", inst.name)
    orc = oracle.run(inst)
    r = mh.reduce(mh.DeviceInstance(inst))
    assert_same(r, orc, inst.name)
    assert r.rounds == orc.rounds and r.rounds >= 5


def test_transport_small_seeds(mh):
    for s in range(3):
        inst = mhsgen.transport(seed=100 + s, n=1500, m=11000)
        say("transport small", inst.name)
        assert_same(mh.reduce(inst), oracle.run(inst), inst.name)


def test_multidemand_reduced(mh):
    for s in range(2):
        inst = mhsgen.multidemand(seed=200 + s, n=2000, m=20000)
        say("multidemand reduced", inst.name)
        assert_same(mh.reduce(inst), oracle.run(inst), inst.name)


def test_batch_members_mixed(mh):
    insts = [mhsgen.batch_member(seed=3, idx=i, nmax=600) for i in range(24)]
    say("batch members", len(insts))
    res = mh.reduce_batch(insts)
    for inst, r in zip(insts, res):
        assert_same(r, oracle.run(inst), inst.name)
        single = mh.reduce(inst)
        assert_same(single, oracle.run(inst), inst.name + " single")


def test_batch_upload_id_widths(mh):
    """Batched host inputs cross the bus as 16-bit vertex ids when n <= 65536
    and as 32-bit ids otherwise, and are widened on the device; members at
    both sides of the limit (ids up to 65535 and beyond), an empty instance
    between them."""
    rng = np.random.default_rng(23)
    top = [sorted({65535} | set(int(v) for v in rng.choice(65535, size=int(rng.integers(1, 5)), replace=False)))
           for _ in range(400)]
    insts = [mhsgen.transport(seed=23, n=65536, m=3000),
             mhsgen.from_edges(65536, top, name="ids-to-65535"),
             mhsgen.from_edges(5, [], name="empty"),
             mhsgen.transport(seed=24, n=70000, m=3000),
             mhsgen.from_edges(65537, top + [[65536]], name="ids-past-65535"),
             mhsgen.tiny(seed=23, idx=0)]
    say("batch upload id widths")
    for inst, r in zip(insts, mh.reduce_batch(insts)):
        assert_same(r, oracle.run(inst), inst.name)


@pytest.mark.parametrize("case", ["range", "order", "empty", "demand", "ptr"])
def test_batch_rejects_bad_member_like_single(mh, case):
    """A bad member of a batch is reported with its index and the message
    the single call gives for it; the next batch runs normally."""
    good = [mhsgen.tiny(seed=31, idx=i) for i in range(6)]
    ptr = np.array([0, 2, 4], np.int64)
    vtx = {"range": [0, 1, 2, 9], "order": [0, 1, 3, 2], "empty": [0, 1, 2, 3],
           "demand": [0, 1, 2, 3], "ptr": [0, 1, 2, 3]}[case]
    dem = [1, 3] if case == "demand" else [1, 1]
    if case == "empty":
        ptr = np.array([0, 2, 2, 4], np.int64)
        dem = [1, 1, 1]
    if case == "ptr":
        ptr = np.array([0, 3, 2], np.int64)
    bad = mhsgen.Instance(n=5, m=len(ptr) - 1, edge_ptr=ptr, edge_vtx=np.array(vtx, np.int32),
                          demand=np.array(dem, np.int32))
    with pytest.raises(mh.MhsError) as single:
        mh.reduce(bad)
    insts = good[:3] + [bad] + good[3:]
    say("batch with a bad member", case)
    with pytest.raises(mh.MhsError) as batched:
        mh.reduce_batch(insts)
    why = str(single.value).split(": ", 1)[-1]
    assert "instance 3: " in str(batched.value) and why in str(batched.value), (str(single.value), str(batched.value))
    for inst, r in zip(good, mh.reduce_batch(good)):
        assert_same(r, oracle.run(inst), inst.name)


def test_device_input_equals_host_input(mh):
    inst = mhsgen.tiny_dense(seed=14, idx=0, n=200, m=900)
    say("device vs host input")
    a = mh.reduce(inst)
    b = mh.reduce(mh.DeviceInstance(inst))
    assert_same(a, oracle.run(inst))
    assert_same(b, oracle.run(inst))


def test_graph_and_direct_launches_agree(mh):
    """Rounds replayed from a hipGraph and launched directly (the defaults of
    a set and of one instance, both forced either way), single and batched;
    asking for both is rejected."""
    inst = mhsgen.transport(seed=5, n=2000, m=15000)
    say("graph vs direct", inst.name)
    orc = oracle.run(inst)
    for flags in (0, mh.MHS_NO_GRAPH, mh.MHS_GRAPH, mh.MHS_PROFILE):
        for _ in range(3):     # replays of the cached graph
            assert_same(mh.reduce(inst, flags=flags), orc, f"{inst.name} flags={flags}")
    insts = [inst, mhsgen.tiny_dense(seed=5, n=300, m=900)]
    refs = [orc, oracle.run(insts[1])]
    for flags in (0, mh.MHS_NO_GRAPH, mh.MHS_GRAPH):
        say("graph vs direct batched", flags)
        for _ in range(2):
            for r, ref, i in zip(mh.reduce_batch(insts, flags=flags), refs, insts):
                assert_same(r, ref, f"{i.name} batched flags={flags}")
    with pytest.raises(mh.MhsError):
        mh.reduce(inst, flags=mh.MHS_GRAPH | mh.MHS_NO_GRAPH)


@pytest.mark.parametrize("k", ["1", "3"])
def test_mixed_set_concurrent_branches(mh, monkeypatch, k):
    """A set with sparse and dense members (HYBRID: interval instances take
    int8 tiles, uniform ones sparse counts) runs each phase's two branches on
    two streams: replayed from round graphs of k rounds, launched directly,
    and in order under MHS_PROFILE, every replay equal to the oracle."""
    monkeypatch.setenv("MHSK_ROUNDS_PER_LAUNCH", k)
    insts = [mhsgen.transport(seed=9, n=2000, m=15000), mhsgen.tiny_dense(seed=9, n=300, m=900)] + \
            [mhsgen.batch_member(seed=9, idx=i, nmax=900) for i in range(6)]
    refs = [oracle.run(i) for i in insts]
    hyb = mh.MHS_VARIANT_HYBRID
    for flags in (hyb, hyb | mh.MHS_GRAPH, hyb | mh.MHS_NO_GRAPH, hyb | mh.MHS_PROFILE):
        say("mixed set", k, flags)
        for _ in range(3):
            res = mh.reduce_batch(insts, flags=flags)
            for r, ref, i in zip(res, refs, insts):
                assert_same(r, ref, f"{i.name} mixed flags={flags} k={k}")
    # the set holds both kinds (otherwise nothing here ran concurrently):
    # sparse members count terms, dense ones issue MFMA work (counted when
    # profiling)
    kinds = {(r.stats["terms"] > 0, r.stats["issued_ops"] > 0)
             for r in mh.reduce_batch(insts, flags=hyb | mh.MHS_PROFILE)}
    assert (True, False) in kinds and (False, True) in kinds, kinds


@pytest.mark.parametrize("k", ["1", "2", "3", "4"])
def test_rounds_per_graph_launch(mh, monkeypatch, k):
    """Graphs of k rounds: rounds queued past the fixpoint (up to 2k - 1 of
    them) do nothing and still publish their end; single and batched,
    instances that stop after 1..several rounds."""
    monkeypatch.setenv("MHSK_ROUNDS_PER_LAUNCH", k)
    insts = [mhsgen.transport(seed=5, n=2000, m=15000), mhsgen.tiny_dense(seed=41, n=300, m=900),
             mhsgen.plain(seed=41)]
    refs = [oracle.run(i) for i in insts]
    for inst, ref in zip(insts, refs):
        say("rounds per launch", k, inst.name)
        for _ in range(2):
            assert_same(mh.reduce(inst, flags=mh.MHS_GRAPH), ref, f"{inst.name} k={k}")
    say("rounds per launch batched", k)
    for r, ref, i in zip(mh.reduce_batch(insts, flags=mh.MHS_GRAPH), refs, insts):
        assert_same(r, ref, f"{i.name} batched k={k}")


def test_repeat_is_deterministic(mh):
    inst = mhsgen.multidemand(seed=7, n=1000, m=8000)
    say("determinism", inst.name)
    a = mh.reduce(inst)
    for _ in range(3):
        b = mh.reduce(inst)
        assert (a.death_e == b.death_e).all() and (a.death_v == b.death_v).all()


def test_degenerate(mh):
    cases = [
        mhsgen.from_edges(0, [], []),
        mhsgen.from_edges(5, [], []),
        mhsgen.from_edges(1, [[0]], [1]),
        mhsgen.from_edges(3, [[0, 1, 2]] * 7, [2] * 7),          # identical hyperedges
        mhsgen.from_edges(300, [[299]], [1]),                    # isolated vertices
        mhsgen.from_edges(129, [[i] for i in range(129)], [1] * 129),   # tightness example, ragged tile
        mhsgen.from_edges(200, [list(range(200))] * 3 + [list(range(0, 200, 2))], [150, 200, 100, 50]),
    ]
    for inst in cases:
        say("degenerate", inst.n, inst.m)
        assert_same(mh.reduce(inst), oracle.run(inst), f"n={inst.n} m={inst.m}")
    res = mh.reduce_batch(cases)
    for inst, r in zip(cases, res):
        assert_same(r, oracle.run(inst), f"batched n={inst.n} m={inst.m}")


def test_invalid_device_input_rejected(mh):
    bad = mhsgen.Instance(n=3, m=1, edge_ptr=np.array([0, 2], np.int64),
                          edge_vtx=np.array([0, 7], np.int32), demand=np.array([1], np.int32))
    say("invalid device input")
    with pytest.raises(mh.MhsError) as ei:
        mh.reduce(mh.DeviceInstance(bad))
    assert ei.value.code == -1


def test_workspace_too_small(mh):
    import torch
    inst = mhsgen.plain(seed=0)
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    say("small workspace")
    from paper_2109_06042_amd import _lib
    import ctypes
    st, keep = mh._host_struct(inst)
    h = ctypes.c_void_p()
    rc = _lib.load().mhs_run(ctypes.byref(st), 0, ctypes.c_void_p(ws.data_ptr()), 4096, None, ctypes.byref(h))
    assert rc == _lib.MHS_ENOSPC


@pytest.mark.parametrize("family,kw", [
    ("tiny_dense", dict(n=300, m=1500)),
    ("multidemand", dict(n=1500, m=15000)),
    ("transport", dict(n=2000, m=15000)),
])
def test_bitset_variant(mh, family, kw):
    """The bit-packed AND + popcount contraction gives the same trajectory."""
    for i in range(2):
        inst = mhsgen.make(family, seed=300 + i, **kw)
        say("bitset", inst.name)
        orc = oracle.run(inst)
        assert_same(mh.reduce(inst, flags=mh.MHS_VARIANT_BITSET), orc, inst.name + " bitset")


def test_bitset_variant_batched(mh):
    insts = [mhsgen.tiny(seed=15, idx=i) for i in range(200)] + \
            [mhsgen.batch_member(seed=4, idx=i, nmax=500) for i in range(8)]
    say("bitset batch")
    for inst, r in zip(insts, mh.reduce_batch(insts, flags=mh.MHS_VARIANT_BITSET)):
        assert_same(r, oracle.run(inst), inst.name)


def test_autotuner(mh):
    """Every tuned candidate (variant x grid) returns identical results; AUTO
    then uses the recorded class and stays bit-exact."""
    sample = [mhsgen.batch_member(seed=6, idx=i, nmax=400) for i in range(6)]
    say("autotune")
    mh.tune_reset()
    rep = mh.tune(sample)
    assert rep["candidates"] == 36
    assert rep["best_flags"] & 0xff in (mh.MHS_VARIANT_INT8, mh.MHS_VARIANT_BITSET, mh.MHS_VARIANT_HYBRID,
                                        mh.MHS_VARIANT_SPARSE)
    assert rep["best_ms"] > 0 and rep["default_ms"] > 0
    res = mh.reduce_batch(sample)          # AUTO -> tuned class
    for inst, r in zip(sample, res):
        assert_same(r, oracle.run(inst), inst.name)
    for k in range(5):
        r = mh.reduce(sample[0], flags=mh.MHS_VARIANT_INT8 | mh._lib.MHS_GRID_LOG2(k))
        assert_same(r, oracle.run(sample[0]), f"grid 2^{k}")
    for g in range(3):
        r = mh.reduce(sample[1], flags=mh.MHS_VARIANT_INT8 | mh._lib.MHS_GEMM_SCHED(g))
        assert_same(r, oracle.run(sample[1]), f"operand staging {g}")
    mh.tune_reset()


def test_autotuner_device_sample(mh):
    """The autotuner on device-resident instances (MHS_INPUT_DEVICE: the
    host-to-device copies stay out of its timings) records the class of the
    device batch, which AUTO on the same DeviceInstances then uses; results
    stay bit-exact."""
    insts = [mhsgen.batch_member(seed=16, idx=i, nmax=500) for i in range(8)]
    dev = [mh.DeviceInstance(i) for i in insts]
    say("autotune device sample")
    mh.tune_reset()
    rep = mh.tune(dev)
    assert rep["candidates"] == 36 and rep["best_ms"] > 0
    for inst, r in zip(insts, mh.reduce_batch(dev, flags=mh.MHS_VARIANT_AUTO)):
        assert_same(r, oracle.run(inst), inst.name + " AUTO")
    mh.tune_reset()


@pytest.mark.parametrize("family,kw", [
    ("tiny_dense", dict(n=300, m=1500)),
    ("multidemand", dict(n=1500, m=15000)),
    ("transport", dict(n=2000, m=15000)),
])
def test_sparse_variant(mh, family, kw):
    """Hash-counted nonzero product terms give the same trajectory."""
    for i in range(2):
        inst = mhsgen.make(family, seed=400 + i, **kw)
        say("sparse", inst.name)
        assert_same(mh.reduce(inst, flags=mh.MHS_VARIANT_SPARSE), oracle.run(inst), inst.name + " sparse")


def test_sparse_variant_long_outer_lists(mh):
    """Victims whose outer list spans more than one wave while their terms
    still fit a wave's table: vertices of degree ~75 in hyperedges of two or
    three vertices (and hyperedges whose outer lists fit one wave)."""
    rng = np.random.default_rng(21)
    edges = [sorted(int(v) for v in rng.choice(100, size=int(rng.integers(2, 4)), replace=False))
             for _ in range(3000)]
    mixed = mhsgen.from_edges(100, edges, [1 + (i % 2) for i in range(3000)], name="long-outer")
    # distinct pairs: no hyperedge dominates another, so the vertex phase
    # still sees degrees ~70
    pairs = [(a, b) for a in range(100) for b in range(a + 1, 100)]
    pick = rng.choice(len(pairs), size=3500, replace=False)
    distinct = mhsgen.from_edges(100, [list(pairs[i]) for i in pick], name="distinct-pairs")
    for inst in (mixed, distinct):
        say("sparse long outer lists", inst.name)
        assert_same(mh.reduce(inst, flags=mh.MHS_VARIANT_SPARSE), oracle.run(inst), inst.name)
        assert_same(mh.reduce(inst, flags=mh.MHS_VARIANT_SPARSE | mh.MHS_RULE_SE),
                    oracle.run(inst, rule=oracle.RULE_SE), inst.name + " SE")


def test_sparse_variant_batched_and_overflow(mh):
    insts = [mhsgen.tiny(seed=16, idx=i) for i in range(200)] + \
            [mhsgen.batch_member(seed=5, idx=i, nmax=500) for i in range(8)]
    # a hub vertex in every hyperedge: its partner lists exceed the hash table
    # (overflow path), and many hyperedges share it
    rng = np.random.default_rng(3)
    edges = [sorted({0} | set(int(v) for v in rng.choice(np.arange(1, 3000), size=int(rng.integers(1, 6)), replace=False)))
             for _ in range(9000)]
    hub = mhsgen.from_edges(3000, edges, [1 + (i % 2) for i in range(9000)], name="hub")
    insts.append(hub)
    say("sparse batch + hub")
    for inst, r in zip(insts, mh.reduce_batch(insts, flags=mh.MHS_VARIANT_SPARSE)):
        assert_same(r, oracle.run(inst), inst.name)
    assert_same(mh.reduce(hub, flags=mh.MHS_VARIANT_SPARSE), oracle.run(hub), "hub single")


def test_sparse_variant_range_fallback(mh, monkeypatch):
    """The sparse variant's overflow path (dense ranges of partner ids),
    forced on every victim, gives the same trajectory."""
    monkeypatch.setenv("MHSK_SPARSE_FORCE_RANGE", "1")
    insts = [mhsgen.tiny_dense(seed=17, idx=0, n=300, m=1500), mhsgen.transport(seed=17, n=9000, m=12000),
             mhsgen.multidemand(seed=17, n=5000, m=9000)]
    for inst in insts:
        say("sparse range fallback", inst.name)
        assert_same(mh.reduce(inst, flags=mh.MHS_VARIANT_SPARSE), oracle.run(inst), inst.name)


def _slack_class(s):
    """The sparse variant's slack classes (monotone): 0..7 exact, then
    [8, 10), [10, 12), [12, 15), [15, 19), [19, 24), [24, 32), [32, 64),
    [64, inf)."""
    s = np.asarray(s, np.int64)
    c = np.minimum(s, 8)
    for t in (10, 12, 15, 19, 24, 32, 64):
        c = c + (s >= t)
    return c


def _sparse_terms(inst, ref, rounds):
    """Nonzero product terms the sparse variant visits over `rounds` executed
    rounds, from the oracle's death rounds: in round r every hyperedge alive
    at the round's start counts, over its alive vertices, their degrees in
    the hyperedges alive at the round's start (itself included) -- in round
    1 only the hyperedges whose slack |e| - f(e) falls in a class no higher
    than its own, on lists of at most 512 entries (a hyperedge of higher
    slack dominates under neither DP nor SE); every vertex alive at the
    round's start that keeps a hyperedge after the round's edge deletions
    counts the full sizes of the hyperedges it keeps."""
    ep = np.asarray(inst.edge_ptr, np.int64)
    ev = np.asarray(inst.edge_vtx, np.int64)
    de, dv = np.asarray(ref.death_e), np.asarray(ref.death_v)
    sizes = np.diff(ep)
    eid = np.repeat(np.arange(inst.m), sizes)
    cls = _slack_class(np.minimum(sizes - np.asarray(inst.demand, np.int64), 254))
    total = 0
    for r in range(1, rounds + 1):
        ae = (de == 0) | (de >= r)
        av = (dv == 0) | (dv >= r)
        deg = np.bincount(ev[ae[eid]], minlength=inst.n)
        if r == 1:
            # per vertex, how many of its hyperedges fall in each class or below
            per = np.zeros((inst.n, 16), np.int64)
            np.add.at(per, (ev, cls[eid]), 1)
            upto = np.cumsum(per, axis=1)[ev, cls[eid]]
            total += int(np.where(deg[ev] <= 512, upto, deg[ev]).sum())
        else:
            total += int(deg[ev[ae[eid] & av[ev]]].sum())
        kept = ((de == 0) | (de > r))[eid]
        d2 = np.bincount(ev[kept], minlength=inst.n)
        w = np.bincount(ev[kept], weights=sizes[eid[kept]], minlength=inst.n)
        total += int(w[av & (d2 > 0)].sum())
    return total


def test_sparse_terms_count(mh):
    """The sparse variant's term counter (the work figure of its roofline)
    equals the count derived from the oracle's trajectory when every victim
    is counted in full (SE rule), for victims on every path: 16- and 32-lane
    groups, one per wave, the whole workgroup (a hub vertex, whose list is
    too long for the round-1 slack order), and lists of both sorting widths.
    Under DP the groups stop a victim that a partner of slack 0 deletes at
    the term step that meets one, so the count there is at most the full
    one."""
    rng = np.random.default_rng(3)
    edges = [sorted({0} | set(int(v) for v in rng.choice(np.arange(1, 3000), size=int(rng.integers(1, 6)),
                                                         replace=False))) for _ in range(9000)]
    hub = mhsgen.from_edges(3000, edges, [1 + (i % 2) for i in range(9000)], name="hub")
    insts = [mhsgen.batch_member(seed=7, idx=i, nmax=700) for i in range(6)] + \
            [mhsgen.multidemand(seed=7, n=1500, m=15000), mhsgen.transport(seed=7, n=600, m=6000), hub]
    for rule, flag in ((oracle.RULE_SE, mh.MHS_RULE_SE), (oracle.RULE_DP, 0)):
        refs = [oracle.run(i, rule=rule) for i in insts]
        singles = [mh.reduce(i, flags=mh.MHS_VARIANT_SPARSE | flag) for i in insts]
        batched = mh.reduce_batch(insts, flags=mh.MHS_VARIANT_SPARSE | flag)
        for inst, ref, a, b in zip(insts, refs, singles, batched):
            say("sparse terms", inst.name, "SE" if flag else "DP")
            assert_same(a, ref, inst.name)
            assert_same(b, ref, inst.name + " batched")
            executed = int(a.stats["iterations"])
            assert executed == ref.rounds + 1, (inst.name, executed, ref.rounds)
            want = _sparse_terms(inst, ref, executed)
            if flag:
                assert a.stats["terms"] == want, (inst.name, a.stats["terms"], want)
                assert b.stats["terms"] == want, (inst.name, b.stats["terms"], want)
            else:
                assert 0 < a.stats["terms"] <= want, (inst.name, a.stats["terms"], want)
                assert 0 < b.stats["terms"] <= want, (inst.name, b.stats["terms"], want)


@pytest.mark.parametrize("kernel", ["lds", "direct", "async"])
def test_int8_kernels(mh, monkeypatch, kernel):
    """The int8 contraction kernels (LDS staged through registers, direct
    fragment loads, asynchronous global-to-LDS copies), single and batched;
    the multi-demand instance has windows of ~24 K chunks (long pipelines),
    the tile-spanning one odd tile counts."""
    monkeypatch.setenv("MHSK_GEMM", kernel)
    insts = [mhsgen.tiny_dense(seed=18, idx=0, n=520, m=2100), mhsgen.multidemand(seed=18, n=1500, m=15000),
             mhsgen.transport(seed=18, n=2500, m=18000)]
    refs = [oracle.run(i) for i in insts]
    for inst, ref in zip(insts, refs):
        say("int8", kernel, inst.name)
        assert_same(mh.reduce(inst, flags=mh.MHS_VARIANT_INT8), ref, f"{inst.name} {kernel}")
    say("int8 batched", kernel)
    for inst, ref, r in zip(insts, refs, mh.reduce_batch(insts, flags=mh.MHS_VARIANT_INT8)):
        assert_same(r, ref, f"{inst.name} {kernel} batched")


def test_device_input_nnz_hint(mh):
    """Device inputs with the nnz hint, without it, and with a wrong one."""
    inst = mhsgen.transport(seed=19, n=1200, m=9000)
    d = mh.DeviceInstance(inst)
    orc = oracle.run(inst)
    say("nnz hint")
    assert_same(mh.reduce(d), orc)
    d.nnz = 0                      # library reads edge_ptr[m] itself
    assert_same(mh.reduce(d), orc)
    d.nnz = inst.nnz - 5           # too small: rejected on the device
    with pytest.raises(mh.MhsError):
        mh.reduce(d)
    d.nnz = inst.nnz + 7           # too large: rejected on the device
    with pytest.raises(mh.MhsError):
        mh.reduce(d)



@pytest.mark.parametrize("variant", ["INT8", "BITSET", "SPARSE"])
def test_superedge_rule(mh, variant):
    """The superedge rule SE in place of DP, every contraction variant."""
    se = mh._lib.MHS_RULE_SE
    flags = getattr(mh, "MHS_VARIANT_" + variant) | se
    insts = [mhsgen.tiny(seed=24, idx=i) for i in range(150)] + \
            [mhsgen.tiny_dense(seed=24, idx=0, n=300, m=1500), mhsgen.multidemand(seed=24, n=1500, m=12000)]
    say("superedge", variant)
    for inst, r in zip(insts, mh.reduce_batch(insts, flags=flags)):
        assert_same(r, oracle.run(inst, rule=oracle.RULE_SE), inst.name + " SE")
    big = mhsgen.transport(seed=24, n=2500, m=18000)
    big.demand[:] = 1 + (np.arange(big.m) % 2) * (np.diff(big.edge_ptr) > 1)
    assert_same(mh.reduce(big, flags=flags), oracle.run(big, rule=oracle.RULE_SE), "transport SE")



def assert_same_fe(r, orc, name=""):
    assert_same(r, orc, name)
    assert (r.forced_v == orc.forced_v).all(), f"{name}: forced sets differ"
    kept = orc.death_e == 0
    assert (r.demand_out[kept] == orc.demand_out[kept]).all(), f"{name}: demands differ"
    assert r.n_forced == orc.n_forced


@pytest.mark.parametrize("variant", ["INT8", "BITSET", "SPARSE"])
def test_full_edge_rule(mh, variant):
    """KernelGPU-FE (FE alternated with DP + MD), every contraction variant,
    single and batched, against the oracle's FE driver."""
    flags = getattr(mh, "MHS_VARIANT_" + variant) | mh.MHS_RULE_FE
    insts = [mhsgen.tiny(seed=27, idx=i) for i in range(200)] + \
            [mhsgen.tiny_dense(seed=27, idx=i, n=200, m=700) for i in range(3)] + \
            [mhsgen.batch_member(seed=27, idx=i, nmax=500) for i in range(6)]
    say("full edge", variant)
    for inst, r in zip(insts, mh.reduce_batch(insts, flags=flags)):
        assert_same_fe(r, oracle.run_fe(inst), inst.name + " FE")
    for inst in insts[-4:]:
        assert_same_fe(mh.reduce(inst, flags=flags), oracle.run_fe(inst), inst.name + " FE single")


@pytest.mark.parametrize("wide", [False, True])
def test_batch_result_layouts(mh, wide):
    """A batch's results travel as 16-bit values when every death round and
    final demand fits (rounds run and vertex counts below 2^16), else as
    int32 (a member with n >= 2^16): both, under FE (demands and forced sets
    change), through the caller's arrays (mhs_run_batch_into) and through
    result objects (mhs_run_batch), against the oracle's FE driver."""
    import ctypes
    import torch
    from paper_2109_06042_amd import _lib
    lib = _lib.load()
    flags = mh.MHS_VARIANT_HYBRID | mh.MHS_RULE_FE
    insts = [mhsgen.tiny(seed=29, idx=i) for i in range(40)] + \
            [mhsgen.batch_member(seed=29, idx=i, nmax=900) for i in range(6)]
    if wide:
        big = mhsgen.transport(seed=29, n=70000, m=4000)
        assert big.n >= 1 << 16
        insts.insert(7, big)
    refs = [oracle.run_fe(i) for i in insts]
    say("result layout", "wide" if wide else "narrow")
    for inst, ref, r in zip(insts, refs, mh.reduce_batch(insts, flags=flags)):
        assert_same_fe(r, ref, inst.name + " into")
    arr, keep, fl = mh._batch_structs(insts, flags)
    need = int(lib.mhs_batch_workspace_bytes(arr, len(insts), fl))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    outs = (ctypes.c_void_p * len(insts))()
    _lib.check(lib.mhs_run_batch(arr, len(insts), fl, ctypes.c_void_p(ws.data_ptr()), need, None, outs))
    try:
        for inst, ref, h in zip(insts, refs, outs):
            de = np.empty(max(inst.m, 1), np.int32)
            dv = np.empty(max(inst.n, 1), np.int32)
            dm = np.empty(max(inst.m, 1), np.int32)
            fv = np.empty(max(inst.n, 1), np.uint8)
            _lib.check(lib.mhs_result_deaths(h, de.ctypes.data, dv.ctypes.data))
            _lib.check(lib.mhs_result_demands(h, dm.ctypes.data))
            _lib.check(lib.mhs_result_forced(h, fv.ctypes.data))
            name = inst.name + " objects"
            assert np.array_equal(de[:inst.m], ref.death_e), name
            assert np.array_equal(dv[:inst.n], ref.death_v), name
            kept = ref.death_e == 0
            assert np.array_equal(dm[:inst.m][kept], ref.demand_out[kept]), name
            assert np.array_equal(fv[:inst.n].astype(bool), np.asarray(ref.forced_v, bool)), name
    finally:
        for h in outs:
            lib.mhs_result_free(h)
    del keep


def test_full_edge_with_superedge_rule(mh):
    flags = mh.MHS_RULE_FE | mh.MHS_RULE_SE
    insts = [mhsgen.tiny(seed=28, idx=i) for i in range(150)]
    say("full edge + superedge")
    for inst, r in zip(insts, mh.reduce_batch(insts, flags=flags)):
        assert_same_fe(r, oracle.run_fe(inst, rule=oracle.RULE_SE), inst.name + " FE+SE")


def long_rows_instance(seed):
    """Interval hyperedges plus a hub vertex in ~6 % of them (degree ~1000,
    beyond the per-lane entry cache of the vertex rows), a long interval
    hyperedge every 150 (70..200 vertices, beyond the edge rows' cache) and an
    isolated vertex; several productive rounds."""
    base = mhsgen.transport(seed=seed, n=2500, m=16000)
    rng = np.random.default_rng(seed)
    edges = [list(e) for e in base.edges()]
    for e in edges:
        if rng.random() < 0.06:
            e.append(base.n)
    for i in range(0, len(edges), 150):
        s = int(rng.integers(0, base.n - 200))
        edges[i] = sorted(set(edges[i]) | set(range(s, s + int(rng.integers(70, 200)))))
    edges = [sorted(set(e)) for e in edges]
    return mhsgen.from_edges(base.n + 2, edges, [1] * len(edges), name=f"long_rows{seed}")


@pytest.mark.parametrize("variant", ["INT8", "BITSET"])
def test_long_rows(mh, variant):
    """Rows longer than the encoder's register cache (reloaded entries) and
    the in-place alive-first partition of vertex lists over many rounds."""
    insts = [long_rows_instance(s) for s in range(3)]
    flag = getattr(mh, "MHS_VARIANT_" + variant)
    refs = [oracle.run(i) for i in insts]
    assert max(r.rounds for r in refs) >= 6
    for inst, ref in zip(insts, refs):
        say("long rows", variant, inst.name)
        assert_same(mh.reduce(inst, flags=flag), ref, inst.name)
    say("long rows batched", variant)
    for inst, ref, r in zip(insts, refs, mh.reduce_batch(insts, flags=flag)):
        assert_same(r, ref, inst.name + " batched")


@pytest.mark.parametrize("variant", ["INT8", "BITSET"])
def test_pair_enumeration(mh, variant):
    """The contraction enumerates tile pairs itself, blockDim candidates per
    workgroup and batch: one tile, a few, a banded instance whose 391 edge
    tiles give more candidates (76,636) than one batch of the grid covers
    (256 per workgroup), and a set whose candidates run on across instances
    of very different tile counts, also with sparse members in between."""
    flag = getattr(mh, "MHS_VARIANT_" + variant)
    insts = [mhsgen.tiny_dense(seed=32, idx=0, n=60, m=100), mhsgen.tiny_dense(seed=32, idx=1, n=300, m=700),
             mhsgen.transport(seed=32, n=6000, m=50000), long_rows_instance(6)]
    refs = [oracle.run(i) for i in insts]
    for inst, ref in zip(insts, refs):
        say("pairs", variant, inst.name)
        assert_same(mh.reduce(inst, flags=flag), ref, inst.name)
    say("pairs batched", variant)
    for inst, ref, r in zip(insts, refs, mh.reduce_batch(insts, flags=flag)):
        assert_same(r, ref, inst.name + " batched")
    if variant == "INT8":
        say("pairs hybrid")
        for inst, ref, r in zip(insts, refs, mh.reduce_batch(insts, flags=mh.MHS_VARIANT_HYBRID)):
            assert_same(r, ref, inst.name + " hybrid")


def test_device_batch_equals_host_batch(mh):
    """Batches of device-resident instances (MHS_INPUT_DEVICE): the same
    results as host batches and the oracle, and the hybrid rule picks the
    same contraction per member (sparse members visit product terms, dense
    ones none) from the span sums computed on the device."""
    insts = [mhsgen.batch_member(seed=33, idx=i, nmax=700) for i in range(24)] + \
            [mhsgen.tiny(seed=33, idx=i) for i in range(40)] + [mhsgen.from_edges(7, [], [])]
    refs = [oracle.run(i) for i in insts]
    dev = [mh.DeviceInstance(i) for i in insts]
    for flags in (mh.MHS_VARIANT_AUTO, mh.MHS_VARIANT_HYBRID, mh.MHS_VARIANT_INT8, mh.MHS_VARIANT_SPARSE,
                  mh.MHS_VARIANT_BITSET):
        say("device batch", flags)
        host_res = mh.reduce_batch(insts, flags=flags)
        dev_res = mh.reduce_batch(dev, flags=flags)
        for inst, ref, a, b in zip(insts, refs, host_res, dev_res):
            assert_same(b, ref, f"{inst.name} device batch flags={flags}")
            assert_same(a, ref, f"{inst.name} host batch flags={flags}")
            assert (a.stats["terms"] > 0) == (b.stats["terms"] > 0), (inst.name, flags)
    styles = {i.meta.get("style") for i in insts[:24]}
    assert styles == {"interval", "uniform"}


def test_device_batch_rejects_bad_member(mh):
    good = [mhsgen.tiny(seed=34, idx=i) for i in range(5)]
    bad = mhsgen.Instance(n=3, m=1, edge_ptr=np.array([0, 2], np.int64), edge_vtx=np.array([0, 7], np.int32),
                          demand=np.array([1], np.int32))
    dev = [mh.DeviceInstance(i) for i in good[:2] + [bad] + good[2:]]
    say("device batch with a bad member")
    with pytest.raises(mh.MhsError) as ei:
        mh.reduce_batch(dev)
    assert "instance 2: " in str(ei.value) and "range" in str(ei.value), str(ei.value)
    nohint = [mh.DeviceInstance(i) for i in good]
    nohint[1].nnz = 0
    with pytest.raises(mh.MhsError) as ei:
        mh.reduce_batch(nohint)
    assert "instance 1: " in str(ei.value) and "nnz" in str(ei.value)
    for inst, r in zip(good, mh.reduce_batch([mh.DeviceInstance(i) for i in good])):
        assert_same(r, oracle.run(inst), inst.name)
