"""GPU parity at the measured configurations' full sizes: the HIP path
(through the C ABI) against the CPU oracle, bit-exact, round by round (the
deletion round of every hyperedge and vertex), for

* the plain instance (n=200, m=1000), default and int8 MFMA contraction;
* the multi-demand instance (n=20000, m=200000) with the int8 MFMA, bitset
  and sparse contractions;
* every member of the 512-instance batch, under the default (hybrid) and the
  int8 schedule;
* a stream of serving requests over the whole log-uniform size range, two of
  them the largest size (n=30000, m=300000), checked in the mix;
* a set of more than 1024 instances (instance prefixes then stay in global
  memory instead of LDS).

The oracle runs in spawned host processes (tests/oracle_pool.py)."""
import time

import numpy as np
import pytest

import mhsgen
import oracle
import oracle_pool
from gpu_common import say, assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2109_06042_amd as mh
    mh._lib.load()
    return mh


def test_plain_config_int8_and_default(mh):
    inst = mhsgen.plain(seed=0)
    orc = oracle.run(inst)
    for flags in (0, mh.MHS_VARIANT_INT8, mh.MHS_VARIANT_INT8 | mh.MHS_GRAPH):
        say("plain config", inst.name, "flags", flags)
        assert_same(mh.reduce(inst, flags=flags), orc, f"{inst.name} flags={flags}")
        assert_same(mh.reduce(mh.DeviceInstance(inst), flags=flags), orc, f"{inst.name} device flags={flags}")


@pytest.fixture(scope="module")
def multidemand():
    inst = mhsgen.multidemand(seed=0)
    say("multidemand oracle", inst.name)
    return inst, oracle.run(inst)


@pytest.mark.parametrize("variant", ["INT8", "BITSET", "SPARSE"])
def test_multidemand_config_full(mh, multidemand, variant):
    import torch
    inst, orc = multidemand
    dev = mh.DeviceInstance(inst)
    flags = getattr(mh, "MHS_VARIANT_" + variant)
    ws = torch.empty(mh.workspace_bytes(inst.n, inst.m, inst.nnz, mh.MHS_INPUT_DEVICE), dtype=torch.uint8,
                     device="cuda")
    say("multidemand full", variant)
    assert_same(mh.reduce(dev, flags=flags, workspace=ws), orc, f"{inst.name} {variant}")
    del ws


@pytest.fixture(scope="module")
def batch512():
    t = time.time()
    insts = mhsgen.batch(512)
    say(f"batch of 512 generated in {time.time() - t:.1f} s; oracle on {oracle_pool.workers()} processes")
    t = time.time()
    refs = oracle_pool.run_all([("batch", 0, i, {}) for i in range(512)])
    say(f"batch oracle {time.time() - t:.1f} s")
    return insts, refs


@pytest.mark.parametrize("variant", ["AUTO", "INT8"])
def test_batch_config_every_member(mh, batch512, variant):
    insts, refs = batch512
    say("batch of 512", variant)
    res = mh.reduce_batch(insts, flags=getattr(mh, "MHS_VARIANT_" + variant))
    assert len(res) == len(insts)
    for inst, r, ref in zip(insts, res, refs):
        assert_same(r, ref, f"{inst.name} {variant}")


def test_set_beyond_lds_prefix(mh):
    """1100 tiny instances with larger ones in between: a set of more than
    1024 members maps its work units through prefixes in global memory."""
    insts = [mhsgen.tiny(seed=51, idx=i) for i in range(1100)]
    for k, i in enumerate(range(37, 1100, 137)):
        insts.insert(i, mhsgen.batch_member(seed=51, idx=k, nmax=300))
    refs = [oracle.run(i) for i in insts]
    for variant in ("AUTO", "INT8", "BITSET", "SPARSE"):
        say("set of", len(insts), variant)
        for inst, ref, r in zip(insts, refs, mh.reduce_batch(insts, flags=getattr(mh, "MHS_VARIANT_" + variant))):
            assert_same(r, ref, f"{inst.name} {variant}")


def test_serving_stream_full_range(mh):
    """200 requests over the whole log-uniform range plus the largest size
    in both styles, arriving while earlier ones are resident; every result
    in the mix equals the oracle's."""
    specs = [("serve", 9, i, {}) for i in range(200)]
    specs += [("serve", 9, 200, {"u": 1.0, "style": "interval"}), ("serve", 9, 201, {"u": 1.0, "style": "uniform"})]
    t = time.time()
    reqs = [mhsgen.make(f, seed=s, idx=i, **kw) for f, s, i, kw in specs]
    say(f"serving stream generated in {time.time() - t:.1f} s: {len(reqs)} requests, "
        f"max n={max(r.n for r in reqs)} max m={max(r.m for r in reqs)}")
    assert max(r.n for r in reqs) >= 25000 and max(r.m for r in reqs) >= 250000
    t = time.time()
    # the largest first: they set the pool's critical path
    order = sorted(range(len(specs)), key=lambda i: -reqs[i].m)
    refs_sorted = oracle_pool.run_all([specs[i] for i in order])
    refs = [None] * len(specs)
    for i, r in zip(order, refs_sorted):
        refs[i] = r
    say(f"serving oracle {time.time() - t:.1f} s")
    srv = mh.Server(arena_bytes=64 << 30, max_slots=128)
    got = {}
    t0 = time.time()
    # requests arrive in four waves, each while the earlier ones are on the GPU
    waves = np.array_split(np.arange(len(reqs)), 4)
    for w in waves:
        for i in w:
            srv.submit(reqs[i], int(i))
        for _ in range(3):
            for rid, r in srv.poll():
                got[rid] = r
    while len(got) < len(reqs):
        for rid, r in srv.poll():
            got[rid] = r
        assert time.time() - t0 < 240, "server did not finish"
    srv.close()
    say(f"served {len(reqs)} in {time.time() - t0:.1f} s")
    for i, inst in enumerate(reqs):
        assert not isinstance(got[i], Exception), got[i]
        assert_same(got[i], refs[i], inst.name)


@pytest.mark.parametrize("variant", ["AUTO", "INT8", "BITSET", "SPARSE"])
def test_paper_shaped_standins(mh, variant):
    """The paper's aspect ratio (vertices far outnumber hyperedges, so the
    vertex phase dominates): NCI60-shaped (n=7124, m=152) and GIRG-shaped
    (n=15015, m=1903) instances at several demand caps alpha, single and
    batched."""
    flags = getattr(mh, "MHS_VARIANT_" + variant)
    insts = [mhsgen.nci60_shaped(seed=0, alpha=a) for a in (1, 5, 20, 60)]
    insts += [mhsgen.girg_shaped(seed=0, idx=i, alpha=a) for i, a in enumerate((1, 5, 10, 30))]
    refs = [oracle.run(i) for i in insts]
    for inst, ref in zip(insts, refs):
        say("paper-shaped", variant, inst.name)
        assert_same(mh.reduce(inst, flags=flags), ref, f"{inst.name} {variant}")
    say("paper-shaped batched", variant)
    for inst, ref, r in zip(insts, refs, mh.reduce_batch(insts, flags=flags)):
        assert_same(r, ref, f"{inst.name} {variant} batched")
