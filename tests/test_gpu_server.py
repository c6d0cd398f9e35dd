"""Serving (continuous batching): results in a mix equal results alone and
the oracle's, bit-exact; admission by footprint never overcommits the arena;
oversized requests are rejected; submit works from another thread."""
import threading
import time

import numpy as np
import pytest

import mhsgen
import oracle
from gpu_common import say, assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import torch
    assert torch.cuda.is_available()
    import paper_2109_06042_amd as mh
    mh._lib.load()
    return mh


def _drain(srv, expect, budget_s=120.0):
    got = {}
    t0 = time.time()
    while len(got) < expect:
        for rid, r in srv.poll():
            got[rid] = r
        assert time.time() - t0 < budget_s, "server did not finish"
    return got


def test_mix_equals_alone_and_oracle(mh):
    insts = [mhsgen.serve_request(seed=1, idx=i, scale_max=0.45) for i in range(40)]
    insts += [mhsgen.tiny_dense(seed=2, idx=i, n=150, m=700) for i in range(6)]
    say("server mix of", len(insts))
    srv = mh.Server(arena_bytes=8 << 30, max_slots=64)
    for i, inst in enumerate(insts[:20]):
        srv.submit(inst, i)
    got = {}
    # the rest arrive while the first ones are resident (continuous batching)
    for _ in range(3):
        for rid, r in srv.poll():
            got[rid] = r
    for i, inst in enumerate(insts[20:], start=20):
        srv.submit(inst, i)
    got.update(_drain(srv, len(insts) - len(got)))
    for i, inst in enumerate(insts):
        orc = oracle.run(inst)
        assert_same(got[i], orc, "mix " + inst.name)
    # alone: a fresh server with one request, and the plain path
    for i in (0, 7, 21, 41):
        srv1 = mh.Server(arena_bytes=2 << 30, max_slots=4)
        srv1.submit(insts[i], 99)
        alone = _drain(srv1, 1)[99]
        srv1.close()
        assert_same(alone, got[i], "alone vs mix " + insts[i].name)
        assert_same(mh.reduce(insts[i]), got[i], "plain vs mix " + insts[i].name)
    srv.close()


def test_request_id_widths(mh):
    """Requests are kept on the host with 16-bit vertex ids when n <= 65536
    (ids up to 65535) and 32-bit ids beyond, and widened when uploaded."""
    rng = np.random.default_rng(29)
    top = [sorted({65535} | set(int(v) for v in rng.choice(65535, size=int(rng.integers(1, 5)), replace=False)))
           for _ in range(300)]
    insts = [mhsgen.from_edges(65536, top, name="ids-to-65535"),
             mhsgen.transport(seed=29, n=70000, m=2500),
             mhsgen.from_edges(65537, top + [[65536]], name="ids-past-65535"),
             mhsgen.serve_request(seed=29, idx=0, scale_max=0.3)]
    say("server id widths")
    srv = mh.Server(arena_bytes=2 << 30, max_slots=8)
    for i, inst in enumerate(insts):
        srv.submit(inst, i)
    got = _drain(srv, len(insts))
    srv.close()
    for i, inst in enumerate(insts):
        assert_same(got[i], oracle.run(inst), inst.name)


def test_admission_never_overcommits(mh):
    insts = [mhsgen.plain(seed=s, n=400, m=3000) for s in range(10)]
    fp = mh.workspace_bytes(400, 3000, int(insts[0].nnz) + 64)
    arena = int(2.5 * fp) + (64 << 10)   # room for two requests plus the control blocks
    say("admission arena", arena)
    srv = mh.Server(arena_bytes=arena, max_slots=16)
    for i, inst in enumerate(insts):
        srv.submit(inst, i)
    got = {}
    peak_res = 0
    t0 = time.time()
    while len(got) < len(insts):
        for rid, r in srv.poll():
            got[rid] = r
        q, res = srv.pending()
        peak_res = max(peak_res, res)
        assert srv.arena_used() <= arena
        assert time.time() - t0 < 120
    assert 1 <= peak_res <= 2
    for i, inst in enumerate(insts):
        assert_same(got[i], oracle.run(inst), inst.name)
    srv.close()


def test_reject_oversized(mh):
    srv = mh.Server(arena_bytes=64 << 20, max_slots=4)
    big = mhsgen.multidemand(seed=0, n=5000, m=50000)
    say("reject oversized")
    with pytest.raises(mh.MhsError) as ei:
        srv.submit(big, 1)
    assert ei.value.code == -5
    small = mhsgen.plain(seed=0)
    srv.submit(small, 2)
    got = _drain(srv, 1)
    assert_same(got[2], oracle.run(small))
    srv.close()


def test_submit_from_other_thread(mh):
    insts = [mhsgen.serve_request(seed=3, idx=i, scale_max=0.3) for i in range(16)]
    srv = mh.Server(arena_bytes=4 << 30, max_slots=8)
    say("threaded submit")

    def producer():
        for i, inst in enumerate(insts):
            srv.submit(inst, i)
            time.sleep(0.002)

    th = threading.Thread(target=producer)
    th.start()
    got = {}
    t0 = time.time()
    while len(got) < len(insts):
        for rid, r in srv.poll():
            got[rid] = r
        assert time.time() - t0 < 120
    th.join()
    for i, inst in enumerate(insts):
        assert_same(got[i], oracle.run(inst), inst.name)
    srv.close()


def test_poisoned_arena(mh):
    """Regression: the resident set's global counters must be cleared when the
    set is built (the arena is caller memory with arbitrary contents)."""
    import torch
    insts = [mhsgen.serve_request(seed=4, idx=i, scale_max=0.3) for i in range(6)]
    srv = mh.Server(arena_bytes=1 << 30, max_slots=8)
    srv.arena.fill_(255)
    torch.cuda.synchronize()
    say("poisoned arena")
    for i, inst in enumerate(insts):
        srv.submit(inst, i)
    got = _drain(srv, len(insts))
    for i, inst in enumerate(insts):
        assert_same(got[i], oracle.run(inst), inst.name)
    srv.close()
