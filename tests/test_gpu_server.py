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


def test_poll_never_waits(mh):
    """A poll only takes stock and queues work: while a long reduction (the
    multi-demand instance with dense int8 tiles, hundreds of ms per round)
    is on the device, polls return at once, and the results still match."""
    big = mhsgen.multidemand(seed=0)
    small = [mhsgen.serve_request(seed=6, idx=i, scale_max=0.3) for i in range(8)]
    srv = mh.Server(arena_bytes=16 << 30, max_slots=16, flags=mh.MHS_VARIANT_INT8)
    say("poll never waits")
    srv.submit(big, 100)
    for i, inst in enumerate(small):
        srv.submit(inst, i)
    got, slow = {}, []
    t0 = time.time()
    while len(got) < len(small) + 1:
        t = time.perf_counter()
        out = srv.poll()
        slow.append(time.perf_counter() - t)
        for rid, r in out:
            got[rid] = r
        assert time.time() - t0 < 120
    wall = time.time() - t0
    srv.close()
    say(f"polls: {len(slow)}, longest {max(slow) * 1e3:.1f} ms, wall {wall:.2f} s")
    assert wall > 0.3 and max(slow) < 0.1, (wall, max(slow))
    assert_same(got[100], oracle.run(big), big.name)
    for i, inst in enumerate(small):
        assert_same(got[i], oracle.run(inst), inst.name)


def test_drain(mh):
    insts = [mhsgen.serve_request(seed=7, idx=i, scale_max=0.4) for i in range(24)]
    srv = mh.Server(arena_bytes=4 << 30, max_slots=8)
    say("drain")
    for i, inst in enumerate(insts):
        srv.submit(inst, i)
    srv.drain()
    assert srv.pending() == (0, 0)
    got = {}
    for _ in range(4):                 # the finished results, a few per poll
        for rid, r in srv.poll(cap=10):
            got[rid] = r
    assert sorted(got) == list(range(len(insts)))
    assert srv.poll() == []            # idle
    srv.drain()                        # nothing to do
    for i, inst in enumerate(insts):
        assert_same(got[i], oracle.run(inst), inst.name)
    srv.close()


def test_failed_request_reported(mh, monkeypatch):
    """A request whose device-side check fails (its upload is corrupted by
    the MHSK_SERVER_FAIL_ID test hook: a demand of 0) comes back as an error
    for that request alone; the others are reduced normally."""
    monkeypatch.setenv("MHSK_SERVER_FAIL_ID", "3")
    insts = [mhsgen.serve_request(seed=8, idx=i, scale_max=0.3) for i in range(6)]
    srv = mh.Server(arena_bytes=2 << 30, max_slots=8)
    say("failed request")
    for i, inst in enumerate(insts):
        srv.submit(inst, i)
    got = _drain(srv, len(insts))
    srv.close()
    assert isinstance(got[3], mh.MhsError) and got[3].code == -1 and "demand" in str(got[3]), got[3]
    for i, inst in enumerate(insts):
        if i != 3:
            assert_same(got[i], oracle.run(inst), inst.name)
    monkeypatch.delenv("MHSK_SERVER_FAIL_ID")
    srv = mh.Server(arena_bytes=2 << 30, max_slots=8)
    srv.submit(insts[3], 3)
    got = _drain(srv, 1)
    srv.close()
    assert_same(got[3], oracle.run(insts[3]), insts[3].name)


def test_result_copy_and_round_on_live_results(mh):
    """mhs_result_copy and mhs_result_round on live results of mhs_run: kept
    ids ascending and every productive round's deletions, against the
    oracle's kept ids and per-round deletion lists."""
    import ctypes
    import torch
    from paper_2109_06042_amd import _lib
    lib = _lib.load()
    for inst in (mhsgen.transport(seed=3, n=2000, m=15000), mhsgen.multidemand(seed=3, n=1500, m=12000),
                 mhsgen.from_edges(5, [], [])):
        say("result copy / round", inst.name)
        orc = oracle.run(inst)
        st, keep = mh._host_struct(inst)
        need = mh.workspace_bytes(inst.n, inst.m, inst.nnz)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        _lib.check(lib.mhs_run(ctypes.byref(st), _lib.MHS_TRACE_ROUNDS, ctypes.c_void_p(ws.data_ptr()), need,
                               None, ctypes.byref(h)))
        try:
            assert lib.mhs_result_status(h) == _lib.MHS_OK
            s = _lib.MhsSummary()
            _lib.check(lib.mhs_result_summary(h, ctypes.byref(s)))
            assert (s.n_kept, s.m_kept, s.rounds, s.n_forced, s.k_out) == \
                (len(orc.kept_v), len(orc.kept_e), orc.rounds, 0, inst.k)
            kv = np.full(max(s.n_kept, 1), -1, np.int32)
            ke = np.full(max(s.m_kept, 1), -1, np.int32)
            _lib.check(lib.mhs_result_copy(h, kv.ctypes.data, ke.ctypes.data, None))
            assert np.array_equal(kv[:s.n_kept], orc.kept_v) and np.array_equal(ke[:s.m_kept], orc.kept_e)
            for r in range(1, s.rounds + 1):
                ne, nv = ctypes.c_int32(-1), ctypes.c_int32(-1)
                _lib.check(lib.mhs_result_round(h, r, ctypes.byref(ne), None, ctypes.byref(nv), None))
                de = np.full(max(ne.value, 1), -1, np.int32)
                dv = np.full(max(nv.value, 1), -1, np.int32)
                _lib.check(lib.mhs_result_round(h, r, ctypes.byref(ne), de.ctypes.data, ctypes.byref(nv),
                                                dv.ctypes.data))
                oe, ov = orc.round_deletions(r)
                assert np.array_equal(de[:ne.value], oe) and np.array_equal(dv[:nv.value], ov), r
            assert lib.mhs_result_round(h, s.rounds + 1, None, None, None, None) == _lib.MHS_EINVAL
            assert lib.mhs_result_round(h, 0, None, None, None, None) == _lib.MHS_EINVAL
        finally:
            lib.mhs_result_free(h)
        del keep
