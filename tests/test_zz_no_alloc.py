"""mhs_run_static, the entry point that allocates nothing (its workspace is
the library's static device scratch), against mhs_run on the same inputs,
bit-exact: two calls in a row, the second with a smaller instance, host and
device inputs; an instance larger than the scratch is refused."""
import numpy as np
import pytest

import mhsgen
from gpu_common import say, assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2109_06042_amd as mh
    mh._lib.load()
    return mh


def _same_summary(a, b, name):
    assert a.rounds == b.rounds and a.k_out == b.k_out and a.n_forced == b.n_forced, name
    assert len(a.kept_v) == len(b.kept_v) and len(a.kept_e) == len(b.kept_e), name


def test_static_matches_run_two_calls(mh):
    from paper_2109_06042_amd import _lib
    big = mhsgen.plain(seed=0)
    small = mhsgen.tiny_dense(seed=61, idx=0, n=64, m=96)
    for inst in (big, small):
        assert mh.workspace_bytes(inst.n, inst.m, inst.nnz) <= _lib.MHS_STATIC_SCRATCH_BYTES
    for inst in (big, small):           # the second call is smaller than the first
        say("static vs run", inst.name)
        ref = mh.reduce(inst)
        got = mh.reduce_static(inst)
        assert_same(got, ref, inst.name + " static")
        _same_summary(got, ref, inst.name)
    # device inputs, the other order, and a multi-round instance with demands
    multi = mhsgen.tiny_dense(seed=62, idx=1, n=300, m=1500)
    for inst in (multi, small):
        say("static vs run, device input", inst.name)
        ref = mh.reduce(mh.DeviceInstance(inst))
        got = mh.reduce_static(mh.DeviceInstance(inst))
        assert_same(got, ref, inst.name + " static device")
        _same_summary(got, ref, inst.name)
    for flags in (mh.MHS_VARIANT_SPARSE, mh.MHS_RULE_SE, mh.MHS_RULE_FE):
        ref = mh.reduce(multi, flags=flags)
        got = mh.reduce_static(multi, flags=flags)
        assert_same(got, ref, f"{multi.name} static flags={flags}")
        _same_summary(got, ref, multi.name)


def test_static_refuses_oversized_and_bad_flags(mh):
    from paper_2109_06042_amd import _lib
    big = mhsgen.transport(seed=0)
    assert mh.workspace_bytes(big.n, big.m, big.nnz) > _lib.MHS_STATIC_SCRATCH_BYTES
    say("static oversized")
    with pytest.raises(mh.MhsError) as ei:
        mh.reduce_static(big)
    assert ei.value.code == _lib.MHS_ENOSPC and "scratch" in str(ei.value)
    with pytest.raises(mh.MhsError) as ei:
        mh.reduce_static(mhsgen.plain(seed=0), flags=mh.MHS_GRAPH)
    assert ei.value.code == _lib.MHS_EINVAL
    # the scratch still serves a normal call afterwards
    inst = mhsgen.plain(seed=1)
    assert_same(mh.reduce_static(inst), mh.reduce(inst), inst.name)
    empty = mhsgen.from_edges(0, [], [])
    assert mh.reduce_static(empty).rounds == 0
