"""The paper-shaped stand-in generators draw valid instances of the stated
shape (CPU only)."""
import numpy as np
import pytest

import mhsgen
import oracle


@pytest.mark.parametrize("alpha", [1, 5, 20, 60])
def test_nci60_shaped(alpha):
    inst = mhsgen.nci60_shaped(seed=0, alpha=alpha)
    sizes = np.diff(inst.edge_ptr)
    assert (inst.n, inst.m) == (7124, 152)
    assert oracle.validate(inst) == 0
    assert (sizes >= 1).all() and np.array_equal(inst.demand, np.minimum(alpha, sizes))
    deg = np.bincount(inst.edge_vtx, minlength=inst.n)
    assert (deg >= 1).all() and 4.0 < deg.mean() < 6.0      # 1 + Poisson(4), capped at m
    again = mhsgen.nci60_shaped(seed=0, alpha=alpha)
    assert np.array_equal(again.edge_vtx, inst.edge_vtx)    # a pure function of the seed


@pytest.mark.parametrize("alpha", [1, 5, 30])
def test_girg_shaped(alpha):
    inst = mhsgen.girg_shaped(seed=0, alpha=alpha)
    sizes = np.diff(inst.edge_ptr)
    assert (inst.n, inst.m) == (15015, 1903)
    assert oracle.validate(inst) == 0
    assert 7.0 < sizes.mean() < 9.0
    assert np.array_equal(inst.demand, np.minimum(alpha, sizes))
    # interval hyperedges: members span at most 18 consecutive ids
    for e in range(0, inst.m, 97):
        vs = inst.edge_vtx[inst.edge_ptr[e]:inst.edge_ptr[e + 1]]
        assert vs[-1] - vs[0] < 18


def test_serve_request_size_override():
    a = mhsgen.serve_request(seed=0, idx=3)
    b = mhsgen.serve_request(seed=0, idx=3)
    assert np.array_equal(a.edge_vtx, b.edge_vtx)
    big = mhsgen.serve_request(seed=0, idx=3, u=1.0, style="uniform")
    assert (big.n, big.m) == (30000, 300000) and big.meta["style"] == "uniform"
