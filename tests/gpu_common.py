"""Shared helpers of the GPU tests (parity of the HIP path with the oracle)."""
import sys

import numpy as np


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def assert_same(gpu, orc, name=""):
    """Bit-exact parity: productive rounds and the deletion round of every
    hyperedge and vertex (which is the round-by-round deletion trace)."""
    assert gpu.rounds == orc.rounds, f"{name}: rounds {gpu.rounds} != {orc.rounds}"
    de = np.nonzero(gpu.death_e != orc.death_e)[0]
    dv = np.nonzero(gpu.death_v != orc.death_v)[0]
    assert de.size == 0, f"{name}: {de.size} hyperedge deaths differ, first {de[:8]} gpu {gpu.death_e[de[:8]]} oracle {orc.death_e[de[:8]]}"
    assert dv.size == 0, f"{name}: {dv.size} vertex deaths differ, first {dv[:8]} gpu {gpu.death_v[dv[:8]]} oracle {orc.death_v[dv[:8]]}"
