"""The oracle over many generated instances on the host cores (test
infrastructure): spawned worker processes regenerate each instance from its
(family, seed, idx, options) and run the CPU oracle on it; nothing here
touches the GPU."""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def workers() -> int:
    # the machine's CPU share for one GPU is 16 cores, whatever the machine shows
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _one(spec):
    import mhsgen
    import oracle
    family, seed, idx, kw = spec
    inst = mhsgen.make(family, seed=seed, idx=idx, **kw)
    r = oracle.run(inst)
    return r.rounds, r.death_e, r.death_v


class Ref:
    def __init__(self, rounds, death_e, death_v):
        self.rounds = rounds
        self.death_e = np.asarray(death_e)
        self.death_v = np.asarray(death_v)


def run_all(specs):
    """Oracle results of the instances named by specs [(family, seed, idx,
    kwargs)], in order; the largest are started first."""
    with ProcessPoolExecutor(max_workers=workers(), mp_context=mp.get_context("spawn")) as ex:
        out = list(ex.map(_one, specs, chunksize=1))
    return [Ref(*o) for o in out]
