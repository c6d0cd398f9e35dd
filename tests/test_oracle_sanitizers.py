"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc) runs the fixtures and random instances cleanly and gives the same
trajectories as the normal build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import golden_io
import mhsgen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    out = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", out,
                           os.path.join(ROOT, "oracle", "mhs_oracle.c"),
                           os.path.join(HERE, "native", "oracle_driver.c")])
    return out


def _text(inst, mode):
    lines = [f"{inst.n} {inst.m} {mode}"]
    for e, f in zip(inst.edges(), inst.demand.tolist()):
        lines.append(" ".join(str(x) for x in [f, len(e)] + e))
    return "\n".join(lines) + "\n"


def test_sanitized_oracle_matches(driver):
    insts = [golden_io.load(f)[0] for f in golden_io.all_fixtures()]
    insts += [mhsgen.tiny(seed=20, idx=i) for i in range(60)]
    insts += [mhsgen.tiny_dense(seed=20, idx=0, n=120, m=400), mhsgen.from_edges(0, [], []),
              mhsgen.from_edges(4, [], [])]
    for mode in (oracle.ALLPAIRS, oracle.PRUNED):
        text = "".join(_text(i, mode) for i in insts)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1")
        res = subprocess.run([driver], input=text, capture_output=True, text=True, env=env, timeout=300)
        assert res.returncode == 0, res.stderr[-2000:]
        lines = res.stdout.splitlines()
        assert len(lines) == 3 * len(insts)
        for k, inst in enumerate(insts):
            rc, rounds = (int(x) for x in lines[3 * k].split())
            ref = oracle.run(inst, mode)
            assert rc == 0 and rounds == ref.rounds
            assert [int(x) for x in lines[3 * k + 1].split()] == ref.death_e.tolist()
            assert [int(x) for x in lines[3 * k + 2].split()] == ref.death_v.tolist()
