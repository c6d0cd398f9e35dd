"""Benchmark: kernelizations per second of the DP + MD reduction (Algorithm 3)
on one MI355X, with latency percentiles, the batched path, the roofline of
the dominant kernel and the single-core oracle as CPU baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-batch] [--no-serve]

One step = one kernelization of the transport workload (n=8000 vertices on a
line, m=60000 interval hyperedges of length 5..40 with members kept with
p=0.8, f=1): the CSR is resident in HBM before the timed region; a step runs
every round to the fixpoint and returns the surviving ids and the per-round
deletion trace to host memory.  Every timed configuration is first checked
bit-exact against the oracle.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# published MI355X peaks
PEAK_INT8_OPS = 5.0e15     # dense int8 MFMA, ops/s
PEAK_HBM = 8.0e12          # bytes/s


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-multidemand", action="store_true")
    ap.add_argument("--no-plain-small", action="store_true")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-arena-gb", type=int, default=96)
    ap.add_argument("--serve-slots", type=int, default=256)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (HBM counter calibration)")
    return ap.parse_args()


def committed_traffic(kernel, tag="transport_plain"):
    """HBM bytes per launch of `kernel` (both phases averaged) from the committed
    rocprofv3 --pmc summary, or None when there is none or the kernel source
    changed since the counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(here, "paper_2109_06042_amd", "csrc", "kernels.hip")
    path = os.path.join(here, "profiles", f"hbm_traffic_{tag}.txt")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    vals = []
    for line in open(path):
        f = line.split()
        if len(f) == 4 and f[0] == "traffic" and f[1].split("<")[0] == kernel and f[2] == f"sha={sha}":
            vals.append(float(f[3].split("=")[1]))
    return sum(vals) / len(vals) if vals else None


def same(a, b):
    return a.rounds == b.rounds and np.array_equal(a.death_e, b.death_e) and np.array_equal(a.death_v, b.death_v)


def pct(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the library has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copied 1 GiB x 5")
        return
    import mhsgen
    import oracle
    import paper_2109_06042_amd as mh

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)

    # ---------------------------------------------------------- plain path
    inst = mhsgen.transport(seed=0)
    log(f"workload {inst.name}: nnz={inst.nnz}")
    t = time.time()
    ref = oracle.run(inst)
    oracle_one = time.time() - t
    dev = mh.DeviceInstance(inst)
    torch.cuda.synchronize()
    need = mh.workspace_bytes(inst.n, inst.m, inst.nnz, mh.MHS_INPUT_DEVICE)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    first = mh.reduce(dev, workspace=ws)
    if not same(first, ref):
        log("PARITY FAILURE against the oracle on the bench workload")
        sys.exit(1)
    log(f"parity ok: rounds={ref.rounds} kept_e={len(ref.kept_e)} kept_v={len(ref.kept_v)}")
    for _ in range(args.warmup):
        mh.reduce(dev, workspace=ws)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s = time.perf_counter()
        r = mh.reduce(dev, workspace=ws)
        lat.append((time.perf_counter() - s) * 1e3)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = args.steps / el
    if not same(r, ref):
        log("PARITY FAILURE in the timed loop")
        sys.exit(1)
    log(f"plain: {value:.1f} kernelizations/s, {el / args.steps * 1e3:.3f} ms/step")

    # host-input (PCIe-inclusive) rate, for reference
    hws = torch.empty(mh.workspace_bytes(inst.n, inst.m, inst.nnz, 0), dtype=torch.uint8, device="cuda")
    mh.reduce(inst, workspace=hws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nh = max(5, args.steps // 5)
    for _ in range(nh):
        mh.reduce(inst, workspace=hws)
    torch.cuda.synchronize()
    host_rate = nh / (time.perf_counter() - t1)
    del hws

    # ------------------------------------------- dominant kernel (events)
    # Profiled runs time every step of every round with HIP events on the
    # stream the kernels run on (a bounded device delay first lets the host
    # enqueue the round, so the kernels run back to back).
    prof = [mh.reduce(dev, flags=mh.MHS_PROFILE, workspace=ws) for _ in range(5)]
    st = {k: float(np.median([p.stats[k] for p in prof])) for k in prof[0].stats}
    launches = max(int(st["gemm_launches"]), 1)      # one launch per phase per round
    steps = {"k_rows_encode": st["rows_ms"],
             "k_gemm_lds": st["gemm_ms"], "k_compact": st["compact_ms"],
             "k_round_end": st["round_end_ms"]}
    gemm_ms = st["gemm_ms"] / launches
    gemm_rate = st["issued_ops"] / launches / (gemm_ms * 1e-3) if gemm_ms > 0 else 0.0
    rows_ms = st["rows_ms"] / launches
    rows_rate = st["encode_bytes"] / launches / (rows_ms * 1e-3) if rows_ms > 0 else 0.0
    gemm_roof = {"kernel": "k_gemm_lds (fused int8 MFMA contraction + DP/MD test)", "bound": "mfma",
                 "achieved": gemm_rate / 1e12, "peak": PEAK_INT8_OPS / 1e12, "unit": "TOPS",
                 "frac": gemm_rate / PEAK_INT8_OPS, "traffic": committed_traffic("k_gemm_lds"),
                 "ops_per_launch": st["issued_ops"] / launches, "us_per_launch": gemm_ms * 1e3,
                 "launches_per_step": launches}
    rows_roof = {"kernel": "k_rows_encode (rows, windows, tile encoding)", "bound": "hbm",
                 "achieved": rows_rate / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                 "frac": rows_rate / PEAK_HBM, "traffic": committed_traffic("k_rows_encode"),
                 "bytes_per_launch": st["encode_bytes"] / launches, "us_per_launch": rows_ms * 1e3,
                 "launches_per_step": launches}
    dominant = max(steps, key=steps.get)
    roofline = rows_roof if dominant == "k_rows_encode" else gemm_roof
    roofline["dominant_by_event_time"] = dominant
    log("per-step event time per kernelization (ms): " + ", ".join(f"{k} {v:.3f}" for k, v in steps.items()))
    log(f"k_gemm: {gemm_ms * 1e3:.1f} us/launch, {gemm_rate / 1e12:.2f} TOPS; "
        f"k_rows_encode: {rows_ms * 1e3:.1f} us/launch, {rows_rate / 1e9:.1f} GB/s")

    out = {
        "metric": "kernelizations/sec + p50/p99 latency, batched vs plain, bit-exact to oracle",
        "value": value,
        "unit": "kernelizations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {
            "workload": "transport: n=8000 vertices on a line, m=60000 interval hyperedges "
                        "(length U{5..40}, members kept p=0.8), f=1, seed 0, CSR resident in HBM",
            "rounds": int(ref.rounds),
            "kept_e": int(len(ref.kept_e)),
            "kept_v": int(len(ref.kept_v)),
            "path": "plain (one instance per call, rounds launched directly, one round queued ahead)",
        },
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "host_input_rate": host_rate,
        "roofline": roofline,
        "roofline_other": rows_roof if roofline is gemm_roof else gemm_roof,
        "step_ms_per_kernelization": steps,
    }

    # ---------------------------------- small plain instance (n=200, m=1000)
    if not args.no_plain_small:
        try:
            small = mhsgen.plain(seed=0)
            sref = oracle.run(small)
            sdev = mh.DeviceInstance(small)
            sws = torch.empty(mh.workspace_bytes(small.n, small.m, small.nnz, mh.MHS_INPUT_DEVICE),
                              dtype=torch.uint8, device="cuda")
            if not same(mh.reduce(sdev, workspace=sws), sref):
                raise RuntimeError("plain-small parity failure")
            for _ in range(3):
                mh.reduce(sdev, workspace=sws)
            slat = []
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(100):
                s0 = time.perf_counter()
                mh.reduce(sdev, workspace=sws)
                slat.append((time.perf_counter() - s0) * 1e3)
            sel = time.perf_counter() - t
            out["plain_small"] = {"workload": "plain: n=200, m=1000, |e|~U{2..8} uniform members, f=1",
                                  "kernelizations_per_s": 100 / sel, "p50_ms": pct(slat, 50),
                                  "p99_ms": pct(slat, 99), "rounds": int(sref.rounds)}
            log(f"plain small: {100 / sel:.1f}/s")
        except Exception as e:
            log(f"plain-small section failed: {e!r}")
            out["plain_small"] = {"error": repr(e)}

    # -------------------------------------------------------- batched path
    if not args.no_batch:
        try:
            out["batched"] = bench_batch(mh, torch, oracle, mhsgen, args)
        except Exception as e:  # report, keep the main line
            log(f"batched section failed: {e!r}")
            out["batched"] = {"error": repr(e)}

    # --------------------------------- multiple demands: int8 vs bitset
    if not args.no_multidemand:
        try:
            out["multidemand"] = bench_multidemand(mh, torch, oracle, mhsgen, args)
        except Exception as e:
            log(f"multidemand section failed: {e!r}")
            out["multidemand"] = {"error": repr(e)}

    # --------------------------------------------------------- served path
    if not args.no_serve:
        try:
            out["served"] = bench_serve(mh, torch, oracle, mhsgen, args)
        except Exception as e:
            log(f"served section failed: {e!r}")
            out["served"] = {"error": repr(e)}

    # --------------------------------------------------------- CPU oracle
    if not args.no_cpu:
        n = 0
        t = time.time()
        while True:
            oracle.run(mhsgen.transport(seed=n))
            n += 1
            if time.time() - t >= args.cpu_seconds:
                break
        cel = time.time() - t
        out["cpu_baseline"] = {
            "value": n / cel, "unit": "kernelizations/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} full-size transport instances (seeds 0..{n - 1}), pruned-candidate "
                      f"oracle, single thread, {cel:.1f} s",
        }
    print(json.dumps(out), flush=True)


def bench_batch(mh, torch, oracle, mhsgen, args):
    insts = mhsgen.batch(args.batch_count)
    log(f"batch: {len(insts)} instances, sum m={sum(i.m for i in insts)}, sum n={sum(i.n for i in insts)}")
    need = mh.batch_workspace_bytes(insts)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    log(f"batch workspace {need / 2**30:.2f} GiB")
    res = mh.reduce_batch(insts, workspace=ws)
    # parity: a sample against the oracle, the rest against the plain GPU path
    rng = np.random.default_rng(0)
    sample = rng.choice(len(insts), size=min(12, len(insts)), replace=False)
    for i in sample:
        if not same(res[i], oracle.run(insts[i])):
            raise RuntimeError(f"batched parity failure on {insts[i].name}")
    # schedule autotuner on a 64-instance sample of the batch
    tsample = [insts[i] for i in rng.choice(len(insts), size=min(64, len(insts)), replace=False)]
    tw = torch.empty(mh.batch_workspace_bytes(tsample), dtype=torch.uint8, device="cuda")
    t = time.perf_counter()
    rep = mh.tune(tsample, workspace=tw)
    tune_s = time.perf_counter() - t
    del tw
    best = rep["best_flags"]
    log(f"autotune: best flags {best:#x} ({rep['best_ms']:.1f} ms vs default {rep['default_ms']:.1f} ms on the sample)")
    timings = {}
    for name, flags in (("default", mh.MHS_VARIANT_INT8), ("hybrid", mh.MHS_VARIANT_HYBRID), ("tuned", best)):
        res_t = mh.reduce_batch(insts, flags=flags, workspace=ws)
        for i in sample:
            if not same(res_t[i], res[i]):
                raise RuntimeError(f"{name} batch differs")
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = 2
        for _ in range(reps):
            mh.reduce_batch(insts, flags=flags, workspace=ws)
        torch.cuda.synchronize()
        timings[name] = (time.perf_counter() - t) / reps
    el = min(timings.values())
    # plain path over a subset for the batched-vs-plain comparison
    sub = [insts[i] for i in sample]
    pws = torch.empty(max(mh.workspace_bytes(i.n, i.m, i.nnz) for i in sub), dtype=torch.uint8, device="cuda")
    t = time.perf_counter()
    for i, inst in zip(sample, sub):
        if not same(mh.reduce(inst, workspace=pws), res[i]):
            raise RuntimeError("batched != plain")
    plain_el = (time.perf_counter() - t) / len(sub)
    return {
        "workload": f"{len(insts)} instances, n~U{{100..4000}}, m=n*U(5,10), interval/uniform 50/50, f in {{1,2}}",
        "kernelizations_per_s": len(insts) / el,
        "batch_ms": el * 1e3,
        "default_schedule_kernelizations_per_s": len(insts) / timings["default"],
        "hybrid_schedule_kernelizations_per_s": len(insts) / timings["hybrid"],
        "tuned_schedule_kernelizations_per_s": len(insts) / timings["tuned"],
        "tuned_flags": hex(best),
        "tune_s": tune_s,
        "plain_kernelizations_per_s_same_mix": 1.0 / plain_el,
        "oracle_checked": int(len(sample)),
        "oracle_all_cores": oracle_all_cores(args.cpu_seconds),
    }


def bench_multidemand(mh, torch, oracle, mhsgen, args):
    inst = mhsgen.multidemand(seed=0)
    log(f"multidemand {inst.name}: nnz={inst.nnz}; oracle...")
    t = time.time()
    ref = oracle.run(inst)
    oracle_s = time.time() - t
    dev = mh.DeviceInstance(inst)
    ws = torch.empty(mh.workspace_bytes(inst.n, inst.m, inst.nnz, mh.MHS_INPUT_DEVICE), dtype=torch.uint8,
                     device="cuda")
    out = {"workload": "multidemand: n=20000, m=200000, |e| power law 2.2 on [2,200], f~U{1,2,3} capped",
           "rounds": int(ref.rounds), "oracle_s": oracle_s}
    for name, flag, peak, env in (("int8", mh.MHS_VARIANT_INT8, PEAK_INT8_OPS, "lds"),
                                  ("int8_direct_loads", mh.MHS_VARIANT_INT8, PEAK_INT8_OPS, "direct"),
                                  ("bitset", mh.MHS_VARIANT_BITSET, None, "lds"),
                                  ("sparse", mh.MHS_VARIANT_SPARSE, None, "lds")):
        os.environ["MHSK_GEMM"] = env
        r = mh.reduce(dev, flags=flag, workspace=ws)
        if not same(r, ref):
            raise RuntimeError(f"multidemand parity failure ({name})")
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = 1
        for _ in range(reps):
            mh.reduce(dev, flags=flag, workspace=ws)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t) / reps
        p = mh.reduce(dev, flags=flag | mh.MHS_PROFILE, workspace=ws).stats
        launches = max(p["gemm_launches"], 1)
        rate = p["issued_ops"] / (p["gemm_ms"] * 1e-3) if p["gemm_ms"] > 0 else 0.0
        ent = {"kernelizations_per_s": 1.0 / el, "ms": el * 1e3, "gemm_ms": p["gemm_ms"],
               "edge_gemm_ms": p["edge_gemm_ms"], "vertex_gemm_ms": p["vertex_gemm_ms"],
               "issued_ops": p["issued_ops"], "gemm_launches": launches,
               "contraction_rate_tops": rate / 1e12, "nonzero_terms": p["terms"]}
        if peak:
            ent["frac_of_int8_peak"] = rate / peak
        out[name] = ent
        log(f"multidemand {name}: {el * 1e3:.1f} ms/kernelization, gemm {p['gemm_ms']:.1f} ms, {rate / 1e12:.1f} TOPS")
    os.environ.pop("MHSK_GEMM", None)
    return out


def _serve_pass(mh, reqs, arena, slots, arrivals):
    """Submit request i at arrivals[i] (seconds from start); poll until all
    are done.  Returns (latencies_ms, wall_s, results)."""
    srv = mh.Server(arena, max_slots=slots)
    n = len(reqs)
    done = {}
    lat = np.zeros(n)
    nxt = 0
    t0 = time.perf_counter()
    while len(done) < n:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            srv.submit(reqs[nxt], nxt)
            nxt += 1
        q, res = srv.pending()
        if q == 0 and res == 0 and nxt < n:
            time.sleep(max(0.0, min(0.002, arrivals[nxt] - now)))
            continue
        for rid, r in srv.poll():
            done[rid] = r
            lat[rid] = (time.perf_counter() - t0 - arrivals[rid]) * 1e3
    wall = time.perf_counter() - t0
    srv.close()
    return lat, wall, done


def _gen_requests(lo, hi):
    import mhsgen
    return [mhsgen.serve_request(seed=0, idx=i) for i in range(lo, hi)]


def _oracle_batch_worker(w, P, seconds):
    """Oracle over batch members w, w + P, ... for `seconds`; (count, elapsed)."""
    import mhsgen
    import oracle
    t = time.time()
    n, i = 0, w
    while time.time() - t < seconds:
        oracle.run(mhsgen.batch_member(seed=0, idx=i))
        n += 1
        i += P
    return n, time.time() - t


def _cpu_pool(P):
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    # spawned workers: they import numpy and the generators only, never the GPU
    return ProcessPoolExecutor(max_workers=P, mp_context=mp.get_context("spawn"))


def cpu_workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def oracle_all_cores(seconds):
    """The oracle on every host core at once (independent instances of the
    batched mix), as the all-core CPU throughput beside the batched GPU path."""
    P = cpu_workers()
    with _cpu_pool(P) as ex:
        res = list(ex.map(_oracle_batch_worker, range(P), [P] * P, [seconds] * P))
    n = sum(r[0] for r in res)
    el = max(r[1] for r in res)
    return {"kernelizations_per_s": n / el, "cores": P, "kind": "oracle",
            "sample": f"{n} batch-mix instances on {P} processes, {el:.1f} s"}


def bench_serve(mh, torch, oracle, mhsgen, args):
    R = args.serve_requests
    P = cpu_workers()
    step = (R + P - 1) // P
    with _cpu_pool(P) as ex:
        parts = list(ex.map(_gen_requests, range(0, R, step), [min(R, i + step) for i in range(0, R, step)]))
    reqs = [r for part in parts for r in part]
    arena = args.serve_arena_gb << 30
    log(f"serve: {R} requests, sum m={sum(r.m for r in reqs)}, arena {args.serve_arena_gb} GiB")
    # saturation throughput: everything submitted at t=0
    lat0, wall0, res0 = _serve_pass(mh, reqs, arena, args.serve_slots, np.zeros(R))
    sat = R / wall0
    # parity: small requests against the oracle, any size against the plain path
    rng = np.random.default_rng(1)
    smalls = [i for i in range(R) if reqs[i].m <= 40000]
    for i in rng.choice(smalls, size=min(6, len(smalls)), replace=False):
        if not same(res0[i], oracle.run(reqs[i])):
            raise RuntimeError(f"served parity failure on {reqs[i].name}")
    for i in rng.choice(R, size=min(4, R), replace=False):
        if not same(res0[i], mh.reduce(reqs[i])):
            raise RuntimeError(f"served != plain on {reqs[i].name}")
    out = {
        "workload": f"{R} requests, n=round(100*300^u), m=round(500*600^u), u~U(0,1), interval/uniform 50/50, f in {{1,2,3}}",
        "arena_gib": args.serve_arena_gb,
        "saturation_kernelizations_per_s": sat,
        "saturation_p50_ms": pct(lat0, 50),
        "saturation_p99_ms": pct(lat0, 99),
        "rates": [],
    }
    for frac in (0.5, 0.8):
        lam = frac * sat
        arr = np.cumsum(np.random.default_rng(2).exponential(1.0 / lam, size=R))
        arr -= arr[0]
        lat, wall, res = _serve_pass(mh, reqs, arena, args.serve_slots, arr)
        for i in rng.choice(R, size=min(4, R), replace=False):
            if not same(res[i], res0[i]):
                raise RuntimeError("served result differs between passes")
        out["rates"].append({"lambda_per_s": lam, "fraction_of_saturation": frac,
                             "throughput_per_s": R / wall, "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99)})
        log(f"serve lambda={lam:.1f}/s: p50 {pct(lat, 50):.1f} ms p99 {pct(lat, 99):.1f} ms")
    return out


if __name__ == "__main__":
    main()
