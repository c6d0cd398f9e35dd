"""Benchmark: kernelizations per second of the DP + MD reduction (Algorithm 3)
on one MI355X, batched against plain, with latency percentiles, the
roofline of the dominant kernel and the oracle on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--only SECTIONS]

One step = one batched kernelization of the 512-instance batch workload
(n ~ U{100..4000}, m = n U(5,10), interval or uniform hyperedges with
probability 1/2 each, f ~ U{1,2} capped at |e|): the instances' CSR arrays
are resident in HBM when the timed region starts; a step reduces every
instance to its fixpoint in shared launches and returns every result
(surviving ids and the per-round deletion trace) to host memory.
value = 512 K / elapsed.  Every timed configuration is first checked
bit-exact against the oracle (all 512 members).  Further sections: the
plain path on the transport, plain and multi-demand workloads, the
paper-shaped stand-ins, the served path, and the oracle and KernelCPU on
the host cores.  Prints ONE JSON line.
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

# published MI355X peaks, and the chip's unit counts for the vector paths
PEAK_INT8_OPS = 5.0e15            # dense int8 MFMA, ops/s
PEAK_HBM = 8.0e12                 # bytes/s
CUS, CLOCK = 256, 2.4e9
PEAK_VALU_I32 = CUS * 4 * 16 * CLOCK    # int32 vector lane-ops/s (4 SIMD x 16 lanes per CU per clock)
PEAK_LDS_ATOMIC = CUS * 32 * CLOCK      # LDS lane-atomics/s (32 banks per CU, one access each per clock)
SECTIONS = ("batch", "transport", "plain", "multidemand", "paper", "serve", "cpu")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed batched kernelizations of the 512-instance batch")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--only", default=",".join(SECTIONS), help="comma list of " + ",".join(SECTIONS))
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--plain-steps", type=int, default=50)
    ap.add_argument("--md-reps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-arena-gb", type=int, default=96)
    ap.add_argument("--serve-slots", type=int, default=256)
    ap.add_argument("--parity", choices=("all", "sample"), default="all",
                    help="batch parity: every member against the oracle on the host cores, or 16 in-process "
                         "(profiler runs: no worker processes)")
    ap.add_argument("--md-variants", default="int8,int8_direct_loads,bitset,sparse")
    ap.add_argument("--flags", type=lambda x: int(x, 0), default=None,
                    help="batch schedule flags (skips the autotuner)")
    ap.add_argument("--lean", action="store_true",
                    help="profiler runs: only the timed loops (no other schedules, host inputs, plain same mix, "
                         "event-profiled runs)")
    ap.add_argument("--batch-profiled-only", action="store_true",
                    help="profiler runs: only the event-profiled batch leg the roofline comes from (the sparse "
                         "and dense branches in order, a bounded delay before each round)")
    ap.add_argument("--kernelcpu-transport", action="store_true",
                    help="also time KernelCPU on the full transport instance (minutes on one core)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (HBM counter calibration)")
    return ap.parse_args()


def host_info():
    model, mhz = "", None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name") and not model:
                model = line.split(":", 1)[1].strip()
            if line.startswith("cpu MHz") and mhz is None:
                mhz = float(line.split(":", 1)[1])
    except OSError:
        pass
    return {"cpu_model": model, "cpu_mhz": mhz, "nproc": os.cpu_count(),
            "affinity_cores": len(os.sched_getaffinity(0))}


def committed_traffic(kernel, tag):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary, or None when there is none or the kernel source changed since
    the counters were taken."""
    import hashlib
    src = os.path.join(ROOT, "paper_2109_06042_amd", "csrc", "kernels.hip")
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{tag}.txt")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    # one line per template instance: "traffic <name> sha=<h> bytes_per_launch=<b> [dispatches=<d>]";
    # instances are weighted by their dispatch counts
    num = den = 0.0
    for line in open(path):
        f = line.split()
        if len(f) in (4, 5) and f[0] == "traffic" and f[1].split("<")[0] == kernel and f[2] == f"sha={sha}":
            w = float(f[4].split("=")[1]) if len(f) == 5 else 1.0
            num += w * float(f[3].split("=")[1])
            den += w
    return num / den if den else None


def dense_kernel(flags):
    """Name of the int8 contraction kernel a flag word selects (its operand
    staging, MHS_GEMM_SCHED k: 0 LDS via registers, 1 direct loads, 2
    asynchronous copies; none asked: the library default, LDS)."""
    k = ((flags >> 20) & 3) - 1
    return {1: "k_gemm", 2: "k_gemm_async"}.get(k, "k_gemm_lds")


def same(a, b):
    return a.rounds == b.rounds and np.array_equal(a.death_e, b.death_e) and np.array_equal(a.death_v, b.death_v)


def pct(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


# ----------------------------------------------------------- host workers
def cpu_workers():
    # one GPU's share of the machine's host cores is 16, whatever nproc shows
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _cpu_pool(P):
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    # spawned workers import numpy, the generators and the oracle only: never the GPU
    return ProcessPoolExecutor(max_workers=P, mp_context=mp.get_context("spawn"))


def _oracle_members(w, P, count):
    """Oracle over batch members w, w + P, ... < count, each generated
    before its timer starts; returns ([(idx, rounds, death_e, death_v)],
    oracle seconds)."""
    import mhsgen
    import oracle
    out, busy = [], 0.0
    for i in range(w, count, P):
        inst = mhsgen.batch_member(seed=0, idx=i)
        t = time.perf_counter()
        r = oracle.run(inst)
        busy += time.perf_counter() - t
        out.append((i, r.rounds, r.death_e, r.death_v))
    return out, busy


class _Ref:
    def __init__(self, rounds, de, dv):
        self.rounds, self.death_e, self.death_v = rounds, de, dv


def oracle_all_members(count):
    """The oracle on every batch member, on the host's cores at once: the
    parity reference and the all-core CPU throughput on the full workload."""
    P = cpu_workers()
    t = time.perf_counter()
    with _cpu_pool(P) as ex:
        parts = list(ex.map(_oracle_members, range(P), [P] * P, [count] * P))
    wall = time.perf_counter() - t
    refs = [None] * count
    for part, _ in parts:
        for i, r, de, dv in part:
            refs[i] = _Ref(r, de, dv)
    busy = max(b for _, b in parts)
    return refs, {"kernelizations_per_s": count / busy, "cores": P, "kind": "oracle",
                  "sample": f"all {count} batch members on {P} processes (the box's host-core share for one "
                            f"GPU), {busy:.1f} s of oracle time on the busiest, {wall:.1f} s wall with generation",
                  **host_info()}


def _pinned_leg(kind, family, kw, seconds, core, max_items=None):
    """One core (sched_setaffinity to `core`): the oracle or KernelCPU over
    instances idx = 0, 1, ... of a family until `seconds` of reduction time
    are spent; generation is outside the timer."""
    import mhsgen
    import oracle
    os.sched_setaffinity(0, {core})
    fn = oracle.run if kind == "oracle" else oracle.kernelcpu
    n, busy, i = 0, 0.0, 0
    while busy < seconds and (max_items is None or n < max_items):
        inst = mhsgen.make(family, seed=0, idx=i, **kw)
        t = time.perf_counter()
        fn(inst)
        busy += time.perf_counter() - t
        n += 1
        i += 1
    return n, busy


def pinned(kind, family, kw, seconds, max_items=None):
    core = sorted(os.sched_getaffinity(0))[0]
    with _cpu_pool(1) as ex:
        return ex.submit(_pinned_leg, kind, family, kw, seconds, core, max_items).result()


def all_cores(kind, family, kw, seconds):
    P = cpu_workers()
    cores = sorted(os.sched_getaffinity(0))
    with _cpu_pool(P) as ex:
        res = list(ex.map(_strided_leg, [kind] * P, [family] * P, [kw] * P, [seconds] * P, range(P), [P] * P,
                          cores[:P]))
    n = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    return n, busy, P


def _strided_leg(kind, family, kw, seconds, w, P, core):
    import mhsgen
    import oracle
    os.sched_setaffinity(0, {core})
    fn = oracle.run if kind == "oracle" else oracle.kernelcpu
    n, busy, i = 0, 0.0, w
    while busy < seconds:
        inst = mhsgen.make(family, seed=0, idx=i, **kw)
        t = time.perf_counter()
        fn(inst)
        busy += time.perf_counter() - t
        n += 1
        i += P
    return n, busy


# ------------------------------------------------------------- sections
def profile_set(mh, run):
    """Median profiled statistics of a reduction (per-step HIP events on the
    stream the kernels run on; a bounded device delay before every round
    lets the host enqueue it, so its kernels run back to back)."""
    profs = [run() for _ in range(3)]
    return {k: float(np.median([p[k] for p in profs])) for k in profs[0]}


def bench_batch(mh, torch, mhsgen, oracle, args, out):
    count = args.batch_count
    insts = mhsgen.batch(count)
    sum_m, sum_n = sum(i.m for i in insts), sum(i.n for i in insts)
    log(f"batch: {count} instances, sum m={sum_m}, sum n={sum_n}, sum nnz={sum(i.nnz for i in insts)}")
    if args.parity == "all":
        refs, all_core = oracle_all_members(count)
        checked = list(range(count))
    else:
        checked = list(np.random.default_rng(0).choice(count, size=min(16, count), replace=False))
        refs = [None] * count
        for i in checked:
            refs[i] = oracle.run(insts[i])
        all_core = None
    dev = [mh.DeviceInstance(i) for i in insts]
    torch.cuda.synchronize()
    ws = torch.empty(mh.batch_workspace_bytes(dev), dtype=torch.uint8, device="cuda")
    log(f"batch workspace {ws.numel() / 2**30:.2f} GiB")
    # schedule autotuner on the batch itself, its arrays resident in HBM as
    # in the timed loop (untimed: the tuning is not part of a step)
    t = time.perf_counter()
    if args.flags is None:
        rep = mh.tune(dev, workspace=ws)
        flags = rep["best_flags"]
        log(f"autotune: flags {flags:#x} ({rep['best_ms']:.1f} ms vs int8 {rep['default_ms']:.1f} ms on the batch)")
    else:
        flags = args.flags
    tune_s = time.perf_counter() - t

    def check(res, what):
        for i in checked:
            if not same(res[i], refs[i]):
                raise SystemExit(f"PARITY FAILURE ({what}) on {insts[i].name}")

    # the dominant kernel: per-step event times of a profiled batch
    def prof_run(what=None):
        res = mh.reduce_batch(dev, flags=flags | mh.MHS_PROFILE, workspace=ws)
        if what:
            check(res, what)
        st = dict(res[0].stats)
        st["terms"] = float(sum(x.stats["terms"] for x in res))
        st["issued_ops"] = float(sum(x.stats["issued_ops"] for x in res))
        # the set runs rounds until its last member is done
        st["iterations"] = float(max(x.stats["iterations"] for x in res))
        return st
    if args.batch_profiled_only:
        # every batch launch of this run is a profiled one (parity checked on
        # the first one's results)
        prof_run("batched, profiled")
        log(f"parity ok: {len(checked)} members against the oracle")
        st = profile_set(mh, prof_run)
        log(f"profiled batch: sparse counting {st['sparse_ms']:.2f} ms, contraction {st['gemm_ms'] - st['sparse_ms']:.2f}"
            f" ms per step, {st['terms']:.4g} terms")
        out.update({"value": None, "config": {"workload": f"batch: {count} instances (profiled leg only)",
                                              "schedule": hex(flags)}, "profiled": st})
        return

    first = mh.reduce_batch(dev, flags=flags, workspace=ws)
    check(first, "batched, tuned schedule")
    log(f"parity ok: {len(checked)} members against the oracle")
    for _ in range(args.warmup):
        mh.reduce_batch(dev, flags=flags, workspace=ws)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s = time.perf_counter()
        last = mh.reduce_batch(dev, flags=flags, workspace=ws)
        lat.append((time.perf_counter() - s) * 1e3)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for i in range(count):
        if not same(last[i], first[i]):
            raise SystemExit(f"timed batch differs from the checked one on {insts[i].name}")
    value = count * args.steps / el
    log(f"batched: {value:.1f} kernelizations/s, {el / args.steps * 1e3:.2f} ms per batch")
    if args.lean:
        out.update({"value": value, "ms_per_step": el / args.steps * 1e3,
                    "config": {"workload": f"batch: {count} instances (lean profiler run)", "schedule": hex(flags)},
                    "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)}})
        return

    # other schedules on the same device-resident batch (context)
    sched = {}
    for name, f in (("hybrid_default", mh.MHS_VARIANT_HYBRID), ("int8_all", mh.MHS_VARIANT_INT8)):
        r = mh.reduce_batch(dev, flags=f, workspace=ws)
        check(r, name)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(2):
            mh.reduce_batch(dev, flags=f, workspace=ws)
        torch.cuda.synchronize()
        sched[name] = count * 2 / (time.perf_counter() - t)
    # host inputs (PCIe-inclusive, for reference)
    r = mh.reduce_batch(insts, flags=flags)
    check(r, "host inputs")
    t = time.perf_counter()
    for _ in range(3):
        mh.reduce_batch(insts, flags=flags)
    host_rate = count * 3 / (time.perf_counter() - t)
    # plain path on the same mix: every member, one call each
    pws = torch.empty(max(mh.workspace_bytes(i.n, i.m, i.nnz, mh.MHS_INPUT_DEVICE) for i in insts),
                      dtype=torch.uint8, device="cuda")
    plain_lat = []
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i, d in enumerate(dev):
        s = time.perf_counter()
        r = mh.reduce(d, workspace=pws)
        plain_lat.append((time.perf_counter() - s) * 1e3)
        if not same(r, first[i]):
            raise SystemExit(f"plain path differs from the batched one on {insts[i].name}")
    plain_el = time.perf_counter() - t
    del pws

    st = profile_set(mh, prof_run)
    rounds = max(int(st["iterations"]), 1)
    steps_ms = {"k_sp_count (sparse counting)": st["sparse_ms"],
                f"{dense_kernel(flags)} (int8 MFMA contraction)": st["gemm_ms"] - st["sparse_ms"],
                "rows / encode": st["rows_ms"], "k_compact": st["compact_ms"], "round end": st["round_end_ms"]}
    log("batch event time per step (ms): " + ", ".join(f"{k} {v:.2f}" for k, v in steps_ms.items()))
    sp_launches = 2 * rounds
    sp_rate = st["terms"] / (st["sparse_ms"] * 1e-3) if st["sparse_ms"] > 0 else 0.0
    roof_sp = {"kernel": "k_sp_count (sparse counting: one LDS hash insert per nonzero product term)",
               "bound": "alu", "achieved": sp_rate / 1e12, "peak": PEAK_LDS_ATOMIC / 1e12, "unit": "Tops/s",
               "frac": sp_rate / PEAK_LDS_ATOMIC, "traffic": committed_traffic("k_sp_count", "batch"),
               "op": "product term (LDS hash insert)", "terms_per_step": st["terms"],
               "terms_per_launch": st["terms"] / sp_launches, "us_per_launch": st["sparse_ms"] * 1e3 / sp_launches,
               "launches_per_step": sp_launches}
    dense_ms = st["gemm_ms"] - st["sparse_ms"]
    dn_rate = st["issued_ops"] / (dense_ms * 1e-3) if dense_ms > 0 else 0.0
    roof_dn = {"kernel": f"{dense_kernel(flags)} (int8 MFMA contraction + DP/MD test)", "bound": "mfma",
               "achieved": dn_rate / 1e12, "peak": PEAK_INT8_OPS / 1e12, "unit": "TOPS",
               "frac": dn_rate / PEAK_INT8_OPS, "traffic": committed_traffic(dense_kernel(flags), "batch"),
               "ops_per_step": st["issued_ops"], "us_per_launch": dense_ms * 1e3 / (2 * rounds),
               "launches_per_step": 2 * rounds}
    dominant = max(steps_ms, key=steps_ms.get)
    out.update({
        "value": value,
        "ms_per_step": el / args.steps * 1e3,
        "config": {"workload": f"batch: {count} instances, n~U{{100..4000}}, m=round(n*U(5,10)), interval or "
                               f"uniform hyperedges (1/2 each), f~U{{1,2}} capped at |e|, seed 0; CSR resident "
                               f"in HBM; results (survivors, per-round trace) returned to host memory",
                   "instances": count, "sum_m": sum_m, "sum_n": sum_n,
                   "schedule": f"autotuned flags {flags:#x}", "rounds_max": int(max(r.rounds for r in first))},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99),
                       "note": "batch latency: every result of a step arrives when the step ends"},
        "roofline": roof_sp if dominant.startswith("k_sp_count") else roof_dn,
    })
    out["batched"] = {
        "kernelizations_per_s": value, "batch_ms": el / args.steps * 1e3, "hyperedges_per_s": sum_m * value / count,
        "tuned_flags": hex(flags), "tune_s": tune_s, "schedules_kernelizations_per_s": sched,
        "host_input_kernelizations_per_s": host_rate,
        "plain_same_mix": {"kernelizations_per_s": count / plain_el, "p50_ms": pct(plain_lat, 50),
                           "p99_ms": pct(plain_lat, 99)},
        "oracle_checked": len(checked), "oracle_all_cores": all_core,
        "step_event_ms": steps_ms, "dominant_by_event_time": dominant,
        "roofline_sparse": roof_sp, "roofline_dense": roof_dn,
    }
    del ws


def bench_transport(mh, torch, mhsgen, oracle, args, out):
    inst = mhsgen.transport(seed=0)
    t = time.time()
    ref = oracle.run(inst)
    log(f"transport {inst.name}: nnz={inst.nnz}, oracle {time.time() - t:.1f} s")
    dev = mh.DeviceInstance(inst)
    ws = torch.empty(mh.workspace_bytes(inst.n, inst.m, inst.nnz, mh.MHS_INPUT_DEVICE), dtype=torch.uint8,
                     device="cuda")
    if not same(mh.reduce(dev, workspace=ws), ref):
        raise SystemExit("PARITY FAILURE on the transport workload")
    for _ in range(5):
        mh.reduce(dev, workspace=ws)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.plain_steps):
        s = time.perf_counter()
        r = mh.reduce(dev, workspace=ws)
        lat.append((time.perf_counter() - s) * 1e3)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if not same(r, ref):
        raise SystemExit("PARITY FAILURE in the timed transport loop")
    if args.lean:
        out["transport_plain"] = {"kernelizations_per_s": args.plain_steps / el, "p50_ms": pct(lat, 50)}
        log(f"transport plain: {args.plain_steps / el:.1f}/s, {el / args.plain_steps * 1e3:.3f} ms")
        return
    hws = torch.empty(mh.workspace_bytes(inst.n, inst.m, inst.nnz, 0), dtype=torch.uint8, device="cuda")
    mh.reduce(inst, workspace=hws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(10):
        mh.reduce(inst, workspace=hws)
    host_rate = 10 / (time.perf_counter() - t1)
    del hws
    st = profile_set(mh, lambda: dict(mh.reduce(dev, flags=mh.MHS_PROFILE, workspace=ws).stats))
    launches = max(int(st["gemm_launches"]), 1)
    gemm_ms = st["gemm_ms"] / launches
    gemm_rate = st["issued_ops"] / launches / (gemm_ms * 1e-3) if gemm_ms > 0 else 0.0
    rows_ms = st["rows_ms"] / launches
    rows_rate = st["encode_bytes"] / launches / (rows_ms * 1e-3) if rows_ms > 0 else 0.0
    out["transport_plain"] = {
        "workload": "transport: n=8000 vertices on a line, m=60000 interval hyperedges (length U{5..40}, members "
                    "kept p=0.8), f=1, seed 0, CSR resident in HBM; plain path, one instance per call",
        "kernelizations_per_s": args.plain_steps / el, "ms": el / args.plain_steps * 1e3,
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "rounds": int(ref.rounds),
        "host_input_kernelizations_per_s": host_rate,
        "step_event_ms": {"k_rows_encode": st["rows_ms"], "k_gemm_lds": st["gemm_ms"],
                          "k_compact": st["compact_ms"], "k_round_end": st["round_end_ms"]},
        "roofline_gemm": {"kernel": "k_gemm_lds (fused int8 MFMA contraction + DP/MD test)", "bound": "mfma",
                          "achieved": gemm_rate / 1e12, "peak": PEAK_INT8_OPS / 1e12, "unit": "TOPS",
                          "frac": gemm_rate / PEAK_INT8_OPS,
                          "traffic": committed_traffic("k_gemm_lds", "transport_plain"),
                          "ops_per_launch": st["issued_ops"] / launches, "us_per_launch": gemm_ms * 1e3,
                          "launches_per_step": launches},
        "roofline_rows": {"kernel": "k_rows_encode (rows, windows, tile encoding)", "bound": "hbm",
                          "achieved": rows_rate / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                          "frac": rows_rate / PEAK_HBM,
                          "traffic": committed_traffic("k_rows_encode", "transport_plain"),
                          "bytes_per_launch": st["encode_bytes"] / launches, "us_per_launch": rows_ms * 1e3,
                          "launches_per_step": launches},
    }
    log(f"transport plain: {args.plain_steps / el:.1f}/s, {el / args.plain_steps * 1e3:.3f} ms; k_gemm "
        f"{gemm_ms * 1e3:.1f} us/launch {gemm_rate / 1e12:.1f} TOPS")
    del ws


def bench_plain_small(mh, torch, mhsgen, oracle, args, out):
    small = mhsgen.plain(seed=0)
    sref = oracle.run(small)
    sdev = mh.DeviceInstance(small)
    sws = torch.empty(mh.workspace_bytes(small.n, small.m, small.nnz, mh.MHS_INPUT_DEVICE), dtype=torch.uint8,
                      device="cuda")
    ent = {"workload": "plain: n=200, m=1000, |e|~U{2..8} uniform members, f=1, seed 0", "rounds": int(sref.rounds)}
    for name, f in (("default", 0), ("int8", mh.MHS_VARIANT_INT8)):
        if not same(mh.reduce(sdev, flags=f, workspace=sws), sref):
            raise SystemExit(f"PARITY FAILURE on the plain workload ({name})")
        for _ in range(3):
            mh.reduce(sdev, flags=f, workspace=sws)
        slat = []
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(200):
            s0 = time.perf_counter()
            mh.reduce(sdev, flags=f, workspace=sws)
            slat.append((time.perf_counter() - s0) * 1e3)
        sel = time.perf_counter() - t
        ent[name] = {"kernelizations_per_s": 200 / sel, "p50_ms": pct(slat, 50), "p99_ms": pct(slat, 99)}
    out["plain_small"] = ent
    log(f"plain small: {ent['default']['kernelizations_per_s']:.1f}/s")


def product_terms(inst, death_e, death_v, rounds):
    """Nonzero product terms of the two contractions over `rounds` executed
    rounds (each a shared incidence of a victim and a partner, the victim
    itself included), from a result's death rounds: round r's edge phase
    has, for every alive hyperedge, the degrees of its alive vertices among
    the hyperedges alive at the round's start; its vertex phase has, for
    every alive vertex that keeps a hyperedge after the round's edge
    deletions, the sizes of the hyperedges it keeps."""
    ep = np.asarray(inst.edge_ptr, np.int64)
    ev = np.asarray(inst.edge_vtx, np.int64)
    de, dv = np.asarray(death_e), np.asarray(death_v)
    sizes = np.diff(ep)
    eid = np.repeat(np.arange(inst.m), sizes)
    total = 0
    for r in range(1, rounds + 1):
        ae = (de == 0) | (de >= r)
        av = (dv == 0) | (dv >= r)
        deg = np.bincount(ev[ae[eid]], minlength=inst.n)
        total += int(deg[ev[ae[eid] & av[ev]]].sum())
        kept = ((de == 0) | (de > r))[eid]
        d2 = np.bincount(ev[kept], minlength=inst.n)
        w = np.bincount(ev[kept], weights=sizes[eid[kept]], minlength=inst.n)
        total += int(w[av & (d2 > 0)].sum())
    return total


def bench_multidemand(mh, torch, mhsgen, oracle, args, out):
    inst = mhsgen.multidemand(seed=0)
    t = time.time()
    ref = oracle.run(inst)
    oracle_s = time.time() - t
    log(f"multidemand {inst.name}: nnz={inst.nnz}; oracle {oracle_s:.1f} s")
    dev = mh.DeviceInstance(inst)
    ws = torch.empty(mh.workspace_bytes(inst.n, inst.m, inst.nnz, mh.MHS_INPUT_DEVICE), dtype=torch.uint8,
                     device="cuda")
    ent_all = {"workload": "multidemand: n=20000, m=200000, |e| power law 2.2 on [2,200], f~U{1,2,3} capped, "
                           "seed 0, CSR resident in HBM", "rounds": int(ref.rounds), "oracle_s": oracle_s}
    variants = {"int8": (mh.MHS_VARIANT_INT8, "lds"), "int8_direct_loads": (mh.MHS_VARIANT_INT8, "direct"),
                "bitset": (mh.MHS_VARIANT_BITSET, "lds"), "sparse": (mh.MHS_VARIANT_SPARSE, "lds")}
    nonzero = None
    for name in args.md_variants.split(","):
        flag, env = variants[name]
        os.environ["MHSK_GEMM"] = env
        r0 = mh.reduce(dev, flags=flag, workspace=ws)
        if not same(r0, ref):
            raise SystemExit(f"PARITY FAILURE on the multidemand workload ({name})")
        if nonzero is None and not args.lean:
            nonzero = product_terms(inst, r0.death_e, r0.death_v, int(r0.stats["iterations"]))
            ent_all["nonzero_product_terms"] = nonzero
        times = []
        for _ in range(args.md_reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            mh.reduce(dev, flags=flag, workspace=ws)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
        el = float(np.median(times))
        if args.lean:
            ent_all[name] = {"ms": el * 1e3}
            log(f"multidemand {name}: {el * 1e3:.1f} ms")
            continue
        p = mh.reduce(dev, flags=flag | mh.MHS_PROFILE, workspace=ws).stats
        launches = max(p["gemm_launches"], 1)
        ent = {"kernelizations_per_s": 1.0 / el, "ms": el * 1e3, "ms_reps": [x * 1e3 for x in times],
               "gemm_ms": p["gemm_ms"], "edge_gemm_ms": p["edge_gemm_ms"], "vertex_gemm_ms": p["vertex_gemm_ms"],
               "gemm_launches": launches}
        if name.startswith("int8"):
            rate = p["issued_ops"] / (p["gemm_ms"] * 1e-3)
            ent.update({"issued_ops": p["issued_ops"], "contraction_rate_tops": rate / 1e12,
                        "frac_of_int8_peak": rate / PEAK_INT8_OPS})
        elif name == "bitset":
            # 65,536 int32 vector ops per (tile pair, 64-column chunk): 128 x 128 pairs x (2 AND + 2 popcount)
            # on 32-bit words, i.e. the dense-equivalent int8 count / 32
            valu = p["issued_ops"] / 32.0
            ent.update({"valu_int32_ops": valu, "valu_rate_tops": valu / (p["gemm_ms"] * 1e-3) / 1e12,
                        "frac_of_valu_peak": valu / (p["gemm_ms"] * 1e-3) / PEAK_VALU_I32})
        else:
            # the terms the count walks (round 1 skips partners of higher slack class than the victim's)
            ent.update({"terms_walked": p["terms"], "terms_rate_tops": p["terms"] / (p["gemm_ms"] * 1e-3) / 1e12,
                        "frac_of_lds_atomic_peak": p["terms"] / (p["gemm_ms"] * 1e-3) / PEAK_LDS_ATOMIC})
        ent_all[name] = ent
        log(f"multidemand {name}: {el * 1e3:.1f} ms, contraction {p['gemm_ms']:.1f} ms")
    os.environ.pop("MHSK_GEMM", None)
    if nonzero:
        for name in ("int8", "int8_direct_loads"):
            if name in ent_all:
                # the nonzero product terms beside the dense operations the int8 path issues
                ent_all[name]["nonzero_terms"] = nonzero
                ent_all[name]["dense_ops_per_nonzero_term"] = ent_all[name]["issued_ops"] / nonzero
    out["multidemand"] = ent_all
    del ws


def bench_paper_shaped(mh, torch, mhsgen, oracle, args, out):
    res = {"note": "stand-ins with the paper's aspect ratio (vertices far outnumber hyperedges): "
                   "NCI60-shaped n=7124, m=152 and GIRG-shaped n=15015, m=1903; plain path, CSR in HBM"}
    cases = [("nci60_shaped", a, mhsgen.nci60_shaped(seed=0, alpha=a)) for a in (1, 5, 20, 60)]
    cases += [("girg_shaped", a, mhsgen.girg_shaped(seed=0, alpha=a)) for a in (1, 5, 10, 30)]
    for fam, a, inst in cases:
        ref = oracle.run(inst)
        dev = mh.DeviceInstance(inst)
        ws = torch.empty(mh.workspace_bytes(inst.n, inst.m, inst.nnz, mh.MHS_INPUT_DEVICE), dtype=torch.uint8,
                         device="cuda")
        if not same(mh.reduce(dev, workspace=ws), ref):
            raise SystemExit(f"PARITY FAILURE on {inst.name}")
        lat = []
        torch.cuda.synchronize()
        for _ in range(30):
            s = time.perf_counter()
            mh.reduce(dev, workspace=ws)
            lat.append((time.perf_counter() - s) * 1e3)
        p = mh.reduce(dev, flags=mh.MHS_PROFILE, workspace=ws).stats
        t = time.perf_counter()
        oracle.run(inst)
        res[f"{fam}_alpha{a}"] = {"n": inst.n, "m": inst.m, "nnz": inst.nnz, "rounds": int(ref.rounds),
                                  "kept_v": int(len(ref.kept_v)), "kept_e": int(len(ref.kept_e)),
                                  "kernelizations_per_s": 1e3 / pct(lat, 50), "p50_ms": pct(lat, 50),
                                  "p99_ms": pct(lat, 99), "edge_gemm_ms": p["edge_gemm_ms"],
                                  "vertex_gemm_ms": p["vertex_gemm_ms"],
                                  "oracle_one_core_s": time.perf_counter() - t}
        del ws
    out["paper_shaped"] = res
    log("paper-shaped: " + ", ".join(f"{k} {v['p50_ms']:.3f} ms" for k, v in res.items() if k != "note"))


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
        got = srv.poll()
        if not got and nxt < n and srv.pending() == (0, 0):
            time.sleep(max(0.0, min(0.001, arrivals[nxt] - now)))
        for rid, r in got:
            if isinstance(r, Exception):
                raise r
            done[rid] = r
            lat[rid] = (time.perf_counter() - t0 - arrivals[rid]) * 1e3
    wall = time.perf_counter() - t0
    srv.close()
    return lat, wall, done


def _gen_requests(lo, hi):
    import mhsgen
    return [mhsgen.serve_request(seed=0, idx=i) for i in range(lo, hi)]


def bench_serve(mh, torch, mhsgen, oracle, args, out):
    R = args.serve_requests
    P = cpu_workers()
    step = (R + P - 1) // P
    with _cpu_pool(P) as ex:
        parts = list(ex.map(_gen_requests, range(0, R, step), [min(R, i + step) for i in range(0, R, step)]))
    reqs = [r for part in parts for r in part]
    arena = args.serve_arena_gb << 30
    sum_m = sum(r.m for r in reqs)
    log(f"serve: {R} requests, sum m={sum_m}, arena {args.serve_arena_gb} GiB")
    # saturation throughput: everything submitted at t=0
    lat0, wall0, res0 = _serve_pass(mh, reqs, arena, args.serve_slots, np.zeros(R))
    sat = R / wall0
    rng = np.random.default_rng(1)
    smalls = [i for i in range(R) if reqs[i].m <= 40000]
    for i in rng.choice(smalls, size=min(6, len(smalls)), replace=False):
        if not same(res0[i], oracle.run(reqs[i])):
            raise SystemExit(f"served parity failure on {reqs[i].name}")
    for i in rng.choice(R, size=min(4, R), replace=False):
        if not same(res0[i], mh.reduce(reqs[i])):
            raise SystemExit(f"served != plain on {reqs[i].name}")
    ent = {"workload": f"{R} requests, n=round(100*300^u), m=round(500*600^u), u~U(0,1), interval/uniform 50/50, "
                       f"f in {{1,2,3}}, host inputs",
           "arena_gib": args.serve_arena_gb, "slots": args.serve_slots,
           "saturation_kernelizations_per_s": sat, "saturation_hyperedges_per_s": sum_m / wall0,
           "saturation_p50_ms": pct(lat0, 50), "saturation_p99_ms": pct(lat0, 99), "rates": []}
    for frac in (0.5, 0.8):
        lam = frac * sat
        arr = np.cumsum(np.random.default_rng(2).exponential(1.0 / lam, size=R))
        arr -= arr[0]
        lat, wall, res = _serve_pass(mh, reqs, arena, args.serve_slots, arr)
        for i in rng.choice(R, size=min(8, R), replace=False):
            if not same(res[i], res0[i]):
                raise SystemExit("served result differs between passes")
        ent["rates"].append({"lambda_per_s": lam, "fraction_of_saturation": frac, "throughput_per_s": R / wall,
                             "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99)})
        log(f"serve lambda={lam:.1f}/s: p50 {pct(lat, 50):.1f} ms p99 {pct(lat, 99):.1f} ms")
    out["served"] = ent


def bench_cpu(args, out):
    """The oracle on one pinned core over the headline workload's members
    (generation outside the timer), KernelCPU (Algorithms 4-6, the paper's
    serial reduction) beside it, one core and all cores."""
    hi = host_info()
    n, busy = pinned("oracle", "batch", {}, args.cpu_seconds)
    out["cpu_baseline"] = {
        "value": n / busy, "unit": "kernelizations/s", "cores": 1, "kind": "oracle",
        "sample": f"batch members 0..{n - 1} of the headline workload, pruned-candidate oracle on one pinned core "
                  f"(sched_setaffinity), {busy:.1f} s of reduction time (generation excluded)", **hi}
    kc = {}
    for fam, kw, label in (("plain", {}, "plain n=200 m=1000"),
                           ("batch", {"nmax": 600}, "batch mix truncated to n<=600 (full members take 10-40 s each)")):
        secs = min(args.cpu_seconds, 4.0)
        on, ob = pinned("oracle", fam, kw, secs)
        kn, kb = pinned("kernelcpu", fam, kw, secs)
        an, ab, P = all_cores("kernelcpu", fam, kw, secs)
        kc[fam] = {"workload": label, "oracle_one_core_per_s": on / ob, "kernelcpu_one_core_per_s": kn / kb,
                   "kernelcpu_all_cores_per_s": an / ab, "all_cores": P,
                   "samples": {"oracle": on, "kernelcpu": kn, "kernelcpu_all_cores": an}}
    if args.kernelcpu_transport:
        kn, kb = pinned("kernelcpu", "transport", {}, 1.0, max_items=1)
        on, ob = pinned("oracle", "transport", {}, 1.0, max_items=1)
        kc["transport"] = {"workload": "transport n=8000 m=60000", "kernelcpu_one_core_s": kb, "oracle_one_core_s": ob}
    out["kernelcpu"] = kc
    log(f"cpu: oracle one core {n / busy:.1f}/s on batch members")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
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

    only = set(args.only.split(","))
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    lib = mh._lib.load()       # refuses a library built from other sources than the tree's
    version = lib.mhs_version().decode()
    log(version)
    out = {
        "metric": "kernelizations/sec + p50/p99 latency, batched vs plain, bit-exact to oracle",
        "value": None, "unit": "kernelizations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int8",
        "data": "synthetic", "config": None, "library": version,
    }
    sections = [("batch", bench_batch), ("transport", bench_transport), ("plain", bench_plain_small),
                ("multidemand", bench_multidemand), ("paper", bench_paper_shaped), ("serve", bench_serve)]
    for name, fn in sections:
        if name not in only:
            continue
        if name == "batch":
            fn(mh, torch, mhsgen, oracle, args, out)   # the headline: a failure ends the run
            continue
        try:
            fn(mh, torch, mhsgen, oracle, args, out)
        except SystemExit:
            raise
        except Exception as e:  # report, keep the main line
            log(f"{name} section failed: {e!r}")
            out[name] = {"error": repr(e)}
    if "cpu" in only:
        bench_cpu(args, out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
