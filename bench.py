#!/usr/bin/env python3
"""Throughput of filter -> sort-based equi-join -> group-by (+ top-100) on one MI355X.

Workload (default): the 60M-row fact table joined to the 15M-row mid table,
date < 2400, group by custkey (about 1.5M groups), exact int64 sum and count,
then ORDER BY sum DESC, custkey ASC LIMIT 100.  Inputs are seeded synthetic
columns (the generator in datagen/), resident in HBM before timing starts.

A step is one whole fragment: the filter, both key sorts, the join, the
group-key sort, the bucket aggregation and the top-100, launched on the
caller's stream (the mid-side sort on a forked side stream).  W untimed
warm-up steps, then exactly K timed steps between two events after a device
synchronisation; value = fact rows / second.

Then the same K steps run again with the library's per-launch profiler on
(HIP events recorded on the launch stream around every kernel): the roofline
figure uses the dominant kernel family's measured durations and its
algorithmic bytes (what the kernel must read and write), from the actual row
counts; ms_per_step_profiled is that run's step time.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fact rows/s filter→join→group-by (% of HBM peak); p50/p99 fragment latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(plan, N, n_f, M, J, G, PB):
    """Bytes per step each kernel family must read and write in this design, summed over its
    launches in one step (the row counts are the actual ones; PB is the revenue payload width in
    bytes, 8 or 4)."""
    R = 4 + PB                                                # a (key, revenue) row
    return {
        "radix_hist": 8 * N + N // 8 + 4 * M,                 # fact fk+date in, predicate bits out; mid pk
        "fact_pass_fused": 20 * N + N // 8 + R * n_f,         # fk, price, disc, predicate bit per row; key+revenue per kept row
        "fact_pass": 2 * R * n_f * (plan["fact_passes"] - 1),
        "mid_pass_first": 16 * M,                             # pk, custkey in; key+custkey out
        "mid_pass": 16 * M * (plan["mid_passes"] - 1),
        "finish_sort": 16 * M,                                # mid (key, custkey) in and out
        "join_count": 4 * n_f + 4 * M,                        # sorted fact keys, mid keys
        "join_keyval": R * n_f + 8 * M + R * J,               # sorted fact pairs, mid keys+custkey; (custkey, revenue) out
        "group_pass": 2 * R * J * plan["group_passes"],
        "bucket_agg": R * J + 20 * G,
        "topk_filter": 12 * G,
    }


def launch_bytes(plan, N, n_f, M, J, G, PB):
    """Algorithmic bytes of each launch of the kernel families the roofline may describe."""
    R = 4 + PB
    return {
        "fact_pass_fused": [20 * N + N // 8 + R * n_f],
        "fact_pass": [2 * R * n_f] * (plan["fact_passes"] - 1),
        "group_pass": [2 * R * J] * plan["group_passes"],
        "join_keyval": [R * n_f + 8 * M + R * J],
        "bucket_agg": [R * J + 20 * G],
    }


def roofline_families(PB):
    """Kernel families the roofline may describe: the kernel (as the profiler names it, shortened)
    and the sources whose hash must match the committed counter summary for its traffic figure to
    be used."""
    v = "u64" if PB == 8 else "u32"
    a = "long" if PB == 8 else "u32"
    cfg = "RadixCfg<8,512,%d,8,16>" % (12 if PB == 8 else 16)      # 8-bit digits, 512 threads x 12 or 16 items
    radix = ("radix.hpp", "dev.hpp", "host.hpp")
    return {
        "fact_pass_fused": ("k_radix_pass<%s, SrcFilterRevenue<%s, true>, %s, 1>" % (cfg, v, v), radix),
        "fact_pass": ("k_radix_pass<%s, SrcPairs<%s>, %s, 1>" % (cfg, v, v), radix),
        "group_pass": ("k_radix_pass<%s, SrcPairs<%s>, %s, 3>" % (cfg, v, v), radix),
        "join_keyval": ("k_join<JoinCfg<256,8,2048>, %s, u32, EmitKeyVal<256,8,%s>, 0>" % (v, v),
                        ("join.hpp", "dev.hpp", "fragment.hpp")),
        "bucket_agg": ("k_bucket_agg<1024,8192,%s,0,false>" % a, ("segreduce.hpp", "dev.hpp")),
    }


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "cfg2_hbm_traffic.md")


def source_hash(files):
    import hashlib
    return hashlib.sha256(b"".join(open(os.path.join(ROOT, "paper_2203_01877_amd", "csrc", f), "rb").read()
                                   for f in files)).hexdigest()


def measured_traffic(family, files, PB):
    """HBM bytes per launch of a kernel family from the committed rocprofv3 counter summary, or None
    when the family's sources have changed since the counters were taken (or they were taken with
    another payload width)."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and not line.startswith(" "))
    if fields.get("revenue_bytes") != str(PB):
        return None
    if fields.get("source_sha256[%s]" % family) != source_hash(files):
        return None
    try:
        return int(fields["traffic_bytes_per_launch[%s]" % family])
    except (KeyError, ValueError):
        return None


def reference_model_bytes(N, n_f, M, J, G, P, Pm, Pg):
    """The sort-based method's reference pass structure (each pass reads its input and writes its
    output once; 8-bit digits), evaluated with the actual counts."""
    F1 = 8 * N + 8 * n_f
    F2 = 5 * M + 8 * M
    S1 = 4 * n_f + 16 * P * n_f
    S2 = 4 * M + 16 * Pm * M
    J1 = 4 * (n_f + M)
    J2 = 8 * (n_f + M) + 8 * J
    G1 = 8 * J + 20 * J + 12 * J
    A1 = 4 * J + 2 * Pg * 12 * J
    A2 = 12 * J + 28 * G
    T1 = 12 * G
    return F1 + F2 + S1 + S2 + J1 + J2 + G1 + A1 + A2 + T1


def host_cpu():
    """Model name of the host CPU and the number of cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0)), os.cpu_count()


def cpu_baseline(fr, N, M, gpu):
    """The oracle (plain C++, one thread) timed on this host, pinned to one core of the cores this
    process may use (the affinity is restored afterwards).  One warm-up run over the whole workload,
    whose every group (key, sum, count), join size and top-k are compared with the GPU's; then three
    timed runs over a bounded sample, the first quarter of the fact rows against the whole mid
    table; the value is the median of the three, in fact rows per second."""
    import numpy as np

    import oracle
    model, usable, ncpu = host_cpu()
    saved = os.sched_getaffinity(0)
    core = sorted(saved)[len(saved) // 2]
    os.sched_setaffinity(0, {core})
    try:
        t1 = time.perf_counter()
        want = oracle.fragment_cust(fr.fact, fr.mid, fr.D, fr.k, gcap=max(1, min(N, fr.cust_hi)))
        full_s = time.perf_counter() - t1
        ok = (want["groups"] == gpu["groups"] and want["join_rows"] == gpu["join_rows"]
              and np.array_equal(want["key"], gpu["key"]) and np.array_equal(want["sum"], gpu["sum"])
              and np.array_equal(want["cnt"], gpu["cnt"])
              and np.array_equal(want["top_key"], gpu["top_key"]) and np.array_equal(want["top_sum"], gpu["top_sum"])
              and np.array_equal(want["top_cnt"], gpu["top_cnt"]))
        ns = N // 4
        sample = {k: v[:ns] for k, v in fr.fact.items()}
        times = []
        for _ in range(3):
            t1 = time.perf_counter()
            oracle.fragment_cust(sample, fr.mid, fr.D, fr.k, gcap=max(1, min(N, fr.cust_hi)))
            times.append(time.perf_counter() - t1)
    finally:
        os.sched_setaffinity(0, saved)
    med = sorted(times)[1]
    log("oracle: whole workload %.1f s (matches GPU: %s); sample runs %s s" % (full_s, ok, [round(t, 2) for t in times]))
    return {"value": round(ns / med, 1), "unit": "fact rows/s", "cores": 1, "kind": "oracle",
            "sample": "fact rows [0, %d) of %d against all %d mid rows, date < %d, group by custkey, top-%d; "
                      "one thread pinned to core %d; median of 3 timed runs (%s s) after one warm-up run over the "
                      "whole workload (%.1f s)" % (ns, N, M, fr.D, fr.k, core,
                                                   ", ".join("%.2f" % t for t in times), full_s),
            "host_cpu": model, "host_nproc": ncpu, "host_usable_cores": usable,
            "matches_gpu": bool(ok), "matches_gpu_compares": "every group (key, sum, count), join size, top-k rows"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--digit-bits", type=int, default=8, choices=[4, 8, 11])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without the per-launch events")
    ap.add_argument("--with-copy", action="store_true",
                    help="after the steps, run a plain 1 GiB device copy (calibrates HBM counters)")
    ap.add_argument("--rows", type=int, default=0, help="fact rows (0: the full 60M workload)")
    ap.add_argument("--revenue-bits", type=int, default=32, choices=[32, 64],
                    help="declared width of the revenue price*(100-disc) carried through sort, join and "
                         "group-by (the workload's maximum is about 1.05e9 < 2^32; sums are int64 either way, "
                         "and a row outside the declared width sets a device error flag)")
    ap.add_argument("--date-lt", type=int, default=None,
                    help="config 2 with another filter constant D (date < D; the workload uses 2400)")
    ap.add_argument("--config", type=int, default=2, choices=[2, 3, 4, 5, 6, 7, 8, 9, 10],
                    help="2: the 60M-row custkey fragment (default); 3: 256 flags fragments, batched vs plain; "
                         "4: served mix under Poisson arrivals, concurrent vs serial; 5: the join kinds on the "
                         "config-2 join inputs; 6: hash join vs sort join from unsorted inputs, 1 to 64 rows per key; "
                         "7: hash vs sort group-by over 60M rows, 6 to 15M groups; 8: a chain of three joins; 9: expression programs; "
                         "10: the custkey workload as a general fragment (tqp_fragment_run) against the fused one")
    ap.add_argument("--rates", default="25,50,100,200,400,800,1600,3200",
                    help="arrival rates (fragments/s) for --config 4, swept until no mode keeps up")
    ap.add_argument("--requests", type=int, default=2000, help="least requests per rate for --config 4")
    ap.add_argument("--min-seconds", type=float, default=0.0,
                    help="--config 4: at least this many seconds of arrivals per rate")
    ap.add_argument("--modes", default="continuous,serial",
                    help="--config 4 server modes: continuous, serial, serial_same_plan (the first is the headline)")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--max-batch", type=int, default=32)
    ap.add_argument("--fragments", type=int, default=256, help="fragments of the batched workload")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_2203_01877_amd as tqp

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.config == 3:
        return bench_batch(args)
    if args.config == 5:
        return bench_joins(args)
    if args.config == 6:
        return bench_hash_vs_sort(args)
    if args.config == 7:
        return bench_groupby(args)
    if args.config == 8:
        return bench_chain(args)
    if args.config == 9:
        return bench_expr(args)
    if args.config == 10:
        return bench_general(args)
    if args.config == 4:
        return bench_serve(args)

    t0 = time.time()
    if args.rows:
        m = max(1, args.rows // 4)
        fr = datagen.config2(n=args.rows, m=m, cust_hi=max(1, args.rows // 40))
    else:
        fr = datagen.config2()
    if args.date_lt is not None:
        fr.D = args.date_lt
    N, M = len(fr.fact["fk"]), len(fr.mid["pk"])
    n_f = int(np.count_nonzero(fr.fact["date"] < fr.D))
    log("generated %d fact rows, %d mid rows in %.1fs" % (N, M, time.time() - t0))

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    fact = tqp.to_device({k: fr.fact[k] for k in ("fk", "date", "price", "disc")}, dev)
    mid = tqp.to_device(fr.mid, dev)
    key_bits = datagen.bits_for(max(int(fr.fact["fk"].max()), M - 1) + 1)
    cust_bits = datagen.bits_for(fr.cust_hi)
    ctx = tqp.Context(0)
    ctx.set_digit_bits(args.digit_bits)
    PB = args.revenue_bits // 8
    run = tqp.CustFragmentRunner(ctx, fact, mid, fr.D, fr.k, key_bits=key_bits, cust_bits=cust_bits,
                                 gcap=min(N, fr.cust_hi), revenue_bits=args.revenue_bits)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        run.run()
    torch.cuda.synchronize()
    log("warmup done")

    def timed_steps(profiled):
        """K steps between two stream events after a device synchronisation; with
        profiled, the library also records an event pair around every launch."""
        if profiled:
            ctx.profile_read()              # drop earlier records
            ctx.set_profiling(True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for i in range(args.steps):
            run.run()
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        recs = ctx.profile_read() if profiled else []
        ctx.set_profiling(False)
        step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
        return ev[0].elapsed_time(ev[-1]) / args.steps, recs, step_ms

    # the step time comes from a run without per-launch events; the per-kernel
    # durations of the roofline from a second, profiled run of the same steps
    ms, _, step_ms = timed_steps(False)
    log("timed %d steps: %.3f ms/step" % (args.steps, ms))
    ms_prof, recs, _ = (None, [], None) if args.no_profile else timed_steps(True)
    if ms_prof is not None:
        log("timed %d profiled steps: %.3f ms/step" % (args.steps, ms_prof))

    res = run.result(all_groups=False)
    J, G = res["join_rows"], res["groups"]
    errors = ctx.errors()
    if errors:
        log("device error flags: %#x" % errors)
        sys.exit(3)

    # ---------------------------------------------------------------- per-kernel figures
    per = {}
    for name, t in recs:
        per.setdefault(name, []).append(t)
    stage_ms = {k: round(sum(v) / args.steps, 4) for k, v in sorted(per.items())}
    stage_bytes = algorithmic_bytes(run.plan(), N, n_f, M, J, G, PB) if per else {}
    step_bytes = sum(algorithmic_bytes(run.plan(), N, n_f, M, J, G, PB).values())
    stage_gbps = {k: round(b / (stage_ms[k] * 1e-3) / 1e9, 1) for k, b in stage_bytes.items()
                  if stage_ms.get(k)}
    # roofline: the family with the most measured time per step among the big single-stream kernels
    roofline = None
    plan = run.plan()
    lbytes = launch_bytes(plan, N, n_f, M, J, G, PB)
    families = roofline_families(PB)
    timed = {f: sum(per[f]) for f in lbytes if f in per}
    if args.digit_bits == 8 and timed:
        fam = max(timed, key=timed.get)
        durs = per[fam]
        sizes = lbytes[fam]
        if len(durs) == len(sizes) * args.steps:
            bytes_total = sum(sizes) * args.steps
            achieved = bytes_total / (sum(durs) * 1e-3) / 1e9
            roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(fam, families[fam][1], PB),
                        "kernel": families[fam][0], "family": fam,
                        "launches": len(durs), "avg_launch_ms": round(sum(durs) / len(durs), 4),
                        "bytes_per_launch": round(bytes_total / len(durs)),
                        "share_of_profiled_step": round(sum(durs) / args.steps / ms_prof, 3)}
        else:
            log("kernel %s: launch count %d does not match %d per step x %d steps"
                % (fam, len(durs), len(sizes), args.steps))

    P = max(1, -(-key_bits // 8))
    Pm = max(1, -(-datagen.bits_for(M) // 8))
    Pg = max(1, -(-cust_bits // 8))
    bref = reference_model_bytes(N, n_f, M, J, G, P, Pm, Pg)
    value = N / (ms * 1e-3)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "fact rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": ("60M-row fact x 15M-row mid: date<%d, fk=pk, group by custkey, sum+count, "
                                "top-100 by sum desc" % fr.D) if not args.rows else "scaled custkey fragment",
                   "fact_rows": N, "mid_rows": M, "filtered_fact_rows": n_f, "join_rows": J, "groups": G,
                   "digit_bits": args.digit_bits, "key_bits": key_bits, "cust_bits": cust_bits,
                   "revenue_bits": args.revenue_bits,
                   "plan": run.plan()},
        "roofline": roofline,
        # the step's own algorithmic bytes (every kernel family of this design) over its time
        "step_algorithmic_bytes": step_bytes,
        "step_hbm_fraction": round(step_bytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
        # a speed ratio, not a bandwidth: the paper's pass structure (full sorts, every pass
        # reading and writing its rows) priced in bytes, over this step's time and the peak
        "ref_model_speed_ratio": round(bref / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
        "ref_model_bytes": bref,
        "stage_ms": stage_ms,
        "stage_gbps": stage_gbps,
        "ms_per_step_profiled": None if ms_prof is None else round(ms_prof, 4),
        # one step = one whole fragment, back to back on the stream: its latency on the device
        "step_ms_p50": round(float(np.percentile(step_ms, 50)), 4),
        "step_ms_p99": round(float(np.percentile(step_ms, 99)), 4),
    }

    if args.with_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        ctx.set_profiling(True)
        for _ in range(3):
            ctx.copy(dst, src, 1 << 30)
        copy_ms = [t for _, t in ctx.profile_read()]
        ctx.set_profiling(False)
        out["copy_1GiB_ms"] = round(sum(copy_ms) / len(copy_ms), 4)
        out["copy_GBps"] = round(2 * (1 << 30) / (sum(copy_ms) / len(copy_ms) * 1e-3) / 1e9, 1)

    if not args.no_cpu_baseline:
        res_all = run.result(all_groups=True)
        out["cpu_baseline"] = cpu_baseline(fr, N, M, res_all)
    print(json.dumps(out), flush=True)


def bench_joins(args):
    """The join kinds (inner, left semi, left anti, left outer) on the config-2 join's inputs: the
    56.3M fact keys that pass date < 2400, sorted, against the 15M sorted mid keys.  Per kind: the
    kernels' own event durations (windows + counting + expansion), the output rows, and the
    expansion's algorithmic bytes per second; the counts are checked against numpy's searchsorted."""
    import numpy as np
    import torch

    import datagen
    import paper_2203_01877_amd as tqp

    fr = datagen.config2()
    lkey = np.sort(fr.fact["fk"][fr.fact["date"] < fr.D]).astype(np.int32)
    rkey = np.sort(fr.mid["pk"]).astype(np.int32)
    nl, nr = len(lkey), len(rkey)
    hits = np.searchsorted(rkey, lkey, "right") - np.searchsorted(rkey, lkey, "left")
    want = {tqp.JOIN_INNER: int(hits.sum()), tqp.JOIN_LEFT_SEMI: int((hits > 0).sum()),
            tqp.JOIN_LEFT_ANTI: int((hits == 0).sum()), tqp.JOIN_LEFT_OUTER: int(np.maximum(hits, 1).sum())}
    dev = torch.device("cuda", 0)
    lk, rk = torch.from_numpy(lkey).to(dev), torch.from_numpy(rkey).to(dev)
    ctx = tqp.Context(0)
    names = {tqp.JOIN_INNER: "inner", tqp.JOIN_LEFT_SEMI: "left_semi", tqp.JOIN_LEFT_ANTI: "left_anti",
             tqp.JOIN_LEFT_OUTER: "left_outer"}
    expansion = {tqp.JOIN_INNER: "join_pairs", tqp.JOIN_LEFT_SEMI: "join_semi", tqp.JOIN_LEFT_ANTI: "join_anti",
                 tqp.JOIN_LEFT_OUTER: "join_outer"}
    out = {}
    for kind, name in names.items():
        cap = want[kind]
        for _ in range(args.warmup):
            tqp.join(ctx, lk, rk, cap=cap, kind=kind)
        torch.cuda.synchronize()
        ctx.profile_read()
        ctx.set_profiling(True)
        for _ in range(args.steps):
            _, _, cnt = tqp.join(ctx, lk, rk, cap=cap, kind=kind)
        torch.cuda.synchronize()
        recs = ctx.profile_read()
        ctx.set_profiling(False)
        got = int(cnt.item())
        if got != want[kind] or ctx.errors():
            log("join %s: %d rows, expected %d" % (name, got, want[kind]))
            sys.exit(3)
        ms = sum(t for _, t in recs) / args.steps
        ems = sum(t for k, t in recs if k == expansion[kind]) / args.steps
        # expansion: left keys 4 B, window keys 4 B, output (left, right) positions 8 B per row
        eb = 4 * nl + 4 * nr + 8 * got
        out[name] = {"ms": round(ms, 4), "expansion_ms": round(ems, 4), "rows_out": got,
                     "left_rows_per_s": round(nl / (ms * 1e-3), 1),
                     "expansion_gbps": round(eb / (ems * 1e-3) / 1e9, 1)}
        log("%s: %s" % (name, out[name]))
    # band join |l - r| <= 1 (the non-equi variant) on the same keys
    wband = 1
    want_b = int((np.searchsorted(rkey, lkey.astype(np.int64) + wband, "right")
                  - np.searchsorted(rkey, lkey.astype(np.int64) - wband, "left")).sum())
    for _ in range(args.warmup):
        tqp.join_band(ctx, lk, rk, wband, cap=want_b)
    torch.cuda.synchronize()
    ctx.profile_read()
    ctx.set_profiling(True)
    for _ in range(args.steps):
        _, _, cnt = tqp.join_band(ctx, lk, rk, wband, cap=want_b)
    torch.cuda.synchronize()
    recs = ctx.profile_read()
    ctx.set_profiling(False)
    got = int(cnt.item())
    if got != want_b or ctx.errors():
        log("band join: %d rows, expected %d" % (got, want_b))
        sys.exit(3)
    ms = sum(t for _, t in recs) / args.steps
    ems = sum(t for k, t in recs if k == "band_expand") / args.steps
    out["band_w1"] = {"ms": round(ms, 4), "expansion_ms": round(ems, 4), "rows_out": got,
                      "left_rows_per_s": round(nl / (ms * 1e-3), 1),
                      "expansion_gbps": round((4 * nl + 4 * nr + 8 * got) / (ems * 1e-3) / 1e9, 1)}
    log("band_w1: %s" % out["band_w1"])
    print(json.dumps({"metric": "left rows/s per join kind (sorted 56.3M x 15M keys)", "unit": "left rows/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
                      "data": "synthetic", "dtype": "int32",
                      "config": {"workload": "config-2 join inputs: %d sorted fact keys (date < %d) x %d sorted mid "
                                             "keys, row positions as payloads" % (nl, fr.D, nr)},
                      "kinds": out, "counts_match_numpy": True}), flush=True)


def bench_hash_vs_sort(args):
    """Hash join against the sort-based join from unsorted inputs (Section 5.3's comparison): n left
    and n right rows, r right rows per key (keys i // r, shuffled), left keys uniform over the same
    key range, r = 1, 2, 4, ..., 64.  Sort-based = stable sort of both sides (with their
    permutations) + the sort join; hash-based = tqp_hash_join (partitioned).  Times from the library's
    own kernel events; the two join sizes must agree, and at r = 1 the two sets of pairs too."""
    import numpy as np
    import torch

    import paper_2203_01877_amd as tqp

    n = args.rows or 8_000_000
    dev = torch.device("cuda", 0)
    ctx = tqp.Context(0)
    rng = np.random.default_rng(17)
    sweep = []
    for r in (1, 2, 4, 8, 16, 32, 64):
        dom = max(1, n // r)
        rkey = rng.permutation(np.arange(n, dtype=np.int64) // r).astype(np.int32)
        lkey = rng.integers(0, dom, n).astype(np.int32)
        want = int((np.bincount(lkey, minlength=dom).astype(np.int64) *
                    np.bincount(rkey, minlength=dom).astype(np.int64)).sum())
        lk, rk = torch.from_numpy(lkey).to(dev), torch.from_numpy(rkey).to(dev)
        kb = max(1, int(dom - 1).bit_length())

        def sort_join():
            ls, lp = tqp.sort(ctx, lk, key_bits=kb, perm=True)
            rs, rp = tqp.sort(ctx, rk, key_bits=kb, perm=True)
            return tqp.join(ctx, ls, rs, lp, rp, cap=want)[2]

        def hash_join():
            return tqp.hash_join(ctx, lk, rk, cap=want)[2]

        if r == 1:
            # the same pairs: (left, right) positions, compared as sorted sets
            ls, lp = tqp.sort(ctx, lk, key_bits=kb, perm=True)
            rs, rp = tqp.sort(ctx, rk, key_bits=kb, perm=True)
            a_l, a_r, _ = tqp.join(ctx, ls, rs, lp, rp, cap=want)
            b_l, b_r, _ = tqp.hash_join(ctx, lk, rk, cap=want)
            ka = np.sort(a_l[:want].cpu().numpy().astype(np.int64) * n + a_r[:want].cpu().numpy())
            kb_ = np.sort(b_l[:want].cpu().numpy().astype(np.int64) * n + b_r[:want].cpu().numpy())
            if not np.array_equal(ka, kb_):
                log("r = 1: the hash join's pairs differ from the sort join's")
                sys.exit(3)
            del ls, lp, rs, rp, a_l, a_r, b_l, b_r

        res = {"rows_per_key": r, "join_rows": want}
        for name, fn in (("sort", sort_join), ("hash", hash_join)):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            ctx.profile_read()
            ctx.set_profiling(True)
            for _ in range(args.steps):
                cnt = fn()
            torch.cuda.synchronize()
            recs = ctx.profile_read()
            ctx.set_profiling(False)
            if int(cnt.item()) != want or ctx.errors():
                log("%s join, r = %d: %d rows, expected %d" % (name, r, int(cnt.item()), want))
                sys.exit(3)
            res[name + "_ms"] = round(sum(t for _, t in recs) / args.steps, 4)
            per = {}
            for k, t in recs:
                per[k] = per.get(k, 0.0) + t / args.steps
            res[name + "_kernels_ms"] = {k: round(v, 4) for k, v in sorted(per.items())}
        res["hash_speedup"] = round(res["sort_ms"] / res["hash_ms"], 2)
        log(str(res))
        sweep.append(res)
        del lk, rk
        torch.cuda.empty_cache()
    faster = [x["rows_per_key"] for x in sweep if x["hash_ms"] < x["sort_ms"]]
    print(json.dumps({"metric": "join ms from unsorted inputs, hash vs sort", "unit": "ms", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "higher_is_better": False, "data": "synthetic",
                      "dtype": "int32", "config": {"workload": "%d x %d rows, r right rows per key" % (n, n)},
                      "hash_faster_at_rows_per_key": faster, "sweep": sweep}), flush=True)


def bench_groupby(args):
    """Hash-based against sort-based group-by (Section 6 credits the hash-based systems' lead on
    aggregation to this difference): N rows (60M, the fact table of the custkey fragment), G
    uniform keys, G = 6 .. 15M; SUM and COUNT per group.  Sort-based = tqp_groupby_agg (radix sort
    of the key, trimmed to its width, then the run reduction); hash-based = tqp_hash_groupby; hash
    with every aggregate adds MIN, MAX and COUNT(DISTINCT) of a second column; hash_distinct is COUNT
    and COUNT(DISTINCT) alone.  Times from the library's own kernel events; the outputs are compared
    in full."""
    import numpy as np
    import torch

    import paper_2203_01877_amd as tqp

    n = args.rows or 60_000_000
    dev = torch.device("cuda", 0)
    ctx = tqp.Context(0)
    rng = np.random.default_rng(23)
    val_h = rng.integers(0, 1_000_000, n).astype(np.int64)
    dv_h = rng.integers(0, 64, n).astype(np.int32)
    val, dv = torch.from_numpy(val_h).to(dev), torch.from_numpy(dv_h).to(dev)
    sweep = []
    for G in (6, 1000, 150_000, 1_500_000, 15_000_000):
        key_h = rng.integers(0, G, n).astype(np.int32)
        gk = torch.from_numpy(key_h).to(dev)
        kb = max(1, int(G - 1).bit_length())
        runs = {"sort": lambda: tqp.groupby_agg(ctx, gk, val, key_bits=kb, gcap=G),
                "hash": lambda: tqp.hash_groupby(ctx, gk, val, gcap=G),
                "hash_all": lambda: tqp.hash_groupby(ctx, gk, val, dv, gcap=G, minmax=True),
                "hash_distinct": lambda: tqp.hash_groupby(ctx, gk, dval=dv, gcap=G)}
        res = {"groups": G}
        outs = {}
        for name, fn in runs.items():
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            ctx.profile_read()
            ctx.set_profiling(True)
            for _ in range(args.steps):
                out = fn()
            torch.cuda.synchronize()
            recs = ctx.profile_read()
            ctx.set_profiling(False)
            ng = int(out["d_ngroups"].item())
            if ctx.errors() or ng > G:
                log("%s group-by, G = %d: %d groups, device errors %d" % (name, G, ng, ctx.errors()))
                sys.exit(3)
            k = out["key"][:ng].cpu().numpy()
            o = np.argsort(k)
            outs[name] = (k[o], out["cnt"][:ng].cpu().numpy()[o]) + (
                (out["sum"][:ng].cpu().numpy()[o],) if out["sum"] is not None else ())
            res[name + "_ms"] = round(sum(t for _, t in recs) / args.steps, 4)
            per = {}
            for kname, t in recs:
                per[kname] = per.get(kname, 0.0) + t / args.steps
            res[name + "_kernels_ms"] = {kk: round(v, 4) for kk, v in sorted(per.items())}
        for name in ("hash", "hash_all", "hash_distinct"):
            if not all(np.array_equal(a, b) for a, b in zip(outs["sort"], outs[name])):
                log("G = %d: %s and sort group-by differ" % (G, name))
                sys.exit(3)
        res["hash_speedup"] = round(res["sort_ms"] / res["hash_ms"], 2)
        log(str(res))
        sweep.append(res)
        del gk
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "group-by ms, hash vs sort", "unit": "ms", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "higher_is_better": False, "data": "synthetic", "dtype": "int64",
                      "config": {"workload": "%d rows, G uniform int32 keys, int64 values" % n},
                      "sweep": sweep}), flush=True)


def bench_chain(args):
    """A chain of three sort-based joins in the shape of the paper's multi-join plans: fact (60M rows,
    key into mid) -> mid (15M rows, primary key in order, key into cust) -> cust (1.5M rows, primary
    key shuffled, key into nation) -> nation (25 rows, in order).  Every fact row matches one row per
    hop, so 60M tuples of 4 row positions come out.  Timed with the rule that treats a key column
    equal to 0..M-1 as dense (mid and nation: a filter instead of sort and join), with the rule that
    only skips the sort of a key column already in order, and with neither; kernel times from the library's
    events, wall time includes the one host read of each hop's size.  The result count is checked."""
    import numpy as np
    import torch

    import paper_2203_01877_amd as tqp

    n = args.rows or 60_000_000
    m, c, q = max(1, n // 4), max(1, n // 40), 25
    dev = torch.device("cuda", 0)
    ctx = tqp.Context(0)
    rng = np.random.default_rng(29)
    cols = {"fact_fk": rng.integers(0, m, n), "mid_pk": np.arange(m), "mid_fk": rng.integers(0, c, m),
            "cust_pk": rng.permutation(c), "cust_fk": rng.integers(0, q, c), "nation_pk": np.arange(q)}
    d = {k: torch.from_numpy(v.astype(np.int32)).to(dev) for k, v in cols.items()}
    outs = [d["fact_fk"], d["mid_fk"], d["cust_fk"]]
    pks = [d["mid_pk"], d["cust_pk"], d["nation_pk"]]
    kb = [int(x - 1).bit_length() for x in (m, c, q)]      # key widths of the three hops
    res = {"key_bits": kb}
    ref = {}
    for name, rule, dense in (("dense_keys", [True, False, True], [True, False, True]),
                              ("skip_sorted", [True, False, True], None), ("sort_all", [False, False, False], None)):
        caps = [n, n, n]
        for _ in range(args.warmup):
            tqp.join_chain(ctx, outs, pks, pk_sorted=rule, key_bits=kb, caps=caps, pk_dense=dense)
        torch.cuda.synchronize()
        ctx.profile_read()
        ctx.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, J = tqp.join_chain(ctx, outs, pks, pk_sorted=rule, key_bits=kb, caps=caps, pk_dense=dense)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / args.steps
        recs = ctx.profile_read()
        ctx.set_profiling(False)
        if J != n:
            log("join chain (%s): %d tuples, expected %d" % (name, J, n))
            sys.exit(3)
        # the same tuples from every plan (their order is free): each fact row matches once, so
        # the tuples ordered by their fact row must agree column by column
        out_cols, _ = tqp.join_chain(ctx, outs, pks, pk_sorted=rule, key_bits=kb, caps=caps, pk_dense=dense)
        first, order = torch.sort(out_cols[0][:J])
        tup = [first] + [col[:J][order] for col in out_cols[1:]]
        if "first" not in ref:
            ref["first"] = tup
        elif not all(torch.equal(a, b) for a, b in zip(ref["first"], tup)):
            log("join chain (%s): tuples differ from the first plan's" % name)
            sys.exit(3)
        per = {}
        for k, t in recs:
            per[k] = per.get(k, 0.0) + t / args.steps
        res[name] = {"kernel_ms": round(sum(per.values()), 4), "wall_ms": round(wall, 4),
                     "kernels_ms": {k: round(v, 4) for k, v in sorted(per.items())}}
        log("%s: %s" % (name, res[name]))
    print(json.dumps({"metric": "join chain ms, 3 joins", "unit": "ms", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "higher_is_better": False, "data": "synthetic", "dtype": "int32",
                      "config": {"workload": "%d fact -> %d mid -> %d cust -> %d nation rows, %d result tuples"
                                 % (n, m, c, q, n)}, "result": res}), flush=True)


def bench_expr(args):
    """Expression programs over 60M rows: the revenue expression price * (100 - disc) and a CASE
    (date < D ? price * (100 - disc) : 0) + flag over int64 / int32 / int8 columns, as one tqp_eval
    launch each.  Reports the kernel time and the rate of algorithmic bytes (columns read once,
    int64 result written once) against the 8 TB/s HBM peak; one result is checked against numpy."""
    import numpy as np
    import torch

    import paper_2203_01877_amd as tqp
    from paper_2203_01877_amd import _lib

    n = args.rows or 60_000_000
    dev = torch.device("cuda", 0)
    ctx = tqp.Context(0)
    rng = np.random.default_rng(31)
    h = {"price": rng.integers(90_000, 10_500_000, n).astype(np.int64), "disc": rng.integers(0, 11, n).astype(np.int64),
         "date": rng.integers(0, 2557, n).astype(np.int32), "flag": rng.integers(0, 3, n).astype(np.int8)}
    d = {k: torch.from_numpy(v).to(dev) for k, v in h.items()}
    X = _lib
    progs = {
        "revenue": ([d["price"], d["disc"]], [(X.TQP_X_COL, 0), (X.TQP_X_CONST, 100), (X.TQP_X_COL, 1),
                                                (X.TQP_X_SUB, 0), (X.TQP_X_MUL, 0)], 8 + 8 + 8),
        "case": ([d["date"], d["price"], d["disc"], d["flag"]],
                 [(X.TQP_X_COL, 0), (X.TQP_X_CONST, 2400), (X.TQP_X_LT, 0), (X.TQP_X_COL, 1), (X.TQP_X_CONST, 100),
                  (X.TQP_X_COL, 2), (X.TQP_X_SUB, 0), (X.TQP_X_MUL, 0), (X.TQP_X_CONST, 0), (X.TQP_X_SELECT, 0),
                  (X.TQP_X_COL, 3), (X.TQP_X_ADD, 0)], 4 + 8 + 8 + 1 + 8),
    }
    res = {}
    for name, (cols, prog, bpr) in progs.items():
        for _ in range(args.warmup):
            out = tqp.eval_expr(ctx, cols, prog)
        torch.cuda.synchronize()
        ctx.profile_read()
        ctx.set_profiling(True)
        for _ in range(args.steps):
            out = tqp.eval_expr(ctx, cols, prog)
        torch.cuda.synchronize()
        recs = ctx.profile_read()
        ctx.set_profiling(False)
        ms = sum(t for _, t in recs) / args.steps
        res[name] = {"ms": round(ms, 4), "bytes_per_row": bpr, "GB/s": round(n * bpr / ms / 1e6, 1),
                     "frac_of_8TBps": round(n * bpr / ms / 1e6 / 8000.0, 3)}
        log("%s: %s" % (name, res[name]))
    want = h["price"] * (100 - h["disc"])
    got = tqp.eval_expr(ctx, [d["price"], d["disc"]], progs["revenue"][1]).cpu().numpy()
    if not np.array_equal(got, want) or ctx.errors():
        log("expression result differs from numpy")
        sys.exit(3)
    print(json.dumps({"metric": "expression ms and GB/s", "unit": "ms", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "higher_is_better": False, "data": "synthetic", "dtype": "int64",
                      "config": {"workload": "%d rows, two expression programs" % n}, "result": res}), flush=True)


def bench_general(args):
    """The config-2 custkey workload (60M fact x 15M mid rows) written as a general fragment
    descriptor (tqp_fragment_run: predicate program, join, group column, SUM and COUNT over value
    programs, top-100) against the fused custkey fragment, both timed as launch sequences on the
    stream, each with the revenue declared 32-bit and 64-bit; then config 1's flags fragment, fused
    and as a descriptor.  The general results must equal the fused ones (every group, the join
    size, the top rows)."""
    import numpy as np
    import torch

    import datagen
    import paper_2203_01877_amd as tqp
    from paper_2203_01877_amd import _lib as X

    fr = datagen.config2() if not args.rows else datagen.config2(n=args.rows, m=max(1, args.rows // 4),
                                                                  cust_hi=max(1, args.rows // 40))
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    N, M = len(fr.fact["fk"]), len(fr.mid["pk"])
    fact = tqp.to_device({k: fr.fact[k] for k in ("fk", "date", "price", "disc")}, dev)
    mid = tqp.to_device(fr.mid, dev)
    key_bits = datagen.bits_for(max(int(fr.fact["fk"].max()), M - 1) + 1)
    cust_bits = datagen.bits_for(fr.cust_hi)
    ctx = tqp.Context(0)
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(args.steps):
            out = fn()
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / args.steps, out

    res = {}
    fused = {}
    for bits in (32, 64):
        run = tqp.CustFragmentRunner(ctx, fact, mid, fr.D, fr.k, key_bits=key_bits, cust_bits=cust_bits,
                                     gcap=min(N, fr.cust_hi), revenue_bits=bits)
        ms, _ = timed(lambda: run.run())
        fused[bits] = run.result()
        res["fused_rev%d_ms" % bits] = round(ms, 4)
        log("fused custkey fragment, %d-bit revenue: %.3f ms" % (bits, ms))
    cols = [fact["fk"], fact["date"], fact["price"], fact["disc"]]
    dcols = [mid["pk"], mid["custkey"]]
    rev = [(X.TQP_X_COL, 2), (X.TQP_X_CONST, 100), (X.TQP_X_COL, 3), (X.TQP_X_SUB, 0), (X.TQP_X_MUL, 0)]
    pred = [(X.TQP_X_COL, 1), (X.TQP_X_CONST, fr.D), (X.TQP_X_LT, 0)]
    f = fused[64]
    ok = all(np.array_equal(fused[32][x], fused[64][x]) for x in ("key", "sum", "cnt", "top_key"))
    for vb in (64, 32):
        # the revenue declared int32 (value_bits = 32) or int64, as the fused fragment's revenue_bits
        gen = lambda vb=vb: tqp.fragment_run(ctx, cols, dcols, pred, [], 0, 0, [(5, cust_bits)],
                                             [(X.AGG_SUM, rev), (X.AGG_COUNT, [])], topk=fr.k, key_bits=key_bits,
                                             join_cap=N, gcap=fr.cust_hi, value_bits=vb)
        ms, out = timed(gen)
        res["general_ms" if vb == 32 else "general_v64_ms"] = round(ms, 4)
        log("general fragment, %d-bit value: %.3f ms" % (vb, ms))
        G = int(out["d_ngroups"].item())
        k = int(out["d_topk"].item())
        ok = (ok and G == f["groups"] and int(out["d_join"].item()) == f["join_rows"] and ctx.errors() == 0
              and np.array_equal(out["key"][:G].cpu().numpy(), f["key"])
              and np.array_equal(out["vals"][0][:G].cpu().numpy(), f["sum"])
              and np.array_equal(out["vals"][1][:G].cpu().numpy(), f["cnt"])
              and np.array_equal(out["top_key"][:k].cpu().numpy(), f["top_key"]))
    # kernel time of one general call (32-bit value) by the library's events
    ctx.profile_read()
    ctx.set_profiling(True)
    gen()
    torch.cuda.synchronize()
    recs = ctx.profile_read()
    ctx.set_profiling(False)
    per = {}
    for name, t in recs:
        per[name] = round(per.get(name, 0.0) + t, 4)
    res["general_kernels_ms"] = per
    # the flags fragment of config 1 (6M fact x 150k dim rows, date < D and seg == c, six groups
    # by flagA, flagB: SUM revenue, COUNT, AVG price) fused and as a descriptor (the direct group-by)
    fr1 = datagen.config1()
    f1, d1 = tqp.to_device(fr1.fact, dev), tqp.to_device(fr1.dim, dev)
    frun = tqp.FlagsFragmentRunner(ctx, f1, d1, fr1.D, fr1.c, key_bits=fr1.key_bits)
    ms, _ = timed(lambda: frun.run())
    res["flags_fused_ms"] = round(ms, 4)
    ff = frun.result()
    gflags = lambda: tqp.fragment_run(ctx, [f1[k] for k in ("fk", "date", "price", "disc", "flagA", "flagB")],
                                      [d1["pk"], d1["seg"]], [(X.TQP_X_COL, 1), (X.TQP_X_CONST, fr1.D), (X.TQP_X_LT, 0)],
                                      [(X.TQP_X_COL, 1), (X.TQP_X_CONST, fr1.c), (X.TQP_X_EQ, 0)], 0, 0, [(4, 2), (5, 1)],
                                      [(X.AGG_SUM, rev), (X.AGG_COUNT, []), (X.AGG_AVG, [(X.TQP_X_COL, 2)])],
                                      key_bits=fr1.key_bits, gcap=8)
    ms, out = timed(gflags)
    res["flags_general_ms"] = round(ms, 4)
    G = int(out["d_ngroups"].item())
    ok = (ok and G == len(ff["key"]) and int(out["d_join"].item()) == ff["join_rows"] and ctx.errors() == 0
          and np.array_equal(out["key"][:G].cpu().numpy(), ff["key"])
          and np.array_equal(out["vals"][0][:G].cpu().numpy(), ff["sum"])
          and np.array_equal(out["vals"][1][:G].cpu().numpy(), ff["cnt"])
          and np.array_equal(out["vals"][2][:G].cpu().numpy().view(np.int64), ff["avg"].view(np.int64)))
    log("flags fragment (config 1): fused %.3f ms, general %.3f ms" % (res["flags_fused_ms"], res["flags_general_ms"]))
    if not ok:
        log("general flags fragment result differs from the fused one")
        sys.exit(3)
    res["general_vs_fused_rev32"] = round(res["general_ms"] / res["fused_rev32_ms"], 2)
    res["general_v64_vs_fused_rev64"] = round(res["general_v64_ms"] / res["fused_rev64_ms"], 2)
    res["general_fact_rows_per_s"] = round(N / (res["general_ms"] * 1e-3), 1)
    print(json.dumps({"metric": "custkey fragment ms, general descriptor vs fused", "unit": "ms", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "higher_is_better": False, "data": "synthetic",
                      "dtype": "int64", "config": {"workload": "%d fact x %d mid rows: date<%d, fk=pk, group by "
                                                             "custkey, sum+count, top-%d" % (N, M, fr.D, fr.k),
                                                    "groups": G},
                      "result": res, "results_equal": True}), flush=True)


def bench_batch(args):
    """256 flags fragments of log-uniform size: plain per-fragment launches vs one batched launch
    sequence (autotuned) vs its hipGraph replay, same data, results checked against the oracle."""
    import numpy as np
    import torch

    import datagen
    import paper_2203_01877_amd as tqp

    t0 = time.time()
    spec = datagen.config3_spec(count=args.fragments)
    host = [datagen.config3_fragment(spec, i) for i in range(args.fragments)]
    rows = sum(len(f.fact["fk"]) for f in host)
    log("generated %d fragments, %d fact rows in %.1fs" % (len(host), rows, time.time() - t0))
    dev = torch.device("cuda", 0)
    frags = [{"fact": tqp.to_device(f.fact, dev), "dim": tqp.to_device(f.dim, dev), "D": f.D, "c": f.c,
              "key_bits": f.key_bits} for f in host]
    ctx = tqp.Context(0)
    plain = [tqp.FlagsFragmentRunner(ctx, fr["fact"], fr["dim"], fr["D"], fr["c"], fr["key_bits"]) for fr in frags]
    batch = tqp.BatchRunner(ctx, frags)
    stream = torch.cuda.current_stream()

    def timed(fn, steps):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def run_plain():
        for r in plain:
            r.run()

    for _ in range(args.warmup):
        run_plain()
        batch.run()
    plain_ms = timed(run_plain, args.steps)
    tune = batch.autotune(reps=2)
    cfg = batch.config()
    for _ in range(args.warmup):
        batch.run()
    batch_ms = timed(batch.run, args.steps)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        batch.capture(side)
        for _ in range(args.warmup):
            batch.replay(side)
        side.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(side)
        for _ in range(args.steps):
            batch.replay(side)
        e1.record(side)
        side.synchronize()
        graph_ms = e0.elapsed_time(e1) / args.steps
    got = batch.results()
    ok_plain = True
    for r, g in zip(plain, got):
        a = r.result()
        ok_plain &= (a["join_rows"] == g["join_rows"] and np.array_equal(a["sum"], g["sum"])
                     and np.array_equal(a["cnt"], g["cnt"]) and np.array_equal(a["key"], g["key"]))
    out = {"metric": METRIC, "value": round(rows / (graph_ms * 1e-3), 1), "unit": "fact rows/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(graph_ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "%d flags fragments, fact rows log-uniform in [1e3, 4e6], dim = fact/40, "
                                  "own D and c each; batched + hipGraph replay" % len(frags),
                      "fragments": len(frags), "fact_rows": rows, "chosen": cfg[2]},
           "plain_ms": round(plain_ms, 4), "batched_ms": round(batch_ms, 4), "graph_ms": round(graph_ms, 4),
           "speedup_vs_plain": round(plain_ms / graph_ms, 2), "autotune_ms": {k: round(v, 4) for k, v in tune.items()},
           "fragments_per_s": round(len(frags) / (graph_ms * 1e-3), 1), "batch_equals_plain": bool(ok_plain)}
    if not args.no_cpu_baseline:
        import oracle
        t1 = time.perf_counter()
        ok = True
        for f, g in zip(host, got):
            w = oracle.fragment_flags(f.fact, f.dim, f.D, f.c)
            ok &= (w["join_rows"] == g["join_rows"] and np.array_equal(w["sum"], g["sum"])
                   and np.array_equal(w["avg"].view(np.int64), g["avg"].view(np.int64)))
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(rows / dt, 1), "unit": "fact rows/s", "cores": 1, "kind": "oracle",
                               "sample": "all %d fragments (%d fact rows), one run, single thread, %.1f s"
                                         % (len(host), rows, dt), "matches_gpu": bool(ok)}
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Served mix (half 60M-row custkey fragments with their own D, half flags fragments over a
    log-uniform row range of the resident fact table with their own D and c) under Poisson arrivals
    at each rate: the continuous-batching server (slots, micro-batches) against the same server
    with one slot and no batching (one request per launch sequence, serial)."""
    import threading

    import numpy as np
    import torch

    import datagen
    import paper_2203_01877_amd as tqp

    t0 = time.time()
    tabs = datagen.config4_tables()
    n_fact = len(tabs["fact"]["fk"])
    dev = {"fact": tqp.to_device(tabs["fact"]), "mid": tqp.to_device(tabs["mid"]), "dim": tqp.to_device(tabs["dim"])}
    log("resident tables: %d fact, %d mid, %d dim rows (%.1fs)" % (n_fact, len(tabs["mid"]["pk"]),
                                                                      len(tabs["dim"]["pk"]), time.time() - t0))
    kb_mid = datagen.bits_for(int(tabs["fact"]["fk"].max()) + 1)
    kb_dim = datagen.bits_for(len(tabs["dim"]["pk"]))
    cb = datagen.bits_for(tabs["cust_hi"])

    def run_trace(srv, reqs, gaps):
        launches0 = srv.stats()["launches"]
        arrivals = np.cumsum(gaps)
        base = srv.now() + 0.05

        def submitter():
            for r, t in zip(reqs, arrivals):
                while srv.now() < base + t:
                    d = base + t - srv.now()
                    if d > 2e-4:
                        time.sleep(d - 1e-4)
                srv.submit(0 if r["kind"] == "cust" else 1, r["D"], c=r["c"], k=100, row0=r["start"],
                           n_rows=r["len"])

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        srv.drain()
        res = srv.poll()
        lat = np.array([r["t_done"] - r["t_arrival"] for r in res])
        rows = sum(n_fact if r["kind"] == "cust" else r["len"] for r in reqs)
        span = max(r["t_done"] for r in res) - min(r["t_arrival"] for r in res)
        bad = sum(1 for r in res if r["status"] != 0)
        return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "rows_per_s": round(rows / span, 1), "fragments_per_s": round(len(res) / span, 1),
                "errors": bad, "launches": srv.stats()["launches"] - launches0}, res

    rates = [float(x) for x in args.rates.split(",") if x]
    modes = {
        # continuous batching: several slots, waiting flags requests coalesced, the mid table
        # sorted once at start-up, revenue carried in 32 bits (the workload's maximum is 1.05e9)
        "continuous": dict(slots=args.slots, max_batch=args.max_batch, presort_mid=True, revenue_bits=32),
        # plain per-query launches, one at a time: every custkey request sorts the mid table again
        "serial": dict(slots=1, max_batch=1, presort_mid=False, revenue_bits=0),
        # one at a time, but with the continuous server's per-request plan (sorted mid, 32-bit revenue)
        "serial_same_plan": dict(slots=1, max_batch=1, presort_mid=True, revenue_bits=32),
    }
    names = [m for m in args.modes.split(",") if m]
    servers = {m: tqp.Server(dev, key_bits_mid=kb_mid, key_bits_dim=kb_dim, cust_bits=cb, **modes[m]) for m in names}
    # warm-up: one request of each kind per server
    for srv in servers.values():
        srv.submit(0, 2400, k=100)
        srv.submit(1, 2400, c=1, row0=0, n_rows=100_000)
        srv.drain()
        srv.poll()
    sweep = []
    same = True
    for i, lam in enumerate(rates):
        seed = datagen.SEED_BASE + 4 + 1000 * (i + 1)
        nreq = max(args.requests, int(lam * args.min_seconds))
        reqs = datagen.config4_requests(seed, nreq, n_fact)
        gaps = datagen.poisson_gaps(seed, nreq, lam)
        row = {"rate": lam, "requests": nreq}
        outs = {}
        for name, srv in servers.items():
            row[name], outs[name] = run_trace(srv, reqs, gaps)
            log("rate %g %s: %s" % (lam, name, row[name]))
        ref = outs[names[0]]
        a = {r["id"] - min(x["id"] for x in ref): r for r in ref}
        for name in names[1:]:
            b = {r["id"] - min(x["id"] for x in outs[name]): r for r in outs[name]}
            for k in a:
                ka = {kk: a[k].get(kk) for kk in ("join_rows", "groups", "sum", "cnt", "top_key", "top_sum")}
                kb = {kk: b[k].get(kk) for kk in ("join_rows", "groups", "sum", "cnt", "top_key", "top_sum")}
                same &= ka == kb
        sweep.append(row)
        # saturated: no mode keeps up with the offered rate any more
        if all(row[m]["fragments_per_s"] < 0.8 * lam for m in names):
            break
    best = max(sweep, key=lambda r: r[names[0]]["rows_per_s"])
    below = [r for r in sweep if r[names[0]]["fragments_per_s"] >= 0.9 * r["rate"]]
    head = below[-1] if below else sweep[0]
    out = {"metric": METRIC, "value": best[names[0]]["rows_per_s"], "unit": "fact rows/s", "n_gpus": 1,
           "steps": sum(r["requests"] for r in sweep), "warmup": 1, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "served mix: 50% 60M-row custkey fragments, 50% flags fragments over log-uniform "
                                  "row ranges [1e3, 4e6] of a resident 60M-row fact table (15M-row mid, 150k-row "
                                  "dim); Poisson arrivals",
                      "modes": {m: modes[m] for m in names}, "budget_bytes": 200 << 30},
           "latency_at_highest_unsaturated_rate": {"rate": head["rate"],
                                                   **{m: {"p50_ms": head[m]["p50_ms"], "p99_ms": head[m]["p99_ms"]}
                                                      for m in names}},
           "sweep": sweep, "results_equal_across_modes": bool(same)}
    for srv in servers.values():
        srv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
