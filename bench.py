"""Benchmark: key-switches per second at N=2^16 on one MI355X.

One step is one pass of the hot path over one batch of synthetic input at
N=2^16, L=36 (36 + 12 primes < 2^30, dnum 3): HMult with relinearisation,
rescale of its result, and HRot by a uniform rotation; 2 key-switches per
step.  Inputs are uniform residues from the seeded generator, already in
HBM when the timed region starts.  Also reported on the same line: HMult
latency p50/p99 (each call bracketed by HIP events, at N=2^16 and at N=2^12),
the roofline position of the dominant kernel (algorithmic bytes of a
key-switch over its measured time, and its VALU issue rate), the batched
rates (8 HMults; the 64-job mixed-level batch), a short run of the
bootstrapping-shaped trace, a short serving run under Poisson arrivals, and
the CPU oracle timed on a bounded sample on the host cores.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
    python bench.py --boot-trace      # the bootstrapping-shaped trace alone, more runs
    python bench.py --serve           # the serving loop alone, with an HBM-budget sweep
    python bench.py --batched         # the batched comparison alone
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LIMB_BYTES = 4  # uint32 residues
HBM_PEAK_GBPS = 8000.0
# VALU issue: 256 CUs x 4 SIMDs, a wave64 instruction every 4 cycles per SIMD at 2.4 GHz
SIMDS = 1024
CLOCK_HZ = 2.4e9
CYCLES_PER_WAVE_INST = 4


# Sources whose change invalidates a stored PMC figure of the key-switching kernels.
KERNEL_SOURCES = ["paper_2512_18345_amd/csrc/" + f for f in
                  ("keyswitch.hip", "keyswitch.h", "ntt_tile.h", "arith.h", "ctx.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k5s_ntt_blks_ip_n16_l36_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "keyswitch_n16_l36_valu.txt")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_values(path):
    """The machine-readable "key: value" lines of a committed profile summary,
    or None when the summary is missing or the kernel sources changed after
    its counters were taken."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                key, _, v = line.partition(":")
                vals[key.strip()] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash():
        return None
    return vals


def stored_traffic():
    """HBM bytes per launch of the dominant kernel from the committed PMC
    summary (FETCH_SIZE and WRITE_SIZE passes scaled by the copy
    calibration), or None when the summary is missing or stale."""
    vals = stored_values(TRAFFIC_FILE)
    if not vals or "bytes_per_launch" not in vals:
        return None
    return int(vals["bytes_per_launch"])


def stored_valu():
    """Wave64 VALU instructions per launch of the dominant kernel and per
    benchmark step, from the committed SQ counter summary (None if stale)."""
    vals = stored_values(VALU_FILE)
    if not vals or "valu_insts_k5" not in vals or "valu_insts_per_step" not in vals:
        return None
    return int(vals["valu_insts_k5"]), int(vals["valu_insts_per_step"])


def valu_frac(wave_insts, seconds):
    """Fraction of the chip's VALU issue rate: wave-instructions x 4 cycles over
    (time x 2.4 GHz x 1024 SIMDs)."""
    return wave_insts * CYCLES_PER_WAVE_INST / (seconds * CLOCK_HZ * SIMDS)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--latency-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-trace", action="store_true", help="skip the short bootstrapping-shaped trace run")
    ap.add_argument("--no-serve", action="store_true", help="skip the short serving run")
    ap.add_argument("--no-tune", action="store_true", help="keep the default kernel schedule")
    ap.add_argument("--schedule", type=str, default="", metavar="UP,DOWN,SMALL[,SHAPE]",
                    help="run under this kernel schedule instead of the autotuned one")
    ap.add_argument("--batch-reps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--small-reps", type=int, default=10000,
                    help="HMult latency samples at N=2^12, 4+1 primes, dnum 4 (0 = skip)")
    ap.add_argument("--trace-runs", type=int, default=5, help="timed runs of the trace in the default line")
    ap.add_argument("--serve-budgets", type=str, default="0.25,1,64",
                    help="HBM budgets (GiB) of the extra saturated serving runs (--serve)")
    ap.add_argument("--boot-trace", action="store_true",
                    help="only run the bootstrapping-shaped operation trace (132 key-switches)")
    ap.add_argument("--batched", action="store_true",
                    help="only run the batched comparison (8 HMults; the 64-job mixed batch)")
    ap.add_argument("--serve", action="store_true",
                    help="only run the serving-loop benchmark (Poisson arrivals, p50/p99, budget sweep)")
    ap.add_argument("--serve-requests", type=int, default=300)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--source-hash", action="store_true",
                    help="print the hash of the key-switching kernel sources (stored with PMC figures)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (for scaling HBM counters)")
    return ap.parse_args()


def calibrate_copy(mib: int):
    """A plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE counters
    give the factor between counter units and bytes moved."""
    import torch
    torch.cuda.set_device(0)
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": n * 4, "copies": 3}), flush=True)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32).copy()).cuda()


def main():
    args = parse()
    if args.source_hash:
        print(kernel_source_hash())
        return
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not supported "
              "(batch-level data parallelism across GPUs needs no collective and is not run here).",
              file=sys.stderr)
        sys.exit(2)
    if args.serve:
        print(json.dumps({"serving": serve_numbers(args.serve_requests, args.serve_budget_gib,
                                                   args.serve_budgets)}), flush=True)
        return
    if args.boot_trace:
        print(json.dumps({"boot_trace": boot_trace_numbers(args.steps)}), flush=True)
        return

    import torch
    import ckks_inputs as ci
    import paper_2512_18345_amd as P

    torch.cuda.set_device(0)
    spec = ci.get("n16_l36")
    L, N, k = spec.L_max, spec.N, spec.k
    rng = ci.Rng(spec.seed)
    ct1 = rng.polys(2, spec.q, N)
    ct2 = rng.polys(2, spec.q, N)
    ctr = rng.polys(2, spec.q, N)
    rot = rng.rotation(N)
    rlk = rng.evk(spec)
    rotk = rng.evk(spec)
    d_ct1, d_ct2, d_ctr, d_rlk, d_rotk = map(_dev, (ct1, ct2, ctr, rlk, rotk))
    ctx = P.Context.from_spec(spec)
    h = ctx.handle
    ws = ctx.workspace("HMULT", L)
    ws_rot = ctx.workspace("HROT", L)
    ws_rs = ctx.workspace("RESCALE", L)
    out_m = torch.empty((2, L, N), dtype=torch.int32, device="cuda")
    out_r = torch.empty((2, L, N), dtype=torch.int32, device="cuda")
    out_s = torch.empty((2, L - 1, N), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    if args.batched:
        print(json.dumps({"batched": batched_numbers(P, ci, ctx, spec, d_rlk, args.batch_reps)}), flush=True)
        return

    # kernel schedule picked by the library's autotuner (before any timing)
    schedule = None
    if args.schedule:
        P.ckks_ctx_set_schedule(h, *[int(v) for v in args.schedule.split(",")])
        schedule = dict(P.ckks_ctx_get_schedule(h), fixed=True)
    elif not args.no_tune:
        sched, sched_us = P.ckks_ctx_tune(h, L, 3, stream)
        schedule = dict(sched, hmult_us=round(sched_us, 2))

    def step():
        P.ckks_hmult(h, d_ct1, d_ct2, L, d_rlk, out_m, ws, stream)
        P.ckks_rescale(h, out_m, L, out_s, ws_rs, stream)
        P.ckks_hrot(h, d_ctr, L, rot, d_rotk, out_r, ws_rot, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # Dominant kernel: NTT block pass fused with the key inner product (stage 2
    # of key-switching), timed by events the runtime records at the start and
    # end of each of its dispatches inside the timed region.
    ip_launches = 2 * args.steps
    P.ckks_trace_begin(h, P.STAGE["NTT_IP"], ip_launches)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ip_ms = P.ckks_trace_end(h, ip_launches)
    ks_per_step = 2
    value = ks_per_step * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    # HMult latency distribution: each call bracketed by events on its stream
    lat = []
    for _ in range(args.latency_reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.ckks_hmult(h, d_ct1, d_ct2, L, d_rlk, out_m, ws, stream)
        e1.record(stream)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1) * 1e3)
    lat = np.array(lat)
    small = None if args.small_reps <= 0 else small_hmult_latency(P, ci, args.small_reps)

    beta = ctx.beta(L)
    R = L + k
    limb = N * LIMB_BYTES
    # Algorithmic bytes of one key-switch at level L: the switched polynomial
    # in, the key rows of level L in, both output components out (the
    # intermediates are assumed on chip).  One K5 launch of the step processes
    # one key-switch.
    ks_bytes = _op_limbs("KEYSWITCH", L, k, beta) * limb
    # K5's own input and output: the beta*R ModUp rows and 2*beta*R key rows
    # in, the 2*R accumulator rows out
    ip_io_bytes = (3 * beta + 2) * R * limb
    ip_s = 1e-3 * float(np.mean(ip_ms))
    achieved = ks_bytes / ip_s / 1e9
    roofline = {
        "kernel": "k5s_ntt_blks_ip",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBPS, 4),
        "traffic": stored_traffic(),
        "avg_us": round(1e6 * ip_s, 2),
        "launches": len(ip_ms),
        "key_switches_per_launch": 1,
        "algorithmic_bytes_per_launch": ks_bytes,
        "kernel_io_bytes_per_launch": ip_io_bytes,
        "kernel_io_frac": round(ip_io_bytes / ip_s / 1e9 / HBM_PEAK_GBPS, 4),
    }
    valu = stored_valu()
    if valu:
        roofline["valu"] = {"wave_insts_per_launch": valu[0], "frac": round(valu_frac(valu[0], ip_s), 4)}

    batched = None
    if not args.no_batched:
        batched = batched_numbers(P, ci, ctx, spec, d_rlk, args.batch_reps)
    boot = None if args.no_trace else boot_trace_numbers(args.trace_runs)
    serving = None if args.no_serve else serve_numbers(args.serve_requests, args.serve_budget_gib, "")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(spec, ct1, ct2, ctr, rot, rlk, rotk, args.cpu_seconds)

    # Whole step against the HBM roofline with per-op algorithmic bytes
    # (inputs + evk rows + outputs; intermediates on chip), and its VALU issue rate
    step_bytes = (_op_limbs("HMULT", L, k, beta) + _op_limbs("RESCALE", L, k, beta)
                  + _op_limbs("HROT", L, k, beta)) * limb
    path = {"bytes_per_step": step_bytes,
            "GBps": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
            "frac": round(step_bytes / (ms_per_step * 1e-3) / 8e12, 4)}
    if valu:
        path["valu_wave_insts_per_step"] = valu[1]
        path["valu_frac"] = round(valu_frac(valu[1], ms_per_step * 1e-3), 4)
    rec = {
        "metric": "key-switches/sec at N=2^16 (single-op HMult + rescale + HRot per step)",
        "value": round(value, 2),
        "unit": "key-switches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "hmult+rescale+hrot N=2^16 L=36 k=12 dnum=3, 2 key-switches/step",
                   "logN": 16, "L": L, "k": k, "dnum": spec.dnum, "mode": "single-op"},
        "hmult_latency_us": {"p50": round(float(np.percentile(lat, 50)), 2),
                             "p99": round(float(np.percentile(lat, 99)), 2),
                             "reps": int(len(lat))},
        "hmult_latency_us_n12_l4": small,
        "schedule": schedule,
        "path": path,
        "batched": batched,
        "boot_trace": boot,
        "serving": serving,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    ctx.close()


def small_hmult_latency(P, ci, reps):
    """Latency distribution of one HMult at N=2^12 with 4 + 1 primes, dnum 4:
    each call bracketed by events on its stream (a launch-latency-bound case),
    as a plain ckks_hmult call and as a one-job graph batch (graph_p50/p99)."""
    import torch
    spec = ci.get("n12_l4")
    rng = ci.Rng(spec.seed)
    L = spec.L_max
    ct1, ct2 = _dev(rng.polys(2, spec.q, spec.N)), _dev(rng.polys(2, spec.q, spec.N))
    rlk = _dev(rng.evk(spec))
    ctx = P.Context.from_spec(spec)
    ws = ctx.workspace("HMULT", L)
    out = torch.empty((2, L, spec.N), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def dist(call):
        for _ in range(20):
            call()
        torch.cuda.synchronize()
        lat = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            call()
            e1.record(stream)
            e1.synchronize()
            lat.append(e0.elapsed_time(e1) * 1e3)
        return np.array(lat)

    lat = dist(lambda: P.ckks_hmult(ctx.handle, ct1, ct2, L, rlk, out, ws, stream))
    # the same HMult as a one-job graph batch: one submission per call
    b = P.ckks_batch_create(ctx.handle, [dict(op=P.JOB["HMULT"], L=L, in0=ct1, in1=ct2, key=rlk, out=out)],
                            use_graph=True)
    glat = dist(lambda: P.ckks_batch_launch(b, stream))
    P.ckks_batch_destroy(b)
    ctx.close()
    return {"p50": round(float(np.percentile(lat, 50)), 2), "p99": round(float(np.percentile(lat, 99)), 2),
            "reps": int(reps),
            "graph_p50": round(float(np.percentile(glat, 50)), 2),
            "graph_p99": round(float(np.percentile(glat, 99)), 2)}


def _op_limbs(op, L, k, beta):
    """Algorithmic HBM limbs of one job: inputs + evk rows at level L + output."""
    if op == "RESCALE":
        return 2 * L + 2 * (L - 1)
    key = 2 * beta * (L + k)
    return {"KEYSWITCH": L, "HMULT": 4 * L, "HROT": 2 * L}[op] + key + 2 * L


def batched_numbers(P, ci, ctx, spec, d_rlk, reps):
    """Batched key-switches/s on the same GPU: (a) 8 HMults at L=36, each with
    its own pair of ciphertexts and one shared relinearisation key, as one
    batch (one captured graph) vs 8 single calls; (b) the 64-job mixed-level
    batch (levels uniform in 4..36; HMult 0.4, HRot 0.4 over 8 rotation keys,
    rescale 0.2) as one captured graph.  Each batch is timed with the default
    plan and again after ckks_batch_tune picked its plan and kernel schedule."""
    import torch
    N, L, k = spec.N, spec.L_max, spec.k
    limb = N * LIMB_BYTES
    stream = torch.cuda.current_stream()

    def timed(fn, n_ks):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return n_ks * reps / (time.perf_counter() - t0)

    def default_and_tuned(b, n_ks):
        default = timed(lambda: P.ckks_batch_launch(b, stream), n_ks)
        plan, _ = P.ckks_batch_tune(b, 2, stream)
        tuned = timed(lambda: P.ckks_batch_launch(b, stream), n_ks)
        log = [[p["jobs_per_launch"], p["streams"], p["split"], round(us, 1)]
               for p, us in P.ckks_batch_tune_log(b)]
        return default, tuned, dict(plan, schedule=P.ckks_batch_get_schedule(b), candidates_B_S_split_us=log)

    # (a) same work, batched vs single-op; every HMult has its own inputs
    rng = ci.Rng(6)
    pairs = [(_dev(rng.polys(2, spec.q, N)), _dev(rng.polys(2, spec.q, N))) for _ in range(8)]
    outs = [torch.empty((2, L, N), dtype=torch.int32, device="cuda") for _ in range(8)]
    ws = ctx.workspace("HMULT", L)
    single = timed(lambda: [P.ckks_hmult(ctx.handle, a, b, L, d_rlk, o, ws, stream)
                            for (a, b), o in zip(pairs, outs)], 8)
    b8 = P.ckks_batch_create(ctx.handle, [dict(op=P.JOB["HMULT"], L=L, in0=a, in1=b, key=d_rlk, out=o)
                                          for (a, b), o in zip(pairs, outs)], use_graph=True)
    batched8, tuned8, plan8 = default_and_tuned(b8, 8)
    P.ckks_batch_destroy(b8)
    del outs, ws, pairs

    # (b) the 64-job mixed batch
    keys_h, jobs_h = ci.batch_jobs(spec)
    keys = [_dev(kh) for kh in keys_h]
    jobs, n_ks, keep = [], 0, []
    per_op, key_level = 0, {}
    for j in jobs_h:
        Lj = j["L"]
        a = _dev(j["in0"])
        keep.append(a)
        bj = ctx.beta(Lj)
        if j["op"] == "HMULT":
            b = _dev(j["in1"])
            keep.append(b)
            o = torch.empty((2, Lj, N), dtype=torch.int32, device="cuda")
            jobs.append(dict(op=P.JOB["HMULT"], L=Lj, in0=a, in1=b, key=keys[j["key"]], out=o))
        elif j["op"] == "HROT":
            o = torch.empty((2, Lj, N), dtype=torch.int32, device="cuda")
            jobs.append(dict(op=P.JOB["HROT"], L=Lj, rot=j["rot"], in0=a, key=keys[j["key"]], out=o))
        else:
            o = torch.empty((2, Lj - 1, N), dtype=torch.int32, device="cuda")
            jobs.append(dict(op=P.JOB["RESCALE"], L=Lj, in0=a, out=o))
        if j["op"] != "RESCALE":
            n_ks += 1
            key_level[j["key"]] = max(key_level.get(j["key"], 0), Lj)
        per_op += _op_limbs(j["op"], Lj, k, bj)
        keep.append(o)
    # workload-compulsory: every distinct key read once (rows of its largest level)
    keys_once = sum(2 * ctx.beta(Lk) * (Lk + k) for Lk in key_level.values())
    key_per_op = sum(2 * ctx.beta(j["L"]) * (j["L"] + k) for j in jobs if j["op"] != P.JOB["RESCALE"])
    compulsory = per_op - key_per_op + keys_once
    b64 = P.ckks_batch_create(ctx.handle, jobs, use_graph=True)
    mixed, mixed_tuned, plan64 = default_and_tuned(b64, n_ks)
    P.ckks_batch_destroy(b64)
    launch_s = n_ks / mixed_tuned
    return {"hmult_L36_x8": {"single_op_ks_per_s": round(single, 1),
                             "batched_graph_ks_per_s": round(batched8, 1),
                             "tuned_ks_per_s": round(tuned8, 1), "tuned_plan": plan8,
                             "speedup": round(max(batched8, tuned8) / single, 3),
                             "inputs": "8 distinct ciphertext pairs, one shared relinearisation key"},
            "mixed_64_jobs_L4_36": {"ks_per_s": round(mixed, 1), "tuned_ks_per_s": round(mixed_tuned, 1),
                                    "tuned_plan": plan64, "key_switches": n_ks, "jobs": len(jobs), "graph": True,
                                    "per_op_bytes": per_op * limb, "compulsory_bytes": compulsory * limb,
                                    "per_op_GBps": round(per_op * limb / launch_s / 1e9, 1),
                                    "compulsory_GBps": round(compulsory * limb / launch_s / 1e9, 1),
                                    "compulsory_frac": round(compulsory * limb / launch_s / 8e12, 4)}}


def boot_trace_numbers(runs):
    """The bootstrapping-shaped trace at N=2^16 from L=36 (2^15 slots): two
    runs to warm up, then `runs` runs each timed on its own (synchronised
    before and after); ms per trace is their median (min and max beside it),
    eager and as one captured hipGraph replayed (its output checked bitwise
    against the eager run's)."""
    import torch
    import ckks_inputs as ci
    import paper_2512_18345_amd as P
    from paper_2512_18345_amd import trace
    torch.cuda.set_device(0)
    spec = ci.get("boot_trace_n16")
    shape = ci.BOOT_TRACE
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(spec.seed)
    ct = _dev(rng.polys(2, spec.q, spec.N))
    rots = sorted(set(shape["baby"]) | set(shape["giant"]))
    keys = {r: _dev(rng.evk(spec)) for r in rots}
    rlk = _dev(rng.evk(spec))
    pts = [_dev(rng.residues(spec.q, spec.N)) for _ in range(len(shape["baby"]) * len(shape["giant"]))]
    stream = torch.cuda.current_stream()

    def timed(fn):
        times = []
        for _ in range(runs):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        return float(np.median(times)), min(times), max(times), r

    for _ in range(2):
        trace.run(ctx, ct, spec.L_max, shape, keys, rlk, pts, stream)
    dt, dmin, dmax, (out, Lf) = timed(lambda: trace.run(ctx, ct, spec.L_max, shape, keys, rlk, pts, stream))
    nks = trace.key_switches(shape)
    # the same trace captured once as a hipGraph (stream capture through torch,
    # intermediates in the graph's pool) and replayed: one submission per trace
    graph = torch.cuda.CUDAGraph()
    gc.collect()  # no destructor (a freed context's hipFree) may run inside the capture
    gc.disable()
    try:
        with torch.cuda.graph(graph):
            gout, _ = trace.run(ctx, ct, spec.L_max, shape, keys, rlk, pts)
    finally:
        gc.enable()
    graph.replay()
    torch.cuda.synchronize()
    same = bool(torch.equal(gout, out))
    gdt, gmin, gmax, _ = timed(graph.replay)
    same = same and bool(torch.equal(gout, out))
    del graph
    ctx.close()
    ms = lambda x: round(x * 1e3, 3)
    return {"ms_per_trace": ms(dt), "ms_min_max": [ms(dmin), ms(dmax)], "key_switches": nks,
            "ks_per_s": round(nks / dt, 1), "L_start": spec.L_max, "L_end": Lf, "runs": runs,
            "graph_ms_per_trace": ms(gdt), "graph_ms_min_max": [ms(gmin), ms(gmax)],
            "graph_ks_per_s": round(nks / gdt, 1), "graph_equals_eager": same}


def serve_numbers(n_requests, budget_gib, sweep_budgets):
    """Serving loop under Poisson arrivals.  A request is b ~ U{1..32} jobs
    (key-switch or HMult, equally likely) at one N in {2^15, 2^16} and one level
    L ~ U{2..36}; request latency = last job's completion - arrival.  First a
    closed-loop flood measures the saturated job rate; then arrivals at 0.5,
    0.8 and 0.95 of it; then (sweep_budgets, GiB) saturated runs under smaller
    HBM budgets."""
    import random
    import torch
    import ckks_inputs as ci
    import paper_2512_18345_amd as P
    torch.cuda.set_device(0)
    specs = [ci.get("serve_n15"), ci.get("serve_n16")]
    ctxs = [P.Context.from_spec(s) for s in specs]
    rng = ci.Rng(5)
    keys = [_dev(rng.evk(s)) for s in specs]
    # one input pair per (N, L); a ring of output buffers per N
    ins = {}
    for c, s in enumerate(specs):
        full1, full2 = rng.polys(2, s.q, s.N), rng.polys(2, s.q, s.N)
        for L in range(2, s.L_max + 1):
            ins[(c, L)] = (_dev(full1[:, :L]), _dev(full2[:, :L]))
    RING = 256
    outs = [[torch.empty(2 * s.L_max * s.N, dtype=torch.int32, device="cuda") for _ in range(RING)]
            for s in specs]
    torch.cuda.synchronize()
    max_slots = 32
    counter = [0]

    def make_request(r):
        c = r.randrange(2)
        L = r.randint(2, specs[c].L_max)
        b = r.randint(1, 32)
        op = P.JOB["KEYSWITCH"] if r.random() < 0.5 else P.JOB["HMULT"]
        a1, a2 = ins[(c, L)]
        jobs = []
        for _ in range(b):
            o = outs[c][counter[0] % RING]
            counter[0] += 1
            if op == P.JOB["KEYSWITCH"]:
                jobs.append(dict(op=op, L=L, in0=a1[0], key=keys[c], out=o))
            else:
                jobs.append(dict(op=op, L=L, in0=a1, in1=a2, key=keys[c], out=o))
        return c, jobs

    def run(n_req, rate, seed, srv):
        r = random.Random(seed)
        reqs = [make_request(r) for _ in range(n_req)]
        first = P.ckks_server_stats(srv)["submitted"]
        spans = []
        t0 = time.perf_counter()
        next_t = t0
        for c, jobs in reqs:
            if rate:
                next_t += r.expovariate(rate)
                while time.perf_counter() < next_t:
                    pass
            t_first = None
            for j in jobs:
                tk = P.ckks_server_submit(srv, c, j)
                t_first = tk if t_first is None else t_first
            spans.append((t_first, len(jobs)))
        P.ckks_server_drain(srv)
        wall = time.perf_counter() - t0
        n_jobs = sum(n for _, n in spans)
        sub, done = P.ckks_server_times(srv, first, n_jobs)
        lat = []
        for t_first, n in spans:
            i = t_first - first
            lat.append(max(done[i:i + n]) - sub[i])
        lat = np.array(lat)
        return {"requests": n_req, "jobs": n_jobs, "jobs_per_s": round(n_jobs / wall, 1),
                "p50_us": round(float(np.percentile(lat, 50)), 1),
                "p99_us": round(float(np.percentile(lat, 99)), 1)}

    srv = P.ckks_server_create([c.handle for c in ctxs], int(budget_gib * (1 << 30)), max_slots)
    run(20, 0, 1, srv)  # warm-up
    sat = run(n_requests, 0, 2, srv)
    mean_b = 16.5
    loads = {}
    for rho in (0.5, 0.8, 0.95):
        loads[str(rho)] = run(n_requests, rho * sat["jobs_per_s"] / mean_b, 3 + int(rho * 100), srv)
    st = P.ckks_server_stats(srv)
    P.ckks_server_destroy(srv)
    res = {"saturated": sat, "poisson": loads, "max_slots": max_slots,
           "budget_bytes": st["budget_bytes"], "peak_bytes": st["peak_bytes"], "batches": st["batches"]}
    # saturated throughput under smaller HBM budgets (admission by scratch bytes)
    budgets = {}
    for gib in [float(v) for v in sweep_budgets.split(",") if v.strip()]:
        s2 = P.ckks_server_create([c.handle for c in ctxs], int(gib * (1 << 30)), max_slots)
        r = run(max(n_requests // 2, 20), 0, 7, s2)
        st2 = P.ckks_server_stats(s2)
        r.update(peak_bytes=st2["peak_bytes"], batches=st2["batches"], rejected=st2["rejected"])
        budgets[str(gib)] = r
        P.ckks_server_destroy(s2)
    if budgets:
        res["budget_sweep_gib"] = budgets
    for c in ctxs:
        c.close()
    return res


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return None


def cpu_baseline(spec, ct1, ct2, ctr, rot, rlk, rotk, budget_s):
    """The oracle, as it stands, on the host cores: whole steps (HMult,
    rescale, HRot at the same sizes) on all cores until about budget_s
    seconds, then one whole step on one thread."""
    import oracle as O
    par = O.Params.from_spec(spec)
    L = spec.L_max
    O.ntt(par, ct1[0][:1], spec.q[:1])  # build + load the C loops outside the timing
    cores = O.num_threads()

    def one_step():
        m = O.hmult(par, ct1, ct2, L, rlk)
        O.rescale(par, m, L)
        O.hrot(par, ctr, L, rot, rotk)

    steps = 0
    t0 = time.perf_counter()
    while True:
        one_step()
        steps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    O.set_num_threads(1)
    t1 = time.perf_counter()
    one_step()
    dt1 = time.perf_counter() - t1
    O.set_num_threads(cores)
    return {"value": round(2 * steps / dt, 4), "unit": "key-switches/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{steps} full steps (HMult + rescale + HRot at N=2^16, L=36) in {dt:.1f} s",
            "single_thread": {"value": round(2 / dt1, 4), "unit": "key-switches/s", "cores": 1,
                              "sample": f"1 full step in {dt1:.1f} s"},
            "cpu_model": cpu_model()}


if __name__ == "__main__":
    main()
