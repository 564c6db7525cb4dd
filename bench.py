"""Benchmark: key-switches per second at N=2^16 on one MI355X.

One step is one pass of the hot path over one batch of synthetic input at
N=2^16, L=36 (36 + 12 primes < 2^30, dnum 3): HMult with relinearisation,
rescale of its result, and HRot by a uniform rotation; 2 key-switches per
step.  Inputs are uniform residues from the seeded generator, already in
HBM when the timed region starts.  Also reported: HMult latency p50/p99
(each call bracketed by HIP events), the roofline position of the dominant
kernel, and the CPU oracle timed on a bounded sample on the host cores.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
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

LIMB_BYTES = 4  # uint32 residues


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--latency-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-reps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
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


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(batch-level data parallelism across GPUs needs no collective and is not run here).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import ckks_inputs as ci
    import paper_2512_18345_amd as P

    torch.cuda.set_device(0)
    spec = ci.get("n16_l36")
    L, N, k = spec.L_max, spec.N, spec.k
    rng = ci.Rng(spec.seed)

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32).copy()).cuda()

    ct1 = rng.polys(2, spec.q, N)
    ct2 = rng.polys(2, spec.q, N)
    ctr = rng.polys(2, spec.q, N)
    rot = rng.rotation(N)
    rlk = rng.evk(spec)
    rotk = rng.evk(spec)
    d_ct1, d_ct2, d_ctr, d_rlk, d_rotk = map(dev, (ct1, ct2, ctr, rlk, rotk))
    ctx = P.Context.from_spec(spec)
    h = ctx.handle
    ws = ctx.workspace("HMULT", L)
    ws_rot = ctx.workspace("HROT", L)
    ws_rs = ctx.workspace("RESCALE", L)
    out_m = torch.empty((2, L, N), dtype=torch.int32, device="cuda")
    out_r = torch.empty((2, L, N), dtype=torch.int32, device="cuda")
    out_s = torch.empty((2, L - 1, N), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        P.ckks_hmult(h, d_ct1, d_ct2, L, d_rlk, out_m, ws, stream)
        P.ckks_rescale(h, out_m, L, out_s, ws_rs, stream)
        P.ckks_hrot(h, d_ctr, L, rot, d_rotk, out_r, ws_rot, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # Dominant kernel: NTT block pass fused with the key inner product (stage 2
    # of key-switching), timed by events around each of its launches on the
    # stream it runs on, inside the timed region.
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

    beta = ctx.beta(L)
    R = L + k
    limb = N * LIMB_BYTES
    # per launch: the beta*R ModUp rows in, the 2*beta*R key rows in, the 2*R
    # accumulator rows out
    ip_bytes = (3 * beta + 2) * R * limb
    ip_us = 1e3 * float(np.mean(ip_ms))
    achieved = ip_bytes / (ip_us * 1e-6) / 1e9
    roofline = {
        "kernel": "k5_ntt_blks_ip",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": 8000.0,
        "unit": "GB/s",
        "frac": round(achieved / 8000.0, 4),
        "traffic": None,
        "avg_us": round(ip_us, 2),
        "launches": len(ip_ms),
        "bytes_per_launch": ip_bytes,
    }

    batched = None
    if not args.no_batched:
        batched = batched_numbers(P, ci, ctx, spec, dev, d_ct1, d_ct2, d_rlk, args.batch_reps)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(spec, ct1, ct2, ctr, rot, rlk, rotk, args.cpu_seconds)

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
        "batched": batched,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    ctx.close()


def batched_numbers(P, ci, ctx, spec, dev, d_ct1, d_ct2, d_rlk, reps):
    """Batched key-switches/s on the same GPU: (a) 8 HMults at L=36, one
    batch (one captured graph) vs 8 single calls; (b) the 64-job mixed-level
    batch (levels uniform in 4..36; HMult 0.4, HRot 0.4 over 8 rotation keys,
    rescale 0.2) as one captured graph."""
    import torch
    N, L = spec.N, spec.L_max
    stream = torch.cuda.current_stream()

    def timed(fn, n_ks):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return n_ks * reps / (time.perf_counter() - t0)

    # (a) same work, batched vs single-op
    outs = [torch.empty((2, L, N), dtype=torch.int32, device="cuda") for _ in range(8)]
    ws = ctx.workspace("HMULT", L)
    single = timed(lambda: [P.ckks_hmult(ctx.handle, d_ct1, d_ct2, L, d_rlk, o, ws, stream) for o in outs], 8)
    b8 = P.ckks_batch_create(ctx.handle, [dict(op=P.JOB["HMULT"], L=L, in0=d_ct1, in1=d_ct2, key=d_rlk,
                                               out=o) for o in outs], use_graph=True)
    batched8 = timed(lambda: P.ckks_batch_launch(b8, stream), 8)
    P.ckks_batch_destroy(b8)
    del outs, ws

    # (b) the 64-job mixed batch
    rng = ci.Rng(3)
    keys = [dev(rng.evk(spec)) for _ in range(9)]  # 8 rotation keys + the relinearisation key
    jobs, n_ks, keep = [], 0, []
    for _ in range(64):
        Lj = int(rng.integers(4, 37))
        u = float(rng.integers(0, 10)) / 10.0
        a = dev(rng.polys(2, spec.q[:Lj], N))
        keep.append(a)
        if u < 0.4:
            b = dev(rng.polys(2, spec.q[:Lj], N))
            keep.append(b)
            o = torch.empty((2, Lj, N), dtype=torch.int32, device="cuda")
            jobs.append(dict(op=P.JOB["HMULT"], L=Lj, in0=a, in1=b, key=keys[8], out=o))
            n_ks += 1
        elif u < 0.8:
            o = torch.empty((2, Lj, N), dtype=torch.int32, device="cuda")
            r = int(rng.integers(0, 8))
            jobs.append(dict(op=P.JOB["HROT"], L=Lj, rot=1 + r, in0=a, key=keys[r], out=o))
            n_ks += 1
        else:
            o = torch.empty((2, Lj - 1, N), dtype=torch.int32, device="cuda")
            jobs.append(dict(op=P.JOB["RESCALE"], L=Lj, in0=a, out=o))
        keep.append(o)
    b64 = P.ckks_batch_create(ctx.handle, jobs, use_graph=True)
    mixed = timed(lambda: P.ckks_batch_launch(b64, stream), n_ks)
    P.ckks_batch_destroy(b64)
    return {"hmult_L36_x8": {"single_op_ks_per_s": round(single, 1),
                             "batched_graph_ks_per_s": round(batched8, 1),
                             "speedup": round(batched8 / single, 3)},
            "mixed_64_jobs_L4_36": {"ks_per_s": round(mixed, 1), "key_switches": n_ks,
                                    "jobs": 64, "graph": True}}


def cpu_baseline(spec, ct1, ct2, ctr, rot, rlk, rotk, budget_s):
    """The oracle, as it stands, on the host cores: whole steps (HMult,
    rescale, HRot at the same sizes) until about budget_s seconds."""
    import oracle as O
    par = O.Params.from_spec(spec)
    L = spec.L_max
    O.ntt(par, ct1[0][:1], spec.q[:1])  # build + load the C loops outside the timing
    steps = 0
    t0 = time.perf_counter()
    while True:
        m = O.hmult(par, ct1, ct2, L, rlk)
        O.rescale(par, m, L)
        O.hrot(par, ctr, L, rot, rotk)
        steps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": round(2 * steps / dt, 4), "unit": "key-switches/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} full steps (HMult + rescale + HRot at N=2^16, L=36) in {dt:.1f} s"}


if __name__ == "__main__":
    main()
