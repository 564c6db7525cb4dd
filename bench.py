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
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def main():
    args = parse()
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
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
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

    # Dominant kernel: the evaluation-key inner product (stage 2), one kernel per call.
    beta = ctx.beta(L)
    R = L + k
    M = torch.randint(0, 2 ** 29, (beta, R, N), dtype=torch.int32, device="cuda")
    acc = torch.empty((2, R, N), dtype=torch.int32, device="cuda")
    for _ in range(3):
        P.ckks_inner_product(h, M, L, d_rlk, acc, stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.kernel_reps):
        P.ckks_inner_product(h, M, L, d_rlk, acc, stream)
    e1.record(stream)
    e1.synchronize()
    ip_us = e0.elapsed_time(e1) * 1e3 / args.kernel_reps
    limb = N * LIMB_BYTES
    ip_bytes = (beta * R + 2 * beta * R + 2 * R) * limb  # read M and the key rows, write acc
    achieved = ip_bytes / (ip_us * 1e-6) / 1e9
    roofline = {
        "kernel": "k_inner_product",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": 8000.0,
        "unit": "GB/s",
        "frac": round(achieved / 8000.0, 4),
        "traffic": None,
        "avg_us": round(ip_us, 2),
        "bytes_per_launch": ip_bytes,
    }

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
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    ctx.close()


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
