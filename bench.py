#!/usr/bin/env python3
"""Benchmark of the gfx950 Pohlig-Hellman generator (one GPU).

Headline workload: 4096 seeded 32-bit instances (distinct admissible primes
n in [2^31, 2^32), e drawn from {9, 17} coprime to n - 1, start position 0),
2^18 draws each per step -- 1,073,741,824 uniforms per step written to HBM as
u32 ciphertexts plus FP64 uniforms.  A step is one batched persistent
launch over all 4096 streams; each step continues every stream where the
previous one ended and overwrites the same output arrays.  The same
workload is also timed in the plain form (one launch per instance), and the
CPU oracle is timed on a bounded sample of it.

Prints one JSON line.  `value` is whole-job throughput (Guniforms/s) with
all inputs resident on the device.
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

SEED_B = 0x14112484 + 1
N_INST = 4096
PER = 1 << 18
HBM_PEAK_GBS = 8000.0         # MI355X published HBM3E bandwidth
ALU_PEAK_OPS = 256 * 64 * 2.4e9  # 256 CUs x 64 lanes x 2.4 GHz, one VALU op per lane per clock


def algorithmic_ops_32(e):
    """VALU operations per width-32 draw in the minimal instruction model of
    algorithm (9): skip 6, message 4, Montgomery products 6 each (e = 9: 5,
    e = 17: 6, e = 3: 3, e = 5: 4), uniform 5."""
    chain = {3: 3, 5: 4, 9: 5, 17: 6}[int(e)]
    return 6 + 4 + 6 * chain + 5


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(e_arr, n_arr, target_s=12.0):
    """The oracle on the host's cores over a bounded sample of the headline
    workload (the first M instances, 2^18 draws each from position 0)."""
    import oracle
    nthreads = min(os.cpu_count() or 1, 16)
    p, a = oracle.lcg_params(32)
    # calibrate on 8 instances
    t0 = time.perf_counter()
    oracle.generate_many(p, a, n_arr[:8], e_arr[:8], 0, 1, np.full(8, PER, dtype=np.uint64), nthreads=min(8, nthreads))
    dt = time.perf_counter() - t0
    per_inst_thread_s = dt * min(8, nthreads) / 8
    m = int(max(nthreads, min(N_INST, target_s * nthreads / max(per_inst_thread_s, 1e-9))))
    m = (m // nthreads) * nthreads or nthreads
    done = 0
    t0 = time.perf_counter()
    while done < m:
        b = min(256, m - done)
        oracle.generate_many(p, a, n_arr[done:done + b], e_arr[done:done + b], 0, 1,
                             np.full(b, PER, dtype=np.uint64), want_c=True, want_r=True, nthreads=nthreads)
        done += b
    el = time.perf_counter() - t0
    draws = m * PER
    return {"value": draws / el / 1e9, "unit": "Guniforms/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d of the 4096 instances x 2^18 draws from position 0 (%d draws), %.1f s" % (m, draws, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="autotune the launch shape before timing")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU share of the generator "
              "(instances shard across GPUs with no communication); --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1411_2484_amd as ph

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    ctx = ph.Context(0, max_instances=N_INST)
    ids = ctx.seed_instances(32, SEED_B, N_INST, (9, 17), 0, 0)
    params = [ctx.get_params(int(i)) for i in ids]
    n_arr = np.array([p[0] for p in params], dtype=np.uint64)
    e_arr = np.array([p[1] for p in params], dtype=np.uint64)
    total = N_INST * PER
    c32 = torch.empty(total, dtype=torch.int32, device=dev)
    r = torch.empty(total, dtype=torch.float64, device=dev)
    reqs = ph.make_requests(ids, [PER] * N_INST, np.arange(N_INST, dtype=np.uint64) * PER)
    if args.autotune:
        log("autotune: %s" % ctx.autotune(1 << 27))
    tuning = ctx.get_tuning()

    def step(mode=ph.PHPRNG_MODE_PERSISTENT):
        ctx.generate(reqs, c32, None, r, capacity=total, mode=mode)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing_reset()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, kcalls = ctx.timing_read()
    ms_per_step = wall * 1e3 / args.steps
    value = total * args.steps / wall / 1e9
    kernel_ms = kms / max(kcalls, 1)
    log("persistent: %.3f ms/step wall, %.3f ms kernel, %.1f Guniforms/s" % (ms_per_step, kernel_ms, value))

    plain = None
    if not args.no_plain:
        step(ph.PHPRNG_MODE_PLAIN)
        torch.cuda.synchronize()
        ctx.timing_reset()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            step(ph.PHPRNG_MODE_PLAIN)
        torch.cuda.synchronize()
        pw = time.perf_counter() - t0
        pk, pc = ctx.timing_read()
        plain = {"value": total * args.plain_steps / pw / 1e9, "unit": "Guniforms/s",
                 "ms_per_step": pw * 1e3 / args.plain_steps, "kernel_ms": pk / max(pc, 1),
                 "launches_per_step": N_INST}
        log("plain: %s" % plain)

    # roofline of the generation kernel: algorithmic bytes / ops per launch
    ops_per_draw = float(np.mean([algorithmic_ops_32(e) for e in e_arr]))
    bytes_per_draw = 12.0
    achieved_gbs = total * bytes_per_draw / (kernel_ms * 1e-3) / 1e9
    achieved_ops = total * ops_per_draw / (kernel_ms * 1e-3)
    hbm = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": None}
    alu = {"bound": "alu", "achieved": achieved_ops / 1e12, "peak": ALU_PEAK_OPS / 1e12, "unit": "Top/s",
           "frac": achieved_ops / ALU_PEAK_OPS, "ops_per_draw": ops_per_draw}
    roof, other = (hbm, alu) if hbm["frac"] >= alu["frac"] else (alu, hbm)
    roof = dict(roof)
    roof["kernel"] = "gen_persistent"
    roof["kernel_ms"] = kernel_ms
    roof["units_per_launch"] = total

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(e_arr, n_arr)
        log("cpu baseline: %s" % cpu)

    out = {
        "metric": "Guniforms/s (32/64-bit moduli), batched vs plain launch; serve p50/p99 latency",
        "value": value,
        "unit": "Guniforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "4096 seeded 32-bit instances x 2^18 draws per step (u32 c + f64 R to HBM), "
                        "one batched persistent launch per step",
            "instances": N_INST, "draws_per_instance": PER, "width": 32, "e_set": [9, 17],
            "start_position": 0, "tuning": tuning,
        },
        "plain": plain,
        "roofline": roof,
        "roofline_other": other,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
