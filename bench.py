#!/usr/bin/env python3
"""Benchmark of the gfx950 Pohlig-Hellman generator (one GPU).

Headline workload: 4096 seeded 32-bit instances (distinct admissible primes
n in [2^31, 2^32), e drawn from {9, 17} coprime to n - 1, start position 0),
2^18 draws each per step -- 1,073,741,824 uniforms per step written to HBM as
FP64 uniforms (a variant also writes the u32 ciphertexts).  A step is one batched persistent
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
    workload: batches of 256 of the instances, 2^18 draws each from position
    0, cycling over the 4096 instances until about target_s seconds."""
    import oracle
    nthreads = min(os.cpu_count() or 1, 16)
    p, a = oracle.lcg_params(32)
    done_inst = 0
    t0 = time.perf_counter()
    while True:
        lo = done_inst % N_INST
        b = min(256, N_INST - lo)
        oracle.generate_many(p, a, n_arr[lo:lo + b], e_arr[lo:lo + b], 0, 1, np.full(b, PER, dtype=np.uint64),
                             want_c=True, want_r=True, nthreads=nthreads)
        done_inst += b
        el = time.perf_counter() - t0
        if el >= target_s:
            break
    draws = done_inst * PER
    return {"value": draws / el / 1e9, "unit": "Guniforms/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d instance-streams of the headline workload (2^18 draws each from position 0, "
                      "%d draws) in %.1f s" % (done_inst, draws, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-ciphertexts", action="store_true", help="skip the u32 + f64 output variant")
    ap.add_argument("--autotune", action="store_true", help="autotune the launch shape before timing")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="first run one device copy of this many GiB (known-size kernel for traffic counters)")
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
    r = torch.empty(total, dtype=torch.float64, device=dev)
    reqs = ph.make_requests(ids, [PER] * N_INST, np.arange(N_INST, dtype=np.uint64) * PER)
    if args.calib_copy_gib > 0:
        nel = int(args.calib_copy_gib * (1 << 30) / 8)
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (nel * 8, nel * 8))
        del src, dst
    if args.autotune:
        log("autotune: %s" % ctx.autotune(1 << 27))
    tuning = ctx.get_tuning()

    def measure(steps, warmup, mode, c32=None):
        """Time `steps` generation calls; returns (wall ms/step, kernel ms/call)."""
        for _ in range(warmup):
            ctx.generate(reqs, c32, None, r, capacity=total, mode=mode)
        torch.cuda.synchronize()
        ctx.timing_reset()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.generate(reqs, c32, None, r, capacity=total, mode=mode)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms, kcalls = ctx.timing_read()
        return wall * 1e3 / steps, kms / max(kcalls, 1)

    # headline: FP64 uniforms only, as the workload defines its output
    ms_per_step, kernel_ms = measure(args.steps, args.warmup, ph.PHPRNG_MODE_PERSISTENT)
    value = total / (ms_per_step * 1e-3) / 1e9
    log("persistent: %.3f ms/step wall, %.3f ms kernel, %.1f Guniforms/s" % (ms_per_step, kernel_ms, value))

    plain = None
    if not args.no_plain:
        pms, pk = measure(args.plain_steps, 1, ph.PHPRNG_MODE_PLAIN)
        plain = {"value": total / (pms * 1e-3) / 1e9, "unit": "Guniforms/s", "ms_per_step": pms,
                 "kernel_ms": pk, "launches_per_step": N_INST, "speedup_of_batched": pms / ms_per_step}
        log("plain: %s" % plain)

    with_c = None
    if not args.no_ciphertexts:
        c32 = torch.empty(total, dtype=torch.int32, device=dev)
        cms, ck = measure(max(args.steps // 2, 1), 1, ph.PHPRNG_MODE_PERSISTENT, c32)
        with_c = {"value": total / (cms * 1e-3) / 1e9, "unit": "Guniforms/s", "ms_per_step": cms,
                  "kernel_ms": ck, "outputs": "u32 c + f64 R (12 B per draw)",
                  "hbm_gbs": total * 12.0 / (ck * 1e-3) / 1e9}
        log("with ciphertexts: %s" % with_c)
        del c32

    # roofline of the generation kernel: algorithmic bytes / ops per launch
    ops_per_draw = float(np.mean([algorithmic_ops_32(e) for e in e_arr]))
    bytes_per_draw = 8.0
    achieved_gbs = total * bytes_per_draw / (kernel_ms * 1e-3) / 1e9
    achieved_ops = total * ops_per_draw / (kernel_ms * 1e-3)
    hbm = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": None, "bytes_per_draw": bytes_per_draw}
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
        "dtype": "u32/f64",
        "data": "synthetic",
        "config": {
            "workload": "4096 seeded 32-bit instances x 2^18 draws per step (1.07e9 FP64 uniforms to HBM), "
                        "one batched persistent launch per step",
            "instances": N_INST, "draws_per_instance": PER, "width": 32, "e_set": [9, 17],
            "start_position": 0, "tuning": tuning,
        },
        "plain": plain,
        "with_ciphertexts": with_c,
        "roofline": roof,
        "roofline_other": other,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
