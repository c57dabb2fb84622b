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


KERNEL_SOURCES = ["paper_1411_2484_amd/csrc/kernels.hip", "paper_1411_2484_amd/csrc/arith.hpp",
                  "paper_1411_2484_amd/csrc/layout.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gen_persistent_traffic.json")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel sources (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t.get("traffic_bytes_per_launch")


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
            "ns_per_uniform_per_core": el * nthreads / draws * 1e9,
            "sample": "%d instance-streams of the headline workload (2^18 draws each from position 0, "
                      "%d draws) in %.1f s" % (done_inst, draws, el)}


def common_line(metric_value, unit, steps, warmup, ms_per_step, config, **extra):
    out = {
        "metric": "Guniforms/s (32/64-bit moduli), batched vs plain launch; serve p50/p99 latency",
        "value": metric_value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32/u64/f64", "data": "synthetic", "config": config,
    }
    out.update(extra)
    return out


def timed_steps(ctx, torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ctx.timing_reset()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, kc = ctx.timing_read()
    return wall * 1e3 / steps, kms / max(kc, 1)


def workload_a(args, torch, ph):
    """One seeded 32-bit instance, 10^6 draws per step (u32 c + f64 R)."""
    dev = torch.device("cuda:0")
    ctx = ph.Context(0, max_instances=1)
    ids = ctx.seed_instances(32, 0x14112484, 1, (9, 17), 0, 0)
    N = 10 ** 6
    c32 = torch.empty(N, dtype=torch.int32, device=dev)
    r = torch.empty(N, dtype=torch.float64, device=dev)
    reqs = ph.make_requests(ids, [N], [0])
    res = {}
    for name, mode in (("persistent", ph.PHPRNG_MODE_PERSISTENT), ("plain", ph.PHPRNG_MODE_PLAIN)):
        ms, kms = timed_steps(ctx, torch, lambda: ctx.generate(reqs, c32, None, r, mode=mode), args.steps,
                              args.warmup)
        res[name] = {"ms_per_step": ms, "kernel_ms": kms, "value": N / (ms * 1e-3) / 1e9}
    ctx.close()
    return common_line(res["persistent"]["value"], "Guniforms/s", args.steps, args.warmup,
                       res["persistent"]["ms_per_step"],
                       {"workload": "1 seeded 32-bit instance x 10^6 draws from position 0 (u32 c + f64 R)"},
                       plain=res["plain"], persistent=res["persistent"])


def workload_c(args, torch, ph):
    """65,536 seeded 32-bit instances, log-uniform stream lengths in
    [2^10, 2^22], random starts in [0, 2^40), one persistent launch per step.
    Outputs (u32 c + f64 R) go to a reused arena of 2^32 elements: streams
    are placed one after another and wrap to the start of the arena."""
    dev = torch.device("cuda:0")
    nin = 65536
    ctx = ph.Context(0, max_instances=nin)
    ids = ctx.seed_instances(32, 0x14112484 + 2, nin, (9, 17), 0, 1 << 40)
    rng = np.random.default_rng(0x14112484 + 2)
    lens = np.floor(2.0 ** (10 + 12 * rng.random(nin))).astype(np.uint64)
    arena = 1 << 32
    offs = np.zeros(nin, dtype=np.uint64)
    cur = 0
    for i in range(nin):
        if cur + int(lens[i]) > arena:
            cur = 0
        offs[i] = cur
        cur += int(lens[i])
    total = int(lens.sum())
    c32 = torch.empty(arena, dtype=torch.int32, device=dev)
    r = torch.empty(arena, dtype=torch.float64, device=dev)
    reqs = ph.make_requests(ids, lens, offs)
    steps = max(2, args.steps // 5)
    ms, kms = timed_steps(ctx, torch, lambda: ctx.generate(reqs, c32, None, r, capacity=arena), steps, 1)
    rms, rkms = timed_steps(ctx, torch, lambda: ctx.generate(reqs, None, None, r, capacity=arena), steps, 1)
    # draw-weighted algorithmic op count over the instances' exponents
    es = np.array([ctx.get_params(int(i))[1] for i in ids])
    ops = float(np.sum(lens.astype(np.float64) * np.array([algorithmic_ops_32(e) for e in es])) / total)
    ctx.close()
    value = total / (ms * 1e-3) / 1e9
    gbs = total * 12.0 / (kms * 1e-3) / 1e9
    alu = total * ops / (kms * 1e-3)
    roofs = {"alu": {"achieved": alu / 1e12, "peak": ALU_PEAK_OPS / 1e12, "unit": "Top/s",
                     "frac": alu / ALU_PEAK_OPS, "ops_per_draw": ops},
             "hbm": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "bytes_per_draw": 12.0}}
    return common_line(value, "Guniforms/s", steps, 1, ms,
                       {"workload": "65536 seeded 32-bit instances, log-uniform lengths 2^10..2^22 (%d draws), "
                                    "random starts in [0, 2^40), one persistent launch, u32 c + f64 R" % total},
                       kernel_ms=kms, hbm_gbs=gbs, roofline_fractions=roofs,
                       uniforms_only={"value": total / (rms * 1e-3) / 1e9, "kernel_ms": rkms})


def workload_d(args, torch, ph):
    """1024 64-bit + 1024 32-bit instances x 2^20 draws, mixed in one launch."""
    dev = torch.device("cuda:0")
    ctx = ph.Context(0, max_instances=2048)
    i64 = ctx.seed_instances(64, 0x14112484 + 3, 1024, (9, 17), 0, 0)
    i32 = ctx.seed_instances(32, 0x14112484 + 4, 1024, (9, 17), 0, 0)
    per = 1 << 20
    total = 2048 * per
    c32 = torch.empty(total, dtype=torch.int32, device=dev)
    c64 = torch.empty(total, dtype=torch.int64, device=dev)
    r = torch.empty(total, dtype=torch.float64, device=dev)
    steps = max(2, args.steps // 4)
    res = {}
    for name, ids in (("mixed", np.concatenate([i64, i32])), ("w64_only", i64), ("w32_only", i32)):
        reqs = ph.make_requests(ids, [per] * len(ids), np.arange(len(ids), dtype=np.uint64) * per)
        ms, kms = timed_steps(ctx, torch, lambda: ctx.generate(reqs, c32, c64, r, capacity=total), steps, 1)
        res[name] = {"value": len(ids) * per / (ms * 1e-3) / 1e9, "ms_per_step": ms, "kernel_ms": kms}
    ctx.close()
    return common_line(res["mixed"]["value"], "Guniforms/s", steps, 1, res["mixed"]["ms_per_step"],
                       {"workload": "1024 64-bit (n in [2^62, 2^63)) + 1024 32-bit instances x 2^20 draws, one "
                                    "mixed persistent launch, u32/u64 c + f64 R"}, **res)


def workload_e(args, torch, ph):
    """Serving: 10^6 resident instances (900,000 32-bit, 100,000 64-bit),
    open-loop Poisson arrivals, each request log-uniform 2^8..2^20 FP64
    uniforms from a uniformly chosen instance, continuous batching."""
    n32, n64 = args.serve_instances * 9 // 10, args.serve_instances // 10
    ctx = ph.Context(0, max_instances=n32 + n64)
    t0 = time.perf_counter()
    ctx.seed_instances(32, 0x14112484 + 5, n32, (9, 17), 0, 1 << 40)
    ctx.seed_instances(64, 0x14112484 + 6, n64, (9, 17), 0, 1 << 32)
    log("serve: %d instances seeded in %.1f s" % (n32 + n64, time.perf_counter() - t0))
    srv = ph.Server(ctx, arena_doubles=args.serve_arena, streams=args.serve_streams,
                    max_inflight=args.serve_inflight)
    # untimed warm-up: first-use costs (staging slots, pinned buffers, the
    # per-instance scratch) stay out of the first load point
    wrng = np.random.default_rng(0x14112484 + 8)
    warm = np.zeros(2000, dtype=ph.ARRIVAL_DTYPE)
    warm["t_ns"] = np.cumsum(wrng.exponential(1e4, warm.size)).astype(np.int64)
    warm["instance"] = wrng.integers(0, n32 + n64, warm.size)
    warm["count"] = np.floor(2.0 ** (8 + 12 * wrng.random(warm.size))).astype(np.uint64)
    srv.replay(warm)
    rng = np.random.default_rng(0x14112484 + 7)
    points = []
    for lam in args.serve_rates:
        n = int(min(args.serve_max_requests, max(2000, lam * args.serve_seconds)))
        arr = np.zeros(n, dtype=ph.ARRIVAL_DTYPE)
        arr["t_ns"] = np.cumsum(rng.exponential(1e9 / lam, n)).astype(np.int64)
        arr["instance"] = rng.integers(0, n32 + n64, n)
        arr["count"] = np.floor(2.0 ** (8 + 12 * rng.random(n))).astype(np.uint64)
        srv.counters(reset=True)
        lat, adm, wall = srv.replay_detail(arr)
        cnt = srv.counters(reset=True)
        draws = int(arr["count"].sum())
        pt = {"rate_req_s": lam, "requests": n, "uniforms_per_s": draws / wall / 1e9,
              "p50_ms": float(np.percentile(lat, 50)) / 1e6, "p99_ms": float(np.percentile(lat, 99)) / 1e6,
              "admit_p50_ms": float(np.percentile(adm, 50)) / 1e6, "admit_p99_ms": float(np.percentile(adm, 99)) / 1e6,
              "offered_guniforms_s": float(draws / (arr["t_ns"][-1] * 1e-9) / 1e9), "wall_s": wall,
              "batches": cnt["batches"], "requests_per_batch": cnt["requests"] / max(cnt["batches"], 1),
              "launch_us_mean": cnt["launch_ns"] / max(cnt["batches"], 1) / 1e3,
              "launch_us_max": cnt["launch_ns_max"] / 1e3,
              "form_us_mean": cnt["form_ns"] / max(cnt["batches"], 1) / 1e3,
              "retire_us_mean": cnt["retire_ns"] / max(cnt["batches"], 1) / 1e3,
              "arena_stalls": cnt["arena_stalls"],
              "arena_peak": cnt["arena_peak"]}
        log("serve: %s" % pt)
        points.append(pt)
    srv.close()
    ctx.close()
    best = max(points, key=lambda p: p["uniforms_per_s"])
    return common_line(best["uniforms_per_s"], "Guniforms/s", len(points), 0, None,
                       {"workload": "serving: %d resident instances (90%% 32-bit, 10%% 64-bit), Poisson arrivals, "
                                    "log-uniform 2^8..2^20 FP64 uniforms per request" % (n32 + n64),
                        "streams": args.serve_streams, "inflight": args.serve_inflight or min(args.serve_streams + 1, 6)},
                       serve=points)


BATTERY_KEYS_PER_DRAW = 1 + 1 / 2 + 1 / 3 + 1 / 4 + 1 / 5   # frequency + serial 2..5 histogram keys
# per 128-block chunk, the counting stage writes and reads 2 slices of 159
# partitions x 2^15 u32 counts and updates 159 x 2^15 u64 histogram cells
BATTERY_COUNT_FIXED_BYTES = 2 * (159 * 2 * (1 << 15) * 4) + 2 * (159 * (1 << 15) * 8)
BATTERY_BYTES_PER_DRAW = {  # algorithmic HBM bytes per tested uniform, per battery kernel
    "hist": 8.0 + 1.0 / 8 + 2 * BATTERY_KEYS_PER_DRAW,  # read R, write one bit and 2-byte bucket keys
    "collision": 8.0,           # read R
    "runs": 1.0 / 8,            # read the bits
    "fft_pass1": 16.0,          # read R, write 8 B of complex rows per uniform
    "fft_pass2": 8.0,           # read the rows
    "hist_count": 2 * BATTERY_KEYS_PER_DRAW + BATTERY_COUNT_FIXED_BYTES / float(128 << 20),
}


def battery_cpu_baseline(r_host, target_s=12.0):
    """The oracle battery on host copies of whole blocks of the tested
    sequence, repeated until about target_s seconds."""
    from oracle import battery as OB
    done = 0
    t0 = time.perf_counter()
    while True:
        OB.run_battery(r_host)
        done += r_host.size
        el = time.perf_counter() - t0
        if el >= target_s:
            break
    return {"value": done / el / 1e9, "unit": "Guniforms/s", "cores": 1, "kind": "oracle",
            "sample": "the nine tests on %d generator uniforms (%d blocks of 2^20), %d passes in %.1f s"
                      % (r_host.size, r_host.size >> 20, done // r_host.size, el)}


def workload_f(args, torch, ph):
    """The statistical battery of the Tests section on the generator's output:
    1024 seeded 32-bit instances x 2^20 draws per step (each block of the
    tested sequence is one stream: intrastream), generation plus the nine
    tests; the interstream variant interleaves the 1024 streams first."""
    dev = torch.device("cuda:0")
    nst, per = 1024, 1 << 20
    total = nst * per
    ctx = ph.Context(0, max_instances=nst)
    ids = ctx.seed_instances(32, 0x14112484 + 8, nst, (9, 17), 0, 0)
    r = torch.empty(total, dtype=torch.float64, device=dev)
    inter = torch.empty(total, dtype=torch.float64, device=dev)
    reqs = ph.make_requests(ids, [per] * nst, np.arange(nst, dtype=np.uint64) * per)
    steps = max(2, args.steps // 4)
    res = {}
    for order in ("intrastream", "interstream"):
        bat = ph.Battery(0)

        def step():
            ctx.generate(reqs, None, None, r, capacity=total)
            if order == "interstream":
                ph.interleave(r, inter, nst, per)
                bat.accumulate(inter)
            else:
                bat.accumulate(r)

        step()
        torch.cuda.synchronize()
        bat.reset()
        ctx.timing_reset()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = bat.timing()
        gen_ms, gen_calls = ctx.timing_read()
        rep = bat.report()
        draws = total * steps
        kernels = {}
        for k, (ms, n) in kt.items():
            gbs = draws * BATTERY_BYTES_PER_DRAW[k] / (ms * 1e-3) / 1e9
            kernels[k] = {"ms_per_step": ms / steps, "launches": n, "achieved_gbs": gbs,
                          "bytes_per_draw": BATTERY_BYTES_PER_DRAW[k]}
        bat_ms = sum(v[0] for v in kt.values()) / steps
        res[order] = {"value": draws / wall / 1e9, "ms_per_step": wall * 1e3 / steps,
                      "generation_ms_per_step": gen_ms / max(gen_calls, 1), "battery_kernel_ms_per_step": bat_ms,
                      "battery_only_guniforms_s": total / (bat_ms * 1e-3) / 1e9, "kernels": kernels,
                      "tests": {name: {"chi2": v[0], "dof": v[1], "p": v[2], "samples": v[3]}
                                for name, v in rep.items()},
                      "min_p": min(v[2] for v in rep.values())}
        log("battery %s: %.1f Guniforms/s tested (battery kernels %.2f ms/step), min P %.3g"
            % (order, res[order]["value"], bat_ms, res[order]["min_p"]))
        bat.close()
    # the paper's largest interleaving shape tried here: N_p = 2^20 streams,
    # 1024 draws each, tested in the interstream order
    ctx.close()
    np_streams, np_len = 1 << 20, 1024
    big = ph.Context(0, max_instances=np_streams)
    t0 = time.perf_counter()
    bids = big.seed_instances(32, 0x14112484 + 10, np_streams, (9, 17), 0, 0)
    seed_s = time.perf_counter() - t0
    breqs = ph.make_requests(bids, [np_len] * np_streams, np.arange(np_streams, dtype=np.uint64) * np_len)
    bat = ph.Battery(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    big.generate(breqs, None, None, r, capacity=total)
    ph.interleave(r, inter, np_streams, np_len)
    bat.accumulate(inter)
    rep = bat.report()
    wall = time.perf_counter() - t0
    res["interstream_np_2p20"] = {"streams": np_streams, "draws_per_stream": np_len, "seconds": wall,
                                  "seeding_seconds": seed_s,
                                  "tests": {k: {"chi2": v[0], "p": v[2]} for k, v in rep.items()},
                                  "min_p": min(v[2] for v in rep.values())}
    log("battery interstream N_p = 2^20: %.2f s, min P %.3g" % (wall, res["interstream_np_2p20"]["min_p"]))
    bat.close()
    big.close()
    # constant skip b = p(p-1)/2 mod n over its whole period n (Sec. II): every
    # ciphertext occurs once, so the one-dimensional test sees a distribution
    # that is uniform to within one count per bin (far below the chi^2 median)
    n_ex, e_ex, p31 = 4294967087, 9, (1 << 31) - 1
    b_ex = (p31 * (p31 - 1) // 2) % n_ex
    cs = ph.Context(0, max_instances=1)
    cid = cs.add_instances_skip(32, [n_ex], [e_ex], [b_ex])
    nblk = n_ex // (1 << 20)
    bat = ph.Battery(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < nblk:
        nb = min(1024, nblk - done)
        cs.generate(ph.make_requests(cid, [nb << 20], [0]), None, None, r, capacity=total)
        bat.accumulate(r[: nb << 20])
        done += nb
    rep = bat.report()
    wall = time.perf_counter() - t0
    res["constant_skip_full_period"] = {
        "n": n_ex, "e": e_ex, "b": b_ex, "uniforms": nblk << 20, "seconds": wall,
        "tests": {k: {"chi2": v[0], "dof": v[1], "p": v[2]} for k, v in rep.items()}}
    log("battery constant skip over its period: %.2f s, P = %s" % (wall, {k: "%.3g" % v[2] for k, v in rep.items()}))
    bat.close()
    cs.close()
    ctx = None
    if args.battery_uniforms > 0:
        # one long stream of the paper's example instance (Sec. II tested single
        # streams of 10^11 to 10^13 uniforms), in steps of 2^30
        lc = ph.Context(0, max_instances=1)
        lid = lc.add_instances(32, [4294967087], [9])
        nsteps = max(1, int(args.battery_uniforms) >> 30)
        lreq = ph.make_requests(lid, [total], [0])
        bat = ph.Battery(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(nsteps):
            lc.generate(lreq, None, None, r, capacity=total)
            bat.accumulate(r)
            if (i + 1) % 128 == 0:
                torch.cuda.synchronize()
                log("battery long stream: %d of %d steps" % (i + 1, nsteps))
        rep = bat.report()
        wall = time.perf_counter() - t0
        res["long_stream"] = {"n": 4294967087, "e": 9, "uniforms": nsteps * total, "seconds": wall,
                              "guniforms_s": nsteps * total / wall / 1e9,
                              "tests": {k: {"chi2": v[0], "dof": v[1], "p": v[2]} for k, v in rep.items()},
                              "min_p": min(v[2] for v in rep.values())}
        log("battery long stream: %.3g uniforms in %.1f s, P = %s"
            % (nsteps * total, wall, {k: "%.3g" % v[2] for k, v in rep.items()}))
        bat.close()
        lc.close()
    intra = res["intrastream"]
    dom = max(intra["kernels"], key=lambda k: intra["kernels"][k]["ms_per_step"])
    dk = intra["kernels"][dom]
    roof = {"bound": "hbm", "achieved": dk["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dk["achieved_gbs"] / HBM_PEAK_GBS, "traffic": None, "kernel": dom,
            "bytes_per_draw": dk["bytes_per_draw"], "units_per_launch": 128 << 20}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = battery_cpu_baseline(r[: 8 << 20].cpu().numpy())
        log("battery cpu baseline: %s" % cpu)
    line = common_line(intra["value"], "Guniforms/s", steps, 1, intra["ms_per_step"],
                       {"workload": "statistical battery (nine chi-square tests, blocks of 2^20) on 1024 seeded "
                                    "32-bit streams x 2^20 draws per step, generation included"},
                       roofline=roof, cpu_baseline=cpu, **res)
    line["metric"] = "uniforms tested per second by the nine-test battery (generation + tests)"
    line["dtype"] = "f64"
    return line


def pattern_ops_per_tuple(dim, e=9):
    """VALU operations per tuple of the pattern kernel in the minimal model:
    per following point one modular add (3), the encryption chain (6 per
    Montgomery product) and the bin (8); one skip step (6) per point after
    the first."""
    chain = {3: 3, 5: 4, 9: 5, 17: 6}[int(e)]
    return (dim - 1) * (3 + 6 * chain + 8) + (dim - 2) * 6


def workload_g(args, torch, ph):
    """Full-period local pattern of Sec. III with the Tests section's sizes:
    the paper's safe prime n = 4294967087, e = 9, the 128 first points
    [0, 128), every skip of the period [1, p), D = 3, 4, 5 in 2^24 cells."""
    import oracle
    n, e, l0 = 4294967087, 9, 128
    p31 = (1 << 31) - 1
    res = {}
    for dim, bins in ((3, 4096), (4, 256), (5, 64)):
        spec = ph.pattern_spec(n, e, 0, l0, dim, bins, 1, p31)
        hist = torch.zeros(bins ** (dim - 1), dtype=torch.int64, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ph.pattern_histogram(spec, hist)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        chi2, pv, total = ph.pattern_chi2(spec, hist)
        tuples = l0 * (p31 - 1)
        ops = pattern_ops_per_tuple(dim, e)
        res["D%d" % dim] = {"seconds": wall, "tuples": tuples, "gtuples_s": tuples / wall / 1e9,
                            "chi2": chi2, "dof": bins ** (dim - 1) - 1, "p": pv, "total": total,
                            "alu_frac": tuples * ops / wall / ALU_PEAK_OPS, "ops_per_tuple": ops}
        log("pattern D=%d: %.2f s, %.1f Gtuples/s, chi2 %.1f, P %.3g" % (dim, wall, tuples / wall / 1e9, chi2, pv))
        del hist
    # the oracle on a bounded sample: one first point, 2^22 skips, D = 3
    p, a = oracle.lcg_params(32)
    t0 = time.perf_counter()
    reps = 0
    while time.perf_counter() - t0 < 10.0:
        oracle.pattern_hist(n, e, p, a, reps, 1, 3, 4096, 1, 1 + (1 << 22))
        reps += 1
    el = time.perf_counter() - t0
    cpu = {"value": reps * (1 << 22) / el / 1e9, "unit": "Gtuples/s", "cores": 1, "kind": "oracle",
           "sample": "%d first points x 2^22 skips, D = 3, 4096^2 cells, in %.1f s" % (reps, el)}
    d3 = res["D3"]
    roof = {"bound": "alu", "achieved": d3["tuples"] * d3["ops_per_tuple"] / d3["seconds"] / 1e12,
            "peak": ALU_PEAK_OPS / 1e12, "unit": "Top/s", "frac": d3["alu_frac"], "traffic": None,
            "kernel": "pattern_kernel<9, 3>", "ops_per_tuple": d3["ops_per_tuple"]}
    total_s = sum(v["seconds"] for v in res.values())
    line = common_line(d3["gtuples_s"], "Gtuples/s", 1, 0, d3["seconds"] * 1e3,
                       {"workload": "full-period local pattern: n = 4294967087, e = 9, first points [0, 128), "
                                    "skips [1, 2^31 - 1), 2^24 cells, D = 3 (value), 4, 5"},
                       roofline=roof, cpu_baseline=cpu, all_dims_seconds=total_s, **res)
    line["metric"] = "full-period pattern tuples per second (D = 3)"
    line["dtype"] = "u32"
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-ciphertexts", action="store_true", help="skip the u32 + f64 output variant")
    ap.add_argument("--no-graph", action="store_true", help="skip the captured-graph replay variant")
    ap.add_argument("--no-unit-skip", action="store_true", help="skip the unit-skip schedule variant")
    ap.add_argument("--no-w64", action="store_true", help="skip the 64-bit-moduli variant")
    ap.add_argument("--autotune", action="store_true", help="autotune the launch shape before timing")
    ap.add_argument("--workload", default="B", choices=["A", "B", "C", "D", "E", "F", "G"],
                    help="B (default): the headline batch; A, C, D, E: the other workload shapes; "
                         "F: the statistical battery on the generator's output; G: the full-period pattern")
    ap.add_argument("--battery-uniforms", type=float, default=0,
                    help="workload F: also test one stream of this many uniforms (multiple of 2^30)")
    ap.add_argument("--serve-instances", type=int, default=1000000)
    ap.add_argument("--serve-arena", type=int, default=1 << 31, help="serving arena, FP64 uniforms")
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[1e3, 3e3, 1e4, 3e4, 1e5, 3e5, 1e6, 3e6])
    ap.add_argument("--serve-seconds", type=float, default=1.0)
    ap.add_argument("--serve-max-requests", type=int, default=200000)
    ap.add_argument("--serve-streams", type=int, default=2, help="streams of the server")
    ap.add_argument("--serve-inflight", type=int, default=0,
                    help="batches in flight (0: the server's default, streams + 1)")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="first run one device copy of this many GiB (known-size kernel for traffic counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: it measures the single-GPU share of the generator "
              "(instances shard across GPUs with no communication); --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1411_2484_amd as ph

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.workload != "B":
        fn = {"A": workload_a, "C": workload_c, "D": workload_d, "E": workload_e, "F": workload_f,
              "G": workload_g}[args.workload]
        print(json.dumps(fn(args, torch, ph)), flush=True)
        return
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

    graph = None
    if not args.no_graph:
        g = ctx.graph(reqs, None, None, r, capacity=total)
        gms, gk = timed_steps(ctx, torch, g.launch, args.steps, 3)
        g.close()
        graph = {"value": total / (gms * 1e-3) / 1e9, "unit": "Guniforms/s", "ms_per_step": gms, "kernel_ms": gk,
                 "note": "captured plan + persistent kernel + position advance, replayed each step"}
        log("graph replay: %s" % graph)

    unit = None
    if not args.no_unit_skip:
        # the same moduli and exponents on the unit-skip schedule (counter mode):
        # the encryption path alone, without the skip generator and prefix
        uctx = ph.Context(0, max_instances=N_INST)
        uids = uctx.add_instances_skip(32, n_arr, e_arr, np.ones(N_INST, dtype=np.uint64))
        ureqs = ph.make_requests(uids, [PER] * N_INST, np.arange(N_INST, dtype=np.uint64) * PER)
        ums, uk = timed_steps(uctx, torch, lambda: uctx.generate(ureqs, None, None, r, capacity=total), args.steps, 3)
        unit = {"value": total / (ums * 1e-3) / 1e9, "unit": "Guniforms/s", "ms_per_step": ums, "kernel_ms": uk,
                "note": "same 4096 (n, e), unit-skip schedule m_k = m_0 + k"}
        log("unit skip: %s" % unit)
        uctx.close()

    w64 = None
    if not args.no_w64:
        # 64-bit moduli (n in [2^62, 2^63)), 1024 seeded instances x 2^20 draws, FP64 only
        wctx = ph.Context(0, max_instances=1024)
        wids = wctx.seed_instances(64, 0x14112484 + 3, 1024, (9, 17), 0, 0)
        wreqs = ph.make_requests(wids, [1 << 20] * 1024, np.arange(1024, dtype=np.uint64) << 20)
        wms, wk = timed_steps(wctx, torch, lambda: wctx.generate(wreqs, None, None, r, capacity=total),
                              max(args.steps // 2, 2), 3)
        w64 = {"value": total / (wms * 1e-3) / 1e9, "unit": "Guniforms/s", "ms_per_step": wms, "kernel_ms": wk,
               "workload": "1024 seeded 64-bit instances x 2^20 draws, FP64 uniforms"}
        log("width 64: %s" % w64)
        wctx.close()

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
           "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": measured_traffic(), "bytes_per_draw": bytes_per_draw}
    alu = {"bound": "alu", "achieved": achieved_ops / 1e12, "peak": ALU_PEAK_OPS / 1e12, "unit": "Top/s",
           "frac": achieved_ops / ALU_PEAK_OPS, "ops_per_draw": ops_per_draw}
    roof, other = (hbm, alu) if hbm["frac"] >= alu["frac"] else (alu, hbm)
    roof = dict(roof)
    roof["traffic"] = measured_traffic()
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
        "graph_replay": graph,
        "unit_skip": unit,
        "width64": w64,
        "roofline": roof,
        "roofline_other": other,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
