#!/usr/bin/env python3
"""Benchmark of the gfx950 Pohlig-Hellman generator on one GPU.

One JSON line.  `value` is the headline: 4096 seeded width-32 instances
(distinct admissible primes n in [2^31, 2^32), e from {9, 17} coprime to
n - 1, start position 0), 2^18 draws each per step, FP64 uniforms written
to HBM, one batched persistent launch per step (1,073,741,824 uniforms per
step; each step continues every stream).  Beside it, in the same run:

  - the same batch as one launch per instance (the plain form), as a
    captured-graph replay, with u32 ciphertexts too, on the unit skip;
  - 1 instance x 10^6 draws (c + R);
  - 65,536 instances with log-uniform lengths in [2^10, 2^22] and starts in
    [0, 2^40) (c + R over the fewest launches whose outputs fit the device,
    and R only in one launch);
  - 1024 width-64 + 1024 width-32 instances x 2^20 in one launch (c + R),
    and each width alone;
  - serving: 10^6 resident instances, Poisson arrivals at three rates, p50
    and p99 latency;
  - the CPU oracle on the host's cores over a bounded sample of the headline
    batch.

Every workload runs on synthetic seeded instances; inputs are resident on
the device when the timed region starts.  Launch shapes are autotuned per
batch class (width 32, width 64, mixed) before timing and reported.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from tests import workloads as W  # noqa: E402

METRIC = "Guniforms/s (32/64-bit moduli), batched vs plain launch; serve p50/p99 latency"
SEED_B = W.SEED0 + 1
N_INST = 4096
PER = 1 << 18
HBM_PEAK_GBS = 8000.0            # MI355X published HBM3E bandwidth
CUS, CLOCK_HZ = 256, 2.4e9       # MI355X compute units and peak engine clock
ALU_PEAK_OPS = CUS * 64 * CLOCK_HZ  # one wave64 VALU instruction per CU per clock

KERNEL_SOURCES = ["paper_1411_2484_amd/csrc/kernels.hip", "paper_1411_2484_amd/csrc/arith.hpp",
                  "paper_1411_2484_amd/csrc/layout.hpp"]
COUNTERS_FILE = os.path.join(ROOT, "profiles", "gen_persistent_counters.json")
COUNTERS_FILE_W64 = os.path.join(ROOT, "profiles", "gen_width64_counters.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_counters(path=COUNTERS_FILE):
    """Per-launch counter figures (headline kernel, or the width-64 path) from
    the committed rocprofv3 runs, when they were taken on the current kernel
    sources."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t


def algorithmic_ops_32(e):
    """VALU operations per width-32 draw in the minimal instruction model of
    algorithm (9): skip 6, message 4, Montgomery products 6 each (e = 9: 5,
    e = 17: 6, e = 3: 3, e = 5: 4), uniform 5."""
    chain = {3: 3, 5: 4, 9: 5, 17: 6}[int(e)]
    return 6 + 4 + 6 * chain + 5


def algorithmic_ops_64(e):
    """VALU operations per width-64 draw in the same model with 32-bit limbs:
    skip mod 2^61 - 1 (a 64 x 64 product, four multiply-adds, and the
    Mersenne fold) 10, message 4, Montgomery products 19 each (full x y,
    low q = lo(x y) n', high q n, borrow), uniform 9 (two conversions, five
    FP64 operations)."""
    chain = {3: 3, 5: 4, 9: 5, 17: 6}[int(e)]
    return 10 + 4 + 19 * chain + 9


def roofline(draws, kernel_ms, ops_per_draw, bytes_per_draw):
    """ALU and HBM fractions of a generation launch (algorithmic work only)."""
    sec = kernel_ms * 1e-3
    ops = draws * ops_per_draw / sec
    gbs = draws * bytes_per_draw / sec / 1e9
    return {"alu": {"achieved": ops / 1e12, "peak": ALU_PEAK_OPS / 1e12, "unit": "Top/s",
                    "frac": ops / ALU_PEAK_OPS, "ops_per_draw": ops_per_draw},
            "hbm": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                    "bytes_per_draw": bytes_per_draw}}


def timed(ctx, torch, fn, steps, warmup):
    """(wall ms per step, generation-kernel ms per step) of `steps` calls of fn."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ctx.timing_reset()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, _ = ctx.timing_read()
    return wall * 1e3 / steps, kms / steps


def release(torch):
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(n_arr, e_arr, target_s):
    """The oracle on all of the host's cores over a bounded sample of the
    headline workload: batches of 256 of its instances, 2^18 draws each from
    position 0, cycling over the 4096 instances for about target_s seconds."""
    import oracle
    nthreads = host_cores()
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
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "ns_per_uniform_per_core": el * nthreads / draws * 1e9,
            "sample": "%d instance-streams of the headline batch (2^18 draws each from position 0, u32 c + f64 R, "
                      "%d draws) in %.1f s on %d threads" % (done_inst, draws, el, nthreads)}


# ---------------------------------------------------------------------------
# headline: 4096 x 2^18, width 32
# ---------------------------------------------------------------------------

def section_headline(args, torch, ph, out):
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
    if not args.no_autotune:
        t0 = time.perf_counter()
        ctx.autotune(total)  # on the batch itself: 4096 streams x 2^18
        log("autotune (width 32): %s in %.1f s" % (ctx.get_tuning_class(ph.PHPRNG_CLASS_W32),
                                                    time.perf_counter() - t0))
    tuning = ctx.get_tuning_class(ph.PHPRNG_CLASS_W32)

    def gen(mode=ph.PHPRNG_MODE_PERSISTENT, c32=None):
        ctx.generate(reqs, c32, None, r, capacity=total, mode=mode)

    ms, kms = timed(ctx, torch, gen, args.steps, args.warmup)
    value = total / (ms * 1e-3) / 1e9
    log("persistent: %.3f ms/step wall, %.3f ms kernel, %.1f Guniforms/s" % (ms, kms, value))
    ops_per_draw = float(np.mean([algorithmic_ops_32(e) for e in e_arr]))
    roofs = roofline(total, kms, ops_per_draw, 8.0)
    roof = dict(roofs["alu"])
    roof.update({"bound": "alu", "kernel": "gen_persistent<%d, %d, false>" % (tuning["block_threads"],
                                                                           tuning["unroll"]),
                 "kernel_ms": kms, "units_per_launch": total, "traffic": None})
    cnt = committed_counters()
    if cnt:
        roof["traffic"] = cnt.get("traffic_bytes_per_launch")
        # per launch from the counter runs, against this run's kernel time:
        #   issued: VALU lane-instructions / (time x 64 lane-ops per CU per
        #           clock at 2.4 GHz);
        #   cycle-weighted: each issued instruction costed at the measured
        #           chip-wide rate of its class (opcode mix of the kernel's
        #           per-draw code), summed, / time;
        #   sclk: busy cycles per XCD (GRBM_GUI_ACTIVE) / time.
        n_valu = cnt.get("valu_insts_per_launch")
        if n_valu:
            roof["issued_valu_frac"] = n_valu * 64 / (kms * 1e-3) / ALU_PEAK_OPS
            if cnt.get("valu_seconds_per_inst"):
                roof["cycle_weighted_frac"] = n_valu * cnt["valu_seconds_per_inst"] / (kms * 1e-3)
                roof["cycle_weighted_model"] = cnt.get("cycle_weighted_model")
        if cnt.get("grbm_cycles_per_xcd"):
            roof["sclk_ghz_est"] = cnt["grbm_cycles_per_xcd"] / (kms * 1e-3) / 1e9
    out.update({"value": value, "ms_per_step": ms, "roofline": roof, "roofline_hbm": roofs["hbm"]})
    out["config"].update({"tuning": tuning})

    if not args.no_plain:
        pms, pk = timed(ctx, torch, lambda: gen(ph.PHPRNG_MODE_PLAIN), args.plain_steps, 1)
        out["plain"] = {"value": total / (pms * 1e-3) / 1e9, "unit": "Guniforms/s", "ms_per_step": pms,
                        "kernel_ms": pk, "launches_per_step": N_INST, "speedup_of_batched": pms / ms}
        log("plain: %s" % out["plain"])
    if not args.no_graph:
        g = ctx.graph(reqs, None, None, r, capacity=total)
        # graph replays warm up as long as the headline does: the first few
        # dozen replays of a fresh graph run slower
        gms, gk = timed(ctx, torch, g.launch, args.steps, args.warmup)
        g.close()
        out["graph_replay"] = {"value": total / (gms * 1e-3) / 1e9, "unit": "Guniforms/s", "ms_per_step": gms,
                               "kernel_ms": gk,
                               "note": "request block copied, then the captured persistent kernel replayed"}
        log("graph replay: %s" % out["graph_replay"])
    if not args.no_ciphertexts:
        c32 = torch.empty(total, dtype=torch.int32, device=dev)
        cms, ck = timed(ctx, torch, lambda: gen(c32=c32), max(args.steps // 2, 1), max(args.warmup // 4, 2))
        out["with_ciphertexts"] = {"value": total / (cms * 1e-3) / 1e9, "unit": "Guniforms/s", "ms_per_step": cms,
                                   "kernel_ms": ck, "outputs": "u32 c + f64 R (12 B per draw)",
                                   "roofline": roofline(total, ck, ops_per_draw, 12.0)}
        log("with ciphertexts: %s" % out["with_ciphertexts"])
        del c32
    if not args.no_unit_skip:
        uctx = ph.Context(0, max_instances=N_INST)
        uids = uctx.add_instances_skip(32, n_arr, e_arr, np.ones(N_INST, dtype=np.uint64))
        ureqs = ph.make_requests(uids, [PER] * N_INST, np.arange(N_INST, dtype=np.uint64) * PER)
        ums, uk = timed(uctx, torch, lambda: uctx.generate(ureqs, None, None, r, capacity=total), args.steps,
                        max(args.warmup // 4, 3))
        out["unit_skip"] = {"value": total / (ums * 1e-3) / 1e9, "unit": "Guniforms/s", "ms_per_step": ums,
                            "kernel_ms": uk, "note": "same 4096 (n, e), unit-skip schedule m_k = m_0 + k"}
        log("unit skip: %s" % out["unit_skip"])
        uctx.close()
    ctx.close()
    del r
    release(torch)
    return n_arr, e_arr


# ---------------------------------------------------------------------------
# 1 instance x 10^6
# ---------------------------------------------------------------------------

def section_a(args, torch, ph, out):
    dev = torch.device("cuda:0")
    ctx = ph.Context(0, max_instances=1)
    ids = ctx.seed_instances(32, W.SEED0, 1, (9, 17), 0, 0)
    N = 10 ** 6
    c32 = torch.empty(N, dtype=torch.int32, device=dev)
    r = torch.empty(N, dtype=torch.float64, device=dev)
    reqs = ph.make_requests(ids, [N], [0])
    res = {}
    for name, mode in (("persistent", ph.PHPRNG_MODE_PERSISTENT), ("plain", ph.PHPRNG_MODE_PLAIN)):
        def call():
            ctx.generate(reqs, c32, None, r, mode=mode)
        # calls this short are bound by the host call: the wall time is taken
        # with per-call timing off (one event record fewer per call), the
        # kernel time in a second, timed pass
        ctx.set_timing(False)
        ms, _ = timed(ctx, torch, call, 20, 5)
        ctx.set_timing(True)
        ms_timed, kms = timed(ctx, torch, call, 20, 5)
        res[name] = {"value": N / (ms * 1e-3) / 1e9, "ms_per_step": ms, "kernel_ms": kms,
                     "ms_per_step_timed": ms_timed}
    res["workload"] = "1 seeded width-32 instance x 10^6 draws from position 0 (u32 c + f64 R)"
    res["note"] = ("value and ms_per_step: calls with per-call kernel timing off; kernel_ms and "
                   "ms_per_step_timed: the same calls with timing on")
    out["one_instance"] = res
    log("one instance: %s" % res)
    ctx.close()


# ---------------------------------------------------------------------------
# 65,536 log-uniform streams
# ---------------------------------------------------------------------------

def section_c(args, torch, ph, out):
    dev = torch.device("cuda:0")
    nin = W.C_INSTANCES
    lens = W.config_c_lengths(nin)
    total = int(lens.sum())
    ctx = ph.Context(0, max_instances=nin)
    ids = ctx.seed_instances(32, W.C_SEED, nin, (9, 17), 0, W.C_START_HI)
    es = np.array([ctx.get_params(int(i))[1] for i in ids])
    ops = float(np.sum(lens.astype(np.float64) * np.array([algorithmic_ops_32(e) for e in es])) / total)
    res = {"workload": "65,536 seeded width-32 instances, lengths floor(2^(10 + 12u)) in [2^10, 2^22] "
                       "(%d draws), starts uniform in [0, 2^40)" % total, "draws": total}
    steps = max(1, args.big_steps)
    # u32 c + f64 R: 12 B per draw exceed the device, so the streams run in
    # the fewest groups whose outputs fit; one persistent launch per group
    free, _ = torch.cuda.mem_get_info()
    groups = W.groups_for_memory(lens, 12, free)
    arena = max(g[3] for g in groups)
    c32 = torch.empty(arena, dtype=torch.int32, device=dev)
    r = torch.empty(arena, dtype=torch.float64, device=dev)
    greqs = [ph.make_requests(ids[a:b], lens[a:b], offs) for a, b, offs, _ in groups]

    def step_cr():
        for q in greqs:
            ctx.generate(q, c32, None, r, capacity=arena)

    ms, kms = timed(ctx, torch, step_cr, steps, 1)
    res["c_and_r"] = {"value": total / (ms * 1e-3) / 1e9, "ms_per_step": ms, "kernel_ms": kms,
                      "launches_per_step": len(groups), "arena_elements": arena,
                      "roofline": roofline(total, kms, ops, 12.0)}
    log("C (c + R, %d launches): %s" % (len(groups), res["c_and_r"]))
    del c32, r
    release(torch)
    # f64 R only: 8 B per draw; the whole batch in one launch when it fits
    free, _ = torch.cuda.mem_get_info()
    groups = W.groups_for_memory(lens, 8, free, fill=0.9)
    arena = max(g[3] for g in groups)
    r = torch.empty(arena, dtype=torch.float64, device=dev)
    greqs = [ph.make_requests(ids[a:b], lens[a:b], offs) for a, b, offs, _ in groups]

    def step_r():
        for q in greqs:
            ctx.generate(q, None, None, r, capacity=arena)

    ms, kms = timed(ctx, torch, step_r, steps, 1)
    res["r_only"] = {"value": total / (ms * 1e-3) / 1e9, "ms_per_step": ms, "kernel_ms": kms,
                     "launches_per_step": len(groups), "arena_elements": arena,
                     "roofline": roofline(total, kms, ops, 8.0)}
    log("C (R only, %d launches): %s" % (len(groups), res["r_only"]))
    del r
    ctx.close()
    release(torch)
    out["log_uniform_65536"] = res


# ---------------------------------------------------------------------------
# 1024 width-64 + 1024 width-32 x 2^20
# ---------------------------------------------------------------------------

def section_d(args, torch, ph, out):
    dev = torch.device("cuda:0")
    per = 1 << 20
    res = {"workload": "1024 seeded width-64 instances (n in [2^62, 2^63)) + 1024 width-32 instances, 2^20 draws "
                       "each from position 0, u64/u32 c + f64 R"}
    if not args.no_autotune:
        # width-64-only shapes, tuned on a context of the 64-bit instances
        # alone, with 2^18 draws per instance: enough chunks to keep every
        # candidate grid busy, as the timed 2^20-draw streams do (a smaller
        # tuning batch favours grids too small for the timed one)
        t64 = ph.Context(0, max_instances=1024)
        t64.seed_instances(64, W.SEED0 + 3, 1024, (9, 17), 0, 0)
        t64.autotune(1 << 28)
        t64.close()
    ctx = ph.Context(0, max_instances=2048)
    i64 = ctx.seed_instances(64, W.SEED0 + 3, 1024, (9, 17), 0, 0)
    i32 = ctx.seed_instances(32, W.SEED0 + 4, 1024, (9, 17), 0, 0)
    if not args.no_autotune:
        ctx.autotune(1 << 29)
    res["tuning"] = {"width64": ctx.get_tuning_class(ph.PHPRNG_CLASS_W64),
                     "mixed": ctx.get_tuning_class(ph.PHPRNG_CLASS_MIXED),
                     "width32": ctx.get_tuning_class(ph.PHPRNG_CLASS_W32)}
    e64 = np.array([ctx.get_params(int(i))[1] for i in i64])
    e32 = np.array([ctx.get_params(int(i))[1] for i in i32])
    ops64 = float(np.mean([algorithmic_ops_64(e) for e in e64]))
    ops32 = float(np.mean([algorithmic_ops_32(e) for e in e32]))
    total = 2048 * per
    c32 = torch.empty(total, dtype=torch.int32, device=dev)
    c64 = torch.empty(total, dtype=torch.int64, device=dev)
    r = torch.empty(total, dtype=torch.float64, device=dev)
    for name, ids, ops, bpd in (("mixed", np.concatenate([i64, i32]), (ops64 + ops32) / 2, 14.0),
                                ("w64_only", i64, ops64, 16.0), ("w32_only", i32, ops32, 12.0)):
        reqs = ph.make_requests(ids, [per] * len(ids), np.arange(len(ids), dtype=np.uint64) * per)
        # one untimed call per staging slot of the library (8) and one more:
        # each slot sizes its width-64 tile arrays on first use at this size,
        # and an allocation there would stall the timed calls
        ms, kms = timed(ctx, torch, lambda: ctx.generate(reqs, c32, c64, r, capacity=total), args.big_steps, 9)
        draws = len(ids) * per
        res[name] = {"value": draws / (ms * 1e-3) / 1e9, "ms_per_step": ms, "kernel_ms": kms,
                     "roofline": roofline(draws, kms, ops, bpd)}
        cnt = committed_counters(COUNTERS_FILE_W64) if name == "w64_only" else None
        if cnt and cnt.get("valu_insts_per_launch"):
            # reduce + scan + generation instructions of this launch against
            # the time of all three (HIP events around the call's kernels)
            alu = res[name]["roofline"]["alu"]
            alu["issued_valu_frac"] = cnt["valu_insts_per_launch"] * 64 / (kms * 1e-3) / ALU_PEAK_OPS
            if cnt.get("valu_seconds_per_inst"):
                alu["cycle_weighted_frac"] = cnt["valu_insts_per_launch"] * cnt["valu_seconds_per_inst"] / (kms * 1e-3)
        log("D %s: %s" % (name, res[name]))
    del c32, c64, r
    ctx.close()
    release(torch)
    out["mixed_widths"] = res


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

def section_e(args, torch, ph, out):
    n32, n64 = args.serve_instances * 9 // 10, args.serve_instances // 10
    ctx = ph.Context(0, max_instances=n32 + n64)
    t0 = time.perf_counter()
    ctx.seed_instances(32, W.SEED0 + 5, n32, (9, 17), 0, 1 << 40)
    ctx.seed_instances(64, W.SEED0 + 6, n64, (9, 17), 0, 1 << 32)
    seed_s = time.perf_counter() - t0
    log("serve: %d instances seeded in %.1f s" % (n32 + n64, seed_s))
    # a serving loop reads no per-call kernel times: one event record fewer per batch
    ctx.set_timing(False)
    srv = ph.Server(ctx, arena_doubles=args.serve_arena, streams=args.serve_streams,
                    max_inflight=args.serve_inflight)
    # untimed warm-up: first-use costs stay out of the first load point
    wrng = np.random.default_rng(W.SEED0 + 8)
    warm = np.zeros(2000, dtype=ph.ARRIVAL_DTYPE)
    warm["t_ns"] = np.cumsum(wrng.exponential(1e4, warm.size)).astype(np.int64)
    warm["instance"] = wrng.integers(0, n32 + n64, warm.size)
    warm["count"] = np.floor(2.0 ** (8 + 12 * wrng.random(warm.size))).astype(np.uint64)
    srv.replay(warm)
    rng = np.random.default_rng(W.SEED0 + 7)
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
              "offered_guniforms_s": float(draws / (arr["t_ns"][-1] * 1e-9) / 1e9),
              "p50_ms": float(np.percentile(lat, 50)) / 1e6, "p99_ms": float(np.percentile(lat, 99)) / 1e6,
              "admit_p50_ms": float(np.percentile(adm, 50)) / 1e6, "admit_p99_ms": float(np.percentile(adm, 99)) / 1e6,
              "wall_s": wall, "batches": cnt["batches"], "requests_per_batch": cnt["requests"] / max(cnt["batches"], 1),
              "launch_us_mean": cnt["launch_ns"] / max(cnt["batches"], 1) / 1e3,
              "form_us_mean": cnt["form_ns"] / max(cnt["batches"], 1) / 1e3,
              "arena_stalls": cnt["arena_stalls"]}
        log("serve: %s" % pt)
        points.append(pt)
    srv.close()
    ctx.close()
    release(torch)
    out["serving"] = {"workload": "%d resident instances (90%% width 32, starts in [0, 2^40); 10%% width 64, starts "
                                  "in [0, 2^32)), Poisson arrivals, each request log-uniform 2^8..2^20 FP64 uniforms "
                                  "from a uniformly chosen instance, latency from the scheduled arrival to the "
                                  "completion seen by the host" % (n32 + n64),
                      "streams": args.serve_streams, "seeding_s": seed_s,
                      "inflight": args.serve_inflight or min(args.serve_streams + 1, 6), "points": points}


def common_line(metric_value, unit, steps, warmup, ms_per_step, config, **extra):
    out = {"metric": METRIC, "value": metric_value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u32/u64/f64", "data": "synthetic", "config": config}
    out.update(extra)
    return out


# ---------------------------------------------------------------------------
# battery and pattern workloads (separate lines, --workload F / G)
# ---------------------------------------------------------------------------

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
    ctx.close()
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
    """Full-period local pattern of Sec. II, Figs. 3-4 with the Tests section's sizes:
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
    ap.add_argument("--steps", type=int, default=100, help="timed steps of the headline batch")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--big-steps", type=int, default=3,
                    help="timed steps of the 65,536-stream and the mixed-width batches")
    ap.add_argument("--sections", default="B,A,C,D,E",
                    help="comma-separated: B headline (with its variants), A one instance, C 65,536 log-uniform "
                         "streams, D mixed widths, E serving")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle time on the host for the baseline")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-ciphertexts", action="store_true", help="skip the u32 + f64 output variant")
    ap.add_argument("--no-graph", action="store_true", help="skip the captured-graph replay variant")
    ap.add_argument("--no-unit-skip", action="store_true", help="skip the unit-skip schedule variant")
    ap.add_argument("--no-autotune", action="store_true", help="time the library's default launch shapes")
    ap.add_argument("--workload", default=None, choices=["F", "G"],
                    help="instead of the generation line: F the statistical battery on the generator's output, "
                         "G the full-period pattern")
    ap.add_argument("--serve-instances", type=int, default=1000000)
    ap.add_argument("--serve-arena", type=int, default=1 << 31, help="serving arena, FP64 uniforms")
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[1e5, 1e6, 3e6])
    ap.add_argument("--serve-seconds", type=float, default=0.5)
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
    if args.workload:
        fn = {"F": workload_f, "G": workload_g}[args.workload]
        print(json.dumps(fn(args, torch, ph)), flush=True)
        return
    out = {
        "metric": METRIC, "value": None, "unit": "Guniforms/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32/u64/f64", "data": "synthetic",
        "config": {"workload": "4096 seeded width-32 instances x 2^18 draws per step (1.07e9 FP64 uniforms to HBM), "
                               "one batched persistent launch per step",
                   "instances": N_INST, "draws_per_instance": PER, "width": 32, "e_set": [9, 17],
                   "start_position": 0},
    }
    sections = [s.strip().upper() for s in args.sections.split(",") if s.strip()]
    n_arr = e_arr = None
    t_start = time.perf_counter()
    if "B" in sections:
        n_arr, e_arr = section_headline(args, torch, ph, out)
    if "A" in sections:
        section_a(args, torch, ph, out)
    if "C" in sections:
        section_c(args, torch, ph, out)
    if "D" in sections:
        section_d(args, torch, ph, out)
    if "E" in sections:
        section_e(args, torch, ph, out)
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline and n_arr is not None:
        out["cpu_baseline"] = cpu_baseline(n_arr, e_arr, args.cpu_seconds)
        log("cpu baseline: %s" % out["cpu_baseline"])
    out["bench_seconds"] = time.perf_counter() - t_start
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
