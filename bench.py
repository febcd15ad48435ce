#!/usr/bin/env python3
"""Benchmark: BLS12-377 G1 multi-scalar multiplication on one MI355X (gfx950).

One step = one full MSM (msm_run: digit sort, bucket accumulation, bucket
aggregation, group aggregation, affine result) over n = 2^20 seeded synthetic
points P_i = k_i G with uniform scalars mod r -- the n = 2^20 workload the
headline metric is quoted on.  Points are generated and prepared on the GPU
before the timed region (preparation is reported separately).

value = PADDs/s: the point additions and doublings one MSM executes (every
non-zero digit's mixed addition, the aggregation tree's additions, the window
and group Horner steps; split-bucket merges are not counted) divided by the
MSM time; ms_per_step = MSM latency.

Prints one JSON line.  Extra keys: the window sweep, per-phase times, the
standalone PADD kernel (2^22 independent pairs), the roofline of the dominant
kernel, the CPU oracle baseline, and the batched (64 MSMs of log-uniform
sizes) and served (Poisson arrivals) workloads against the plain path.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_POINTS = 1 << 20
# (encoding, window width) candidates of the n = 2^20 sweep
SWEEP = [("signed", c) for c in (15, 16, 17)] + [("glv", c) for c in (13, 15, 16, 19)]
ENCODINGS = {"signed": 0, "unsigned": 1, "glv": 2}
MAD_PER_MUL = 276          # 144 a*b + 132 m*p word products per Montgomery multiply
MULS_MIXED = 7             # mixed PADD (Z2 = 1, U2 = k T2)
MULS_COMPLETE = 9          # complete PADD with k T2 formed on the fly
# gfx950 VALU: 256 CUs x 4 SIMDs x 16 lanes, v_mad_u64_u32 at full rate, 2.4 GHz
PEAK_MAD_PER_S = 256 * 64 * 2.4e9
# Chip-wide issue rates measured by --microbench (profiles/valu_rates.md), as
# fractions of PEAK_MAD_PER_S: independent v_mad_u64_u32 and v_addc_co_u32.
# The field multiply issues one carry add per multiply-add, so its mads can
# reach at most 1 / (1/MAD_RATE + 1/ADDC_RATE) of the peak.
MAD_RATE = 0.71
ADDC_RATE = 0.80
MAD_WITH_CARRY_CEILING = 1.0 / (1.0 / MAD_RATE + 1.0 / ADDC_RATE)


def padd_count_formula(n, c):
    """Unsigned-digit Pippenger count n W + 2 (2^c - 1) W + W c + W - 1."""
    W = -(-253 // c)
    return n * W + 2 * ((1 << c) - 1) * W + W * c + W - 1


def num_windows(c, encoding):
    bits = {"signed": 254, "unsigned": 253, "glv": 128}[encoding]
    return -(-bits // c)


def padd_count_executed(entries, c, encoding="signed", jobs=1):
    """Additions and doublings the implementation executes for one MSM:
    accumulation (one mixed addition per non-zero digit), the aggregation
    tree (2^(bb+1) - bb - 2 per window), the window Horner steps and the
    group Horner steps (c doublings and one addition per window but the top)."""
    signed = encoding != "unsigned"
    W = num_windows(c, encoding)
    bb = c - 1 if signed else c
    S = W * jobs
    tree = S * ((1 << (bb + 1)) - bb - 2)
    combine = S * (2 * bb - 1 + (1 if signed else 0))
    horner = jobs * (W - 1) * (c + 1)
    return entries + tree + combine + horner


# ---------------------------------------------------------------------------
# CPU baseline: the oracle, timed on the host cores (runs before the GPU is
# touched, so the worker processes are forked from a GPU-free process)
# ---------------------------------------------------------------------------

def _oracle_worker(args):
    seed, seconds = args
    import random
    from oracle import curve, points
    from oracle.field import R_ORDER
    rng = random.Random(seed)
    pts = [points.fixed_base_mul(rng.randrange(1, R_ORDER)) for _ in range(32)]
    acc = pts[0]
    adds = 0
    t0 = time.perf_counter()
    elapsed = 0.0
    while elapsed < seconds:
        for j in range(256):
            acc = curve.add(acc, pts[j & 31])   # one affine PADD (chord law)
        adds += 256
        elapsed = time.perf_counter() - t0
    return adds, elapsed


def cpu_baseline(c, seconds=8.0):
    import multiprocessing as mp
    cores = max(1, min(os.cpu_count() or 1, 16))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(1000 + i, seconds) for i in range(cores)])
    wall = time.perf_counter() - t0
    adds = sum(r[0] for r in res)
    rate = adds / max(r[1] for r in res)
    return {
        "value": rate,
        "unit": "PADD/s",
        "cores": cores,
        "kind": "oracle",
        "sample": ("CPU oracle point additions (affine Weierstrass chord law, one Fermat "
                   "inverse per add), %d dependent adds in %.1f s on %d processes; the MSM time "
                   "at n=2^20, c=%d is extrapolated from this rate by the PADD count"
                   % (adds, wall, cores, c)),
        "msm_ms_extrapolated": None,
    }


# ---------------------------------------------------------------------------
# GPU side
# ---------------------------------------------------------------------------

def timed(fn, reps, torch):
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def glv_halves(sw_np):
    """Scalar words -> words of the endomorphism halves (s0, s1) per scalar."""
    import numpy as np
    from paper_2502_11660_amd import inputs
    lam = 0x8508C00000000001 ** 2 - 1
    ints = [inputs.words_to_int(r) for r in sw_np.reshape(-1, 8)]
    halves = []
    for v in ints:
        halves += [v % lam, v // lam]
    return np.asarray(inputs.ints_to_words(halves, 8), dtype=np.uint32)


def nonzero_digit_entries(sw_np, c, encoding="signed"):
    """Number of (point, window) pairs with a non-zero digit: the mixed PADDs
    bucket accumulation performs."""
    import numpy as np
    signed = encoding != "unsigned"
    W = num_windows(c, encoding)
    if encoding == "glv":
        sw_np = glv_halves(sw_np)
    words = sw_np.reshape(-1, 8).astype(np.uint64)
    carry = np.zeros(words.shape[0], dtype=np.uint64)
    total = 0
    for w in range(W):
        pos = w * c
        wi, sh = pos // 32, pos % 32
        lo = words[:, wi] if wi < 8 else np.zeros(words.shape[0], dtype=np.uint64)
        hi = words[:, wi + 1] if wi + 1 < 8 else np.zeros_like(lo)
        d = ((lo | (hi << np.uint64(32))) >> np.uint64(sh)) & np.uint64((1 << c) - 1)
        if signed:
            v = d + carry
            neg = (v >= np.uint64(1 << (c - 1))) & (w + 1 < W)
            mag = np.where(neg, np.uint64(1 << c) - v, v)
            carry = neg.astype(np.uint64)
            total += int(np.count_nonzero(mag))
        else:
            total += int(np.count_nonzero(d))
    return total


def padd_kernel_bench(torch, api, xyu_pool, pool_n, pairs, reps):
    """Standalone batched PADD (2^22 independent pairs, SoA) -- the paper's
    'task' measured as a stream of independent additions."""
    import numpy as np
    dev = xyu_pool.device
    aos = xyu_pool.view(pool_n, 3, 12)
    soa_b = aos.permute(1, 2, 0).contiguous()             # (3, 12, pool) prepared
    ident = torch.zeros(4, 12, pool_n, dtype=torch.int32, device=dev)
    one = api.to_device(np.array([0xffffff68, 0x02cdffff, 0x7fffffb1, 0x51409f83, 0x8a7d3ff2,
                                  0x9f7db3a9, 0x6e7c6305, 0x7b4e97b7, 0x803c84e8, 0x4cf495bf,
                                  0xe2fdf49a, 0x008d6661], dtype=np.uint32), dev)
    ident[1] = one.view(12, 1)
    ident[3] = one.view(12, 1)
    # projective points with Z != 1: identity + P, then + another pool point
    a_pool = api.padd_batch(ident.reshape(-1), soa_b.reshape(-1), pool_n, api.MSM_FORM_XYU)
    rot = torch.roll(soa_b, 1, dims=2).contiguous()
    a_pool = api.padd_batch(a_pool, rot.reshape(-1), pool_n, api.MSM_FORM_XYU)
    g = torch.Generator(device="cpu").manual_seed(20250219)
    ja = torch.randint(0, pool_n, (pairs,), generator=g).to(dev)
    jb = torch.randint(0, pool_n, (pairs,), generator=g).to(dev)
    A = a_pool.view(4, 12, pool_n).index_select(2, ja).contiguous().view(-1)
    Bm = soa_b.index_select(2, jb).contiguous().view(-1)
    Bc = a_pool.view(4, 12, pool_n).index_select(2, jb).contiguous().view(-1)
    out = torch.empty_like(A)
    res = {"_a_pool": a_pool}
    for name, B, form, muls, nbytes in (("mixed", Bm, api.MSM_FORM_XYU, MULS_MIXED, 48 * 4 * 2 + 36 * 4),
                                        ("complete", Bc, api.MSM_FORM_XYTZ, MULS_COMPLETE, 48 * 4 * 3)):
        fn = lambda: api.padd_batch(A, B, pairs, form, out=out)
        fn()
        ms = timed(fn, reps, torch)
        rate = pairs / (ms * 1e-3)
        res[name] = {
            "pairs": pairs,
            "ms": ms,
            "padd_per_s": rate,
            "mad_per_s": rate * muls * MAD_PER_MUL,
            "frac_of_valu_mad_peak": rate * muls * MAD_PER_MUL / PEAK_MAD_PER_S,
            "hbm_GBps": rate * nbytes / 1e9,
        }
    return res


def chain_and_stream_bench(torch, api, xyu_pool, a_pool_soa, pool_n):
    """The paper's latency workload (a dependent chain of complete additions
    over 2^18 points) and its throughput workload (independent accumulators
    fed prepared points, result returned once)."""
    recs = a_pool_soa.view(48, pool_n).t().contiguous()          # AoS XYTZ
    out = {"paper_latency_us_per_padd": 1.05, "paper_throughput_mtask_per_s": 67.0}
    chain = {}
    for name, unit, count in (("wide", api.MSM_UNIT_WIDE, 1 << 18), ("quad", api.MSM_UNIT_QUAD, 1 << 18),
                              ("lane", api.MSM_UNIT_LANE, 1 << 16)):
        pts = recs.repeat((count + pool_n - 1) // pool_n, 1)[:count].contiguous().view(-1)
        api.padd_chain(pts, 64, unit)
        ms = timed(lambda: api.padd_chain(pts, count, unit), 1, torch)
        chain[name] = {"count": count, "ms": ms, "us_per_padd": ms * 1e3 / count}
    out["latency_chain_complete_padd"] = chain
    npool = xyu_pool.numel() // 36
    stream = {}
    for n, A in ((1 << 18, 10), (1 << 18, 1 << 14), (1 << 20, 1 << 17)):
        n = min(n, npool)
        api.accumulate_stream(xyu_pool, n, A)
        ms = timed(lambda: api.accumulate_stream(xyu_pool, n, A), 3, torch)
        stream["n%d_A%d" % (n, A)] = {"points": n, "accumulators": A, "ms": ms,
                                       "mtask_per_s": n / (ms * 1e-3) / 1e6}
    out["accumulation_stream_mixed_padd"] = stream
    return out


def field_core_bench(torch, api, inputs, count=1 << 20, rounds=64):
    """Montgomery vs Barrett vs Karatsuba-Montgomery field multiplies:
    count lanes, each chaining `rounds` products."""
    a = api.to_device(inputs.base_field_elements(inputs.config_seed(2), count, stream=7).T.copy())
    b = api.to_device(inputs.base_field_elements(inputs.config_seed(2), count, stream=8).T.copy())
    out = api.words(12 * count)
    res = {}
    for name, var, mads in (("montgomery", api.MSM_MUL_MONT, MAD_PER_MUL),
                            ("barrett_k378", api.MSM_MUL_BARRETT, 144 + 99 + 78),
                            ("karatsuba_montgomery", api.MSM_MUL_KARATSUBA, 3 * 36 + 132)):
        api.fe_mul_chain(a, b, count, var, 2, out=out)
        ms = timed(lambda: api.fe_mul_chain(a, b, count, var, rounds, out=out), 3, torch)
        rate = count * rounds / (ms * 1e-3)
        res[name] = {"ms": ms, "mul_per_s": rate, "word_mads_per_mul": mads,
                     "mad_per_s": rate * mads, "frac_of_valu_mad_peak": rate * mads / PEAK_MAD_PER_S}
    res["lanes"] = count
    res["rounds"] = rounds
    return res


def microbench():
    """Issue rates of v_mad_u64_u32 / v_addc_co_u32 and HBM copy bandwidth."""
    import torch
    from paper_2502_11660_amd import api
    torch.cuda.set_device(0)
    out = {}
    buf = torch.empty(2048 * 256 * 2, dtype=torch.int32, device="cuda")
    threads = 2048 * 256
    for name, kind in (("v_mad_u64_u32", api._lib.MSM_MB_MAD64), ("v_addc_co_u32", api._lib.MSM_MB_ADDC)):
        iters = 4000
        api.microbench(kind, 10, buf)
        ms = timed(lambda: api.microbench(kind, iters, buf), 3, torch)
        rate = 16.0 * iters * threads / (ms * 1e-3)
        out[name] = {"ops_per_s": rate, "frac_of_peak": rate / PEAK_MAD_PER_S,
                     "lane_ops_per_cu_per_clk_at_2.4GHz": rate / (256 * 2.4e9)}
    for name, kind, per in (("lone_wave_mad64_8_chains", api._lib.MSM_MB_MAD64_LONE, 16),
                            ("lone_wave_mad64_dependent", api._lib.MSM_MB_MAD64_DEP, 16),
                            ("lone_wave_fe_mul_dependent", api._lib.MSM_MB_FEMUL_DEP, 1)):
        iters = 20000 if per == 16 else 2000
        api.microbench(kind, 10, buf)
        ms = timed(lambda: api.microbench(kind, iters, buf), 3, torch)
        ops = per * iters
        out[name] = {"ops": ops, "ms": ms, "ns_per_op": ms * 1e6 / ops,
                     "cycles_per_op_at_2.4GHz": ms * 1e-3 * 2.4e9 / ops}
    nbytes = 1 << 31
    big = torch.empty(2 * nbytes // 4, dtype=torch.int32, device="cuda")
    api.microbench(api._lib.MSM_MB_COPY, nbytes, big)
    ms = timed(lambda: api.microbench(api._lib.MSM_MB_COPY, nbytes, big), 5, torch)
    out["hbm_copy"] = {"bytes_read": nbytes, "bytes_written": nbytes, "ms": ms,
                       "GBps_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}
    out["peak_mad_per_s_derived"] = PEAK_MAD_PER_S
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--c", type=int, default=0,
                    help="window width (0: sweep the encodings and widths, take the best)")
    ap.add_argument("--encoding", default="glv", choices=sorted(ENCODINGS),
                    help="digit encoding used with --c")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-padd-kernel", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-serve", action="store_true", help="skip the served workload")
    ap.add_argument("--serve-seconds", type=float, default=6.0,
                    help="measured seconds of the served trace (after 1 s of warm-up)")
    ap.add_argument("--serve-full", action="store_true",
                    help="served trace of 5 s warm-up + 30 s, plus a run with a 2 GB budget")
    ap.add_argument("--microbench", action="store_true",
                    help="only measure the VALU mad / carry-add issue rates and HBM copy bandwidth")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X and has no "
              "multi-GPU path (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.microbench:
        print(json.dumps(microbench()))
        return

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(16)

    import numpy as np
    import torch

    from paper_2502_11660_amd import api, inputs

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    n = N_POINTS
    seed = inputs.config_seed(3)
    kw = inputs.nonzero_scalars_mod_r(seed, n, stream=1)
    sw = inputs.scalars_mod_r(seed, n, stream=2)
    k_dev = api.to_device(kw, dev)
    s_dev = api.to_device(sw, dev)

    print("[bench] generating %d points on the GPU ..." % n, file=sys.stderr, flush=True)
    xy, inf = api.gen_points(k_dev, n)
    torch.cuda.synchronize()
    xyu = None

    def prep():
        nonlocal xyu
        xyu, _ = api.points_prepare(xy, n, inf=inf, out=xyu)

    prep()
    prepare_ms = timed(prep, 3, torch)
    xyu_endo = None

    def prep_endo():
        nonlocal xyu_endo
        xyu_endo, _ = api.points_prepare(xy, n, inf=inf, out=xyu_endo, endo=True)

    prep_endo()
    prepare_endo_ms = timed(prep_endo, 3, torch)
    pts_for = {"signed": xyu, "unsigned": xyu, "glv": xyu_endo}

    # (encoding, window) sweep
    sweep = {}
    cands = [(args.encoding, args.c)] if args.c else SWEEP
    for enc, c in cands:
        ws = api.workspace(n, c, ENCODINGS[enc], device=dev)
        res = api.words(api.MSM_RESULT_WORDS, dev)
        fn = lambda: api.msm_run(pts_for[enc], s_dev, n, c, ENCODINGS[enc], result=res, ws=ws)
        fn()
        sweep[(enc, c)] = timed(fn, 2, torch)
        del ws
        print("[bench] %s c=%d: %.3f ms" % (enc, c, sweep[(enc, c)]), file=sys.stderr, flush=True)
    best_enc, best_c = min(sweep, key=sweep.get)

    ws = api.workspace(n, best_c, ENCODINGS[best_enc], device=dev)
    res = api.words(api.MSM_RESULT_WORDS, dev)
    step = lambda: api.msm_run(pts_for[best_enc], s_dev, n, best_c, ENCODINGS[best_enc],
                               result=res, ws=ws)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for ph in ("sort", "accum", "merge", "agg", "horner"):
        api.profile_read(ph)
    # timed steps: the accumulation kernel carries start / stop events on its
    # own dispatch (no event records between kernels)
    api.profile_enable(api.MSM_PROFILE_ACCUM_KERNEL)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(args.steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    api.profile_enable(api.MSM_PROFILE_OFF)
    ms_per_step = t0.elapsed_time(t1) / args.steps
    tot, cnt = api.profile_read("accum")
    accum_tot_ms = tot / max(cnt, 1)
    # phase split from separate steps with events around every phase (which
    # stall the stream briefly at each phase boundary)
    api.profile_enable(api.MSM_PROFILE_PHASES)
    for _ in range(min(args.steps, 3)):
        step()
    torch.cuda.synchronize()
    api.profile_enable(api.MSM_PROFILE_OFF)
    phases = {}
    for ph in ("sort", "accum", "merge", "agg", "horner"):
        tot, cnt = api.profile_read(ph)
        phases[ph] = tot / max(cnt, 1)
    # the result of the timed runs, against the closed form
    from oracle import msm as msm_oracle
    ok_result = api.decode_result(api.to_host(res)) == (
        msm_oracle.closed_form([inputs.words_to_int(r) for r in sw],
                               [inputs.words_to_int(r) for r in kw]), 0)

    entries = nonzero_digit_entries(sw, best_c, best_enc)
    padds = padd_count_executed(entries, best_c, best_enc)
    value = padds / (ms_per_step * 1e-3)
    accum_mads = entries * MULS_MIXED * MAD_PER_MUL
    achieved = accum_mads / (accum_tot_ms * 1e-3)

    padd_k = None
    chain_stream = None
    if not args.no_padd_kernel:
        pool_n = 8192
        padd_k = padd_kernel_bench(torch, api, xyu[:pool_n * 36], pool_n, 1 << 22, 5)
        chain_stream = chain_and_stream_bench(torch, api, xyu, padd_k.pop("_a_pool"), pool_n)
        chain_stream["field_cores"] = field_core_bench(torch, api, inputs)

    if cpu is not None:
        cpu["msm_ms_extrapolated"] = padds / cpu["value"] * 1e3
        cpu["sample"] = cpu["sample"].replace("c=16", "c=%d" % best_c)

    del ws
    ks_pool = [inputs.words_to_int(r) for r in kw[:N_CHECK_POOL]]
    batched = None
    if not args.no_batch:
        batched = batched_bench(torch, api, inputs, pts_for, ks_pool, args)
    served = None
    if not args.no_serve:
        served = served_bench(torch, api, inputs, pts_for, ks_pool, args)

    out = {
        "metric": "PADDs/s and MSM latency (ms) at n=2^20; batched/served MSMs/s + p99 vs plain",
        "value": value,
        "unit": "PADD/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "BLS12-377 G1 MSM, n=2^20 points k_i*G, uniform scalars mod r",
                   "n": n, "c": best_c, "digits": best_enc,
                   "windows": num_windows(best_c, best_enc), "seed": seed,
                   "padds_per_msm": padds,
                   "padds_per_msm_unsigned_formula": padd_count_formula(n, best_c)},
        "msm_ms": ms_per_step,
        "result_matches_closed_form": bool(ok_result),
        "prepare_ms": prepare_ms,
        "prepare_endo_ms": prepare_endo_ms,
        "sweep_ms": {"%s_c%d" % k: v for k, v in sweep.items()},
        "phase_ms": phases,
        "roofline": {
            "kernel": "k_accum (bucket accumulation, mixed PADD)",
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_MAD_PER_S / 1e12,
            "unit": "Tmad/s (32x32->64 multiply-adds)",
            "frac": achieved / PEAK_MAD_PER_S,
            "mad_with_carry_ceiling_frac": MAD_WITH_CARRY_CEILING,
            "frac_of_that_ceiling": achieved / PEAK_MAD_PER_S / MAD_WITH_CARRY_CEILING,
            "traffic": accum_traffic(),
            "work_per_launch": {"mixed_padds": entries, "mad_per_padd": MULS_MIXED * MAD_PER_MUL},
            "launch_ms": accum_tot_ms,
        },
        "padd_kernel": padd_k,
        "padd_workloads": chain_stream,
        "batched": batched,
        "served": served,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


# ---------------------------------------------------------------------------
# batched and served workloads
# ---------------------------------------------------------------------------

N_CHECK_POOL = 1 << 18   # pool points whose discrete logs the checks use


def _closed_form_ok(msm_oracle, api, inputs, res_words, sc_words, ks):
    ss = [inputs.words_to_int(r) for r in sc_words]
    return api.decode_result(res_words) == (msm_oracle.closed_form(ss, ks), 0)


def batched_bench(torch, api, inputs, pools, ks_pool, args):
    """64 MSMs, n_j = floor(2^u), u ~ U[10, 18]: one graph-replayed batch with
    autotuned widths (signed digits and the endomorphism split), against 64
    sequential msm_run calls with the static width."""
    xyu_pool = pools["signed"]
    import numpy as np
    from oracle import msm as msm_oracle
    from paper_2502_11660_amd import autotune

    seed = inputs.config_seed(4)
    sizes = [int(x) for x in inputs.log_uniform_sizes(seed, 64, 10, 18)]
    npool = xyu_pool.numel() // 36
    ntot = sum(sizes)
    sw = inputs.scalars_mod_r(seed, ntot, stream=2)
    s_dev = api.to_device(sw)
    rng = np.random.Generator(np.random.PCG64([seed, 3]))
    offs = [int(rng.integers(0, N_CHECK_POOL - n + 1)) if n <= N_CHECK_POOL // 2
            else int(rng.integers(0, npool - n + 1)) for n in sizes]
    bu = sorted({autotune.n_bucket(n) for n in sizes})
    tuners = {}
    t0 = time.perf_counter()
    for enc in ("signed", "glv"):
        tuners[enc] = autotune.Autotuner(encoding=ENCODINGS[enc], context="batch")
        for u in bu:
            tuners[enc].tune(u, pools[enc], s_dev)
    tune_s = time.perf_counter() - t0
    print("[bench] autotuned %d size classes x 2 encodings in %.1f s" % (len(bu), tune_s),
          file=sys.stderr, flush=True)

    def jobs_with(enc, cfun, results):
        rec = 2 if enc == "glv" else 1
        jobs, so = [], 0
        for j, n in enumerate(sizes):
            o = offs[j]
            jobs.append((pools[enc][rec * o * 36:rec * (o + n) * 36], s_dev[so * 8:(so + n) * 8],
                         results[j], n, cfun(n)))
            so += n
        return jobs

    reps = 5
    out = {"jobs": 64, "points": ntot, "sizes_log2_range": [10, 18], "seed": seed,
           "autotune_s": tune_s,
           "tuned_c": {enc: {"u%d" % u: t.choose(1 << u) for u in bu} for enc, t in tuners.items()}}
    res_b = {enc: [api.words(api.MSM_RESULT_WORDS) for _ in sizes] for enc in tuners}
    for enc, t in tuners.items():
        for graph in (True, False):
            b = api.Batch(jobs_with(enc, t.choose, res_b[enc]), ENCODINGS[enc], use_graph=graph)
            b.run()
            ms = timed(b.run, reps, torch)
            out["batched_%s_%s" % (enc, "graph" if graph else "nograph")] = {
                "ms": ms, "msms_per_s": 64 / (ms * 1e-3),
                "classes": len({t.choose(n) for n in sizes})}
            b.destroy()
    best = min((k for k in out if k.startswith("batched_")), key=lambda k: out[k]["ms"])
    out["batched_best"] = best
    maxws = max(api.workspace_bytes(n, api.default_window(n)) for n in sizes)
    ws = torch.empty((maxws + 3) // 4, dtype=torch.int32, device=xyu_pool.device)
    res_p = [api.words(api.MSM_RESULT_WORDS) for _ in sizes]
    jobs = jobs_with("signed", api.default_window, res_p)

    def seq():
        for (x, sc, r, n, c) in jobs:
            api.msm_run(x, sc, n, c, result=r, ws=ws)
    seq()
    ms = timed(seq, reps, torch)
    out["plain_static_c"] = {"ms": ms, "msms_per_s": 64 / (ms * 1e-3),
                             "what": "64 sequential msm_run, signed digits, msm_default_window"}
    torch.cuda.synchronize()
    same = all(np.array_equal(api.to_host(a), api.to_host(b))
               for enc in res_b for a, b in zip(res_b[enc], res_p))
    checked = 0
    so = 0
    ok = True
    for j, n in enumerate(sizes):
        if offs[j] + n <= len(ks_pool) and checked < 8:
            ok &= _closed_form_ok(msm_oracle, api, inputs, api.to_host(res_p[j]),
                                  sw[so:so + n], ks_pool[offs[j]:offs[j] + n])
            checked += 1
        so += n
    out["results_equal_plain_vs_batched"] = bool(same)
    out["closed_form_checked_jobs"] = checked
    out["closed_form_ok"] = bool(ok)
    out["speedup_vs_plain_static"] = out["plain_static_c"]["ms"] / out[best]["ms"]
    print("[bench] batched (%s) %.2f ms vs plain %.2f ms" % (best, out[best]["ms"],
                                                           out["plain_static_c"]["ms"]),
          file=sys.stderr, flush=True)
    return out


def served_bench(torch, api, inputs, pools, ks_pool, args):
    """Poisson arrivals at 200/s, n = floor(2^u), u ~ U[12, 20], replayed
    through the MSM server (endomorphism split, solo-tuned widths) and
    through the plain path one at a time (msm_run, signed digits, static
    width)."""
    xyu_pool = pools["signed"]
    import numpy as np
    from oracle import msm as msm_oracle
    from paper_2502_11660_amd import autotune, serve

    seed = inputs.config_seed(5)
    warm, meas = (5.0, 30.0) if args.serve_full else (1.0, args.serve_seconds)
    arrivals = inputs.poisson_arrivals(seed, 200.0, warm + meas)
    nreq = len(arrivals)
    sizes = [int(x) for x in inputs.log_uniform_sizes(seed, nreq, 12, 20, stream=1)]
    npool = xyu_pool.numel() // 36
    spool_n = 1 << 21
    sw = inputs.scalars_mod_r(seed, spool_n, stream=2)
    s_dev = api.to_device(sw)
    rng = np.random.Generator(np.random.PCG64([seed, 3]))
    poffs = [int(rng.integers(0, npool - n + 1)) for n in sizes]
    soffs = [int(rng.integers(0, spool_n - n + 1)) for n in sizes]
    tuner = autotune.Autotuner(encoding=ENCODINGS["glv"], context="solo")
    for u in range(12, 21):
        if not tuner.tuned(u):
            tuner.tune(u, pools["glv"], s_dev)
    out_tuned = {"u%d" % u: tuner.choose(1 << u) for u in range(12, 21)}
    results = torch.zeros(nreq, api.MSM_RESULT_WORDS, dtype=torch.int32, device=xyu_pool.device)

    def jobs_for(enc, cfun):
        rec = 2 if enc == "glv" else 1
        return [(pools[enc][rec * po * 36:rec * (po + n) * 36], s_dev[so * 8:(so + n) * 8],
                 results[i], n, cfun(n))
                for i, (n, po, so) in enumerate(zip(sizes, poffs, soffs))]

    measured = np.asarray(arrivals) >= warm
    free, _ = torch.cuda.mem_get_info()
    out = {"rate_per_s": 200.0, "warmup_s": warm, "measured_s": meas, "requests": nreq,
           "sizes_log2_range": [12, 20], "seed": seed, "streams": 4,
           "tuned_c_solo": out_tuned}
    budgets = [("half_free_hbm", int(free * 0.5))]
    if args.serve_full:
        budgets.append(("2GB", 2 << 30))
    served_words = None
    for name, budget in budgets:
        srv = api.Server(budget, streams=4, encoding=ENCODINGS["glv"])
        print("[bench] serving %d requests, budget %.1f GB ..." % (nreq, budget / 1e9),
              file=sys.stderr, flush=True)
        lat, wall = serve.replay_served(srv, arrivals, jobs_for("glv", tuner.choose),
                                        progress_every=5.0)
        srv.destroy()
        out[name] = serve.summarize(lat, wall, measured)
        out[name]["budget_bytes"] = budget
        if served_words is None:
            torch.cuda.synchronize()
            served_words = results.cpu().numpy().copy()
    results.zero_()
    maxws = max(api.workspace_bytes(n, 0) for n in set(sizes))
    ws = torch.empty((maxws + 3) // 4, dtype=torch.int32, device=xyu_pool.device)
    print("[bench] plain replay ...", file=sys.stderr, flush=True)
    lat_p, wall_p = serve.replay_plain(arrivals, jobs_for("signed", lambda n: 0),
                                       workspaces=lambda n, c: ws, progress_every=5.0)
    out["plain_fifo"] = serve.summarize(lat_p, wall_p, measured)
    plain_words = results.cpu().numpy()
    out["results_equal_served_vs_plain"] = bool(np.array_equal(served_words, plain_words))
    ok, checked = True, 0
    for i, n in enumerate(sizes):
        if poffs[i] + n <= len(ks_pool) and checked < 6:
            ok &= _closed_form_ok(msm_oracle, api, inputs, plain_words[i].view(np.uint32),
                                  sw[soffs[i]:soffs[i] + n], ks_pool[poffs[i]:poffs[i] + n])
            checked += 1
    out["closed_form_checked_requests"] = checked
    out["closed_form_ok"] = bool(ok)
    return out


def accum_traffic():
    """HBM bytes per accumulation launch from the committed rocprofv3 counter
    summary, if it was taken on the current accumulation kernel sources."""
    from paper_2502_11660_amd import profsum
    path = os.path.join(ROOT, "profiles", "k_accum_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != profsum.sources_sha256(rec.get("sources", [])):
        return None
    return rec.get("bytes_per_launch")


if __name__ == "__main__":
    main()
