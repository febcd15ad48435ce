#!/usr/bin/env python3
"""Benchmark: BLS12-377 G1 multi-scalar multiplication on one MI355X (gfx950).

One step = one full MSM (msm_run: digit sort, bucket accumulation, bucket
aggregation, group aggregation, affine result) over n = 2^20 seeded synthetic
points P_i = k_i G with uniform scalars mod r -- the n = 2^20 workload the
headline metric is quoted on.  Points are generated and prepared on the GPU
before the timed region (preparation is reported separately, beside the
headline).

value = PADDs/s: the point additions and doublings one MSM executes (every
non-zero digit's mixed addition, the aggregation tree's additions, the window
and group Horner steps; split-bucket merges are not counted) divided by the
MSM time; ms_per_step = MSM latency.

Prints one JSON line.  Besides the headline it reports the five workloads:
  1  n = 1024, c = 8, plain unsigned slices, against the naive MSM;
  2  the batched PADD kernel alone on 2^22 pairs (both forms), 4096 sampled
     outputs checked;
  3  n = 2^20 swept over c = 10..16 (and wider) for the unsigned slices, the
     signed digits and the endomorphism split, every width checked;
  4  64 MSMs of log-uniform sizes batched, against 64 plain launches with the
     static and with the same tuned widths, every job checked;
  5  a Poisson request stream served, against the plain path one request at
     a time with the same encoding and widths, at 200/s and at saturation,
     plus a 2 GB budget that forces queueing; several hundred requests
     checked.
and the roofline of the dominant kernel.

The oracle is used only in the cpu_baseline leg (cpu_leg and
cpu_leg_compare below).  cpu_leg runs before the GPU is touched: it times the
oracle on a bounded slice of the n = 2^20 workload (the CPU baseline) and
computes the expected results of every output the GPU legs check (the closed
form sum s_i (k_i G) = ((sum s_i k_i) mod r) G, the naive MSM of workload 1,
and the affine sums of the sampled PADD pairs); cpu_leg_compare normalises
the sampled PADD outputs after the GPU legs.  The GPU legs compute nothing
with the oracle.
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

import numpy as np  # noqa: E402

N_POINTS = 1 << 20
ENCODINGS = {"signed": 0, "unsigned": 1, "glv": 2}
# window widths swept at n = 2^20, per encoding (requested widths; widths
# that the library lowers to the same window layout run once)
SWEEP = {"unsigned": list(range(10, 17)), "signed": list(range(10, 18)),
         "glv": list(range(10, 21))}
DIGIT_BITS = {"signed": 254, "unsigned": 253, "glv": 128}
MAD_PER_MUL = 276          # 144 a*b + 132 m*p 32x32-bit word products per Montgomery multiply
MULS_MIXED = 7             # mixed PADD (Z2 = 1, U2 = k T2)
MULS_COMPLETE = 9          # complete PADD with k T2 formed on the fly
# gfx950 VALU: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz, one 32-bit lane op
# (a v_mad_u64_u32 among them) per lane per cycle
PEAK_LANE_OPS = 256 * 64 * 2.4e9

PAIRS = 1 << 22            # workload 2
PAIR_POOL = 8192
PAIR_SAMPLE = 4096
JOBS = 64                  # workload 4
SERVE_RATE = 200.0         # workload 5
SERVE_CHECKED = 400
SATURATION_REQUESTS = 600
CPU_SLICE = 1 << 11        # oracle naive MSM slice of the n = 2^20 workload


def padd_count_formula(n, c):
    """Unsigned-digit Pippenger count n W + 2 (2^c - 1) W + W c + W - 1."""
    W = -(-253 // c)
    return n * W + 2 * ((1 << c) - 1) * W + W * c + W - 1


def num_windows(c, encoding):
    return -(-DIGIT_BITS[encoding] // c)


def window_bits(c, encoding):
    """The width the library runs for a requested c (msm_window_bits): the
    window count of c, and the smallest width that covers the digit bits
    with that many windows."""
    return -(-DIGIT_BITS[encoding] // num_windows(c, encoding))


def padd_count_executed(entries, c, encoding="signed", jobs=1):
    """Additions and doublings the implementation executes for one MSM at
    the effective width c (window_bits): accumulation (one mixed addition
    per non-zero digit), the aggregation tree (2^(bb+1) - bb - 2 per window),
    the window Horner steps and the group Horner steps (c doublings and one
    addition per window but the top)."""
    signed = encoding != "unsigned"
    W = num_windows(c, encoding)
    bb = c - 1 if signed else c
    S = W * jobs
    tree = S * ((1 << (bb + 1)) - bb - 2)
    combine = S * (2 * bb - 1 + (1 if signed else 0))
    horner = jobs * (W - 1) * (c + 1)
    return entries + tree + combine + horner


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_cores():
    return max(1, min(os.cpu_count() or 1, 16))


# ---------------------------------------------------------------------------
# workloads: seeded host-side definitions shared by the GPU legs and the
# oracle (random draws only, no arithmetic of the method)
# ---------------------------------------------------------------------------

class Workloads:
    def __init__(self, args):
        from paper_2502_11660_amd import inputs
        self.inputs = inputs
        n = N_POINTS
        self.seed3 = inputs.config_seed(3)
        self.kw = inputs.nonzero_scalars_mod_r(self.seed3, n, stream=1)   # P_i = k_i G
        self.sw = inputs.scalars_mod_r(self.seed3, n, stream=2)           # MSM scalars
        # workload 1: the first 1024 points, their own scalars
        self.seed1 = inputs.config_seed(1)
        self.s1 = inputs.scalars_mod_r(self.seed1, 1024, stream=2)
        # workload 2: pairs over the first PAIR_POOL points; a-operands are
        # P_j + P_{j-1} (built on the GPU), b-operands P_j (mixed) or
        # P_j + P_{j-1} (complete)
        seed2 = inputs.config_seed(2)
        rng = np.random.Generator(np.random.PCG64([seed2, 1]))
        self.ja = rng.integers(0, PAIR_POOL, PAIRS)
        self.jb = rng.integers(0, PAIR_POOL, PAIRS)
        self.pair_sample = np.sort(rng.choice(PAIRS, PAIR_SAMPLE, replace=False))
        self.pair_sample[-1] = PAIRS - 1
        # workload 4: 64 jobs, n = floor(2^u), u ~ U[10, 18], slices of the pool
        self.seed4 = inputs.config_seed(4)
        self.sizes4 = [int(x) for x in inputs.log_uniform_sizes(self.seed4, JOBS, 10, 18)]
        self.s4 = inputs.scalars_mod_r(self.seed4, sum(self.sizes4), stream=2)
        rng = np.random.Generator(np.random.PCG64([self.seed4, 3]))
        self.offs4 = [int(rng.integers(0, n - m + 1)) for m in self.sizes4]
        self.soffs4 = np.concatenate([[0], np.cumsum(self.sizes4)[:-1]]).astype(int).tolist()
        # workload 5: Poisson arrivals, n = floor(2^u), u ~ U[12, 20]
        self.seed5 = inputs.config_seed(5)
        self.serve_warm, self.serve_meas = args.serve_warmup, args.serve_seconds
        self.arrivals = inputs.poisson_arrivals(self.seed5, SERVE_RATE,
                                                self.serve_warm + self.serve_meas)
        nreq = len(self.arrivals)
        self.sizes5 = [int(x) for x in inputs.log_uniform_sizes(self.seed5, nreq, 12, 20, stream=1)]
        self.spool5 = 1 << 21
        self.s5 = inputs.scalars_mod_r(self.seed5, self.spool5, stream=2)
        rng = np.random.Generator(np.random.PCG64([self.seed5, 3]))
        self.poffs5 = [int(rng.integers(0, n - m + 1)) for m in self.sizes5]
        self.soffs5 = [int(rng.integers(0, self.spool5 - m + 1)) for m in self.sizes5]
        rng = np.random.Generator(np.random.PCG64([self.seed5, 4]))
        self.check5 = sorted(rng.choice(nreq, min(SERVE_CHECKED, nreq), replace=False).tolist())


# ---------------------------------------------------------------------------
# cpu_baseline leg: the oracle (runs before the GPU is touched, so worker
# processes are forked from a GPU-free process)
# ---------------------------------------------------------------------------

_WL = None   # the workloads, inherited by forked workers


def _naive_slice(args):
    """Oracle naive MSM sum s_i P_i over points [lo, hi) of the n = 2^20
    workload; returns the partial sum and the wall time."""
    lo, hi = args
    from oracle import curve, msm, points
    inp = _WL.inputs
    pts = [points.fixed_base_mul(inp.words_to_int(r)) for r in _WL.kw[lo:hi]]
    ss = [inp.words_to_int(r) for r in _WL.sw[lo:hi]]
    t0 = time.perf_counter()
    part = msm.msm_naive(ss, pts)
    dt = time.perf_counter() - t0
    # additions and doublings of double-and-add: bits - 1 doublings and
    # popcount additions per scalar (one more addition into the sum)
    ops = sum(max(0, s.bit_length() - 1) + bin(s).count("1") for s in ss) + len(ss)
    return part, dt, ops


def _naive_config1(args):
    lo, hi = args
    from oracle import msm, points
    inp = _WL.inputs
    pts = [points.fixed_base_mul(inp.words_to_int(r)) for r in _WL.kw[lo:hi]]
    ss = [inp.words_to_int(r) for r in _WL.s1[lo:hi]]
    t0 = time.perf_counter()
    part = msm.msm_naive(ss, pts)
    return part, time.perf_counter() - t0


def _pool_point(j):
    from oracle import points
    return points.fixed_base_mul(_WL.inputs.words_to_int(_WL.kw[j]))


def _closed_form(args):
    """Expected MSM result of scalars s_words with points k_words G."""
    which, idx = args
    from oracle import msm
    if which == "slice":
        return msm.closed_form_words(_WL.sw[:CPU_SLICE], _WL.kw[:CPU_SLICE])
    if which == "c3":
        return msm.closed_form_words(_WL.sw, _WL.kw)
    if which == "c4":
        m, o, so = _WL.sizes4[idx], _WL.offs4[idx], _WL.soffs4[idx]
        return msm.closed_form_words(_WL.s4[so:so + m], _WL.kw[o:o + m])
    m, o, so = _WL.sizes5[idx], _WL.poffs5[idx], _WL.soffs5[idx]
    return msm.closed_form_words(_WL.s5[so:so + m], _WL.kw[o:o + m])


def cpu_leg(wl, skip_baseline=False):
    """Oracle work: the timed CPU baseline and the expected values of every
    checked GPU output."""
    global _WL
    import multiprocessing as mp
    from oracle import curve
    _WL = wl
    cores = cpu_cores()
    ctx = mp.get_context("fork")
    out = {"expected": {}}
    with ctx.Pool(cores) as pool:
        if not skip_baseline:
            # baseline: naive MSM (double-and-add per point, affine additions)
            # over the first CPU_SLICE points of the n = 2^20 workload
            step = CPU_SLICE // (4 * cores)
            chunks = [(lo, min(lo + step, CPU_SLICE)) for lo in range(0, CPU_SLICE, step)]
            t0 = time.perf_counter()
            res = pool.map(_naive_slice, chunks)
            wall = time.perf_counter() - t0
            acc = curve.INF
            for part, _, _ in res:
                acc = curve.add(acc, part)
            ops = sum(r[2] for r in res)
            cpu_s = sum(r[1] for r in res)
            out["baseline"] = {
                "value": ops / wall,
                "unit": "PADD/s",
                "cores": cores,
                "kind": "oracle",
                "sample": ("naive MSM (double-and-add, affine Weierstrass additions) of the first "
                           "%d points and scalars of the n=2^20 workload on %d processes: %d "
                           "additions and doublings in %.2f s wall (%.1f s of CPU time); value "
                           "= those operations per wall second" % (CPU_SLICE, cores, ops, wall,
                                                                  cpu_s)),
                "cpu_model": cpu_model(),
                "points_per_s": CPU_SLICE / wall,
                "msm_n2p20_s_extrapolated": N_POINTS * wall / CPU_SLICE,
                "slice_equals_closed_form": acc == _closed_form(("slice", 0)),
            }
            # workload 1: the full naive MSM at n = 1024
            t0 = time.perf_counter()
            res1 = pool.map(_naive_config1, [(lo, lo + 64) for lo in range(0, 1024, 64)])
            wall1 = time.perf_counter() - t0
            acc1 = curve.INF
            for part, _ in res1:
                acc1 = curve.add(acc1, part)
            out["baseline"]["config1_msm_naive_wall_ms"] = wall1 * 1e3
            out["baseline"]["config1_msm_naive_cpu_ms"] = sum(r[1] for r in res1) * 1e3
            out["expected"]["c1"] = acc1
        else:
            res1 = pool.map(_naive_config1, [(lo, lo + 64) for lo in range(0, 1024, 64)])
            acc1 = curve.INF
            for part, _ in res1:
                acc1 = curve.add(acc1, part)
            out["expected"]["c1"] = acc1
        # workload 2: affine sums of the sampled pairs
        need = set()
        for i in wl.pair_sample:
            for j in (wl.ja[i], wl.jb[i]):
                need.update((int(j), int((j - 1) % PAIR_POOL)))
        need = sorted(need)
        t0 = time.perf_counter()
        P = dict(zip(need, pool.map(_pool_point, need, chunksize=64)))
        mixed, complete = [], []
        t1 = time.perf_counter()
        for i in wl.pair_sample:
            a, b = int(wl.ja[i]), int(wl.jb[i])
            pa = curve.add(P[a], P[(a - 1) % PAIR_POOL])
            mixed.append(curve.add(pa, P[b]))
            complete.append(curve.add(pa, curve.add(P[b], P[(b - 1) % PAIR_POOL])))
        t2 = time.perf_counter()
        out["expected"]["c2_mixed"] = mixed
        out["expected"]["c2_complete"] = complete
        out["pair_sample_oracle"] = {"points_s": t1 - t0, "adds": 5 * len(wl.pair_sample),
                                     "adds_s_one_core": t2 - t1}
        # workloads 3, 4, 5: closed forms
        tasks = [("c3", 0)] + [("c4", j) for j in range(JOBS)] + [("c5", i) for i in wl.check5]
        t0 = time.perf_counter()
        vals = pool.map(_closed_form, tasks, chunksize=4)
        out["closed_forms_s"] = time.perf_counter() - t0
        out["expected"]["c3"] = vals[0]
        out["expected"]["c4"] = vals[1:1 + JOBS]
        out["expected"]["c5"] = dict(zip(wl.check5, vals[1 + JOBS:]))
    return out


def cpu_leg_compare(expected, gathered):
    """The oracle side of the checks, after the GPU legs: the sampled PADD
    outputs (canonical Montgomery-form extended records) normalised to
    Weierstrass affine points and compared with the oracle's sums.  MSM
    results are affine already and are compared as decoded."""
    from oracle import te
    from tests import helpers as H
    out = {}
    for form, smp in gathered.items():
        got = [te.te_to_w(H.normalize_extended_mont(tuple(
            sum(int(smp[c * 12 + l, t]) << (32 * l) for l in range(12)) for c in range(4))))
            for t in range(smp.shape[1])]
        out[form] = got == expected["c2_" + form]
    return out


# ---------------------------------------------------------------------------
# GPU legs
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
    """Scalar words -> words of the endomorphism halves (s0, s1) per scalar
    (host-side count of the digits, not a step of the MSM)."""
    from paper_2502_11660_amd import inputs
    lam = 0x8508C00000000001 ** 2 - 1
    ints = [inputs.words_to_int(r) for r in sw_np.reshape(-1, 8)]
    halves = []
    for v in ints:
        halves += [v % lam, v // lam]
    return np.asarray(inputs.ints_to_words(halves, 8), dtype=np.uint32)


def nonzero_digit_entries(sw_np, c, encoding="signed"):
    """Number of (point, window) pairs with a non-zero digit at the effective
    width c (window_bits): the mixed PADDs bucket accumulation performs."""
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


def sweep_leg(torch, api, wl, pts_for, s_dev, args):
    """Workload 3: every encoding at every width of SWEEP."""
    dev = s_dev.device
    out = {}
    req = [(args.encoding, args.c)] if args.c else [(e, c) for e in SWEEP for c in SWEEP[e]]
    cands = []
    for enc, c in req:   # effective widths, each once
        if (enc, window_bits(c, enc)) not in cands:
            cands.append((enc, window_bits(c, enc)))
    for enc, c in cands:
        ws = api.workspace(N_POINTS, c, ENCODINGS[enc], device=dev)
        res = api.words(api.MSM_RESULT_WORDS, dev)
        fn = lambda: api.msm_run(pts_for[enc], s_dev, N_POINTS, c, ENCODINGS[enc],
                                 result=res, ws=ws)
        fn()
        ms = timed(fn, 2, torch)
        out[(enc, c)] = (ms, api.to_host(res).copy())
        del ws
        print("[bench] %s c=%d: %.3f ms" % (enc, c, ms), file=sys.stderr, flush=True)
    return out


def padd_kernel_leg(torch, api, wl, xyu_pool, reps):
    """Workload 2: the batched PADD kernel on 2^22 independent pairs (SoA),
    both forms.  Pool records: prepared b_j = P_j; extended a_j = P_j +
    P_{j-1} (two mixed additions from the identity), so every a has Z != 1."""
    dev = xyu_pool.device
    aos = xyu_pool[:PAIR_POOL * 36].view(PAIR_POOL, 3, 12)
    soa_b = aos.permute(1, 2, 0).contiguous()             # (3, 12, pool) prepared
    ident = torch.zeros(4, 12, PAIR_POOL, dtype=torch.int32, device=dev)
    one = api.to_device(np.array([0xffffff68, 0x02cdffff, 0x7fffffb1, 0x51409f83, 0x8a7d3ff2,
                                  0x9f7db3a9, 0x6e7c6305, 0x7b4e97b7, 0x803c84e8, 0x4cf495bf,
                                  0xe2fdf49a, 0x008d6661], dtype=np.uint32), dev)
    ident[1] = one.view(12, 1)
    ident[3] = one.view(12, 1)
    a_pool = api.padd_batch(ident.reshape(-1), soa_b.reshape(-1), PAIR_POOL, api.MSM_FORM_XYU)
    rot = torch.roll(soa_b, 1, dims=2).contiguous()       # column j holds P_{j-1}
    a_pool = api.padd_batch(a_pool, rot.reshape(-1), PAIR_POOL, api.MSM_FORM_XYU)
    ja = torch.from_numpy(wl.ja).to(dev)
    jb = torch.from_numpy(wl.jb).to(dev)
    A = a_pool.view(4, 12, PAIR_POOL).index_select(2, ja).contiguous().view(-1)
    Bm = soa_b.index_select(2, jb).contiguous().view(-1)
    Bc = a_pool.view(4, 12, PAIR_POOL).index_select(2, jb).contiguous().view(-1)
    out = torch.empty_like(A)
    smp = torch.from_numpy(wl.pair_sample).to(dev)
    res = {"_a_pool": a_pool}
    for name, B, form, muls, nbytes in (("mixed", Bm, api.MSM_FORM_XYU, MULS_MIXED, 48 * 4 * 2 + 36 * 4),
                                        ("complete", Bc, api.MSM_FORM_XYTZ, MULS_COMPLETE, 48 * 4 * 3)):
        fn = lambda: api.padd_batch(A, B, PAIRS, form, out=out)
        fn()
        ms = timed(fn, reps, torch)
        rate = PAIRS / (ms * 1e-3)
        sample = out.view(48, PAIRS).index_select(1, smp).cpu().numpy().view(np.uint32).copy()
        res[name] = {
            "pairs": PAIRS,
            "ms": ms,
            "padd_per_s": rate,
            "word_mad_per_s": rate * muls * MAD_PER_MUL,
            "frac_of_valu_lane_peak": rate * muls * MAD_PER_MUL / PEAK_LANE_OPS,
            "hbm_GBps": rate * nbytes / 1e9,
            "_sample": sample,
        }
    return res


def chain_and_stream_leg(torch, api, xyu_pool, a_pool_soa):
    """The paper's latency workload (a dependent chain of complete additions
    over 2^18 points) and its throughput workload (independent accumulators
    fed prepared points, result returned once)."""
    recs = a_pool_soa.view(48, PAIR_POOL).t().contiguous()          # AoS XYTZ
    out = {"paper_latency_us_per_padd": 1.05, "paper_throughput_mtask_per_s": 67.0}
    chain = {}
    for name, unit, count in (("wide", api.MSM_UNIT_WIDE, 1 << 18), ("quad", api.MSM_UNIT_QUAD, 1 << 18),
                              ("lane", api.MSM_UNIT_LANE, 1 << 16)):
        pts = recs.repeat((count + PAIR_POOL - 1) // PAIR_POOL, 1)[:count].contiguous().view(-1)
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


def field_core_leg(torch, api, inputs, count=1 << 20, rounds=64):
    """Field-multiplication cores: count lanes, each chaining `rounds`
    products.  Word products per multiply are the 32x32-bit products of the
    12-word forms (the carry-free core's own 28-bit products in brackets)."""
    a = api.to_device(inputs.base_field_elements(inputs.config_seed(2), count, stream=7).T.copy())
    b = api.to_device(inputs.base_field_elements(inputs.config_seed(2), count, stream=8).T.copy())
    out = api.words(12 * count)
    res = {}
    for name, var, mads in (("montgomery", api.MSM_MUL_MONT, MAD_PER_MUL),
                            ("barrett_k378", api.MSM_MUL_BARRETT, 144 + 99 + 78),
                            ("karatsuba_montgomery", api.MSM_MUL_KARATSUBA, 3 * 36 + 132),
                            ("carry_free_28bit_montgomery", api.MSM_MUL_F28, 378)):
        api.fe_mul_chain(a, b, count, var, 2, out=out)
        ms = timed(lambda: api.fe_mul_chain(a, b, count, var, rounds, out=out), 3, torch)
        rate = count * rounds / (ms * 1e-3)
        res[name] = {"ms": ms, "mul_per_s": rate, "mads_per_mul": mads,
                     "mad_per_s": rate * mads, "frac_of_valu_lane_peak": rate * mads / PEAK_LANE_OPS}
    res["lanes"] = count
    res["rounds"] = rounds
    return res


def batched_leg(torch, api, wl, pools, s_all, isolated_run=False):
    """Workload 4: 64 MSMs, n_j = floor(2^u), u ~ U[10, 18]: one batch with
    autotuned widths (graph replay and plain enqueue, signed digits and the
    endomorphism split), against 64 sequential msm_run calls with the static
    width and with the batch's own encoding and widths."""
    from paper_2502_11660_amd import autotune
    dev = s_all.device
    s_dev = api.to_device(wl.s4, dev)
    bu = sorted({autotune.n_bucket(n) for n in wl.sizes4})
    tuners = {}
    t0 = time.perf_counter()
    for enc in ("signed", "glv"):
        tuners[enc] = autotune.Autotuner(encoding=ENCODINGS[enc], context="batch")
        for u in bu:
            tuners[enc].tune(u, pools[enc], s_all)
    tune_s = time.perf_counter() - t0
    print("[bench] autotuned %d size classes x 2 encodings in %.1f s" % (len(bu), tune_s),
          file=sys.stderr, flush=True)

    def jobs_with(enc, cfun, results, sfun=None):
        rec = 2 if enc == "glv" else 1
        jobs = []
        for j, n in enumerate(wl.sizes4):
            o, so = wl.offs4[j], wl.soffs4[j]
            jobs.append((pools[enc][rec * o * 36:rec * (o + n) * 36], s_dev[so * 8:(so + n) * 8],
                         results[j], n, cfun(n), sfun(n) if sfun else None))
        return jobs

    reps = 5
    out = {"jobs": JOBS, "points": int(sum(wl.sizes4)), "sizes_log2_range": [10, 18],
           "seed": wl.seed4, "autotune_s": tune_s,
           "tuned_c": {enc: {"u%d" % u: t.choose(1 << u) for u in bu} for enc, t in tuners.items()},
           "tuned_schedule": {enc: {"u%d" % u: t.schedule(1 << u) for u in bu}
                              for enc, t in tuners.items()}}
    res_b = {enc: [api.words(api.MSM_RESULT_WORDS, dev) for _ in wl.sizes4] for enc in tuners}
    for enc, t in tuners.items():
        for graph in (True, False):
            b = api.Batch(jobs_with(enc, t.choose, res_b[enc], t.schedule), ENCODINGS[enc],
                          use_graph=graph)
            b.run()
            ms = timed(b.run, reps, torch)
            out["batched_%s_%s" % (enc, "graph" if graph else "nograph")] = {
                "ms": ms, "msms_per_s": JOBS / (ms * 1e-3),
                "classes": len({(t.choose(n), tuple(sorted(t.schedule(n).items())))
                                for n in wl.sizes4})}
            b.destroy()
    # the best encoding's batch with widths tuned but the default schedule
    enc_s = min(("signed", "glv"), key=lambda e: min(out["batched_%s_graph" % e]["ms"],
                                                      out["batched_%s_nograph" % e]["ms"]))
    b = api.Batch(jobs_with(enc_s, tuners[enc_s].choose, res_b[enc_s]), ENCODINGS[enc_s],
                  use_graph=False)
    b.run()
    ms = timed(b.run, reps, torch)
    out["batched_%s_nograph_default_schedule" % enc_s] = {"ms": ms, "msms_per_s": JOBS / (ms * 1e-3)}
    b.destroy()
    best = min((k for k in out if k.startswith("batched_") and "default_schedule" not in k),
               key=lambda k: out[k]["ms"])
    best_enc = best.split("_")[1]
    out["batched_best"] = best
    maxws = max(max(api.workspace_bytes(n, api.default_window(n)) for n in wl.sizes4),
                max(api.workspace_bytes(n, tuners[best_enc].choose(n), ENCODINGS[best_enc])
                    for n in wl.sizes4))
    ws = torch.empty((maxws + 3) // 4, dtype=torch.int32, device=dev)

    def seq_leg(enc, cfun, results):
        jobs = jobs_with(enc, cfun, results)

        def seq():
            for (x, sc, r, n, c, _) in jobs:
                api.msm_run(x, sc, n, c, ENCODINGS[enc], result=r, ws=ws)
        seq()
        return timed(seq, reps, torch)

    res_p = [api.words(api.MSM_RESULT_WORDS, dev) for _ in wl.sizes4]
    ms = seq_leg("signed", api.default_window, res_p)
    out["plain_static_c"] = {"ms": ms, "msms_per_s": JOBS / (ms * 1e-3),
                             "what": "64 sequential msm_run, signed digits, msm_default_window"}
    res_t = [api.words(api.MSM_RESULT_WORDS, dev) for _ in wl.sizes4]
    ms = seq_leg(best_enc, tuners[best_enc].choose, res_t)
    out["plain_tuned_c"] = {"ms": ms, "msms_per_s": JOBS / (ms * 1e-3),
                            "what": "64 sequential msm_run with the best batch's encoding (%s) "
                                    "and per-job widths" % best_enc}
    out["speedup_vs_plain_static"] = out["plain_static_c"]["ms"] / out[best]["ms"]
    out["speedup_vs_plain_tuned"] = out["plain_tuned_c"]["ms"] / out[best]["ms"]
    torch.cuda.synchronize()
    out["_results"] = {"batched": [api.to_host(r).copy() for r in res_b[best_enc]],
                       "plain_static": [api.to_host(r).copy() for r in res_p],
                       "plain_tuned": [api.to_host(r).copy() for r in res_t]}
    print("[bench] batched (%s) %.2f ms vs plain %.2f (static c) / %.2f ms (same c)"
          % (best, out[best]["ms"], out["plain_static_c"]["ms"], out["plain_tuned_c"]["ms"]),
          file=sys.stderr, flush=True)
    if isolated_run:
        # one more run of the best batch with the device idle for 50 ms before
        # and after, so that a kernel trace shows it as a cluster of its own
        t = tuners[best_enc]
        b = api.Batch(jobs_with(best_enc, t.choose, res_b[best_enc], t.schedule),
                      ENCODINGS[best_enc], use_graph=best.endswith("_graph"))
        b.run()
        torch.cuda.synchronize()
        time.sleep(0.05)
        out["isolated_run_ms"] = timed(b.run, 1, torch)
        time.sleep(0.05)
        b.destroy()
    return out


def served_leg(torch, api, wl, pools, args):
    """Workload 5: Poisson arrivals at 200/s, n = floor(2^u), u ~ U[12, 20],
    replayed through the MSM server (endomorphism split, solo-tuned widths)
    and through the plain path one request at a time with the same encoding
    and widths; then every request submitted at once (saturation), and the
    200/s trace again under a 2 GB budget that forces queueing."""
    from paper_2502_11660_amd import autotune, serve
    dev = pools["glv"].device
    enc = "glv"
    s_dev = api.to_device(wl.s5, dev)
    tuner = autotune.Autotuner(encoding=ENCODINGS[enc], context="solo")
    for u in range(12, 21):
        if not tuner.tuned(u):
            tuner.tune(u, pools[enc], s_dev)
    nreq = len(wl.arrivals)
    results = torch.zeros(nreq, api.MSM_RESULT_WORDS, dtype=torch.int32, device=dev)

    def jobs_for(idx):
        return [(pools[enc][2 * wl.poffs5[i] * 36:2 * (wl.poffs5[i] + wl.sizes5[i]) * 36],
                 s_dev[wl.soffs5[i] * 8:(wl.soffs5[i] + wl.sizes5[i]) * 8],
                 results[i], wl.sizes5[i], tuner.choose(wl.sizes5[i])) for i in idx]

    measured = np.asarray(wl.arrivals) >= wl.serve_warm
    free, _ = torch.cuda.mem_get_info()
    out = {"rate_per_s": SERVE_RATE, "warmup_s": wl.serve_warm, "measured_s": wl.serve_meas,
           "requests": nreq, "sizes_log2_range": [12, 20], "seed": wl.seed5, "streams": 4,
           "encoding": enc, "tuned_c_solo": {"u%d" % u: tuner.choose(1 << u) for u in range(12, 21)}}
    maxws = max(api.workspace_bytes(n, tuner.choose(n), ENCODINGS[enc]) for n in set(wl.sizes5))
    ws = torch.empty((maxws + 3) // 4, dtype=torch.int32, device=dev)
    words = {}
    all_idx = list(range(nreq))
    budget = int(free * 0.5)
    # 200/s, half of the free HBM
    srv = api.Server(budget, streams=4, encoding=ENCODINGS[enc])
    print("[bench] serving %d requests, budget %.1f GB ..." % (nreq, budget / 1e9),
          file=sys.stderr, flush=True)
    lat, wall = serve.replay_served(srv, wl.arrivals, jobs_for(all_idx), progress_every=5.0)
    srv.destroy()
    out["served_200"] = serve.summarize(lat, wall, measured)
    out["served_200"]["budget_bytes"] = budget
    torch.cuda.synchronize()
    words["served_200"] = results.cpu().numpy().view(np.uint32).copy()
    results.zero_()
    print("[bench] plain replay ...", file=sys.stderr, flush=True)
    lat_p, wall_p = serve.replay_plain(wl.arrivals, jobs_for(all_idx), encoding=ENCODINGS[enc],
                                       workspaces=lambda n, c: ws, progress_every=5.0)
    out["plain_200"] = serve.summarize(lat_p, wall_p, measured)
    words["plain_200"] = results.cpu().numpy().view(np.uint32).copy()
    # saturation: the first SATURATION_REQUESTS requests all arrive at t = 0
    sat = list(range(min(SATURATION_REQUESTS, nreq)))
    zero = np.zeros(len(sat))
    allm = np.ones(len(sat), dtype=bool)
    results.zero_()
    srv = api.Server(budget, streams=4, encoding=ENCODINGS[enc])
    lat_s, wall_s = serve.replay_served(srv, zero, jobs_for(sat))
    srv.destroy()
    out["served_saturation"] = serve.summarize(lat_s, wall_s, allm)
    out["served_saturation"]["requests_at_t0"] = len(sat)
    torch.cuda.synchronize()
    words["served_saturation"] = results.cpu().numpy().view(np.uint32)[:len(sat)].copy()
    results.zero_()
    lat_ps, wall_ps = serve.replay_plain(zero, jobs_for(sat), encoding=ENCODINGS[enc],
                                         workspaces=lambda n, c: ws)
    out["plain_saturation"] = serve.summarize(lat_ps, wall_ps, allm)
    words["plain_saturation"] = results.cpu().numpy().view(np.uint32)[:len(sat)].copy()
    # 200/s under a 2 GB budget (a 2^20-point request needs about 0.3 GB)
    if not args.no_serve_2gb:
        results.zero_()
        srv = api.Server(2 << 30, streams=4, encoding=ENCODINGS[enc])
        print("[bench] serving %d requests, budget 2 GB ..." % nreq, file=sys.stderr, flush=True)
        lat2, wall2 = serve.replay_served(srv, wl.arrivals, jobs_for(all_idx), progress_every=5.0)
        srv.destroy()
        out["served_200_2GB"] = serve.summarize(lat2, wall2, measured)
        out["served_200_2GB"]["budget_bytes"] = 2 << 30
        torch.cuda.synchronize()
        words["served_200_2GB"] = results.cpu().numpy().view(np.uint32).copy()
    out["msms_per_s_served_over_plain_saturation"] = (
        out["served_saturation"]["msms_per_s"] / out["plain_saturation"]["msms_per_s"])
    out["_words"] = words
    return out


def host_to_device_leg(torch, xyu, xyu_endo, s_dev):
    """PCIe copy of the MSM's inputs from pinned host memory (outside `value`,
    whose inputs are resident): the prepared points, with or without the
    endomorphism images, and the scalars."""
    out = {}
    for name, t in (("prepared_points", xyu), ("prepared_points_with_images", xyu_endo),
                    ("scalars", s_dev)):
        host = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
        host.copy_(t)
        dst = torch.empty_like(t)
        ms = timed(lambda: dst.copy_(host, non_blocking=True), 3, torch)
        out[name] = {"bytes": t.numel() * t.element_size(), "ms": ms,
                     "GBps": t.numel() * t.element_size() / (ms * 1e6)}
        del host, dst
    return out


def bucket_scatter_figure(phases_ms, entries, n, records):
    """Algorithmic HBM bytes of the digit slicing and bucket sort at n points
    with `entries` digit slots (non-zero and zero digits alike are slotted),
    per the layout: 32 B of scalar read per point; per slot a 4-byte digit
    written and read, a staging entry written and read (one 4-byte word for
    jobs of at most 2^23 point records, else an 8-byte index and key pair),
    and the sorted key and index written (8 B); and the bytes the committed
    rocprofv3 counter summary measured for the sort phase's kernels, per
    slot, times these slots (null when the sort sources changed since)."""
    staged = 4 if records <= (1 << 23) else 8
    nbytes = 32 * n + entries * (4 + 4 + staged + staged + 8)
    ms = phases_ms.get("sort")
    out = {"algorithmic_bytes": nbytes, "phase_ms": ms,
           "GBps": nbytes / (ms * 1e-3) / 1e9 if ms else None,
           "traffic_bytes": None, "traffic_GBps": None}
    from paper_2502_11660_amd import profsum
    try:
        with open(os.path.join(ROOT, "profiles", "sort_phase_traffic.json")) as f:
            rec = json.load(f)
        if rec.get("sources_sha256") == profsum.sources_sha256(rec.get("sources", [])):
            tb = rec["bytes_per_entry"] * entries
            out["traffic_bytes"] = tb
            out["traffic_GBps"] = tb / (ms * 1e-3) / 1e9 if ms else None
    except (OSError, ValueError, KeyError):
        pass
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
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the timed oracle baseline (expected values are still computed)")
    ap.add_argument("--no-checks", action="store_true",
                    help="skip the oracle leg entirely (no baseline, no result checks)")
    ap.add_argument("--no-padd-kernel", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-serve", action="store_true", help="skip the served workload")
    ap.add_argument("--no-serve-2gb", action="store_true", help="skip the 2 GB served leg")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="measured seconds of the served trace")
    ap.add_argument("--serve-warmup", type=float, default=5.0,
                    help="warm-up seconds of the served trace")
    ap.add_argument("--msm-only", action="store_true",
                    help="only the n = 2^20 MSM at --c/--encoding (for profiling): no oracle leg, "
                         "no n = 1024 run, no PADD, batched or served workloads")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 64-job batched workload (no oracle leg), followed by one "
                         "batch run isolated by idle gaps, for kernel traces")
    ap.add_argument("--microbench", action="store_true",
                    help="only measure the VALU issue rates and HBM copy bandwidth")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X and has no "
              "multi-GPU path (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.microbench:
        print(json.dumps(microbench()))
        return
    if args.msm_only or args.batch_only:
        args.no_checks = args.no_padd_kernel = args.no_batch = args.no_serve = True

    wl = Workloads(args)
    cpu = None
    if not args.no_checks:
        print("[bench] oracle leg (CPU baseline and expected values) ...", file=sys.stderr,
              flush=True)
        t0 = time.perf_counter()
        cpu = cpu_leg(wl, skip_baseline=args.no_cpu_baseline)
        print("[bench] oracle leg done in %.1f s" % (time.perf_counter() - t0), file=sys.stderr,
              flush=True)
    expected = cpu["expected"] if cpu else None

    import torch

    from paper_2502_11660_amd import api

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    n = N_POINTS
    k_dev = api.to_device(wl.kw, dev)
    s_dev = api.to_device(wl.sw, dev)

    def check(res_words, want):
        return None if expected is None else api.decode_result(res_words) == (want, 0)

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
    if args.batch_only:
        b = batched_leg(torch, api, wl, {"signed": xyu, "unsigned": xyu, "glv": xyu_endo}, s_dev,
                        isolated_run=True)
        b.pop("_results", None)
        print(json.dumps({"batched": b}, default=lambda o: o.item() if hasattr(o, "item")
                         else str(o)))
        return
    h2d = host_to_device_leg(torch, xyu, xyu_endo, s_dev)

    # workload 1: n = 1024, c = 8, the paper's unsigned slices
    config1 = None
    if not args.msm_only:
        res1 = api.words(api.MSM_RESULT_WORDS, dev)
        f1 = lambda: api.msm_run(xyu[:1024 * 36], api.to_device(wl.s1, dev), 1024, 8,
                                 ENCODINGS["unsigned"], result=res1)
        f1()
        config1 = {"n": 1024, "c": 8, "digits": "unsigned", "ms": timed(f1, 5, torch),
                   "result_ok": check(api.to_host(res1), expected["c1"] if expected else None)}

    # workload 3: the width sweep (every result checked)
    sweep = sweep_leg(torch, api, wl, pts_for, s_dev, args)
    best_enc, best_c = min(sweep, key=lambda k: sweep[k][0])
    sweep_out = {}
    for (enc, c), (ms, words) in sweep.items():
        ent = nonzero_digit_entries(wl.sw, c, enc)
        pc = padd_count_executed(ent, c, enc)
        sweep_out["%s_c%d" % (enc, c)] = {
            "ms": ms, "padd_per_s": pc / (ms * 1e-3), "padds": pc,
            "windows": num_windows(c, enc),
            "requested_c": [r for r in SWEEP[enc] if window_bits(r, enc) == c] if not args.c
            else [args.c],
            "ok": check(words, expected["c3"] if expected else None)}

    # the headline: timed steps at the best (encoding, width)
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
    accum_ms = tot / max(cnt, 1)
    result_ok = check(api.to_host(res), expected["c3"] if expected else None)
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
    del ws

    entries = nonzero_digit_entries(wl.sw, best_c, best_enc)
    padds = padd_count_executed(entries, best_c, best_enc)
    value = padds / (ms_per_step * 1e-3)
    accum_work = entries * MULS_MIXED * MAD_PER_MUL
    achieved = accum_work / (accum_ms * 1e-3)
    slots = (2 if best_enc == "glv" else 1) * n * num_windows(best_c, best_enc)

    padd_k = chain_stream = None
    if not args.no_padd_kernel:
        padd_k = padd_kernel_leg(torch, api, wl, xyu, 5)
        chain_stream = chain_and_stream_leg(torch, api, xyu, padd_k.pop("_a_pool"))
        from paper_2502_11660_amd import inputs
        chain_stream["field_cores"] = field_core_leg(torch, api, inputs)

    pools = {"signed": xyu, "unsigned": xyu, "glv": xyu_endo}
    batched = served = None
    if not args.no_batch:
        batched = batched_leg(torch, api, wl, pools, s_dev)
    if not args.no_serve:
        served = served_leg(torch, api, wl, pools, args)

    # ---- comparisons against the oracle's expected values ----
    checks = {}
    if expected is not None:
        checks["config1_ok"] = config1["result_ok"]
        checks["sweep_ok"] = {k: v["ok"] for k, v in sweep_out.items()}
        checks["sweep_all_ok"] = all(v["ok"] for v in sweep_out.values())
        checks["headline_ok"] = result_ok
        if padd_k is not None:
            smps = {form: padd_k[form].pop("_sample") for form in ("mixed", "complete")}
            oks = cpu_leg_compare(expected, smps)
            for form in ("mixed", "complete"):
                padd_k[form]["sample_checked"] = int(smps[form].shape[1])
                padd_k[form]["sample_ok"] = bool(oks[form])
            checks["padd_sample_ok"] = bool(padd_k["mixed"]["sample_ok"]
                                            and padd_k["complete"]["sample_ok"])
        if batched is not None:
            r = batched.pop("_results")
            ok_b = [api.decode_result(w) == (want, 0) for w, want in zip(r["batched"], expected["c4"])]
            batched["closed_form_checked_jobs"] = len(ok_b)
            batched["closed_form_ok"] = all(ok_b)
            batched["results_equal_plain_vs_batched"] = all(
                np.array_equal(a, b) for a, b in zip(r["batched"], r["plain_tuned"]))
            checks["batched_ok"] = all(ok_b)
        if served is not None:
            w = served.pop("_words")
            ok5, n5 = True, 0
            for leg, arr in w.items():
                for i in wl.check5:
                    if i < arr.shape[0]:
                        ok5 &= api.decode_result(arr[i]) == (expected["c5"][i], 0)
                        n5 += 1
            served["closed_form_checked"] = n5
            served["closed_form_checked_requests"] = len(wl.check5)
            served["closed_form_ok"] = bool(ok5)
            served["results_equal_served_vs_plain"] = bool(
                np.array_equal(w["served_200"], w["plain_200"]))
            checks["served_ok"] = bool(ok5)
    else:
        if padd_k is not None:
            for form in ("mixed", "complete"):
                padd_k[form].pop("_sample", None)
        if batched is not None:
            batched.pop("_results", None)
        if served is not None:
            served.pop("_words", None)

    cpu_baseline = None
    if cpu is not None and "baseline" in cpu:
        cpu_baseline = dict(cpu["baseline"])
        cpu_baseline["msm_ms_extrapolated"] = cpu_baseline["msm_n2p20_s_extrapolated"] * 1e3
        ps = cpu["pair_sample_oracle"]
        # the workload-2 sample's additions on one core (the oracle's affine
        # additions computing the expected sums of the 4096 sampled pairs)
        cpu_baseline["pair_sample_adds_per_s_one_core"] = ps["adds"] / ps["adds_s_one_core"]

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
                   "windows": num_windows(best_c, best_enc), "seed": wl.seed3,
                   "padds_per_msm": padds,
                   "padds_per_msm_unsigned_formula": padd_count_formula(n, best_c)},
        "msm_ms": ms_per_step,
        "result_matches_closed_form": result_ok,
        "prepare_ms": prepare_ms,
        "prepare_endo_ms": prepare_endo_ms,
        "prepare_plus_msm_ms": ms_per_step + (prepare_endo_ms if best_enc == "glv" else prepare_ms),
        "host_to_device": h2d,
        "config1": config1,
        "sweep": sweep_out,
        "phase_ms": phases,
        "bucket_scatter": bucket_scatter_figure(phases, slots, n,
                                                (2 if best_enc == "glv" else 1) * n),
        "roofline": {
            "kernel": "k_accum (bucket accumulation, mixed PADD)",
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_LANE_OPS / 1e12,
            "unit": "T word-products/s (32x32-bit products of the 12-word Montgomery form)",
            "frac": achieved / PEAK_LANE_OPS,
            "traffic": accum_traffic(entries),
            "work_per_launch": {"mixed_padds": entries, "word_products_per_padd": MULS_MIXED * MAD_PER_MUL},
            "launch_ms": accum_ms,
        },
        "padd_kernel": padd_k,
        "padd_workloads": chain_stream,
        "batched": batched,
        "served": served,
        "checks": checks,
        "cpu_baseline": cpu_baseline,
    }
    print(json.dumps(out, default=lambda o: o.item() if hasattr(o, "item") else str(o)))


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
        out[name] = {"ops_per_s": rate, "frac_of_peak": rate / PEAK_LANE_OPS,
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
    out["peak_lane_ops_per_s"] = PEAK_LANE_OPS
    return out


def accum_traffic(entries):
    """HBM bytes per accumulation launch from the committed rocprofv3 counter
    summary, if it was taken on the current accumulation kernel sources: the
    profiled bytes per digit entry times this launch's entries (the profile
    may be of another window width), or the profiled bytes per launch."""
    from paper_2502_11660_amd import profsum
    path = os.path.join(ROOT, "profiles", "k_accum_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != profsum.sources_sha256(rec.get("sources", [])):
        return None
    if rec.get("bytes_per_entry"):
        return rec["bytes_per_entry"] * entries
    return rec.get("bytes_per_launch")


if __name__ == "__main__":
    main()
