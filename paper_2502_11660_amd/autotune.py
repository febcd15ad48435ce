"""Autotuner of the window width and the schedule for batched and served MSMs.

For a size class (n-bucket u = floor(log2 n)) it times MSMs of size 2^u:
first the window width c at candidates around the static heuristic
(msm_default_window), then, in the batch context and at the chosen width,
the schedule of the job's pipeline one parameter at a time: the
accumulation chunk (digit entries per lane: the default that fills one
resident round of lanes, half of it, twice it) and the aggregation tree's
unit thresholds (the output counts below which a level runs on the four-lane
unit, and up to which on the wide two-wave unit).  A candidate replaces the
current choice only when it is faster by more than 2%, so the defaults stay
unless a change pays.

The timing context matters: in a batch many jobs share the chip, so narrower
windows (less aggregation, more accumulation) win; a served request mostly
runs alone, where latency favours the solo optimum.  Context "batch" times
batches of up to 64 jobs (about 2^20 points in all), context "solo" one job
at a time (width only: the plain path takes no schedule).  Results are cached
per device (name and architecture), encoding, context and n-bucket in a JSON
file, by default ~/.cache/paper_2502_11660_amd/autotune.json
(MSM_AUTOTUNE_CACHE overrides it).  Timing runs the library's own kernels on
the current stream; nothing here computes any part of an MSM.
"""

import json
import math
import os

import torch

from . import api

# schedule candidates (0 = the library's default)
CHUNK_SCALES = (0.5, 2.0)                 # times the default chunk of the class
TREE_QUAD = (16384, 262144)               # default 65536
TREE_WIDE = (256, 4096)                   # default 1024
MIN_GAIN = 0.02


def cache_path():
    return os.environ.get("MSM_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2502_11660_amd", "autotune.json")


def device_key(device=None):
    p = torch.cuda.get_device_properties(device or torch.cuda.current_device())
    return "%s|%s" % (p.name, getattr(p, "gcnArchName", ""))


def n_bucket(n):
    return max(0, int(math.floor(math.log2(max(1, int(n))))))


def default_chunk(total_entries, cus=256):
    """The average length of the library's default accumulation chunks for a
    class with this many digit entries: one chunk per lane of a resident
    round (256 CUs x 4 SIMDs x 3 waves x 64), at least 16 entries; the
    library splits that into lengths K and K + 4 (multiples of 4)."""
    lanes = cus * 4 * 3 * 64
    return max(16, -(-int(total_entries) // lanes))


class Autotuner:
    def __init__(self, path=None, encoding=api.MSM_DIGITS_SIGNED, context="batch"):
        if context not in ("batch", "solo"):
            raise ValueError("context must be 'batch' or 'solo'")
        self.path = path or cache_path()
        self.encoding = encoding
        self.context = context
        self.table = {}
        try:
            with open(self.path) as f:
                self.table = json.load(f)
        except (OSError, ValueError):
            self.table = {}

    def _key(self, u):
        return "%s|enc%d|%s|u%d" % (device_key(), self.encoding, self.context, u)

    def tuned(self, u):
        return self._key(u) in self.table

    def choose(self, n):
        """Tuned width for n's size class, else the static heuristic."""
        ent = self.table.get(self._key(n_bucket(n)))
        return int(ent["c"]) if ent else api.default_window(int(n))

    def schedule(self, n):
        """Tuned schedule for n's size class ({} = defaults)."""
        ent = self.table.get(self._key(n_bucket(n)))
        return dict(ent.get("schedule", {})) if ent else {}

    def _time(self, jobs_n, n, c, sched, xyu_pool, scalar_pool, npool, rec, reps, results):
        jobs = []
        for j in range(jobs_n):
            off = (j * 7919) % (npool - n + 1)
            jobs.append((xyu_pool[rec * off * 36:rec * (off + n) * 36],
                         scalar_pool[off * 8:(off + n) * 8], results[j], n, c, sched))
        b = api.Batch(jobs, self.encoding, use_graph=True)
        b.run()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            b.run()
        e.record()
        torch.cuda.synchronize()
        b.destroy()
        return s.elapsed_time(e) / reps / jobs_n

    def tune(self, u, xyu_pool, scalar_pool, span=(-3, 2), reps=3, batch_points=1 << 20):
        """Time jobs of size 2^u over pool slices -- batches of about
        batch_points points (at most 64 jobs) in context "batch", single jobs
        in context "solo" -- and store and return the best width (and, in
        context "batch", schedule).  With the endomorphism encoding the pool
        holds two records per point."""
        n = 1 << u
        rec = 2 if self.encoding == api.MSM_DIGITS_GLV else 1  # records per point
        npool = xyu_pool.numel() // (api.XYU_WORDS * rec)
        if n > npool or n > scalar_pool.numel() // api.SCALAR_WORDS:
            raise ValueError("pool smaller than 2^%d" % u)
        jobs_n = max(1, min(64, batch_points // n)) if self.context == "batch" else 1
        c0 = api.default_window(n)
        cands = [c for c in range(c0 + span[0], c0 + span[1] + 1) if 2 <= c <= 20]
        results = [api.words(api.MSM_RESULT_WORDS) for _ in range(jobs_n)]
        t = lambda c, sched: self._time(jobs_n, n, c, sched, xyu_pool, scalar_pool, npool, rec,
                                        reps, results)
        times = {c: t(c, {}) for c in cands}
        best = min(times, key=times.get)
        ent = {"c": best, "ms_per_job": times[best],
               "candidates_ms_per_job": {str(k): v for k, v in times.items()},
               "jobs_per_batch": jobs_n, "schedule": {}, "schedule_trials_ms_per_job": {}}
        if self.context == "batch":
            sched, cur = {}, times[best]
            W = api.num_windows(best, self.encoding)
            k0 = default_chunk(jobs_n * rec * n * W)
            trials = [("chunk", max(4, int(k0 * f))) for f in CHUNK_SCALES]
            trials += [("tree_quad", v) for v in TREE_QUAD] + [("tree_wide", v) for v in TREE_WIDE]
            for name, v in trials:
                cand = dict(sched)
                cand[name] = v
                ms = t(best, cand)
                ent["schedule_trials_ms_per_job"]["%s=%d" % (name, v)] = ms
                if ms < cur * (1.0 - MIN_GAIN):
                    sched, cur = cand, ms
            ent["schedule"] = sched
            ent["ms_per_job"] = cur
        self.table[self._key(u)] = ent
        return best

    def save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(self.path, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
