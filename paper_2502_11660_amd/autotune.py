"""Window-width autotuner for batched and served MSMs.

For a size class (n-bucket u = floor(log2 n)) it times MSMs of size 2^u at
candidate window widths around the static heuristic (msm_default_window) and
keeps the fastest.  The timing context matters: in a batch many jobs share
the chip, so narrower windows (less aggregation, more accumulation) win; a
served request mostly runs alone, where latency favours the solo optimum.
Context "batch" times batches of up to 64 jobs (about 2^20 points in all),
context "solo" one job at a time.  Results are cached per device (name and
architecture), context and n-bucket in a JSON file, by default
~/.cache/paper_2502_11660_amd/autotune.json (MSM_AUTOTUNE_CACHE overrides it).
Timing runs the library's own kernels on the current stream; nothing here
computes any part of an MSM.
"""

import json
import math
import os

import torch

from . import api


def cache_path():
    return os.environ.get("MSM_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2502_11660_amd", "autotune.json")


def device_key(device=None):
    p = torch.cuda.get_device_properties(device or torch.cuda.current_device())
    return "%s|%s" % (p.name, getattr(p, "gcnArchName", ""))


def n_bucket(n):
    return max(0, int(math.floor(math.log2(max(1, int(n))))))


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

    def tune(self, u, xyu_pool, scalar_pool, span=(-3, 2), reps=3, batch_points=1 << 20):
        """Time jobs of size 2^u over pool slices -- batches of about
        batch_points points (at most 64 jobs) in context "batch", single jobs
        in context "solo" -- and store and return the best width.  With the
        endomorphism encoding the pool holds two records per point."""
        n = 1 << u
        rec = 2 if self.encoding == api.MSM_DIGITS_GLV else 1  # records per point
        npool = xyu_pool.numel() // (api.XYU_WORDS * rec)
        if n > npool or n > scalar_pool.numel() // api.SCALAR_WORDS:
            raise ValueError("pool smaller than 2^%d" % u)
        jobs_n = max(1, min(64, batch_points // n)) if self.context == "batch" else 1
        c0 = api.default_window(n)
        cands = [c for c in range(c0 + span[0], c0 + span[1] + 1) if 2 <= c <= 20]
        times = {}
        results = [api.words(api.MSM_RESULT_WORDS) for _ in range(jobs_n)]
        for c in cands:
            jobs = []
            for j in range(jobs_n):
                off = (j * 7919) % (npool - n + 1)
                jobs.append((xyu_pool[rec * off * 36:rec * (off + n) * 36],
                             scalar_pool[off * 8:(off + n) * 8], results[j], n, c))
            b = api.Batch(jobs, self.encoding, use_graph=True)
            b.run()
            torch.cuda.synchronize()
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            for _ in range(reps):
                b.run()
            e.record()
            torch.cuda.synchronize()
            times[c] = s.elapsed_time(e) / reps / jobs_n
            b.destroy()
            del b
        best = min(times, key=times.get)
        self.table[self._key(u)] = {"c": best, "ms_per_job": times[best],
                                    "candidates_ms_per_job": {str(k): v for k, v in times.items()},
                                    "jobs_per_batch": jobs_n}
        return best

    def save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(self.path, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
