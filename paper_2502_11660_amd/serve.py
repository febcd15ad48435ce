"""Trace replay for served MSMs: requests arrive at given times and are
either submitted to an MSM server as they arrive (continuous admission,
overlapping on the device) or run by the plain path one at a time, first in
first out.  Latency is completion time minus arrival time on the host clock.
"""

import sys
import time

import numpy as np
import torch

from . import api


def replay_served(server, arrivals, jobs, progress_every=None):
    """arrivals[i] (s, ascending) and jobs[i] = (xyu, scalars, result, n, c).
    Returns per-request latency (s) and the wall time of the replay."""
    nreq = len(arrivals)
    lat = np.full(nreq, np.nan)
    ticket_of = {}
    t0 = time.perf_counter()
    i = 0
    done = 0
    last_report = 0.0
    while done < nreq:
        now = time.perf_counter() - t0
        while i < nreq and arrivals[i] <= now:
            ticket_of[server.submit(*jobs[i])] = i
            i += 1
        fin = server.progress()
        if fin:
            tf = time.perf_counter() - t0
            for t in fin:
                k = ticket_of.pop(t)
                lat[k] = tf - arrivals[k]
            done += len(fin)
        if progress_every and now - last_report >= progress_every:
            last_report = now
            fl, q, b = server.stats()
            print("[serve] t=%.1fs submitted=%d done=%d in_flight=%d queued=%d arena=%.2f GB"
                  % (now, i, done, fl, q, b / 1e9), file=sys.stderr, flush=True)
    return lat, time.perf_counter() - t0


def replay_plain(arrivals, jobs, encoding=api.MSM_DIGITS_SIGNED, workspaces=None,
                 progress_every=None):
    """The plain path: msm_run of one request at a time, in arrival order, each
    started when it has arrived and the previous one has finished."""
    nreq = len(arrivals)
    lat = np.full(nreq, np.nan)
    t0 = time.perf_counter()
    last_report = 0.0
    for i in range(nreq):
        while time.perf_counter() - t0 < arrivals[i]:
            pass
        xyu, sc, res, n, c = jobs[i][:5]
        ws = workspaces(n, c) if workspaces else None
        api.msm_run(xyu, sc, n, c, encoding, result=res, ws=ws)
        torch.cuda.current_stream().synchronize()
        lat[i] = time.perf_counter() - t0 - arrivals[i]
        now = time.perf_counter() - t0
        if progress_every and now - last_report >= progress_every:
            last_report = now
            print("[plain] t=%.1fs done=%d" % (now, i + 1), file=sys.stderr, flush=True)
    return lat, time.perf_counter() - t0


def summarize(lat_s, wall_s, measured):
    """p50/p99 latency (ms) and MSMs/s over the measured requests."""
    lm = lat_s[measured] * 1e3
    return {
        "requests": int(measured.sum()),
        "p50_ms": float(np.percentile(lm, 50)),
        "p99_ms": float(np.percentile(lm, 99)),
        "mean_ms": float(lm.mean()),
        "msms_per_s": float(len(lat_s) / wall_s),
    }
