"""Python binding of the C ABI (include/msm.h), one function per entry point.

Argument marshalling only: torch provides device memory (int32 tensors used as
raw 32-bit words) and the current HIP stream; every step of the computation
runs in the library's kernels.  Calls are asynchronous on the current stream,
like the C functions they wrap.
"""

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (MSM_DIGITS_GLV, MSM_DIGITS_SIGNED, MSM_DIGITS_UNSIGNED,  # noqa: F401
                   MSM_FLAG_EXCEPT,
                   MSM_FLAG_OFFCURVE, MSM_FLAG_RANGE, MSM_FORM_XYTZ, MSM_FORM_XYU,
                   MSM_MUL_BARRETT, MSM_MUL_F28, MSM_MUL_KARATSUBA, MSM_MUL_MONT, MSM_MUL_WIDE,
                   MSM_PROFILE_ACCUM_KERNEL, MSM_PROFILE_OFF, MSM_PROFILE_PHASES,
                   MSM_RESULT_WORDS,
                   MSM_UNIT_LANE, MSM_UNIT_QUAD, MSM_UNIT_WIDE, MSMError, MsmJob)

WORDS = 12
XYU_WORDS = 36
XYTZ_WORDS = 48
SCALAR_WORDS = 8


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA/HIP tensor" % name)
    if t.dtype != torch.int32 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous int32 tensor (raw 32-bit words)" % name)
    return t


def words(n, device="cuda"):
    return torch.empty(int(n), dtype=torch.int32, device=device)


def to_device(arr_u32, device="cuda"):
    """numpy uint32 array -> contiguous int32 device tensor with the same bits."""
    a = np.ascontiguousarray(arr_u32, dtype=np.uint32).reshape(-1)
    return torch.from_numpy(a.view(np.int32).copy()).to(device)


def to_host(t):
    """device tensor of 32-bit words -> numpy uint32 array (synchronises)."""
    return t.detach().cpu().numpy().view(np.uint32)


def padd_batch(a_xytz, b, count, b_form, out=None):
    """out_i = a_i + b_i (SoA layouts, see msm_padd_batch)."""
    _dev(a_xytz, "a_xytz")
    _dev(b, "b")
    nb = 4 if b_form == MSM_FORM_XYTZ else 3
    if a_xytz.numel() != 4 * WORDS * count or b.numel() != nb * WORDS * count:
        raise ValueError("operand sizes do not match count")
    if out is None:
        out = words(4 * WORDS * count, a_xytz.device)
    _dev(out, "out")
    _lib.check("msm_padd_batch", _lib.lib().msm_padd_batch(
        _ptr(a_xytz), _ptr(b), _ptr(out), count, b_form, _stream()))
    return out


def padd_chain(pts_xytz, count, unit=MSM_UNIT_QUAD, out=None):
    """Sum of count AoS XYTZ records added one after another (latency chain)."""
    _dev(pts_xytz, "pts_xytz")
    if pts_xytz.numel() < XYTZ_WORDS * count:
        raise ValueError("pts_xytz smaller than count records")
    if out is None:
        out = words(XYTZ_WORDS, pts_xytz.device)
    _lib.check("msm_padd_chain", _lib.lib().msm_padd_chain(
        _ptr(pts_xytz), count, unit, _ptr(out), _stream()))
    return out


def accumulate_stream(xyu, n, accumulators, out=None):
    """accumulators independent mixed-PADD running sums over strided points."""
    _dev(xyu, "xyu")
    if xyu.numel() < XYU_WORDS * n:
        raise ValueError("xyu smaller than n records")
    if out is None:
        out = words(XYTZ_WORDS * accumulators, xyu.device)
    _lib.check("msm_accumulate_stream", _lib.lib().msm_accumulate_stream(
        _ptr(xyu), n, accumulators, _ptr(out), _stream()))
    return out


def fe_mul_batch(a, b, count, canonical=True, out=None):
    _dev(a, "a")
    _dev(b, "b")
    if a.numel() != WORDS * count or b.numel() != WORDS * count:
        raise ValueError("operand sizes do not match count")
    if out is None:
        out = words(WORDS * count, a.device)
    _lib.check("msm_fe_mul_batch", _lib.lib().msm_fe_mul_batch(
        _ptr(a), _ptr(b), _ptr(out), count, 1 if canonical else 0, _stream()))
    return out


def fe_mul_chain(a, b, count, variant=MSM_MUL_MONT, rounds=1, out=None):
    """out_i = a_i * b_i^rounds with the chosen field-multiplication core."""
    _dev(a, "a")
    _dev(b, "b")
    if a.numel() != WORDS * count or b.numel() != WORDS * count:
        raise ValueError("operand sizes do not match count")
    if out is None:
        out = words(WORDS * count, a.device)
    _lib.check("msm_fe_mul_chain", _lib.lib().msm_fe_mul_chain(
        _ptr(a), _ptr(b), _ptr(out), count, variant, rounds, _stream()))
    return out


def points_prepare(xy_std, n, inf=None, out=None, status=None, endo=False):
    """Weierstrass affine (SoA) -> prepared Edwards XYU records (AoS); with
    endo, 2n records: the points, then their endomorphism images."""
    _dev(xy_std, "xy_std")
    if xy_std.numel() != 2 * WORDS * n:
        raise ValueError("xy_std size does not match n")
    if inf is not None:
        _dev(inf, "inf")
    if out is None:
        out = words(XYU_WORDS * n * (2 if endo else 1), xy_std.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=xy_std.device)
    fn = "msm_points_prepare_endo" if endo else "msm_points_prepare"
    _lib.check(fn, getattr(_lib.lib(), fn)(
        _ptr(xy_std), _ptr(inf), _ptr(out), n, _ptr(status), _stream()))
    return out, status


def gen_points(k, n, xy_out=None, inf_out=None):
    """P_i = k_i G as Weierstrass affine points (SoA) plus infinity flags."""
    _dev(k, "k")
    if k.numel() != SCALAR_WORDS * n:
        raise ValueError("k size does not match n")
    if xy_out is None:
        xy_out = words(2 * WORDS * n, k.device)
    if inf_out is None:
        inf_out = words(n, k.device)
    _lib.check("msm_gen_points", _lib.lib().msm_gen_points(
        _ptr(k), n, _ptr(xy_out), _ptr(inf_out), _stream()))
    return xy_out, inf_out


def num_windows(c, encoding=MSM_DIGITS_SIGNED):
    return _lib.lib().msm_num_windows(c, encoding)


def window_bits(c, encoding=MSM_DIGITS_SIGNED):
    return _lib.lib().msm_window_bits(c, encoding)


def buckets_per_window(c, encoding=MSM_DIGITS_SIGNED):
    cb = window_bits(c, encoding)
    return 1 << (cb if encoding == MSM_DIGITS_UNSIGNED else cb - 1)


def default_window(n):
    return _lib.lib().msm_default_window(n)


def workspace_bytes(n, c, encoding=MSM_DIGITS_SIGNED):
    return _lib.lib().msm_workspace_bytes(n, c, encoding)


def workspace(n, c, encoding=MSM_DIGITS_SIGNED, device="cuda"):
    nbytes = workspace_bytes(n, c, encoding)
    if nbytes == 0:
        raise ValueError("invalid (n, c, encoding) = (%d, %d, %d)" % (n, c, encoding))
    return torch.empty((nbytes + 3) // 4, dtype=torch.int32, device=device)


def bucket_accumulate(xyu, scalars, n, c, encoding=MSM_DIGITS_SIGNED, buckets=None, ws=None):
    _dev(xyu, "xyu")
    _dev(scalars, "scalars")
    if xyu.numel() != XYU_WORDS * _records(n, encoding) or scalars.numel() != SCALAR_WORDS * n:
        raise ValueError("input sizes do not match n")
    W = num_windows(c, encoding)
    if buckets is None:
        buckets = words(XYTZ_WORDS * W * buckets_per_window(c, encoding), xyu.device)
    if ws is None:
        ws = workspace(n, c, encoding, xyu.device)
    _lib.check("msm_bucket_accumulate", _lib.lib().msm_bucket_accumulate(
        _ptr(xyu), _ptr(scalars), n, c, encoding, _ptr(buckets), _ptr(ws), ws.numel() * 4,
        _stream()))
    return buckets, ws


def _records(n, encoding):
    return 2 * n if encoding == MSM_DIGITS_GLV else n


def msm_run(xyu, scalars, n, c=0, encoding=MSM_DIGITS_SIGNED, result=None, ws=None):
    _dev(xyu, "xyu")
    _dev(scalars, "scalars")
    if xyu.numel() != XYU_WORDS * _records(n, encoding) or scalars.numel() != SCALAR_WORDS * n:
        raise ValueError("input sizes do not match n")
    if result is None:
        result = words(MSM_RESULT_WORDS, xyu.device)
    if ws is None:
        ws = workspace(n, c, encoding, xyu.device)
    _lib.check("msm_run", _lib.lib().msm_run(
        _ptr(xyu), _ptr(scalars), n, c, encoding, _ptr(result), _ptr(ws), ws.numel() * 4,
        _stream()))
    return result


def msm_run_noalloc(xyu, scalars, n, c=0, encoding=MSM_DIGITS_SIGNED, result=None):
    """msm_run on the library's own device scratch (msm_run_noalloc): no
    workspace argument; the call allocates nothing (pass `result` to keep
    the caller side allocation-free too)."""
    _dev(xyu, "xyu")
    _dev(scalars, "scalars")
    if xyu.numel() != XYU_WORDS * _records(n, encoding) or scalars.numel() != SCALAR_WORDS * n:
        raise ValueError("input sizes do not match n")
    if result is None:
        result = words(MSM_RESULT_WORDS, xyu.device)
    _dev(result, "result")
    _lib.check("msm_run_noalloc", _lib.lib().msm_run_noalloc(
        _ptr(xyu), _ptr(scalars), n, c, encoding, _ptr(result), _stream()))
    return result


def _job_array(jobs, encoding=MSM_DIGITS_SIGNED):
    """jobs: (xyu, scalars, result, n, c) or (xyu, scalars, result, n, c,
    schedule) tuples; schedule is a dict with any of chunk, tree_quad,
    tree_wide (msm_job's schedule fields; missing or 0 = default)."""
    arr = (MsmJob * len(jobs))()
    for a, job in zip(arr, jobs):
        xyu, scalars, result, n, c = job[:5]
        sched = job[5] if len(job) > 5 and job[5] else {}
        for t, name in ((xyu, "xyu"), (scalars, "scalars"), (result, "result")):
            _dev(t, name)
        if xyu.numel() < XYU_WORDS * _records(n, encoding) or scalars.numel() < SCALAR_WORDS * n:
            raise ValueError("job inputs smaller than n")
        if result.numel() < MSM_RESULT_WORDS:
            raise ValueError("job result buffer too small")
        a.xyu, a.scalars, a.result = xyu.data_ptr(), scalars.data_ptr(), result.data_ptr()
        a.n, a.c = int(n), int(c)
        a.chunk = int(sched.get("chunk", 0))
        a.tree_quad = int(sched.get("tree_quad", 0))
        a.tree_wide = int(sched.get("tree_wide", 0))
    return arr


def batch_workspace_bytes(jobs, encoding=MSM_DIGITS_SIGNED):
    """jobs: list of (xyu, scalars, result, n, c) tuples (c = 0: default width)."""
    arr = _job_array(jobs, encoding)
    return _lib.lib().msm_batch_workspace_bytes(arr, len(jobs), encoding)


class Batch:
    """A planned batch of independent MSMs (msm_batch_create / run / destroy).

    The tensors named by the jobs must stay alive and in place while the batch
    exists; the batch holds references to them and to its workspace.
    """

    def __init__(self, jobs, encoding=MSM_DIGITS_SIGNED, use_graph=False):
        arr = _job_array(jobs, encoding)
        nbytes = _lib.lib().msm_batch_workspace_bytes(arr, len(jobs), encoding)
        if nbytes == 0:
            raise ValueError("invalid batch jobs")
        dev = jobs[0][0].device
        self.ws = torch.empty((nbytes + 3) // 4, dtype=torch.int32, device=dev)
        self._keep = [t for j in jobs for t in j[:3]]
        h = ctypes.c_void_p()
        _lib.check("msm_batch_create", _lib.lib().msm_batch_create(
            arr, len(jobs), encoding, _ptr(self.ws), self.ws.numel() * 4,
            1 if use_graph else 0, ctypes.byref(h)))
        self._h = h

    def run(self):
        if self._h is None:
            raise RuntimeError("batch destroyed")
        _lib.check("msm_batch_run", _lib.lib().msm_batch_run(self._h, _stream()))

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _lib.lib().msm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.destroy()


def constants():
    buf = (ctypes.c_uint32 * 96)()
    _lib.check("msm_constants", _lib.lib().msm_constants(ctypes.cast(buf, ctypes.c_void_p), 96))
    return np.frombuffer(bytes(buf), dtype=np.uint32).copy()


def decode_result(res_u32):
    """Host view of a result buffer: (x, y) ints or None for infinity, flags."""
    r = np.asarray(res_u32, dtype=np.uint32)
    flags = int(r[2 * WORDS + 1])
    if r[2 * WORDS]:
        return None, flags
    x = sum(int(w) << (32 * i) for i, w in enumerate(r[:WORDS]))
    y = sum(int(w) << (32 * i) for i, w in enumerate(r[WORDS:2 * WORDS]))
    return (x, y), flags


def profile_enable(mode=MSM_PROFILE_PHASES):
    """Timing mode (msm_profile_enable): MSM_PROFILE_OFF, MSM_PROFILE_PHASES
    (events around every phase) or MSM_PROFILE_ACCUM_KERNEL (events attached
    to the accumulation kernel's dispatch only); True / False mean phases /
    off."""
    if mode is True:
        mode = MSM_PROFILE_PHASES
    elif mode is False:
        mode = MSM_PROFILE_OFF
    _lib.check("msm_profile_enable", _lib.lib().msm_profile_enable(int(mode)))


def profile_read(phase):
    """(total_ms, launches) of one phase since the last read (synchronises)."""
    tot = ctypes.c_double(0.0)
    cnt = ctypes.c_int(0)
    _lib.check("msm_profile_read", _lib.lib().msm_profile_read(
        phase.encode(), ctypes.byref(tot), ctypes.byref(cnt)))
    return tot.value, cnt.value


def microbench(kind, param, buf):
    """Launch one microbenchmark kernel (see msm_microbench) on the current stream."""
    _dev(buf, "buf")
    _lib.check("msm_microbench", _lib.lib().msm_microbench(
        kind, param, _ptr(buf), buf.numel() * 4, _stream()))


class Server:
    """MSM request server (msm_server_*): HBM-budget admission, concurrent
    streams, retirement by completion events.  Tensors of a submitted job are
    referenced until its ticket is reported finished."""

    def __init__(self, budget_bytes, streams=4, encoding=MSM_DIGITS_SIGNED):
        h = ctypes.c_void_p()
        _lib.check("msm_server_create", _lib.lib().msm_server_create(
            int(budget_bytes), int(streams), int(encoding), ctypes.byref(h)))
        self._h = h
        self.encoding = encoding
        self._live = {}
        self._buf = (ctypes.c_uint64 * 1024)()

    def submit(self, xyu, scalars, result, n, c=0, schedule=None):
        """Queue one MSM; it runs after the work already enqueued on the
        current stream (the producer of its inputs).  schedule: as for a
        batch job (chunk, tree_quad, tree_wide)."""
        arr = _job_array([(xyu, scalars, result, n, c, schedule)], self.encoding)
        t = ctypes.c_uint64(0)
        _lib.check("msm_server_submit", _lib.lib().msm_server_submit(
            self._h, arr, _stream(), ctypes.byref(t)))
        self._live[t.value] = (xyu, scalars, result)
        return t.value

    def progress(self):
        """Tickets finished since the last call (their results are valid)."""
        out = []
        while True:
            k = ctypes.c_size_t(0)
            _lib.check("msm_server_progress", _lib.lib().msm_server_progress(
                self._h, self._buf, len(self._buf), ctypes.byref(k)))
            out.extend(self._buf[i] for i in range(k.value))
            if k.value < len(self._buf):
                break
        for t in out:
            self._live.pop(t, None)
        return out

    def drain(self):
        _lib.check("msm_server_drain", _lib.lib().msm_server_drain(self._h))

    def stats(self):
        a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _lib.check("msm_server_stats", _lib.lib().msm_server_stats(
            self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _lib.lib().msm_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        self.destroy()
