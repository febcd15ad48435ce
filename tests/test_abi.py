"""Host-side checks of the C ABI: the library loads, exports every function
declared in include/msm.h, validates arguments, and its built-in constants
equal the oracle's independently derived values.  No GPU work is launched."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import field, te
from paper_2502_11660_amd import _lib
from tests.helpers import words_int

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(msm_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("library not built: " + _lib.LIB_PATH)
    return _lib.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, "binding does not declare " + n


def test_constants_match_oracle(lib):
    buf = (ctypes.c_uint32 * 96)()
    assert lib.msm_constants(ctypes.cast(buf, ctypes.c_void_p), 96) == 0
    w = np.frombuffer(bytes(buf), dtype=np.uint32)
    g = lambda i: words_int(w[12 * i:12 * i + 12])
    P = field.P
    assert g(0) == P
    assert g(1) == field.R_MONT % P
    assert g(2) == field.R2_MONT
    assert field.from_mont(g(3)) == te.K_TE
    assert field.from_mont(g(4)) == te.ALPHA
    assert field.from_mont(g(5)) == te.BETA
    assert field.from_mont(g(6)) == field.G_X
    assert field.from_mont(g(7)) == field.G_Y
    assert lib.msm_constants(None, 96) == _lib.MSM_EINVAL
    assert lib.msm_constants(ctypes.cast(buf, ctypes.c_void_p), 10) == _lib.MSM_EINVAL


def test_argument_validation_without_gpu(lib):
    # invalid arguments are rejected on the host before anything is enqueued
    p = ctypes.c_void_p(16)
    assert lib.msm_padd_batch(None, p, p, 4, 0, None) == _lib.MSM_EINVAL
    assert lib.msm_padd_batch(p, p, p, 0, 0, None) == _lib.MSM_EINVAL
    assert lib.msm_padd_batch(p, p, p, 4, 7, None) == _lib.MSM_EINVAL
    assert lib.msm_fe_mul_batch(p, None, p, 4, 1, None) == _lib.MSM_EINVAL
    assert lib.msm_points_prepare(p, None, p, 0, p, None) == _lib.MSM_EINVAL
    assert lib.msm_gen_points(p, 0, p, p, None) == _lib.MSM_EINVAL
    S, U = _lib.MSM_DIGITS_SIGNED, _lib.MSM_DIGITS_UNSIGNED
    assert lib.msm_run(p, p, 0, 8, S, p, p, 1 << 30, None) == _lib.MSM_EINVAL
    assert lib.msm_run(p, p, 16, 21, S, p, p, 1 << 30, None) == _lib.MSM_EINVAL
    assert lib.msm_run(p, p, 16, 1, S, p, p, 1 << 30, None) == _lib.MSM_EINVAL  # signed: c >= 2
    assert lib.msm_run(p, p, 16, 8, 7, p, p, 1 << 30, None) == _lib.MSM_EINVAL
    assert lib.msm_run(p, p, 16, 8, S, p, p, 100, None) == _lib.MSM_ENOSPC
    assert lib.msm_run_noalloc(None, p, 16, 8, S, p, None) == _lib.MSM_EINVAL
    assert lib.msm_run_noalloc(p, p, 0, 8, S, p, None) == _lib.MSM_EINVAL
    assert lib.msm_run_noalloc(p, p, 16, 21, S, p, None) == _lib.MSM_EINVAL
    # more than the library's scratch: refused before any device call
    assert lib.msm_run_noalloc(p, p, 1 << 20, 16, S, p, None) == _lib.MSM_ENOSPC
    assert lib.msm_bucket_accumulate(p, p, 16, 8, U, None, p, 1 << 30, None) == _lib.MSM_EINVAL
    assert lib.msm_bucket_accumulate(p, p, 1 << 26, 8, U, p, p, 1 << 40, None) == _lib.MSM_EINVAL
    assert lib.msm_workspace_bytes(0, 8, S) == 0
    assert lib.msm_workspace_bytes(1024, 21, S) == 0
    assert lib.msm_workspace_bytes(1024, 1, S) == 0
    assert lib.msm_workspace_bytes(1024, 1, U) > 0
    assert lib.msm_workspace_bytes(1024, 8, S) > 0
    assert lib.msm_padd_chain(p, 0, 0, p, None) == _lib.MSM_EINVAL
    assert lib.msm_padd_chain(p, 4, 5, p, None) == _lib.MSM_EINVAL
    assert lib.msm_padd_chain(None, 4, 0, p, None) == _lib.MSM_EINVAL
    assert lib.msm_accumulate_stream(p, 0, 4, p, None) == _lib.MSM_EINVAL
    assert lib.msm_accumulate_stream(p, 4, 0, p, None) == _lib.MSM_EINVAL
    # timing modes: host state only
    assert lib.msm_profile_enable(3) == _lib.MSM_EINVAL
    assert lib.msm_profile_enable(-1) == _lib.MSM_EINVAL
    for mode in (_lib.MSM_PROFILE_ACCUM_KERNEL, _lib.MSM_PROFILE_PHASES, _lib.MSM_PROFILE_OFF):
        assert lib.msm_profile_enable(mode) == _lib.MSM_OK
    # batches: validated on the host
    Job = _lib.MsmJob
    jobs = (Job * 2)(Job(16, 16, 16, 100, 8), Job(16, 16, 16, 0, 8))
    assert lib.msm_batch_workspace_bytes(jobs, 2, S) == 0          # n = 0
    assert lib.msm_batch_workspace_bytes(jobs, 1, S) > 0
    assert lib.msm_batch_workspace_bytes(jobs, 0, S) == 0
    neg = (Job * 1)(Job(16, 16, 16, 100, 8, -1, 0, 0))
    assert lib.msm_batch_workspace_bytes(neg, 1, S) == 0          # negative schedule value
    sch = (Job * 2)(Job(16, 16, 16, 100, 8), Job(16, 16, 16, 100, 8, 7, 16, 4096))
    assert lib.msm_batch_workspace_bytes(sch, 2, S) > lib.msm_batch_workspace_bytes(sch, 1, S)
    h = ctypes.c_void_p()
    assert lib.msm_batch_create(jobs, 2, S, p, 1 << 40, 0, ctypes.byref(h)) == _lib.MSM_EINVAL
    assert lib.msm_batch_create(jobs, 1, S, p, 100, 0, ctypes.byref(h)) == _lib.MSM_ENOSPC
    assert h.value is None
    assert lib.msm_batch_run(None, None) == _lib.MSM_EINVAL
    assert lib.msm_batch_destroy(None) == _lib.MSM_OK
    # server: argument checks come before any device call
    srv = ctypes.c_void_p()
    assert lib.msm_server_create(0, 4, S, ctypes.byref(srv)) == _lib.MSM_EINVAL
    assert lib.msm_server_create(1 << 30, 0, S, ctypes.byref(srv)) == _lib.MSM_EINVAL
    assert lib.msm_server_create(1 << 30, 17, S, ctypes.byref(srv)) == _lib.MSM_EINVAL
    assert lib.msm_server_create(1 << 30, 4, 9, ctypes.byref(srv)) == _lib.MSM_EINVAL
    assert lib.msm_server_create(1 << 30, 4, S, None) == _lib.MSM_EINVAL
    t = ctypes.c_uint64()
    assert lib.msm_server_submit(None, jobs, None, ctypes.byref(t)) == _lib.MSM_EINVAL
    k = ctypes.c_size_t()
    assert lib.msm_server_progress(None, None, 0, ctypes.byref(k)) == _lib.MSM_EINVAL
    assert lib.msm_server_drain(None) == _lib.MSM_EINVAL
    assert lib.msm_server_stats(None, None, None, None) == _lib.MSM_EINVAL
    assert lib.msm_server_destroy(None) == _lib.MSM_OK
    assert lib.msm_status_string(_lib.MSM_ENOSPC).startswith(b"MSM_ENOSPC")


def test_window_helpers(lib):
    S, U = _lib.MSM_DIGITS_SIGNED, _lib.MSM_DIGITS_UNSIGNED
    for c in range(1, 21):
        assert lib.msm_num_windows(c, U) == -(-253 // c)
        assert lib.msm_num_windows(c, S) == (-(-254 // c) if c >= 2 else 0)
    assert lib.msm_num_windows(0, U) == 0
    assert lib.msm_num_windows(8, 5) == 0
    for n in (1, 1024, 1 << 16, 1 << 20):
        c = lib.msm_default_window(n)
        assert 2 <= c <= 20
        assert lib.msm_workspace_bytes(n, 0, S) == lib.msm_workspace_bytes(n, c, S)
    # signed digits halve the bucket storage
    assert lib.msm_workspace_bytes(1 << 16, 16, S) < lib.msm_workspace_bytes(1 << 16, 16, U)
    # window widths are lowered to cover the digit bits with the same windows
    G = _lib.MSM_DIGITS_GLV
    for enc, bits in ((U, 253), (S, 254), (G, 128)):
        for c in range(2, 21):
            W = lib.msm_num_windows(c, enc)
            cb = lib.msm_window_bits(c, enc)
            assert cb <= c and W * cb >= bits and W * (cb - 1) < bits, (enc, c)
    assert lib.msm_window_bits(17, G) == 16 and lib.msm_window_bits(18, S) == 17
    assert lib.msm_workspace_bytes(1 << 12, 17, G) == lib.msm_workspace_bytes(1 << 12, 16, G)
    assert lib.msm_window_bits(1, S) == 0 and lib.msm_window_bits(21, U) == 0
    # a batch of one job needs what a single MSM needs
    Job = _lib.MsmJob
    one = (Job * 1)(Job(16, 16, 16, 5000, 11))
    assert lib.msm_batch_workspace_bytes(one, 1, S) == lib.msm_workspace_bytes(5000, 11, S)


def test_size_limits_plan_at_every_width(lib):
    """Single MSMs plan up to the interface's n = 2^26 - 1 points at every
    width and encoding whose digit slots (points x windows, twice the points
    with the split) stay below 2^31 (entry positions are 32-bit words): the
    sort groups tiles and splits the bucket bits so that its count matrix
    fits the two-level scan.  n = 2^26 is refused.  The split digits' c = 0
    choice is c' = 16 at n = 2^20 and c' = 19 from ~2^22 on; the signed
    model's reaches c = 20 at 2^24."""
    S, U, G = _lib.MSM_DIGITS_SIGNED, _lib.MSM_DIGITS_UNSIGNED, _lib.MSM_DIGITS_GLV
    top = (1 << 26) - 1
    planned = 0
    for enc in (S, U, G):
        for c in range(2, 21):
            slots = (2 if enc == G else 1) * top * lib.msm_num_windows(c, enc)
            b = lib.msm_workspace_bytes(top, c, enc)
            if slots < (1 << 31):
                assert 0 < b < (48 << 30), (enc, c)  # well inside one GPU's memory
                planned += 1
            else:
                assert b == 0, (enc, c)
            assert lib.msm_workspace_bytes(1 << 26, c, enc) == 0, (enc, c)
    assert planned >= 3 * 12  # c = 8 .. 20 at least, in every encoding
    assert lib.msm_default_window(1 << 24) == 20
    assert lib.msm_workspace_bytes(1 << 20, 0, G) == lib.msm_workspace_bytes(1 << 20, 16, G)
    assert lib.msm_workspace_bytes(1 << 24, 0, G) == lib.msm_workspace_bytes(1 << 24, 19, G)
    assert lib.msm_workspace_bytes(1 << 24, 0, G) != lib.msm_workspace_bytes(1 << 24, 16, G)
