/*
 * msm.h -- C ABI of the gfx950 BLS12-377 G1 multi-scalar multiplication library.
 *
 * The library computes MSM = sum_i s_i P_i over G1 of BLS12-377 (Abstract,
 * Sec. II-C) by Pippenger's method: scalars are cut into c-bit windows, points
 * are accumulated into buckets by their window digits (bucket accumulation),
 * buckets are combined per window (bucket aggregation), and windows are
 * combined into the result (group aggregation) (Sec. II-C).  Points are kept
 * in twisted-Edwards extended coordinates (X, Y, T, Z); inputs to bucket
 * accumulation are prepared as (X, Y, U = k T) with Z = 1 and added with the
 * mixed addition, while aggregation uses the complete addition (Sec. II-D).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - A field element (FE) is 12 little-endian uint32 words.  Device-side FEs
 *    crossing this boundary are canonical (< p).  Twisted-Edwards data is in
 *    Montgomery form (value * 2^384 mod p); Weierstrass affine input/output
 *    ("std") is in ordinary form.
 *  - Scalars are 8 little-endian uint32 words each, one scalar after another,
 *    and must be < 2^253 (values >= 2^253 are flagged, see MSM_FLAG_RANGE).
 *  - Every pointer argument is a DEVICE pointer owned by the caller unless
 *    stated otherwise; the library never frees or keeps caller memory.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls validate their
 *    arguments on the host, enqueue work on `stream` and return without
 *    synchronising; results are valid once the stream has reached them.
 *    Calls on distinct workspaces may run concurrently.
 *  - Return value: MSM_OK (0) or a negative MSM_E* code.  Nothing is enqueued
 *    when a call returns an error from argument validation.
 *
 * Layouts
 *  - SoA ("structure of arrays", limb-major): coordinate c, word l of element
 *    i is at word index (c*12 + l)*count + i.
 *  - AoS records: element i occupies a contiguous record; an XYU record is
 *    36 words (X, Y, U), an XYTZ record 48 words (X, Y, T, Z).
 */
#ifndef MSM_H_
#define MSM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSM_OK 0
#define MSM_EINVAL (-1) /* null pointer, zero/oversized count, c out of [1, 20] */
#define MSM_ENOSPC (-2) /* workspace smaller than msm_workspace_bytes() */
#define MSM_EHIP (-3)   /* HIP launch/runtime error; see msm_last_hip_error() */

/* device-written status flags (bit set = condition detected) */
#define MSM_FLAG_RANGE 1u    /* a scalar >= 2^253 (its bits >= 253 were ignored) */
#define MSM_FLAG_OFFCURVE 2u /* an input point is not on y^2 = x^3 + 1 */
#define MSM_FLAG_EXCEPT 4u   /* an input point is exceptional for the Edwards map
                                (it cannot lie in the prime-order subgroup) */

#define MSM_FORM_XYTZ 0 /* second PADD operand in extended coordinates */
#define MSM_FORM_XYU 1  /* second PADD operand prepared: (X, Y, U = kT), Z = 1 */

#define MSM_RESULT_WORDS 32 /* x[12], y[12], inf, flags, 6 reserved */

/* Digit encodings of the scalars (Sec. II-C slices the scalars into c-bit
 * windows and assigns each point to the bucket of its slice value).
 *  MSM_DIGITS_UNSIGNED: the plain slices d_w = (s >> w c) mod 2^c,
 *    W = ceil(253 / c) windows, 2^c buckets per window, bucket b = d_w
 *    (bucket 0 stays the identity).
 *  MSM_DIGITS_SIGNED: the slices recoded into d_w in [-2^(c-1), 2^(c-1)] with
 *    s = sum_w d_w 2^(w c): from the lowest window up, a slice plus the
 *    incoming carry that reaches 2^(c-1) becomes d_w = v - 2^c with a carry of
 *    one into the next window; the top window is never recoded.
 *    W = ceil(254 / c) windows; a point with d_w != 0 is added with the sign
 *    of d_w to bucket m = |d_w| - 1, 2^(c-1) buckets per window, and the window
 *    sum weights bucket m by m + 1.  Same MSM, half the buckets to aggregate.
 *    Requires c >= 2. */
#define MSM_DIGITS_SIGNED 0
#define MSM_DIGITS_UNSIGNED 1
/*  MSM_DIGITS_GLV: the endomorphism split (not in the paper; the same MSM
 *    with half-length scalars).  phi(x, y) = (omega x, y) multiplies G1 by
 *    lambda = x0^2 - 1, and lambda^2 + lambda + 1 = r, so each scalar splits
 *    as s = s1 lambda + s0 with s0, s1 < 2^127 and s P = s0 P + s1 phi(P).
 *    The prepared points must come from msm_points_prepare_endo (2n records:
 *    each point followed by its image); the 2n half-scalars use signed
 *    digits with W = ceil(128 / c) windows and 2^(c-1) buckets per window,
 *    bucket entries indexed by record (record 2i: s0 of scalar i; record
 *    2i + 1: s1 of scalar i).  Requires c >= 2; scalars are given as for
 *    the other encodings. */
#define MSM_DIGITS_GLV 2

/* Batched point addition out_i = a_i + b_i (Sec. II-D; the paper's "task").
 * a_xytz: SoA, 4 coordinates x 12 words x count.  b: SoA, 4 coordinates
 * (MSM_FORM_XYTZ, complete addition) or 3 coordinates (MSM_FORM_XYU, mixed
 * addition with Z2 = 1).  out_xytz: SoA like a_xytz, canonical; may alias a.
 * Errors: MSM_EINVAL for null pointers, count = 0 or count >= 2^29 (larger
 * batches exceed the device memory anyway), or an unknown b_form. */
int msm_padd_batch(const uint32_t* a_xytz, const uint32_t* b, uint32_t* out_xytz, size_t count,
                   int b_form, void* stream);

/* The paper's two PADD workloads outside an MSM (Sec. IV).
 *
 * msm_padd_chain -- latency: out = P_0 + P_1 + ... + P_{count-1}, added one
 *   after another into a single accumulator (starting at the identity), each
 *   addition waiting for the previous one, with the complete addition.
 *   pts_xytz: AoS XYTZ records (48 words each, Montgomery form, coordinates
 *   < 2p).  unit: MSM_UNIT_WIDE (two waves share one point, each
 *   coordinate spread over 16 lanes as 24-bit limbs, a third wave preparing
 *   k T of the next point: the latency unit group aggregation uses),
 *   MSM_UNIT_QUAD (four lanes share one point: the latency unit of the
 *   aggregation tree) or MSM_UNIT_LANE (one lane does the whole addition).
 *   out_xytz: one AoS XYTZ record, lazily reduced (< 2p).
 *   Errors: MSM_EINVAL (null pointers, count = 0 or >= 2^31, unknown unit).
 *
 * msm_accumulate_stream -- throughput: `accumulators` independent running
 *   sums; accumulator a = sum of the prepared points i = a, a + A, a + 2A, ...
 *   (A = accumulators), mixed addition, each sum written once at the end.
 *   xyu: AoS prepared records (msm_points_prepare).  out_xytz: A AoS XYTZ
 *   records (lazily reduced; accumulators without points hold the identity).
 *   Up to 1024 accumulators run one wide unit each (the latency unit
 *   above), more run one lane each.
 *   Errors: MSM_EINVAL (null pointers, n = 0, A = 0, n or A >= 2^31). */
#define MSM_UNIT_QUAD 0
#define MSM_UNIT_LANE 1
#define MSM_UNIT_WIDE 2
int msm_padd_chain(const uint32_t* pts_xytz, size_t count, int unit, uint32_t* out_xytz,
                   void* stream);
int msm_accumulate_stream(const uint32_t* xyu, size_t n, size_t accumulators, uint32_t* out_xytz,
                          void* stream);

/* Batched Montgomery product out_i = a_i * b_i * 2^-384 mod p (the field core
 * of every PADD, Sec. III-B/III-C with Montgomery reduction as proposed in
 * Sec. V-C).  a, b, out: SoA with one coordinate (12 x count words).  Inputs
 * may be any values with a_i * b_i < 2^384 p.  canonical != 0 reduces the
 * output to [0, p); otherwise it is the lazily reduced value in [0, 2p).
 * Errors: MSM_EINVAL as for msm_padd_batch. */
int msm_fe_mul_batch(const uint32_t* a, const uint32_t* b, uint32_t* out, size_t count,
                     int canonical, void* stream);

/* Field-multiplication cores compared (the paper's future work, Sec. V-C:
 * Montgomery reduction and Karatsuba multiplication): out_i = a_i * b_i^rounds
 * in the variant's arithmetic, each product waiting for the previous one.
 *  MSM_MUL_MONT: the production Montgomery multiply (R = 2^384):
 *    out = a b^rounds R^-rounds mod p.
 *  MSM_MUL_BARRETT: plain residues, Barrett reduction with k = 378:
 *    out = a b^rounds mod p.
 *  MSM_MUL_KARATSUBA: Montgomery with one Karatsuba level over 6-word halves
 *    and a separate reduction: same output as MSM_MUL_MONT.
 *  MSM_MUL_WIDE: the Montgomery product spread over lanes (16 limbs of 24
 *    bits, one per lane, two elements per wave), with the reduction digits
 *    formed as one product m = (a b mod R)(-p^-1) mod R: the latency-oriented
 *    form; same output as MSM_MUL_MONT.
 *  MSM_MUL_F28: the carry-free core of the one-lane PADD unit: 14 limbs of
 *    28 bits, one per 32-bit word, so a column of 32x32->64 multiply-adds
 *    needs no carry word; Montgomery with R' = 2^392:
 *    out = a b^rounds 2^(-392 rounds) mod p.
 * a, b, out: SoA, one coordinate (12 x count words); inputs canonical
 * (< p); output canonical.  Errors: MSM_EINVAL (null pointers, count = 0 or
 * >= 2^31, rounds < 1, unknown variant), MSM_EHIP. */
#define MSM_MUL_MONT 0
#define MSM_MUL_BARRETT 1
#define MSM_MUL_KARATSUBA 2
#define MSM_MUL_WIDE 3
#define MSM_MUL_F28 4
int msm_fe_mul_chain(const uint32_t* a, const uint32_t* b, uint32_t* out, size_t count,
                     int variant, int rounds, void* stream);

/* Convert Weierstrass affine points (x, y), y^2 = x^3 + 1, to prepared
 * twisted-Edwards form (Sec. II-D: inputs as (X, Y, U = k T), Z = 1).
 * xy_std: SoA, 2 coordinates x 12 words x n, ordinary form, canonical.
 * inf: n uint32 flags (non-zero = point at infinity) or NULL.
 * xyu: AoS, 36 words per point, Montgomery form, canonical.
 * status: one device uint32 that receives MSM_FLAG_OFFCURVE / MSM_FLAG_EXCEPT
 * bits (OR-ed in; the caller clears it).  Points in the prime-order subgroup
 * are never exceptional.  Errors: MSM_EINVAL for null pointers or n = 0. */
int msm_points_prepare(const uint32_t* xy_std, const uint32_t* inf, uint32_t* xyu, size_t n,
                       uint32_t* status, void* stream);

/* As msm_points_prepare, and also the images phi(P_i) = (omega x_i, y_i)
 * of the points under the curve's order-3 automorphism (for
 * MSM_DIGITS_GLV): xyu receives 2n AoS records, record 2i = P_i and
 * record 2i + 1 = phi(P_i), so the records of a slice of the points are a
 * slice of the records.  Errors: MSM_EINVAL for null pointers, n = 0 or
 * n >= 2^30. */
int msm_points_prepare_endo(const uint32_t* xy_std, const uint32_t* inf, uint32_t* xyu, size_t n,
                            uint32_t* status, void* stream);

/* Synthetic-workload generator: P_i = k_i G for the conventional generator G
 * of BLS12-377 G1, written as Weierstrass affine points.  k: 8 words per
 * scalar (any value < 2^256).  xy_std: SoA, 2 x 12 x n words, ordinary form,
 * canonical.  inf: n uint32 flags (1 where k_i G is the point at infinity).
 * Errors: MSM_EINVAL for null pointers or n = 0. */
int msm_gen_points(const uint32_t* k, size_t n, uint32_t* xy_std, uint32_t* inf, void* stream);

/* Number of windows W for window width c and a digit encoding (0 when c is
 * out of range for the encoding). */
int msm_num_windows(int c, int encoding);

/* Bits per window for a requested width c: the windows keep their count
 * W = msm_num_windows(c, encoding), and the width is lowered to the smallest
 * one that still covers the digit bits (253 unsigned, 254 signed, 128 for the
 * endomorphism halves) with W windows, so that the top window is not left
 * with a few bits whose digits would crowd a handful of buckets.  Bucket
 * arrays have 2^c' (unsigned) or 2^(c'-1) buckets per window for this c'.
 * Returns 0 when c is out of range for the encoding. */
int msm_window_bits(int c, int encoding);

/* Workspace (device bytes) needed by msm_bucket_accumulate / msm_run for n
 * points, window width c (c = 0: the width msm_run would pick) and a digit
 * encoding.  Returns 0 for invalid arguments. */
size_t msm_workspace_bytes(size_t n, int c, int encoding);

/* Window width msm_run picks for n points when called with c = 0 and signed
 * or unsigned digits (a cost model: n W entries plus the aggregation of W
 * windows of buckets, widths 4..20).  With the endomorphism split, c = 0
 * picks from a model of its own (2n W entries of W = ceil(127 / c') windows):
 * c' = 16 up to n ~ 2^21 and 19 (seven windows) above. */
int msm_default_window(size_t n);

/* Bucket accumulation (Sec. II-C), digits of c' = msm_window_bits(c,
 * encoding) bits.  With unsigned digits B[w][b] = sum of the P_i whose w-th
 * digit d_w(s_i) equals b, 0 <= b < 2^c' (bucket 0 holds the identity); with
 * signed digits B[w][m] = sum of sign(d_w(s_i)) P_i over the i with
 * |d_w(s_i)| = m + 1, 0 <= m < 2^(c'-1).  xyu: AoS prepared points
 * (msm_points_prepare).  scalars: 8 words per scalar.  buckets: AoS XYTZ
 * records, record index w * (buckets per window) + bucket, Montgomery form,
 * lazily reduced (< 2p; compare after normalisation -- any projective
 * multiple is the same point).  ws: device workspace of
 * ws_bytes >= msm_workspace_bytes(n, c, encoding); word 0 of ws receives the
 * status flags (MSM_FLAG_RANGE).
 * Errors: MSM_EINVAL (null, n = 0, n >= 2^26, 2^31 or more digit slots --
 * n times the window count, twice that with the endomorphism split; e.g.
 * widths below 8 at n near 2^26 -- c not in [1, 20] -- [2, 20]
 * for signed digits -- or an unknown encoding), MSM_ENOSPC, MSM_EHIP. */
int msm_bucket_accumulate(const uint32_t* xyu, const uint32_t* scalars, size_t n, int c,
                          int encoding, uint32_t* buckets, void* ws, size_t ws_bytes,
                          void* stream);

/* Full MSM: result = sum_i s_i P_i (Sec. II-C), Pippenger with window width
 * c (c = 0 picks msm_default_window(n), or the split digits' own choice)
 * and the given digit encoding.
 * result: MSM_RESULT_WORDS device words: x[12], y[12] (Weierstrass affine,
 * ordinary form, canonical), inf (1 if the sum is the point at infinity, then
 * x = y = 0), flags (MSM_FLAG_RANGE).  Other arguments as for
 * msm_bucket_accumulate.  Errors as for msm_bucket_accumulate. */
int msm_run(const uint32_t* xyu, const uint32_t* scalars, size_t n, int c, int encoding,
            uint32_t* result, void* ws, size_t ws_bytes, void* stream);

/* Full MSM as msm_run, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the workspace is a library-owned device array of
 * MSM_NOALLOC_SCRATCH_BYTES per GPU (reserved when the library is loaded on
 * that GPU and held until the process ends), so the call allocates nothing;
 * the caller passes inputs and the result buffer as for msm_run.  It fits n
 * up to 2^16 points at the default width in every encoding
 * (msm_workspace_bytes(n, c, encoding) must not exceed
 * MSM_NOALLOC_SCRATCH_BYTES).  Every call on a GPU
 * shares that GPU's array: calls whose work overlaps on one GPU (on
 * different streams, or from several threads) race and must be ordered by
 * the caller; each call initialises what it reads of the array.  No timing
 * events are recorded.  Errors: as msm_run, and MSM_ENOSPC when the MSM
 * needs more than the array. */
#define MSM_NOALLOC_SCRATCH_BYTES (128u << 20)
int msm_run_noalloc(const uint32_t* xyu, const uint32_t* scalars, size_t n, int c, int encoding,
                    uint32_t* result, void* stream);

/* Batched MSMs: many independent MSMs of different sizes as one launch
 * sequence (Sec. II-C per job; running many independent units side by side
 * is the paper's way of scaling PADD throughput, Sec. IV).  Jobs with the
 * same window width form a class; each class runs as one pipeline whose
 * kernels cover every window of every job of the class, and the classes run
 * concurrently on internal streams forked from the caller's stream.
 *
 * msm_job: device pointers owned by the caller (prepared points, scalars,
 * MSM_RESULT_WORDS result words), n >= 1 points, window width c (0 = the
 * choice of msm_run with c = 0), and the schedule (0 = the default for
 * each): chunk, the digit entries one lane sums in bucket accumulation
 * (default: enough entries that one resident round of lanes covers the
 * class; every value is rounded up to a multiple of 4, at least 4);
 * tree_quad, aggregation-tree levels
 * with fewer outputs than this run on the four-lane unit (default 65536);
 * tree_wide, levels with at most this many outputs run on the wide two-wave
 * unit (default 1024).  Jobs of a batch with the same width and schedule
 * form one class.  The schedule changes the time, never the result.  A batch
 * keeps the pointers: between runs the caller may rewrite the scalars and
 * points in place, not move them.
 *
 * msm_batch_workspace_bytes: device bytes a batch of these jobs needs
 *   (0 for invalid jobs).
 * msm_batch_create: validates and plans the jobs, copies their tables into
 *   ws (a synchronous host-to-device copy; ws must stay allocated and
 *   untouched until msm_batch_destroy) and creates the internal streams.
 *   use_graph != 0: the first msm_batch_run captures the batch's launches
 *   into a HIP graph and every run launches that graph.  *out receives the
 *   batch handle (host memory owned by the library).
 * msm_batch_run: enqueues one run of every job on `stream` (results valid
 *   once the stream reaches them).  Runs of one batch must not overlap.
 * msm_batch_destroy: waits for the batch's work, frees the handle, its
 *   streams and its graph; NULL is accepted.
 * Errors: MSM_EINVAL (null pointers, njobs = 0, a job with n = 0 or an
 * invalid c, more than 2^26 points or 2^31 digits per class), MSM_ENOSPC,
 * MSM_EHIP. */
typedef struct msm_job {
  const uint32_t* xyu;
  const uint32_t* scalars;
  uint32_t* result;
  size_t n;
  int c;
  int chunk;      /* accumulation entries per lane (0 = default) */
  int tree_quad;  /* quad-unit threshold of the aggregation tree (0 = 65536) */
  int tree_wide;  /* wide-unit threshold of the aggregation tree (0 = 1024) */
} msm_job;

typedef struct msm_batch msm_batch;

size_t msm_batch_workspace_bytes(const msm_job* jobs, size_t njobs, int encoding);
int msm_batch_create(const msm_job* jobs, size_t njobs, int encoding, void* ws, size_t ws_bytes,
                     int use_graph, msm_batch** out);
int msm_batch_run(msm_batch* batch, void* stream);
int msm_batch_destroy(msm_batch* batch);

/* MSM server: a request loop for MSMs that arrive over time (continuous
 * batching at request granularity; the paper computes one MSM at a time, so
 * this is an addition for serving many of them on one GPU).
 *
 * msm_server_create: allocates an arena of hbm_budget_bytes device bytes (the
 *   server's only device allocation) and `streams` (1..16) streams of default
 *   priority; every request uses the given digit encoding.  *out receives the
 *   handle (host memory owned by the library).
 * msm_server_submit: queues one MSM (job as for msm_batch_create; c = 0
 *   picks as msm_run does).  Its workspace (msm_workspace_bytes) is its
 *   footprint: it is admitted -- launched on the stream with the fewest
 *   requests in flight -- as soon as that much of the arena is free and no
 *   earlier request is still waiting (FIFO).  While fewer than three
 *   requests are in flight, an admitted request's bucket accumulation waits
 *   for the previous request to finish (arrival order at light load); with
 *   more in flight, requests overlap fully.  Ordering: an event is recorded
 *   on `stream` (the producer's stream; NULL = the null stream) at the call,
 *   and the request's kernels wait for it, so work the caller enqueued on
 *   that stream before submitting (writing the points or scalars, clearing
 *   the result) happens first.  The job's buffers must stay valid, and
 *   unwritten, until the request is reported finished; its result is valid
 *   from then on.  *ticket receives the request's id (1, 2, ... in
 *   submission order).  MSM_ENOSPC when the footprint exceeds the whole
 *   budget (nothing is queued).
 * msm_server_progress: non-blocking; retires requests whose work has
 *   finished (their results are then valid), admits waiting ones, and writes
 *   up to cap finished tickets (oldest first) to the HOST array done, their
 *   number to *ndone.  Tickets not returned stay for the next call.
 * msm_server_drain: blocks until every submitted request has finished.
 * msm_server_stats: requests in flight, requests waiting, arena bytes in use
 *   (any output may be NULL).
 * msm_server_destroy: waits for the work in flight, frees the arena, the
 *   streams and the handle; NULL is accepted.
 * A server is driven from one host thread at a time.
 * Errors: MSM_EINVAL (null pointers, invalid job or arguments), MSM_ENOSPC,
 * MSM_EHIP. */
typedef struct msm_server msm_server;

int msm_server_create(size_t hbm_budget_bytes, int streams, int encoding, msm_server** out);
int msm_server_submit(msm_server* server, const msm_job* job, void* stream, uint64_t* ticket);
int msm_server_progress(msm_server* server, uint64_t* done, size_t cap, size_t* ndone);
int msm_server_drain(msm_server* server);
int msm_server_stats(msm_server* server, size_t* in_flight, size_t* queued,
                     size_t* bytes_in_use);
int msm_server_destroy(msm_server* server);

/* Timing for measurement.  msm_profile_enable(mode):
 *   MSM_PROFILE_OFF (0): nothing is recorded.
 *   MSM_PROFILE_PHASES (1): each call records HIP events on its own stream
 *     around its phases: "sort" (histogram, scan, scatter), "accum" (the
 *     bucket accumulation kernel), "merge" (split-bucket merge), "agg"
 *     (bucket aggregation), "horner" (group aggregation and the affine
 *     result).  Each event record stalls the stream briefly between kernels,
 *     so this mode adds several microseconds per phase boundary.
 *   MSM_PROFILE_ACCUM_KERNEL (2): only "accum", from start and stop events
 *     attached to the accumulation kernel's own dispatch: no event records
 *     between kernels, so the stream runs as it does unprofiled.
 * msm_profile_read synchronises on the recorded events, returns the summed
 * milliseconds and the number of recorded launches of one phase since the
 * last read, and forgets them.  Nothing is recorded under graph capture.
 * Errors: MSM_EINVAL (mode out of range, unknown phase, null outputs),
 * MSM_EHIP. */
#define MSM_PROFILE_OFF 0
#define MSM_PROFILE_PHASES 1
#define MSM_PROFILE_ACCUM_KERNEL 2
int msm_profile_enable(int mode);
int msm_profile_read(const char* phase, double* total_ms, int* launches);

/* Microbenchmarks for the roofline denominators (not part of the MSM path).
 * kind MSM_MB_MAD64: 2048 x 256 threads, each issuing 16 * param independent
 *   v_mad_u64_u32 (the field core's 32x32->64 multiply-add);
 * kind MSM_MB_ADDC: the same with v_addc_co_u32 (the carry add);
 *   for both, buf is a device buffer of at least 2048 * 256 * 8 bytes.
 * kind MSM_MB_COPY: copies param bytes (a multiple of 16) from the first half
 *   of buf to the second; buf_bytes >= 2 * param, buf 16-byte aligned.
 * Lone-wave kinds (one wave of 64 lanes; buf >= 512 bytes), for the latency
 * of dependent chains: MSM_MB_MAD64_LONE issues 16 * param mads in 8
 * independent chains, MSM_MB_MAD64_DEP 16 * param mads in one dependent
 * chain, MSM_MB_FEMUL_DEP param dependent Montgomery products.
 * The caller times the launch on `stream`.  Errors: MSM_EINVAL, MSM_EHIP. */
#define MSM_MB_MAD64 0
#define MSM_MB_ADDC 1
#define MSM_MB_COPY 2
#define MSM_MB_MAD64_LONE 3
#define MSM_MB_MAD64_DEP 4
#define MSM_MB_FEMUL_DEP 5
int msm_microbench(int kind, size_t param, void* buf, size_t buf_bytes, void* stream);

/* HIP error code (hipError_t value) behind the last MSM_EHIP on this thread. */
int msm_last_hip_error(void);

/* Human-readable name of a status code. */
const char* msm_status_string(int status);

/* Host copy of the built-in constants the kernels use, for independent
 * checking: words [0,12) p, [12,24) 2^384 mod p, [24,36) 2^768 mod p, then in
 * Montgomery form (value * 2^384 mod p): [36,48) the Edwards constant k,
 * [48,60) alpha, [60,72) beta (the Weierstrass/Edwards map x = alpha u - 1,
 * y = beta v), [72,84) G.x, [84,96) G.y.  out: HOST pointer to at least 96
 * words.  Returns MSM_OK or MSM_EINVAL (null out, words < 96). */
int msm_constants(uint32_t* out, size_t words);

#ifdef __cplusplus
}
#endif

#endif /* MSM_H_ */
