// Declarations shared by the translation units of libmsm_gfx950.so.
#pragma once
#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/msm.h"
#include "curve.hpp"
#include "field.hpp"

namespace msm {

// Constants of the Weierstrass <-> twisted-Edwards map, Montgomery form:
//   x_w = alpha u - 1,  y_w = beta v,  u = (1 + y_e)/(1 - y_e),  v = u / x_e
constexpr uint32_t kAlpha[NL] = {0x8894e1e4u, 0x3fabdfd0u, 0xcc1f55aau, 0xcbf921ddu,
                                 0x460edc0cu, 0xd17deff1u, 0x7897028du, 0xd394e81eu,
                                 0x0912681au, 0xc29c995du, 0xaff9d568u, 0x01515e6cu};
constexpr uint32_t kBeta[NL] = {0xa38cfd11u, 0xface0c97u, 0x0adb8383u, 0x8cc7c229u,
                                0xd44ae9cbu, 0x4765cd5fu, 0x22354029u, 0x9ae986d8u,
                                0x252ab9bdu, 0xc3dc7860u, 0xc8942395u, 0x00486011u};
constexpr uint32_t kBetaOverAlpha[NL] = {0xead605e4u, 0xfb7c0ab8u, 0xe2752c7au, 0x363b93d1u,
                                         0x144be536u, 0xd2246835u, 0x429f2077u, 0xeb8bf6ddu,
                                         0x0234d423u, 0x3a9efda2u, 0xba0c72a4u, 0x013c7943u};
// R^3 mod p: turns a plain inverse of a Montgomery value into Montgomery form
constexpr uint32_t kR3[NL] = {0x8815de20u, 0x581f532fu, 0xbe329585u, 0xe50f4148u,
                              0x0449f513u, 0x2be8b118u, 0xc804a20eu, 0x6a2a9516u,
                              0x13590cb9u, 0x3f725407u, 0xc0e7dda5u, 0x01065ab4u};
// omega (Montgomery form): the cube root of unity for which
// (x, y) -> (omega x, y) is multiplication by lambda = x0^2 - 1 on G1
constexpr uint32_t kOmega[NL] = {0xa5847973u, 0xdacd106du, 0xbac2a79au, 0xd8fe2454u,
                                 0xfd832edcu, 0x1ada4fd6u, 0x9d150908u, 0xfb986844u,
                                 0xea32285eu, 0xd63eb8aeu, 0x6f873fd0u, 0x0167d6a3u};
// conventional generator G of BLS12-377 G1, Weierstrass affine (Montgomery form)
constexpr uint32_t kGx[NL] = {0x772451f4u, 0x260f33b9u, 0x169d5658u, 0xc54dd773u,
                              0x69a510ddu, 0x5c1551c4u, 0x425e1698u, 0x761662e4u,
                              0x6f065272u, 0xc97d78ccu, 0xb361fd4du, 0x00a41206u};
constexpr uint32_t kGy[NL] = {0xb8cb81f3u, 0x8193961fu, 0x5f44adb8u, 0x00638d4cu,
                              0xd4daf54au, 0xfafaf3dau, 0xd655cd18u, 0xc27849e2u,
                              0x01d52814u, 0x2ec3ddb4u, 0x26303c71u, 0x007da933u};
// G in prepared twisted-Edwards form (x_e, y_e, k x_e y_e), Montgomery form
constexpr uint32_t kGteX[NL] = {0x654b417fu, 0x5bab21b3u, 0x1d3e1fe0u, 0x042fff8au,
                                0xdf39dc37u, 0xb702072eu, 0x39426b02u, 0xa5625e78u,
                                0xb51c7d03u, 0xbf2dc368u, 0x28ac3263u, 0x00b3ad90u};
constexpr uint32_t kGteY[NL] = {0xef15101du, 0x3904973cu, 0xb1f14456u, 0xb45ed211u,
                                0x5dfac94eu, 0x90a86b86u, 0xfe3945cdu, 0xcdb19c57u,
                                0xef4f7097u, 0x972a8d46u, 0xa3d9cf77u, 0x00281a91u};
constexpr uint32_t kGteU[NL] = {0x4f3f8d58u, 0x719243efu, 0x4a7b9d48u, 0xf744d1fcu,
                                0xa77008dcu, 0x0ab712e3u, 0x1e09b26fu, 0x53f80798u,
                                0xef3f9f1bu, 0x24125ab8u, 0xfb63f6d1u, 0x01959f77u};

constexpr int SCALAR_BITS = 253;  // scalars are below 2^253
constexpr int GLV_BITS = 127;     // halves of the endomorphism split are below 2^127
constexpr int SCALAR_WORDS = 8;

inline unsigned grid_for(size_t n, unsigned block) { return (unsigned)((n + block - 1) / block); }

// ---------------------------------------------------------------------------
// error reporting and optional per-phase timing (msm_api.hip)
// ---------------------------------------------------------------------------
void set_last_hip_error(int e);

#define HIPCHK(x)                         \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) {               \
      ::msm::set_last_hip_error((int)e_); \
      return MSM_EHIP;                    \
    }                                     \
  } while (0)

enum ProfTag { PT_SORT = 0, PT_ACCUM, PT_MERGE, PT_AGG, PT_HORNER, PT_COUNT };

// Records HIP events around its lifetime on `st` while profiling is enabled.
struct ProfScope {
  bool active = false;
  int tag = 0;
  hipStream_t st = nullptr;
  hipEvent_t a = nullptr;
  ProfScope(int t, hipStream_t s);
  ~ProfScope();
};

// Start and stop events for one kernel dispatch of phase `tag`, when the
// profiling mode times that kernel alone (false otherwise); the caller
// launches with them (hipExtLaunchKernelGGL) and then records the pair.
bool prof_kernel_events(int tag, hipStream_t st, hipEvent_t* a, hipEvent_t* b);
void prof_kernel_record(int tag, hipEvent_t a, hipEvent_t b);

// Digit sort geometry: partitions of uniformly spread digits hold about
// SORT_PART_TARGET entries; pass 2 stages up to SORT_PART_CAP in LDS and
// sorts larger partitions on many blocks, in items of SORT_BIG_ITEM entries.
constexpr uint32_t SORT_PART_TARGET = 4096;
constexpr uint32_t SORT_PART_CAP = 10240;
constexpr uint32_t SORT_BIG_ITEM = 4096;

// ---------------------------------------------------------------------------
// jobs and workspace plans (msm_api.hip)
// ---------------------------------------------------------------------------
// One pipeline runs a batch of J independent MSMs that share the window width
// c and the digit encoding; a single MSM is a batch of one.  Window w of job j
// is segment s = j W + w.  Segment s holds the job's n digits at
// [W pt_off + w n, W pt_off + (w+1) n) of the digit array and owns the
// pass-1 sort tiles [W tile_off + w tps, W tile_off + (w+1) tps).
struct JobDesc {
  const uint32_t* xyu;      // prepared points (AoS XYU records)
  const uint32_t* scalars;  // 8 words per scalar
  uint32_t* result;         // MSM_RESULT_WORDS words
  uint32_t n;               // points of the job
  uint32_t pt_off;          // points of the jobs before it
  uint32_t tile_off;        // tile groups per window of the jobs before it
  uint32_t tps;             // sort tile groups per window, ceil(n / tile_digits)
};

// Kernel-argument view of a batch's jobs: a device table, or (J = 1) the one
// job by value so that a single MSM needs no table upload.
struct JobView {
  const JobDesc* tab;
  JobDesc one;
  uint32_t J;
  __device__ __forceinline__ JobDesc get(uint32_t j) const { return tab ? tab[j] : one; }
};

constexpr uint32_t SORT_TILE = 8192;  // digits per pass-1 sort tile

struct Plan {
  int c = 0, W = 0;
  int encoding = MSM_DIGITS_SIGNED;
  int bb = 0;  // bucket-index bits: c (unsigned digits) or c - 1 (signed)
  uint32_t J = 1;
  size_t N = 0;       // points over all jobs
  size_t max_n = 0;   // largest job
  size_t S = 0;       // segments J W
  size_t M = 0;       // buckets S 2^bb
  size_t NW = 0;      // digits N W
  size_t tiles = 0;   // pass-1 sort tiles over all segments
  size_t chunks = 0;  // accumulation chunks
  uint32_t K = 32;    // entries per accumulation chunk (the first Kx chunks: K + 4)
  uint32_t Kx = 0;    // accumulation chunks of K + 4 entries, before those of K
  uint64_t tree_quad = 65536;  // tree levels with fewer outputs run on quads
  uint64_t tree_wide = 1024;   // levels with at most this many outputs on wide units
  uint32_t lo_bits = 0, hi_bits = 0;  // split of the bb bucket bits in the sort
  uint32_t tpb = 1;                   // pass-1 tiles per block (one histogram per group)
  uint32_t tile_digits = SORT_TILE;   // digits per group, SORT_TILE tpb
  bool tmp_packed = false;            // staged sort entries in one word (jobs <= 2^23 points)
  size_t ncounts = 0, nb = 0;         // sort count matrix size, its scan blocks
  JobDesc one{};  // the job when J = 1; otherwise one.xyu is the base of segment offsets
  // byte offsets into the workspace
  size_t o_flags = 0, o_total = 0, o_offsets = 0, o_counts = 0, o_blocksums = 0, o_digits = 0,
         o_tmp = 0, o_key = 0, o_idx = 0, o_head = 0, o_tail = 0, o_buckets = 0, o_lvl0 = 0,
         o_lvl1 = 0, o_wsum = 0, o_qstate = 0, o_longlist = 0, o_big = 0, o_bigdesc = 0, o_bigcnt = 0, o_bigitem = 0, o_jobs = 0, o_segoff = 0, bytes = 0;
};

int num_windows(int c, int encoding);
int window_bits(int c, int encoding);
int default_window(size_t n);                     // signed-digit model (msm_default_window)
int default_window_for(size_t n, int encoding);   // the width c = 0 picks for an encoding
// schedule of a plan (0 = default for each; msm_job's chunk, tree_quad,
// tree_wide)
struct Schedule {
  int chunk = 0, tree_quad = 0, tree_wide = 0;
  bool operator<(const Schedule& o) const {
    if (chunk != o.chunk) return chunk < o.chunk;
    if (tree_quad != o.tree_quad) return tree_quad < o.tree_quad;
    return tree_wide < o.tree_wide;
  }
};

// plan of a batch with job sizes ns[0..J); false for invalid sizes, c or
// schedule values
bool make_plan(const size_t* ns, uint32_t J, int c, int encoding, Plan& pl,
               const Schedule& sched = Schedule());

template <typename T>
inline T* ws_at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// every phase of a planned batch on one stream (msm_api.hip); with an event
// `accum_after`, the accumulation first waits for that event's last recording
// (the digit sort does not)
int enqueue_msm(const Plan& pl, void* ws, hipStream_t st, hipEvent_t accum_after = nullptr);

inline JobView job_view(const Plan& pl, void* ws) {
  JobView v;
  v.tab = pl.J == 1 ? nullptr : ws_at<const JobDesc>(ws, pl.o_jobs);
  v.one = pl.one;
  v.J = pl.J;
  return v;
}

// ---------------------------------------------------------------------------
// kernel launchers (each returns MSM_OK or MSM_EHIP)
// ---------------------------------------------------------------------------
// k_sort.hip: digits -> CSR offsets, sorted (key, idx | sign << 31); empty
// buckets set to the identity
// fills lo_bits, hi_bits, tpb, tile_digits, tiles (groups over all segments),
// ncounts, nb for jobs of mult * ns[j] points
void sort_geometry(Plan& pl, const size_t* ns, uint32_t J, size_t mult);
int launch_sort(const Plan& pl, uint32_t* buckets, void* ws, hipStream_t st);
// k_accum.hip: bucket accumulation and split-bucket merge
int launch_accumulate(const Plan& pl, uint32_t* buckets, void* ws, hipStream_t st);
// k_agg.hip: bucket aggregation (window sums), group aggregation and the
// affine results of every job
int launch_aggregate(const Plan& pl, const uint32_t* buckets, void* ws, hipStream_t st);
int launch_horner(const Plan& pl, void* ws, hipStream_t st);
// k_elementwise.hip
int launch_fe_mul(const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t count,
                  int canonical, hipStream_t st);
int launch_padd(const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t count, int form,
                hipStream_t st);
int launch_prepare(const uint32_t* xy, const uint32_t* inf, uint32_t* xyu, uint32_t n,
                   uint32_t* status, bool endo, hipStream_t st);
int launch_gen_points(const uint32_t* k, uint32_t* xy, uint32_t* inf, uint32_t n, hipStream_t st);
int launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st);

}  // namespace msm
