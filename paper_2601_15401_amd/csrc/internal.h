// Internal structures shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mick.h"
#include "modarith.h"

namespace mick {

constexpr int kMaxK = 12;     // largest k of a k-input multiply
constexpr int kKipTileLog = 10;  // log2 of the key-product kernel's tile (elements)
constexpr int kModupTileLog = 13;  // log2 of the ModUp kernel's tile (elements)
constexpr int kMaxJobs = 64;  // jobs per batched launch sequence

// Device pointers to the per-prime tables.  Prime index j < L is q_j,
// L + i is p_i.
struct DevTables {
  const uint32_t* mod;    // [L+K]
  const uint32_t* minv;   // [L+K] m^-1 mod 2^32 (Montgomery)
  const Red64* red;       // [L+K]
  const uint32_t* tw;     // [L+K][N][2] forward twiddle, Shoup companion; pass-B stages transposed
  const uint32_t* itw;    // [L+K][N][2] inverse twiddles, same layout
  const uint32_t* nfix;   // [L+K][4]: N^-1, Shoup; (stage-0 inverse twiddle) N^-1, Shoup
  const uint32_t* rpow;   // [L+K][2*(kMaxK+1)]: R^e mod m and Shoup, e = 0..kMaxK
};

// Where the limbs of one transform launch live and which prime each uses.
// Limb i: group g = i / period, position pos = i % period; data at
// base + g * group_stride + pos * N (+ blockIdx.z * job_stride); prime
// pos + off_lo if pos < split, else pos + off_hi.  nfix_pos, when set,
// replaces the per-prime N^-1 constants of an inverse transform by
// per-position ones (4 words each), folding a per-limb factor into it.
struct LimbMap {
  int period;
  long long group_stride;
  int split, off_lo, off_hi;
  long long job_stride;
  const uint32_t* nfix_pos;
};

// Workspace of one k-input multiply at `level`, in elements: the tensor
// product D [k+1][level][N], the scaled coefficient-domain d_2..d_k
// [k-1][level][N], the ModUp pass-A outputs [k-1][B][level+K][N] and the two
// accumulators [2][level+K][N].
struct WsLayout {
  size_t D, dcoef, X, acc, total;
  __host__ __device__ WsLayout(int k, int level, int K, int alpha, int log_n) {
    const size_t N = (size_t)1 << log_n;
    const int E = level + K, B = (level + alpha - 1) / alpha;
    D = 0;
    dcoef = D + (size_t)(k + 1) * level * N;
    X = dcoef + (size_t)(k - 1) * level * N;
    acc = X + (size_t)(k - 1) * B * E * N;
    total = acc + 2 * (size_t)E * N;
  }
};

// Heterogeneous batches: every stage of the multiply is one launch over a
// table of jobs of one ring degree (the jobs' k and level may differ); each
// block finds its job by binary search over the jobs' first blocks.
enum Stage { S_TENSOR, S_INTT_D, S_MODUP, S_KIP, S_INTT_ACC, S_MODDOWN, S_NTT_OUT, kStages };

// One rank of a job-adjacent block order (seg_block): the job at that rank
// (its index in the table), its groups of 8 units, where its segment starts.
struct Seg {
  int job, groups, base;
};

struct JobDesc {
  const uint32_t* in[kMaxK];  // input ciphertexts [2][level][N]
  uint32_t* out;              // output [2][level-k+1][N]
  uint32_t* ws;               // the job's workspace (WsLayout)
  int k, level;
  int blk0[kStages];          // first block of the job in each stage's launch (multiple of 8)
  // job-adjacent block orders (seg_block): [0] the tensor launch of the
  // job's run of equal k, [1] the key-product launch over the whole table
  Seg seg[2];
};

// A job-adjacent block order over n jobs ranked by unit count, descending.
// Blocks go by unit group g (8 units, one per XCD), then by rank: within
// group g the ranks whose units reach it, 8 blocks each.  Those ranks are a
// prefix 0..c_g - 1, and c_g steps down at each rank's group count: rank r's
// segment holds the groups [groups(r + 1), groups(r)) with r + 1 ranks each,
// from block group base(r) on (base(n - 1) = 0; a segment's end is the
// previous rank's base).  Block b -> (rank, unit); unit >= the job's units:
// padding.  The jobs of one unit then run back to back on one XCD and share
// what the unit reads (twiddles, key words) in its L2.
template <int ORDER>
__device__ __forceinline__ void seg_block(const JobDesc* jt, int n, int b, int& rank, int& unit) {
  const int xcd = b & 7, seq = b >> 3;
  int lo = 0, hi = n - 1;  // the first rank whose segment starts at or before seq
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (jt[mid].seg[ORDER].base <= seq)
      hi = mid;
    else
      lo = mid + 1;
  }
  const int r = lo;
  const int g_lo = r + 1 < n ? jt[r + 1].seg[ORDER].groups : 0;
  const int off = seq - jt[r].seg[ORDER].base;
  rank = off % (r + 1);
  unit = (g_lo + off / (r + 1)) * 8 + xcd;
}

// Index (relative to jt) of the last job whose first block in `stage` is <= b.
__device__ __forceinline__ int find_job(const JobDesc* jt, int n, int stage, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jt[mid].blk0[stage] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Per parameter set and key set: what the table kernels read besides the
// job table.  Offsets are element offsets into the parameter tables.
struct GroupConsts {
  const uint32_t* modup_tab;
  const uint32_t* modup_off;   // [L][dnum]: offset of the (level, digit) table
  const uint32_t* rs_tab;
  const uint32_t* rs_off;      // [L+1][L+1]: offset of the (level, mu) table
  const uint32_t* dscale;
  const uint32_t* dscale_off;  // [L+1]
  const uint32_t* md;          // ModDown constants
  const uint32_t* evk;
  int log_n, L, K, dnum, alpha;
};

struct mick_params_impl;

}  // namespace mick

namespace mick {

// Device allocator of long-lived objects (mick_set_allocator); null
// functions mean hipMalloc / hipFree.  Each object keeps the allocator that
// created it and frees its memory with the same one.
struct Allocator {
  mick_alloc_fn alloc = nullptr;
  mick_free_fn release = nullptr;
  void* ctx = nullptr;
};
Allocator current_allocator();
int dev_alloc_bytes(const Allocator& a, void** p, size_t bytes);
void dev_free(const Allocator& a, void* p);

}  // namespace mick

struct mick_params {
  int log_n, N, L, K, dnum, alpha;
  mick::Allocator alloc;
  std::vector<uint32_t> q, p, mods;  // mods = q ++ p
  int device;
  // device allocations
  void* d_tables = nullptr;  // one allocation for all per-prime tables
  mick::DevTables dt;
  // ModUp basis conversion tables per (level, digit): offsets into d_modup
  uint32_t* d_modup = nullptr;
  std::vector<size_t> modup_off;  // index (level - 1) * dnum + digit
  // ModDown tables: phinv (+Shoup) [K][2], pinvq [K][L]
  uint32_t* d_moddown = nullptr;
  // rescale tables per (level, mu)
  uint32_t* d_rescale = nullptr;
  // per level: N^-1 constants of the ModUp inverse transform with each limb's
  // qhat_j^-1 (within its digit) folded in, [level][4]
  uint32_t* d_dscale = nullptr;
  std::vector<size_t> dscale_off;  // index level
  // device copies of modup_off, rescale_off and dscale_off (uint32)
  uint32_t* d_offsets = nullptr;
  std::vector<size_t> rescale_off;  // index level * (L + 1) + mu
  // P^-1 and P mod q_j (host)
  std::vector<uint32_t> pinv_q, p_mod_q;
  // host copies of psi per prime
  std::vector<uint32_t> psi;
  int split_a, split_b;  // log2 rows of the two NTT passes
  int tensor_method;     // TensorMethod of the fused tensor kernels
  int modup_targets;     // ModUp targets per workgroup for digits of 5..8 primes (1 or 2)
  // the last mick_autotune's timings: (first-pass log, tensor method, ModUp
  // targets, microseconds per multiply)
  std::vector<std::vector<double>> tune_table;
};

// A heterogeneous batch ready to run: the job table lives in the caller's
// workspace, the launch sizes here.
struct mick_plan {
  const mick_params* prm;
  const mick_keys* keys;
  mick::JobDesc* table;
  int n_jobs;
  int blocks[mick::kStages];
  struct Run {  // jobs [j0, next j0) share k
    int j0, k, tensor_blocks, moddown_blocks;
  };
  std::vector<Run> runs;
  // source of the asynchronous copy of the job table: lives as long as the
  // plan, which the caller keeps until the copy has run
  std::vector<mick::JobDesc> host_table;
};

struct mick_keys {
  const mick_params* prm;
  mick::Allocator alloc;
  int k_max;
  uint64_t seed;
  std::vector<int64_t> s;  // host copy of the secret
  uint32_t* d_S = nullptr;    // [L+K][N] NTT(s)
  uint32_t* d_pk = nullptr;   // [2][L][N] (b, a)
  uint32_t* d_evk = nullptr;  // [t = 2..k_max][dnum][2][L+K][N], q rows x P^-1
};

namespace mick {

// Launch sites the optional profiler distinguishes.  A transform site's
// pass A is the listed value, its pass B the next one.
enum ProfSite {
  P_TENSOR,
  P_INTT_D,
  P_INTT_D_B,
  P_MODUP,
  P_NTT_X,
  P_NTT_X_B,
  P_KIP,
  P_INTT_ACC,
  P_INTT_ACC_B,
  P_MODDOWN_RS,
  P_NTT_OUT,
  P_NTT_OUT_B,
  P_RS_SUMS,
  P_RS_COMBINE,
  P_OTHER,
  P_OTHER_B,
  P_TENSOR_IB,
  P_COUNT
};

// Records a pair of HIP events around one launch on `s` when profiling is
// enabled (mick_profile_enable); free otherwise.
struct ProfScope {
  ProfScope(int site, hipStream_t s);
  ~ProfScope();
  int site, idx;
  hipStream_t stream;
};

// Error reporting (thread-local message).
int set_error(int status, const std::string& msg);
int hip_error(hipError_t e, const char* what);

#define MICK_TRY(expr)              \
  do {                              \
    int _st = (expr);               \
    if (_st != MICK_OK) return _st; \
  } while (0)
#define MICK_HIP(expr, what) MICK_TRY(::mick::hip_error((expr), (what)))

// Transforms (ntt.hip).  src may equal dst.
int ntt_launch(const mick_params* prm, const uint32_t* src, uint32_t* dst, const LimbMap& map, int n_limbs, int n_jobs,
               bool inverse, hipStream_t s, int site = P_OTHER);
// The inverse transform's second pass (pass A, with N^-1) alone, in place:
// for limbs whose first pass (pass B) already ran elsewhere.
int intt_pass_a_launch(const mick_params* prm, uint32_t* buf, const LimbMap& map, int n_limbs, int n_jobs,
                       hipStream_t s, int site);
LimbMap simple_map(const mick_params* prm, int first_prime, int n_limbs);
// Frees the standalone basis-conversion tables built for `prm` (bconv.hip).
void bconv_release(const mick_params* prm);

inline size_t evk_offset(const mick_params* prm, int t, int b, int l) {
  size_t limbs = (size_t)(prm->L + prm->K);
  return ((((size_t)(t - 2) * prm->dnum + b) * 2 + l) * limbs) << prm->log_n;
}

inline int digits_at(const mick_params* prm, int level) { return (level + prm->alpha - 1) / prm->alpha; }

// Job tables (api.hip).  job_ws_bytes: one job's workspace (aligned);
// table_bytes: a table of n_jobs entries (aligned).  check_job validates
// one job's shape, keys and pointers; check_jobs every job.  plan_jobs
// writes the table of n_jobs jobs (job i using the workspace job_ws[i]) to
// table_dev with an asynchronous copy from the plan's own host table, so the
// plan must outlive that copy.
// One multiply's workspace in words (D, scaled d_t, ModUp outputs,
// accumulators) and the relinearisation of the degree-k product D at the
// start of `ws` followed by mu rescales (api.hip).
size_t mul_ws_words(const mick_params* prm, int k, int level);
int relin_rescale_one(const mick_params* prm, const mick_keys* keys, int k, int level, int mu, uint32_t* ws,
                      uint32_t* out, hipStream_t s);

size_t job_ws_bytes(const mick_params* prm, int k, int level);
size_t table_bytes(int n_jobs);
int check_job(const mick_params* prm, const mick_keys* keys, const mick_job& job);
int check_jobs(const mick_params* prm, const mick_keys* keys, const mick_job* jobs, int n_jobs);
int plan_jobs(const mick_params* prm, const mick_keys* keys, const mick_job* jobs, int n_jobs,
              uint32_t* const* job_ws, JobDesc* table_dev, hipStream_t s, mick_plan** out);

}  // namespace mick
