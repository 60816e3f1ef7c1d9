// C ABI of libmick: parameter tables, key generation, encryption,
// decryption and the orchestration of the k-input multiply.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "host_math.h"
#include "internal.h"
#include "rns.h"

using namespace mick;

// Workspace of the allocation-free multiply (mick_mul_relin_rescale_noalloc):
// one copy per device, held from the code object's load until the process
// ends.  Host code never passes this name as an address: each device's copy
// is reached through the pointer hipGetSymbolAddress returns for it, looked
// up once per device and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) uint32_t scratch[kScratchBytes / 4];

namespace mick {

static thread_local std::string g_last_error;

int set_error(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int hip_error(hipError_t e, const char* what) {
  if (e == hipSuccess) return MICK_OK;
  return set_error(MICK_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- profiler
namespace {
const char* const kSiteNames[P_COUNT] = {
    "tensor",       "intt_d.passA",  "intt_d.passB",  "modup_bconv_passA", "unused.passA", "unused.passB",
    "passB_kip",    "intt_acc.passA", "intt_acc.passB", "moddown_rescale", "ntt_out.passA", "ntt_out.passB",
    "rescale_sums", "rescale_combine", "ntt_other.passA", "ntt_other.passB", "tensor_inttB"};
std::mutex g_prof_mu;
bool g_prof_on = false;
uint32_t g_prof_mask = ~0u;  // sites that record while profiling is on
std::vector<hipEvent_t> g_prof_events;            // pool, two per record
std::vector<std::pair<int, int>> g_prof_records;  // (site, first event index)
}  // namespace

ProfScope::ProfScope(int site_, hipStream_t s) : site(site_), idx(-1), stream(s) {
  if (!g_prof_on || !((g_prof_mask >> site) & 1u)) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  size_t need = 2 * (g_prof_records.size() + 1);
  while (g_prof_events.size() < need) {
    // timing only: these events order nothing for the host, so they skip
    // the system-scope fence a default event performs when it is reached
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return;
    g_prof_events.push_back(e);
  }
  idx = (int)(2 * g_prof_records.size());
  g_prof_records.push_back({site, idx});
  (void)hipEventRecord(g_prof_events[idx], s);
}

ProfScope::~ProfScope() {
  if (idx < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  (void)hipEventRecord(g_prof_events[idx + 1], stream);
}

}  // namespace mick

namespace {

constexpr int kSecretWeight = 64;
constexpr double kSigma = 3.2;


uint32_t inv_pow2_32(uint32_t m) {  // m^-1 mod 2^32 by Newton iteration
  uint32_t x = m;
  for (int i = 0; i < 5; i++) x *= 2 - m * x;
  return x;
}

int brv(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; i++) r |= ((x >> i) & 1) << (bits - 1 - i);
  return r;
}

template <typename T>
int upload(T* dst, const std::vector<T>& src, hipStream_t s) {
  MICK_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
  MICK_HIP(hipStreamSynchronize(s), "upload sync");
  return MICK_OK;
}

template <typename T>
int dev_alloc(const Allocator& a, T** p, size_t count) {
  void* v = nullptr;
  MICK_TRY(dev_alloc_bytes(a, &v, std::max<size_t>(count, 1) * sizeof(T)));
  *p = (T*)v;
  return MICK_OK;
}

// Residues of an integer polynomial over the moduli with prime indices
// [first, first + rows).
std::vector<uint32_t> residues(const mick_params* prm, const int64_t* poly, int first, int rows) {
  std::vector<uint32_t> out((size_t)rows * prm->N);
  for (int r = 0; r < rows; r++) {
    int64_t m = prm->mods[first + r];
    for (int i = 0; i < prm->N; i++) {
      int64_t v = poly[i] % m;
      out[(size_t)r * prm->N + i] = (uint32_t)(v < 0 ? v + m : v);
    }
  }
  return out;
}

int build_tables(mick_params* prm) {
  const int N = prm->N, log_n = prm->log_n, L = prm->L, K = prm->K, E = L + K;
  const int la = prm->split_a;
  // ---- per-prime tables, one allocation
  size_t n_mod = E, n_red = (size_t)E * 4, n_tw = (size_t)E * N * 2, n_fix = (size_t)E * 4,
         n_rpow = (size_t)E * 2 * (kMaxK + 1);
  size_t total = n_mod * 2 + n_red + n_tw * 2 + n_fix + n_rpow;
  std::vector<uint32_t> h(total, 0);
  uint32_t* h_mod = h.data();
  uint32_t* h_minv = h_mod + n_mod;
  uint32_t* h_red = h_minv + n_mod;
  uint32_t* h_tw = h_red + n_red;
  uint32_t* h_itw = h_tw + n_tw;
  uint32_t* h_fix = h_itw + n_tw;
  uint32_t* h_rpow = h_fix + n_fix;
  prm->psi.resize(E);
  std::vector<uint32_t> pw(2 * (size_t)N);
  for (int r = 0; r < E; r++) {
    const uint32_t m = prm->mods[r];
    h_mod[r] = m;
    h_minv[r] = inv_pow2_32(m);
    const uint32_t r32 = (uint32_t)(((uint64_t)1 << 32) % m);
    h_red[4 * r + 0] = m;
    h_red[4 * r + 1] = r32;
    h_red[4 * r + 2] = shoup_companion(r32, m);
    h_red[4 * r + 3] = (uint32_t)(((uint64_t)1 << 32) / m);
    const uint32_t psi = smallest_psi(m, N);
    prm->psi[r] = psi;
    uint64_t v = 1;
    for (int i = 0; i < 2 * N; i++) {
      pw[i] = (uint32_t)v;
      v = v * psi % m;
    }
    uint32_t* tw = h_tw + (size_t)r * N * 2;
    uint32_t* itw = h_itw + (size_t)r * N * 2;
    for (int s = 0; s < log_n; s++) {
      for (int b = 0; b < (1 << s); b++) {
        int k = (1 << s) + b;
        int e = brv(k, log_n);
        uint32_t w = pw[e], wi = pw[(2 * N - e) % (2 * N)];
        int pos = k;
        if (s >= la) {  // pass-B stage: b = blk 2^sl + rr stored at rr 2^la + blk
          int sl = s - la;
          int blk = b >> sl, rr = b & ((1 << sl) - 1);
          pos = (1 << s) + (rr << la) + blk;
        }
        tw[2 * pos] = 0u - w;  // stored negated: the forward butterfly forms -(Shoup product)
        tw[2 * pos + 1] = shoup_companion(w, m);
        itw[2 * pos] = wi;
        itw[2 * pos + 1] = shoup_companion(wi, m);
      }
    }
    const uint32_t ninv = (uint32_t)invmod(N, m);
    const uint32_t w1 = pw[(2 * N - brv(1, log_n)) % (2 * N)];
    const uint32_t w1n = (uint32_t)((uint64_t)w1 * ninv % m);
    h_fix[4 * r + 0] = ninv;
    h_fix[4 * r + 1] = shoup_companion(ninv, m);
    h_fix[4 * r + 2] = w1n;
    h_fix[4 * r + 3] = shoup_companion(w1n, m);
    uint64_t R = ((uint64_t)1 << 32) % m, rp = 1;
    for (int e = 0; e <= kMaxK; e++) {
      h_rpow[(size_t)r * 2 * (kMaxK + 1) + 2 * e] = (uint32_t)rp;
      h_rpow[(size_t)r * 2 * (kMaxK + 1) + 2 * e + 1] = shoup_companion((uint32_t)rp, m);
      rp = rp * R % m;
    }
  }
  MICK_TRY(dev_alloc(prm->alloc, (uint32_t**)&prm->d_tables, total));
  uint32_t* d = (uint32_t*)prm->d_tables;
  MICK_HIP(hipMemcpy(d, h.data(), total * 4, hipMemcpyHostToDevice), "table upload");
  prm->dt.mod = d;
  prm->dt.minv = d + n_mod;
  prm->dt.red = reinterpret_cast<const Red64*>(d + 2 * n_mod);
  prm->dt.tw = d + 2 * n_mod + n_red;
  prm->dt.itw = prm->dt.tw + n_tw;
  prm->dt.nfix = prm->dt.itw + n_tw;
  prm->dt.rpow = prm->dt.nfix + n_fix;

  // ---- ModUp tables per (level, digit), rows padded with zeros to the
  // kernel's digit width
  const int a = prm->alpha, arows = modup_rows(a);
  std::vector<uint32_t> mu;
  prm->modup_off.assign((size_t)L * prm->dnum, 0);
  for (int level = 1; level <= L; level++) {
    const int El = level + K;
    for (int b = 0; b < prm->dnum; b++) {
      int lo = b * a, hi = std::min(lo + a, level);
      prm->modup_off[(size_t)(level - 1) * prm->dnum + b] = mu.size();
      if (lo >= hi) continue;
      int cnt = hi - lo;
      std::vector<uint32_t> qh(arows, 0), qhs(arows, 0), C((size_t)arows * El, 0);
      for (int j = 0; j < cnt; j++) {
        uint32_t qj = prm->q[lo + j];
        uint64_t x = 1;
        for (int i = 0; i < cnt; i++)
          if (i != j) x = x * invmod(prm->q[lo + i] % qj, qj) % qj;
        qh[j] = (uint32_t)x;
        qhs[j] = shoup_companion((uint32_t)x, qj);
        for (int e = 0; e < El; e++) {  // qhat_j R mod m_e (Montgomery form)
          uint32_t me = e < level ? prm->q[e] : prm->p[e - level];
          uint64_t y = ((uint64_t)1 << 32) % me;
          for (int i = 0; i < cnt; i++)
            if (i != j) y = y * (prm->q[lo + i] % me) % me;
          C[(size_t)j * El + e] = (uint32_t)y;
        }
      }
      mu.insert(mu.end(), qh.begin(), qh.end());
      mu.insert(mu.end(), qhs.begin(), qhs.end());
      mu.insert(mu.end(), C.begin(), C.end());
    }
  }
  MICK_TRY(dev_alloc(prm->alloc, &prm->d_modup, mu.size()));
  MICK_HIP(hipMemcpy(prm->d_modup, mu.data(), mu.size() * 4, hipMemcpyHostToDevice), "modup upload");

  // ---- per level: the inverse transform's N^-1 constants times qhat_j^-1
  // of limb j within its digit (the scaling step of eq. (basis conversion))
  std::vector<uint32_t> ds;
  prm->dscale_off.assign((size_t)L + 1, 0);
  for (int level = 1; level <= L; level++) {
    prm->dscale_off[level] = ds.size();
    for (int j = 0; j < level; j++) {
      const int lo = (j / a) * a, hi = std::min(lo + a, level);
      const uint32_t qj = prm->q[j];
      uint64_t sc = 1;
      for (int i = lo; i < hi; i++)
        if (i != j) sc = sc * invmod(prm->q[i] % qj, qj) % qj;
      const uint32_t* nf = h_fix + 4 * (size_t)j;
      const uint32_t f0 = (uint32_t)(nf[0] * sc % qj), f2 = (uint32_t)(nf[2] * sc % qj);
      ds.push_back(f0);
      ds.push_back(shoup_companion(f0, qj));
      ds.push_back(f2);
      ds.push_back(shoup_companion(f2, qj));
    }
  }
  MICK_TRY(dev_alloc(prm->alloc, &prm->d_dscale, ds.size()));
  MICK_HIP(hipMemcpy(prm->d_dscale, ds.data(), ds.size() * 4, hipMemcpyHostToDevice), "dscale upload");

  // ---- ModDown tables and the chain constants q_d^-1 mod q_t
  std::vector<uint32_t> md;
  for (int i = 0; i < K; i++) {
    uint32_t pi = prm->p[i];
    uint64_t x = 1;
    for (int i2 = 0; i2 < K; i2++)
      if (i2 != i) x = x * invmod(prm->p[i2] % pi, pi) % pi;
    md.push_back((uint32_t)x);
    md.push_back(shoup_companion((uint32_t)x, pi));
  }
  for (int i = 0; i < K; i++)
    for (int j = 0; j < L; j++) md.push_back((uint32_t)invmod(prm->p[i] % prm->q[j], prm->q[j]));
  for (int d2 = 0; d2 < L; d2++) {
    for (int t = 0; t < L; t++) {
      uint32_t v = d2 == t ? 0 : (uint32_t)invmod(prm->q[d2] % prm->q[t], prm->q[t]);
      md.push_back(v);
      md.push_back(shoup_companion(v, prm->q[t]));
    }
  }
  MICK_TRY(dev_alloc(prm->alloc, &prm->d_moddown, md.size()));
  MICK_HIP(hipMemcpy(prm->d_moddown, md.data(), md.size() * 4, hipMemcpyHostToDevice), "moddown upload");

  // ---- rescale constants g^{mu,t}_eta per (level, mu), eq. (g(u,t,eta))
  std::vector<uint32_t> rs;
  prm->rescale_off.assign((size_t)(L + 1) * (L + 1), 0);
  for (int level = 2; level <= L; level++) {
    for (int m2 = 1; m2 < level && m2 <= 16; m2++) {
      prm->rescale_off[(size_t)level * (L + 1) + m2] = rs.size();
      int top = level - m2;
      std::vector<uint32_t> g((size_t)top * m2);
      for (int eta = 0; eta < top; eta++) {
        uint32_t qe = prm->q[eta];
        uint64_t x = 1;
        for (int t = level - m2; t < level; t++) {
          x = x * invmod(prm->q[t] % qe, qe) % qe;
          g[(size_t)eta * m2 + (t - (level - m2))] = (uint32_t)x;
        }
        rs.push_back((uint32_t)x);  // g^{mu,l-1}_eta
        rs.push_back(shoup_companion((uint32_t)x, qe));
      }
      rs.insert(rs.end(), g.begin(), g.end());
    }
  }
  MICK_TRY(dev_alloc(prm->alloc, &prm->d_rescale, rs.size()));
  if (!rs.empty()) MICK_HIP(hipMemcpy(prm->d_rescale, rs.data(), rs.size() * 4, hipMemcpyHostToDevice), "rs upload");

  // device copies of the table offsets, for the job-table kernels
  {
    std::vector<uint32_t> off;
    for (size_t v : prm->modup_off) off.push_back((uint32_t)v);
    for (size_t v : prm->rescale_off) off.push_back((uint32_t)v);
    for (size_t v : prm->dscale_off) off.push_back((uint32_t)v);
    MICK_TRY(dev_alloc(prm->alloc, &prm->d_offsets, off.size()));
    MICK_HIP(hipMemcpy(prm->d_offsets, off.data(), off.size() * 4, hipMemcpyHostToDevice), "offset upload");
  }

  // host constants
  prm->pinv_q.resize(L);
  prm->p_mod_q.resize(L);
  for (int j = 0; j < L; j++) {
    uint64_t P = 1;
    for (int i = 0; i < K; i++) P = P * (prm->p[i] % prm->q[j]) % prm->q[j];
    prm->p_mod_q[j] = (uint32_t)P;
    prm->pinv_q[j] = (uint32_t)invmod(P, prm->q[j]);
  }
  return MICK_OK;
}

MdArgs md_args(const mick_params* prm, int level, int mu) {
  MdArgs A{};
  A.md = prm->d_moddown;
  A.qinvq = prm->d_moddown + 2 * prm->K + (size_t)prm->K * prm->L;
  A.rs = mu > 0 ? prm->d_rescale + prm->rescale_off[(size_t)level * (prm->L + 1) + mu] : nullptr;
  A.log_n = prm->log_n;
  A.level = level;
  A.L = prm->L;
  A.K = prm->K;
  A.E = level + prm->K;
  return A;
}

struct Layout {  // per-job workspace of the multiply, in elements
  size_t D, dcoef, X, acc, total;
};

Layout mul_layout(const mick_params* prm, int k, int level) {
  const size_t N = prm->N;
  const int E = level + prm->K, B = digits_at(prm, level);
  Layout l;
  l.D = 0;
  l.dcoef = l.D + (size_t)(k + 1) * level * N;
  l.X = l.dcoef + (size_t)(k - 1) * level * N;
  l.acc = l.X + (size_t)(k - 1) * B * E * N;
  l.total = l.acc + 2 * (size_t)E * N;
  return l;
}

// The keys for the fused tensor kernel's own-digit sums.
OwnKeys own_keys(const mick_params* prm, const mick_keys* keys) {
  OwnKeys o{};
  o.evk = keys->d_evk;
  o.dnum = prm->dnum;
  o.alpha = prm->alpha;
  o.key_poly = (long long)(prm->L + prm->K) * prm->N;
  return o;
}

int check_mul(const mick_params* prm, const mick_keys* keys, int k, int level) {
  if (!prm || !keys) return set_error(MICK_E_ARG, "NULL params or keys");
  if (keys->prm != prm) return set_error(MICK_E_ARG, "keys belong to other params");
  if (k < 2 || k > kMaxK) return set_error(MICK_E_ARG, "k must be in 2..12");
  if (level < k || level > prm->L) return set_error(MICK_E_LEVEL, "level must be in k..L");
  if (k > keys->k_max) return set_error(MICK_E_KEY, "k exceeds the key set's k_max");
  return MICK_OK;
}

// Relinearisation and rescale of jobs whose tensor products are already in
// the workspace (D at the start of each job block).  d_pass_b: the first pass
// of d_2..d_k's INTT has run too (k_tensor_ib), its output in dcoef, and D
// holds the own-digit key sums (with d_0, d_1) in place of d_0..d_k.
int relin_rescale_ws(const mick_params* prm, const mick_keys* keys, int k, int level, int mu, uint32_t* ws,
                     size_t job_stride, int n_jobs, uint32_t* out, size_t out_job, hipStream_t s,
                     bool d_pass_b = false) {
  const Layout lay = mul_layout(prm, k, level);
  const int N = prm->N, L = prm->L, K = prm->K, E = level + K, B = digits_at(prm, level);
  // ModUp: INTT of d_2..d_k, each limb also multiplied by its qhat_j^-1
  LimbMap m = simple_map(prm, 0, level);
  m.job_stride = (long long)job_stride;
  m.nfix_pos = prm->d_dscale + prm->dscale_off[level];
  if (d_pass_b)
    MICK_TRY(intt_pass_a_launch(prm, ws + lay.dcoef, m, (k - 1) * level, n_jobs, s, P_INTT_D));
  else
    MICK_TRY(ntt_launch(prm, ws + lay.D + 2 * (size_t)level * N, ws + lay.dcoef, m, (k - 1) * level, n_jobs, true, s,
                        P_INTT_D));
  // basis conversion from each digit fused with pass A of the new limbs' NTT
  ModupArgs ma{};
  ma.tab = prm->d_modup;
  for (int b = 0; b < B; b++) ma.tab_off[b] = (int)prm->modup_off[(size_t)(level - 1) * prm->dnum + b];
  ma.log_n = prm->log_n;
  ma.level = level;
  ma.L = L;
  ma.E = E;
  ma.B = B;
  ma.alpha = prm->alpha;
  ma.groups = (k - 1) * B;
  ma.dcoef_job = (long long)job_stride;
  ma.x_job = (long long)job_stride;
  MICK_TRY(launch_modup_a(prm, ws + lay.dcoef, ws + lay.X, ma, n_jobs, s));
  // pass B fused with the key inner product, combined over t, with D_l added
  // on the q rows
  KipArgs ka{};
  ka.log_n = prm->log_n;
  ka.level = level;
  ka.L = L;
  ka.E = E;
  ka.B = B;
  ka.alpha = prm->alpha;
  ka.dnum = prm->dnum;
  ka.k = k;
  ka.n_jobs = n_jobs;
  ka.key_poly = (long long)(L + K) * N;
  ka.d_job = ka.x_job = ka.acc_job = (long long)job_stride;
  ka.own_sums = d_pass_b;  // the fused tensor kernel formed them
  MICK_TRY(launch_kip_b(prm, ws + lay.X, ws + lay.D, keys->d_evk, ws + lay.acc, ka, s));
  // relocated ModDown: INTT of every accumulator limb (its first pass ran in
  // the key-product kernel)
  LimbMap ma2 = simple_map(prm, 0, E);
  ma2.split = level;
  ma2.off_hi = L - level;
  ma2.job_stride = (long long)job_stride;
  MICK_TRY(intt_pass_a_launch(prm, ws + lay.acc, ma2, 2 * E, n_jobs, s, P_INTT_ACC));
  // scaled BConv, subtraction and the combined rescale, then the final NTT
  MdArgs A = md_args(prm, level, mu);
  A.acc_job = (long long)job_stride;
  A.out_job = (long long)out_job;
  MICK_TRY(launch_moddown_rs(prm, ws + lay.acc, out, A, mu, n_jobs, s));
  LimbMap mo = simple_map(prm, 0, level - mu);
  mo.job_stride = (long long)out_job;
  MICK_TRY(ntt_launch(prm, out, out, mo, 2 * (level - mu), n_jobs, false, s, P_NTT_OUT));
  return MICK_OK;
}

}  // namespace

namespace mick {

size_t mul_ws_words(const mick_params* prm, int k, int level) { return mul_layout(prm, k, level).total; }

int relin_rescale_one(const mick_params* prm, const mick_keys* keys, int k, int level, int mu, uint32_t* ws,
                      uint32_t* out, hipStream_t s) {
  return relin_rescale_ws(prm, keys, k, level, mu, ws, mul_layout(prm, k, level).total, 1, out, 0, s);
}

}  // namespace mick

// ====================================================================== C ABI

extern "C" {

const char* mick_strerror(int status) {
  switch (status) {
    case MICK_OK: return "ok";
    case MICK_E_ARG: return "invalid argument";
    case MICK_E_LEVEL: return "invalid level";
    case MICK_E_KEY: return "k exceeds the key set";
    case MICK_E_NOMEM: return "out of memory";
    case MICK_E_HIP: return "HIP runtime error";
    case MICK_E_RANGE: return "value out of range";
    case MICK_E_WS: return "workspace too small";
    case MICK_E_BUSY: return "over the queue's budget, or already running";
    case MICK_E_CANCELLED: return "cancelled";
    case MICK_PENDING: return "pending";
    default: return "unknown status";
  }
}

const char* mick_last_error(void) { return g_last_error.c_str(); }

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// This device's copy of `scratch`, looked up once with that device current.
int scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return set_error(MICK_E_ARG, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    MICK_HIP(hipGetDevice(&cur), "hipGetDevice");
    if (cur != device) MICK_HIP(hipSetDevice(device), "hipSetDevice");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    MICK_HIP(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(MICK_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return MICK_OK;
}

}  // namespace

int mick_params_create(int log_n, int L, int K, int dnum, mick_params** out) {
  if (!out) return set_error(MICK_E_ARG, "NULL out");
  *out = nullptr;
  if (log_n < 13 || log_n > 16) return set_error(MICK_E_ARG, "log_n must be in 13..16");
  if (L < 1 || L > 60 || K < 1 || K > kMaxKp || dnum < 1 || dnum > L)
    return set_error(MICK_E_ARG, "need 1 <= L <= 60, 1 <= K <= 24, 1 <= dnum <= L");
  const int alpha = (L + dnum - 1) / dnum;
  if (alpha > kMaxAlpha || (L + alpha - 1) / alpha > 16)
    return set_error(MICK_E_ARG, "ceil(L / dnum) must be at most 32, with at most 16 digits");
  std::unique_ptr<mick_params> p(new mick_params());
  p->log_n = log_n;
  p->N = 1 << log_n;
  p->L = L;
  p->K = K;
  p->dnum = dnum;
  p->alpha = alpha;
  p->alloc = current_allocator();
  p->q = ntt_primes(30, 2 * (uint64_t)p->N, L);
  p->p = ntt_primes(31, 2 * (uint64_t)p->N, K);
  if ((int)p->q.size() < L || (int)p->p.size() < K) return set_error(MICK_E_ARG, "not enough NTT-friendly primes");
  p->mods = p->q;
  p->mods.insert(p->mods.end(), p->p.begin(), p->p.end());
  static const int split_a[17] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 7, 7, 8, 8};
  p->split_a = split_a[log_n];
  p->split_b = log_n - p->split_a;
  p->tensor_method = kTensorChain;
  p->modup_targets = 2;
  MICK_HIP(hipGetDevice(&p->device), "hipGetDevice");
  void* scratch_dev = nullptr;  // the allocation-free multiply's workspace on this device
  MICK_TRY(scratch_address(p->device, &scratch_dev));
  int st = build_tables(p.get());
  if (st != MICK_OK) {
    mick_params_destroy(p.release());
    return st;
  }
  *out = p.release();
  return MICK_OK;
}

static void free_tables(mick_params* prm) {
  for (void** p : {(void**)&prm->d_tables, (void**)&prm->d_modup, (void**)&prm->d_moddown, (void**)&prm->d_rescale,
                   (void**)&prm->d_dscale, (void**)&prm->d_offsets}) {
    dev_free(prm->alloc, *p);
    *p = nullptr;
  }
}

void mick_params_destroy(mick_params* prm) {
  if (prm) bconv_release(prm);
  if (!prm) return;
  free_tables(prm);
  delete prm;
}

static bool schedule_ok(int log_n, int a) { return (a == 7 || a == 8) && log_n - a >= 6 && log_n - a <= 8; }

int mick_params_set_schedule(mick_params* prm, int first_pass_log) {
  if (!prm) return set_error(MICK_E_ARG, "NULL params");
  if (!schedule_ok(prm->log_n, first_pass_log))
    return set_error(MICK_E_ARG, "first pass must be 7 or 8 stages with 6..8 left for the second");
  if (first_pass_log == prm->split_a) return MICK_OK;
  MICK_HIP(hipDeviceSynchronize(), "schedule sync");
  const int old = prm->split_a;
  free_tables(prm);
  prm->split_a = first_pass_log;
  prm->split_b = prm->log_n - first_pass_log;
  int st = build_tables(prm);
  if (st != MICK_OK) {  // restore the previous schedule
    free_tables(prm);
    prm->split_a = old;
    prm->split_b = prm->log_n - old;
    (void)build_tables(prm);
  }
  return st;
}

int mick_params_schedule(const mick_params* prm) { return prm ? prm->split_a : set_error(MICK_E_ARG, "NULL params"); }

int mick_params_set_tensor_method(mick_params* prm, int method) {
  if (!prm) return set_error(MICK_E_ARG, "NULL params");
  if (method < 0 || method >= kTensorMethods) return set_error(MICK_E_ARG, "tensor method must be 0, 1 or 2");
  prm->tensor_method = method;
  return MICK_OK;
}

int mick_params_tensor_method(const mick_params* prm) {
  return prm ? prm->tensor_method : set_error(MICK_E_ARG, "NULL params");
}

int mick_params_set_modup_targets(mick_params* prm, int targets) {
  if (!prm) return set_error(MICK_E_ARG, "NULL params");
  if (targets != 1 && targets != 2) return set_error(MICK_E_ARG, "ModUp targets per workgroup must be 1 or 2");
  if (targets == 2 && !modup_two_targets(prm->alpha))
    return set_error(MICK_E_ARG, "two targets per workgroup need digits of 5 to 8 primes");
  prm->modup_targets = targets;
  return MICK_OK;
}

int mick_params_modup_targets(const mick_params* prm) {
  if (!prm) return set_error(MICK_E_ARG, "NULL params");
  return modup_pairs_on(prm) ? 2 : 1;
}

namespace {

struct TuneConfig {
  int a, tm, mt;
};

// Device time of `reps` fused multiplies of a batch of `jobs` with the
// current settings (synthetic keys and inputs: the timing does not depend
// on the values).
int time_multiply(const mick_params* prm, const mick_keys* keys, int k, int level, int jobs, const uint32_t* cts,
                  uint32_t* out, uint32_t* ws, size_t ws_bytes, int reps, hipEvent_t e0, hipEvent_t e1,
                  double* us) {
  MICK_TRY(mick_mul_relin_rescale_batch(prm, keys, cts, jobs, k, level, out, ws, ws_bytes, nullptr));  // warm-up
  MICK_HIP(hipEventRecord(e0, nullptr), "event");
  for (int r = 0; r < reps; r++)
    MICK_TRY(mick_mul_relin_rescale_batch(prm, keys, cts, jobs, k, level, out, ws, ws_bytes, nullptr));
  MICK_HIP(hipEventRecord(e1, nullptr), "event");
  MICK_HIP(hipEventSynchronize(e1), "event");
  float ms = 0;
  MICK_HIP(hipEventElapsedTime(&ms, e0, e1), "event");
  *us = 1e3 * ms / (reps * jobs);
  return MICK_OK;
}

}  // namespace

int mick_autotune(mick_params* prm, const char* cache_path) {
  if (!prm) return set_error(MICK_E_ARG, "NULL params");
  std::vector<TuneConfig> cand;
  for (int a : {7, 8})
    if (schedule_ok(prm->log_n, a))
      for (int tm = 0; tm < kTensorMethods; tm++)
        for (int mt : {2, 1})
          if (mt == 1 || modup_two_targets(prm->alpha)) cand.push_back({a, tm, mt});
  const char* path = cache_path ? cache_path : getenv("MICK_AUTOTUNE_CACHE");
  hipDeviceProp_t prop;
  MICK_HIP(hipGetDeviceProperties(&prop, prm->device), "device properties");
  char key[256];
  snprintf(key, sizeof key, "%s %d %d %d %d %d", prop.gcnArchName, prop.multiProcessorCount, prm->log_n, prm->L,
           prm->K, prm->dnum);
  for (char* c = key; *c; c++)
    if (*c == ':') *c = '_';  // keep the arch name one token
  auto apply = [&](const TuneConfig& c) -> int {
    if (prm->split_a != c.a) MICK_TRY(mick_params_set_schedule(prm, c.a));
    MICK_TRY(mick_params_set_tensor_method(prm, c.tm));
    return mick_params_set_modup_targets(prm, c.mt);
  };
  if (path) {
    if (FILE* f = fopen(path, "r")) {
      char line[512];
      int found = 0;
      TuneConfig best{};
      while (fgets(line, sizeof line, f)) {
        char arch[128];
        int cus, ln, l, k, d, a, tm, mt;
        double us;
        if (sscanf(line, "mick-tune %127s %d %d %d %d %d %d %d %d %lf", arch, &cus, &ln, &l, &k, &d, &a, &tm, &mt,
                   &us) != 10)
          continue;
        char k2[256];
        snprintf(k2, sizeof k2, "%s %d %d %d %d %d", arch, cus, ln, l, k, d);
        for (const TuneConfig& c : cand)
          if (strcmp(k2, key) == 0 && c.a == a && c.tm == tm && c.mt == mt) {
            best = c;  // the last valid entry wins
            found = 1;
          }
      }
      fclose(f);
      if (found) return apply(best);
    }
  }
  // time the fused multiply of a batch of two jobs at k = min(8, L), level L
  // under every candidate, in interleaved rounds (the median of each is kept)
  const int k = std::min(8, prm->L), level = prm->L, jobs = 2;
  if (k < 2) return MICK_OK;  // a single prime: no multiply to time
  const size_t N = prm->N, E = (size_t)prm->L + prm->K;
  const size_t evk_words = (size_t)(k - 1) * prm->dnum * 2 * E * N;
  const size_t in_words = (size_t)jobs * k * 2 * level * N;
  const size_t out_words = (size_t)jobs * 2 * (level - k + 1) * N;
  const size_t ws_bytes = mick_batch_workspace_bytes(prm, jobs, k, level);
  uint32_t *evk = nullptr, *in = nullptr, *out = nullptr, *ws = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  mick_keys fake;  // synthetic key set: only the evaluation-key words are read
  fake.prm = prm;
  fake.k_max = k;
  fake.seed = 0;
  const TuneConfig start{prm->split_a, prm->tensor_method, prm->modup_targets};
  std::vector<std::vector<double>> times(cand.size());
  int st = [&]() -> int {
    MICK_TRY(dev_alloc(prm->alloc, &evk, evk_words));
    MICK_TRY(dev_alloc(prm->alloc, &in, in_words));
    MICK_TRY(dev_alloc(prm->alloc, &out, out_words));
    MICK_TRY(dev_alloc(prm->alloc, &ws, ws_bytes / 4 + 1));
    // residues 0x11111111 < 2^29 are canonical for every prime here
    MICK_HIP(hipMemset(evk, 0x11, evk_words * 4), "autotune fill");
    MICK_HIP(hipMemset(in, 0x11, in_words * 4), "autotune fill");
    MICK_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence), "event");
    MICK_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence), "event");
    fake.d_evk = evk;
    constexpr int kRounds = 3, kReps = 4;
    for (int round = 0; round < kRounds; round++)
      for (size_t i = 0; i < cand.size(); i++) {
        MICK_TRY(apply(cand[i]));
        double us = 0;
        MICK_TRY(time_multiply(prm, &fake, k, level, jobs, in, out, ws, ws_bytes, kReps, e0, e1, &us));
        times[i].push_back(us);
      }
    return MICK_OK;
  }();
  fake.d_evk = nullptr;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipDeviceSynchronize();
  for (uint32_t* b : {evk, in, out, ws}) dev_free(prm->alloc, b);
  if (st != MICK_OK) {
    (void)apply(start);
    return st;
  }
  size_t best = 0;
  prm->tune_table.clear();
  std::vector<double> med(cand.size());
  for (size_t i = 0; i < cand.size(); i++) {
    std::sort(times[i].begin(), times[i].end());
    med[i] = times[i][times[i].size() / 2];
    prm->tune_table.push_back({(double)cand[i].a, (double)cand[i].tm, (double)cand[i].mt, med[i]});
    if (med[i] < med[best]) best = i;
  }
  MICK_TRY(apply(cand[best]));
  if (path) {
    if (FILE* f = fopen(path, "a")) {
      fprintf(f, "mick-tune %s %d %d %d %.2f\n", key, cand[best].a, cand[best].tm, cand[best].mt, med[best]);
      fclose(f);
    }
  }
  return MICK_OK;
}

int mick_autotune_report(const mick_params* prm, int max, int* configs, double* us) {
  if (!prm || (max > 0 && (!configs || !us))) return set_error(MICK_E_ARG, "NULL argument");
  const int n = std::min(max, (int)prm->tune_table.size());
  for (int i = 0; i < n; i++) {
    for (int j = 0; j < 3; j++) configs[3 * i + j] = (int)prm->tune_table[i][j];
    us[i] = prm->tune_table[i][3];
  }
  return (int)prm->tune_table.size();
}

int mick_params_moduli(const mick_params* prm, uint32_t* q_host, uint32_t* p_host) {
  if (!prm || !q_host || !p_host) return set_error(MICK_E_ARG, "NULL argument");
  memcpy(q_host, prm->q.data(), prm->L * 4);
  memcpy(p_host, prm->p.data(), prm->K * 4);
  return MICK_OK;
}

int mick_params_shape(const mick_params* prm, int* out5) {
  if (!prm || !out5) return set_error(MICK_E_ARG, "NULL argument");
  out5[0] = prm->log_n;
  out5[1] = prm->L;
  out5[2] = prm->K;
  out5[3] = prm->dnum;
  out5[4] = prm->alpha;
  return MICK_OK;
}

int mick_keygen(const mick_params* prm, uint64_t seed, int k_max, void* stream, mick_keys** out) {
  if (!prm || !out) return set_error(MICK_E_ARG, "NULL argument");
  *out = nullptr;
  if (k_max < 2 || k_max > kMaxK) return set_error(MICK_E_ARG, "k_max must be in 2..12");
  hipStream_t s = (hipStream_t)stream;
  const int N = prm->N, L = prm->L, K = prm->K, E = L + K;
  const size_t NE = (size_t)E * N;
  std::unique_ptr<mick_keys> keys(new mick_keys());
  keys->prm = prm;
  keys->alloc = current_allocator();
  keys->k_max = k_max;
  keys->seed = seed;
  keys->s = sample_ternary(stream_key(seed, "SK"), N, kSecretWeight);
  const int st_alloc = [&]() -> int {
    MICK_TRY(dev_alloc(keys->alloc, &keys->d_S, NE));
    MICK_TRY(dev_alloc(keys->alloc, &keys->d_pk, 2 * (size_t)L * N));
    return dev_alloc(keys->alloc, &keys->d_evk, (size_t)(k_max - 1) * prm->dnum * 2 * NE);
  }();
  if (st_alloc != MICK_OK) {
    mick_keys_destroy(keys.release());
    return st_alloc;
  }
  uint32_t *tE = nullptr, *tA = nullptr, *tSt = nullptr, *tRow = nullptr;
  auto cleanup = [&]() {
    dev_free(keys->alloc, tE);
    dev_free(keys->alloc, tA);
    dev_free(keys->alloc, tSt);
    dev_free(keys->alloc, tRow);
  };
  int st = [&]() -> int {
    MICK_TRY(dev_alloc(keys->alloc, &tE, NE));
    MICK_TRY(dev_alloc(keys->alloc, &tA, NE));
    MICK_TRY(dev_alloc(keys->alloc, &tSt, NE));
    MICK_TRY(dev_alloc(keys->alloc, &tRow, (size_t)E * 4));
    const GaussTable gt = gauss_table(kSigma);
    // S = NTT(s) over every modulus
    MICK_TRY(upload(keys->d_S, residues(prm, keys->s.data(), 0, E), s));
    MICK_TRY(ntt_launch(prm, keys->d_S, keys->d_S, simple_map(prm, 0, E), E, 1, false, s));
    // public key
    std::vector<uint32_t> ha((size_t)L * N);
    for (int j = 0; j < L; j++) sample_uniform(stream_key(seed, "PK_A", j), prm->q[j], N, ha.data() + (size_t)j * N);
    MICK_TRY(upload(keys->d_pk + (size_t)L * N, ha, s));
    std::vector<int64_t> e = sample_gauss(stream_key(seed, "PK_E"), N, gt);
    MICK_TRY(upload(tE, residues(prm, e.data(), 0, L), s));
    MICK_TRY(ntt_launch(prm, tE, tE, simple_map(prm, 0, L), L, 1, false, s));
    MICK_TRY(launch_pk(prm, tE, keys->d_pk + (size_t)L * N, keys->d_S, keys->d_pk, s));
    // evaluation keys for s^t, t = 2..k_max, one per digit
    MICK_HIP(hipMemcpyAsync(tSt, keys->d_S, NE * 4, hipMemcpyDeviceToDevice, s), "copy S");
    std::vector<uint32_t> hrow((size_t)E * 4);
    std::vector<uint32_t> hA(NE);
    for (int t = 2; t <= k_max; t++) {
      MICK_TRY(launch_mul_rows(prm, tSt, keys->d_S, E, s));
      for (int b = 0; b < prm->dnum; b++) {
        for (int r = 0; r < E; r++)
          sample_uniform(stream_key(seed, "EVK_A", t, b, r), prm->mods[r], N, hA.data() + (size_t)r * N);
        MICK_TRY(upload(tA, hA, s));
        std::vector<int64_t> ee = sample_gauss(stream_key(seed, "EVK_E", t, b), N, gt);
        MICK_TRY(upload(tE, residues(prm, ee.data(), 0, E), s));
        MICK_TRY(ntt_launch(prm, tE, tE, simple_map(prm, 0, E), E, 1, false, s));
        const int lo = b * prm->alpha, hi = std::min(lo + prm->alpha, L);
        for (int r = 0; r < E; r++) {
          uint32_t m = prm->mods[r];
          uint32_t g = (r < L && r >= lo && r < hi) ? prm->p_mod_q[r] : 0;
          // device copy: q rows times [P^-1] (Sec. IV), every row times
          // R = 2^32 (Montgomery form for the key inner product)
          const uint64_t R = ((uint64_t)1 << 32) % m;
          uint32_t f = (uint32_t)((r < L ? prm->pinv_q[r] : 1) * R % m);
          hrow[4 * r + 0] = g;
          hrow[4 * r + 1] = f;
          hrow[4 * r + 2] = shoup_companion(f, m);
          hrow[4 * r + 3] = 0;
        }
        MICK_TRY(upload(tRow, hrow, s));
        uint32_t* k0 = keys->d_evk + evk_offset(prm, t, b, 0);
        uint32_t* k1 = keys->d_evk + evk_offset(prm, t, b, 1);
        MICK_TRY(launch_evk(prm, tE, tA, keys->d_S, tSt, k0, k1, tRow, s));
      }
    }
    MICK_HIP(hipStreamSynchronize(s), "keygen sync");
    return MICK_OK;
  }();
  cleanup();
  if (st != MICK_OK) {
    mick_keys_destroy(keys.release());
    return st;
  }
  *out = keys.release();
  return MICK_OK;
}

void mick_keys_destroy(mick_keys* keys) {
  if (!keys) return;
  dev_free(keys->alloc, keys->d_S);
  dev_free(keys->alloc, keys->d_pk);
  dev_free(keys->alloc, keys->d_evk);
  delete keys;
}

int mick_keys_kmax(const mick_keys* keys) { return keys ? keys->k_max : MICK_E_ARG; }

int mick_keys_export(const mick_keys* keys, int what, int t, int b, void* host_out, void* stream) {
  if (!keys || !host_out) return set_error(MICK_E_ARG, "NULL argument");
  const mick_params* prm = keys->prm;
  hipStream_t s = (hipStream_t)stream;
  const size_t N = prm->N;
  const int L = prm->L, E = prm->L + prm->K;
  if (what == 0) {
    memcpy(host_out, keys->s.data(), N * 8);
    return MICK_OK;
  }
  if (what == 1) {
    MICK_HIP(hipMemcpyAsync(host_out, keys->d_pk, 2 * L * N * 4, hipMemcpyDeviceToHost, s), "export pk");
    MICK_HIP(hipStreamSynchronize(s), "export sync");
    return MICK_OK;
  }
  if (what == 2) {
    if (t < 2 || t > keys->k_max || b < 0 || b >= prm->dnum) return set_error(MICK_E_ARG, "no such key");
    uint32_t* o = (uint32_t*)host_out;
    MICK_HIP(hipMemcpyAsync(o, keys->d_evk + evk_offset(prm, t, b, 0), 2 * E * N * 4, hipMemcpyDeviceToHost, s),
             "export evk");
    MICK_HIP(hipStreamSynchronize(s), "export sync");
    for (int l = 0; l < 2; l++)
      for (int r = 0; r < E; r++) {  // undo the [P^-1] of the q rows and the factor R
        const uint64_t m = prm->mods[r];
        const uint64_t Rinv = invmod(((uint64_t)1 << 32) % m, m);
        const uint64_t f = (r < L ? prm->p_mod_q[r] : 1) * Rinv % m;
        uint32_t* row = o + ((size_t)l * E + r) * N;
        for (size_t i = 0; i < N; i++) row[i] = (uint32_t)(row[i] * f % m);
      }
    return MICK_OK;
  }
  return set_error(MICK_E_ARG, "unknown export kind");
}

int mick_encode(const mick_params* prm, const double* re, const double* im, size_t n_slots, double scale,
                int64_t* m_host) {
  if (!prm || !re || !im || !m_host) return set_error(MICK_E_ARG, "NULL argument");
  if (n_slots != (size_t)prm->N / 2) return set_error(MICK_E_ARG, "n_slots must be N/2");
  ckks_encode(prm->N, re, im, scale, m_host);
  return MICK_OK;
}

int mick_decode(const mick_params* prm, const int64_t* m_host, double scale, double* re, double* im,
                size_t n_slots) {
  if (!prm || !re || !im || !m_host) return set_error(MICK_E_ARG, "NULL argument");
  if (n_slots != (size_t)prm->N / 2) return set_error(MICK_E_ARG, "n_slots must be N/2");
  ckks_decode(prm->N, m_host, scale, re, im);
  return MICK_OK;
}

int mick_encrypt(const mick_params* prm, const mick_keys* keys, const int64_t* m_host, int level, uint64_t seed,
                 uint64_t ct_id, uint32_t* ct_dev, void* stream) {
  if (!prm || !keys || !m_host || !ct_dev) return set_error(MICK_E_ARG, "NULL argument");
  if (level < 1 || level > prm->L) return set_error(MICK_E_LEVEL, "level must be in 1..L");
  hipStream_t s = (hipStream_t)stream;
  const int N = prm->N;
  const size_t LN = (size_t)level * N;
  const GaussTable gt = gauss_table(kSigma);
  std::vector<int64_t> v = sample_ternary(stream_key(seed, "ENC_V", ct_id), N, N / 2);
  std::vector<int64_t> e0 = sample_gauss(stream_key(seed, "ENC_E0", ct_id), N, gt);
  std::vector<int64_t> e1 = sample_gauss(stream_key(seed, "ENC_E1", ct_id), N, gt);
  std::vector<uint32_t> hm = residues(prm, m_host, 0, level), he0 = residues(prm, e0.data(), 0, level);
  for (size_t i = 0; i < LN; i++) {
    uint32_t m = prm->q[i / N];
    hm[i] = (uint32_t)(((uint64_t)hm[i] + he0[i]) % m);
  }
  uint32_t* tmp = nullptr;
  MICK_TRY(dev_alloc(prm->alloc, &tmp, 3 * LN));
  int st = [&]() -> int {
    MICK_TRY(upload(tmp, residues(prm, v.data(), 0, level), s));
    MICK_TRY(upload(tmp + LN, hm, s));
    MICK_TRY(upload(tmp + 2 * LN, residues(prm, e1.data(), 0, level), s));
    LimbMap mp = simple_map(prm, 0, level);
    MICK_TRY(ntt_launch(prm, tmp, tmp, mp, 3 * level, 1, false, s));
    MICK_TRY(launch_enc(prm, tmp, tmp + LN, tmp + 2 * LN, keys->d_pk, ct_dev, level, s));
    MICK_HIP(hipStreamSynchronize(s), "encrypt sync");
    return MICK_OK;
  }();
  dev_free(prm->alloc, tmp);
  return st;
}

static int decrypt_res(const mick_params* prm, const mick_keys* keys, const uint32_t* ct_dev, int level,
                       uint32_t* res_host, hipStream_t s) {
  const size_t LN = (size_t)level * prm->N;
  uint32_t* tmp = nullptr;
  MICK_TRY(dev_alloc(prm->alloc, &tmp, LN));
  int st = [&]() -> int {
    MICK_TRY(launch_dec(prm, ct_dev, keys->d_S, tmp, level, s));
    MICK_TRY(ntt_launch(prm, tmp, tmp, simple_map(prm, 0, level), level, 1, true, s));
    MICK_HIP(hipMemcpyAsync(res_host, tmp, LN * 4, hipMemcpyDeviceToHost, s), "decrypt copy");
    MICK_HIP(hipStreamSynchronize(s), "decrypt sync");
    return MICK_OK;
  }();
  dev_free(prm->alloc, tmp);
  return st;
}

int mick_decrypt_residues(const mick_params* prm, const mick_keys* keys, const uint32_t* ct_dev, int level,
                          uint32_t* res_host, void* stream) {
  if (!prm || !keys || !ct_dev || !res_host) return set_error(MICK_E_ARG, "NULL argument");
  if (level < 1 || level > prm->L) return set_error(MICK_E_LEVEL, "level must be in 1..L");
  return decrypt_res(prm, keys, ct_dev, level, res_host, (hipStream_t)stream);
}

int mick_decrypt(const mick_params* prm, const mick_keys* keys, const uint32_t* ct_dev, int level, int64_t* m_host,
                 void* stream) {
  if (!prm || !keys || !ct_dev || !m_host) return set_error(MICK_E_ARG, "NULL argument");
  if (level < 1 || level > prm->L) return set_error(MICK_E_LEVEL, "level must be in 1..L");
  const int N = prm->N;
  std::vector<uint32_t> res((size_t)level * N);
  MICK_TRY(decrypt_res(prm, keys, ct_dev, level, res.data(), (hipStream_t)stream));
  std::vector<uint32_t> qs(prm->q.begin(), prm->q.begin() + level);
  Crt crt(qs);
  std::vector<uint32_t> col(level);
  for (int i = 0; i < N; i++) {
    for (int j = 0; j < level; j++) col[j] = res[(size_t)j * N + i];
    if (!crt.centred(col.data(), &m_host[i])) return set_error(MICK_E_RANGE, "coefficient exceeds 62 bits");
  }
  return MICK_OK;
}

size_t mick_workspace_bytes(const mick_params* prm, int op, int k, int level) {
  if (!prm || level < 1 || level > prm->L) return 0;
  const size_t N = prm->N;
  switch (op) {
    case MICK_OP_MUL_RELIN_RESCALE:
      if (k < 2 || k > kMaxK || level < k) return 0;
      return mul_layout(prm, k, level).total * 4;
    case MICK_OP_RELIN:
      if (k < 2 || k > kMaxK || level < k) return 0;
      return mul_layout(prm, k, level).total * 4;
    case MICK_OP_RESCALE:
      if (k < 1 || k >= level) return 0;
      return 2 * (size_t)level * N * 4;
    default: return 0;
  }
}

int mick_mul_k(const mick_params* prm, const uint32_t* const* cts_host, int k, int level, uint32_t* d_dev,
               void* stream) {
  if (!prm || !cts_host || !d_dev) return set_error(MICK_E_ARG, "NULL argument");
  if (k < 2 || k > kMaxK) return set_error(MICK_E_ARG, "k must be in 2..12");
  if (level < 1 || level > prm->L) return set_error(MICK_E_LEVEL, "level must be in 1..L");
  CtPtrs in{};
  for (int u = 0; u < k; u++) {
    if (!cts_host[u]) return set_error(MICK_E_ARG, "NULL ciphertext pointer");
    in.p[u] = cts_host[u];
  }
  return launch_tensor(prm, in, 0, k, level, d_dev, 0, 1, (hipStream_t)stream);
}

int mick_relin_k(const mick_params* prm, const mick_keys* keys, const uint32_t* d_dev, int k, int level,
                 uint32_t* ct_out_dev, void* ws, size_t ws_bytes, void* stream) {
  MICK_TRY(check_mul(prm, keys, k, level));
  if (!d_dev || !ct_out_dev || !ws) return set_error(MICK_E_ARG, "NULL argument");
  if (ws_bytes < mick_workspace_bytes(prm, MICK_OP_MUL_RELIN_RESCALE, k, level))
    return set_error(MICK_E_WS, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const Layout lay = mul_layout(prm, k, level);
  uint32_t* w = (uint32_t*)ws;
  // stage D in the workspace so that one layout serves every step
  MICK_HIP(hipMemcpyAsync(w + lay.D, d_dev, (size_t)(k + 1) * level * prm->N * 4, hipMemcpyDeviceToDevice, s),
           "stage d");
  return relin_rescale_ws(prm, keys, k, level, 0, w, lay.total, 1, ct_out_dev, 0, s);
}

}  // extern "C"

namespace mick {

// Algorithm 1 on `polys` NTT-domain polynomials in[polys][level][N] ->
// out[polys][level-mu][N]; ws holds polys level N words.
int rescale_polys(const mick_params* prm, const uint32_t* in, int polys, int level, int mu, uint32_t* out,
                  uint32_t* ws, hipStream_t s) {
  const size_t N = prm->N;
  const int top = level - mu;
  uint32_t* topc = ws;
  uint32_t* bb = topc + (size_t)polys * mu * N;
  // step 1: INTT of the mu dropped limbs of every polynomial
  MICK_HIP(hipMemcpy2DAsync(topc, (size_t)mu * N * 4, in + (size_t)top * N, (size_t)level * N * 4,
                            (size_t)mu * N * 4, polys, hipMemcpyDeviceToDevice, s),
           "stage dropped limbs");
  MICK_TRY(ntt_launch(prm, topc, topc, simple_map(prm, top, mu), polys * mu, 1, true, s));
  // steps 2 and 3: chain, sums, NTT, combine
  MdArgs A = md_args(prm, level, mu);
  MICK_TRY(launch_rs_sums(prm, topc, bb, A, mu, polys, s));
  MICK_TRY(ntt_launch(prm, bb, bb, simple_map(prm, 0, top), polys * top, 1, false, s));
  return launch_rs_combine(prm, in, bb, out, A, mu, polys, s);
}

}  // namespace mick

extern "C" {

int mick_rescale_multi(const mick_params* prm, const uint32_t* ct_in_dev, int level, int mu, uint32_t* ct_out_dev,
                       void* ws, size_t ws_bytes, void* stream) {
  if (!prm || !ct_in_dev || !ct_out_dev || !ws) return set_error(MICK_E_ARG, "NULL argument");
  if (level < 2 || level > prm->L || mu < 1 || mu >= level) return set_error(MICK_E_LEVEL, "need 1 <= mu < level <= L");
  if (mu > 16) return set_error(MICK_E_ARG, "mu must be at most 16");
  if (ws_bytes < mick_workspace_bytes(prm, MICK_OP_RESCALE, mu, level)) return set_error(MICK_E_WS, "workspace too small");
  return rescale_polys(prm, ct_in_dev, 2, level, mu, ct_out_dev, (uint32_t*)ws, (hipStream_t)stream);
}

int mick_mul_relin_rescale(const mick_params* prm, const mick_keys* keys, const uint32_t* const* cts_host, int k,
                           int level, uint32_t* ct_out_dev, void* ws, size_t ws_bytes, void* stream) {
  MICK_TRY(check_mul(prm, keys, k, level));
  if (!cts_host || !ct_out_dev || !ws) return set_error(MICK_E_ARG, "NULL argument");
  if (ws_bytes < mick_workspace_bytes(prm, MICK_OP_MUL_RELIN_RESCALE, k, level))
    return set_error(MICK_E_WS, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const Layout lay = mul_layout(prm, k, level);
  uint32_t* w = (uint32_t*)ws;
  CtPtrs in{};
  for (int u = 0; u < k; u++) {
    if (!cts_host[u]) return set_error(MICK_E_ARG, "NULL ciphertext pointer");
    in.p[u] = cts_host[u];
  }
  const bool fuse = tensor_takes_pass_b(k);
  if (fuse)
    MICK_TRY(launch_tensor_ib(prm, in, 0, k, level, w, 0, (long long)lay.D, (long long)lay.dcoef, 1,
                              own_keys(prm, keys), s));
  else
    MICK_TRY(launch_tensor(prm, in, 0, k, level, w + lay.D, 0, 1, s));
  return relin_rescale_ws(prm, keys, k, level, k - 1, w, lay.total, 1, ct_out_dev, 0, s, fuse);
}

int mick_mul_relin_rescale_noalloc(const mick_params* prm, const mick_keys* keys, const uint32_t* const* cts_host,
                                   int k, int level, uint32_t* ct_out_dev, void* stream) {
  MICK_TRY(check_mul(prm, keys, k, level));
  const size_t need = mick_workspace_bytes(prm, MICK_OP_MUL_RELIN_RESCALE, k, level);
  if (need > kScratchBytes)
    return set_error(MICK_E_WS, "this multiply needs " + std::to_string(need) +
                                    " bytes of workspace; the library's static workspace holds " +
                                    std::to_string(kScratchBytes));
  void* ws = nullptr;
  MICK_TRY(scratch_address(prm->device, &ws));
  return mick_mul_relin_rescale(prm, keys, cts_host, k, level, ct_out_dev, ws, kScratchBytes, stream);
}

size_t mick_batch_workspace_bytes(const mick_params* prm, int n_jobs, int k, int level) {
  if (n_jobs < 1 || n_jobs > kMaxJobs) return 0;
  return (size_t)n_jobs * mick_workspace_bytes(prm, MICK_OP_MUL_RELIN_RESCALE, k, level);
}

int mick_mul_relin_rescale_batch(const mick_params* prm, const mick_keys* keys, const uint32_t* cts_dev, int n_jobs,
                                 int k, int level, uint32_t* outs_dev, void* ws, size_t ws_bytes, void* stream) {
  MICK_TRY(check_mul(prm, keys, k, level));
  if (!cts_dev || !outs_dev || !ws) return set_error(MICK_E_ARG, "NULL argument");
  if (n_jobs < 1 || n_jobs > kMaxJobs) return set_error(MICK_E_ARG, "n_jobs must be in 1..64");
  if (ws_bytes < mick_batch_workspace_bytes(prm, n_jobs, k, level)) return set_error(MICK_E_WS, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const size_t N = prm->N;
  const Layout lay = mul_layout(prm, k, level);
  uint32_t* w = (uint32_t*)ws;
  CtPtrs in{};
  const size_t ct_elems = 2 * (size_t)level * N;
  for (int u = 0; u < k; u++) in.p[u] = cts_dev + (size_t)u * ct_elems;
  const bool fuse = tensor_takes_pass_b(k);
  if (fuse)
    MICK_TRY(launch_tensor_ib(prm, in, (long long)(k * ct_elems), k, level, w, (long long)lay.total,
                              (long long)lay.D, (long long)lay.dcoef, n_jobs, own_keys(prm, keys), s));
  else
    MICK_TRY(launch_tensor(prm, in, (long long)(k * ct_elems), k, level, w + lay.D, (long long)lay.total, n_jobs, s));
  const size_t out_job = 2 * (size_t)(level - k + 1) * N;
  return relin_rescale_ws(prm, keys, k, level, k - 1, w, lay.total, n_jobs, outs_dev, out_job, s, fuse);
}

int mick_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return MICK_OK;
}

int mick_profile_select(const char* sites) {
  static_assert(P_COUNT <= 32, "one mask bit per site");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!sites || !*sites) {
    g_prof_mask = ~0u;
    return MICK_OK;
  }
  uint32_t mask = 0;
  std::string all(sites);
  size_t pos = 0;
  while (pos <= all.size()) {
    const size_t end = std::min(all.find(',', pos), all.size());
    const std::string name = all.substr(pos, end - pos);
    int found = -1;
    for (int i = 0; i < P_COUNT; i++)
      if (name == kSiteNames[i]) found = i;
    if (found < 0) return set_error(MICK_E_ARG, "unknown profiling site: " + name);
    mask |= 1u << found;
    pos = end + 1;
  }
  g_prof_mask = mask;
  return MICK_OK;
}

int mick_profile_collect(int max, const char** names, double* total_ms, int* launches) {
  if (max < 0 || (max > 0 && (!names || !total_ms || !launches))) return set_error(MICK_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double ms[P_COUNT] = {0};
  int cnt[P_COUNT] = {0};
  for (auto& r : g_prof_records) {
    MICK_HIP(hipEventSynchronize(g_prof_events[r.second + 1]), "profile sync");
    float t = 0;
    MICK_HIP(hipEventElapsedTime(&t, g_prof_events[r.second], g_prof_events[r.second + 1]), "profile elapsed");
    ms[r.first] += t;
    cnt[r.first]++;
  }
  g_prof_records.clear();
  int n = 0;
  for (int i = 0; i < P_COUNT && n < max; i++) {
    if (!cnt[i]) continue;
    names[n] = kSiteNames[i];
    total_ms[n] = ms[i];
    launches[n] = cnt[i];
    n++;
  }
  return n;
}

}  // extern "C"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Blocks of one job in each stage's launch (see the job-table kernels).
void job_blocks(const mick_params* prm, int k, int level, int (&nb)[kStages]) {
  const int tiles = 1 << (prm->log_n - 13);
  const int E = level + prm->K, B = digits_at(prm, level);
  auto pad8 = [](int x) { return (x + 7) / 8 * 8; };
  nb[S_TENSOR] = pad8((prm->N >> tib_tile_log(k)) * level);  // k_tensor_ib_jt
  nb[S_INTT_D] = pad8(tiles * (k - 1) * level);
  nb[S_MODUP] = pad8((k - 1) * B * (1 << (prm->log_n - kModupTileLog))) *
                (modup_pairs_on(prm) ? modup_pairs(level, E) : E);
  nb[S_KIP] = pad8(E * (1 << (prm->log_n - kKipTileLog)));
  nb[S_INTT_ACC] = pad8(tiles * 2 * E);
  nb[S_MODDOWN] = pad8(2 * (prm->N / 256));
  nb[S_NTT_OUT] = pad8(tiles * 2 * (level - k + 1));
}

GroupConsts group_consts(const mick_params* prm, const mick_keys* keys) {
  GroupConsts G{};
  G.modup_tab = prm->d_modup;
  G.modup_off = prm->d_offsets;
  G.rs_tab = prm->d_rescale;
  G.rs_off = prm->d_offsets + prm->modup_off.size();
  G.dscale = prm->d_dscale;
  G.dscale_off = G.rs_off + prm->rescale_off.size();
  G.md = prm->d_moddown;
  G.evk = keys->d_evk;
  G.log_n = prm->log_n;
  G.L = prm->L;
  G.K = prm->K;
  G.dnum = prm->dnum;
  G.alpha = prm->alpha;
  return G;
}

}  // namespace

namespace mick {

namespace {
std::mutex g_alloc_mu;
Allocator g_alloc;
}  // namespace

Allocator current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}

int dev_alloc_bytes(const Allocator& a, void** p, size_t bytes) {
  *p = nullptr;
  if (a.alloc) {
    *p = a.alloc(bytes, a.ctx);
    if (!*p) return set_error(MICK_E_NOMEM, "registered allocator returned NULL");
    if (((uintptr_t)*p & 255) != 0) {
      a.release(*p, a.ctx);
      *p = nullptr;
      return set_error(MICK_E_NOMEM, "registered allocator returned a pointer not aligned to 256 bytes");
    }
    return MICK_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return set_error(MICK_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return MICK_OK;
}

void dev_free(const Allocator& a, void* p) {
  if (!p) return;
  if (a.release)
    a.release(p, a.ctx);
  else
    (void)hipFree(p);
}

size_t job_ws_bytes(const mick_params* prm, int k, int level) {
  return align_up(WsLayout(k, level, prm->K, prm->alpha, prm->log_n).total * 4);
}

size_t table_bytes(int n_jobs) { return align_up((size_t)n_jobs * sizeof(JobDesc)); }

int check_job(const mick_params* prm, const mick_keys* keys, const mick_job& jb) {
  MICK_TRY(check_mul(prm, keys, jb.k, jb.level));
  if (!jb.out) return set_error(MICK_E_ARG, "NULL output pointer");
  for (int u = 0; u < jb.k; u++)
    if (!jb.cts[u]) return set_error(MICK_E_ARG, "NULL ciphertext pointer");
  return MICK_OK;
}

int check_jobs(const mick_params* prm, const mick_keys* keys, const mick_job* jobs, int n_jobs) {
  for (int i = 0; i < n_jobs; i++) MICK_TRY(check_job(prm, keys, jobs[i]));
  return MICK_OK;
}

int plan_jobs(const mick_params* prm, const mick_keys* keys, const mick_job* jobs, int n_jobs,
              uint32_t* const* job_ws, JobDesc* table_dev, hipStream_t s, mick_plan** out) {
  std::unique_ptr<mick_plan> plan(new mick_plan());
  plan->prm = prm;
  plan->keys = keys;
  plan->table = table_dev;
  plan->n_jobs = n_jobs;
  // jobs of equal k are contiguous in the table (the tensor and rescale kernels
  // are specialised on k), and within a run sorted by level, descending (the
  // tensor launch's job-adjacent order, seg_block)
  std::vector<int> order(n_jobs);
  for (int i = 0; i < n_jobs; i++) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return jobs[a].k != jobs[b].k ? jobs[a].k < jobs[b].k : jobs[a].level > jobs[b].level;
  });
  std::vector<JobDesc>& jt = plan->host_table;
  jt.assign(n_jobs, JobDesc{});
  int total[kStages] = {0};
  for (int r = 0; r < n_jobs; r++) {
    const mick_job& jb = jobs[order[r]];
    JobDesc& d = jt[r];
    memset(&d, 0, sizeof(d));
    for (int u = 0; u < jb.k; u++) d.in[u] = jb.cts[u];
    d.out = jb.out;
    d.ws = job_ws[order[r]];
    d.k = jb.k;
    d.level = jb.level;
    int nb[kStages];
    job_blocks(prm, jb.k, jb.level, nb);
    for (int st = 0; st < kStages; st++) {
      // tensor and rescale launches restart at each run of equal k
      const bool per_k = st == S_TENSOR || st == S_MODDOWN;
      if (per_k && r > 0 && jt[r - 1].k != jb.k) {
        if (st == S_TENSOR) plan->runs.push_back({r, 0, 0, 0});
        total[st] = 0;
      }
      if (per_k && r == 0 && st == S_TENSOR) plan->runs.push_back({0, 0, 0, 0});
      d.blk0[st] = total[st];
      total[st] += nb[st];
    }
    auto& run = plan->runs.back();
    run.k = jb.k;
    run.tensor_blocks = total[S_TENSOR];
    run.moddown_blocks = total[S_MODDOWN];
  }
  for (int st = 0; st < kStages; st++) plan->blocks[st] = total[st];
  // job-adjacent block orders (seg_block): the segment bases from the last
  // rank up
  auto segments = [&](int order, int r0, int r1) {
    jt[r1 - 1].seg[order].base = 0;
    for (int r = r1 - 2; r >= r0; r--) {
      const int i = r - r0;  // rank i + 1's segment: groups [G(i + 2), G(i + 1)), i + 2 ranks each
      const int g_next = r + 2 < r1 ? jt[r + 2].seg[order].groups : 0;
      jt[r].seg[order].base = jt[r + 1].seg[order].base + (jt[r + 1].seg[order].groups - g_next) * (i + 2);
    }
  };
  // [0] each run's tensor launch: the run is already in rank order
  for (size_t ri = 0; ri < plan->runs.size(); ri++) {
    const int j0 = plan->runs[ri].j0;
    const int j1 = ri + 1 < plan->runs.size() ? plan->runs[ri + 1].j0 : n_jobs;
    for (int r = j0; r < j1; r++) {
      int nb[kStages];
      job_blocks(prm, jt[r].k, jt[r].level, nb);
      jt[r].seg[0] = {r, nb[S_TENSOR] / 8, 0};
    }
    segments(0, j0, j1);
  }
  // [1] the key-product launch over the table: ranks by level, descending
  if (n_jobs > 0) {
    std::vector<int> rank(n_jobs);
    for (int r = 0; r < n_jobs; r++) rank[r] = r;
    std::stable_sort(rank.begin(), rank.end(), [&](int a, int b) { return jt[a].level > jt[b].level; });
    for (int r = 0; r < n_jobs; r++) {
      int nb[kStages];
      job_blocks(prm, jt[rank[r]].k, jt[rank[r]].level, nb);
      jt[r].seg[1] = {rank[r], nb[S_KIP] / 8, 0};
    }
    segments(1, 0, n_jobs);
  }
  if (n_jobs > 0)
    MICK_HIP(hipMemcpyAsync(table_dev, jt.data(), n_jobs * sizeof(JobDesc), hipMemcpyHostToDevice, s), "job table");
  *out = plan.release();
  return MICK_OK;
}

}  // namespace mick

extern "C" {

int mick_set_allocator(mick_alloc_fn alloc, mick_free_fn release, void* ctx) {
  if ((alloc == nullptr) != (release == nullptr)) return set_error(MICK_E_ARG, "give both functions or neither");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc.alloc = alloc;
  g_alloc.release = release;
  g_alloc.ctx = alloc ? ctx : nullptr;
  return MICK_OK;
}

size_t mick_jobs_workspace_bytes(const mick_params* prm, const mick_job* jobs, int n_jobs) {
  if (!prm || !jobs || n_jobs < 1) return 0;
  size_t total = table_bytes(n_jobs);
  for (int i = 0; i < n_jobs; i++) {
    const int k = jobs[i].k, level = jobs[i].level;
    if (k < 2 || k > kMaxK || level < k || level > prm->L) {
      if (jobs[i].status) continue;  // left out of the batch
      return 0;
    }
    total += job_ws_bytes(prm, k, level);
  }
  return total;
}

int mick_jobs_plan(const mick_params* prm, const mick_keys* keys, const mick_job* jobs, int n_jobs, void* ws,
                   size_t ws_bytes, void* stream, mick_plan** out) {
  if (!out) return set_error(MICK_E_ARG, "NULL out");
  *out = nullptr;
  if (!prm || !keys || !jobs || !ws) return set_error(MICK_E_ARG, "NULL argument");
  if (keys->prm != prm) return set_error(MICK_E_ARG, "keys belong to other params");
  if (n_jobs < 1 || n_jobs > 65536) return set_error(MICK_E_ARG, "n_jobs must be in 1..65536");
  // every job is checked before anything is written: a job with a status
  // word that fails is left out, one without fails the call
  std::vector<int> st(n_jobs, MICK_OK);
  std::string first_error;
  for (int i = 0; i < n_jobs; i++) {
    st[i] = check_job(prm, keys, jobs[i]);
    if (st[i] != MICK_OK && !jobs[i].status) return st[i];
    if (st[i] != MICK_OK && first_error.empty()) first_error = mick_last_error();
  }
  std::vector<mick_job> valid;
  valid.reserve(n_jobs);
  for (int i = 0; i < n_jobs; i++)
    if (st[i] == MICK_OK) valid.push_back(jobs[i]);
  const int nv = (int)valid.size();
  // table (sized for every job) first, then the valid jobs' workspaces
  size_t off = table_bytes(n_jobs), need = off;
  for (const mick_job& jb : valid) need += job_ws_bytes(prm, jb.k, jb.level);
  if (ws_bytes < need) return set_error(MICK_E_WS, "workspace too small");
  std::vector<uint32_t*> job_ws(nv);
  char* base = (char*)ws;
  for (int i = 0; i < nv; i++) {
    job_ws[i] = (uint32_t*)(base + off);
    off += job_ws_bytes(prm, valid[i].k, valid[i].level);
  }
  MICK_TRY(plan_jobs(prm, keys, valid.data(), nv, job_ws.data(), (JobDesc*)ws, (hipStream_t)stream, out));
  for (int i = 0; i < n_jobs; i++)
    if (jobs[i].status) *jobs[i].status = st[i];
  if (!first_error.empty()) set_error(MICK_OK, first_error);  // detail of the first refused job
  return MICK_OK;
}

int mick_plan_execute(const mick_plan* plan, void* stream) {
  if (!plan) return set_error(MICK_E_ARG, "NULL plan");
  hipStream_t s = (hipStream_t)stream;
  const mick_params* prm = plan->prm;
  const JobDesc* djt = plan->table;
  const int n = plan->n_jobs;
  if (n == 0) return MICK_OK;  // every job was refused
  const GroupConsts G = group_consts(prm, plan->keys);
  for (size_t i = 0; i < plan->runs.size(); i++) {
    const auto& r = plan->runs[i];
    const int j1 = i + 1 < plan->runs.size() ? plan->runs[i + 1].j0 : n;
    MICK_TRY(launch_tensor_ib_jt(prm, djt, r.j0, j1 - r.j0, r.k, r.tensor_blocks, own_keys(prm, plan->keys),
                                 s));
  }
  MICK_TRY(launch_ntt_jt(prm, djt, n, S_INTT_D, plan->blocks[S_INTT_D], G, s));
  MICK_TRY(launch_modup_a_jt(prm, djt, n, plan->blocks[S_MODUP], G, s));
  MICK_TRY(launch_kip_b_jt(prm, djt, n, plan->blocks[S_KIP], G, s));
  MICK_TRY(launch_ntt_jt(prm, djt, n, S_INTT_ACC, plan->blocks[S_INTT_ACC], G, s));
  for (size_t i = 0; i < plan->runs.size(); i++) {
    const auto& r = plan->runs[i];
    const int j1 = i + 1 < plan->runs.size() ? plan->runs[i + 1].j0 : n;
    MICK_TRY(launch_moddown_rs_jt(prm, djt, r.j0, j1 - r.j0, r.k - 1, r.moddown_blocks, G, s));
  }
  return launch_ntt_jt(prm, djt, n, S_NTT_OUT, plan->blocks[S_NTT_OUT], G, s);
}

void mick_plan_destroy(mick_plan* plan) { delete plan; }

namespace {
void destroy_plan_cb(void* plan) { mick_plan_destroy(static_cast<mick_plan*>(plan)); }
}  // namespace

int mick_mul_relin_rescale_jobs(const mick_params* prm, const mick_keys* keys, const mick_job* jobs, int n_jobs,
                                void* ws, size_t ws_bytes, void* stream) {
  // this call frees its plan from a host function on the stream, which a
  // graph would replay: capture takes mick_jobs_plan + mick_plan_execute
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  MICK_HIP(hipStreamIsCapturing((hipStream_t)stream, &cap), "capture status");
  if (cap != hipStreamCaptureStatusNone)
    return set_error(MICK_E_ARG, "stream is capturing: plan with mick_jobs_plan and capture mick_plan_execute");
  mick_plan* plan = nullptr;
  MICK_TRY(mick_jobs_plan(prm, keys, jobs, n_jobs, ws, ws_bytes, stream, &plan));
  const int st = mick_plan_execute(plan, stream);
  // the plan holds the source of the table copy: free it once the stream
  // has passed that copy (a host function queued behind the launches), or
  // after a synchronisation if no host function can be queued
  if (hipLaunchHostFunc((hipStream_t)stream, destroy_plan_cb, plan) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize((hipStream_t)stream);
    mick_plan_destroy(plan);
  }
  return st;
}

int mick_output_scale(const mick_params* prm, const double* scales_host, int k, int level, double* out_host) {
  if (!prm || !scales_host || !out_host) return set_error(MICK_E_ARG, "NULL argument");
  if (k < 2 || k > kMaxK) return set_error(MICK_E_ARG, "k must be in 2..12");
  if (level < k || level > prm->L) return set_error(MICK_E_LEVEL, "level must be in k..L");
  double sc = 1.0;
  for (int u = 0; u < k; u++) sc *= scales_host[u];
  for (int t = level - k + 1; t < level; t++) sc /= (double)prm->q[t];
  *out_host = sc;
  return MICK_OK;
}

int mick_ntt(const mick_params* prm, uint32_t* data_dev, int n_limbs, int first_prime, int inverse, void* stream) {
  if (!prm || !data_dev) return set_error(MICK_E_ARG, "NULL argument");
  if (n_limbs < 1 || first_prime < 0 || first_prime + n_limbs > prm->L + prm->K)
    return set_error(MICK_E_ARG, "limb range outside the prime set");
  return ntt_launch(prm, data_dev, data_dev, simple_map(prm, first_prime, n_limbs), n_limbs, 1, inverse != 0,
                    (hipStream_t)stream);
}

}  // extern "C"
