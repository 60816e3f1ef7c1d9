// Launch arguments and launchers of the pointwise RNS kernels.
#pragma once
#include "internal.h"

namespace mick {

constexpr int kMaxAlpha = 32;  // primes per key-switching digit
constexpr int kMaxKp = 24;     // special primes p_i

// Rows of a digit's conversion table as the ModUp kernel reads them: the
// digit width rounded up to 1, 2, 4, 8, 16, 24 or 32 (padded rows are zero).
inline int modup_rows(int alpha) {
  if (alpha > 8) return (alpha + 7) / 8 * 8;
  int r = 1;
  while (r < alpha) r <<= 1;
  return r;
}

// The same-shape ModUp launch converts into two targets per workgroup for
// digits of 5 to 8 primes (one source load feeds both); wider digits leave
// no registers for a second target, and narrower ones read too few source
// rows to gain.
inline bool modup_two_targets(int alpha) { return modup_rows(alpha) == 8; }

// Workgroups per source tile of the two-target kernel: ceil(level / 2) +
// ceil(K / 2), an upper bound on the pairs of q targets plus the pairs of
// special primes.
__host__ __device__ inline int modup_pairs(int level, int E) { return (level + 1) / 2 + (E - level + 1) / 2; }

struct CtPtrs {
  const uint32_t* p[kMaxK];
};

struct ModupArgs {
  const uint32_t* tab;  // ModUp tables
  int tab_off[16];      // per digit offset of this level's table inside `tab`
  int log_n, level, L, E, B, alpha;
  int groups;           // (k - 1) B source groups per job
  int tiles, units;     // set by the launcher
  long long dcoef_job, x_job;
};

struct KipArgs {
  int log_n, level, L, E, B, alpha, dnum, k, n_jobs;
  int tiles;           // set by the launcher
  long long key_poly;  // elements per key polynomial ((L+K) N)
  long long d_job, x_job, acc_job;
};

struct MdArgs {
  const uint32_t* md;     // [K][2] phat_i^-1 (+Shoup), then [K][L] p_i^-1 mod q_j
  const uint32_t* qinvq;  // [L][L][2] q_d^-1 mod q_t (+Shoup)
  const uint32_t* rs;     // (level, mu) block: [top][2] g^{mu,l-1}_eta (+Shoup), [top][mu] g^{mu,t}_eta
  int log_n, level, L, K, E;
  long long acc_job, out_job;
};

int launch_tensor(const mick_params* prm, const CtPtrs& in, long long in_job_stride, int k, int level, uint32_t* D,
                  long long d_job_stride, int n_jobs, hipStream_t s);
// ModUp basis conversion fused with pass A of the forward transform of the
// new limbs (ntt.hip).  dsc: the d_t limbs in the coefficient domain, each
// already multiplied by its qhat_j^-1.
int launch_modup_a(const mick_params* prm, const uint32_t* dsc, uint32_t* X, ModupArgs A, int n_jobs, hipStream_t s);
// Pass B of those transforms fused with the key inner product, followed by
// the first pass (pass B) of the accumulators' inverse transform; acc holds
// that pass's output (ntt.hip).
int launch_kip_b(const mick_params* prm, const uint32_t* X, const uint32_t* D, const uint32_t* evk, uint32_t* acc,
                 KipArgs A, hipStream_t s);
int launch_moddown_rs(const mick_params* prm, const uint32_t* acc, uint32_t* out, const MdArgs& A, int mu, int n_jobs,
                      hipStream_t s);
// Job-table forms (heterogeneous batches): jobs [j0, j0 + nj) of the table,
// all with the given k (mu = k - 1); `blocks` covers their block ranges.
int launch_tensor_jt(const mick_params* prm, const JobDesc* jt, int j0, int nj, int k, int blocks, hipStream_t s);
int launch_moddown_rs_jt(const mick_params* prm, const JobDesc* jt, int j0, int nj, int mu, int blocks,
                         const GroupConsts& G, hipStream_t s);
int launch_ntt_jt(const mick_params* prm, const JobDesc* jt, int nj, int stage, int blocks, const GroupConsts& G,
                  hipStream_t s);
int launch_modup_a_jt(const mick_params* prm, const JobDesc* jt, int nj, int blocks, const GroupConsts& G,
                      hipStream_t s);
int launch_kip_b_jt(const mick_params* prm, const JobDesc* jt, int nj, int blocks, const GroupConsts& G,
                    hipStream_t s);

// Algorithm 1 steps 2-3 over `polys` polynomials ([polys][...] layouts).
int launch_rs_sums(const mick_params* prm, const uint32_t* topc, uint32_t* bout, const MdArgs& A, int mu, int polys,
                   hipStream_t s);
int launch_rs_combine(const mick_params* prm, const uint32_t* Ain, const uint32_t* Bn, uint32_t* out, const MdArgs& A,
                      int mu, int polys, hipStream_t s);
// Algorithm 1 on polys NTT-domain polynomials (api.hip); ws: polys level N words.
int rescale_polys(const mick_params* prm, const uint32_t* in, int polys, int level, int mu, uint32_t* out,
                  uint32_t* ws, hipStream_t s);
int launch_pk(const mick_params* prm, const uint32_t* E, const uint32_t* a, const uint32_t* S, uint32_t* b,
              hipStream_t s);
int launch_mul_rows(const mick_params* prm, uint32_t* X, const uint32_t* Y, int rows, hipStream_t s);
int launch_evk(const mick_params* prm, const uint32_t* E, const uint32_t* a, const uint32_t* S, const uint32_t* St,
               uint32_t* k0, uint32_t* k1, const uint32_t* rowc, hipStream_t s);
int launch_enc(const mick_params* prm, const uint32_t* V, const uint32_t* M0, const uint32_t* E1, const uint32_t* pk,
               uint32_t* ct, int level, hipStream_t s);
int launch_dec(const mick_params* prm, const uint32_t* ct, const uint32_t* S, uint32_t* X, int level, hipStream_t s);

}  // namespace mick
