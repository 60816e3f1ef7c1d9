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

// The ModUp kernels convert into two targets per workgroup for digits of 5
// to 8 primes (one source load feeds both); wider digits leave no registers
// for a second target, and narrower ones read too few source rows to gain.
inline bool modup_two_targets(int alpha) { return modup_rows(alpha) == 8; }
// Whether a parameter set's ModUp launches take two targets per workgroup:
// digits of 5 to 8 primes, unless set to one target (mick_params_set_modup_targets).
inline bool modup_pairs_on(const mick_params* prm) {
  return modup_two_targets(prm->alpha) && prm->modup_targets == 2;
}

// Workgroups per source tile of the two-target kernel: ceil(level / 2) +
// ceil(K / 2), an upper bound on the pairs of q targets plus the pairs of
// special primes.
__host__ __device__ inline int modup_pairs(int level, int E) { return (level + 1) / 2 + (E - level + 1) / 2; }

struct CtPtrs {
  const uint32_t* p[kMaxK];
};

// eq. (d_u formula for n-ct mult): prod_u (c0^u + c1^u Y) = sum_t d_t Y^t for
// four consecutive residues (uint4 index n) of limb j, built one factor at a
// time.  Every partial product picks up one R^-1 per factor, removed at the
// end by R^(K-1); P[t] = d_t, canonical.  The two products of canonical
// residues in a step are summed exactly (below 2 m^2 < m 2^32) and reduced
// once: the same residue, with the same factor R^-1, as two Montgomery
// products and a modular add.
template <int K>
__device__ __forceinline__ void tensor4(const uint32_t* const (&inp)[K], int level, int log_n, int j, size_t n,
                                        const DevTables& T, uint4 (&P)[K + 1]) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t m = T.mod[j], minv = T.minv[j];
  const size_t limb = (size_t)j * N;
  const size_t poly = (size_t)level * N;
  P[0] = reinterpret_cast<const uint4*>(inp[0] + limb)[n];
  P[1] = reinterpret_cast<const uint4*>(inp[0] + poly + limb)[n];
#pragma unroll
  for (int u = 1; u < K; u++) {
    const uint4 a = reinterpret_cast<const uint4*>(inp[u] + limb)[n];
    const uint4 b = reinterpret_cast<const uint4*>(inp[u] + poly + limb)[n];
    // new_t = P_t a + P_{t-1} b, t = u+1 .. 0 (descending keeps P_{t-1} intact)
    P[u + 1].x = mont_mul(P[u].x, b.x, m, minv);
    P[u + 1].y = mont_mul(P[u].y, b.y, m, minv);
    P[u + 1].z = mont_mul(P[u].z, b.z, m, minv);
    P[u + 1].w = mont_mul(P[u].w, b.w, m, minv);
#pragma unroll
    for (int t = u; t >= 1; t--) {
      P[t].x = redc((uint64_t)P[t].x * a.x + (uint64_t)P[t - 1].x * b.x, m, minv);
      P[t].y = redc((uint64_t)P[t].y * a.y + (uint64_t)P[t - 1].y * b.y, m, minv);
      P[t].z = redc((uint64_t)P[t].z * a.z + (uint64_t)P[t - 1].z * b.z, m, minv);
      P[t].w = redc((uint64_t)P[t].w * a.w + (uint64_t)P[t - 1].w * b.w, m, minv);
    }
    P[0].x = mont_mul(P[0].x, a.x, m, minv);
    P[0].y = mont_mul(P[0].y, a.y, m, minv);
    P[0].z = mont_mul(P[0].z, a.z, m, minv);
    P[0].w = mont_mul(P[0].w, a.w, m, minv);
  }
  const uint32_t* rp = T.rpow + (size_t)j * 2 * (kMaxK + 1);
  const uint32_t f = rp[2 * (K - 1)], fsh = rp[2 * (K - 1) + 1];
#pragma unroll
  for (int t = 0; t <= K; t++) {
    P[t].x = shoup(P[t].x, f, fsh, m);
    P[t].y = shoup(P[t].y, f, fsh, m);
    P[t].z = shoup(P[t].z, f, fsh, m);
    P[t].w = shoup(P[t].w, f, fsh, m);
  }
}

// Ways of forming d_0..d_k (all give the same canonical residues):
//  kTensorChain  one linear factor at a time (tensor4);
//  kTensorTree   a balanced binary tree of products of polynomials in Y, each
//                node's coefficients exact 64-bit sums of products reduced
//                once (Montgomery);
//  kTensorFilter the same tree with the fast filtering forms of Sec. II and
//                Sec. V-A at its nodes: Karatsuba for two linear factors and
//                for two cubics (two levels), the 3-parallel fast filter for
//                two quadratics, schoolbook sums elsewhere.
enum TensorMethod { kTensorChain = 0, kTensorTree = 1, kTensorFilter = 2, kTensorMethods = 3 };

// Montgomery reduction of a sum of `terms` products of canonical residues
// below m < 2^30: below 4 m^2 < m 2^32 for up to four terms, below 8 m^2 <
// 2 m 2^32 for up to eight.
template <int TERMS>
__device__ __forceinline__ uint32_t redc_terms(uint64_t t, uint32_t m, uint32_t minv) {
  static_assert(TERMS >= 1 && TERMS <= 8, "at most eight products per sum");
  if constexpr (TERMS <= 4)
    return redc(t, m, minv);
  else
    return redc_2m(t, m, minv);
}

__device__ __forceinline__ uint64_t mul64(uint32_t a, uint32_t b) { return (uint64_t)a * b; }

// C = A B for polynomials in Y with canonical coefficients below m < 2^30;
// every coefficient of C is the exact sum of its products, reduced once, so
// it carries one factor R^-1.
template <int NA, int NB, bool FF>
__device__ __forceinline__ void poly_mul(const uint32_t (&A)[NA], const uint32_t (&B)[NB],
                                         uint32_t (&C)[NA + NB - 1], uint32_t m, uint32_t minv) {
  if constexpr (FF && NA == 2 && NB == 2) {
    // Karatsuba: a0 b1 + a1 b0 = (a0 + a1)(b0 + b1) - a0 b0 - a1 b1
    const uint64_t lo = mul64(A[0], B[0]), hi = mul64(A[1], B[1]);
    const uint64_t mid = mul64(A[0] + A[1], B[0] + B[1]) - lo - hi;
    C[0] = redc_terms<1>(lo, m, minv);
    C[1] = redc_terms<2>(mid, m, minv);
    C[2] = redc_terms<1>(hi, m, minv);
  } else if constexpr (FF && NA == 3 && NB == 3) {
    // 3-parallel fast filter: six products for the nine of the schoolbook form
    const uint64_t p0 = mul64(A[0], B[0]), p1 = mul64(A[1], B[1]), p2 = mul64(A[2], B[2]);
    const uint64_t p01 = mul64(A[0] + A[1], B[0] + B[1]);
    const uint64_t p12 = mul64(A[1] + A[2], B[1] + B[2]);
    const uint64_t p012 = mul64(A[0] + A[1] + A[2], B[0] + B[1] + B[2]);  // < 9 m^2
    C[0] = redc_terms<1>(p0, m, minv);
    C[1] = redc_terms<2>(p01 - p0 - p1, m, minv);
    C[2] = redc_terms<3>(p012 + 2 * p1 - p01 - p12, m, minv);  // a0 b2 + a1 b1 + a2 b0
    C[3] = redc_terms<2>(p12 - p1 - p2, m, minv);
    C[4] = redc_terms<1>(p2, m, minv);
  } else if constexpr (FF && NA == 4 && NB == 4) {
    // Karatsuba on halves A = A0 + Y^2 A1, B = B0 + Y^2 B1, each half product
    // itself by Karatsuba, all in exact 64-bit sums: A0 B0, A1 B1 and
    // (A0 + A1)(B0 + B1) (sums of halves below 2m, their sums below 4m)
    uint64_t lo[3], hi[3], md[3];
    auto kara = [](uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1, uint64_t (&r)[3]) {
      r[0] = mul64(a0, b0);
      r[2] = mul64(a1, b1);
      r[1] = mul64(a0 + a1, b0 + b1) - r[0] - r[2];
    };
    kara(A[0], A[1], B[0], B[1], lo);
    kara(A[2], A[3], B[2], B[3], hi);
    kara(A[0] + A[2], A[1] + A[3], B[0] + B[2], B[1] + B[3], md);
    for (int i = 0; i < 3; i++) md[i] -= lo[i] + hi[i];
    C[0] = redc_terms<1>(lo[0], m, minv);
    C[1] = redc_terms<2>(lo[1], m, minv);
    C[2] = redc_terms<3>(lo[2] + md[0], m, minv);
    C[3] = redc_terms<4>(md[1], m, minv);
    C[4] = redc_terms<3>(md[2] + hi[0], m, minv);
    C[5] = redc_terms<2>(hi[1], m, minv);
    C[6] = redc_terms<1>(hi[2], m, minv);
  } else {
#pragma unroll
    for (int t = 0; t < NA + NB - 1; t++) {
      constexpr int kMin = NA < NB ? NA : NB;
      uint64_t acc = 0;
#pragma unroll
      for (int i = 0; i < NA; i++)
        if (t - i >= 0 && t - i < NB) acc += mul64(A[i], B[t - i]);
      C[t] = redc_terms<kMin>(acc, m, minv);
    }
  }
}

// prod_{u in [U0, U1)} (c0^u + c1^u Y) by a balanced binary tree: the left
// half of the factors times the right half, recursively.  Every internal
// node adds one factor R^-1, so the root carries R^-(U1 - U0 - 1).
template <int U0, int U1, bool FF>
struct TensorTree {
  static constexpr int N = U1 - U0;
  static constexpr int H = (N + 1) / 2;
  template <int K>
  __device__ static void run(const uint32_t (&a)[K], const uint32_t (&b)[K], uint32_t (&P)[N + 1], uint32_t m,
                             uint32_t minv) {
    if constexpr (N == 1) {
      P[0] = a[U0];
      P[1] = b[U0];
    } else {
      uint32_t L[H + 1], R[N - H + 1];
      TensorTree<U0, U0 + H, FF>::run(a, b, L, m, minv);
      TensorTree<U0 + H, U1, FF>::run(a, b, R, m, minv);
      poly_mul<H + 1, N - H + 1, FF>(L, R, P, m, minv);
    }
  }
};

// The tensor product of tensor4 by the product tree (FF: fast filtering
// nodes); same inputs, same canonical outputs.
template <int K, bool FF>
__device__ __forceinline__ void tensor4_tree(const uint32_t* const (&inp)[K], int level, int log_n, int j, size_t n,
                                             const DevTables& T, uint4 (&P)[K + 1]) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t m = T.mod[j], minv = T.minv[j];
  const size_t limb = (size_t)j * N;
  const size_t poly = (size_t)level * N;
  uint4 a4[K], b4[K];
#pragma unroll
  for (int u = 0; u < K; u++) {
    a4[u] = reinterpret_cast<const uint4*>(inp[u] + limb)[n];
    b4[u] = reinterpret_cast<const uint4*>(inp[u] + poly + limb)[n];
  }
  const uint32_t* rp = T.rpow + (size_t)j * 2 * (kMaxK + 1);
  const uint32_t f = rp[2 * (K - 1)], fsh = rp[2 * (K - 1) + 1];
  uint32_t a[K], b[K], r[K + 1];
#define MICK_TREE_LANE(C)                                        \
  for (int u = 0; u < K; u++) {                                  \
    a[u] = a4[u].C;                                              \
    b[u] = b4[u].C;                                              \
  }                                                              \
  TensorTree<0, K, FF>::run(a, b, r, m, minv);                   \
  for (int t = 0; t <= K; t++) P[t].C = shoup(r[t], f, fsh, m);
  MICK_TREE_LANE(x)
  MICK_TREE_LANE(y)
  MICK_TREE_LANE(z)
  MICK_TREE_LANE(w)
#undef MICK_TREE_LANE
}

template <int K, int TM>
__device__ __forceinline__ void tensor4_by(const uint32_t* const (&inp)[K], int level, int log_n, int j, size_t n,
                                           const DevTables& T, uint4 (&P)[K + 1]) {
  if constexpr (TM == kTensorChain)
    tensor4<K>(inp, level, log_n, j, n, T, P);
  else
    tensor4_tree<K, TM == kTensorFilter>(inp, level, log_n, j, n, T, P);
}

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
  // 1: the tensor kernel has summed each q limb's own-digit key products
  // and d_0, d_1 (OwnKeys) into D's slots 0 and 1; those pairs are skipped
  // here and D is not added at the end
  int own_sums;
};

// The evaluation keys as the fused tensor kernel reads them for the own
// digit of each q limb (evk == nullptr: d_0..d_k are written instead).
struct OwnKeys {
  const uint32_t* evk;
  int dnum, alpha;
  long long key_poly;  // elements per key polynomial ((L+K) N)
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
// Tensor product of n_jobs same-shape multiplies fused with pass B of the
// INTT of d_2..d_k: D (all k + 1 polynomials) at ws + d_off and the pass-B
// outputs at ws + dc_off, per job ws_job words apart.  At N = 2^16, k = 8,
// batch 8: tensor 0.36 ms + pass B 0.29 ms -> 0.55 ms.  Every k takes it
// now (tile sizes by k, tib_tile_log); the predicate is the one switch
// between it and the plain tensor launch + two-pass INTT in the fused
// multiply.
inline bool tensor_takes_pass_b(int k) { return k >= 2; }

// Residues per tile of the fused kernel (log2): 1024 from k = 5; 2048 for
// k = 3, 4 and 4096 for k = 2, so that the k - 1 tiles' pass-B items (64 per
// 1024 residues at 256 rows per block) still cover a workgroup's 256 threads.
__host__ __device__ constexpr int tib_tile_log(int k) { return k >= 5 ? 10 : (k >= 3 ? 11 : 12); }

// Job-table form: jobs [j0, j0 + nj) of equal k, blocks as job_blocks counts
// them; every job of a table takes it (the table's INTT of d_2..d_k then
// runs its pass A only).  With own.evk set both forms write the own-digit
// sums (with d_0, d_1 folded in) into D's slots 0 and 1 in place of d_0..d_k.
int launch_tensor_ib_jt(const mick_params* prm, const JobDesc* jt, int j0, int nj, int k, int blocks,
                        const OwnKeys& own, hipStream_t s);
int launch_tensor_ib(const mick_params* prm, const CtPtrs& in, long long in_job_stride, int k, int level,
                     uint32_t* ws, long long ws_job, long long d_off, long long dc_off, int n_jobs,
                     const OwnKeys& own, hipStream_t s);
int launch_kip_b(const mick_params* prm, const uint32_t* X, const uint32_t* D, const uint32_t* evk, uint32_t* acc,
                 KipArgs A, hipStream_t s);
int launch_moddown_rs(const mick_params* prm, const uint32_t* acc, uint32_t* out, const MdArgs& A, int mu, int n_jobs,
                      hipStream_t s);
// Job-table forms (heterogeneous batches): jobs [j0, j0 + nj) of the table,
// all with the given k (mu = k - 1); `blocks` covers their block ranges.
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
