// Pointwise RNS kernels of the k-input multiply: tensor product, relocated
// ModDown fused with the combined multi-level rescale, the steps of
// Algorithm 1, and the small pointwise operations of key generation,
// encryption and decryption.  (The ModUp basis conversion and the key inner
// product are fused into transform passes in ntt.hip.)
#include "internal.h"
#include "rns.h"

namespace mick {

namespace {

constexpr int kThreads = 256;

// a * b mod m for two variables: two Montgomery products, the second by
// R^2 mod m, remove both R^-1 factors.
__device__ __forceinline__ uint32_t mul_var(uint32_t a, uint32_t b, uint32_t m, uint32_t minv, uint32_t r2) {
  return mont_mul(mont_mul(a, b, m, minv), r2, m, minv);
}

// ------------------------------------------------------------------ tensor
// The k + 1 limbs j of D at residues 4n .. 4n + 3 (tensor4).
template <int K>
__device__ __forceinline__ void tensor_body(const uint32_t* const (&inp)[K], int level, int log_n, uint32_t* D, int j,
                                            size_t n, const DevTables& T) {
  uint4 P[K + 1];
  tensor4<K>(inp, level, log_n, j, n, T, P);
  const size_t N = (size_t)1 << log_n;
  uint32_t* out = D + (size_t)j * N;
#pragma unroll
  for (int t = 0; t <= K; t++) reinterpret_cast<uint4*>(out + (size_t)t * level * N)[n] = P[t];
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_tensor(CtPtrs in, long long in_job_stride, int level, int log_n,
                                                     uint32_t* D, long long d_job_stride, DevTables T) {
  const size_t job_in = (size_t)blockIdx.z * (size_t)in_job_stride;
  const uint32_t* inp[K];
#pragma unroll
  for (int u = 0; u < K; u++) inp[u] = in.p[u] + job_in;
  tensor_body<K>(inp, level, log_n, D + (size_t)blockIdx.z * (size_t)d_job_stride, blockIdx.y,
                 (size_t)blockIdx.x * kThreads + threadIdx.x, T);
}

// ------------------------------------------------------------------ ModDown + multi-rescale
// Input: acc after the INTT, coefficient domain: rows q_0..q_{l-1} hold
// INTT(D + P^-1 C~) (eq. (moddown improved 2)), rows p_i hold INTT(C~^(p)).
// c*_j = row_j - scBConv(p rows)_j (eq. (scBconv)), then mu rescalings by
// eq. (multi rs): the dropped limbs run the chain of Algorithm 1 step 2,
// every kept limb eta takes g^{mu,l-1}_eta c*_eta - sum_t g^{mu,t}_eta a_t.
// Output coefficient domain, limbs 0..l-mu-1 (the final NTT follows).
// Constants of one launch staged in LDS (every thread reads them with
// uniform addresses): phat_i^-1 (+Shoup) [K][2], p_i^-1 mod q_j [K][level],
// the chain's q_d^-1 mod q_t (+Shoup) [MU][MU][2], g^{mu,l-1}_eta (+Shoup)
// [top][2] and g^{mu,t}_eta [top][MU].
// KP: special primes the kernel is built for (8 or 24; rows beyond K are zero).
template <int KP>
constexpr int md_lds_words() { return 2 * KP + KP * 60 + 2 * 12 * 12 + 2 * 60 + 60 * 12; }

// Loads up to IT x kThreads words: v[it] = get(i) for i = it kThreads + tid < n.
template <int IT, typename Get>
__device__ __forceinline__ void gather_words(uint32_t (&v)[IT], int n, Get get) {
#pragma unroll
  for (int it = 0; it < IT; it++) {
    const int i = it * kThreads + threadIdx.x;
    if (i < n) v[it] = get(i);
  }
}

template <int IT>
__device__ __forceinline__ void put_words(const uint32_t (&v)[IT], int n, uint32_t* dst) {
#pragma unroll
  for (int it = 0; it < IT; it++) {
    const int i = it * kThreads + threadIdx.x;
    if (i < n) dst[i] = v[it];
  }
}

// Stages the ModDown and rescale constants in LDS.  Every load is issued
// before the first LDS store, so staging costs one memory latency.
template <int MU, int KP>
__device__ __forceinline__ void moddown_stage(const MdArgs& A, uint32_t* c) {
  constexpr int M1 = MU > 0 ? MU : 1;
  const int top = A.level - MU;
  uint32_t* phinv = c;
  uint32_t* pinvq = phinv + 2 * KP;
  uint32_t* chain = pinvq + KP * 60;
  uint32_t* gtop = chain + 2 * 12 * 12;
  uint32_t* gt = gtop + 2 * 60;
  // rows i >= K are zero, so the loops over the special primes need no bounds
  uint32_t vph[1], vpi[(KP * 60 + kThreads - 1) / kThreads], vch[2], vgtop[1], vgt[(60 * M1 + kThreads - 1) / kThreads];
  gather_words(vph, 2 * KP, [&](int i) { return i < 2 * A.K ? A.md[i] : 0u; });
  gather_words(vpi, KP * A.level, [&](int i) {
    const int pi = i / A.level, j = i - pi * A.level;
    return pi < A.K ? A.md[2 * A.K + (size_t)pi * A.L + j] : 0u;
  });
  // chain: rescale u drops q_{l-u}; entry (u, t) is q_{l-u}^-1 mod q_{top+t}
  // (+Shoup), for u >= 1 and t < MU - u
  auto chain_src = [&](int i) -> const uint32_t* {
    const int u = i / M1, t = i - u * M1;
    return (u >= 1 && t < MU - u) ? A.qinvq + 2 * ((size_t)(A.level - u) * A.L + top + t) : nullptr;
  };
  if constexpr (MU > 0) {
    gather_words(vch, 2 * MU * MU, [&](int i) {
      const uint32_t* ci = chain_src(i >> 1);
      return ci ? ci[i & 1] : 0u;
    });
    gather_words(vgtop, 2 * top, [&](int i) { return A.rs[i]; });
    gather_words(vgt, top * MU, [&](int i) { return A.rs[2 * top + i]; });
  }
  put_words(vph, 2 * KP, phinv);
  put_words(vpi, KP * A.level, pinvq);
  if constexpr (MU > 0) {
    put_words(vch, 2 * MU * MU, chain);
    put_words(vgtop, 2 * top, gtop);
    put_words(vgt, top * MU, gt);
  }
  __syncthreads();
}

template <int MU, int KP>
__device__ __forceinline__ void moddown_body(const uint32_t* acc, uint32_t* out, const MdArgs& A, int l, size_t n,
                                             const uint32_t* c, const DevTables& T) {
  const size_t N = (size_t)1 << A.log_n;
  const uint32_t* row = acc + (size_t)l * A.E * N + n;
  uint32_t* o = out + (size_t)l * (A.level - MU) * N + n;
  const uint32_t* phinv = c;
  const uint32_t* pinvq = phinv + 2 * KP;
  const uint32_t* chain = pinvq + KP * 60;
  const uint32_t* gtop = chain + 2 * 12 * 12;
  const uint32_t* gt = gtop + 2 * 60;
  // scaled p residues z_i = [phat_i^-1 x_i]_{p_i}; for i >= K the staged
  // constant is 0 (and the row read is the last special prime's)
  uint32_t z[KP];
#pragma unroll
  for (int i = 0; i < KP; i++) {
    const int ii = min(i, A.K - 1);
    z[i] = shoup(row[(size_t)(A.level + ii) * N], phinv[2 * i], phinv[2 * i + 1], T.mod[A.L + ii]);
  }
  // each product z_i [p_i^-1]_{q_j} is below 2^61, so eight of them fit 64
  // bits: wider special bases reduce every eight terms
  auto cstar = [&](int j, uint32_t x) -> uint32_t {
    const Red64 rc = T.red[j];
    uint32_t r = 0;
#pragma unroll
    for (int i0 = 0; i0 < KP; i0 += 8) {
      uint64_t s = 0;
#pragma unroll
      for (int i = i0; i < i0 + 8 && i < KP; i++) s += (uint64_t)z[i] * pinvq[i * A.level + j];
      r = i0 == 0 ? reduce64(s, rc) : add_mod(r, reduce64(s, rc), rc.m);
    }
    return sub_mod(x, r, rc.m);
  };
  if constexpr (MU == 0) {
    for (int j = 0; j < A.level; j++) o[(size_t)j * N] = cstar(j, row[(size_t)j * N]);
  } else {
    const int top = A.level - MU;
    uint32_t fin[MU];
    {
      uint32_t cur[MU];
#pragma unroll
      for (int i = 0; i < MU; i++) cur[i] = row[(size_t)(top + i) * N];
#pragma unroll
      for (int i = 0; i < MU; i++) cur[i] = cstar(top + i, cur[i]);
      fin[MU - 1] = cur[MU - 1];
      // the u-th rescale drops q_{l-u}
#pragma unroll
      for (int u = 1; u < MU; u++) {
        const uint32_t cd = cur[MU - u];
#pragma unroll
        for (int i = 0; i < MU - u; i++) {
          const uint32_t qt = T.mod[top + i];
          const uint32_t* ci = chain + 2 * (u * MU + i);
          cur[i] = shoup(cur[i] + qt - cd, ci[0], ci[1], qt);
        }
        fin[MU - 1 - u] = cur[MU - 1 - u];
      }
    }
    // four output limbs per round: their loads issue together
    int eta = 0;
    for (; eta + 4 <= top; eta += 4) {
      uint32_t x[4];
#pragma unroll
      for (int v = 0; v < 4; v++) x[v] = row[(size_t)(eta + v) * N];
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int e = eta + v;
        const Red64 rc = T.red[e];
        uint64_t s = 0;
#pragma unroll
        for (int i = 0; i < MU; i++) s += (uint64_t)fin[i] * gt[e * MU + i];
        const uint32_t a = shoup(cstar(e, x[v]), gtop[2 * e], gtop[2 * e + 1], rc.m);
        o[(size_t)e * N] = sub_mod(a, reduce64(s, rc), rc.m);
      }
    }
    for (; eta < top; eta++) {
      const Red64 rc = T.red[eta];
      uint64_t s = 0;
#pragma unroll
      for (int i = 0; i < MU; i++) s += (uint64_t)fin[i] * gt[eta * MU + i];
      const uint32_t a = shoup(cstar(eta, row[(size_t)eta * N]), gtop[2 * eta], gtop[2 * eta + 1], rc.m);
      o[(size_t)eta * N] = sub_mod(a, reduce64(s, rc), rc.m);
    }
  }
}

template <int MU, int KP>
__global__ __launch_bounds__(kThreads) void k_moddown_rs(const uint32_t* acc, uint32_t* out, MdArgs A, DevTables T) {
  __shared__ uint32_t c[md_lds_words<KP>()];
  moddown_stage<MU, KP>(A, c);
  const size_t job = blockIdx.z;
  moddown_body<MU, KP>(acc + job * (size_t)A.acc_job, out + job * (size_t)A.out_job, A, blockIdx.y,
                   (size_t)blockIdx.x * kThreads + threadIdx.x, c, T);
}

// Job-table form: jobs [j0, j0 + nj) of equal k = MU + 1; blocks per job 2 N / 256.
template <int MU, int KP>
__global__ __launch_bounds__(kThreads) void k_moddown_rs_jt(const JobDesc* jt, int j0, int nj, GroupConsts G,
                                                            DevTables T) {
  const int j = j0 + find_job(jt + j0, nj, S_MODDOWN, blockIdx.x);
  const int local = blockIdx.x - jt[j].blk0[S_MODDOWN];
  const int xb = 1 << (G.log_n - 8);
  if (local >= 2 * xb) return;
  const int level = jt[j].level;
  MdArgs A{};
  A.md = G.md;
  A.qinvq = G.md + 2 * G.K + (size_t)G.K * G.L;
  A.rs = MU > 0 ? G.rs_tab + G.rs_off[level * (G.L + 1) + MU] : nullptr;
  A.log_n = G.log_n;
  A.level = level;
  A.L = G.L;
  A.K = G.K;
  A.E = level + G.K;
  const WsLayout lay(MU + 1, level, G.K, G.alpha, G.log_n);
  __shared__ uint32_t c[md_lds_words<KP>()];
  moddown_stage<MU, KP>(A, c);
  moddown_body<MU, KP>(jt[j].ws + lay.acc, jt[j].out, A, local / xb, (size_t)(local % xb) * kThreads + threadIdx.x, c,
                   T);
}

// Algorithm 1 step 2 and the sums of step 3 on coefficient-domain dropped
// limbs `topc` ([polys][MU][N], polynomial blockIdx.y):
// b_eta = sum_t g^{mu,t}_eta a^(t),{l-1-t}.  The chain constants and the g
// table are staged in LDS.
template <int MU>
__global__ __launch_bounds__(kThreads) void k_rs_sums(const uint32_t* topc, uint32_t* bout, MdArgs A, DevTables T) {
  __shared__ uint32_t chain[2 * MU * MU];  // [u][t][2], rescale u dropping q_{l-u}
  __shared__ uint32_t gt[60 * MU];         // [top <= 60][MU]
  {
    const int top = A.level - MU;
    uint32_t vch[2], vgt[(60 * MU + kThreads - 1) / kThreads];
    gather_words(vch, 2 * MU * MU, [&](int i) {
      const int u = (i >> 1) / MU, t = (i >> 1) - u * MU;
      return (u >= 1 && t < MU - u) ? A.qinvq[2 * ((size_t)(A.level - u) * A.L + top + t) + (i & 1)] : 0u;
    });
    gather_words(vgt, top * MU, [&](int i) { return A.rs[2 * top + i]; });
    put_words(vch, 2 * MU * MU, chain);
    put_words(vgt, top * MU, gt);
    __syncthreads();
  }
  const size_t N = (size_t)1 << A.log_n;
  const size_t n = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const int l = blockIdx.y;
  const int top = A.level - MU;
  const uint32_t* src = topc + (size_t)l * MU * N + n;
  uint32_t* o = bout + (size_t)l * top * N + n;
  uint32_t cur[MU], fin[MU];
#pragma unroll
  for (int i = 0; i < MU; i++) cur[i] = src[(size_t)i * N];
  fin[MU - 1] = cur[MU - 1];
#pragma unroll
  for (int u = 1; u < MU; u++) {
    const uint32_t cd = cur[MU - u];
#pragma unroll
    for (int i = 0; i < MU - u; i++) {
      const uint32_t qt = T.mod[top + i];
      const uint32_t* ci = chain + 2 * (u * MU + i);
      cur[i] = shoup(cur[i] + qt - cd, ci[0], ci[1], qt);
    }
    fin[MU - 1 - u] = cur[MU - 1 - u];
  }
  int eta = 0;
  for (; eta + 4 <= top; eta += 4) {
#pragma unroll
    for (int v = 0; v < 4; v++) {
      uint64_t s = 0;
#pragma unroll
      for (int i = 0; i < MU; i++) s += (uint64_t)fin[i] * gt[(eta + v) * MU + i];
      o[(size_t)(eta + v) * N] = reduce64(s, T.red[eta + v]);
    }
  }
  for (; eta < top; eta++) {
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < MU; i++) s += (uint64_t)fin[i] * gt[eta * MU + i];
    o[(size_t)eta * N] = reduce64(s, T.red[eta]);
  }
}

// Algorithm 1 step 3, last line: A^(eta),{mu} = g^{mu,l-1}_eta A^(eta) - B^(eta).
__global__ __launch_bounds__(kThreads) void k_rs_combine(const uint32_t* Ain, const uint32_t* Bn, uint32_t* out,
                                                         MdArgs A, int mu, DevTables T) {
  const size_t N = (size_t)1 << A.log_n;
  const size_t n = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const int eta = blockIdx.y, l = blockIdx.z;
  const int top = A.level - mu;
  const uint32_t m = T.mod[eta];
  const uint32_t a = Ain[((size_t)l * A.level + eta) * N + n];
  const uint32_t b = Bn[((size_t)l * top + eta) * N + n];
  out[((size_t)l * top + eta) * N + n] = sub_mod(shoup(a, A.rs[2 * eta], A.rs[2 * eta + 1], m), b, m);
}

// ------------------------------------------------------------------ key generation / encryption
// Pointwise helpers over rows of the extended basis.  Row r uses prime
// index prime0 + r.
__global__ void k_pk(const uint32_t* E, const uint32_t* a, const uint32_t* S, uint32_t* b, int log_n, DevTables T) {
  const size_t N = (size_t)1 << log_n;
  const int r = blockIdx.y;
  const size_t i = (size_t)r * N + (size_t)blockIdx.x * kThreads + threadIdx.x;
  const uint32_t m = T.mod[r], minv = T.minv[r], r2 = T.rpow[(size_t)r * 2 * (kMaxK + 1) + 4];
  b[i] = sub_mod(E[i], mul_var(a[i], S[i], m, minv, r2), m);
}

__global__ void k_mul_rows(uint32_t* X, const uint32_t* Y, int log_n, DevTables T) {
  const size_t N = (size_t)1 << log_n;
  const int r = blockIdx.y;
  const size_t i = (size_t)r * N + (size_t)blockIdx.x * kThreads + threadIdx.x;
  const uint32_t m = T.mod[r], minv = T.minv[r], r2 = T.rpow[(size_t)r * 2 * (kMaxK + 1) + 4];
  X[i] = mul_var(X[i], Y[i], m, minv, r2);
}

// ek_{t,b,0} = E - a S + g_r S^t, ek_{t,b,1} = a, then q rows times [P^-1].
// Rows 0..L-1 are q_j, rows L.. are p_i (prime index = row).
__global__ void k_evk(const uint32_t* E, const uint32_t* a, const uint32_t* S, const uint32_t* St, uint32_t* k0,
                      uint32_t* k1, const uint32_t* rowc /*[L+K][4]: g, f, f_sh*/, int log_n, DevTables T) {
  const size_t N = (size_t)1 << log_n;
  const int r = blockIdx.y;
  const size_t i = (size_t)r * N + (size_t)blockIdx.x * kThreads + threadIdx.x;
  const uint32_t m = T.mod[r], minv = T.minv[r], r2 = T.rpow[(size_t)r * 2 * (kMaxK + 1) + 4];
  const uint32_t g = rowc[4 * r], f = rowc[4 * r + 1], fsh = rowc[4 * r + 2];
  uint32_t v = sub_mod(E[i], mul_var(a[i], S[i], m, minv, r2), m);
  v = add_mod(v, mul_var(St[i], g, m, minv, r2), m);
  k0[i] = shoup(v, f, fsh, m);
  k1[i] = shoup(a[i], f, fsh, m);
}

// c0 = V b + M0, c1 = V a + E1 (rows are q_0..q_{level-1}).
__global__ void k_enc(const uint32_t* V, const uint32_t* M0, const uint32_t* E1, const uint32_t* pk, uint32_t* ct,
                      int level, int L, int log_n, DevTables T) {
  const size_t N = (size_t)1 << log_n;
  const int r = blockIdx.y;
  const size_t n = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const size_t i = (size_t)r * N + n;
  const uint32_t m = T.mod[r], minv = T.minv[r], r2 = T.rpow[(size_t)r * 2 * (kMaxK + 1) + 4];
  const uint32_t b = pk[i], a = pk[((size_t)L + r) * N + n];
  ct[i] = add_mod(mul_var(V[i], b, m, minv, r2), M0[i], m);
  ct[(size_t)level * N + i] = add_mod(mul_var(V[i], a, m, minv, r2), E1[i], m);
}

// X = c0 + c1 S (NTT domain).
__global__ void k_dec(const uint32_t* ct, const uint32_t* S, uint32_t* X, int level, int log_n, DevTables T) {
  const size_t N = (size_t)1 << log_n;
  const int r = blockIdx.y;
  const size_t n = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const size_t i = (size_t)r * N + n;
  const uint32_t m = T.mod[r], minv = T.minv[r], r2 = T.rpow[(size_t)r * 2 * (kMaxK + 1) + 4];
  X[i] = add_mod(ct[i], mul_var(ct[(size_t)level * N + i], S[i], m, minv, r2), m);
}

}  // namespace

// ------------------------------------------------------------------ launchers

int launch_tensor(const mick_params* prm, const CtPtrs& in, long long in_job_stride, int k, int level, uint32_t* D,
                  long long d_job_stride, int n_jobs, hipStream_t s) {
  dim3 grid((unsigned)(prm->N / (kThreads * 4)), (unsigned)level, (unsigned)n_jobs);
  const DevTables& T = prm->dt;
  const int ln = prm->log_n;
  ProfScope ps(P_TENSOR, s);
  switch (k) {
#define MICK_T(KK) \
  case KK: k_tensor<KK><<<grid, kThreads, 0, s>>>(in, in_job_stride, level, ln, D, d_job_stride, T); break;
    MICK_T(2) MICK_T(3) MICK_T(4) MICK_T(5) MICK_T(6) MICK_T(7) MICK_T(8) MICK_T(9) MICK_T(10) MICK_T(11) MICK_T(12)
#undef MICK_T
    default: return set_error(MICK_E_ARG, "k out of range");
  }
  return hip_error(hipGetLastError(), "tensor launch");
}

int launch_moddown_rs(const mick_params* prm, const uint32_t* acc, uint32_t* out, const MdArgs& A, int mu, int n_jobs,
                      hipStream_t s) {
  dim3 grid((unsigned)(prm->N / kThreads), 2, (unsigned)n_jobs);
  const DevTables& T = prm->dt;
  ProfScope ps(P_MODDOWN_RS, s);
  const bool wide = A.K > 8;
  switch (mu) {
#define MICK_M(MM)                                                          \
  case MM:                                                                  \
    if (wide)                                                               \
      k_moddown_rs<MM, 24><<<grid, kThreads, 0, s>>>(acc, out, A, T);       \
    else                                                                    \
      k_moddown_rs<MM, 8><<<grid, kThreads, 0, s>>>(acc, out, A, T);        \
    break;
    MICK_M(0) MICK_M(1) MICK_M(2) MICK_M(3) MICK_M(4) MICK_M(5) MICK_M(6) MICK_M(7) MICK_M(8) MICK_M(9) MICK_M(10)
    MICK_M(11)
#undef MICK_M
    default: return set_error(MICK_E_ARG, "mu out of range for the fused rescale");
  }
  return hip_error(hipGetLastError(), "moddown launch");
}

int launch_moddown_rs_jt(const mick_params* prm, const JobDesc* jt, int j0, int nj, int mu, int blocks,
                         const GroupConsts& G, hipStream_t s) {
  if (blocks <= 0) return MICK_OK;
  const DevTables& T = prm->dt;
  ProfScope ps(P_MODDOWN_RS, s);
  const bool wide = G.K > 8;
  switch (mu) {
#define MICK_M(MM)                                                               \
  case MM:                                                                       \
    if (wide)                                                                    \
      k_moddown_rs_jt<MM, 24><<<blocks, kThreads, 0, s>>>(jt, j0, nj, G, T);     \
    else                                                                         \
      k_moddown_rs_jt<MM, 8><<<blocks, kThreads, 0, s>>>(jt, j0, nj, G, T);      \
    break;
    MICK_M(1) MICK_M(2) MICK_M(3) MICK_M(4) MICK_M(5) MICK_M(6) MICK_M(7) MICK_M(8) MICK_M(9) MICK_M(10) MICK_M(11)
#undef MICK_M
    default: return set_error(MICK_E_ARG, "mu out of range for the fused rescale");
  }
  return hip_error(hipGetLastError(), "moddown launch");
}

int launch_rs_sums(const mick_params* prm, const uint32_t* topc, uint32_t* bout, const MdArgs& A, int mu, int polys,
                   hipStream_t s) {
  dim3 grid((unsigned)(prm->N / kThreads), (unsigned)polys, 1);
  const DevTables& T = prm->dt;
  ProfScope ps(P_RS_SUMS, s);
  switch (mu) {
#define MICK_R(MM) \
  case MM: k_rs_sums<MM><<<grid, kThreads, 0, s>>>(topc, bout, A, T); break;
    MICK_R(1) MICK_R(2) MICK_R(3) MICK_R(4) MICK_R(5) MICK_R(6) MICK_R(7) MICK_R(8) MICK_R(9) MICK_R(10) MICK_R(11)
    MICK_R(12) MICK_R(13) MICK_R(14) MICK_R(15) MICK_R(16)
#undef MICK_R
    default: return set_error(MICK_E_ARG, "mu out of range (1..16)");
  }
  return hip_error(hipGetLastError(), "rescale sums launch");
}

int launch_rs_combine(const mick_params* prm, const uint32_t* Ain, const uint32_t* Bn, uint32_t* out, const MdArgs& A,
                      int mu, int polys, hipStream_t s) {
  dim3 grid((unsigned)(prm->N / kThreads), (unsigned)(A.level - mu), (unsigned)polys);
  ProfScope ps(P_RS_COMBINE, s);
  k_rs_combine<<<grid, kThreads, 0, s>>>(Ain, Bn, out, A, mu, prm->dt);
  return hip_error(hipGetLastError(), "rescale combine launch");
}

int launch_pk(const mick_params* prm, const uint32_t* E, const uint32_t* a, const uint32_t* S, uint32_t* b,
              hipStream_t s) {
  dim3 grid((unsigned)(prm->N / kThreads), (unsigned)prm->L, 1);
  k_pk<<<grid, kThreads, 0, s>>>(E, a, S, b, prm->log_n, prm->dt);
  return hip_error(hipGetLastError(), "pk launch");
}

int launch_mul_rows(const mick_params* prm, uint32_t* X, const uint32_t* Y, int rows, hipStream_t s) {
  dim3 grid((unsigned)(prm->N / kThreads), (unsigned)rows, 1);
  k_mul_rows<<<grid, kThreads, 0, s>>>(X, Y, prm->log_n, prm->dt);
  return hip_error(hipGetLastError(), "mul launch");
}

int launch_evk(const mick_params* prm, const uint32_t* E, const uint32_t* a, const uint32_t* S, const uint32_t* St,
               uint32_t* k0, uint32_t* k1, const uint32_t* rowc, hipStream_t s) {
  dim3 grid((unsigned)(prm->N / kThreads), (unsigned)(prm->L + prm->K), 1);
  k_evk<<<grid, kThreads, 0, s>>>(E, a, S, St, k0, k1, rowc, prm->log_n, prm->dt);
  return hip_error(hipGetLastError(), "evk launch");
}

int launch_enc(const mick_params* prm, const uint32_t* V, const uint32_t* M0, const uint32_t* E1, const uint32_t* pk,
               uint32_t* ct, int level, hipStream_t s) {
  dim3 grid((unsigned)(prm->N / kThreads), (unsigned)level, 1);
  k_enc<<<grid, kThreads, 0, s>>>(V, M0, E1, pk, ct, level, prm->L, prm->log_n, prm->dt);
  return hip_error(hipGetLastError(), "encrypt launch");
}

int launch_dec(const mick_params* prm, const uint32_t* ct, const uint32_t* S, uint32_t* X, int level, hipStream_t s) {
  dim3 grid((unsigned)(prm->N / kThreads), (unsigned)level, 1);
  k_dec<<<grid, kThreads, 0, s>>>(ct, S, X, level, prm->log_n, prm->dt);
  return hip_error(hipGetLastError(), "decrypt launch");
}

}  // namespace mick
