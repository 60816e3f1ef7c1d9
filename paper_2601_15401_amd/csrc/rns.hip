// Pointwise RNS kernels of the k-input multiply: tensor product, ModUp basis
// conversion, key inner product, relocated ModDown fused with the combined
// multi-level rescale, the steps of Algorithm 1, and the small pointwise
// operations of key generation, encryption and decryption.
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
// eq. (d_u formula for n-ct mult): prod_u (c0^u + c1^u Y) = sum_t d_t Y^t,
// built one factor at a time; every partial product picks up one R^-1 per
// factor, removed at the end by R^(k-1).
template <int K>
__global__ __launch_bounds__(kThreads) void k_tensor(CtPtrs in, long long in_job_stride, int level, int log_n,
                                                     uint32_t* D, long long d_job_stride, DevTables T) {
  const int j = blockIdx.y;
  const size_t n = (size_t)blockIdx.x * kThreads + threadIdx.x;  // uint4 index
  const size_t N = (size_t)1 << log_n;
  const uint32_t m = T.mod[j], minv = T.minv[j];
  const size_t job_in = (size_t)blockIdx.z * (size_t)in_job_stride;
  const size_t limb = (size_t)j * N;
  const size_t poly = (size_t)level * N;
  uint4 P[K + 1];
  {
    const uint4* c = reinterpret_cast<const uint4*>(in.p[0] + job_in + limb);
    P[0] = c[n];
    P[1] = reinterpret_cast<const uint4*>(in.p[0] + job_in + poly + limb)[n];
  }
#pragma unroll
  for (int u = 1; u < K; u++) {
    const uint4 a = reinterpret_cast<const uint4*>(in.p[u] + job_in + limb)[n];
    const uint4 b = reinterpret_cast<const uint4*>(in.p[u] + job_in + poly + limb)[n];
    // new_t = P_t a + P_{t-1} b, t = u+1 .. 0 (descending keeps P_{t-1} intact)
    P[u + 1].x = mont_mul(P[u].x, b.x, m, minv);
    P[u + 1].y = mont_mul(P[u].y, b.y, m, minv);
    P[u + 1].z = mont_mul(P[u].z, b.z, m, minv);
    P[u + 1].w = mont_mul(P[u].w, b.w, m, minv);
#pragma unroll
    for (int t = u; t >= 1; t--) {
      P[t].x = add_mod(mont_mul(P[t].x, a.x, m, minv), mont_mul(P[t - 1].x, b.x, m, minv), m);
      P[t].y = add_mod(mont_mul(P[t].y, a.y, m, minv), mont_mul(P[t - 1].y, b.y, m, minv), m);
      P[t].z = add_mod(mont_mul(P[t].z, a.z, m, minv), mont_mul(P[t - 1].z, b.z, m, minv), m);
      P[t].w = add_mod(mont_mul(P[t].w, a.w, m, minv), mont_mul(P[t - 1].w, b.w, m, minv), m);
    }
    P[0].x = mont_mul(P[0].x, a.x, m, minv);
    P[0].y = mont_mul(P[0].y, a.y, m, minv);
    P[0].z = mont_mul(P[0].z, a.z, m, minv);
    P[0].w = mont_mul(P[0].w, a.w, m, minv);
  }
  const uint32_t* rp = T.rpow + (size_t)j * 2 * (kMaxK + 1);
  const uint32_t f = rp[2 * (K - 1)], fsh = rp[2 * (K - 1) + 1];
  uint32_t* out = D + (size_t)blockIdx.z * (size_t)d_job_stride + limb;
#pragma unroll
  for (int t = 0; t <= K; t++) {
    uint4 v;
    v.x = shoup(P[t].x, f, fsh, m);
    v.y = shoup(P[t].y, f, fsh, m);
    v.z = shoup(P[t].z, f, fsh, m);
    v.w = shoup(P[t].w, f, fsh, m);
    reinterpret_cast<uint4*>(out + (size_t)t * poly)[n] = v;
  }
}

// ------------------------------------------------------------------ ModUp
// eq. (basis conversion): for digit b of the active primes, y_j =
// [x_j qhat_j^-1]_{q_j}, then [sum_j y_j qhat_j]_m for every other modulus m
// of the extended basis.  Input coefficient domain, output coefficient
// domain (the NTT follows).  Table of (level, digit), padded to ALPHA rows
// with zeros when the digit is truncated at this level:
//   [ALPHA] qhat_j^-1, [ALPHA] Shoup companions, [ALPHA][E] qhat_j mod m_e.
// The table and the targets' reduction constants are staged in LDS; each
// thread converts 4 neighbouring coefficients.
template <int ALPHA>
__global__ __launch_bounds__(kThreads) void k_modup(const uint32_t* dcoef, uint32_t* X, ModupArgs A, DevTables T) {
  __shared__ uint32_t s_c[ALPHA * kMaxE];
  __shared__ Red64 s_red[kMaxE];
  const size_t N = (size_t)1 << A.log_n;
  const size_t n = ((size_t)blockIdx.x * kThreads + threadIdx.x) * 4;
  const int tb = blockIdx.y;  // (t - 2) * B + b
  const int t2 = tb / A.B, b = tb - t2 * A.B;
  const int lo = b * A.alpha;
  const int a = min(A.alpha, A.level - lo);
  const uint32_t* tab = A.tab + A.tab_off[b];
  const int E = A.E;
  for (int i = threadIdx.x; i < ALPHA * E; i += kThreads) s_c[i] = tab[2 * ALPHA + i];
  for (int e = threadIdx.x; e < E; e += kThreads) s_red[e] = T.red[e < A.level ? e : A.L + (e - A.level)];
  const size_t job = (size_t)blockIdx.z;
  const uint32_t* src = dcoef + job * (size_t)A.dcoef_job + ((size_t)t2 * A.level + lo) * N + n;
  uint32_t* dst = X + job * (size_t)A.x_job + ((size_t)tb * E) * N + n;
  uint4 y[ALPHA];
#pragma unroll
  for (int j = 0; j < ALPHA; j++) {
    const int row = min(j, a - 1);  // padded rows read a valid limb, scaled by 0
    const uint32_t qj = T.mod[lo + row];
    const uint4 v = *reinterpret_cast<const uint4*>(src + (size_t)row * N);
    const uint32_t w = tab[j], wsh = tab[ALPHA + j];
    y[j].x = shoup(v.x, w, wsh, qj);
    y[j].y = shoup(v.y, w, wsh, qj);
    y[j].z = shoup(v.z, w, wsh, qj);
    y[j].w = shoup(v.w, w, wsh, qj);
  }
  __syncthreads();
  for (int e = 0; e < E; e++) {
    if (e >= lo && e < lo + a) continue;
    const Red64 rc = s_red[e];
    uint64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
    for (int j = 0; j < ALPHA; j++) {
      const uint64_t c = s_c[j * E + e];
      s0 += y[j].x * c;
      s1 += y[j].y * c;
      s2 += y[j].z * c;
      s3 += y[j].w * c;
    }
    uint4 o;
    o.x = reduce64(s0, rc);
    o.y = reduce64(s1, rc);
    o.z = reduce64(s2, rc);
    o.w = reduce64(s3, rc);
    *reinterpret_cast<uint4*>(dst + (size_t)e * N) = o;
  }
}

// ------------------------------------------------------------------ key inner product
// Acc_l[e] = sum_t sum_b X_{t,b}[e] ek'_{t,b,l}[e] over the extended basis,
// X_{t,b}[e] = D_t[e] on the digit's own primes (Sec. III combined sum; the
// q rows of ek' carry P^-1, Sec. IV).  On the q rows the relocated ModDown
// input D_l + P^-1 C~ is formed here.  Up to JB jobs share each key load.
template <int JB>
__global__ __launch_bounds__(kThreads) void k_kip(const uint32_t* D, const uint32_t* X, const uint32_t* evk,
                                                  uint32_t* acc, KipArgs A, DevTables T) {
  const size_t N = (size_t)1 << A.log_n;
  const size_t n = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const int e = blockIdx.y;
  const int job0 = blockIdx.z * JB;
  const int nj = min(JB, A.n_jobs - job0);
  const int pe = e < A.level ? e : A.L + (e - A.level);
  const Red64 rc = T.red[pe];
  const int chunk = rc.m < (1u << 30) ? 16 : 4;  // products < m^2, sums stay below 2^64
  const size_t key_row = ((size_t)pe << A.log_n) + n;
  uint64_t a0[JB], a1[JB];
  uint32_t r0[JB], r1[JB];
#pragma unroll
  for (int i = 0; i < JB; i++) {
    a0[i] = a1[i] = 0;
    r0[i] = r1[i] = 0;
  }
  int cnt = 0;
  for (int t = 2; t <= A.k; t++) {
    for (int b = 0; b < A.B; b++) {
      const int lo = b * A.alpha;
      const bool own = e >= lo && e < min(lo + A.alpha, A.level);
      const size_t ko = (((size_t)(t - 2) * A.dnum + b) * 2) * A.key_poly;
      const uint32_t k0 = evk[ko + key_row];
      const uint32_t k1 = evk[ko + A.key_poly + key_row];
#pragma unroll
      for (int i = 0; i < JB; i++) {
        if (i < nj) {
          const size_t jo = (size_t)(job0 + i);
          const uint32_t x = own ? D[jo * (size_t)A.d_job + ((size_t)t * A.level + e) * N + n]
                                 : X[jo * (size_t)A.x_job + (((size_t)(t - 2) * A.B + b) * A.E + e) * N + n];
          a0[i] += (uint64_t)x * k0;
          a1[i] += (uint64_t)x * k1;
        }
      }
      if (++cnt == chunk) {
        cnt = 0;
#pragma unroll
        for (int i = 0; i < JB; i++) {
          r0[i] = add_mod(r0[i], reduce64(a0[i], rc), rc.m);
          r1[i] = add_mod(r1[i], reduce64(a1[i], rc), rc.m);
          a0[i] = a1[i] = 0;
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < JB; i++) {
    if (i < nj) {
      const size_t jo = (size_t)(job0 + i);
      uint32_t v0 = add_mod(r0[i], reduce64(a0[i], rc), rc.m);
      uint32_t v1 = add_mod(r1[i], reduce64(a1[i], rc), rc.m);
      if (e < A.level) {
        v0 = add_mod(v0, D[jo * (size_t)A.d_job + (size_t)e * N + n], rc.m);
        v1 = add_mod(v1, D[jo * (size_t)A.d_job + ((size_t)A.level + e) * N + n], rc.m);
      }
      uint32_t* o = acc + jo * (size_t)A.acc_job + (size_t)e * N + n;
      o[0] = v0;
      o[(size_t)A.E * N] = v1;
    }
  }
}

// ------------------------------------------------------------------ ModDown + multi-rescale
// Input: acc after the INTT, coefficient domain: rows q_0..q_{l-1} hold
// INTT(D + P^-1 C~) (eq. (moddown improved 2)), rows p_i hold INTT(C~^(p)).
// c*_j = row_j - scBConv(p rows)_j (eq. (scBconv)), then mu rescalings by
// eq. (multi rs): the dropped limbs run the chain of Algorithm 1 step 2,
// every kept limb eta takes g^{mu,l-1}_eta c*_eta - sum_t g^{mu,t}_eta a_t.
// Output coefficient domain, limbs 0..l-mu-1 (the final NTT follows).
template <int MU>
__global__ __launch_bounds__(kThreads) void k_moddown_rs(const uint32_t* acc, uint32_t* out, MdArgs A, DevTables T) {
  const size_t N = (size_t)1 << A.log_n;
  const size_t n = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const int l = blockIdx.y;
  const size_t job = blockIdx.z;
  const uint32_t* row = acc + job * (size_t)A.acc_job + (size_t)l * A.E * N + n;
  uint32_t* o = out + job * (size_t)A.out_job + (size_t)l * (A.level - MU) * N + n;
  // scaled p residues z_i = [phat_i^-1 x_i]_{p_i}
  uint32_t z[kMaxKp];
#pragma unroll
  for (int i = 0; i < kMaxKp; i++) {
    if (i < A.K) {
      const uint32_t pi = T.mod[A.L + i];
      z[i] = shoup(row[(size_t)(A.level + i) * N], A.md[2 * i], A.md[2 * i + 1], pi);
    }
  }
  const uint32_t* pinvq = A.md + 2 * A.K;  // [K][L]
  auto cstar = [&](int j) -> uint32_t {
    const Red64 rc = T.red[j];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < kMaxKp; i++) {
      if (i < A.K) s += (uint64_t)z[i] * pinvq[(size_t)i * A.L + j];
    }
    return sub_mod(row[(size_t)j * N], reduce64(s, rc), rc.m);
  };
  if constexpr (MU == 0) {
    for (int j = 0; j < A.level; j++) o[(size_t)j * N] = cstar(j);
  } else {
    const int top = A.level - MU;
    uint32_t fin[MU];
    {
      uint32_t cur[MU];
#pragma unroll
      for (int i = 0; i < MU; i++) cur[i] = cstar(top + i);
      fin[MU - 1] = cur[MU - 1];
      // the u-th rescale drops q_{l-u}; chain constants q_d^-1 mod q_t (+ Shoup)
#pragma unroll
      for (int u = 1; u < MU; u++) {
        const int d = A.level - u;
        const uint32_t cd = cur[MU - u];
#pragma unroll
        for (int i = 0; i < MU - u; i++) {
          const int t = top + i;
          const uint32_t qt = T.mod[t];
          const uint32_t* ci = A.qinvq + 2 * ((size_t)d * A.L + t);
          cur[i] = shoup(cur[i] + qt - cd, ci[0], ci[1], qt);
        }
        fin[MU - 1 - u] = cur[MU - 1 - u];
      }
    }
    const uint32_t* g = A.rs;  // [top][2] gtop (+Shoup), then [top][MU] g
    const uint32_t* gt = g + 2 * (size_t)top;
    for (int eta = 0; eta < top; eta++) {
      const Red64 rc = T.red[eta];
      uint64_t s = 0;
#pragma unroll
      for (int i = 0; i < MU; i++) s += (uint64_t)fin[i] * gt[(size_t)eta * MU + i];
      const uint32_t a = shoup(cstar(eta), g[2 * eta], g[2 * eta + 1], rc.m);
      o[(size_t)eta * N] = sub_mod(a, reduce64(s, rc), rc.m);
    }
  }
}

// Algorithm 1 step 2 and the sums of step 3 on coefficient-domain dropped
// limbs `topc` ([2][MU][N]): b_eta = sum_t g^{mu,t}_eta a^(t),{l-1-t}.
template <int MU>
__global__ __launch_bounds__(kThreads) void k_rs_sums(const uint32_t* topc, uint32_t* bout, MdArgs A, DevTables T) {
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
    const int d = A.level - u;
    const uint32_t cd = cur[MU - u];
#pragma unroll
    for (int i = 0; i < MU - u; i++) {
      const int t = top + i;
      const uint32_t qt = T.mod[t];
      const uint32_t* ci = A.qinvq + 2 * ((size_t)d * A.L + t);
      cur[i] = shoup(cur[i] + qt - cd, ci[0], ci[1], qt);
    }
    fin[MU - 1 - u] = cur[MU - 1 - u];
  }
  const uint32_t* gt = A.rs + 2 * (size_t)top;
  for (int eta = 0; eta < top; eta++) {
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < MU; i++) s += (uint64_t)fin[i] * gt[(size_t)eta * MU + i];
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

int launch_modup(const mick_params* prm, const uint32_t* dcoef, uint32_t* X, const ModupArgs& A, int k, int n_jobs,
                 hipStream_t s) {
  dim3 grid((unsigned)(prm->N / (kThreads * 4)), (unsigned)((k - 1) * A.B), (unsigned)n_jobs);
  ProfScope ps(P_MODUP, s);
  if (A.E > kMaxE) return set_error(MICK_E_ARG, "extended basis too large");
  switch (A.alpha) {
    case 1: k_modup<1><<<grid, kThreads, 0, s>>>(dcoef, X, A, prm->dt); break;
    case 2: k_modup<2><<<grid, kThreads, 0, s>>>(dcoef, X, A, prm->dt); break;
    case 3:
    case 4: k_modup<4><<<grid, kThreads, 0, s>>>(dcoef, X, A, prm->dt); break;
    default: k_modup<8><<<grid, kThreads, 0, s>>>(dcoef, X, A, prm->dt); break;
  }
  return hip_error(hipGetLastError(), "modup launch");
}

int launch_kip(const mick_params* prm, const uint32_t* D, const uint32_t* X, const uint32_t* evk, uint32_t* acc,
               const KipArgs& A, hipStream_t s) {
  const DevTables& T = prm->dt;
  ProfScope ps(P_KIP, s);
  if (A.n_jobs <= 1) {
    dim3 grid((unsigned)(prm->N / kThreads), (unsigned)A.E, 1);
    k_kip<1><<<grid, kThreads, 0, s>>>(D, X, evk, acc, A, T);
  } else {
    dim3 grid((unsigned)(prm->N / kThreads), (unsigned)A.E, (unsigned)((A.n_jobs + 7) / 8));
    k_kip<8><<<grid, kThreads, 0, s>>>(D, X, evk, acc, A, T);
  }
  return hip_error(hipGetLastError(), "kip launch");
}

int launch_moddown_rs(const mick_params* prm, const uint32_t* acc, uint32_t* out, const MdArgs& A, int mu, int n_jobs,
                      hipStream_t s) {
  dim3 grid((unsigned)(prm->N / kThreads), 2, (unsigned)n_jobs);
  const DevTables& T = prm->dt;
  ProfScope ps(P_MODDOWN_RS, s);
  switch (mu) {
#define MICK_M(MM) \
  case MM: k_moddown_rs<MM><<<grid, kThreads, 0, s>>>(acc, out, A, T); break;
    MICK_M(0) MICK_M(1) MICK_M(2) MICK_M(3) MICK_M(4) MICK_M(5) MICK_M(6) MICK_M(7) MICK_M(8) MICK_M(9) MICK_M(10)
    MICK_M(11)
#undef MICK_M
    default: return set_error(MICK_E_ARG, "mu out of range for the fused rescale");
  }
  return hip_error(hipGetLastError(), "moddown launch");
}

int launch_rs_sums(const mick_params* prm, const uint32_t* topc, uint32_t* bout, const MdArgs& A, int mu,
                   hipStream_t s) {
  dim3 grid((unsigned)(prm->N / kThreads), 2, 1);
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
                      int mu, hipStream_t s) {
  dim3 grid((unsigned)(prm->N / kThreads), (unsigned)(A.level - mu), 2);
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
