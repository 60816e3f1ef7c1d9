// Standalone fast basis conversion (Sec. II, eq. (basis conversion)) of one
// key-switching digit, by 32-bit VALU multiply-adds or by the int8 matrix
// cores; both give the same canonical residues.
//
// For digit b = {q_a} at level l, every coefficient of the target limb e is
//   out_e = sum_a y_a (qhat_a mod m_e) mod m_e,  y_a = [x_a qhat_a^-1]_{q_a},
// with qhat_a = Q_b / q_a.  In the fused multiply this conversion runs inside
// the ModUp kernel; this file exists to measure the matrix-core form against
// the VALU form on the same work.
//
// Matrix-core form (v_mfma_i32_32x32x32_i8, 32 targets x 32 coefficients x
// K = 32 per instruction, digits of at most 8 primes):
//  * B (K x coefficients): y_a split into four signed bytes, y = sum_i d_i
//    256^i with d_i in [-128, 128) (the bytes of (y + 0x80808080) XOR
//    0x80808080), row k = 4 a + i;
//  * A_j (targets x K), j = 0..3: byte j of the balanced signed base-256
//    digits of c_{e,a,i} = qhat_a R 256^i mod m_e (taken in (-m/2, m/2)),
//    R = 2^32;
//  * D_j = A_j B + C_j with C_0 = C_2 = 2^28 (offsets that keep the sums
//    below positive), |A_j B| <= 32 128^2 = 2^19;
//  * U = (D_0 + 256 D_1) + 2^16 (D_2 + 256 D_3) = S + 2^28 (1 + 2^16) with
//    S = sum_k c_k d_k congruent to R out_e; one Montgomery reduction of U
//    (< 2^46 < m 2^32) gives out_e + 2^28 (1 + 2^16) R^-1, and a modular
//    subtraction removes the offset.
// A and B take their K index from the same (lane half, byte) positions, so
// the product over K does not depend on how the instruction orders K.
#include <map>
#include <mutex>

#include "internal.h"
#include "rns.h"

namespace mick {

namespace {

constexpr int kBcThreads = 256;
constexpr int kBcTargets = 8;  // targets per thread of the VALU kernel

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Per (level, digit) device tables.
struct BcTables {
  int na = 0, T = 0, ntb = 0;  // sources, targets, target blocks of 32
  uint32_t* src = nullptr;     // [na][4]: q_a, qhat_a^-1 mod q_a, its Shoup companion, 0
  uint32_t* tgt = nullptr;     // [32 ntb][4]: m_e, m_e^-1 mod 2^32, offset R^-1 mod m_e, 0
  uint32_t* valu = nullptr;    // [8][T]: qhat_a R mod m_e (rows >= na zero)
  uint32_t* mfma = nullptr;    // [ntb][4 j][64 lanes][4 words]: the A operands
  Allocator alloc;
};

std::mutex g_bc_mu;
std::map<std::tuple<const mick_params*, int, int>, BcTables> g_bc;

__device__ __forceinline__ uint32_t signed_bytes(uint32_t y) { return (y + 0x80808080u) ^ 0x80808080u; }

// One thread: four consecutive coefficients of one polynomial, kBcTargets
// targets; the sources are loaded once for all of them.
__global__ __launch_bounds__(kBcThreads) void k_bconv_valu(const uint32_t* __restrict__ src,
                                                          uint32_t* __restrict__ dst, const uint32_t* __restrict__ st,
                                                          const uint32_t* __restrict__ tt,
                                                          const uint32_t* __restrict__ C, int na, int T, int log_n) {
  const size_t N = (size_t)1 << log_n;
  const size_t n4 = (size_t)blockIdx.x * kBcThreads + threadIdx.x;  // uint4 index, < N / 4 by the grid
  const size_t poly = blockIdx.z;
  const uint4* s4 = reinterpret_cast<const uint4*>(src + poly * na * N);
  uint4 y[8];
#pragma unroll
  for (int a = 0; a < 8; a++) {
    if (a < na) {
      const uint4 x = s4[(size_t)a * (N / 4) + n4];
      const uint32_t q = st[4 * a], w = st[4 * a + 1], wsh = st[4 * a + 2];
      y[a] = make_uint4(shoup(x.x, w, wsh, q), shoup(x.y, w, wsh, q), shoup(x.z, w, wsh, q), shoup(x.w, w, wsh, q));
    } else {
      y[a] = make_uint4(0, 0, 0, 0);
    }
  }
  const int e0 = blockIdx.y * kBcTargets;
  for (int ei = 0; ei < kBcTargets; ei++) {
    const int e = e0 + ei;
    if (e >= T) break;
    const uint32_t m = tt[4 * e], minv = tt[4 * e + 1];
    uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
    for (int a = 0; a < 8; a++) {
      const uint32_t c = C[a * T + e];
      a0 += (uint64_t)y[a].x * c;
      a1 += (uint64_t)y[a].y * c;
      a2 += (uint64_t)y[a].z * c;
      a3 += (uint64_t)y[a].w * c;
    }
    uint4 o = make_uint4(redc_2m(a0, m, minv), redc_2m(a1, m, minv), redc_2m(a2, m, minv), redc_2m(a3, m, minv));
    reinterpret_cast<uint4*>(dst + (poly * T + e) * N)[n4] = o;
  }
}

// One wave: kBcBlocks blocks of 32 coefficients of one polynomial, every
// target block.  Per target block the lane's A operands and the constants of
// its 16 output rows stay in registers across the coefficient blocks; the
// source constants of its four rows of K stay for the whole launch.
constexpr int kBcBlocks = 8;

__global__ __launch_bounds__(kBcThreads) void k_bconv_mfma(const uint32_t* __restrict__ src,
                                                          uint32_t* __restrict__ dst, const uint32_t* __restrict__ st,
                                                          const uint32_t* __restrict__ tt,
                                                          const uint32_t* __restrict__ A, int na, int T, int ntb,
                                                          int log_n) {
  const size_t N = (size_t)1 << log_n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane >> 5, c = lane & 31;
  const size_t n0 = ((size_t)blockIdx.x * (kBcThreads / 64) + wave) * 32 * kBcBlocks + c;  // < N by the grid
  const size_t poly = blockIdx.y;
  const uint32_t* sp = src + poly * na * N;
  uint32_t sq[4], sqi[4], sqs[4];
#pragma unroll
  for (int w = 0; w < 4; w++) {
    const int a = 4 * h + w;
    sq[w] = a < na ? st[4 * a] : 1;
    sqi[w] = a < na ? st[4 * a + 1] : 0;
    sqs[w] = a < na ? st[4 * a + 2] : 0;
  }
  const v16i off = {1 << 28, 1 << 28, 1 << 28, 1 << 28, 1 << 28, 1 << 28, 1 << 28, 1 << 28,
                    1 << 28, 1 << 28, 1 << 28, 1 << 28, 1 << 28, 1 << 28, 1 << 28, 1 << 28};
  const v16i zero = {};
  for (int tb = 0; tb < ntb; tb++) {
    const v4i* at = reinterpret_cast<const v4i*>(A) + (size_t)tb * 4 * 64 + lane;
    const v4i a0 = at[0], a1 = at[64], a2 = at[128], a3 = at[192];
    uint32_t cm[16], ci[16], co[16];
#pragma unroll
    for (int v = 0; v < 16; v++) {
      const int e = tb * 32 + (v & 3) + 4 * h + 8 * (v >> 2);  // output row of register v
      const bool ok = e < T;
      cm[v] = ok ? tt[4 * e] : 1u;
      ci[v] = ok ? tt[4 * e + 1] : 1u;
      co[v] = ok ? tt[4 * e + 2] : 0u;
    }
    for (int cb = 0; cb < kBcBlocks; cb++) {
      const size_t n = n0 + (size_t)cb * 32;
      v4i b;
#pragma unroll
      for (int w = 0; w < 4; w++) {
        const int a = 4 * h + w;
        const uint32_t y = a < na ? shoup(sp[(size_t)a * N + n], sqi[w], sqs[w], sq[w]) : 0u;
        b[w] = (int)signed_bytes(y);  // sources beyond the digit contribute the digits of 0
      }
      const v16i d0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b, off, 0, 0, 0);
      const v16i d1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b, zero, 0, 0, 0);
      const v16i d2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, b, off, 0, 0, 0);
      const v16i d3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a3, b, zero, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 16; v++) {
        const int e = tb * 32 + (v & 3) + 4 * h + 8 * (v >> 2);
        const uint32_t t1 = (uint32_t)d0[v] + ((uint32_t)d1[v] << 8);
        const uint32_t t2 = (uint32_t)d2[v] + ((uint32_t)d3[v] << 8);
        const uint64_t u = (uint64_t)t2 * 65536u + t1;
        if (e < T) dst[(poly * T + e) * N + n] = sub_mod(redc(u, cm[v], ci[v]), co[v], cm[v]);
      }
    }
  }
}

uint32_t inv_mod_u32(uint64_t a, uint64_t m) {
  int64_t t = 0, nt = 1, r = (int64_t)m, nr = (int64_t)(a % m);
  while (nr) {
    const int64_t qq = r / nr;
    int64_t tmp = t - qq * nt;
    t = nt;
    nt = tmp;
    tmp = r - qq * nr;
    r = nr;
    nr = tmp;
  }
  return (uint32_t)(t < 0 ? t + (int64_t)m : t);
}

uint64_t mulmod_u64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }

int build_bc(const mick_params* prm, int level, int digit, BcTables& t) {
  const int alpha = prm->alpha;
  const int lo = digit * alpha, na = std::min(alpha, level - lo);
  const int E = level + prm->K, T = E - na;
  t.na = na;
  t.T = T;
  t.ntb = (T + 31) / 32;
  t.alloc = prm->alloc;
  std::vector<uint32_t> tgt_m(T);
  for (int e = 0, i = 0; e < E; e++) {
    if (e >= lo && e < lo + na) continue;
    tgt_m[i++] = e < level ? prm->q[e] : prm->p[e - level];
  }
  std::vector<uint32_t> hs(4 * na, 0), ht(4 * 32 * t.ntb, 0), hv(8 * (size_t)T, 0),
      hm((size_t)t.ntb * 4 * 64 * 4, 0);
  for (int a = 0; a < na; a++) {
    const uint64_t q = prm->q[lo + a];
    uint64_t qhat_mod_q = 1;
    for (int b = 0; b < na; b++)
      if (b != a) qhat_mod_q = qhat_mod_q * (prm->q[lo + b] % q) % q;
    const uint32_t qi = inv_mod_u32(qhat_mod_q, q);
    hs[4 * a] = (uint32_t)q;
    hs[4 * a + 1] = qi;
    hs[4 * a + 2] = (uint32_t)(((uint64_t)qi << 32) / q);
  }
  const uint64_t off = ((uint64_t)1 << 28) * (1 + 65536);
  for (int e = 0; e < T; e++) {
    const uint64_t m = tgt_m[e];
    const uint64_t R = ((uint64_t)1 << 32) % m;
    const uint32_t rinv = inv_mod_u32(R, m);
    ht[4 * e] = (uint32_t)m;
    uint32_t minv = 1;  // m^-1 mod 2^32 by Newton iteration
    for (int it = 0; it < 5; it++) minv *= 2 - (uint32_t)m * minv;
    ht[4 * e + 1] = minv;
    ht[4 * e + 2] = (uint32_t)mulmod_u64(off % m, rinv, m);
    for (int a = 0; a < na; a++) {
      uint64_t qhat = 1;  // qhat_a mod m_e
      for (int b = 0; b < na; b++)
        if (b != a) qhat = qhat * (prm->q[lo + b] % m) % m;
      const uint64_t cr = mulmod_u64(qhat, R, m);  // Montgomery form
      hv[(size_t)a * T + e] = (uint32_t)cr;
      for (int i = 0; i < 4; i++) {
        uint64_t c = mulmod_u64(cr, (uint64_t)1 << (8 * i), m);
        int64_t v = c < m / 2 ? (int64_t)c : (int64_t)c - (int64_t)m;  // |v| < 2^30
        const int k = 4 * a + i;                                           // K index
        const int lane = (e & 31) + 32 * (k >> 4), byte = k & 15;
        const int tb = e >> 5;
        for (int j = 0; j < 4; j++) {
          const int64_t d = ((v + 128) & 255) - 128;  // balanced signed base-256 digit
          v = (v - d) / 256;
          uint32_t& w = hm[(((size_t)tb * 4 + j) * 64 + lane) * 4 + (byte >> 2)];
          w |= (uint32_t)(uint8_t)(int8_t)d << (8 * (byte & 3));
        }
      }
    }
  }
  auto up = [&](uint32_t** d, const std::vector<uint32_t>& h) -> int {
    void* p = nullptr;
    MICK_TRY(dev_alloc_bytes(t.alloc, &p, h.size() * 4));
    *d = (uint32_t*)p;
    return hip_error(hipMemcpy(*d, h.data(), h.size() * 4, hipMemcpyHostToDevice), "bconv tables");
  };
  MICK_TRY(up(&t.src, hs));
  MICK_TRY(up(&t.tgt, ht));
  MICK_TRY(up(&t.valu, hv));
  return up(&t.mfma, hm);
}

}  // namespace

void bconv_release(const mick_params* prm) {
  std::lock_guard<std::mutex> lk(g_bc_mu);
  for (auto it = g_bc.begin(); it != g_bc.end();) {
    if (std::get<0>(it->first) != prm) {
      ++it;
      continue;
    }
    for (uint32_t* p : {it->second.src, it->second.tgt, it->second.valu, it->second.mfma}) dev_free(it->second.alloc, p);
    it = g_bc.erase(it);
  }
}

}  // namespace mick

extern "C" int mick_bconv(const mick_params* prm, const uint32_t* src_dev, int n_polys, int level, int digit,
                          uint32_t* dst_dev, int method, void* stream) {
  using namespace mick;
  if (!prm || !src_dev || !dst_dev) return set_error(MICK_E_ARG, "NULL argument");
  if (level < 1 || level > prm->L) return set_error(MICK_E_LEVEL, "level must be in 1..L");
  if (digit < 0 || digit * prm->alpha >= level) return set_error(MICK_E_ARG, "no such digit at this level");
  if (n_polys < 1 || n_polys > 65535) return set_error(MICK_E_ARG, "n_polys must be in 1..65535");
  if (method != 0 && method != 1) return set_error(MICK_E_ARG, "method must be 0 (VALU) or 1 (matrix cores)");
  if (prm->alpha > 8) return set_error(MICK_E_ARG, "digits of at most 8 primes");
  const BcTables* t = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_bc_mu);
    auto key = std::make_tuple(prm, level, digit);
    auto it = g_bc.find(key);
    if (it == g_bc.end()) {
      BcTables nt;
      const int st = build_bc(prm, level, digit, nt);
      if (st != MICK_OK) {
        for (uint32_t* p : {nt.src, nt.tgt, nt.valu, nt.mfma}) dev_free(nt.alloc, p);
        return st;
      }
      it = g_bc.emplace(key, nt).first;
    }
    t = &it->second;
  }
  hipStream_t s = (hipStream_t)stream;
  if (method == 0) {
    dim3 grid((unsigned)(prm->N / 4 / kBcThreads), (unsigned)((t->T + kBcTargets - 1) / kBcTargets),
              (unsigned)n_polys);
    k_bconv_valu<<<grid, kBcThreads, 0, s>>>(src_dev, dst_dev, t->src, t->tgt, t->valu, t->na, t->T, prm->log_n);
  } else {
    dim3 grid((unsigned)(prm->N / (32 * kBcBlocks * (kBcThreads / 64))), (unsigned)n_polys);
    k_bconv_mfma<<<grid, kBcThreads, 0, s>>>(src_dev, dst_dev, t->src, t->tgt, t->mfma, t->na, t->T, t->ntb,
                                             prm->log_n);
  }
  return hip_error(hipGetLastError(), "bconv launch");
}
