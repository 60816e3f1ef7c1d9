// The tensor product of eq. (d_u formula for n-ct mult) fused with the first
// pass (pass B) of the inverse transform of d_2..d_k, same-shape and
// job-table launches.
#include "ntt_core.h"

namespace mick {

namespace {

// ------------------------------------------------------------------ tensor product + pass B of d_2..d_k's INTT

// One tile of one limb of every d_t: the tensor product (four residues per
// thread and step, tensor4), written in the NTT domain (all k + 1 limbs as by
// k_tensor, or given the keys the two own-digit sums of tensor_ib_tile), and
// d_2..d_k also kept in LDS, where the first pass of their inverse transform
// (pass B: both of its rounds, twiddles staged once for the k - 1 limbs)
// runs before its output is written.  The pass then reads nothing back from
// HBM.  Tiles of 1024 residues from k = 5; 2048 for k = 3, 4 and 4096 for
// k = 2, so that the k - 1 tiles' round items (64 per 1024 residues at 256
// rows per block) still cover the 256 threads.

// LDS rows and row blocks of the fused kernel's tiles.  Besides the two
// rounds, the tile is written by the tensor product itself: a lane stores
// four consecutive rows of one column, so a half-wave covers 32 / 2^RB1
// blocks four rows at a time.  Over 32 banks of 4 bytes:
//  * 2048 and 4096 residues (k = 2..4, at most three tiles): padded rows and
//    these block pitches leave at most two lanes of a half-wave on one bank
//    in the consecutive round and none in the strided round or the stores;
//  * 1024 residues (k >= 5, four to eleven tiles) in blocks of 2^7 or 2^8
//    rows: rows of COLS words, no padding, so that a tile takes 1024 + 16
//    XPAD words instead of about 1.5 times that and more workgroups fit a
//    CU's LDS; these pitches leave at most two lanes on one bank in each of
//    the three access patterns (with 2^6-row blocks unpadded rows would put
//    four lanes on one bank in the strided round, so those keep the padding).
constexpr int tib_pad(int logr, int tl) { return tl == 10 && logr >= 7 ? 1 << (tl - logr) : -1; }
constexpr int tib_xpad(int logr, int tl) {
  return logr == 8 ? (tl == 10 ? 2 : tl == 11 ? 5 : 1) : logr == 7 ? (tl == 10 ? 5 : 1) : 2;
}

template <int LOGR, int TL>
using TibGeo = Geo<LOGR, TL, tib_xpad(LOGR, TL), tib_pad(LOGR, TL)>;

template <int LOGR, int K>
constexpr int tib_lds_words() {
  return (K - 1) * TibGeo<LOGR, tib_tile_log(K)>::LDS_WORDS;
}

template <int LOGR, int K, int TL, bool LAZY>
__device__ __forceinline__ void tib_rounds(uint32_t* dc, size_t tpoly, uint32_t* lds, const uint2* ltw, int s0,
                                           int col0, uint32_t q) {
  using G = TibGeo<LOGR, TL>;
  using R1 = Rnd<LOGR, true, false, kThreads, TL>;  // inverse: consecutive round first
  using R2 = Rnd<LOGR, true, true, kThreads, TL>;
  const uint4 nf{};
  for (int it = threadIdx.x; it < (K - 1) * R1::ITEMS; it += kThreads) {
    const int tt = it / R1::ITEMS;
    int cc, rb, hi;
    R1::decode(it - tt * R1::ITEMS, cc, rb, hi);
    uint32_t x[R1::E];
    load_lds<R1, G>(x, lds + tt * G::LDS_WORDS, cc, rb);
    item_bfly_t<R1::RB, false, LAZY, false>(x, TwLds<G::COLS, G::RB0>{ltw, s0, cc}, s0 + R1::SL0, hi, q, nf);
    store_lds<R1, G>(x, lds + tt * G::LDS_WORDS, cc, rb);
  }
  __syncthreads();
  for (int it = threadIdx.x; it < (K - 1) * R2::ITEMS; it += kThreads) {
    const int tt = it / R2::ITEMS;
    int cc, rb, hi;
    R2::decode(it - tt * R2::ITEMS, cc, rb, hi);
    uint32_t x[R2::E];
    load_lds<R2, G>(x, lds + tt * G::LDS_WORDS, cc, rb);
    item_bfly_t<R2::RB, false, LAZY, false>(x, TwLds<G::COLS, G::RB0>{ltw, s0, cc}, s0 + R2::SL0, hi, q, nf);
    store_global<R2>(x, dc + (size_t)tt * tpoly, 0, col0 + cc, rb);
  }
}

// One tile of limb j: inp the k inputs, wsj the job's workspace with D at
// d_off ([k+1][level][N]) and the pass-B outputs at dc_off ([k-1][level][N]).
// With own.evk set, D's slots 0 and 1 receive, for each key polynomial c,
// d_c 2^32 plus the sum over t = 2..k of d_t times the key of s^t for limb
// j's own digit b, reduced mod q, instead of d_0..d_k.  In the key inner
// product a limb's own-digit pairs need no transform (the ModUp image of d_t
// on its own digit is d_t itself), so they are summed here, where d_t is at
// hand, rather than read back from HBM by the key-product kernel; d_c 2^32
// becomes d_c after that kernel's final Montgomery step, which is where the
// relocated ModDown adds it.
template <int LOGR, int K, int TM>
__device__ __forceinline__ void tensor_ib_tile(const uint32_t* const (&inp)[K], int level, int log_n, int j,
                                               int tile, uint32_t* wsj, size_t d_off, size_t dc_off,
                                               const DevTables& T, const OwnKeys& own, uint32_t* lds,
                                               uint2* ltw) {
  constexpr int TL = tib_tile_log(K);
  constexpr int STEPS = 1 << (TL - 10);  // uint4 groups per thread
  using G = TibGeo<LOGR, TL>;
  const size_t N = (size_t)1 << log_n;
  const int s0 = log_n - LOGR;
  const int col0 = tile * G::COLS;
  const uint2* itw = reinterpret_cast<const uint2*>(T.itw) + ((size_t)j << log_n);
  stage_tw_pass_b<G::COLS, LOGR, kThreads, G::RB0>(ltw, itw, s0, col0);
  uint32_t* D = wsj + d_off + (size_t)j * N;
  const size_t tpoly = (size_t)level * N;
  for (int g = 0; g < STEPS; g++) {
    const int local = g * kThreads + threadIdx.x;  // uint4 index within the tile
    const size_t n = (size_t)tile * (STEPS * kThreads) + local;
    uint4 P[K + 1];
    tensor4_by<K, TM>(inp, level, log_n, j, n, T, P);
    if (own.evk != nullptr) {
      // d_c 2^32 (below 2^62) and at most 11 products of canonical residues
      // below 2^30 per sum: exact in 64 bits, reduced once
      const int b = j / own.alpha;
      uint64_t s0[4] = {(uint64_t)P[0].x << 32, (uint64_t)P[0].y << 32, (uint64_t)P[0].z << 32,
                        (uint64_t)P[0].w << 32};
      uint64_t s1[4] = {(uint64_t)P[1].x << 32, (uint64_t)P[1].y << 32, (uint64_t)P[1].z << 32,
                        (uint64_t)P[1].w << 32};
#pragma unroll
      for (int t = 2; t <= K; t++) {
        const uint32_t* kp =
            own.evk + (((size_t)(t - 2) * own.dnum + b) * 2) * (size_t)own.key_poly + (size_t)j * N;
        const uint4 a0 = reinterpret_cast<const uint4*>(kp)[n];
        const uint4 a1 = reinterpret_cast<const uint4*>(kp + own.key_poly)[n];
        s0[0] += (uint64_t)P[t].x * a0.x;
        s0[1] += (uint64_t)P[t].y * a0.y;
        s0[2] += (uint64_t)P[t].z * a0.z;
        s0[3] += (uint64_t)P[t].w * a0.w;
        s1[0] += (uint64_t)P[t].x * a1.x;
        s1[1] += (uint64_t)P[t].y * a1.y;
        s1[2] += (uint64_t)P[t].z * a1.z;
        s1[3] += (uint64_t)P[t].w * a1.w;
      }
      const Red64& rd = T.red[j];
      const uint4 o0{reduce64(s0[0], rd), reduce64(s0[1], rd), reduce64(s0[2], rd), reduce64(s0[3], rd)};
      const uint4 o1{reduce64(s1[0], rd), reduce64(s1[1], rd), reduce64(s1[2], rd), reduce64(s1[3], rd)};
      reinterpret_cast<uint4*>(D)[n] = o0;
      reinterpret_cast<uint4*>(D + tpoly)[n] = o1;
    } else {
#pragma unroll
      for (int t = 0; t <= K; t++) reinterpret_cast<uint4*>(D + (size_t)t * tpoly)[n] = P[t];
    }
    // residues 4 local .. 4 local + 3: one 2^LOGR-residue block (column c)
    const int e = 4 * local;
    // (four rows of one row block: 2^RB1 >= 8)
    const int o = G::off(e & ((1 << LOGR) - 1), e >> LOGR);
#pragma unroll
    for (int t = 2; t <= K; t++) {
      uint32_t* tl = lds + (t - 2) * G::LDS_WORDS + o;
      tl[0] = P[t].x;
      tl[G::PAD] = P[t].y;
      tl[2 * G::PAD] = P[t].z;
      tl[3 * G::PAD] = P[t].w;
    }
  }
  __syncthreads();  // d_t tiles and staged twiddles
  uint32_t* dc = wsj + dc_off + (size_t)j * N;
  const uint32_t q = T.mod[j];
  if (q < (1u << 30))
    tib_rounds<LOGR, K, TL, true>(dc, tpoly, lds, ltw, s0, col0, q);
  else
    tib_rounds<LOGR, K, TL, false>(dc, tpoly, lds, ltw, s0, col0, q);
}

// Grid: ceil(level tiles / 8) 8 n_jobs workgroups over (limb, tile) units
// and jobs; per job ws_job words of workspace.  Block b runs on XCD b mod 8,
// and the jobs of one unit follow each other there, so all but the first
// read the unit's staged twiddles from that XCD's L2.
template <int LOGR, int K, int TM>
__global__ __launch_bounds__(kThreads) void k_tensor_ib(CtPtrs in, long long in_job_stride, int level, int log_n,
                                                        uint32_t* ws, long long ws_job, long long d_off,
                                                        long long dc_off, int n_jobs, OwnKeys own, DevTables T) {
  __shared__ uint32_t lds[tib_lds_words<LOGR, K>()];
  __shared__ uint2 ltw[TibGeo<LOGR, tib_tile_log(K)>::COLS * ((1 << LOGR) - 1)];
  const int xcd = blockIdx.x & 7, seq = blockIdx.x >> 3;
  const int job = seq % n_jobs;
  const int unit = (seq / n_jobs) * 8 + xcd;
  const int tiles = 1 << (log_n - tib_tile_log(K));
  if (unit >= level * tiles) return;  // the last group's padding
  const int j = unit / tiles, tile = unit - j * tiles;
  const size_t job_in = (size_t)job * (size_t)in_job_stride;
  const uint32_t* inp[K];
#pragma unroll
  for (int u = 0; u < K; u++) inp[u] = in.p[u] + job_in;
  tensor_ib_tile<LOGR, K, TM>(inp, level, log_n, j, tile, ws + (size_t)job * (size_t)ws_job, (size_t)d_off,
                              (size_t)dc_off, T, own, lds, ltw);
}

// Job-table form: jobs [j0, j0 + nj) of equal k, sorted by level
// (descending); blocks in the job-adjacent order of seg_block over the
// run's (limb, tile) units, so that the jobs of one unit run back to back on
// one XCD and share its twiddles and key words in L2.  D and the pass-B outputs at their places in
// the job's workspace (WsLayout).
template <int LOGR, int K, int TM>
__global__ __launch_bounds__(kThreads) void k_tensor_ib_jt(const JobDesc* jt, int j0, int nj, int log_n,
                                                           OwnKeys own, DevTables T) {
  __shared__ uint32_t lds[tib_lds_words<LOGR, K>()];
  __shared__ uint2 ltw[TibGeo<LOGR, tib_tile_log(K)>::COLS * ((1 << LOGR) - 1)];
  int rank, local;
  seg_block<0>(jt + j0, nj, blockIdx.x, rank, local);
  const int j = j0 + rank;  // the run is in rank order
  const int tiles = 1 << (log_n - tib_tile_log(K));
  const int level = jt[j].level;
  if (local >= tiles * level) return;  // the job's last group's padding
  const uint32_t* inp[K];
#pragma unroll
  for (int u = 0; u < K; u++) inp[u] = jt[j].in[u];
  const size_t N = (size_t)1 << log_n;
  tensor_ib_tile<LOGR, K, TM>(inp, level, log_n, local / tiles, local % tiles, jt[j].ws, 0,
                              (size_t)(K + 1) * level * N, T, own, lds, ltw);
}

}  // namespace

// The tensor-product form (rns.h TensorMethod) is a template parameter of
// the fused kernels, chosen per parameter set (mick_params_set_tensor_method).
#define MICK_TIB_TM(LR, KK, KERNEL, ARGS, GRID)                                     \
  switch (prm->tensor_method) {                                                     \
    case kTensorTree: KERNEL<LR, KK, kTensorTree><<<GRID, kThreads, 0, s>>> ARGS; break;     \
    case kTensorFilter: KERNEL<LR, KK, kTensorFilter><<<GRID, kThreads, 0, s>>> ARGS; break; \
    default: KERNEL<LR, KK, kTensorChain><<<GRID, kThreads, 0, s>>> ARGS; break;           \
  }

int launch_tensor_ib(const mick_params* prm, const CtPtrs& in, long long in_job_stride, int k, int level,
                     uint32_t* ws, long long ws_job, long long d_off, long long dc_off, int n_jobs,
                     const OwnKeys& own, hipStream_t s) {
  const long long units = (long long)(prm->N >> tib_tile_log(k)) * level;
  dim3 grid((unsigned)(((units + 7) / 8) * 8 * n_jobs));
  const DevTables& T = prm->dt;
  const int ln = prm->log_n;
  ProfScope ps(P_TENSOR_IB, s);
#define MICK_TIB(LR, KK) \
  MICK_TIB_TM(LR, KK, k_tensor_ib, (in, in_job_stride, level, ln, ws, ws_job, d_off, dc_off, n_jobs, own, T), grid)
#define MICK_TIB_K(LR)                                                   \
  switch (k) {                                                           \
    case 2: MICK_TIB(LR, 2); break;                                      \
    case 3: MICK_TIB(LR, 3); break;                                      \
    case 4: MICK_TIB(LR, 4); break;                                      \
    case 5: MICK_TIB(LR, 5); break;                                      \
    case 6: MICK_TIB(LR, 6); break;                                      \
    case 7: MICK_TIB(LR, 7); break;                                      \
    case 8: MICK_TIB(LR, 8); break;                                      \
    case 9: MICK_TIB(LR, 9); break;                                      \
    case 10: MICK_TIB(LR, 10); break;                                    \
    case 11: MICK_TIB(LR, 11); break;                                    \
    case 12: MICK_TIB(LR, 12); break;                                    \
    default: return set_error(MICK_E_ARG, "k out of range");            \
  }
  switch (prm->split_b) {
    case 6: MICK_TIB_K(6) break;
    case 7: MICK_TIB_K(7) break;
    case 8: MICK_TIB_K(8) break;
    default: return set_error(MICK_E_ARG, "pass split out of range");
  }
#undef MICK_TIB_K
#undef MICK_TIB
  return hip_error(hipGetLastError(), "tensor + pass B launch");
}

int launch_tensor_ib_jt(const mick_params* prm, const JobDesc* jt, int j0, int nj, int k, int blocks,
                        const OwnKeys& own, hipStream_t s) {
  if (blocks <= 0) return MICK_OK;
  const DevTables& T = prm->dt;
  const int ln = prm->log_n;
  ProfScope ps(P_TENSOR_IB, s);
#define MICK_TIB(LR, KK) MICK_TIB_TM(LR, KK, k_tensor_ib_jt, (jt, j0, nj, ln, own, T), blocks)
#define MICK_TIB_K(LR)                                                   \
  switch (k) {                                                           \
    case 2: MICK_TIB(LR, 2); break;                                      \
    case 3: MICK_TIB(LR, 3); break;                                      \
    case 4: MICK_TIB(LR, 4); break;                                      \
    case 5: MICK_TIB(LR, 5); break;                                      \
    case 6: MICK_TIB(LR, 6); break;                                      \
    case 7: MICK_TIB(LR, 7); break;                                      \
    case 8: MICK_TIB(LR, 8); break;                                      \
    case 9: MICK_TIB(LR, 9); break;                                      \
    case 10: MICK_TIB(LR, 10); break;                                    \
    case 11: MICK_TIB(LR, 11); break;                                    \
    case 12: MICK_TIB(LR, 12); break;                                    \
    default: return set_error(MICK_E_ARG, "k out of range");            \
  }
  switch (prm->split_b) {
    case 6: MICK_TIB_K(6) break;
    case 7: MICK_TIB_K(7) break;
    case 8: MICK_TIB_K(8) break;
    default: return set_error(MICK_E_ARG, "pass split out of range");
  }
#undef MICK_TIB_K
#undef MICK_TIB
  return hip_error(hipGetLastError(), "tensor + pass B launch");
}

}  // namespace mick
