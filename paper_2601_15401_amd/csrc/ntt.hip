// Negacyclic NTT / INTT for N = 2^13 .. 2^16 on gfx950, and the two fused
// kernels of the ModUp path that are built on the same transform passes.
//
// The transform passes are built from ntt_core.h; the fused tensor-product
// kernel is in tensor.hip.
//
//
// ModUp fusion (Sec. II ModUp, Sec. III combined key products):
//  * k_modup_a: the fast basis conversion of eq. (basis conversion) computed
//    while loading pass A of the forward transform of each new limb, so the
//    converted limbs are never written in the coefficient domain.  The input
//    limbs already carry the factor qhat_j^-1 (merged into the inverse
//    transform that produced them).
//  * k_kip_b: pass B of those forward transforms fused with the key inner
//    product: one workgroup owns one tile of one extended-basis limb and
//    accumulates sum_t sum_b X_{t,b} ek'_{t,b,l} over every (t, b) pair in
//    registers, reusing the limb's pass-B twiddles for all pairs; the
//    transformed limbs are never written.  The finished accumulator tile is
//    already in the inverse transform's first-round layout, so the first
//    pass (pass B) of the accumulators' INTT (Sec. IV relocated ModDown)
//    runs in the same kernel and only its output is written.
#include "ntt_core.h"

namespace mick {

namespace {

// ------------------------------------------------------------------ plain transform pass

// ltwa: LDS twiddles (pass_tw_words) for the second round, which would
// otherwise read per-thread twiddles right after the barrier: the forward
// pass A (its first round's are uniform per wave) and the inverse pass B.
template <int LOGR, bool FWD, bool LAZY, bool PASSB>
__device__ __forceinline__ void pass_body(const uint32_t* src, uint32_t* dst, uint32_t* lds, uint2* ltwa, int s0,
                                          int H, int col0, uint32_t q, const uint2* tw, const uint4& nfix) {
  using G = Geo<LOGR>;
  // forward: strided round first; inverse: consecutive round first
  using R1 = Rnd<LOGR, PASSB, FWD>;
  using R2 = Rnd<LOGR, PASSB, !FWD>;
  constexpr bool FINAL = FWD ? PASSB : !PASSB;  // last pass of the transform
  constexpr bool STAGED = FWD && !PASSB;
  constexpr bool STAGED_B = !FWD && PASSB && LOGR == 8;
  if constexpr (STAGED) stage_tw_pass_a<LOGR>(ltwa, tw);
  if constexpr (STAGED_B) stage_tw_pass_b<G::COLS, G::RB0, kThreads, G::RB0>(ltwa, tw, s0, col0);
#pragma unroll
  for (int i = 0; i < R1::NI; i++) {
    int c, rb, hi;
    R1::decode(i * kThreads + threadIdx.x, c, rb, hi);
    uint32_t x[R1::E];
    load_global<R1>(x, src, H, col0 + c, rb);
    item_bfly<R1::RB, FWD, LAZY, false>(x, tw, s0 + R1::SL0, s0, hi, PASSB ? col0 + c : 0, q, nfix);
    store_lds<R1, G>(x, lds, c, rb);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < R2::NI; i++) {
    int c, rb, hi;
    R2::decode(i * kThreads + threadIdx.x, c, rb, hi);
    uint32_t x[R2::E];
    load_lds<R2, G>(x, lds, c, rb);
    // the inverse's strided round of pass A holds global stage 0
    if constexpr (STAGED)
      item_bfly_t<R2::RB, FWD, LAZY, false>(x, TwPassA{ltwa}, R2::SL0, hi, q, nfix);
    else if constexpr (STAGED_B)
      item_bfly_t<R2::RB, FWD, LAZY, false>(x, TwLds<G::COLS, G::RB0>{ltwa, s0, c}, s0 + R2::SL0, hi, q, nfix);
    else
      item_bfly<R2::RB, FWD, LAZY, !FWD && !PASSB>(x, tw, s0 + R2::SL0, s0, hi, PASSB ? col0 + c : 0, q, nfix);
    if constexpr (FINAL) {
#pragma unroll
      for (int j = 0; j < R2::E; j++) x[j] = canonical<FWD, LAZY>(x[j], q);
    }
    store_global<R2>(x, dst, H, col0 + c, rb);
  }
}

// Launch index y -> limb: group g = y / period, position pos = y % period.
__device__ __forceinline__ void resolve(const LimbMap& mp, int limb, int log_n, int& prime, int& pos, size_t& off) {
  const int g = limb / mp.period;
  pos = limb - g * mp.period;
  prime = pos < mp.split ? pos + mp.off_lo : pos + mp.off_hi;
  off = (size_t)g * (size_t)mp.group_stride + ((size_t)pos << log_n) + (size_t)blockIdx.z * (size_t)mp.job_stride;
}

template <int LOGR, bool FWD, bool PASSB>
__global__ __launch_bounds__(kThreads) void k_ntt_pass(const uint32_t* src, uint32_t* dst, LimbMap mp, DevTables T,
                                                       int log_n, int s0) {
  __shared__ uint32_t lds[Geo<LOGR>::LDS_WORDS];
  __shared__ uint2 ltwa[pass_tw_words<LOGR, FWD, PASSB>()];
  int prime, pos;
  size_t off;
  resolve(mp, blockIdx.y, log_n, prime, pos, off);
  const uint32_t q = T.mod[prime];
  const uint2* tw = reinterpret_cast<const uint2*>(FWD ? T.tw : T.itw) + ((size_t)prime << log_n);
  const uint4 nfix = mp.nfix_pos ? reinterpret_cast<const uint4*>(mp.nfix_pos)[pos]
                                 : reinterpret_cast<const uint4*>(T.nfix)[prime];
  const int H = log_n - s0 - LOGR;  // > 0 in pass A, 0 in pass B
  const int col0 = blockIdx.x * Geo<LOGR>::COLS;
  if (q < (1u << 30))
    pass_body<LOGR, FWD, true, PASSB>(src + off, dst + off, lds, ltwa, s0, H, col0, q, tw, nfix);
  else
    pass_body<LOGR, FWD, false, PASSB>(src + off, dst + off, lds, ltwa, s0, H, col0, q, tw, nfix);
}

template <bool FWD, bool PASSB>
void launch_pass(int logr, dim3 grid, hipStream_t s, const uint32_t* src, uint32_t* dst, const LimbMap& mp,
                 const DevTables& T, int log_n, int s0, int site) {
  ProfScope ps(site, s);
  switch (logr) {
    case 6: k_ntt_pass<6, FWD, PASSB><<<grid, kThreads, 0, s>>>(src, dst, mp, T, log_n, s0); break;
    case 7: k_ntt_pass<7, FWD, PASSB><<<grid, kThreads, 0, s>>>(src, dst, mp, T, log_n, s0); break;
    default: k_ntt_pass<8, FWD, PASSB><<<grid, kThreads, 0, s>>>(src, dst, mp, T, log_n, s0); break;
  }
}

// ------------------------------------------------------------------ ModUp: conversion + pass A

// 32 elements per thread on tiles of 2^kModupTileLog elements.  Unlike the
// key-product kernel, ModUp loses with narrower tiles: its source rows are
// read a tile row at a time, and a 4096- or 2048-element tile reads 64- or
// 32-byte row segments (1262 us per eight-job launch at 8192 elements, 1503
// at 4096, 2322 at 2048).
constexpr int kModupThreads = 1 << (kModupTileLog - 5);

// Workgroup order: the targets of one source tile run back to back on one
// XCD (block b goes to XCD b % 8), so the source tile is read from L2.
// One target per workgroup, except at digits of 5 to 8 primes, which take
// two (k_modup_a2, k_modup_a2_jt).
// The conversion constants carry a factor R = 2^32 (Montgomery form): the
// sum of up to 8 products of a residue below 2^30 and a constant below m
// stays below 2m 2^32, so one Montgomery reduction returns it mod m (wider
// digits reduce every eight rows).
template <int LOGR, int ALPHA, bool LAZY>
__device__ __forceinline__ void modup_a_body(__amdgpu_buffer_rsrc_t src, int na, const uint32_t (&cc)[ALPHA],
                                             uint32_t minv, uint32_t* dst, uint32_t* lds, uint2* ltwa, int H,
                                             int col0, uint32_t q, const uint2* tw) {
  using G = Geo<LOGR, kModupTileLog>;
  using R1 = Rnd<LOGR, false, true, kModupThreads, kModupTileLog>;
  using R2 = Rnd<LOGR, false, false, kModupThreads, kModupTileLog>;
  const uint4 nf{};
  // the second round's twiddles vary per thread: read from LDS after the barrier
  stage_tw_pass_a<LOGR, kModupThreads>(ltwa, tw);
  // the item's rows are 2^NLO_LOG rows apart: a uniform byte step per j
  constexpr uint32_t kRowStep = 4u << R1::NLO_LOG;
  const uint32_t row_bytes = 4u << (H + LOGR);  // one source limb
#pragma unroll
  for (int i = 0; i < R1::NI; i++) {
    int c, rb, hi;
    R1::decode(i * kModupThreads + threadIdx.x, c, rb, hi);
    const uint32_t voff = 4u * R1::gidx(H, col0 + c, R1::row(rb, 0));
    uint32_t vj[R1::E];  // lane offsets of the item's positions in one limb
#pragma unroll
    for (int j = 0; j < R1::E; j++) vj[j] = voff + ((uint32_t)j * kRowStep << H);
    uint64_t acc[R1::E];
#pragma unroll
    for (int j = 0; j < R1::E; j++) acc[j] = 0;
    // source row outermost, double-buffered: the E independent loads of row
    // a + 1 are in flight while row a is accumulated (padded rows reread a
    // valid limb and are multiplied by 0)
    uint32_t v[2][R1::E];
#pragma unroll
    for (int j = 0; j < R1::E; j++) v[0][j] = __builtin_amdgcn_raw_buffer_load_b32(src, vj[j], 0, 0);
    // more than eight rows: every eight rows' sum (below 2m 2^32) is reduced
    // and the partial results are added mod q
    uint32_t part[ALPHA > 8 ? R1::E : 1];
#pragma unroll
    for (int j = 0; j < (ALPHA > 8 ? R1::E : 1); j++) part[j] = 0;
#pragma unroll
    for (int a = 0; a < ALPHA; a++) {
      if (a + 1 < ALPHA) {
        const uint32_t soff = (uint32_t)min(a + 1, na - 1) * row_bytes;
#pragma unroll
        for (int j = 0; j < R1::E; j++)
          v[(a + 1) & 1][j] = __builtin_amdgcn_raw_buffer_load_b32(src, vj[j], soff, 0);
      }
#pragma unroll
      for (int j = 0; j < R1::E; j++) acc[j] += (uint64_t)v[a & 1][j] * cc[a];
      if constexpr (ALPHA > 8) {
        if ((a & 7) == 7 && a + 1 < ALPHA) {
#pragma unroll
          for (int j = 0; j < R1::E; j++) {
            part[j] = add_mod(part[j], redc_2m(acc[j], q, minv), q);
            acc[j] = 0;
          }
        }
      }
    }
    // the lazy butterflies take values below 4q: the sum's reduction stays
    // lazy there (below 3q); the 31-bit primes and the chunked sums of wide
    // digits need it canonical
    uint32_t x[R1::E];
#pragma unroll
    for (int j = 0; j < R1::E; j++) {
      if constexpr (LAZY && ALPHA <= 8)
        x[j] = redc_lazy(acc[j], q, minv);
      else
        x[j] = redc_2m(acc[j], q, minv);
      if constexpr (ALPHA > 8) x[j] = add_mod(part[j], x[j], q);
    }
    item_bfly<R1::RB, true, LAZY, false>(x, tw, R1::SL0, 0, hi, 0, q, nf);
    store_lds<R1, G>(x, lds, c, rb);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < R2::NI; i++) {
    int c, rb, hi;
    R2::decode(i * kModupThreads + threadIdx.x, c, rb, hi);
    uint32_t x[R2::E];
    load_lds<R2, G>(x, lds, c, rb);
    item_bfly_t<R2::RB, true, LAZY, false>(x, TwPassA{ltwa}, R2::SL0, hi, q, nf);
    store_global<R2>(x, dst, H, col0 + c, rb);
  }
}

// Raw buffer descriptor over `bytes` bytes at `base` (gfx9 word 3: 32-bit
// data format, no swizzle, no stride).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <int LOGR, int ALPHA>
__global__ __launch_bounds__(kModupThreads) void k_modup_a(const uint32_t* dsc, uint32_t* X, ModupArgs A,
                                                           DevTables T) {
  __shared__ uint32_t lds[Geo<LOGR, kModupTileLog>::LDS_WORDS];
  __shared__ uint2 ltwa[1 << LOGR];
  const int xcd = blockIdx.x & 7, seq = blockIdx.x >> 3;
  const int e = seq % A.E;
  const int unit = (seq / A.E) * 8 + xcd;  // (job, t, b, tile)
  if (unit >= A.units) return;
  const int tile = unit % A.tiles;
  const int src_grp = unit / A.tiles;
  const int job = src_grp / A.groups;
  const int tb = src_grp - job * A.groups;  // (t - 2) * B + b
  const int t2 = tb / A.B, b = tb - t2 * A.B;
  const int lo = b * A.alpha;
  const int na = min(A.alpha, A.level - lo);
  if (e >= lo && e < lo + na) return;  // the digit's own limbs are the input itself
  const int pe = e < A.level ? e : A.L + (e - A.level);
  const uint32_t q = T.mod[pe], minv = T.minv[pe];
  const uint2* tw = reinterpret_cast<const uint2*>(T.tw) + ((size_t)pe << A.log_n);
  const size_t N = (size_t)1 << A.log_n;
  // [ALPHA][E] qhat_j R mod m_e, zero rows padded
  const uint32_t* C = A.tab + A.tab_off[b] + 2 * ALPHA;
  const uint32_t* base = dsc + (size_t)job * (size_t)A.dcoef_job + ((size_t)t2 * A.level + lo) * N;
  const __amdgpu_buffer_rsrc_t src = buffer_rsrc(base, (uint32_t)(na * N * 4));
  uint32_t cc[ALPHA];
#pragma unroll
  for (int a = 0; a < ALPHA; a++) cc[a] = C[a * A.E + e];
  uint32_t* dst = X + (size_t)job * (size_t)A.x_job + ((size_t)tb * A.E + e) * N;
  const int H = A.log_n - LOGR;
  const int col0 = tile * Geo<LOGR, kModupTileLog>::COLS;
  if (q < (1u << 30))
    modup_a_body<LOGR, ALPHA, true>(src, na, cc, minv, dst, lds, ltwa, H, col0, q, tw);
  else
    modup_a_body<LOGR, ALPHA, false>(src, na, cc, minv, dst, lds, ltwa, H, col0, q, tw);
}

// Two targets per workgroup: each source word loaded feeds both targets'
// conversions, which halves the source traffic through L1.  The first
// target's pass runs through the LDS tile while the second target's
// converted values wait in registers; then the second target's pass.
template <int LOGR, int ALPHA, bool LAZY>
__device__ __forceinline__ void modup_a2_body(__amdgpu_buffer_rsrc_t src, int na, const uint32_t (&c0)[ALPHA],
                                              const uint32_t (&c1)[ALPHA], uint32_t minv0, uint32_t minv1,
                                              uint32_t* dst0, uint32_t* dst1, uint32_t* lds, uint2* ltw0, uint2* ltw1,
                                              int H, int col0, uint32_t q0, uint32_t q1, const uint2* tw0,
                                              const uint2* tw1) {
  using G = Geo<LOGR, kModupTileLog>;
  using R1 = Rnd<LOGR, false, true, kModupThreads, kModupTileLog>;
  using R2 = Rnd<LOGR, false, false, kModupThreads, kModupTileLog>;
  static_assert(ALPHA == 8, "eight rows: one reduction per sum");
  const uint4 nf{};
  stage_tw_pass_a<LOGR, kModupThreads>(ltw0, tw0);
  stage_tw_pass_a<LOGR, kModupThreads>(ltw1, tw1);
  constexpr uint32_t kRowStep = 4u << R1::NLO_LOG;
  const uint32_t row_bytes = 4u << (H + LOGR);
  uint32_t y1[R1::NI][R1::E];
#pragma unroll
  for (int i = 0; i < R1::NI; i++) {
    int c, rb, hi;
    R1::decode(i * kModupThreads + threadIdx.x, c, rb, hi);
    const uint32_t voff = 4u * R1::gidx(H, col0 + c, R1::row(rb, 0));
    uint32_t vj[R1::E];
#pragma unroll
    for (int j = 0; j < R1::E; j++) vj[j] = voff + ((uint32_t)j * kRowStep << H);
    uint64_t a0[R1::E], a1[R1::E];
#pragma unroll
    for (int j = 0; j < R1::E; j++) a0[j] = a1[j] = 0;
    uint32_t v[2][R1::E];
#pragma unroll
    for (int j = 0; j < R1::E; j++) v[0][j] = __builtin_amdgcn_raw_buffer_load_b32(src, vj[j], 0, 0);
#pragma unroll
    for (int a = 0; a < ALPHA; a++) {
      if (a + 1 < ALPHA) {
        const uint32_t soff = (uint32_t)min(a + 1, na - 1) * row_bytes;
#pragma unroll
        for (int j = 0; j < R1::E; j++)
          v[(a + 1) & 1][j] = __builtin_amdgcn_raw_buffer_load_b32(src, vj[j], soff, 0);
      }
#pragma unroll
      for (int j = 0; j < R1::E; j++) {
        a0[j] += (uint64_t)v[a & 1][j] * c0[a];
        a1[j] += (uint64_t)v[a & 1][j] * c1[a];
        // both sums advance with the row (the optimiser would otherwise
        // finish one chain first and keep every source word for the other)
        asm volatile("" : "+v"(a0[j]), "+v"(a1[j]));
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    uint32_t x[R1::E];
#pragma unroll
    for (int j = 0; j < R1::E; j++) {
      // lazy reductions (below 3q) feed the lazy butterflies
      if constexpr (LAZY) {
        x[j] = redc_lazy(a0[j], q0, minv0);
        y1[i][j] = redc_lazy(a1[j], q1, minv1);
      } else {
        x[j] = redc_2m(a0[j], q0, minv0);
        y1[i][j] = redc_2m(a1[j], q1, minv1);
      }
      asm volatile("" : "+v"(x[j]), "+v"(y1[i][j]));  // both sums reduced before the butterflies
    }
    __builtin_amdgcn_sched_barrier(0);
    item_bfly<R1::RB, true, LAZY, false>(x, tw0, R1::SL0, 0, hi, 0, q0, nf);
    store_lds<R1, G>(x, lds, c, rb);
    __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < R2::NI; i++) {
    int c, rb, hi;
    R2::decode(i * kModupThreads + threadIdx.x, c, rb, hi);
    uint32_t x[R2::E];
    load_lds<R2, G>(x, lds, c, rb);
    item_bfly_t<R2::RB, true, LAZY, false>(x, TwPassA{ltw0}, R2::SL0, hi, q0, nf);
    store_global<R2>(x, dst0, H, col0 + c, rb);
  }
  if (!dst1) return;  // uniform: an odd target count leaves one alone
  // The second target's LDS addresses are those of the first: an opaque
  // copy of the thread index makes the compiler recompute them here rather
  // than hold them (in scratch) across both passes.
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  __syncthreads();
#pragma unroll
  for (int i = 0; i < R1::NI; i++) {
    int c, rb, hi;
    R1::decode(i * kModupThreads + tid, c, rb, hi);
    // the second target's first round runs here: its twiddles are not live
    // through the first target's pass
    item_bfly<R1::RB, true, LAZY, false>(y1[i], tw1, R1::SL0, 0, hi, 0, q1, nf);
    store_lds<R1, G>(y1[i], lds, c, rb);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < R2::NI; i++) {
    int c, rb, hi;
    R2::decode(i * kModupThreads + tid, c, rb, hi);
    uint32_t x[R2::E];
    load_lds<R2, G>(x, lds, c, rb);
    item_bfly_t<R2::RB, true, LAZY, false>(x, TwPassA{ltw1}, R2::SL0, hi, q1, nf);
    store_global<R2>(x, dst1, H, col0 + c, rb);
  }
}

// Digits of 5 to 8 primes.  Target pairs of one source
// tile: the digit's q targets (every q limb outside the digit) two by two,
// then the special primes two by two, so both members of a pair take the
// same lazy or canonical butterflies.  modup_pairs() pairs per unit is an
// upper bound; the unused ones return, and an odd group's last target is
// alone (e1 < 0).
// Three waves per SIMD: 148 VGPRs (both targets' 64-bit sums, the next
// source row, the second target's converted values) and no scratch.  Per
// eight-job launch at the eight-input shape: 1277 us for the one-target
// kernel at four waves, 1085 us here; forced to four waves this kernel
// spills and takes 1169 us.
template <int LOGR, int ALPHA>
__global__ __launch_bounds__(kModupThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_modup_a2(
    const uint32_t* dsc, uint32_t* X, ModupArgs A, DevTables T) {
  __shared__ uint32_t lds[Geo<LOGR, kModupTileLog>::LDS_WORDS];
  __shared__ uint2 ltw[2][1 << LOGR];
  const int pairs = modup_pairs(A.level, A.E);
  const int xcd = blockIdx.x & 7, seq = blockIdx.x >> 3;
  const int pr = seq % pairs;
  const int unit = (seq / pairs) * 8 + xcd;  // (job, t, b, tile)
  if (unit >= A.units) return;
  const int tile = unit % A.tiles;
  const int src_grp = unit / A.tiles;
  const int job = src_grp / A.groups;
  const int tb = src_grp - job * A.groups;  // (t - 2) * B + b
  const int t2 = tb / A.B, b = tb - t2 * A.B;
  const int lo = b * A.alpha;
  const int na = min(A.alpha, A.level - lo);
  const int nq = A.level - na;
  const int qp = (nq + 1) / 2;
  int e0, e1;
  if (pr < qp) {
    const int i0 = 2 * pr, i1 = i0 + 1;
    e0 = i0 < lo ? i0 : i0 + na;
    e1 = i1 < nq ? (i1 < lo ? i1 : i1 + na) : -1;
  } else {
    e0 = A.level + 2 * (pr - qp);
    if (e0 >= A.E) return;
    e1 = e0 + 1 < A.E ? e0 + 1 : -1;
  }
  const bool two = e1 >= 0;
  const int f1 = two ? e1 : e0;
  const int p0 = e0 < A.level ? e0 : A.L + (e0 - A.level);
  const int p1 = f1 < A.level ? f1 : A.L + (f1 - A.level);
  const uint32_t q0 = T.mod[p0], q1 = T.mod[p1];
  const uint2* tw0 = reinterpret_cast<const uint2*>(T.tw) + ((size_t)p0 << A.log_n);
  const uint2* tw1 = reinterpret_cast<const uint2*>(T.tw) + ((size_t)p1 << A.log_n);
  const size_t N = (size_t)1 << A.log_n;
  const uint32_t* C = A.tab + A.tab_off[b] + 2 * ALPHA;
  const uint32_t* base = dsc + (size_t)job * (size_t)A.dcoef_job + ((size_t)t2 * A.level + lo) * N;
  const __amdgpu_buffer_rsrc_t src = buffer_rsrc(base, (uint32_t)(na * N * 4));
  uint32_t c0[ALPHA], c1[ALPHA];
#pragma unroll
  for (int a = 0; a < ALPHA; a++) {
    c0[a] = C[a * A.E + e0];
    c1[a] = C[a * A.E + f1];
  }
  uint32_t* xj = X + (size_t)job * (size_t)A.x_job + (size_t)tb * A.E * N;
  uint32_t* dst0 = xj + (size_t)e0 * N;
  uint32_t* dst1 = two ? xj + (size_t)e1 * N : nullptr;
  const int H = A.log_n - LOGR;
  const int col0 = tile * Geo<LOGR, kModupTileLog>::COLS;
  if (q0 < (1u << 30) && q1 < (1u << 30))
    modup_a2_body<LOGR, ALPHA, true>(src, na, c0, c1, T.minv[p0], T.minv[p1], dst0, dst1, lds, ltw[0], ltw[1], H,
                                     col0, q0, q1, tw0, tw1);
  else
    modup_a2_body<LOGR, ALPHA, false>(src, na, c0, c1, T.minv[p0], T.minv[p1], dst0, dst1, lds, ltw[0], ltw[1], H,
                                      col0, q0, q1, tw0, tw1);
}

// ------------------------------------------------------------------ pass B + key inner product

// One wave per workgroup on 1024-element tiles: the pair loop's barriers
// involve a single wave, and eight workgroups share a CU, which is what its
// 219-245 VGPRs allow.  (8192-element tiles with 512 threads: 1121 us per
// eight-job launch; 4096 / 256: 1075; 2048 / 128: 996; 1024 / 64: 955.)
constexpr int kKipThreads = 64;

// The tile, then the staged twiddles (COLS (2^LOGR - 1) pairs), which the
// second accumulator's tile reuses once the pair loop is done.
template <int LOGR>
constexpr int kip_lds_words() {
  using G = Geo<LOGR, kKipTileLog>;
  constexpr int tw_words = 2 * G::COLS * ((1 << LOGR) - 1);
  static_assert(tw_words >= G::LDS_WORDS, "the twiddle area holds a tile");
  static_assert(G::LDS_WORDS % 4 == 0, "16-byte aligned twiddles");
  return G::LDS_WORDS + tw_words;
}

template <int LOGR, bool LAZY>
__device__ __forceinline__ void kip_b_body(const uint32_t* Xe, const uint32_t* De, const uint32_t* evk_e,
                                           uint32_t* acc_e, const KipArgs& A, uint32_t* lds, uint2* ltw, int e,
                                           int col0, uint32_t q, uint32_t minv, const Red64& red, const uint2* tw,
                                           const uint2* itw) {
  using G = Geo<LOGR, kKipTileLog>;
  using R1 = Rnd<LOGR, true, true, kKipThreads, kKipTileLog>;
  using R2 = Rnd<LOGR, true, false, kKipThreads, kKipTileLog>;
  constexpr int V = R1::NI * R1::E;  // words of the tile held by one thread
  static_assert(V == R2::NI * R2::E, "both rounds cover the tile");
  const size_t N = (size_t)1 << A.log_n;
  const int s0 = A.log_n - LOGR;
  const uint4 nf{};
  // every (t, b) pair of this tile uses the same twiddles: stage them once.
  // A limb of the only digit (B = 1, e < level) is its own ModUp image in
  // every pair, so it transforms nothing and skips the staging.
  const bool transforms = A.B > 1 || e >= A.level;
  if (transforms) stage_tw_pass_b<G::COLS, LOGR, kKipThreads, G::RB0>(ltw, tw, s0, col0);
  // pairs p = (t - 2) B + b.  A pair is "own" when limb e belongs to digit b:
  // its ModUp image is D_t itself (NTT domain, second-round layout); otherwise the
  // pass-A output X_{t,b,e} is read in first-round layout.
  // A pair's position (t - 2, b) advances by counting, not by dividing
  // the pair index by B.
  struct Pos {
    int t2, b;
  };
  auto own_of = [&](Pos u) {
    const int lo = u.b * A.alpha;
    return e >= lo && e < min(lo + A.alpha, A.level);
  };
  // With the own-digit sums precomputed, a q limb's pairs of its own digit
  // (one per t) are skipped: the accumulators start from those sums.
  const bool sums = A.own_sums && e < A.level;
  const int P = (A.k - 1) * A.B - (sums ? A.k - 1 : 0);
  auto next = [&](Pos u) {
    do {
      if (++u.b == A.B) {
        u.b = 0;
        ++u.t2;
      }
    } while (sums && u.t2 < A.k - 1 && own_of(u));
    return u;
  };
  // the transform input of one pair
  auto fetch_x = [&](Pos u, uint32_t (&xv)[V]) {
    if (own_of(u)) {
      const uint32_t* d = De + (size_t)(u.t2 + 2) * A.level * N;
#pragma unroll
      for (int i = 0; i < R2::NI; i++) {
        int c, rb, hi;
        R2::decode(i * kKipThreads + threadIdx.x, c, rb, hi);
        uint32_t x[R2::E];
        load_global<R2>(x, d, 0, col0 + c, rb);
#pragma unroll
        for (int j = 0; j < R2::E; j++) xv[i * R2::E + j] = x[j];
      }
    } else {
      const uint32_t* src = Xe + (size_t)(u.t2 * A.B + u.b) * A.E * N;
#pragma unroll
      for (int i = 0; i < R1::NI; i++) {
        int c, rb, hi;
        R1::decode(i * kKipThreads + threadIdx.x, c, rb, hi);
        uint32_t x[R1::E];
        load_global<R1>(x, src, 0, col0 + c, rb);
#pragma unroll
        for (int j = 0; j < R1::E; j++) xv[i * R1::E + j] = x[j];
      }
    }
  };
  // both key words of every second-round position of this thread
  auto fetch_k = [&](Pos u, uint4 (&kv)[V / 2]) {
    const uint32_t* k0p = evk_e + (((size_t)u.t2 * A.dnum + u.b) * 2) * (size_t)A.key_poly;
    const uint32_t* k1p = k0p + A.key_poly;
#pragma unroll
    for (int i = 0; i < R2::NI; i++) {
      int c, rb, hi;
      R2::decode(i * kKipThreads + threadIdx.x, c, rb, hi);
      const uint32_t g = R2::gidx(0, col0 + c, rb);
#pragma unroll
      for (int j = 0; j < R2::E; j += 4) {
        kv[(i * R2::E + j) / 2] = *reinterpret_cast<const uint4*>(k0p + g + j);
        kv[(i * R2::E + j) / 2 + 1] = *reinterpret_cast<const uint4*>(k1p + g + j);
      }
    }
  };
  // exact sums of the products (each below 2^63) in 96 bits; reduced once
  uint64_t l0[V], l1[V];
  uint32_t h0[V], h1[V];
#pragma unroll
  for (int j = 0; j < V; j++) {
    l0[j] = l1[j] = 0;
    h0[j] = h1[j] = 0;
  }
  if (sums) {  // the own-digit sums (residues mod q), in second-round layout
#pragma unroll
    for (int i = 0; i < R2::NI; i++) {
      int c, rb, hi;
      R2::decode(i * kKipThreads + threadIdx.x, c, rb, hi);
      uint32_t o0[R2::E], o1[R2::E];
      load_global<R2>(o0, De, 0, col0 + c, rb);
      load_global<R2>(o1, De + (size_t)A.level * N, 0, col0 + c, rb);
#pragma unroll
      for (int j = 0; j < R2::E; j++) {
        l0[i * R2::E + j] = o0[j];
        l1[i * R2::E + j] = o1[j];
      }
    }
  }
  // One pair: x holds its input (transformed in place), xn receives the
  // next pair's.  The loop runs two pairs per iteration with the buffers'
  // roles swapped, so no copy carries the prefetch from one pair to the next.
  auto pair = [&](Pos u, bool more, uint32_t (&x)[V], uint32_t (&xn)[V]) {
    const bool own = own_of(u);
    // key words of this pair arrive while it is transformed; the next pair's
    // input arrives during this whole pair
    uint4 kk[V / 2];
    fetch_k(u, kk);
    if (more) fetch_x(next(u), xn);
    if (!own) {
      uint32_t* tile = lds;
#pragma unroll
      for (int i = 0; i < R1::NI; i++) {
        int c, rb, hi;
        R1::decode(i * kKipThreads + threadIdx.x, c, rb, hi);
        uint32_t y[R1::E];
#pragma unroll
        for (int j = 0; j < R1::E; j++) y[j] = x[i * R1::E + j];
        item_bfly_t<R1::RB, true, LAZY, false>(y, TwLds<G::COLS, G::RB0>{ltw, s0, c}, s0 + R1::SL0, hi, q, nf);
        store_lds<R1, G>(y, tile, c, rb);
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < R2::NI; i++) {
        int c, rb, hi;
        R2::decode(i * kKipThreads + threadIdx.x, c, rb, hi);
        uint32_t y[R2::E];
        load_lds<R2, G>(y, tile, c, rb);
        item_bfly_t<R2::RB, true, LAZY, false>(y, TwLds<G::COLS, G::RB0>{ltw, s0, c}, s0 + R2::SL0, hi, q, nf);
#pragma unroll
        for (int j = 0; j < R2::E; j++) x[i * R2::E + j] = y[j];
      }
      __syncthreads();  // the tile is read before the next pair writes it
    }
#pragma unroll
    for (int j = 0; j < V; j += 4) {
      const uint4 k0 = kk[j / 2], k1 = kk[j / 2 + 1];
      mac96x4(l0[j], h0[j], l0[j + 1], h0[j + 1], l0[j + 2], h0[j + 2], l0[j + 3], h0[j + 3], x[j], k0.x, x[j + 1],
              k0.y, x[j + 2], k0.z, x[j + 3], k0.w);
      mac96x4(l1[j], h1[j], l1[j + 1], h1[j + 1], l1[j + 2], h1[j + 2], l1[j + 3], h1[j + 3], x[j], k1.x, x[j + 1],
              k1.y, x[j + 2], k1.z, x[j + 3], k1.w);
    }
  };
  uint32_t xa[V], xb[V];
  Pos u{0, 0};
  if (sums && own_of(u)) u = next(u);
  if (P > 0) fetch_x(u, xa);
  __syncthreads();  // twiddles staged
  int p = 0;
  for (; p + 1 < P; p += 2) {
    pair(u, true, xa, xb);
    u = next(u);
    pair(u, p + 2 < P, xb, xa);
    u = next(u);
  }
  if (p < P) pair(u, false, xa, xb);
  // sum mod q, then the key's factor R = 2^32 removed by one Montgomery step
  const uint32_t r32 = red.r32, r32sh = red.r32sh;
  auto finish = [&](uint64_t lo, uint32_t hi) {
    const uint32_t th = shoup(shoup(hi, r32, r32sh, q), r32, r32sh, q);  // hi 2^64 mod q
    return mont_mul(add_mod(reduce64(lo, red), th, q), 1u, q, minv);
  };
  // The finished tile is in the layout of the inverse transform's first
  // round (pass B's consecutive round), so the first pass of the
  // accumulators' INTT runs here: that round in registers, the strided round
  // through the two LDS tiles, and the pass's output is what is written.
  uint32_t y0[R2::NI][R2::E], y1[R2::NI][R2::E];
#pragma unroll
  for (int i = 0; i < R2::NI; i++) {
    int c, rb, hi;
    R2::decode(i * kKipThreads + threadIdx.x, c, rb, hi);
    uint32_t o0[R2::E], o1[R2::E];
#pragma unroll
    for (int j = 0; j < R2::E; j++) {
      o0[j] = finish(l0[i * R2::E + j], h0[i * R2::E + j]);
      o1[j] = finish(l1[i * R2::E + j], h1[i * R2::E + j]);
    }
    if (e < A.level && !sums) {  // relocated ModDown input D_l + P^-1 C~ on the q rows
      uint32_t d0[R2::E], d1[R2::E];
      load_global<R2>(d0, De, 0, col0 + c, rb);
      load_global<R2>(d1, De + (size_t)A.level * N, 0, col0 + c, rb);
#pragma unroll
      for (int j = 0; j < R2::E; j++) {
        o0[j] = add_mod(o0[j], d0[j], q);
        o1[j] = add_mod(o1[j], d1[j], q);
      }
    }
    item_bfly<R2::RB, false, LAZY, false>(o0, itw, s0 + R2::SL0, s0, hi, col0 + c, q, nf);
    item_bfly<R2::RB, false, LAZY, false>(o1, itw, s0 + R2::SL0, s0, hi, col0 + c, q, nf);
#pragma unroll
    for (int j = 0; j < R2::E; j++) {
      y0[i][j] = o0[j];
      y1[i][j] = o1[j];
    }
  }
  __syncthreads();  // every thread is done with the tile and the twiddles
  uint32_t* lds1 = reinterpret_cast<uint32_t*>(ltw);
#pragma unroll
  for (int i = 0; i < R2::NI; i++) {
    int c, rb, hi;
    R2::decode(i * kKipThreads + threadIdx.x, c, rb, hi);
    store_lds<R2, G>(y0[i], lds, c, rb);
    store_lds<R2, G>(y1[i], lds1, c, rb);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < R1::NI; i++) {
    int c, rb, hi;
    R1::decode(i * kKipThreads + threadIdx.x, c, rb, hi);
    uint32_t z0[R1::E], z1[R1::E];
    load_lds<R1, G>(z0, lds, c, rb);
    load_lds<R1, G>(z1, lds1, c, rb);
    item_bfly<R1::RB, false, LAZY, false>(z0, itw, s0 + R1::SL0, s0, hi, col0 + c, q, nf);
    item_bfly<R1::RB, false, LAZY, false>(z1, itw, s0 + R1::SL0, s0, hi, col0 + c, q, nf);
    store_global<R1>(z0, acc_e, 0, col0 + c, rb);
    store_global<R1>(z1, acc_e + (size_t)A.E * N, 0, col0 + c, rb);
  }
}

// Workgroup order: the jobs of one (limb, tile) run back to back on one XCD,
// so the key tiles they share are read from L2.  The special primes come
// first: a q limb skips its own digit's pairs when the tensor kernel has
// summed them, so the longest units are dispatched before the shorter ones
// and the last, partly filled round is made of the shorter ones.
template <int LOGR>
__global__ __launch_bounds__(kKipThreads) void k_kip_b(const uint32_t* X, const uint32_t* D, const uint32_t* evk,
                                                       uint32_t* acc, KipArgs A, DevTables T) {
  __shared__ __align__(16) uint32_t lds[kip_lds_words<LOGR>()];
  uint2* ltw = reinterpret_cast<uint2*>(lds + Geo<LOGR, kKipTileLog>::LDS_WORDS);
  const int xcd = blockIdx.x & 7, seq = blockIdx.x >> 3;
  const int job = seq % A.n_jobs;
  const int unit = (seq / A.n_jobs) * 8 + xcd;  // (prime, tile)
  if (unit >= A.E * A.tiles) return;
  const int u = unit / A.tiles, ks = A.E - A.level;  // K special primes, then the q limbs
  const int tile = unit - u * A.tiles;
  const int e = u < ks ? A.level + u : u - ks;
  const int pe = e < A.level ? e : A.L + (e - A.level);
  const uint32_t q = T.mod[pe], minv = T.minv[pe];
  const uint2* tw = reinterpret_cast<const uint2*>(T.tw) + ((size_t)pe << A.log_n);
  const uint2* itw = reinterpret_cast<const uint2*>(T.itw) + ((size_t)pe << A.log_n);
  const size_t N = (size_t)1 << A.log_n;
  const uint32_t* Xe = X + (size_t)job * (size_t)A.x_job + (size_t)e * N;
  const uint32_t* De = D + (size_t)job * (size_t)A.d_job + (size_t)e * N;
  const uint32_t* evk_e = evk + (size_t)pe * N;
  uint32_t* acc_e = acc + (size_t)job * (size_t)A.acc_job + (size_t)e * N;
  const int col0 = tile * Geo<LOGR, kKipTileLog>::COLS;
  if (q < (1u << 30))
    kip_b_body<LOGR, true>(Xe, De, evk_e, acc_e, A, lds, ltw, e, col0, q, minv, T.red[pe], tw, itw);
  else
    kip_b_body<LOGR, false>(Xe, De, evk_e, acc_e, A, lds, ltw, e, col0, q, minv, T.red[pe], tw, itw);
}

// ------------------------------------------------------------------ job-table forms

// One transform pass over the jobs of a table: stage S_INTT_D (d_2..d_k into
// the scaled coefficient limbs), S_INTT_ACC (the accumulators) or S_NTT_OUT
// (the rescaled output).  Blocks per job: tiles x limbs.
template <int LOGR, bool FWD, bool PASSB>
__global__ __launch_bounds__(kThreads) void k_ntt_pass_jt(const JobDesc* jt, int nj, int stage, GroupConsts G,
                                                          DevTables T, int s0) {
  __shared__ uint32_t lds[Geo<LOGR>::LDS_WORDS];
  __shared__ uint2 ltwa[pass_tw_words<LOGR, FWD, PASSB>()];
  constexpr bool FIRST = FWD ? !PASSB : PASSB;  // the transform's first pass reads the source
  const int j = find_job(jt, nj, stage, blockIdx.x);
  const int local = blockIdx.x - jt[j].blk0[stage];
  const int log_n = G.log_n;
  const int tiles = 1 << (log_n - kTileLog);
  const int tile = local & (tiles - 1), limb = local >> (log_n - kTileLog);
  const int k = jt[j].k, level = jt[j].level;
  const size_t N = (size_t)1 << log_n;
  const WsLayout lay(k, level, G.K, G.alpha, log_n);
  uint32_t* ws = jt[j].ws;
  const uint32_t* src;
  uint32_t* dst;
  int prime;
  uint4 nfix;
  if (stage == S_INTT_D) {
    if (limb >= (k - 1) * level) return;
    const int g = limb / level, pos = limb - g * level;
    prime = pos;
    dst = ws + lay.dcoef + ((size_t)g * level + pos) * N;
    src = FIRST ? ws + lay.D + ((size_t)(g + 2) * level + pos) * N : dst;
    nfix = reinterpret_cast<const uint4*>(G.dscale + G.dscale_off[level])[pos];
  } else if (stage == S_INTT_ACC) {
    const int E = level + G.K;
    if (limb >= 2 * E) return;
    const int g = limb / E, pos = limb - g * E;
    prime = pos < level ? pos : G.L + (pos - level);
    dst = ws + lay.acc + ((size_t)g * E + pos) * N;
    src = dst;
    nfix = reinterpret_cast<const uint4*>(T.nfix)[prime];
  } else {
    const int top = level - (k - 1);
    if (limb >= 2 * top) return;
    const int g = limb / top, pos = limb - g * top;
    prime = pos;
    dst = jt[j].out + ((size_t)g * top + pos) * N;
    src = dst;
    nfix = reinterpret_cast<const uint4*>(T.nfix)[prime];
  }
  const uint32_t q = T.mod[prime];
  const uint2* tw = reinterpret_cast<const uint2*>(FWD ? T.tw : T.itw) + ((size_t)prime << log_n);
  const int H = log_n - s0 - LOGR;
  const int col0 = tile * Geo<LOGR>::COLS;
  if (q < (1u << 30))
    pass_body<LOGR, FWD, true, PASSB>(src, dst, lds, ltwa, s0, H, col0, q, tw, nfix);
  else
    pass_body<LOGR, FWD, false, PASSB>(src, dst, lds, ltwa, s0, H, col0, q, tw, nfix);
}

// ModUp conversion + pass A over the jobs of a table.  Blocks per job:
// ceil(units / 8) 8 E with units = (k - 1) B tiles (each job's first block is
// a multiple of 8, so local and global blocks share their XCD).
template <int LOGR, int ALPHA>
__global__ __launch_bounds__(kModupThreads) void k_modup_a_jt(const JobDesc* jt, int nj, GroupConsts G, DevTables T) {
  __shared__ uint32_t lds[Geo<LOGR, kModupTileLog>::LDS_WORDS];
  __shared__ uint2 ltwa[1 << LOGR];
  const int j = find_job(jt, nj, S_MODUP, blockIdx.x);
  const int local = blockIdx.x - jt[j].blk0[S_MODUP];
  const int log_n = G.log_n;
  const int k = jt[j].k, level = jt[j].level;
  const int E = level + G.K, B = (level + G.alpha - 1) / G.alpha;
  const int tiles = 1 << (log_n - kModupTileLog);
  const int units = (k - 1) * B * tiles;
  const int xcd = local & 7, seq = local >> 3;
  const int e = seq % E;
  const int unit = (seq / E) * 8 + xcd;
  if (unit >= units) return;
  const int tile = unit % tiles;
  const int tb = unit / tiles;  // (t - 2) B + b
  const int t2 = tb / B, b = tb - t2 * B;
  const int lo = b * G.alpha;
  const int na = min(G.alpha, level - lo);
  if (e >= lo && e < lo + na) return;
  const int pe = e < level ? e : G.L + (e - level);
  const uint32_t q = T.mod[pe], minv = T.minv[pe];
  const uint2* tw = reinterpret_cast<const uint2*>(T.tw) + ((size_t)pe << log_n);
  const size_t N = (size_t)1 << log_n;
  const WsLayout lay(k, level, G.K, G.alpha, log_n);
  const uint32_t* C = G.modup_tab + G.modup_off[(level - 1) * G.dnum + b] + 2 * ALPHA;
  const uint32_t* base = jt[j].ws + lay.dcoef + ((size_t)t2 * level + lo) * N;
  const __amdgpu_buffer_rsrc_t src = buffer_rsrc(base, (uint32_t)(na * N * 4));
  uint32_t cc[ALPHA];
#pragma unroll
  for (int a = 0; a < ALPHA; a++) cc[a] = C[a * E + e];
  uint32_t* dst = jt[j].ws + lay.X + ((size_t)tb * E + e) * N;
  const int H = log_n - LOGR;
  const int col0 = tile * Geo<LOGR, kModupTileLog>::COLS;
  if (q < (1u << 30))
    modup_a_body<LOGR, ALPHA, true>(src, na, cc, minv, dst, lds, ltwa, H, col0, q, tw);
  else
    modup_a_body<LOGR, ALPHA, false>(src, na, cc, minv, dst, lds, ltwa, H, col0, q, tw);
}

// Job-table form of k_modup_a2 (digits of 5 to 8 primes).  Blocks per job:
// ceil(units / 8) 8 modup_pairs(level, E).
template <int LOGR, int ALPHA>
__global__ __launch_bounds__(kModupThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_modup_a2_jt(
    const JobDesc* jt, int nj, GroupConsts G, DevTables T) {
  __shared__ uint32_t lds[Geo<LOGR, kModupTileLog>::LDS_WORDS];
  __shared__ uint2 ltw[2][1 << LOGR];
  const int j = find_job(jt, nj, S_MODUP, blockIdx.x);
  const int local = blockIdx.x - jt[j].blk0[S_MODUP];
  const int log_n = G.log_n;
  const int k = jt[j].k, level = jt[j].level;
  const int E = level + G.K, B = (level + G.alpha - 1) / G.alpha;
  const int tiles = 1 << (log_n - kModupTileLog);
  const int units = (k - 1) * B * tiles;
  const int pairs = modup_pairs(level, E);
  const int xcd = local & 7, seq = local >> 3;
  const int pr = seq % pairs;
  const int unit = (seq / pairs) * 8 + xcd;
  if (unit >= units) return;
  const int tile = unit % tiles;
  const int tb = unit / tiles;  // (t - 2) B + b
  const int t2 = tb / B, b = tb - t2 * B;
  const int lo = b * G.alpha;
  const int na = min(G.alpha, level - lo);
  const int nq = level - na;
  const int qp = (nq + 1) / 2;
  int e0, e1;
  if (pr < qp) {
    const int i0 = 2 * pr, i1 = i0 + 1;
    e0 = i0 < lo ? i0 : i0 + na;
    e1 = i1 < nq ? (i1 < lo ? i1 : i1 + na) : -1;
  } else {
    e0 = level + 2 * (pr - qp);
    if (e0 >= E) return;
    e1 = e0 + 1 < E ? e0 + 1 : -1;
  }
  const bool two = e1 >= 0;
  const int f1 = two ? e1 : e0;
  const int p0 = e0 < level ? e0 : G.L + (e0 - level);
  const int p1 = f1 < level ? f1 : G.L + (f1 - level);
  const uint32_t q0 = T.mod[p0], q1 = T.mod[p1];
  const uint2* tw0 = reinterpret_cast<const uint2*>(T.tw) + ((size_t)p0 << log_n);
  const uint2* tw1 = reinterpret_cast<const uint2*>(T.tw) + ((size_t)p1 << log_n);
  const size_t N = (size_t)1 << log_n;
  const WsLayout lay(k, level, G.K, G.alpha, log_n);
  const uint32_t* C = G.modup_tab + G.modup_off[(level - 1) * G.dnum + b] + 2 * ALPHA;
  const uint32_t* base = jt[j].ws + lay.dcoef + ((size_t)t2 * level + lo) * N;
  const __amdgpu_buffer_rsrc_t src = buffer_rsrc(base, (uint32_t)(na * N * 4));
  uint32_t c0[ALPHA], c1[ALPHA];
#pragma unroll
  for (int a = 0; a < ALPHA; a++) {
    c0[a] = C[a * E + e0];
    c1[a] = C[a * E + f1];
  }
  uint32_t* xj = jt[j].ws + lay.X + (size_t)tb * E * N;
  uint32_t* dst0 = xj + (size_t)e0 * N;
  uint32_t* dst1 = two ? xj + (size_t)e1 * N : nullptr;
  const int H = log_n - LOGR;
  const int col0 = tile * Geo<LOGR, kModupTileLog>::COLS;
  if (q0 < (1u << 30) && q1 < (1u << 30))
    modup_a2_body<LOGR, ALPHA, true>(src, na, c0, c1, T.minv[p0], T.minv[p1], dst0, dst1, lds, ltw[0], ltw[1], H,
                                     col0, q0, q1, tw0, tw1);
  else
    modup_a2_body<LOGR, ALPHA, false>(src, na, c0, c1, T.minv[p0], T.minv[p1], dst0, dst1, lds, ltw[0], ltw[1], H,
                                      col0, q0, q1, tw0, tw1);
}

// Pass B + key inner product over the jobs of a table.  Blocks per job:
// ceil(E tiles / 8) 8.
template <int LOGR>
__global__ __launch_bounds__(kKipThreads) void k_kip_b_jt(const JobDesc* jt, int nj, GroupConsts G, DevTables T) {
  __shared__ __align__(16) uint32_t lds[kip_lds_words<LOGR>()];
  uint2* ltw = reinterpret_cast<uint2*>(lds + Geo<LOGR, kKipTileLog>::LDS_WORDS);
  // units (prime, tile) with the special primes first, so that a job's
  // units are a prefix and a unit is the same prime for every job: the jobs
  // of one unit share its key words and twiddles in L2 (seg_block)
  int rank, local;
  seg_block<1>(jt, nj, blockIdx.x, rank, local);
  const int j = jt[rank].seg[1].job;
  const int log_n = G.log_n;
  const int k = jt[j].k, level = jt[j].level;
  KipArgs A{};
  A.log_n = log_n;
  A.level = level;
  A.L = G.L;
  A.E = level + G.K;
  A.B = (level + G.alpha - 1) / G.alpha;
  A.alpha = G.alpha;
  A.dnum = G.dnum;
  A.k = k;
  A.n_jobs = 1;
  A.tiles = 1 << (log_n - kKipTileLog);
  A.key_poly = (long long)(G.L + G.K) << log_n;
  A.own_sums = 1;  // the table's tensor launches always form them
  if (local >= A.E * A.tiles) return;  // the job's last group's padding
  const int u = local / A.tiles;  // K special primes, then the q limbs
  const int tile = local - u * A.tiles;
  const int e = u < G.K ? level + u : u - G.K;
  const int pe = e < level ? e : G.L + (e - level);
  const uint32_t q = T.mod[pe], minv = T.minv[pe];
  const uint2* tw = reinterpret_cast<const uint2*>(T.tw) + ((size_t)pe << log_n);
  const uint2* itw = reinterpret_cast<const uint2*>(T.itw) + ((size_t)pe << log_n);
  const size_t N = (size_t)1 << log_n;
  const WsLayout lay(k, level, G.K, G.alpha, log_n);
  uint32_t* ws = jt[j].ws;
  const int col0 = tile * Geo<LOGR, kKipTileLog>::COLS;
  if (q < (1u << 30))
    kip_b_body<LOGR, true>(ws + lay.X + (size_t)e * N, ws + lay.D + (size_t)e * N, G.evk + (size_t)pe * N,
                           ws + lay.acc + (size_t)e * N, A, lds, ltw, e, col0, q, minv, T.red[pe], tw, itw);
  else
    kip_b_body<LOGR, false>(ws + lay.X + (size_t)e * N, ws + lay.D + (size_t)e * N, G.evk + (size_t)pe * N,
                            ws + lay.acc + (size_t)e * N, A, lds, ltw, e, col0, q, minv, T.red[pe], tw, itw);
}

template <bool FWD, bool PASSB>
void launch_pass_jt(int logr, unsigned blocks, hipStream_t s, const JobDesc* jt, int nj, int stage,
                    const GroupConsts& G, const DevTables& T, int s0) {
  switch (logr) {
    case 6: k_ntt_pass_jt<6, FWD, PASSB><<<blocks, kThreads, 0, s>>>(jt, nj, stage, G, T, s0); break;
    case 7: k_ntt_pass_jt<7, FWD, PASSB><<<blocks, kThreads, 0, s>>>(jt, nj, stage, G, T, s0); break;
    default: k_ntt_pass_jt<8, FWD, PASSB><<<blocks, kThreads, 0, s>>>(jt, nj, stage, G, T, s0); break;
  }
}

}  // namespace

LimbMap simple_map(const mick_params* prm, int first_prime, int n_limbs) {
  LimbMap m{};
  m.period = n_limbs;
  m.group_stride = (long long)n_limbs << prm->log_n;
  m.split = n_limbs;
  m.off_lo = first_prime;
  m.off_hi = first_prime;
  m.job_stride = 0;
  m.nfix_pos = nullptr;
  return m;
}

int ntt_launch(const mick_params* prm, const uint32_t* src, uint32_t* dst, const LimbMap& map, int n_limbs, int n_jobs,
               bool inverse, hipStream_t s, int site) {
  if (n_limbs <= 0 || n_jobs <= 0) return MICK_OK;
  if (n_limbs > 65535 || n_jobs > 65535) return set_error(MICK_E_ARG, "too many limbs for one transform launch");
  const int log_n = prm->log_n;
  dim3 grid(1u << (log_n - kTileLog), (unsigned)n_limbs, (unsigned)n_jobs);
  const int la = prm->split_a, lb = prm->split_b;
  if (!inverse) {
    launch_pass<true, false>(la, grid, s, src, dst, map, prm->dt, log_n, 0, site);
    launch_pass<true, true>(lb, grid, s, dst, dst, map, prm->dt, log_n, la, site + 1);
  } else {
    launch_pass<false, true>(lb, grid, s, src, dst, map, prm->dt, log_n, la, site + 1);
    launch_pass<false, false>(la, grid, s, dst, dst, map, prm->dt, log_n, 0, site);
  }
  return hip_error(hipGetLastError(), "ntt launch");
}

int intt_pass_a_launch(const mick_params* prm, uint32_t* buf, const LimbMap& map, int n_limbs, int n_jobs,
                       hipStream_t s, int site) {
  if (n_limbs <= 0 || n_jobs <= 0) return MICK_OK;
  if (n_limbs > 65535 || n_jobs > 65535) return set_error(MICK_E_ARG, "too many limbs for one transform launch");
  const int log_n = prm->log_n;
  dim3 grid(1u << (log_n - kTileLog), (unsigned)n_limbs, (unsigned)n_jobs);
  launch_pass<false, false>(prm->split_a, grid, s, buf, buf, map, prm->dt, log_n, 0, site);
  return hip_error(hipGetLastError(), "ntt launch");
}

int launch_modup_a(const mick_params* prm, const uint32_t* dsc, uint32_t* X, ModupArgs A, int n_jobs, hipStream_t s) {
  A.tiles = 1 << (prm->log_n - kModupTileLog);
  A.units = n_jobs * A.groups * A.tiles;
  const unsigned blocks =
      (unsigned)(((A.units + 7) / 8) * 8 * (modup_pairs_on(prm) ? modup_pairs(A.level, A.E) : A.E));
  ProfScope ps(P_MODUP, s);
  const DevTables& T = prm->dt;
#define MICK_MA2(LR, AL) k_modup_a2<LR, AL><<<blocks, kModupThreads, 0, s>>>(dsc, X, A, T)
#define MICK_MA(LR, AL) k_modup_a<LR, AL><<<blocks, kModupThreads, 0, s>>>(dsc, X, A, T)
#define MICK_MA_A(LR)                                                   \
  switch (modup_rows(A.alpha)) {                                        \
    case 1: MICK_MA(LR, 1); break;                                      \
    case 2: MICK_MA(LR, 2); break;                                      \
    case 4: MICK_MA(LR, 4); break;                                      \
    case 8:                                                             \
      if (modup_pairs_on(prm))                                          \
        MICK_MA2(LR, 8);                                                \
      else                                                              \
        MICK_MA(LR, 8);                                                 \
      break;                                                            \
    case 16: MICK_MA(LR, 16); break;                                    \
    case 24: MICK_MA(LR, 24); break;                                    \
    case 32: MICK_MA(LR, 32); break;                                    \
    default: return set_error(MICK_E_ARG, "digit width out of range"); \
  }
  if (prm->split_a == 7) {
    MICK_MA_A(7)
  } else {
    MICK_MA_A(8)
  }
#undef MICK_MA_A
#undef MICK_MA
#undef MICK_MA2
  return hip_error(hipGetLastError(), "modup launch");
}

int launch_kip_b(const mick_params* prm, const uint32_t* X, const uint32_t* D, const uint32_t* evk, uint32_t* acc,
                 KipArgs A, hipStream_t s) {
  A.tiles = 1 << (prm->log_n - kKipTileLog);
  const int units = A.E * A.tiles;
  const unsigned blocks = (unsigned)(((units + 7) / 8) * 8 * A.n_jobs);
  ProfScope ps(P_KIP, s);
  const DevTables& T = prm->dt;
  switch (prm->split_b) {
    case 6: k_kip_b<6><<<blocks, kKipThreads, 0, s>>>(X, D, evk, acc, A, T); break;
    case 7: k_kip_b<7><<<blocks, kKipThreads, 0, s>>>(X, D, evk, acc, A, T); break;
    default: k_kip_b<8><<<blocks, kKipThreads, 0, s>>>(X, D, evk, acc, A, T); break;
  }
  return hip_error(hipGetLastError(), "kip launch");
}

}  // namespace mick

namespace mick {

int launch_ntt_jt(const mick_params* prm, const JobDesc* jt, int nj, int stage, int blocks, const GroupConsts& G,
                  hipStream_t s) {
  if (blocks <= 0) return MICK_OK;
  const int la = prm->split_a, lb = prm->split_b;
  const int site = stage == S_INTT_D ? P_INTT_D : (stage == S_INTT_ACC ? P_INTT_ACC : P_NTT_OUT);
  if (stage == S_NTT_OUT) {
    {
      ProfScope ps(site, s);
      launch_pass_jt<true, false>(la, blocks, s, jt, nj, stage, G, prm->dt, 0);
    }
    ProfScope ps(site + 1, s);
    launch_pass_jt<true, true>(lb, blocks, s, jt, nj, stage, G, prm->dt, la);
  } else {
    // pass B of the accumulators ran inside the key-product kernel, and that
    // of d_2..d_k inside the tensor kernel
    if (stage != S_INTT_ACC && stage != S_INTT_D) {
      ProfScope ps(site + 1, s);
      launch_pass_jt<false, true>(lb, blocks, s, jt, nj, stage, G, prm->dt, la);
    }
    ProfScope ps(site, s);
    launch_pass_jt<false, false>(la, blocks, s, jt, nj, stage, G, prm->dt, 0);
  }
  return hip_error(hipGetLastError(), "ntt launch");
}

int launch_modup_a_jt(const mick_params* prm, const JobDesc* jt, int nj, int blocks, const GroupConsts& G,
                      hipStream_t s) {
  if (blocks <= 0) return MICK_OK;
  ProfScope ps(P_MODUP, s);
  const DevTables& T = prm->dt;
#define MICK_MA2(LR, AL) k_modup_a2_jt<LR, AL><<<blocks, kModupThreads, 0, s>>>(jt, nj, G, T)
#define MICK_MA(LR, AL) k_modup_a_jt<LR, AL><<<blocks, kModupThreads, 0, s>>>(jt, nj, G, T)
#define MICK_MA_A(LR)                                                   \
  switch (modup_rows(G.alpha)) {                                        \
    case 1: MICK_MA(LR, 1); break;                                      \
    case 2: MICK_MA(LR, 2); break;                                      \
    case 4: MICK_MA(LR, 4); break;                                      \
    case 8:                                                             \
      if (modup_pairs_on(prm))                                          \
        MICK_MA2(LR, 8);                                                \
      else                                                              \
        MICK_MA(LR, 8);                                                 \
      break;                                                            \
    case 16: MICK_MA(LR, 16); break;                                    \
    case 24: MICK_MA(LR, 24); break;                                    \
    case 32: MICK_MA(LR, 32); break;                                    \
    default: return set_error(MICK_E_ARG, "digit width out of range"); \
  }
  if (prm->split_a == 7) {
    MICK_MA_A(7)
  } else {
    MICK_MA_A(8)
  }
#undef MICK_MA_A
#undef MICK_MA
#undef MICK_MA2
  return hip_error(hipGetLastError(), "modup launch");
}

int launch_kip_b_jt(const mick_params* prm, const JobDesc* jt, int nj, int blocks, const GroupConsts& G,
                    hipStream_t s) {
  if (blocks <= 0) return MICK_OK;
  ProfScope ps(P_KIP, s);
  const DevTables& T = prm->dt;
  switch (prm->split_b) {
    case 6: k_kip_b_jt<6><<<blocks, kKipThreads, 0, s>>>(jt, nj, G, T); break;
    case 7: k_kip_b_jt<7><<<blocks, kKipThreads, 0, s>>>(jt, nj, G, T); break;
    default: k_kip_b_jt<8><<<blocks, kKipThreads, 0, s>>>(jt, nj, G, T); break;
  }
  return hip_error(hipGetLastError(), "kip launch");
}

}  // namespace mick
