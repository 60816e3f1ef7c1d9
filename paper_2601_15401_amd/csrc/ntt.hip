// Negacyclic NTT / INTT for N = 2^13 .. 2^16 on gfx950.
//
// The transform is the merged-twiddle Cooley-Tukey factorisation of
// NTT(a)[k] = a(psi^(2 brv(k) + 1)): stage s (s = 0 .. log N - 1) splits the
// vector into 2^s blocks and butterflies element pairs half a block apart
// with twiddle psi^brv(2^s + b) for block b.  The inverse runs the stages in
// reverse with Gentleman-Sande butterflies and psi^-brv(.), and the factor
// N^-1 is merged into its last stage.
//
// Two passes cover the log N stages: pass A the first LA stages (element
// pairs that differ in the high LA index bits), pass B the last LB stages.
// A workgroup owns an 8192-element tile of one limb: 2^LOGR butterfly rows
// by 8192 / 2^LOGR independent columns (pass A: columns are consecutive low
// indices; pass B: columns are consecutive 2^LB-element blocks).  A pass is
// two radix-8/16 rounds in registers: the "strided" round (the pass's first
// RB0 stages, row stride 2^(LOGR-RB0)) and the "consecutive" round (the last
// RB1 stages, 2^RB1 neighbouring rows).  The first round of a pass loads
// straight from global memory into registers, the tile crosses LDS once
// between the rounds, and the second round stores straight to global
// memory.  Lane-to-item maps are chosen per pass and round so that global
// accesses are coalesced (pass B's consecutive round moves 16 neighbouring
// words per lane with 128-bit accesses); pass-B twiddles are stored
// transposed per stage so that lanes holding neighbouring blocks read
// neighbouring twiddles.
//
// Arithmetic: Shoup products by precomputed twiddles.  Limbs whose prime is
// below 2^30 use Harvey's lazy butterflies (values kept below 4q); the
// 31-bit special primes keep values below 2q with one more conditional
// subtraction per butterfly.  The last pass stores canonical residues.
#include "internal.h"

namespace mick {

namespace {

constexpr int kThreads = 256;
constexpr int kTileLog = 13;

template <bool MODUP>
__device__ __forceinline__ void resolve(const LimbMap& mp, int limb, int log_n, int& prime, size_t& off, bool& skip) {
  int g = limb / mp.period;
  int pos = limb - g * mp.period;
  prime = pos < mp.split ? pos + mp.off_lo : pos + mp.off_hi;
  off = (size_t)g * (size_t)mp.group_stride + ((size_t)pos << log_n) + (size_t)blockIdx.z * (size_t)mp.job_stride;
  skip = false;
  if constexpr (MODUP) {
    int b = g % mp.skip_groups;
    int lo = b * mp.skip_alpha;
    int hi = min(lo + mp.skip_alpha, mp.skip_level);
    skip = pos >= lo && pos < hi;
  }
}

// Forward (Cooley-Tukey) butterfly.
template <bool LAZY>
__device__ __forceinline__ void ct(uint32_t& x, uint32_t& y, uint2 w, uint32_t q) {
  if constexpr (LAZY) {  // x, y < 4q -> outputs < 4q
    uint32_t a = min(x, x - 2 * q);
    uint32_t t = shoup_lazy(y, w.x, w.y, q);
    x = a + t;
    y = a - t + 2 * q;
  } else {  // x, y < 2q -> outputs < 2q
    uint32_t a = red1(x, q);
    uint32_t t = red1(shoup_lazy(y, w.x, w.y, q), q);
    x = a + t;
    y = a - t + q;
  }
}

// Inverse (Gentleman-Sande) butterfly, values < 2q throughout.
template <bool LAZY>
__device__ __forceinline__ void gs(uint32_t& x, uint32_t& y, uint2 w, uint32_t q) {
  if constexpr (LAZY) {
    uint32_t u = x + y;
    uint32_t v = x - y + 2 * q;
    x = min(u, u - 2 * q);
    y = shoup_lazy(v, w.x, w.y, q);
  } else {
    uint32_t a = red1(x, q), b = red1(y, q);
    x = a + b;
    y = shoup_lazy(a - b + q, w.x, w.y, q);
  }
}

// The last inverse stage with N^-1 merged into both outputs.
template <bool LAZY>
__device__ __forceinline__ void gs_last(uint32_t& x, uint32_t& y, const uint4& nf, uint32_t q) {
  if constexpr (LAZY) {
    uint32_t u = x + y, v = x - y + 2 * q;
    x = shoup_lazy(u, nf.x, nf.y, q);
    y = shoup_lazy(v, nf.z, nf.w, q);
  } else {
    uint32_t a = red1(x, q), b = red1(y, q);
    x = shoup_lazy(a + b, nf.x, nf.y, q);
    y = shoup_lazy(a - b + q, nf.z, nf.w, q);
  }
}

template <bool FWD, bool LAZY>
__device__ __forceinline__ uint32_t canonical(uint32_t v, uint32_t q) {
  if constexpr (FWD && LAZY) v = min(v, v - 2 * q);
  return red1(v, q);
}

// One round of a pass.  STRIDED: the pass's first RB0 stages; otherwise its
// last RB1 stages.  Loads from global memory when FROM_G, else from LDS;
// stores to global memory when TO_G, else to LDS.
template <int LOGR, bool FWD, bool LAZY, bool PASSB, bool STRIDED, bool FROM_G, bool TO_G>
__device__ __forceinline__ void nround(const uint32_t* gsrc, uint32_t* gdst,
                                       uint32_t* lds, int s0, int H, int col0, uint32_t q,
                                       const uint2* __restrict__ tw, const uint4& nfix) {
  constexpr int LOGC = kTileLog - LOGR;
  constexpr int COLS = 1 << LOGC;
  constexpr int PAD = COLS + 1;
  constexpr int RB0 = (LOGR == 6) ? 3 : 4;
  constexpr int RB = STRIDED ? RB0 : LOGR - RB0;
  constexpr int E = 1 << RB;
  constexpr int SL0 = STRIDED ? 0 : RB0;          // first local stage of the round
  constexpr int NLO_LOG = STRIDED ? LOGR - RB0 : 0;
  constexpr int NLO = 1 << NLO_LOG;
  constexpr int ITEMS = (1 << kTileLog) >> RB;
  // pass B's strided round walks the rows of a column with consecutive lanes
  constexpr bool LO_FAST = PASSB && STRIDED;
  constexpr bool FINAL = FWD ? PASSB : !PASSB;     // last pass of the transform
  constexpr bool STORE_FINAL = FINAL && TO_G;
  constexpr bool HAS_STAGE0 = !FWD && !PASSB && STRIDED;  // global stage 0 (inverse)
  constexpr bool VEC = PASSB && !STRIDED;           // 16 neighbouring words per lane

#pragma unroll
  for (int it0 = 0; it0 < ITEMS; it0 += kThreads) {
    const int it = it0 + threadIdx.x;
    int c, lo, hi;
    if constexpr (LO_FAST) {
      lo = it & (NLO - 1);
      c = it >> NLO_LOG;
      hi = 0;
    } else {
      c = it & (COLS - 1);
      const int hl = it >> LOGC;
      lo = STRIDED ? hl : 0;
      hi = STRIDED ? 0 : hl;
    }
    const int rbase = (hi << (LOGR - SL0)) + lo;
    const int col = col0 + c;
    const int blk = PASSB ? col : 0;
    uint32_t x[E];
    // ---- load
    if constexpr (FROM_G && VEC) {
#pragma unroll
      for (int j = 0; j < E; j += 4) {
        const uint4 v = *reinterpret_cast<const uint4*>(gsrc + ((size_t)col << LOGR) + rbase + j);
        x[j] = v.x;
        x[j + 1] = v.y;
        x[j + 2] = v.z;
        x[j + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < E; j++) {
        const int r = rbase + (j << NLO_LOG);
        if constexpr (FROM_G) {
          const size_t g = PASSB ? ((size_t)col << LOGR) + r : ((size_t)r << H) + col;
          x[j] = gsrc[g];
        } else {
          x[j] = lds[r * PAD + c];
        }
      }
    }
    // ---- the round's twiddles: stage u uses 2^u of them, w[2^u + g]
    uint2 w[E];
#pragma unroll
    for (int u = 0; u < RB; u++) {
      if (HAS_STAGE0 && u == 0) continue;
      const int s = s0 + SL0 + u;
#pragma unroll
      for (int g = 0; g < (1 << u); g++) {
        const int rr = (hi << u) + g;
        w[(1 << u) + g] = tw[(1 << s) + (rr << s0) + blk];
      }
    }
    // ---- butterflies
    if constexpr (FWD) {
#pragma unroll
      for (int u = 0; u < RB; u++) {
        const int half = 1 << (RB - 1 - u);
#pragma unroll
        for (int j = 0; j < E; j++) {
          if (j & half) continue;
          ct<LAZY>(x[j], x[j + half], w[(1 << u) + (j >> (RB - u))], q);
        }
      }
    } else {
#pragma unroll
      for (int u = RB - 1; u >= 0; u--) {
        const int half = 1 << (RB - 1 - u);
#pragma unroll
        for (int j = 0; j < E; j++) {
          if (j & half) continue;
          if (HAS_STAGE0 && u == 0)
            gs_last<LAZY>(x[j], x[j + half], nfix, q);
          else
            gs<LAZY>(x[j], x[j + half], w[(1 << u) + (j >> (RB - u))], q);
        }
      }
    }
    // ---- store
    if constexpr (STORE_FINAL) {
#pragma unroll
      for (int j = 0; j < E; j++) x[j] = canonical<FWD, LAZY>(x[j], q);
    }
    if constexpr (TO_G && VEC) {
#pragma unroll
      for (int j = 0; j < E; j += 4) {
        uint4 o;
        o.x = x[j];
        o.y = x[j + 1];
        o.z = x[j + 2];
        o.w = x[j + 3];
        *reinterpret_cast<uint4*>(gdst + ((size_t)col << LOGR) + rbase + j) = o;
      }
    } else {
#pragma unroll
      for (int j = 0; j < E; j++) {
        const int r = rbase + (j << NLO_LOG);
        if constexpr (TO_G) {
          const size_t g = PASSB ? ((size_t)col << LOGR) + r : ((size_t)r << H) + col;
          gdst[g] = x[j];
        } else {
          lds[r * PAD + c] = x[j];
        }
      }
    }
  }
}

template <int LOGR, bool FWD, bool LAZY, bool PASSB>
__device__ __forceinline__ void pass_body(const uint32_t* src, uint32_t* dst, uint32_t* lds, int s0, int H, int col0,
                                          uint32_t q, const uint2* tw, const uint4& nfix) {
  // forward: strided round first; inverse: consecutive round first
  nround<LOGR, FWD, LAZY, PASSB, FWD, true, false>(src, dst, lds, s0, H, col0, q, tw, nfix);
  __syncthreads();
  nround<LOGR, FWD, LAZY, PASSB, !FWD, false, true>(src, dst, lds, s0, H, col0, q, tw, nfix);
}

// MODUP: the launch transforms ModUp outputs, whose limbs inside the digit's
// own primes are skipped.  PASSB selects the pass (pass A has s0 = 0).
template <int LOGR, bool FWD, bool MODUP, bool PASSB>
__global__ __launch_bounds__(kThreads) void k_ntt_pass(const uint32_t* src, uint32_t* dst, LimbMap mp, DevTables T,
                                                       int log_n, int s0) {
  constexpr int LOGC = kTileLog - LOGR;
  constexpr int COLS = 1 << LOGC;
  __shared__ uint32_t lds[(1 << LOGR) * (COLS + 1)];
  int prime;
  size_t off;
  bool skip;
  resolve<MODUP>(mp, blockIdx.y, log_n, prime, off, skip);
  if (skip) return;
  const uint32_t q = T.mod[prime];
  const uint2* tw = reinterpret_cast<const uint2*>(FWD ? T.tw : T.itw) + ((size_t)prime << log_n);
  const uint4 nfix = reinterpret_cast<const uint4*>(T.nfix)[prime];
  const int H = log_n - s0 - LOGR;  // > 0 in pass A, 0 in pass B
  const int col0 = blockIdx.x * COLS;
  if (q < (1u << 30))
    pass_body<LOGR, FWD, true, PASSB>(src + off, dst + off, lds, s0, H, col0, q, tw, nfix);
  else
    pass_body<LOGR, FWD, false, PASSB>(src + off, dst + off, lds, s0, H, col0, q, tw, nfix);
}

template <bool FWD, bool MODUP, bool PASSB>
void launch_pass_t(int logr, dim3 grid, hipStream_t s, const uint32_t* src, uint32_t* dst, const LimbMap& mp,
                   const DevTables& T, int log_n, int s0) {
  switch (logr) {
    case 6: k_ntt_pass<6, FWD, MODUP, PASSB><<<grid, kThreads, 0, s>>>(src, dst, mp, T, log_n, s0); break;
    case 7: k_ntt_pass<7, FWD, MODUP, PASSB><<<grid, kThreads, 0, s>>>(src, dst, mp, T, log_n, s0); break;
    default: k_ntt_pass<8, FWD, MODUP, PASSB><<<grid, kThreads, 0, s>>>(src, dst, mp, T, log_n, s0); break;
  }
}

template <bool FWD, bool PASSB>
void launch_pass(int logr, dim3 grid, hipStream_t s, const uint32_t* src, uint32_t* dst, const LimbMap& mp,
                 const DevTables& T, int log_n, int s0, int site) {
  ProfScope ps(site, s);
  if (mp.skip_groups > 0)
    launch_pass_t<FWD, true, PASSB>(logr, grid, s, src, dst, mp, T, log_n, s0);
  else
    launch_pass_t<FWD, false, PASSB>(logr, grid, s, src, dst, mp, T, log_n, s0);
}

}  // namespace

LimbMap simple_map(const mick_params* prm, int first_prime, int n_limbs) {
  LimbMap m{};
  m.period = n_limbs;
  m.group_stride = (long long)n_limbs << prm->log_n;
  m.split = n_limbs;
  m.off_lo = first_prime;
  m.off_hi = first_prime;
  m.skip_groups = 0;
  m.job_stride = 0;
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

}  // namespace mick
