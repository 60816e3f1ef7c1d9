// Negacyclic NTT / INTT for N = 2^13 .. 2^16 on gfx950.
//
// The transform is the merged-twiddle Cooley-Tukey factorisation of
// NTT(a)[k] = a(psi^(2 brv(k) + 1)): stage s (s = 0 .. log N - 1) splits the
// vector into 2^s blocks and butterflies element pairs half a block apart
// with twiddle psi^brv(2^s + b) for block b.  The inverse runs the stages in
// reverse with Gentleman-Sande butterflies and psi^-brv(.), and the factor
// N^-1 is merged into the last stage.
//
// Two passes cover the log N stages: pass A the first LA stages (pairs whose
// indices differ in the high LA bits), pass B the remaining LB stages (the
// low bits).  Each workgroup stages an 8192-element tile of one limb in LDS
// (2^LOGR butterfly rows x 8192 / 2^LOGR independent columns), runs the
// pass's stages as radix-8/16 rounds in registers, and writes the tile back.
// Pass A's columns are consecutive low indices (coalesced along columns);
// pass B's columns are consecutive 2^LB-element blocks (coalesced along
// rows).  Pass-B twiddles are stored transposed per stage so that the lanes
// of a wave, which hold consecutive blocks, read consecutive addresses.
//
// Residues stay in [0, 2m) between stages (2m < 2^32 for m < 2^31) and are
// made canonical when the last pass stores them.
#include "internal.h"

namespace mick {

namespace {

constexpr int kThreads = 256;
constexpr int kTileLog = 13;

__device__ __forceinline__ void resolve(const LimbMap& mp, int limb, int log_n, int& prime, size_t& off, bool& skip) {
  int g = limb / mp.period;
  int pos = limb - g * mp.period;
  prime = pos < mp.split ? pos + mp.off_lo : pos + mp.off_hi;
  off = (size_t)g * (size_t)mp.group_stride + ((size_t)pos << log_n) + (size_t)blockIdx.z * (size_t)mp.job_stride;
  skip = false;
  if (mp.skip_groups > 0) {
    int b = g % mp.skip_groups;
    int lo = b * mp.skip_alpha;
    int hi = min(lo + mp.skip_alpha, mp.skip_level);
    skip = pos >= lo && pos < hi;
  }
}

// One round of RB consecutive stages [sl0, sl0 + RB) of the pass, in
// registers.  Items: (column c, high part hi of the row, low part lo).
template <int LOGR, int RB, bool FWD>
__device__ __forceinline__ void round_rb(uint32_t* lds, int sl0, int s0, int col0, bool colblk, uint32_t q,
                                         const uint2* __restrict__ tw, const uint4& nfix) {
  constexpr int LOGC = kTileLog - LOGR;
  constexpr int COLS = 1 << LOGC;
  constexpr int PAD = COLS + 1;
  constexpr int ITEMS = (1 << kTileLog) >> RB;
  constexpr int E = 1 << RB;
  const int nlo_log = LOGR - sl0 - RB;
  for (int it = threadIdx.x; it < ITEMS; it += kThreads) {
    const int c = it & (COLS - 1);
    const int hl = it >> LOGC;
    const int lo = hl & ((1 << nlo_log) - 1);
    const int hi = hl >> nlo_log;
    const int rbase = (hi << (LOGR - sl0)) + lo;
    const int blk = colblk ? col0 + c : 0;
    uint32_t x[E];
#pragma unroll
    for (int j = 0; j < E; j++) x[j] = lds[(rbase + (j << nlo_log)) * PAD + c];
    if (FWD) {
#pragma unroll
      for (int u = 0; u < RB; u++) {
        const int s = s0 + sl0 + u;
        const int half = 1 << (RB - 1 - u);
#pragma unroll
        for (int j = 0; j < E; j++) {
          if (j & half) continue;
          const int rr = (hi << u) + (j >> (RB - u));
          const uint2 w = tw[(1 << s) + (rr << s0) + blk];
          uint32_t a = red1(x[j], q);
          uint32_t t = red1(shoup_lazy(x[j + half], w.x, w.y, q), q);
          x[j] = a + t;
          x[j + half] = a - t + q;
        }
      }
    } else {
#pragma unroll
      for (int u = RB - 1; u >= 0; u--) {
        const int s = s0 + sl0 + u;
        const int half = 1 << (RB - 1 - u);
#pragma unroll
        for (int j = 0; j < E; j++) {
          if (j & half) continue;
          uint32_t a = red1(x[j], q);
          uint32_t b = red1(x[j + half], q);
          if (s == 0) {
            // last inverse stage: both outputs carry N^-1
            x[j] = shoup_lazy(a + b, nfix.x, nfix.y, q);
            x[j + half] = shoup_lazy(a - b + q, nfix.z, nfix.w, q);
          } else {
            const int rr = (hi << u) + (j >> (RB - u));
            const uint2 w = tw[(1 << s) + (rr << s0) + blk];
            x[j] = a + b;
            x[j + half] = shoup_lazy(a - b + q, w.x, w.y, q);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < E; j++) lds[(rbase + (j << nlo_log)) * PAD + c] = x[j];
  }
}

template <int LOGR, bool FWD>
__global__ __launch_bounds__(kThreads) void k_ntt_pass(const uint32_t* src, uint32_t* dst, LimbMap mp, DevTables T,
                                                       int log_n, int s0, int last) {
  constexpr int R = 1 << LOGR;
  constexpr int LOGC = kTileLog - LOGR;
  constexpr int COLS = 1 << LOGC;
  constexpr int PAD = COLS + 1;
  constexpr int RB0 = (LOGR == 6) ? 3 : 4;
  constexpr int RB1 = LOGR - RB0;
  __shared__ uint32_t lds[R * PAD];

  int prime;
  size_t off;
  bool skip;
  resolve(mp, blockIdx.y, log_n, prime, off, skip);
  if (skip) return;
  const uint32_t q = T.mod[prime];
  const uint2* tw = reinterpret_cast<const uint2*>(FWD ? T.tw : T.itw) + ((size_t)prime << log_n);
  const uint4 nfix = reinterpret_cast<const uint4*>(T.nfix)[prime];
  const int H = log_n - s0 - LOGR;  // > 0 in pass A, 0 in pass B
  const bool colblk = (H == 0);
  const int col0 = blockIdx.x * COLS;
  src += off;
  dst += off;

  for (int i = threadIdx.x; i < R * COLS; i += kThreads) {
    int r, c;
    size_t idx;
    if (H) {
      c = i & (COLS - 1);
      r = i >> LOGC;
      idx = ((size_t)r << H) + (size_t)(col0 + c);
    } else {
      r = i & (R - 1);
      c = i >> LOGR;
      idx = ((size_t)(col0 + c) << LOGR) + (size_t)r;
    }
    lds[r * PAD + c] = src[idx];
  }
  __syncthreads();
  if (FWD) {
    round_rb<LOGR, RB0, FWD>(lds, 0, s0, col0, colblk, q, tw, nfix);
    __syncthreads();
    round_rb<LOGR, RB1, FWD>(lds, RB0, s0, col0, colblk, q, tw, nfix);
  } else {
    round_rb<LOGR, RB1, FWD>(lds, RB0, s0, col0, colblk, q, tw, nfix);
    __syncthreads();
    round_rb<LOGR, RB0, FWD>(lds, 0, s0, col0, colblk, q, tw, nfix);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R * COLS; i += kThreads) {
    int r, c;
    size_t idx;
    if (H) {
      c = i & (COLS - 1);
      r = i >> LOGC;
      idx = ((size_t)r << H) + (size_t)(col0 + c);
    } else {
      r = i & (R - 1);
      c = i >> LOGR;
      idx = ((size_t)(col0 + c) << LOGR) + (size_t)r;
    }
    uint32_t v = lds[r * PAD + c];
    dst[idx] = last ? red1(v, q) : v;
  }
}

template <bool FWD>
void launch_pass(int logr, dim3 grid, hipStream_t s, const uint32_t* src, uint32_t* dst, const LimbMap& mp,
                 const DevTables& T, int log_n, int s0, int last) {
  switch (logr) {
    case 6: k_ntt_pass<6, FWD><<<grid, kThreads, 0, s>>>(src, dst, mp, T, log_n, s0, last); break;
    case 7: k_ntt_pass<7, FWD><<<grid, kThreads, 0, s>>>(src, dst, mp, T, log_n, s0, last); break;
    default: k_ntt_pass<8, FWD><<<grid, kThreads, 0, s>>>(src, dst, mp, T, log_n, s0, last); break;
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
  m.skip_groups = 0;
  m.job_stride = 0;
  return m;
}

int ntt_launch(const mick_params* prm, const uint32_t* src, uint32_t* dst, const LimbMap& map, int n_limbs, int n_jobs,
               bool inverse, hipStream_t s) {
  if (n_limbs <= 0 || n_jobs <= 0) return MICK_OK;
  if (n_limbs > 65535 || n_jobs > 65535) return set_error(MICK_E_ARG, "too many limbs for one transform launch");
  const int log_n = prm->log_n;
  dim3 grid(1u << (log_n - kTileLog), (unsigned)n_limbs, (unsigned)n_jobs);
  const int la = prm->split_a, lb = prm->split_b;
  if (!inverse) {
    launch_pass<true>(la, grid, s, src, dst, map, prm->dt, log_n, 0, 0);
    launch_pass<true>(lb, grid, s, dst, dst, map, prm->dt, log_n, la, 1);
  } else {
    launch_pass<false>(lb, grid, s, src, dst, map, prm->dt, log_n, la, 0);
    launch_pass<false>(la, grid, s, dst, dst, map, prm->dt, log_n, 0, 1);
  }
  return hip_error(hipGetLastError(), "ntt launch");
}

}  // namespace mick
