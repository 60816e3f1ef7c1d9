// Building blocks of the negacyclic transform passes shared by the transform,
// ModUp, key-product and tensor-product kernels (ntt.hip, tensor.hip).
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
// A workgroup owns a tile of one limb (8192 elements; 1024 in the key-product
// kernel): 2^LOGR butterfly rows by tile / 2^LOGR independent columns (pass
// A: columns are consecutive low indices; pass B: columns are consecutive
// 2^LB-element blocks).  A pass is
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
#pragma once
#include "internal.h"
#include "rns.h"

namespace mick {

namespace {

constexpr int kThreads = 256;
constexpr int kTileLog = 13;

// TL: log2 of the tile's element count (8192 for the transform passes).
// XP: extra words between blocks of 2^RB1 rows (-1: the default below).
// PD: row pitch (-1: the padded pitch below).
template <int LOGR, int TL = kTileLog, int XP = -1, int PD = -1>
struct Geo {
  static constexpr int LOGC = TL - LOGR;
  static constexpr int COLS = 1 << LOGC;
  static constexpr int RB0 = (LOGR == 6) ? 3 : 4;
  static constexpr int RB1 = LOGR - RB0;
  // LDS row pitch.  Pass B's strided round gives each column 2^(LOGR-RB0)
  // consecutive lanes (rows lo, lo + 2^(LOGR-RB0), ...), so a 32-lane half
  // touches 32 >> (LOGR-RB0) columns; a pitch of COLS + that count puts
  // their lanes on distinct banks.
  static constexpr int PAD = PD >= 0 ? PD : COLS + (32 >> (LOGR - RB0));
  // Rows are stored in blocks of 2^RB1 (one consecutive-round item per
  // column), BP words apart.  With 32 or more columns a half-wave of the
  // consecutive round reads 32 columns of one row: conflict-free with
  // BP = 2^RB1 PAD, i.e. plain rows of PAD words.  Narrower tiles (the
  // key-product and fused tensor kernels) put 32 / COLS blocks in one
  // half-wave; 2^RB1 PAD is a multiple of 32 there, so every block would hit
  // the same COLS banks.  A block pitch of COLS times an odd number (mod 32)
  // spreads them over all 32 banks, and leaves the strided round's lanes
  // (one block, distinct rows) as they were.
  static constexpr int XPAD = XP >= 0 ? XP : (COLS >= 32 ? 0 : COLS);
  static constexpr int BP = (PAD << RB1) + XPAD;
  static constexpr int LDS_WORDS = BP << RB0;
  __device__ static int off(int r, int c) { return (r >> RB1) * BP + (r & ((1 << RB1) - 1)) * PAD + c; }
};

// Item layout of one round.  An item is one column c and 2^RB rows
// rbase + j 2^NLO_LOG, j < 2^RB.
template <int LOGR, bool PASSB, bool STRIDED, int NT = kThreads, int TL = kTileLog>
struct Rnd {
  using G = Geo<LOGR, TL>;
  static constexpr int RB = STRIDED ? G::RB0 : G::RB1;
  static constexpr int E = 1 << RB;
  static constexpr int SL0 = STRIDED ? 0 : G::RB0;  // first local stage of the round
  static constexpr int NLO_LOG = STRIDED ? LOGR - G::RB0 : 0;
  static constexpr int ITEMS = (1 << TL) >> RB;
  static constexpr int NI = ITEMS / NT;  // items per thread
  // pass B's strided round walks the rows of a column with consecutive lanes
  static constexpr bool LO_FAST = PASSB && STRIDED;
  // pass B's consecutive round moves 2^RB neighbouring words per lane
  static constexpr bool VEC = PASSB && !STRIDED;

  __device__ static void decode(int it, int& c, int& rbase, int& hi) {
    int lo;
    if constexpr (LO_FAST) {
      lo = it & ((1 << NLO_LOG) - 1);
      c = it >> NLO_LOG;
      hi = 0;
    } else {
      c = it & (G::COLS - 1);
      const int hl = it >> G::LOGC;
      lo = STRIDED ? hl : 0;
      hi = STRIDED ? 0 : hl;
    }
    rbase = (hi << (LOGR - SL0)) + lo;
  }
  __device__ static int row(int rbase, int j) { return rbase + (j << NLO_LOG); }
  __device__ static uint32_t gidx(int H, int col, int r) {  // < N <= 2^16
    return PASSB ? ((uint32_t)col << LOGR) + r : ((uint32_t)r << H) + col;
  }
};

// Forward (Cooley-Tukey) butterfly.  The forward twiddle table stores each
// twiddle negated, w.x = 2^32 - w (w.y is the Shoup companion of w itself),
// so one chain of two multiply-adds gives nt = h q - y w mod 2^32 = -t for
// the lazy Shoup product t = y w - h q in [0, 2q), h = floor(y w' / 2^32);
// then x + t and x - t + 2q are a subtraction and one three-operand add.
// Primes above 2^30 (2q < 2^32 <= 4q) keep values below 2q: the chain adds
// q as well, v = q - t mod 2^32, and s = min(v, v + q) lies in [0, q] with
// s = q - t mod q (t < q: s = v; t >= q: v wraps, v + q = 2q - t), so the
// outputs are a + q - s and a + s for the reduced x = a in [0, q): ten
// instructions.
template <bool LAZY>
__device__ __forceinline__ void ct(uint32_t& x, uint32_t& y, uint2 w, uint32_t q) {
  if constexpr (LAZY) {  // x, y < 4q -> outputs < 4q
    const uint32_t nt = mad2_lo(y, w.x, __umulhi(y, w.y), q);
    const uint32_t a = min(x, x - 2 * q);
    x = a - nt;
    y = a + nt + 2 * q;
  } else {  // x < 2q -> outputs < 2q
    const uint32_t v = mad2_lo_add(y, w.x, __umulhi(y, w.y), q, q);
    const uint32_t s = min(v, v + q);
    const uint32_t a = red1(x, q);
    x = a - s + q;
    y = a + s;
  }
}

// Inverse (Gentleman-Sande) butterfly, values < 2q throughout.  The inverse
// table stores twiddles as they are; the Shoup products take 2^32 - q.
template <bool LAZY>
__device__ __forceinline__ void gs(uint32_t& x, uint32_t& y, uint2 w, uint32_t q) {
  if constexpr (LAZY) {
    uint32_t u = x + y;
    uint32_t v = x - y + 2 * q;
    x = min(u, u - 2 * q);
    y = shoup_lazy_neg(v, w.x, w.y, 0u - q);
  } else {
    uint32_t a = red1(x, q), b = red1(y, q);
    x = a + b;
    y = shoup_lazy_neg(a - b + q, w.x, w.y, 0u - q);
  }
}

// The last inverse stage with N^-1 (times a per-limb factor) merged into both
// outputs: nf = (f, f', w1 f, (w1 f)').
template <bool LAZY>
__device__ __forceinline__ void gs_last(uint32_t& x, uint32_t& y, const uint4& nf, uint32_t q) {
  if constexpr (LAZY) {
    uint32_t u = x + y, v = x - y + 2 * q;
    x = shoup_lazy_neg(u, nf.x, nf.y, 0u - q);
    y = shoup_lazy_neg(v, nf.z, nf.w, 0u - q);
  } else {
    uint32_t a = red1(x, q), b = red1(y, q);
    x = shoup_lazy_neg(a + b, nf.x, nf.y, 0u - q);
    y = shoup_lazy_neg(a - b + q, nf.z, nf.w, 0u - q);
  }
}

template <bool FWD, bool LAZY>
__device__ __forceinline__ uint32_t canonical(uint32_t v, uint32_t q) {
  if constexpr (FWD && LAZY) v = min(v, v - 2 * q);
  return red1(v, q);
}

// Butterflies of one item: fetches the round's twiddles (stage u of the
// round uses 2^u of them; TW(s, rr) returns the twiddle of global stage s,
// local block rr), then runs the RB stages in order (forward) or reverse
// order (inverse).  HAS_STAGE0: the round contains global stage 0 of an
// inverse transform, which takes nfix instead of a twiddle.
template <int RB, bool FWD, bool LAZY, bool HAS_STAGE0, typename TW>
__device__ __forceinline__ void item_bfly_t(uint32_t (&x)[1 << RB], const TW& twf, int s_first, int hi, uint32_t q,
                                            const uint4& nfix) {
  constexpr int E = 1 << RB;
  uint2 w[E];
#pragma unroll
  for (int u = 0; u < RB; u++) {
    if (HAS_STAGE0 && u == 0) continue;
#pragma unroll
    for (int g = 0; g < (1 << u); g++) w[(1 << u) + g] = twf(s_first + u, u, (hi << u) + g);
  }
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
}

// Twiddles read from the per-prime table in global memory.
struct TwGlobal {
  const uint2* tw;
  int s0, blk;
  __device__ uint2 operator()(int s, int, int rr) const { return tw[(1 << s) + (rr << s0) + blk]; }
};

// Pass A's twiddles do not depend on the column: a tile uses tw[1 .. 2^LOGR)
// of its prime, staged in LDS once per block.
struct TwPassA {
  const uint2* t;
  __device__ uint2 operator()(int s, int, int rr) const { return t[(1 << s) + rr]; }
};

template <int LOGR, int NT = kThreads>
__device__ __forceinline__ void stage_tw_pass_a(uint2* ltwa, const uint2* tw) {
  for (int i = threadIdx.x; i < (1 << LOGR); i += NT) ltwa[i] = tw[i];
}

// The tile's pass-B twiddles staged in LDS: stage s0 + sl at COLS (2^sl - 1),
// then 2^sl blocks of COLS columns.  The strided round's stages (sl < RB0)
// hold block rr at position rr; every lane of a column reads the same
// entry.  In a stage of the consecutive round (u = sl - RB0) the item with
// row block hi reads blocks rr = hi 2^u + g, g < 2^u; block rr sits at
// position g 2^RB0 + hi, so that for each g the lanes (row block, column)
// of a wave read consecutive entries.
template <int RB0>
__device__ __forceinline__ int tw_pos(int sl, int rr) {
  if (sl < RB0) return rr;
  const int u = sl - RB0;
  return ((rr & ((1 << u) - 1)) << RB0) + (rr >> u);
}

template <int COLS, int RB0>
struct TwLds {
  const uint2* t;
  int s0, c;
  __device__ uint2 operator()(int s, int, int rr) const {
    const int sl = s - s0;
    return t[COLS * ((1 << sl) - 1) + tw_pos<RB0>(sl, rr) * COLS + c];
  }
};

// Stages the pass-B twiddles of the tile's first NSL stages (sl < NSL) in
// the TwLds layout; every load is issued before the first LDS store.
template <int COLS, int NSL, int NT, int RB0>
__device__ __forceinline__ void stage_tw_pass_b(uint2* ltw, const uint2* tw, int s0, int col0) {
  constexpr int LOGC = __builtin_ctz(COLS);
  constexpr int NTW = COLS * ((1 << NSL) - 1);
  constexpr int IT = (NTW + NT - 1) / NT;
  uint2 t[IT];
#pragma unroll
  for (int it = 0; it < IT; it++) {
    const int i = it * NT + threadIdx.x;
    if (i < NTW) {
      const int c = i & (COLS - 1);
      const int k = i >> LOGC;  // (2^sl - 1) + position
      const int sl = 31 - __clz(k + 1);
      const int pos = k + 1 - (1 << sl);
      const int u = sl - RB0;  // the inverse of tw_pos
      const int rr = u < 0 ? pos : ((pos & ((1 << RB0) - 1)) << u) + (pos >> RB0);
      t[it] = tw[(1 << (s0 + sl)) + (rr << s0) + col0 + c];
    }
  }
#pragma unroll
  for (int it = 0; it < IT; it++) {
    const int i = it * NT + threadIdx.x;
    if (i < NTW) ltw[i] = t[it];
  }
}

// LDS twiddle words of a transform pass: the forward pass A stages pass A's
// twiddles; the inverse pass B at LOGR = 8 stages its strided round's
// per-column twiddles (3.75 KB, which keeps four workgroups per CU).
template <int LOGR, bool FWD, bool PASSB>
constexpr int pass_tw_words() {
  return FWD && !PASSB ? 1 << LOGR : (!FWD && PASSB && LOGR == 8 ? Geo<LOGR>::COLS * ((1 << Geo<LOGR>::RB0) - 1) : 1);
}

template <int RB, bool FWD, bool LAZY, bool HAS_STAGE0>
__device__ __forceinline__ void item_bfly(uint32_t (&x)[1 << RB], const uint2* tw, int s_first, int s0, int hi,
                                          int blk, uint32_t q, const uint4& nfix) {
  item_bfly_t<RB, FWD, LAZY, HAS_STAGE0>(x, TwGlobal{tw, s0, blk}, s_first, hi, q, nfix);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Global accesses of one item.  STREAM marks data touched once per pass
// (nontemporal: it should not displace the twiddles other tiles reuse).
template <typename RD, bool STREAM = false>
__device__ __forceinline__ void load_global(uint32_t (&x)[RD::E], const uint32_t* g, int H, int col, int rbase) {
  if constexpr (RD::VEC) {
#pragma unroll
    for (int j = 0; j < RD::E; j += 4) {
      const u32x4* p = reinterpret_cast<const u32x4*>(g + RD::gidx(H, col, rbase + j));
      const u32x4 v = STREAM ? __builtin_nontemporal_load(p) : *p;
      x[j] = v.x;
      x[j + 1] = v.y;
      x[j + 2] = v.z;
      x[j + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < RD::E; j++) {
      const uint32_t* p = g + RD::gidx(H, col, RD::row(rbase, j));
      x[j] = STREAM ? __builtin_nontemporal_load(p) : *p;
    }
  }
}

template <typename RD, bool STREAM = false>
__device__ __forceinline__ void store_global(const uint32_t (&x)[RD::E], uint32_t* g, int H, int col, int rbase) {
  if constexpr (RD::VEC) {
#pragma unroll
    for (int j = 0; j < RD::E; j += 4) {
      u32x4 o;
      o.x = x[j];
      o.y = x[j + 1];
      o.z = x[j + 2];
      o.w = x[j + 3];
      u32x4* p = reinterpret_cast<u32x4*>(g + RD::gidx(H, col, rbase + j));
      if constexpr (STREAM)
        __builtin_nontemporal_store(o, p);
      else
        *p = o;
    }
  } else {
#pragma unroll
    for (int j = 0; j < RD::E; j++) {
      uint32_t* p = g + RD::gidx(H, col, RD::row(rbase, j));
      if constexpr (STREAM)
        __builtin_nontemporal_store(x[j], p);
      else
        *p = x[j];
    }
  }
}

// Element j of an item sits at base + j step: the strided round walks the
// blocks of a column (rows lo + j 2^RB1), the consecutive round the rows of
// one block.
template <typename RD, typename G>
__device__ __forceinline__ void lds_item(int c, int rbase, int& base, int& step) {
  static_assert(RD::NLO_LOG == 0 || RD::NLO_LOG == G::RB1, "rounds of this geometry");
  base = G::off(rbase, c);
  step = RD::NLO_LOG == 0 ? G::PAD : G::BP;
}

template <typename RD, typename G>
__device__ __forceinline__ void load_lds(uint32_t (&x)[RD::E], const uint32_t* lds, int c, int rbase) {
  int base, step;
  lds_item<RD, G>(c, rbase, base, step);
#pragma unroll
  for (int j = 0; j < RD::E; j++) x[j] = lds[base + j * step];
}

template <typename RD, typename G>
__device__ __forceinline__ void store_lds(const uint32_t (&x)[RD::E], uint32_t* lds, int c, int rbase) {
  int base, step;
  lds_item<RD, G>(c, rbase, base, step);
#pragma unroll
  for (int j = 0; j < RD::E; j++) lds[base + j * step] = x[j];
}

}  // namespace

}  // namespace mick
