// Tree-structured n-input multiply (Sec. V-C): products of polynomials in s
// at every node, Algorithm 1 (Sec. V-B) on every polynomial of a non-root
// node, relinearisation and the relocated multi-level rescale at the root;
// and the partition planner that minimises rescale units at depth
// ceil(log2 n).
//
// Trees travel as prefix tokens: g > 0 is a group of g consecutive inputs
// multiplied together, -m (m >= 2) an internal node whose m subtrees follow.
// Every subtree is evaluated at the level at which its result enters its
// parent (its inputs drop their top limbs first).
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "internal.h"
#include "rns.h"

using namespace mick;

namespace {

constexpr int kThreads = 256;
constexpr int kMaxTokens = 64;
constexpr int kMaxPlanInputs = 32;

// ---------------------------------------------------------------- node product

struct Operand {
  const uint32_t* p;  // [deg + 1][stride][N]
  int deg;
  int stride;         // limbs per polynomial of this operand
};

struct ProdArgs {
  Operand op[kMaxK];
  int m;              // operands
  int level;          // limbs of the product (a prefix of every operand's)
  int log_n;
};

// Coefficient t of the product of m polynomials in s is the sum over
// t_1 + ... + t_m = t of the pointwise products (Sec. V-A), accumulated
// operand by operand: acc' [t] = sum_b acc[t - b] op[b].  Every term is a
// product of m factors formed by m - 1 Montgomery products, so one final
// multiplication by R^(m-1) makes all of them exact.  Degrees are uniform
// across the launch, so the skipped (t, b) pairs are uniform branches.
template <int DOUT>
__global__ __launch_bounds__(kThreads) void k_polyprod(ProdArgs A, uint32_t* out, DevTables T) {
  const size_t N = (size_t)1 << A.log_n;
  const size_t n = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const int j = blockIdx.y;
  const uint32_t m = T.mod[j], minv = T.minv[j];
  uint32_t acc[DOUT + 1];
  {
    const Operand o = A.op[0];
#pragma unroll
    for (int i = 0; i <= DOUT; i++) acc[i] = i <= o.deg ? o.p[((size_t)i * o.stride + j) * N + n] : 0u;
  }
  int cur = A.op[0].deg;
  for (int c = 1; c < A.m; c++) {
    const Operand o = A.op[c];
    uint32_t x[DOUT + 1];
#pragma unroll
    for (int b = 0; b <= DOUT; b++) x[b] = b <= o.deg ? o.p[((size_t)b * o.stride + j) * N + n] : 0u;
    uint32_t nw[DOUT + 1];
#pragma unroll
    for (int t = 0; t <= DOUT; t++) {
      nw[t] = 0;
#pragma unroll
      for (int b = 0; b <= t; b++)
        if (b <= o.deg && t - b <= cur) nw[t] = add_mod(nw[t], mont_mul(acc[t - b], x[b], m, minv), m);
    }
#pragma unroll
    for (int t = 0; t <= DOUT; t++) acc[t] = nw[t];
    cur += o.deg;
  }
  const uint32_t* rp = T.rpow + (size_t)j * 2 * (kMaxK + 1) + 2 * (A.m - 1);
  const uint32_t f = rp[0], fsh = rp[1];
#pragma unroll
  for (int t = 0; t <= DOUT; t++) out[((size_t)t * A.level + j) * N + n] = shoup(acc[t], f, fsh, m);
}

int launch_polyprod(const mick_params* prm, const ProdArgs& A, int dout, uint32_t* out, hipStream_t s) {
  dim3 grid((unsigned)(prm->N / kThreads), (unsigned)A.level, 1);
  const DevTables& T = prm->dt;
  ProfScope ps(P_OTHER, s);
  switch (dout) {
#define MICK_P(D) \
  case D: k_polyprod<D><<<grid, kThreads, 0, s>>>(A, out, T); break;
    MICK_P(1) MICK_P(2) MICK_P(3) MICK_P(4) MICK_P(5) MICK_P(6) MICK_P(7) MICK_P(8) MICK_P(9) MICK_P(10) MICK_P(11)
    MICK_P(12)
#undef MICK_P
    default: return set_error(MICK_E_ARG, "product degree out of range (1..12)");
  }
  return hip_error(hipGetLastError(), "node product launch");
}

// ---------------------------------------------------------------- tree shape

struct Node {
  bool leaf;
  int g;                      // leaf: inputs in the group
  std::vector<int> kids;      // internal: node indices
  int first_input;            // leaf: index of its first input
  int n, deg, fan, depth;     // inputs, degree in s, factors of the product, levels consumed
  int prod_level, mu;         // level of the product, rescale depth after it
  size_t prod_off, res_off;   // workspace offsets (words) of the product and the rescaled result
};

struct Tree {
  std::vector<Node> nodes;    // nodes[0] is the root
  int n = 0;
  size_t scratch_off = 0;     // rescale scratch (words)
};

int parse(const int* tok, int len, int& pos, Tree& tr, int& next_input, int& out) {
  if (pos >= len) return set_error(MICK_E_ARG, "tree tokens end early");
  const int v = tok[pos++];
  if (v > kMaxPlanInputs || v < -kMaxTokens) return set_error(MICK_E_ARG, "tree token out of range");
  const int idx = (int)tr.nodes.size();
  tr.nodes.push_back(Node());
  if (v > 0) {
    Node& nd = tr.nodes[idx];
    nd.leaf = true;
    nd.g = v;
    nd.first_input = next_input;
    next_input += v;
    nd.n = nd.deg = nd.fan = v;
    nd.depth = v - 1;
  } else if (v <= -2) {
    std::vector<int> kids;
    for (int c = 0; c < -v; c++) {
      int k;
      MICK_TRY(parse(tok, len, pos, tr, next_input, k));
      kids.push_back(k);
    }
    Node& nd = tr.nodes[idx];
    nd.leaf = false;
    nd.kids = kids;
    nd.fan = -v;
    nd.n = 0;
    nd.depth = 0;
    for (int k : kids) {
      nd.n += tr.nodes[k].n;
      nd.depth = std::max(nd.depth, tr.nodes[k].depth);
    }
    nd.deg = nd.n;
    nd.depth += nd.fan - 1;
  } else {
    return set_error(MICK_E_ARG, "tree token must be a group size >= 1 or a node of >= 2 children (-m)");
  }
  out = idx;
  return MICK_OK;
}

int build_tree(const int* tok, int len, Tree& tr) {
  if (!tok || len < 1 || len > kMaxTokens) return set_error(MICK_E_ARG, "tree needs 1..64 tokens");
  int pos = 0, next = 0, root;
  MICK_TRY(parse(tok, len, pos, tr, next, root));
  if (pos != len) return set_error(MICK_E_ARG, "tree tokens left over after the root");
  tr.n = next;
  return MICK_OK;
}

// Levels top-down: the root's product is at out_level + (fan - 1); each
// child ends where its parent multiplies.
void place(Tree& tr, int idx, int end) {
  Node& nd = tr.nodes[idx];
  nd.mu = nd.fan - 1;
  nd.prod_level = end + nd.mu;
  if (!nd.leaf)
    for (int k : nd.kids) place(tr, k, nd.prod_level);
}

// Workspace: every non-root node that computes a product gets its product
// and its rescaled result; one rescale scratch; the root's multiply
// workspace last.  Returns words.
size_t layout(const mick_params* prm, Tree& tr) {
  const size_t N = prm->N;
  size_t off = 0, scratch = 0;
  for (size_t i = 1; i < tr.nodes.size(); i++) {
    Node& nd = tr.nodes[i];
    if (nd.leaf && nd.g == 1) continue;  // an input used as it is
    nd.prod_off = off;
    off += (size_t)(nd.deg + 1) * nd.prod_level * N;
    nd.res_off = off;
    off += (size_t)(nd.deg + 1) * (nd.prod_level - nd.mu) * N;
    scratch = std::max(scratch, (size_t)(nd.deg + 1) * nd.prod_level * N);
  }
  tr.scratch_off = off;
  off += scratch;
  tr.nodes[0].prod_off = off;  // D of the root multiply workspace
  return off + mul_ws_words(prm, tr.n, tr.nodes[0].prod_level);
}

int check_tree(const mick_params* prm, const int* tok, int len, int level, Tree& tr) {
  MICK_TRY(build_tree(tok, len, tr));
  if (tr.n < 2 || tr.n > kMaxK) return set_error(MICK_E_ARG, "the tree must take 2..12 inputs");
  if (level < 1 || level > prm->L) return set_error(MICK_E_LEVEL, "level must be in 1..L");
  const int out_level = level - tr.nodes[0].depth;
  if (out_level < 1) return set_error(MICK_E_LEVEL, "the tree is deeper than the level allows");
  place(tr, 0, out_level);
  return MICK_OK;
}

// Evaluates node idx (not the root) into its result buffer.
int eval(const mick_params* prm, Tree& tr, int idx, const uint32_t* const* cts, int level_in, uint32_t* ws,
         size_t scratch_off, hipStream_t s);

int node_product(const mick_params* prm, Tree& tr, int idx, const uint32_t* const* cts, int level_in, uint32_t* ws,
                 size_t scratch_off, uint32_t* prod, hipStream_t s) {
  Node& nd = tr.nodes[idx];
  ProdArgs A{};
  A.level = nd.prod_level;
  A.log_n = prm->log_n;
  if (nd.leaf) {
    A.m = nd.g;
    for (int u = 0; u < nd.g; u++) A.op[u] = Operand{cts[nd.first_input + u], 1, level_in};
  } else {
    A.m = (int)nd.kids.size();
    for (int c = 0; c < A.m; c++) {
      const int k = nd.kids[c];
      Node& ch = tr.nodes[k];
      if (ch.leaf && ch.g == 1) {
        A.op[c] = Operand{cts[ch.first_input], 1, level_in};
      } else {
        MICK_TRY(eval(prm, tr, k, cts, level_in, ws, scratch_off, s));
        A.op[c] = Operand{ws + ch.res_off, ch.deg, ch.prod_level - ch.mu};
      }
    }
  }
  return launch_polyprod(prm, A, nd.deg, prod, s);
}

int eval(const mick_params* prm, Tree& tr, int idx, const uint32_t* const* cts, int level_in, uint32_t* ws,
         size_t scratch_off, hipStream_t s) {
  Node& nd = tr.nodes[idx];
  MICK_TRY(node_product(prm, tr, idx, cts, level_in, ws, scratch_off, ws + nd.prod_off, s));
  return rescale_polys(prm, ws + nd.prod_off, nd.deg + 1, nd.prod_level, nd.mu, ws + nd.res_off, ws + scratch_off, s);
}

// ---------------------------------------------------------------- planner

struct Plan {
  bool ok = false;
  int units = 0;
  std::vector<int> tok;
};

void int_partitions(int n, int largest, std::vector<int>& cur, std::vector<std::vector<int>>& out) {
  if (n == 0) {
    out.push_back(cur);
    return;
  }
  for (int p = std::min(n, largest); p >= 1; p--) {
    cur.push_back(p);
    int_partitions(n - p, p, cur, out);
    cur.pop_back();
  }
}

// Fewest rescale units over trees of n inputs and depth <= max_depth: a
// single group first, then splits in descending lexicographic order of the
// part sizes; a later candidate replaces the best only when strictly better.
// A non-root node's product is rescaled (one unit per polynomial, n + 1 of
// them); the root's rescale follows relinearisation and is not counted.
Plan best(int n, int max_depth, bool root, std::map<std::tuple<int, int, bool>, Plan>& memo) {
  const auto key = std::make_tuple(n, max_depth, root);
  auto it = memo.find(key);
  if (it != memo.end()) return it->second;
  Plan b;
  if (n - 1 <= max_depth) {
    b.ok = true;
    b.units = (root || n == 1) ? 0 : n + 1;
    b.tok = {n};
  }
  std::vector<std::vector<int>> parts;
  std::vector<int> cur;
  int_partitions(n, n, cur, parts);
  for (const auto& pp : parts) {
    const int m = (int)pp.size();
    if (m < 2 || m - 1 > max_depth) continue;
    std::vector<Plan> subs;
    bool ok = true;
    int units = root ? 0 : n + 1;
    for (int p : pp) {
      subs.push_back(best(p, max_depth - (m - 1), false, memo));
      if (!subs.back().ok) {
        ok = false;
        break;
      }
      units += subs.back().units;
    }
    if (!ok) continue;
    if (!b.ok || units < b.units) {
      b.ok = true;
      b.units = units;
      b.tok = {-m};
      for (const auto& sp : subs) b.tok.insert(b.tok.end(), sp.tok.begin(), sp.tok.end());
    }
  }
  memo[key] = b;
  return b;
}

int ceil_log2(int n) {
  int d = 0;
  while ((1 << d) < n) d++;
  return d;
}

}  // namespace

extern "C" {

int mick_tree_plan(int n, int* tokens, int max_tokens) {
  if (!tokens) return set_error(MICK_E_ARG, "NULL tokens");
  if (n < 2 || n > kMaxPlanInputs) return set_error(MICK_E_ARG, "n must be in 2..32");
  std::map<std::tuple<int, int, bool>, Plan> memo;
  const Plan p = best(n, ceil_log2(n), true, memo);
  if ((int)p.tok.size() > max_tokens) return set_error(MICK_E_ARG, "max_tokens too small for the plan");
  memcpy(tokens, p.tok.data(), p.tok.size() * sizeof(int));
  return (int)p.tok.size();
}

int mick_tree_shape(const int* tokens, int n_tokens, int* n_inputs, int* depth, int* rs_units) {
  Tree tr;
  MICK_TRY(build_tree(tokens, n_tokens, tr));
  if (n_inputs) *n_inputs = tr.n;
  if (depth) *depth = tr.nodes[0].depth;
  if (rs_units) {
    int u = 0;
    for (size_t i = 1; i < tr.nodes.size(); i++)
      if (tr.nodes[i].fan > 1) u += tr.nodes[i].deg + 1;
    *rs_units = u;
  }
  return MICK_OK;
}

size_t mick_tree_workspace_bytes(const mick_params* prm, const int* tokens, int n_tokens, int level) {
  if (!prm) return 0;
  Tree tr;
  if (check_tree(prm, tokens, n_tokens, level, tr) != MICK_OK) return 0;
  return layout(prm, tr) * 4;
}

int mick_mul_tree(const mick_params* prm, const mick_keys* keys, const uint32_t* const* cts_host, int level,
                  const int* tokens, int n_tokens, uint32_t* ct_out_dev, void* ws, size_t ws_bytes, void* stream) {
  if (!prm || !keys || !cts_host || !ct_out_dev || !ws) return set_error(MICK_E_ARG, "NULL argument");
  if (keys->prm != prm) return set_error(MICK_E_ARG, "keys belong to other params");
  Tree tr;
  MICK_TRY(check_tree(prm, tokens, n_tokens, level, tr));
  if (tr.n > keys->k_max) return set_error(MICK_E_KEY, "the tree needs keys up to s^n beyond the key set's k_max");
  for (int u = 0; u < tr.n; u++)
    if (!cts_host[u]) return set_error(MICK_E_ARG, "NULL ciphertext pointer");
  const size_t words = layout(prm, tr);
  if (ws_bytes < words * 4) return set_error(MICK_E_WS, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  uint32_t* w = (uint32_t*)ws;
  const size_t scratch_off = tr.scratch_off;
  Node& root = tr.nodes[0];
  uint32_t* rws = w + root.prod_off;  // D of the root's multiply workspace is at its start
  MICK_TRY(node_product(prm, tr, 0, cts_host, level, w, scratch_off, rws, s));
  return relin_rescale_one(prm, keys, tr.n, root.prod_level, root.mu, rws, ct_out_dev, s);
}

}  // extern "C"
