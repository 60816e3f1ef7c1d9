// Host-only checks of the library's C++ host code, built by
// tests/test_host_sanitized.py with the address and undefined-behaviour
// sanitizers (no GPU, no HIP):
//
//   host_check arena      random take / give sequences on the workspace
//                         arena of the work queue: blocks never overlap, stay
//                         inside the arena, the used count is exact, and
//                         freeing everything coalesces back to one block;
//   host_check samplers   prints the host samplers' outputs (primes, psi,
//                         stream keys, ternary, Gaussian, uniform, codec,
//                         CRT) as JSON for comparison with the oracle.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <random>
#include <string>
#include <vector>

#include "../../paper_2601_15401_amd/csrc/arena.h"
#include "../../paper_2601_15401_amd/csrc/host_math.h"

namespace {

int fail(const char* what) {
  fprintf(stderr, "FAIL: %s\n", what);
  return 1;
}

int check_arena() {
  std::mt19937_64 rng(12345);
  for (int round = 0; round < 50; round++) {
    const size_t size = (size_t)256 * (1 + rng() % 4096);
    mick::Arena a(size);
    struct Blk {
      size_t off, bytes;
    };
    std::vector<Blk> live;
    size_t used = 0;
    for (int step = 0; step < 4000; step++) {
      const bool take = live.empty() || (rng() % 100) < 55;
      if (take) {
        const size_t bytes = (size_t)256 * (1 + rng() % 64);
        const size_t off = a.take(bytes);
        if (off == SIZE_MAX) {
          if (a.largest_free() >= bytes) return fail("take refused a block that fits");
          continue;
        }
        if (off % 256 || off + bytes > size) return fail("block outside the arena or misaligned");
        for (const Blk& b : live)
          if (off < b.off + b.bytes && b.off < off + bytes) return fail("overlapping blocks");
        live.push_back({off, bytes});
        used += bytes;
      } else {
        const size_t i = rng() % live.size();
        a.give(live[i].off, live[i].bytes);
        used -= live[i].bytes;
        live[i] = live.back();
        live.pop_back();
      }
      if (a.used() != used) return fail("used count");
    }
    // fragment deliberately: free every other block, then the rest
    for (size_t i = 0; i < live.size(); i += 2) a.give(live[i].off, live[i].bytes);
    for (size_t i = 1; i < live.size(); i += 2) a.give(live[i].off, live[i].bytes);
    if (a.used() != 0) return fail("used after freeing everything");
    if (a.free_blocks() != 1 || a.largest_free() != size) return fail("free blocks did not coalesce");
    if (a.take(size) != 0) return fail("whole arena not available again");
    if (a.take(256) != SIZE_MAX) return fail("take from a full arena");
  }
  if (mick::Arena(0).take(256) != SIZE_MAX) return fail("empty arena");
  printf("{\"arena\": \"ok\"}\n");
  return 0;
}

void print_u64s(const char* name, const std::vector<uint64_t>& v, bool last = false) {
  printf("\"%s\": [", name);
  for (size_t i = 0; i < v.size(); i++) printf("%s\"%llu\"", i ? ", " : "", (unsigned long long)v[i]);
  printf("]%s\n", last ? "" : ",");
}

void print_i64s(const char* name, const std::vector<int64_t>& v) {
  printf("\"%s\": [", name);
  for (size_t i = 0; i < v.size(); i++) printf("%s%lld", i ? ", " : "", (long long)v[i]);
  printf("],\n");
}

int samplers() {
  printf("{\n");
  std::vector<uint64_t> q;
  for (uint32_t x : mick::ntt_primes(30, 1u << 14, 4)) q.push_back(x);
  print_u64s("primes30_n8192", q);
  std::vector<uint64_t> psi;
  for (uint64_t x : q) psi.push_back(mick::smallest_psi((uint32_t)x, 1u << 13));
  print_u64s("psi_n8192", psi);
  print_u64s("keys", {mick::stream_key(1, "SK"), mick::stream_key(7, "EVK_A", 3, 1, 5),
                      mick::stream_key(0xFFFFFFFFFFFFFFFFull, "ENC_V", 2)});
  std::vector<uint64_t> d;
  for (int n = 0; n < 8; n++) d.push_back(mick::stream_draw(0, n));
  print_u64s("draws0", d);
  print_i64s("ternary_key0_n4_h2", mick::sample_ternary(0, 4, 2));
  print_i64s("ternary_keyG_n4_h2", mick::sample_ternary(0x9E3779B97F4A7C15ull, 4, 2));
  print_i64s("ternary_sk_n64_h16", mick::sample_ternary(mick::stream_key(3, "SK"), 64, 16));
  const mick::GaussTable g = mick::gauss_table(3.2);
  print_u64s("gauss_table", g.T);
  print_i64s("gauss_64", mick::sample_gauss(mick::stream_key(11, "PK_E"), 64, g));
  std::vector<uint32_t> u(32);
  mick::sample_uniform(mick::stream_key(1, "PK_A", 0), (uint32_t)q[0], 32, u.data());
  print_u64s("uniform_32", std::vector<uint64_t>(u.begin(), u.end()));
  // codec round trip on 16 slots of N = 32
  const int n = 32;
  std::vector<double> re(n / 2), im(n / 2), re2(n / 2), im2(n / 2);
  for (int j = 0; j < n / 2; j++) {
    re[j] = 0.25 * j / n - 0.1;
    im[j] = 0.5 - 0.03 * j;
  }
  std::vector<int64_t> m(n);
  mick::ckks_encode(n, re.data(), im.data(), 1099511627776.0, m.data());
  print_i64s("encode_n32", m);
  mick::ckks_decode(n, m.data(), 1099511627776.0, re2.data(), im2.data());
  double err = 0;
  for (int j = 0; j < n / 2; j++) {
    err = std::max(err, std::abs(re2[j] - re[j]));
    err = std::max(err, std::abs(im2[j] - im[j]));
  }
  printf("\"codec_roundtrip_err\": %.3e,\n", err);
  // CRT of random signed values below 2^61 over the four primes
  std::vector<uint32_t> qs(q.begin(), q.end());
  mick::Crt crt(qs);
  std::mt19937_64 rng(7);
  int crt_bad = 0;
  for (int i = 0; i < 2000; i++) {
    const int64_t v = (int64_t)(rng() >> 3) * ((rng() & 1) ? 1 : -1);
    uint32_t r[4];
    for (int j = 0; j < 4; j++) {
      const int64_t x = v % (int64_t)qs[j];
      r[j] = (uint32_t)(x < 0 ? x + qs[j] : x);
    }
    int64_t out = 0;
    if (!crt.centred(r, &out) || out != v) crt_bad++;
  }
  printf("\"crt_mismatches\": %d,\n", crt_bad);
  printf("\"inv_pow\": [%llu, %llu]\n}\n", (unsigned long long)mick::invmod(12345, q[0]),
         (unsigned long long)mick::powmod(3, q[0] - 1, q[0]));
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) return fail("usage: host_check arena|samplers");
  if (!strcmp(argv[1], "arena")) return check_arena();
  if (!strcmp(argv[1], "samplers")) return samplers();
  return fail("unknown mode");
}
