// Host-side number theory, random streams, samplers, FP64 codec and CRT.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace mick {

// ---------------------------------------------------------------- integers
uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m);
uint64_t powmod(uint64_t a, uint64_t e, uint64_t m);
uint64_t invmod(uint64_t a, uint64_t m);  // m prime
bool is_prime_u64(uint64_t n);
// The `count` largest primes below 2^bits that are 1 mod two_n, descending.
std::vector<uint32_t> ntt_primes(int bits, uint64_t two_n, int count);
// Smallest x >= 2 with x^n = -1 mod m (a primitive 2n-th root of unity).
uint32_t smallest_psi(uint32_t m, uint32_t n);
inline uint32_t shoup_companion(uint32_t w, uint32_t m) { return (uint32_t)(((uint64_t)w << 32) / m); }

// ---------------------------------------------------------------- random streams
// SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014) in counter mode.
uint64_t splitmix_mix(uint64_t z);
// n-th draw of the stream with key `key`: mix(key + (n + 1) * 0x9E3779B97F4A7C15).
uint64_t stream_draw(uint64_t key, uint64_t n);
// Stream key of (seed, tag, a, b, c); tag is up to 8 ASCII characters.
uint64_t stream_key(uint64_t seed, const char* tag, uint64_t a = 0, uint64_t b = 0, uint64_t c = 0);

// Exactly h entries in {+1, -1}, by partial Fisher-Yates over 0..n-1.
std::vector<int64_t> sample_ternary(uint64_t key, int n, int h);
// Discrete Gaussian by inversion of a cumulative table over [-B, B],
// B = floor(6 sigma).
struct GaussTable {
  int B;
  std::vector<uint64_t> T;  // 2B thresholds
};
GaussTable gauss_table(double sigma);
std::vector<int64_t> sample_gauss(uint64_t key, int n, const GaussTable& g);
// draw(key, i) mod m for i < n.
void sample_uniform(uint64_t key, uint32_t m, int n, uint32_t* out);

// ---------------------------------------------------------------- codec
void ckks_encode(int n, const double* re, const double* im, double scale, int64_t* m_out);
void ckks_decode(int n, const int64_t* m, double scale, double* re, double* im);

// ---------------------------------------------------------------- CRT
// Centred CRT of residues r[j], j < l, to a signed value; false if it does
// not fit in 62 bits of magnitude.  Garner's mixed-radix form.
struct Crt {
  std::vector<uint32_t> q;
  std::vector<std::vector<uint32_t>> inv;  // inv[i][j] = (q_j)^-1 mod q_i, j < i
  explicit Crt(const std::vector<uint32_t>& moduli);
  bool centred(const uint32_t* r, int64_t* out) const;
};

}  // namespace mick
