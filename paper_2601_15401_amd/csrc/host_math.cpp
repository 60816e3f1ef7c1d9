// Host-side number theory, random streams, samplers, codec and CRT.
#include "host_math.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>

namespace mick {

// ---------------------------------------------------------------- integers

uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod64(r, a, m);
    a = mulmod64(a, a, m);
    e >>= 1;
  }
  return r;
}

uint64_t invmod(uint64_t a, uint64_t m) { return powmod(a % m, m - 2, m); }

// Deterministic Miller-Rabin; the first 12 prime bases are exact far beyond 2^64.
bool is_prime_u64(uint64_t n) {
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t p : bases) {
    if (n % p == 0) return n == p;
  }
  uint64_t d = n - 1;
  int r = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    r++;
  }
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool composite = true;
    for (int i = 1; i < r; i++) {
      x = mulmod64(x, x, n);
      if (x == n - 1) {
        composite = false;
        break;
      }
    }
    if (composite) return false;
  }
  return true;
}

std::vector<uint32_t> ntt_primes(int bits, uint64_t two_n, int count) {
  std::vector<uint32_t> out;
  uint64_t top = (uint64_t)1 << bits;
  // largest candidate of the form c * two_n + 1 below 2^bits
  uint64_t x = ((top - 2) / two_n) * two_n + 1;
  while ((int)out.size() < count && x > two_n) {
    if (is_prime_u64(x)) out.push_back((uint32_t)x);
    x -= two_n;
  }
  return out;
}

uint32_t smallest_psi(uint32_t m, uint32_t n) {
  // x^n = -1 has exactly n solutions, the odd powers of any one of them.
  uint64_t e = (m - 1) / (2 * (uint64_t)n);
  uint64_t root = 0;
  for (uint64_t g = 2; g < m; g++) {
    uint64_t c = powmod(g, e, m);
    if (powmod(c, n, m) == m - 1) {
      root = c;
      break;
    }
  }
  uint64_t sq = mulmod64(root, root, m), x = root, best = m;
  for (uint32_t i = 0; i < n; i++) {
    best = std::min(best, x);
    x = mulmod64(x, sq, m);
  }
  return (uint32_t)best;
}

// ---------------------------------------------------------------- random streams

static const uint64_t kGamma = 0x9E3779B97F4A7C15ull;

uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t stream_draw(uint64_t key, uint64_t n) { return splitmix_mix(key + (n + 1) * kGamma); }

uint64_t stream_key(uint64_t seed, const char* tag, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t t = 0;
  size_t len = strlen(tag);
  for (size_t i = 0; i < len && i < 8; i++) t |= (uint64_t)(unsigned char)tag[i] << (8 * i);
  uint64_t h = splitmix_mix(seed + kGamma);
  const uint64_t words[4] = {t, a, b, c};
  for (uint64_t w : words) h = splitmix_mix((h ^ w) + kGamma);
  return h;
}

std::vector<int64_t> sample_ternary(uint64_t key, int n, int h) {
  std::vector<int64_t> out(n, 0);
  std::vector<int> idx(n);
  for (int i = 0; i < n; i++) idx[i] = i;
  for (int i = 0; i < h; i++) {
    uint64_t pick = stream_draw(key, 2 * (uint64_t)i);
    uint64_t sign = stream_draw(key, 2 * (uint64_t)i + 1);
    int j = i + (int)(pick % (uint64_t)(n - i));
    std::swap(idx[i], idx[j]);
    out[idx[i]] = (sign & 1) ? -1 : 1;
  }
  return out;
}

GaussTable gauss_table(double sigma) {
  GaussTable g;
  g.B = (int)floor(6.0 * sigma);
  std::vector<double> rho;
  for (int x = -g.B; x <= g.B; x++) rho.push_back(exp(-(double)(x * x) / (2.0 * sigma * sigma)));
  double S = 0.0;
  for (double r : rho) S += r;
  double c = 0.0;
  for (size_t i = 0; i + 1 < rho.size(); i++) {
    c += rho[i];
    g.T.push_back((uint64_t)((c / S) * 18446744073709551616.0));
  }
  return g;
}

std::vector<int64_t> sample_gauss(uint64_t key, int n, const GaussTable& g) {
  std::vector<int64_t> out(n);
  for (int i = 0; i < n; i++) {
    uint64_t u = stream_draw(key, (uint64_t)i);
    // number of thresholds <= u
    int cnt = (int)(std::upper_bound(g.T.begin(), g.T.end(), u) - g.T.begin());
    out[i] = (int64_t)cnt - g.B;
  }
  return out;
}

void sample_uniform(uint64_t key, uint32_t m, int n, uint32_t* out) {
  for (int i = 0; i < n; i++) out[i] = (uint32_t)(stream_draw(key, (uint64_t)i) % m);
}

// ---------------------------------------------------------------- codec

typedef std::complex<double> cplx;

// In-place iterative radix-2 FFT; sign -1: sum x_r exp(-2 pi i r k / n).
static void fft(std::vector<cplx>& a, int sign) {
  size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; i++) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    size_t half = len / 2;
    for (size_t k = 0; k < half; k++) {
      double ang = sign * 2.0 * M_PI * (double)k / (double)len;
      cplx w(cos(ang), sin(ang));
      for (size_t i = 0; i < n; i += len) {
        cplx u = a[i + k], v = a[i + k + half] * w;
        a[i + k] = u + v;
        a[i + k + half] = u - v;
      }
    }
  }
}

static std::vector<int64_t> slot_powers(int n) {
  std::vector<int64_t> r(n / 2);
  int64_t v = 1;
  for (int j = 0; j < n / 2; j++) {
    r[j] = v;
    v = v * 5 % (2 * n);
  }
  return r;
}

void ckks_encode(int n, const double* re, const double* im, double scale, int64_t* m_out) {
  std::vector<cplx> w(2 * (size_t)n, cplx(0, 0));
  std::vector<int64_t> r = slot_powers(n);
  for (int j = 0; j < n / 2; j++) w[r[j]] = cplx(scale * re[j], scale * im[j]);
  fft(w, -1);
  for (int i = 0; i < n; i++) {
    double v = (2.0 / n) * w[i].real();
    double a = floor(fabs(v) + 0.5);
    m_out[i] = (int64_t)(v < 0 ? -a : a);
  }
}

void ckks_decode(int n, const int64_t* m, double scale, double* re, double* im) {
  std::vector<cplx> w(2 * (size_t)n, cplx(0, 0));
  for (int i = 0; i < n; i++) w[i] = cplx((double)m[i], 0.0);
  fft(w, +1);
  std::vector<int64_t> r = slot_powers(n);
  for (int j = 0; j < n / 2; j++) {
    re[j] = w[r[j]].real() / scale;
    im[j] = w[r[j]].imag() / scale;
  }
}

// ---------------------------------------------------------------- CRT

Crt::Crt(const std::vector<uint32_t>& moduli) : q(moduli) {
  inv.resize(q.size());
  for (size_t i = 0; i < q.size(); i++)
    for (size_t j = 0; j < i; j++) inv[i].push_back((uint32_t)invmod(q[j] % q[i], q[i]));
}

// Multi-word helpers on little-endian base-2^32 arrays.
static void big_muladd(std::vector<uint32_t>& x, uint32_t mul, uint32_t add) {
  uint64_t carry = add;
  for (auto& w : x) {
    uint64_t t = (uint64_t)w * mul + carry;
    w = (uint32_t)t;
    carry = t >> 32;
  }
  if (carry) x.push_back((uint32_t)carry);
}

static int big_cmp(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  size_t n = std::max(a.size(), b.size());
  for (size_t i = n; i-- > 0;) {
    uint32_t x = i < a.size() ? a[i] : 0, y = i < b.size() ? b[i] : 0;
    if (x != y) return x < y ? -1 : 1;
  }
  return 0;
}

static std::vector<uint32_t> big_sub(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  std::vector<uint32_t> r(a.size());
  int64_t borrow = 0;
  for (size_t i = 0; i < a.size(); i++) {
    int64_t t = (int64_t)a[i] - (i < b.size() ? b[i] : 0) - borrow;
    borrow = t < 0;
    r[i] = (uint32_t)(t + (borrow << 32));
  }
  return r;
}

bool Crt::centred(const uint32_t* r, int64_t* out) const {
  const size_t l = q.size();
  // mixed-radix digits v_i in [0, q_i): x = v_0 + v_1 q_0 + v_2 q_0 q_1 + ...
  std::vector<uint32_t> v(l);
  for (size_t i = 0; i < l; i++) {
    uint64_t t = r[i] % q[i];
    for (size_t j = 0; j < i; j++) {
      t = (t + q[i] - v[j] % q[i]) % q[i];
      t = t * inv[i][j] % q[i];
    }
    v[i] = (uint32_t)t;
  }
  std::vector<uint32_t> x(1, 0), Q(1, 1);
  for (size_t i = l; i-- > 0;) big_muladd(x, q[i], v[i]);
  for (size_t i = 0; i < l; i++) big_muladd(Q, q[i], 0);
  std::vector<uint32_t> half = Q;  // floor(Q / 2)
  for (size_t i = 0; i < half.size(); i++) {
    half[i] = (half[i] >> 1) | (i + 1 < half.size() ? half[i + 1] << 31 : 0);
  }
  bool neg = big_cmp(x, half) > 0;
  std::vector<uint32_t> mag = neg ? big_sub(Q, x) : x;
  for (size_t i = 2; i < mag.size(); i++)
    if (mag[i]) return false;
  uint64_t m = (uint64_t)mag[0] | ((mag.size() > 1 ? (uint64_t)mag[1] : 0) << 32);
  if (m >> 62) return false;
  *out = neg ? -(int64_t)m : (int64_t)m;
  return true;
}

}  // namespace mick
