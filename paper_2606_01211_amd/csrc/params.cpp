// Parameter registry, CDF tables and AES tables of liblwe_hip (host side).
#include <math.h>
#include <string.h>

#include <deque>
#include <mutex>
#include <vector>

#include "lwe_internal.h"

namespace lwe {

// Error-distribution table of a centred discrete Gaussian of width sigma on [-K, K]:
// T[k] + 1 = round(2^15 * P(|x| <= k)) for k < K and T[K] = 2^15 - 1, where P is the
// Gaussian mass restricted to the support, accumulated in increasing |x| in double.
// A 16-bit keystream word u yields |e| = #{k < K : (u >> 1) > T[k]} and sign bit u & 1.
bool build_cdf(int K, double sigma, uint16_t* T) {
  if (K < 1 || K > MAX_K || !(sigma > 0)) return false;
  std::vector<double> cum(K + 1);
  double s = 1.0;
  cum[0] = s;
  for (int x = 1; x <= K; ++x) {
    const double xd = (double)x;
    s += 2.0 * exp(-(xd * xd) / (2.0 * sigma * sigma));
    cum[x] = s;
  }
  for (int k = 0; k < K; ++k) T[k] = (uint16_t)(floor(32768.0 * (cum[k] / cum[K]) + 0.5) - 1.0);
  T[K] = 32767;
  for (int k = 1; k <= K; ++k)
    if (T[k] <= T[k - 1]) return false;
  return true;
}

static std::mutex g_reg_mu;
// a deque keeps Params addresses stable when sets are registered later
static std::deque<Params>& registry() {
  static std::deque<Params> reg;
  static bool init = false;
  if (!init) {
    init = true;
    // n, logq, B, K, sigma.  n, q and the support follow the evaluated workloads; sigma is
    // the paper's Table 1 value where that leaves mass on the whole support, else K/4.3.
    const struct { int n, logq, B, K; double sigma; } base[] = {
        {640, 15, 2, 12, 2.8},  {976, 16, 3, 10, 2.3},  {1344, 16, 4, 6, 1.4},
        {4096, 16, 4, 6, 1.4},  {8192, 16, 4, 6, 1.4},  {16384, 16, 3, 6, 1.4},
        {32768, 16, 3, 6, 1.4},
    };
    for (const auto& b : base) {
      Params p;
      memset(&p, 0, sizeof(p));
      p.n = b.n;
      p.logq = b.logq;
      p.B = b.B;
      p.K = b.K;
      p.sigma = b.sigma;
      build_cdf(p.K, p.sigma, p.T);
      finish_params(p);
      reg.push_back(p);
    }
    // The paper's own sets, Table 1: n, prime q, sigma of e / r / e1, k of e2 (eta = 3 for s).
    // The Gaussian's support is the largest K whose 15-bit table stays strictly increasing.
    const struct { int n; uint32_t q; double sigma; int ku; } table1[] = {
        {512, 3329, 2.3, 3},    {1024, 12289, 2.3, 3}, {2048, 12289, 2.3, 3}, {4096, 12289, 1.7, 3},
        {8192, 65537, 1.2, 2},  {16384, 65537, 1.2, 2}, {32768, 65537, 1.0, 2},
    };
    for (const auto& b : table1) {
      Params p;
      memset(&p, 0, sizeof(p));
      p.paper = 1;
      p.n = b.n;
      p.q = b.q;
      p.sigma = b.sigma;
      p.ku = b.ku;
      p.eta = 3;
      p.B = 1;
      for (int K = 1; K <= MAX_K; ++K) {
        uint16_t T[MAX_K + 1];
        if (build_cdf(K, p.sigma, T)) p.K = K;
      }
      build_cdf(p.K, p.sigma, p.T);
      int bits = 0;
      while ((1u << bits) < p.q) ++bits;
      p.logq = bits;  // informational: bits of q
      finish_params(p);
      reg.push_back(p);
    }
  }
  return reg;
}

void finish_params(Params& p) {
  p.ldx = (p.n + 63) / 64 * 64;
  if (p.paper) {
    p.nbar = 1;
    p.mbar = PB_BITS;
    p.coef_bytes = p.q > 65536 ? 4 : 2;
    p.pk_bytes = 16 + (size_t)p.n * p.coef_bytes;
    p.sk_bytes = 2 * (size_t)p.n + p.pk_bytes + 64;
    p.ct_bytes = (size_t)PB_BITS * ((size_t)p.n + 1) * p.coef_bytes;
    p.mu_bytes = PB_BITS / 8;
    return;
  }
  p.q = 1u << p.logq;
  p.nbar = NBAR;
  p.mbar = MBAR;
  p.coef_bytes = 2;
  p.pk_bytes = 16 + (size_t)NBAR * p.n * 2;
  p.sk_bytes = (size_t)NBAR * p.n * 2 + p.pk_bytes + 64;
  p.ct_bytes = (size_t)MBAR * p.n * 2 + (size_t)MBAR * NBAR * 2;
  p.mu_bytes = (size_t)MBAR * NBAR * p.B / 8;
}

const Params* get_params(int pid) {
  std::lock_guard<std::mutex> g(g_reg_mu);
  auto& reg = registry();
  if (pid < 0 || pid >= (int)reg.size()) return nullptr;
  return &reg[pid];
}

int find_param(uint32_t n) {
  std::lock_guard<std::mutex> g(g_reg_mu);
  auto& reg = registry();
  for (size_t k = 0; k < reg.size(); ++k)
    if (!reg[k].paper && reg[k].n == (int)n) return (int)k;
  return LWE_EINVAL;
}

int find_param_paper(uint32_t n) {
  std::lock_guard<std::mutex> g(g_reg_mu);
  auto& reg = registry();
  for (size_t k = 0; k < reg.size(); ++k)
    if (reg[k].paper && reg[k].n == (int)n) return (int)k;
  return LWE_EINVAL;
}

int register_param(uint32_t n, uint32_t logq, uint32_t B, uint32_t K, double sigma) {
  if (n % 8 != 0 || n < 8 || n > 32768) return LWE_EINVAL;
  if (logq < 3 || logq > 16 || B < 1 || B > 8 || B >= logq) return LWE_EINVAL;
  if (K < 1 || K > (uint32_t)MAX_K || !(sigma > 0)) return LWE_EINVAL;
  Params p;
  memset(&p, 0, sizeof(p));
  p.n = (int)n;
  p.logq = (int)logq;
  p.B = (int)B;
  p.K = (int)K;
  p.sigma = sigma;
  if (!build_cdf(p.K, p.sigma, p.T)) return LWE_EINVAL;
  finish_params(p);
  std::lock_guard<std::mutex> g(g_reg_mu);
  auto& reg = registry();
  for (size_t k = 0; k < reg.size(); ++k) {
    const Params& r = reg[k];
    if (!r.paper && r.n == p.n && r.logq == p.logq && r.B == p.B && r.K == p.K && r.sigma == p.sigma)
      return (int)k;
  }
  if (reg.size() >= 256) return LWE_ENOMEM;
  reg.push_back(p);
  return (int)reg.size() - 1;
}

// ------------------------------------------------------------------------------------
// AES S-box from its definition (FIPS-197 Sec. 5.1.1): multiplicative inverse in
// GF(2^8) followed by the affine map b ^ rotl(b,1) ^ rotl(b,2) ^ rotl(b,3) ^ rotl(b,4) ^ 0x63.
// The inverse uses exp/log tables over the generator 0x03.
// ------------------------------------------------------------------------------------
static void derive_sbox(uint8_t sb[256]) {
  uint8_t ex[255];
  int lg[256];
  uint8_t x = 1;
  for (int i = 0; i < 255; ++i) {
    ex[i] = x;
    lg[x] = i;
    x = (uint8_t)(x ^ gf_mul2(x));  // x * 3
  }
  for (int a = 0; a < 256; ++a) {
    uint8_t inv = a ? ex[(255 - lg[a]) % 255] : 0;
    uint8_t s = inv;
    for (int r = 1; r <= 4; ++r) s ^= (uint8_t)((inv << r) | (inv >> (8 - r)));
    sb[a] = (uint8_t)(s ^ 0x63);
  }
}

// T0[x] packs the MixColumns column (2S, S, S, 3S) of S = sbox(x) little-endian; the
// other three tables are byte rotations of it.
const uint32_t* aes_T0() {
  static uint32_t T0[256];
  static bool init = false;
  static std::mutex mu;
  std::lock_guard<std::mutex> g(mu);
  if (!init) {
    uint8_t sb[256];
    derive_sbox(sb);
    for (int x = 0; x < 256; ++x) {
      uint8_t s = sb[x], s2 = gf_mul2(s), s3 = (uint8_t)(s2 ^ s);
      T0[x] = (uint32_t)s2 | ((uint32_t)s << 8) | ((uint32_t)s << 16) | ((uint32_t)s3 << 24);
    }
    init = true;
  }
  return T0;
}

const uint8_t* aes_sbox() {
  static uint8_t sb[256];
  static bool init = false;
  static std::mutex mu;
  std::lock_guard<std::mutex> g(mu);
  if (!init) {
    const uint32_t* T0 = aes_T0();
    for (int x = 0; x < 256; ++x) sb[x] = (uint8_t)(T0[x] >> 8);
    init = true;
  }
  return sb;
}

}  // namespace lwe
