/*
 * Plain CPU oracle, part 2: the paper's own parameterisation -- TEST INFRASTRUCTURE ONLY.
 *
 * The scheme exactly as the paper states it: every one of the 256 message bits is
 * encrypted on its own (Alg. 2 run once per bit, Sec. 2.3 and Sec. 3.2), so a ciphertext
 * is 256 pairs (u_r, v_r); the modulus is one of the primes of Table 1; the secret s comes
 * from the centred binomial distribution with eta = 3, the errors e, r, e1 from a discrete
 * Gaussian of Table 1's sigma, and e2 from the centred uniform distribution on [-k, k]
 * (Table 1); decryption thresholds at q/4 and 3q/4 (Alg. 3).  All noise is drawn from an
 * AES-256 CTR_DRBG (Sec. 3.3).  Plain loops, 64-bit accumulators, reduction mod q at the end.
 * Shares nothing with the GPU library; only tests, the smoke check and the benchmark's CPU
 * leg may call it.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "lwe_oracle.h"

/* Table 1: n, q, sigma (e, r, e1), k (e2), eta (s).  The CDF support K is derived. */
int orc_pb_params_for(int n, orc_pb_params* out) {
  static const struct {
    int n, q;
    double sigma;
    int k, eta;
  } reg[] = {
      {512, 3329, 2.3, 3, 3},    {1024, 12289, 2.3, 3, 3},  {2048, 12289, 2.3, 3, 3},
      {4096, 12289, 1.7, 3, 3},  {8192, 65537, 1.2, 2, 3},  {16384, 65537, 1.2, 2, 3},
      {32768, 65537, 1.0, 2, 3},
  };
  for (size_t r = 0; r < sizeof(reg) / sizeof(reg[0]); ++r)
    if (reg[r].n == n) {
      out->n = n;
      out->q = reg[r].q;
      out->sigma = reg[r].sigma;
      out->k = reg[r].k;
      out->eta = reg[r].eta;
      out->K = orc_pb_support(reg[r].sigma);
      return 0;
    }
  return -1;
}

/* The largest support [-K, K] (K <= 40) whose 15-bit CDF table stays strictly increasing,
 * i.e. every value of the support keeps a nonzero probability. */
int orc_pb_support(double sigma) {
  uint16_t T[64];
  int best = 0;
  for (int K = 1; K <= 40; ++K)
    if (orc_cdf_table(K, sigma, T) == 0) best = K;
  return best;
}

size_t orc_pb_coef_bytes(const orc_pb_params* p) { return p->q > 65536 ? 4 : 2; }
size_t orc_pb_pk_bytes(const orc_pb_params* p) { return 16 + (size_t)p->n * orc_pb_coef_bytes(p); }
size_t orc_pb_sk_bytes(const orc_pb_params* p) { return 2 * (size_t)p->n + orc_pb_pk_bytes(p) + 64; }
size_t orc_pb_ct_bytes(const orc_pb_params* p) {
  return (size_t)ORC_PB_BITS * ((size_t)p->n + 1) * orc_pb_coef_bytes(p);
}

/* ---- samplers of one 16-bit DRBG word ---- */
/* centred binomial: (sum of eta bits) - (sum of the next eta bits) */
int orc_pb_binomial(uint16_t w, int eta) {
  int a = 0, b = 0;
  for (int t = 0; t < eta; ++t) {
    a += (w >> t) & 1;
    b += (w >> (eta + t)) & 1;
  }
  return a - b;
}

/* centred uniform on [-k, k]: floor(w (2k + 1) / 2^16) - k */
int orc_pb_uniform(uint16_t w, int k) { return (int)(((uint32_t)w * (uint32_t)(2 * k + 1)) >> 16) - k; }

void orc_pb_noise(const orc_pb_params* p, const uint8_t key[16], uint32_t domain, int dist, size_t count,
                  int16_t* out) {
  uint16_t T[64];
  orc_cdf_table(p->K, p->sigma, T);
  uint16_t* w = (uint16_t*)malloc(sizeof(uint16_t) * (count ? count : 1));
  orc_drbg_words(key, domain, count, w);
  for (size_t i = 0; i < count; ++i) {
    int v;
    if (dist == ORC_PB_BINOMIAL)
      v = orc_pb_binomial(w[i], p->eta);
    else if (dist == ORC_PB_GAUSSIAN)
      v = orc_sample_word(w[i], T, p->K);
    else
      v = orc_pb_uniform(w[i], p->k);
    out[i] = (int16_t)v;
  }
  free(w);
}

/* A = sample(rho) (Alg. 1): A[i][j] = word(j n + i) mod q of the AES-128-CTR keystream of
 * seedA (domain 0), the same keystream and column-major order as the matrix-form sets. */
void orc_pb_expand_A_cols(const orc_pb_params* p, const uint8_t seedA[16], int col0, int ncols, uint32_t* out) {
  const size_t cnt = (size_t)ncols * p->n;
  uint16_t* w = (uint16_t*)malloc(sizeof(uint16_t) * (cnt ? cnt : 1));
  orc_ctr_words(seedA, 0, (uint64_t)col0 * p->n, cnt, w);
  for (size_t k = 0; k < cnt; ++k) out[k] = (uint32_t)w[k] % (uint32_t)p->q;
  free(w);
}

/* row-major copy of A: Arm[i n + j] = A[i][j] */
static uint32_t* pb_full_A(const orc_pb_params* p, const uint8_t seedA[16]) {
  const long n = p->n;
  uint32_t* cols = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n * n);
  orc_pb_expand_A_cols(p, seedA, 0, (int)n, cols);
  uint32_t* Arm = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n * n);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i)
    for (long j = 0; j < n; ++j) Arm[i * n + j] = cols[j * n + i];
  free(cols);
  return Arm;
}

static uint32_t mod_q(long long x, int q) {
  long long r = x % q;
  return (uint32_t)(r < 0 ? r + q : r);
}

/* KeyGen (Alg. 1): s <- chi_eta^n (domain 1), e <- Gaussian^n (domain 2), t = A s + e mod q */
void orc_pb_pke_keygen(const orc_pb_params* p, const uint8_t seedA[16], const uint8_t seedSK[16], int16_t* s,
                       uint32_t* t) {
  const long n = p->n;
  int16_t* e = (int16_t*)malloc(sizeof(int16_t) * n);
  orc_pb_noise(p, seedSK, 1, ORC_PB_BINOMIAL, (size_t)n, s);
  orc_pb_noise(p, seedSK, 2, ORC_PB_GAUSSIAN, (size_t)n, e);
  uint32_t* A = pb_full_A(p, seedA);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i) {
    long long acc = e[i];
    for (long j = 0; j < n; ++j) acc += (long long)A[i * n + j] * s[j];
    t[i] = mod_q(acc, p->q);
  }
  free(A);
  free(e);
}

/* bit r of the message, least significant bit of each byte first */
static int mu_bit(const uint8_t* mu, int r) { return (mu[r >> 3] >> (r & 7)) & 1; }

/* Encrypt (Alg. 2) once per message bit r: r_r <- Gaussian^n (row r of domain 1), e1_r <-
 * Gaussian^n (row r of domain 2), e2_r <- U_k (word r of domain 3);
 * u_r = A^T r_r + e1_r, v_r = t^T r_r + e2_r + bit_r * round(q/2), all mod q. */
void orc_pb_pke_encrypt(const orc_pb_params* p, const uint8_t seedA[16], const uint32_t* t, const uint8_t coins[16],
                        const uint8_t* mu, uint32_t* U, uint32_t* v) {
  const long n = p->n, R = ORC_PB_BITS;
  int16_t* Rm = (int16_t*)malloc(sizeof(int16_t) * R * n);
  int16_t* E1 = (int16_t*)malloc(sizeof(int16_t) * R * n);
  int16_t e2[ORC_PB_BITS];
  orc_pb_noise(p, coins, 1, ORC_PB_GAUSSIAN, (size_t)(R * n), Rm);
  orc_pb_noise(p, coins, 2, ORC_PB_GAUSSIAN, (size_t)(R * n), E1);
  orc_pb_noise(p, coins, 3, ORC_PB_UNIFORM, (size_t)R, e2);
  uint32_t* A = pb_full_A(p, seedA);
  const long long half = (p->q + 1) / 2;
#pragma omp parallel for schedule(static)
  for (long r = 0; r < R; ++r) {
    /* u_r[j] = e1_r[j] + sum_i A[i][j] r_r[i], accumulated row of A by row of A */
    long long* acc = (long long*)malloc(sizeof(long long) * n);
    for (long j = 0; j < n; ++j) acc[j] = E1[r * n + j];
    for (long i = 0; i < n; ++i) {
      const long long ri = Rm[r * n + i];
      for (long j = 0; j < n; ++j) acc[j] += (long long)A[i * n + j] * ri;
    }
    for (long j = 0; j < n; ++j) U[r * n + j] = mod_q(acc[j], p->q);
    free(acc);
    long long vacc = (long long)e2[r] + (mu_bit(mu, (int)r) ? half : 0);
    for (long i = 0; i < n; ++i) vacc += (long long)t[i] * Rm[r * n + i];
    v[r] = mod_q(vacc, p->q);
  }
  free(A);
  free(Rm);
  free(E1);
}

/* Alg. 3's rule for one value x in [0, q): 0 when x <= q/4 or x >= 3q/4 (as real numbers),
 * otherwise 1 (the value q/2). */
int orc_pb_decode(int q, uint32_t x) {
  const long long x4 = 4LL * x;
  return (x4 <= q || x4 >= 3LL * q) ? 0 : 1;
}

/* Decrypt (Alg. 3): mu_r = v_r - s^T u_r mod q, bit_r = decode(mu_r). */
void orc_pb_pke_decrypt(const orc_pb_params* p, const int16_t* s, const uint32_t* U, const uint32_t* v,
                        uint8_t* mu) {
  const long n = p->n;
  memset(mu, 0, ORC_PB_BITS / 8);
  for (long r = 0; r < ORC_PB_BITS; ++r) {
    long long acc = v[r];
    for (long j = 0; j < n; ++j) acc -= (long long)U[r * n + j] * s[j];
    if (orc_pb_decode(p->q, mod_q(acc, p->q))) mu[r >> 3] |= (uint8_t)(1u << (r & 7));
  }
}

/* Exact decryption noise of every bit, e^T r_r - s^T e1_r + e2_r (not reduced); returns
 * the largest magnitude.  Decryption of bit r is correct while it stays below q/4. */
long orc_pb_noise_max(const orc_pb_params* p, const uint8_t seedSK[16], const uint8_t coins[16]) {
  const long n = p->n, R = ORC_PB_BITS;
  int16_t* s = (int16_t*)malloc(sizeof(int16_t) * n);
  int16_t* e = (int16_t*)malloc(sizeof(int16_t) * n);
  int16_t* Rm = (int16_t*)malloc(sizeof(int16_t) * R * n);
  int16_t* E1 = (int16_t*)malloc(sizeof(int16_t) * R * n);
  int16_t e2[ORC_PB_BITS];
  orc_pb_noise(p, seedSK, 1, ORC_PB_BINOMIAL, (size_t)n, s);
  orc_pb_noise(p, seedSK, 2, ORC_PB_GAUSSIAN, (size_t)n, e);
  orc_pb_noise(p, coins, 1, ORC_PB_GAUSSIAN, (size_t)(R * n), Rm);
  orc_pb_noise(p, coins, 2, ORC_PB_GAUSSIAN, (size_t)(R * n), E1);
  orc_pb_noise(p, coins, 3, ORC_PB_UNIFORM, (size_t)R, e2);
  long mx = 0;
  for (long r = 0; r < R; ++r) {
    long acc = e2[r];
    for (long i = 0; i < n; ++i) acc += (long)e[i] * Rm[r * n + i] - (long)s[i] * E1[r * n + i];
    long a = acc < 0 ? -acc : acc;
    if (a > mx) mx = a;
  }
  free(s);
  free(e);
  free(Rm);
  free(E1);
  return mx;
}

/* ---- single entries straight from the definitions (sampled checks at large n) ---- */
uint32_t orc_pb_t_entry(const orc_pb_params* p, const uint8_t seedA[16], const uint8_t seedSK[16], long i) {
  const long n = p->n;
  int16_t* s = (int16_t*)malloc(sizeof(int16_t) * n);
  int16_t* e = (int16_t*)malloc(sizeof(int16_t) * n);
  orc_pb_noise(p, seedSK, 1, ORC_PB_BINOMIAL, (size_t)n, s);
  orc_pb_noise(p, seedSK, 2, ORC_PB_GAUSSIAN, (size_t)n, e);
  long long acc = e[i];
  for (long j = 0; j < n; ++j) {
    uint16_t w;
    orc_ctr_words(seedA, 0, (uint64_t)j * n + (uint64_t)i, 1, &w);
    acc += (long long)((uint32_t)w % (uint32_t)p->q) * s[j];
  }
  free(s);
  free(e);
  return mod_q(acc, p->q);
}

uint32_t orc_pb_u_entry(const orc_pb_params* p, const uint8_t seedA[16], const uint8_t coins[16], int r, long j) {
  const long n = p->n;
  const size_t upto = (size_t)(r + 1) * n;
  int16_t* Rm = (int16_t*)malloc(sizeof(int16_t) * upto);
  int16_t* E1 = (int16_t*)malloc(sizeof(int16_t) * upto);
  uint32_t* col = (uint32_t*)malloc(sizeof(uint32_t) * n);
  orc_pb_noise(p, coins, 1, ORC_PB_GAUSSIAN, upto, Rm);
  orc_pb_noise(p, coins, 2, ORC_PB_GAUSSIAN, upto, E1);
  orc_pb_expand_A_cols(p, seedA, (int)j, 1, col);
  long long acc = E1[(size_t)r * n + j];
  for (long i = 0; i < n; ++i) acc += (long long)col[i] * Rm[(size_t)r * n + i];
  free(Rm);
  free(E1);
  free(col);
  return mod_q(acc, p->q);
}

/* ---- KEM (Alg. 4, 5) over the per-bit PKE ----
 * pk = seedA || t (n coefficients); sk = s (n int16) || pk || H(pk) || z;
 * ct = u_0 .. u_255 (256 x n coefficients) || v_0 .. v_255; coefficients little endian,
 * 2 bytes when q < 2^16, else 4.  H, coins and K as in the matrix-form sets (32-byte m). */
static void put_coef(uint8_t* dst, const uint32_t* src, size_t count, size_t cb) {
  for (size_t k = 0; k < count; ++k)
    for (size_t b = 0; b < cb; ++b) dst[cb * k + b] = (uint8_t)(src[k] >> (8 * b));
}
static void get_coef(uint32_t* dst, const uint8_t* src, size_t count, size_t cb) {
  for (size_t k = 0; k < count; ++k) {
    uint32_t v = 0;
    for (size_t b = 0; b < cb; ++b) v |= (uint32_t)src[cb * k + b] << (8 * b);
    dst[k] = v;
  }
}

static void pb_fo(const uint8_t pkh[32], const uint8_t mu[32], uint8_t coins[16], uint8_t kprime[32]) {
  uint8_t buf[65], h[32];
  buf[0] = 0x01;
  memcpy(buf + 1, pkh, 32);
  memcpy(buf + 33, mu, 32);
  orc_sha3_256(buf, 65, h);
  memcpy(coins, h, 16);
  orc_sha3_256(buf + 1, 64, kprime);
}

void orc_pb_kem_keygen(const orc_pb_params* p, const uint8_t seedA[16], const uint8_t seedSK[16],
                       const uint8_t z[32], uint8_t* pk, uint8_t* sk) {
  const size_t n = (size_t)p->n, cb = orc_pb_coef_bytes(p), pkb = orc_pb_pk_bytes(p);
  int16_t* s = (int16_t*)malloc(sizeof(int16_t) * n);
  uint32_t* t = (uint32_t*)malloc(sizeof(uint32_t) * n);
  orc_pb_pke_keygen(p, seedA, seedSK, s, t);
  memcpy(pk, seedA, 16);
  put_coef(pk + 16, t, n, cb);
  for (size_t k = 0; k < n; ++k) {
    sk[2 * k] = (uint8_t)((uint16_t)s[k] & 0xff);
    sk[2 * k + 1] = (uint8_t)((uint16_t)s[k] >> 8);
  }
  memcpy(sk + 2 * n, pk, pkb);
  orc_sha3_256(pk, pkb, sk + 2 * n + pkb);
  memcpy(sk + 2 * n + pkb + 32, z, 32);
  free(s);
  free(t);
}

static void pb_encrypt_bytes(const orc_pb_params* p, const uint8_t* pk, const uint8_t coins[16], const uint8_t* mu,
                             uint8_t* ct) {
  const size_t n = (size_t)p->n, cb = orc_pb_coef_bytes(p);
  uint32_t* t = (uint32_t*)malloc(sizeof(uint32_t) * n);
  uint32_t* U = (uint32_t*)malloc(sizeof(uint32_t) * ORC_PB_BITS * n);
  uint32_t v[ORC_PB_BITS];
  get_coef(t, pk + 16, n, cb);
  orc_pb_pke_encrypt(p, pk, t, coins, mu, U, v);
  put_coef(ct, U, ORC_PB_BITS * n, cb);
  put_coef(ct + ORC_PB_BITS * n * cb, v, ORC_PB_BITS, cb);
  free(t);
  free(U);
}

void orc_pb_kem_encaps(const orc_pb_params* p, const uint8_t* pk, const uint8_t mu[32], uint8_t* ct,
                       uint8_t ss[32]) {
  uint8_t pkh[32], coins[16], kp[32], buf[64];
  orc_sha3_256(pk, orc_pb_pk_bytes(p), pkh);
  pb_fo(pkh, mu, coins, kp);
  pb_encrypt_bytes(p, pk, coins, mu, ct);
  memcpy(buf, kp, 32);
  orc_sha3_256(ct, orc_pb_ct_bytes(p), buf + 32);
  orc_sha3_256(buf, 64, ss);
}

int orc_pb_kem_decaps(const orc_pb_params* p, const uint8_t* sk, const uint8_t* ct, uint8_t ss[32]) {
  const size_t n = (size_t)p->n, cb = orc_pb_coef_bytes(p), pkb = orc_pb_pk_bytes(p), ctb = orc_pb_ct_bytes(p);
  const uint8_t* pk = sk + 2 * n;
  const uint8_t* pkh = pk + pkb;
  const uint8_t* z = pkh + 32;
  int16_t* s = (int16_t*)malloc(sizeof(int16_t) * n);
  uint32_t* U = (uint32_t*)malloc(sizeof(uint32_t) * ORC_PB_BITS * n);
  uint32_t v[ORC_PB_BITS];
  for (size_t k = 0; k < n; ++k) s[k] = (int16_t)(uint16_t)(sk[2 * k] | (sk[2 * k + 1] << 8));
  get_coef(U, ct, ORC_PB_BITS * n, cb);
  get_coef(v, ct + ORC_PB_BITS * n * cb, ORC_PB_BITS, cb);
  uint8_t mu[32], coins[16], kp[32], buf[64];
  orc_pb_pke_decrypt(p, s, U, v, mu);
  pb_fo(pkh, mu, coins, kp);
  uint8_t* ct2 = (uint8_t*)malloc(ctb);
  pb_encrypt_bytes(p, pk, coins, mu, ct2);
  uint8_t diff = 0;
  for (size_t k = 0; k < ctb; ++k) diff |= (uint8_t)(ct2[k] ^ ct[k]);
  uint8_t keep = (uint8_t)(((unsigned)diff - 1u) >> 8);
  for (int k = 0; k < 32; ++k) buf[k] = (uint8_t)((kp[k] & keep) | (z[k] & (uint8_t)~keep));
  orc_sha3_256(ct, ctb, buf + 32);
  orc_sha3_256(buf, 64, ss);
  free(s);
  free(U);
  free(ct2);
  return keep ? 1 : 0;
}
