/*
 * Plain CPU oracle for the LWE KEM hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Written for readability, not speed: byte-oriented textbook AES-128, a Keccak-f[1600]
 * whose constants are derived from the FIPS 202 definitions at run time, a scan-all
 * CDF sampler, and plain loops with 64-bit accumulators for every product.
 * Shares nothing with the GPU library.  Only tests, the smoke check and the CPU
 * baseline of the benchmark may call it.
 *
 * Where the paper leaves a choice open (PRF, layouts, hash, encodings) the functions
 * follow the readings listed in the design notes; each function names the passage of
 * the paper it implements.
 */
#include "lwe_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------------------ */
/* Parameter registry.  n, q and the support come from the workload definitions; sigma  */
/* follows the paper's Table 1 where that table leaves mass on the whole support,       */
/* otherwise sigma = K/4.3 (rounded to 0.1).                                            */
/* ------------------------------------------------------------------------------------ */
int orc_params_for(int n, orc_params* out) {
  static const orc_params reg[] = {
      {640, 15, 2, 12, 2.8},  {976, 16, 3, 10, 2.3},  {1344, 16, 4, 6, 1.4},
      {4096, 16, 4, 6, 1.4},  {8192, 16, 4, 6, 1.4},  {16384, 16, 3, 6, 1.4},
      {32768, 16, 3, 6, 1.4},
  };
  for (size_t k = 0; k < sizeof(reg) / sizeof(reg[0]); ++k)
    if (reg[k].n == n) {
      *out = reg[k];
      return 0;
    }
  return -1;
}

size_t orc_pk_bytes(const orc_params* p) { return 16 + (size_t)ORC_NBAR * p->n * 2; }
size_t orc_sk_bytes(const orc_params* p) {
  return (size_t)ORC_NBAR * p->n * 2 + orc_pk_bytes(p) + 32 + 32;
}
size_t orc_ct_bytes(const orc_params* p) {
  return (size_t)ORC_MBAR * p->n * 2 + (size_t)ORC_MBAR * ORC_NBAR * 2;
}
size_t orc_mu_bytes(const orc_params* p) { return (size_t)ORC_MBAR * ORC_NBAR * p->B / 8; }

/* ------------------------------------------------------------------------------------ */
/* AES-128, FIPS-197 Sec. 5: state is 4x4 bytes, s[r][c] = in[r + 4c].                  */
/* ------------------------------------------------------------------------------------ */
static const uint8_t SBOX[256] = {
    0x63, 0x7c, 0x77, 0x7b, 0xf2, 0x6b, 0x6f, 0xc5, 0x30, 0x01, 0x67, 0x2b, 0xfe, 0xd7, 0xab, 0x76,
    0xca, 0x82, 0xc9, 0x7d, 0xfa, 0x59, 0x47, 0xf0, 0xad, 0xd4, 0xa2, 0xaf, 0x9c, 0xa4, 0x72, 0xc0,
    0xb7, 0xfd, 0x93, 0x26, 0x36, 0x3f, 0xf7, 0xcc, 0x34, 0xa5, 0xe5, 0xf1, 0x71, 0xd8, 0x31, 0x15,
    0x04, 0xc7, 0x23, 0xc3, 0x18, 0x96, 0x05, 0x9a, 0x07, 0x12, 0x80, 0xe2, 0xeb, 0x27, 0xb2, 0x75,
    0x09, 0x83, 0x2c, 0x1a, 0x1b, 0x6e, 0x5a, 0xa0, 0x52, 0x3b, 0xd6, 0xb3, 0x29, 0xe3, 0x2f, 0x84,
    0x53, 0xd1, 0x00, 0xed, 0x20, 0xfc, 0xb1, 0x5b, 0x6a, 0xcb, 0xbe, 0x39, 0x4a, 0x4c, 0x58, 0xcf,
    0xd0, 0xef, 0xaa, 0xfb, 0x43, 0x4d, 0x33, 0x85, 0x45, 0xf9, 0x02, 0x7f, 0x50, 0x3c, 0x9f, 0xa8,
    0x51, 0xa3, 0x40, 0x8f, 0x92, 0x9d, 0x38, 0xf5, 0xbc, 0xb6, 0xda, 0x21, 0x10, 0xff, 0xf3, 0xd2,
    0xcd, 0x0c, 0x13, 0xec, 0x5f, 0x97, 0x44, 0x17, 0xc4, 0xa7, 0x7e, 0x3d, 0x64, 0x5d, 0x19, 0x73,
    0x60, 0x81, 0x4f, 0xdc, 0x22, 0x2a, 0x90, 0x88, 0x46, 0xee, 0xb8, 0x14, 0xde, 0x5e, 0x0b, 0xdb,
    0xe0, 0x32, 0x3a, 0x0a, 0x49, 0x06, 0x24, 0x5c, 0xc2, 0xd3, 0xac, 0x62, 0x91, 0x95, 0xe4, 0x79,
    0xe7, 0xc8, 0x37, 0x6d, 0x8d, 0xd5, 0x4e, 0xa9, 0x6c, 0x56, 0xf4, 0xea, 0x65, 0x7a, 0xae, 0x08,
    0xba, 0x78, 0x25, 0x2e, 0x1c, 0xa6, 0xb4, 0xc6, 0xe8, 0xdd, 0x74, 0x1f, 0x4b, 0xbd, 0x8b, 0x8a,
    0x70, 0x3e, 0xb5, 0x66, 0x48, 0x03, 0xf6, 0x0e, 0x61, 0x35, 0x57, 0xb9, 0x86, 0xc1, 0x1d, 0x9e,
    0xe1, 0xf8, 0x98, 0x11, 0x69, 0xd9, 0x8e, 0x94, 0x9b, 0x1e, 0x87, 0xe9, 0xce, 0x55, 0x28, 0xdf,
    0x8c, 0xa1, 0x89, 0x0d, 0xbf, 0xe6, 0x42, 0x68, 0x41, 0x99, 0x2d, 0x0f, 0xb0, 0x54, 0xbb, 0x16,
};

/* multiplication by x in GF(2^8) modulo x^8 + x^4 + x^3 + x + 1 (FIPS-197 Sec. 4.2.1) */
static uint8_t xtime(uint8_t b) { return (uint8_t)((b << 1) ^ ((b & 0x80) ? 0x1b : 0x00)); }

/* FIPS-197 Sec. 5.2, Nk = 4, Nr = 10: 44 words, stored as 176 bytes */
void orc_aes128_expand_key(const uint8_t key[16], uint8_t rk[176]) {
  memcpy(rk, key, 16);
  uint8_t rcon = 0x01;
  for (int i = 4; i < 44; ++i) {
    uint8_t t[4];
    memcpy(t, rk + 4 * (i - 1), 4);
    if (i % 4 == 0) {
      uint8_t r0 = t[0]; /* RotWord */
      t[0] = t[1];
      t[1] = t[2];
      t[2] = t[3];
      t[3] = r0;
      for (int b = 0; b < 4; ++b) t[b] = SBOX[t[b]]; /* SubWord */
      t[0] ^= rcon;
      rcon = xtime(rcon);
    }
    for (int b = 0; b < 4; ++b) rk[4 * i + b] = rk[4 * (i - 4) + b] ^ t[b];
  }
}

static void add_round_key(uint8_t s[16], const uint8_t* k) {
  for (int b = 0; b < 16; ++b) s[b] ^= k[b];
}
static void sub_bytes(uint8_t s[16]) {
  for (int b = 0; b < 16; ++b) s[b] = SBOX[s[b]];
}
/* row r of the state is cyclically shifted left by r positions */
static void shift_rows(uint8_t s[16]) {
  uint8_t t[16];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) t[r + 4 * c] = s[r + 4 * ((c + r) % 4)];
  memcpy(s, t, 16);
}
/* each column is multiplied by {03}x^3 + {01}x^2 + {01}x + {02} modulo x^4 + 1 */
static void mix_columns(uint8_t s[16]) {
  for (int c = 0; c < 4; ++c) {
    uint8_t* col = s + 4 * c;
    uint8_t a0 = col[0], a1 = col[1], a2 = col[2], a3 = col[3];
    col[0] = (uint8_t)(xtime(a0) ^ (xtime(a1) ^ a1) ^ a2 ^ a3);
    col[1] = (uint8_t)(a0 ^ xtime(a1) ^ (xtime(a2) ^ a2) ^ a3);
    col[2] = (uint8_t)(a0 ^ a1 ^ xtime(a2) ^ (xtime(a3) ^ a3));
    col[3] = (uint8_t)((xtime(a0) ^ a0) ^ a1 ^ a2 ^ xtime(a3));
  }
}

void orc_aes128_encrypt(const uint8_t rk[176], const uint8_t in[16], uint8_t out[16]) {
  uint8_t s[16];
  memcpy(s, in, 16);
  add_round_key(s, rk);
  for (int round = 1; round < 10; ++round) {
    sub_bytes(s);
    shift_rows(s);
    mix_columns(s);
    add_round_key(s, rk + 16 * round);
  }
  sub_bytes(s);
  shift_rows(s);
  add_round_key(s, rk + 160);
  memcpy(out, s, 16);
}

/* ------------------------------------------------------------------------------------ */
/* CTR mode (SP 800-38A Sec. 6.5, standard incrementing function over the whole block). */
/* The initial counter of domain d is the 128-bit big-endian integer d*2^96, so block b  */
/* is encrypted from d*2^96 + b.  This is the seed-expansion function sample(rho) of     */
/* Alg. 1 and the device-side noise source of Sec. 3.3, with one domain per matrix.    */
/* ------------------------------------------------------------------------------------ */
static void counter_block(uint32_t domain, uint64_t b, uint8_t ctr[16]) {
  /* big-endian 128-bit integer domain*2^96 + b (b < 2^64 here) */
  memset(ctr, 0, 16);
  ctr[0] = (uint8_t)(domain >> 24);
  ctr[1] = (uint8_t)(domain >> 16);
  ctr[2] = (uint8_t)(domain >> 8);
  ctr[3] = (uint8_t)domain;
  for (int k = 0; k < 8; ++k) ctr[15 - k] = (uint8_t)(b >> (8 * k));
}

void orc_ctr_blocks(const uint8_t key[16], uint32_t domain, uint64_t block0, size_t nblocks,
                    uint8_t* out) {
  uint8_t rk[176];
  orc_aes128_expand_key(key, rk);
#pragma omp parallel for schedule(static) if (nblocks > 4096)
  for (long k = 0; k < (long)nblocks; ++k) {
    uint8_t ctr[16];
    counter_block(domain, block0 + (uint64_t)k, ctr);
    orc_aes128_encrypt(rk, ctr, out + 16 * (size_t)k);
  }
}

void orc_ctr_words(const uint8_t key[16], uint32_t domain, uint64_t word0, size_t nwords,
                   uint16_t* out) {
  if (nwords == 0) return;
  uint64_t b0 = word0 / 8, b1 = (word0 + nwords - 1) / 8;
  size_t nb = (size_t)(b1 - b0 + 1);
  uint8_t* ks = (uint8_t*)malloc(16 * nb);
  orc_ctr_blocks(key, domain, b0, nb, ks);
  for (size_t k = 0; k < nwords; ++k) {
    uint64_t w = word0 + k;
    size_t off = (size_t)(w - 8 * b0) * 2;
    out[k] = (uint16_t)(ks[off] | (ks[off + 1] << 8));
  }
  free(ks);
}

/* ------------------------------------------------------------------------------------ */
/* SHA3-256 (FIPS 202).  Lane (x, y) holds bits 64(5y+x) .. of the state string, little */
/* endian.  Rotation offsets and round constants are generated from the definitions    */
/* (Sec. 3.2.2 and 3.2.5) rather than written out.                                      */
/* ------------------------------------------------------------------------------------ */
static uint64_t rotl64(uint64_t v, int r) {
  r &= 63;
  return r ? (v << r) | (v >> (64 - r)) : v;
}

/* rc(t) of FIPS 202 Algorithm 5: an LFSR over GF(2) with feedback taps 0, 4, 5, 6 */
static int keccak_rc_bit(int t) {
  if (t % 255 == 0) return 1;
  unsigned R = 1; /* R[0] = 1, R[1..7] = 0 */
  for (int i = 1; i <= t % 255; ++i) {
    R <<= 1; /* R = 0 || R */
    unsigned r8 = (R >> 8) & 1;
    R ^= r8 | (r8 << 4) | (r8 << 5) | (r8 << 6);
    R &= 0xff; /* Trunc_8 */
  }
  return (int)(R & 1);
}

static void keccak_f1600(uint64_t A[5][5]) {
  /* rho offsets (Algorithm 2) */
  int rho[5][5];
  memset(rho, 0, sizeof(rho));
  {
    int x = 1, y = 0;
    for (int t = 0; t < 24; ++t) {
      rho[x][y] = ((t + 1) * (t + 2) / 2) % 64;
      int nx = y, ny = (2 * x + 3 * y) % 5;
      x = nx;
      y = ny;
    }
  }
  for (int ir = 0; ir < 24; ++ir) {
    /* theta */
    uint64_t C[5], D[5];
    for (int x = 0; x < 5; ++x) C[x] = A[x][0] ^ A[x][1] ^ A[x][2] ^ A[x][3] ^ A[x][4];
    for (int x = 0; x < 5; ++x) D[x] = C[(x + 4) % 5] ^ rotl64(C[(x + 1) % 5], 1);
    for (int x = 0; x < 5; ++x)
      for (int y = 0; y < 5; ++y) A[x][y] ^= D[x];
    /* rho */
    for (int x = 0; x < 5; ++x)
      for (int y = 0; y < 5; ++y) A[x][y] = rotl64(A[x][y], rho[x][y]);
    /* pi: A'[x][y] = A[(x + 3y) mod 5][x] */
    uint64_t P[5][5];
    for (int x = 0; x < 5; ++x)
      for (int y = 0; y < 5; ++y) P[x][y] = A[(x + 3 * y) % 5][x];
    /* chi */
    for (int x = 0; x < 5; ++x)
      for (int y = 0; y < 5; ++y) A[x][y] = P[x][y] ^ ((~P[(x + 1) % 5][y]) & P[(x + 2) % 5][y]);
    /* iota (Algorithm 6) */
    uint64_t RC = 0;
    for (int j = 0; j <= 6; ++j)
      if (keccak_rc_bit(j + 7 * ir)) RC |= (uint64_t)1 << ((1 << j) - 1);
    A[0][0] ^= RC;
  }
}

void orc_sha3_256(const uint8_t* in, size_t len, uint8_t out[32]) {
  const size_t rate = 136; /* (1600 - 2*256) / 8 */
  uint64_t A[5][5];
  memset(A, 0, sizeof(A));
  /* padded message: M || 0x06 || 0x00 ... || 0x80 (the 01 suffix then pad10*1) */
  size_t nblk = len / rate + 1;
  uint8_t block[136];
  for (size_t b = 0; b < nblk; ++b) {
    size_t off = b * rate;
    for (size_t k = 0; k < rate; ++k) {
      size_t pos = off + k;
      block[k] = pos < len ? in[pos] : 0;
    }
    if (b == nblk - 1) {
      block[len - off] ^= 0x06;
      block[rate - 1] ^= 0x80;
    }
    for (int lane = 0; lane < 17; ++lane) {
      uint64_t v = 0;
      for (int k = 0; k < 8; ++k) v |= (uint64_t)block[8 * lane + k] << (8 * k);
      A[lane % 5][lane / 5] ^= v;
    }
    keccak_f1600(A);
  }
  for (int k = 0; k < 32; ++k) {
    int lane = k / 8;
    out[k] = (uint8_t)(A[lane % 5][lane / 5] >> (8 * (k % 8)));
  }
}

/* ------------------------------------------------------------------------------------ */
/* CDF table of a centred discrete Gaussian restricted to [-K, K].                      */
/* C(k) = P(|x| <= k) = (w(0) + 2 sum_{x=1..k} w(x)) / (w(0) + 2 sum_{x=1..K} w(x)),      */
/* w(x) = exp(-x^2 / (2 sigma^2)); T[k] = floor(2^15 C(k) + 1/2) - 1, T[K] = 2^15 - 1.    */
/* Sums are accumulated in increasing x, in IEEE double.                                */
/* ------------------------------------------------------------------------------------ */
int orc_cdf_table(int K, double sigma, uint16_t* T) {
  double partial[64];
  if (K < 1 || K > 63) return -1;
  double acc = 1.0; /* w(0) */
  partial[0] = acc;
  for (int x = 1; x <= K; ++x) {
    acc += 2.0 * exp(-(double)x * (double)x / (2.0 * sigma * sigma));
    partial[x] = acc;
  }
  for (int k = 0; k < K; ++k) {
    double c = partial[k] / partial[K];
    T[k] = (uint16_t)(floor(32768.0 * c + 0.5) - 1.0);
  }
  T[K] = 32767;
  for (int k = 1; k <= K; ++k)
    if (T[k] <= T[k - 1]) return -1;
  return 0;
}

/* One sample from one 16-bit keystream word: bit 0 is the sign, bits 1..15 are compared */
/* with every table entry (no early exit), giving |e|.                                  */
int orc_sample_word(uint16_t u, const uint16_t* T, int K) {
  int r = u >> 1, sgn = u & 1, e = 0;
  for (int k = 0; k < K; ++k) e += (r > T[k]) ? 1 : 0;
  return sgn ? -e : e;
}

void orc_sample_stream(const orc_params* p, const uint8_t key[16], uint32_t domain, uint64_t word0,
                       size_t count, int16_t* out) {
  uint16_t T[64];
  orc_cdf_table(p->K, p->sigma, T);
  uint16_t* w = (uint16_t*)malloc(sizeof(uint16_t) * (count ? count : 1));
  orc_ctr_words(key, domain, word0, count, w);
  for (size_t k = 0; k < count; ++k) out[k] = (int16_t)orc_sample_word(w[k], T, p->K);
  free(w);
}

/* ------------------------------------------------------------------------------------ */
/* A = sample(rho) (Alg. 1): A[i][j] = word(j*n + i) mod q of the domain-0 keystream   */
/* under seedA, i.e. the keystream fills A column by column.                            */
/* ------------------------------------------------------------------------------------ */
void orc_expand_A_cols(const orc_params* p, const uint8_t seedA[16], int col0, int ncols,
                       uint16_t* out) {
  const int n = p->n;
  const uint16_t mask = (uint16_t)((1u << p->logq) - 1u);
  orc_ctr_words(seedA, 0, (uint64_t)col0 * n, (size_t)ncols * n, out);
  for (size_t k = 0; k < (size_t)ncols * n; ++k) out[k] &= mask;
}

/* full A in row-major order: Arm[i*n + j] = A[i][j] */
static uint16_t* full_A_rowmajor(const orc_params* p, const uint8_t seedA[16]) {
  const int n = p->n;
  uint16_t* cols = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)n * n);
  orc_expand_A_cols(p, seedA, 0, n, cols);
  uint16_t* Arm = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)n * n);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i)
    for (long j = 0; j < n; ++j) Arm[i * (size_t)n + j] = cols[j * (size_t)n + i];
  free(cols);
  return Arm;
}

/* ------------------------------------------------------------------------------------ */
/* Encoding (generalises the 1-bit threshold of Alg. 3 to B bits per coefficient).      */
/* Coefficient c = 8r + col carries mu bits c*B .. c*B+B-1, least significant bit first */
/* within each byte; the value k is placed in the top B bits: enc = k * 2^(logq - B).   */
/* ------------------------------------------------------------------------------------ */
uint16_t orc_encode_coeff(const orc_params* p, const uint8_t* mu, int coeff) {
  unsigned k = 0;
  for (int t = 0; t < p->B; ++t) {
    int pos = coeff * p->B + t;
    unsigned bit = (mu[pos / 8] >> (pos % 8)) & 1u;
    k |= bit << t;
  }
  return (uint16_t)(k << (p->logq - p->B));
}

/* nearest multiple of 2^(logq-B), halves rounded up, wrapped mod q */
int orc_decode_value(const orc_params* p, uint16_t x) {
  unsigned q = 1u << p->logq;
  unsigned half = 1u << (p->logq - p->B - 1);
  return (int)(((x + half) % q) >> (p->logq - p->B));
}

/* ------------------------------------------------------------------------------------ */
/* PKE (Alg. 1-3) in matrix form.                                                       */
/* Keystream domains under seedSK: 1 -> S^T[c][j] = sample(c*n + j), 2 -> E^T[c][i].     */
/* Under coins: 1 -> S'[r][i] = sample(r*n + i), 2 -> E'[r][j], 3 -> E''[r][c] =         */
/* sample(8r + c).                                                                       */
/* ------------------------------------------------------------------------------------ */
void orc_pke_keygen(const orc_params* p, const uint8_t seedA[16], const uint8_t seedSK[16],
                    int16_t* St, uint16_t* Bt) {
  const int n = p->n;
  const long qmask = (1L << p->logq) - 1;
  int16_t* Et = (int16_t*)malloc(sizeof(int16_t) * ORC_NBAR * (size_t)n);
  orc_sample_stream(p, seedSK, 1, 0, (size_t)ORC_NBAR * n, St);
  orc_sample_stream(p, seedSK, 2, 0, (size_t)ORC_NBAR * n, Et);
  uint16_t* A = full_A_rowmajor(p, seedA);
  /* B^T[c][i] = sum_j S^T[c][j] A[i][j] + E^T[c][i]   (t = A s + e) */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i)
    for (int c = 0; c < ORC_NBAR; ++c) {
      long acc = 0;
      for (long j = 0; j < n; ++j) acc += (long)St[c * (size_t)n + j] * A[i * (size_t)n + j];
      acc += Et[c * (size_t)n + i];
      Bt[c * (size_t)n + i] = (uint16_t)(acc & qmask);
    }
  free(A);
  free(Et);
}

void orc_pke_encrypt(const orc_params* p, const uint8_t seedA[16], const uint16_t* Bt,
                     const uint8_t coins[16], const uint8_t* mu, uint16_t* Bp, uint16_t* V) {
  const int n = p->n;
  const long qmask = (1L << p->logq) - 1;
  int16_t* Sp = (int16_t*)malloc(sizeof(int16_t) * ORC_MBAR * (size_t)n);
  int16_t* Ep = (int16_t*)malloc(sizeof(int16_t) * ORC_MBAR * (size_t)n);
  int16_t Epp[ORC_MBAR * ORC_NBAR];
  orc_sample_stream(p, coins, 1, 0, (size_t)ORC_MBAR * n, Sp);
  orc_sample_stream(p, coins, 2, 0, (size_t)ORC_MBAR * n, Ep);
  orc_sample_stream(p, coins, 3, 0, ORC_MBAR * ORC_NBAR, Epp);
  uint16_t* A = full_A_rowmajor(p, seedA);
  /* B'[r][j] = sum_i S'[r][i] A[i][j] + E'[r][j]   (u = A^T r + e1) */
#pragma omp parallel for schedule(static)
  for (long j = 0; j < n; ++j)
    for (int r = 0; r < ORC_MBAR; ++r) {
      long acc = 0;
      for (long i = 0; i < n; ++i) acc += (long)Sp[r * (size_t)n + i] * A[i * (size_t)n + j];
      acc += Ep[r * (size_t)n + j];
      Bp[r * (size_t)n + j] = (uint16_t)(acc & qmask);
    }
  /* V[r][c] = sum_i S'[r][i] B[i][c] + E''[r][c] + enc(mu)   (v = t^T r + e2 + m) */
  for (int r = 0; r < ORC_MBAR; ++r)
    for (int c = 0; c < ORC_NBAR; ++c) {
      long acc = 0;
      for (long i = 0; i < n; ++i) acc += (long)Sp[r * (size_t)n + i] * Bt[c * (size_t)n + i];
      acc += Epp[r * ORC_NBAR + c];
      acc += orc_encode_coeff(p, mu, r * ORC_NBAR + c);
      V[r * ORC_NBAR + c] = (uint16_t)(acc & qmask);
    }
  free(A);
  free(Sp);
  free(Ep);
}

/* M[r][c] = V[r][c] - sum_j B'[r][j] S[j][c]   (mu = v - s^T u, Alg. 3) */
void orc_pke_decrypt_M(const orc_params* p, const int16_t* St, const uint16_t* Bp, const uint16_t* V,
                       uint16_t* M) {
  const int n = p->n;
  const long qmask = (1L << p->logq) - 1;
  for (int r = 0; r < ORC_MBAR; ++r)
    for (int c = 0; c < ORC_NBAR; ++c) {
      long acc = V[r * ORC_NBAR + c];
      for (long j = 0; j < n; ++j) acc -= (long)Bp[r * (size_t)n + j] * St[c * (size_t)n + j];
      M[r * ORC_NBAR + c] = (uint16_t)(acc & qmask);
    }
}

void orc_pke_decode(const orc_params* p, const uint16_t* M, uint8_t* mu_out) {
  memset(mu_out, 0, orc_mu_bytes(p));
  for (int coeff = 0; coeff < ORC_MBAR * ORC_NBAR; ++coeff) {
    unsigned k = (unsigned)orc_decode_value(p, M[coeff]);
    for (int t = 0; t < p->B; ++t) {
      int pos = coeff * p->B + t;
      mu_out[pos / 8] |= (uint8_t)(((k >> t) & 1u) << (pos % 8));
    }
  }
}

/* word w of the domain-0 keystream under an expanded key */
static uint16_t word_at(const uint8_t rk[176], uint64_t w) {
  uint8_t ctr[16], ks[16];
  counter_block(0, w / 8, ctr);
  orc_aes128_encrypt(rk, ctr, ks);
  return (uint16_t)(ks[2 * (w % 8)] | (ks[2 * (w % 8) + 1] << 8));
}

uint16_t orc_A_entry(const orc_params* p, const uint8_t seedA[16], long i, long j) {
  uint8_t rk[176];
  orc_aes128_expand_key(seedA, rk);
  return (uint16_t)(word_at(rk, (uint64_t)j * p->n + (uint64_t)i) & ((1u << p->logq) - 1u));
}

/* B^T[c][i] = sum_j S^T[c][j] A[i][j] + E^T[c][i] mod q, with row i of A computed alone */
uint16_t orc_Bt_entry(const orc_params* p, const uint8_t seedA[16], const uint8_t seedSK[16], int c,
                      long i) {
  const int n = p->n;
  uint8_t rk[176];
  orc_aes128_expand_key(seedA, rk);
  int16_t* St = (int16_t*)malloc(sizeof(int16_t) * (size_t)n);
  int16_t e;
  orc_sample_stream(p, seedSK, 1, (uint64_t)c * n, (size_t)n, St);
  orc_sample_stream(p, seedSK, 2, (uint64_t)c * n + (uint64_t)i, 1, &e);
  long acc = e;
  const unsigned mask = (1u << p->logq) - 1u;
  for (long j = 0; j < n; ++j) acc += (long)St[j] * (word_at(rk, (uint64_t)j * n + (uint64_t)i) & mask);
  free(St);
  return (uint16_t)(acc & (long)mask);
}

/* B'[r][j] = sum_i S'[r][i] A[i][j] + E'[r][j] mod q, with column j of A computed alone */
uint16_t orc_Bp_entry(const orc_params* p, const uint8_t seedA[16], const uint8_t coins[16], int r,
                      long j) {
  const int n = p->n;
  int16_t* Sp = (int16_t*)malloc(sizeof(int16_t) * (size_t)n);
  uint16_t* col = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)n);
  int16_t e;
  orc_sample_stream(p, coins, 1, (uint64_t)r * n, (size_t)n, Sp);
  orc_sample_stream(p, coins, 2, (uint64_t)r * n + (uint64_t)j, 1, &e);
  orc_expand_A_cols(p, seedA, (int)j, 1, col);
  long acc = e;
  for (long i = 0; i < n; ++i) acc += (long)Sp[i] * col[i];
  free(Sp);
  free(col);
  return (uint16_t)(acc & ((1L << p->logq) - 1));
}

void orc_pke_V(const orc_params* p, const uint16_t* Bt, const uint8_t coins[16], const uint8_t* mu,
               uint16_t* V) {
  const int n = p->n;
  const long qmask = (1L << p->logq) - 1;
  int16_t* Sp = (int16_t*)malloc(sizeof(int16_t) * ORC_MBAR * (size_t)n);
  int16_t Epp[ORC_MBAR * ORC_NBAR];
  orc_sample_stream(p, coins, 1, 0, (size_t)ORC_MBAR * n, Sp);
  orc_sample_stream(p, coins, 3, 0, ORC_MBAR * ORC_NBAR, Epp);
  for (int r = 0; r < ORC_MBAR; ++r)
    for (int c = 0; c < ORC_NBAR; ++c) {
      long acc = 0;
      for (long i = 0; i < n; ++i) acc += (long)Sp[r * (size_t)n + i] * Bt[c * (size_t)n + i];
      acc += Epp[r * ORC_NBAR + c];
      acc += orc_encode_coeff(p, mu, r * ORC_NBAR + c);
      V[r * ORC_NBAR + c] = (uint16_t)(acc & qmask);
    }
  free(Sp);
}

long orc_noise_max(const orc_params* p, const uint8_t seedSK[16], const uint8_t coins[16]) {
  const int n = p->n;
  size_t sz = (size_t)ORC_NBAR * n;
  int16_t* St = (int16_t*)malloc(sizeof(int16_t) * sz);
  int16_t* Et = (int16_t*)malloc(sizeof(int16_t) * sz);
  int16_t* Sp = (int16_t*)malloc(sizeof(int16_t) * sz);
  int16_t* Ep = (int16_t*)malloc(sizeof(int16_t) * sz);
  int16_t Epp[ORC_MBAR * ORC_NBAR];
  orc_sample_stream(p, seedSK, 1, 0, sz, St);
  orc_sample_stream(p, seedSK, 2, 0, sz, Et);
  orc_sample_stream(p, coins, 1, 0, sz, Sp);
  orc_sample_stream(p, coins, 2, 0, sz, Ep);
  orc_sample_stream(p, coins, 3, 0, ORC_MBAR * ORC_NBAR, Epp);
  /* N = S'E - E'S + E'' */
  long mx = 0;
  for (int r = 0; r < ORC_MBAR; ++r)
    for (int c = 0; c < ORC_NBAR; ++c) {
      long acc = Epp[r * ORC_NBAR + c];
      for (long i = 0; i < n; ++i) acc += (long)Sp[r * (size_t)n + i] * Et[c * (size_t)n + i];
      for (long j = 0; j < n; ++j) acc -= (long)Ep[r * (size_t)n + j] * St[c * (size_t)n + j];
      long a = acc < 0 ? -acc : acc;
      if (a > mx) mx = a;
    }
  free(St);
  free(Et);
  free(Sp);
  free(Ep);
  return mx;
}

/* ------------------------------------------------------------------------------------ */
/* KEM (Alg. 4 and 5).  H = SHA3-256.                                                    */
/*   pk = seedA || B^T (u16 LE);  sk = S^T (i16 LE) || pk || H(pk) || z;                 */
/*   ct = B' (u16 LE) || V (u16 LE).                                                     */
/*   coins = H(0x01 || H(pk) || mu)[0:16],  K' = H(H(pk) || mu),  K = H(K' || H(ct)).     */
/* Decaps re-encrypts with the decoded message and, in constant time, keeps K' when the */
/* ciphertexts agree and z otherwise (implicit rejection).                              */
/* ------------------------------------------------------------------------------------ */
static void put_u16(uint8_t* dst, const uint16_t* src, size_t count) {
  for (size_t k = 0; k < count; ++k) {
    dst[2 * k] = (uint8_t)(src[k] & 0xff);
    dst[2 * k + 1] = (uint8_t)(src[k] >> 8);
  }
}
static void get_u16(uint16_t* dst, const uint8_t* src, size_t count) {
  for (size_t k = 0; k < count; ++k) dst[k] = (uint16_t)(src[2 * k] | (src[2 * k + 1] << 8));
}

void orc_fo_coins(const orc_params* p, const uint8_t pkh[32], const uint8_t* mu, uint8_t coins[16],
                  uint8_t kprime[32]) {
  size_t mb = orc_mu_bytes(p);
  uint8_t buf[1 + 32 + 64];
  uint8_t h[32];
  buf[0] = 0x01;
  memcpy(buf + 1, pkh, 32);
  memcpy(buf + 33, mu, mb);
  orc_sha3_256(buf, 33 + mb, h);
  memcpy(coins, h, 16);
  orc_sha3_256(buf + 1, 32 + mb, kprime);
}

void orc_kem_keygen(const orc_params* p, const uint8_t seedA[16], const uint8_t seedSK[16],
                    const uint8_t z[32], uint8_t* pk, uint8_t* sk) {
  const int n = p->n;
  size_t sz = (size_t)ORC_NBAR * n;
  int16_t* St = (int16_t*)malloc(sizeof(int16_t) * sz);
  uint16_t* Bt = (uint16_t*)malloc(sizeof(uint16_t) * sz);
  orc_pke_keygen(p, seedA, seedSK, St, Bt);
  size_t pkb = orc_pk_bytes(p);
  memcpy(pk, seedA, 16);
  put_u16(pk + 16, Bt, sz);
  put_u16(sk, (const uint16_t*)St, sz); /* two's complement bytes of the int16 values */
  memcpy(sk + 2 * sz, pk, pkb);
  orc_sha3_256(pk, pkb, sk + 2 * sz + pkb);
  memcpy(sk + 2 * sz + pkb + 32, z, 32);
  free(St);
  free(Bt);
}

static void encrypt_to_bytes(const orc_params* p, const uint8_t* pk, const uint8_t coins[16],
                             const uint8_t* mu, uint8_t* ct) {
  const int n = p->n;
  size_t sz = (size_t)ORC_NBAR * n;
  uint16_t* Bt = (uint16_t*)malloc(sizeof(uint16_t) * sz);
  uint16_t* Bp = (uint16_t*)malloc(sizeof(uint16_t) * sz);
  uint16_t V[ORC_MBAR * ORC_NBAR];
  get_u16(Bt, pk + 16, sz);
  orc_pke_encrypt(p, pk, Bt, coins, mu, Bp, V);
  put_u16(ct, Bp, (size_t)ORC_MBAR * n);
  put_u16(ct + 2 * (size_t)ORC_MBAR * n, V, ORC_MBAR * ORC_NBAR);
  free(Bt);
  free(Bp);
}

void orc_kem_encaps(const orc_params* p, const uint8_t* pk, const uint8_t* mu, uint8_t* ct,
                    uint8_t ss[32]) {
  uint8_t pkh[32], coins[16], kp[32], hct[32], buf[64];
  orc_sha3_256(pk, orc_pk_bytes(p), pkh);
  orc_fo_coins(p, pkh, mu, coins, kp);
  encrypt_to_bytes(p, pk, coins, mu, ct);
  orc_sha3_256(ct, orc_ct_bytes(p), hct);
  memcpy(buf, kp, 32);
  memcpy(buf + 32, hct, 32);
  orc_sha3_256(buf, 64, ss);
}

int orc_kem_decaps(const orc_params* p, const uint8_t* sk, const uint8_t* ct, uint8_t ss[32]) {
  const int n = p->n;
  size_t sz = (size_t)ORC_NBAR * n;
  size_t pkb = orc_pk_bytes(p), ctb = orc_ct_bytes(p);
  const uint8_t* pk = sk + 2 * sz;
  const uint8_t* pkh = pk + pkb;
  const uint8_t* z = pkh + 32;
  int16_t* St = (int16_t*)malloc(sizeof(int16_t) * sz);
  uint16_t* Bp = (uint16_t*)malloc(sizeof(uint16_t) * sz);
  uint16_t V[ORC_MBAR * ORC_NBAR], M[ORC_MBAR * ORC_NBAR];
  get_u16((uint16_t*)St, sk, sz);
  get_u16(Bp, ct, (size_t)ORC_MBAR * n);
  get_u16(V, ct + 2 * (size_t)ORC_MBAR * n, ORC_MBAR * ORC_NBAR);
  uint8_t mu[64], coins[16], kp[32], hct[32], buf[64];
  orc_pke_decrypt_M(p, St, Bp, V, M);
  orc_pke_decode(p, M, mu);
  orc_fo_coins(p, pkh, mu, coins, kp);
  uint8_t* ct2 = (uint8_t*)malloc(ctb);
  encrypt_to_bytes(p, pk, coins, mu, ct2);
  /* constant-time comparison and selection */
  uint8_t diff = 0;
  for (size_t k = 0; k < ctb; ++k) diff |= (uint8_t)(ct2[k] ^ ct[k]);
  uint8_t keep = (uint8_t)(((unsigned)diff - 1u) >> 8); /* 0xff when equal, 0 otherwise */
  for (int k = 0; k < 32; ++k) buf[k] = (uint8_t)((kp[k] & keep) | (z[k] & (uint8_t)~keep));
  orc_sha3_256(ct, ctb, hct);
  memcpy(buf + 32, hct, 32);
  orc_sha3_256(buf, 64, ss);
  free(St);
  free(Bp);
  free(ct2);
  return keep ? 1 : 0;
}

/* ------------------------------------------------------------------------------------ */
/* AES-256, FIPS-197 Sec. 5 with Nk = 8, Nr = 14: 60 key-schedule words (240 bytes).    */
/* The paper's device noise source is an AES-256 DRBG (Sec. 3.3).                       */
/* ------------------------------------------------------------------------------------ */
void orc_aes256_expand_key(const uint8_t key[32], uint8_t rk[240]) {
  memcpy(rk, key, 32);
  uint8_t rcon = 0x01;
  for (int i = 8; i < 60; ++i) {
    uint8_t t[4];
    memcpy(t, rk + 4 * (i - 1), 4);
    if (i % 8 == 0) {
      uint8_t r0 = t[0]; /* RotWord */
      t[0] = t[1];
      t[1] = t[2];
      t[2] = t[3];
      t[3] = r0;
      for (int b = 0; b < 4; ++b) t[b] = SBOX[t[b]]; /* SubWord */
      t[0] ^= rcon;
      rcon = xtime(rcon);
    } else if (i % 8 == 4) {
      for (int b = 0; b < 4; ++b) t[b] = SBOX[t[b]]; /* SubWord only (Nk > 6) */
    }
    for (int b = 0; b < 4; ++b) rk[4 * i + b] = rk[4 * (i - 8) + b] ^ t[b];
  }
}

void orc_aes256_encrypt(const uint8_t rk[240], const uint8_t in[16], uint8_t out[16]) {
  uint8_t s[16];
  memcpy(s, in, 16);
  add_round_key(s, rk);
  for (int round = 1; round < 14; ++round) {
    sub_bytes(s);
    shift_rows(s);
    mix_columns(s);
    add_round_key(s, rk + 16 * round);
  }
  sub_bytes(s);
  shift_rows(s);
  add_round_key(s, rk + 224);
  memcpy(out, s, 16);
}

/* ------------------------------------------------------------------------------------ */
/* CTR_DRBG with AES-256 and no derivation function (SP 800-90A Rev. 1, Sec. 10.2.1):    */
/* seedlen = 384 bits, the counter is the whole 128-bit V (big endian), at most 2^19     */
/* bits per Generate request, each request followed by an Update with zero additional   */
/* input.  The paper draws its noise from such a generator (Sec. 3.3).                  */
/* ------------------------------------------------------------------------------------ */
static void v_increment(uint8_t V[16]) {
  for (int k = 15; k >= 0; --k)
    if (++V[k] != 0) break;
}

/* CTR_DRBG_Update (Sec. 10.2.1.2) */
static void drbg_update(const uint8_t provided[48], uint8_t key[32], uint8_t V[16]) {
  uint8_t rk[240], temp[48];
  orc_aes256_expand_key(key, rk);
  for (int b = 0; b < 3; ++b) {
    v_increment(V);
    orc_aes256_encrypt(rk, V, temp + 16 * b);
  }
  for (int k = 0; k < 48; ++k) temp[k] ^= provided[k];
  memcpy(key, temp, 32);
  memcpy(V, temp + 32, 16);
}

void orc_drbg_instantiate(const uint8_t entropy[48], uint8_t key[32], uint8_t V[16]) {
  /* no personalization string: seed_material = entropy_input; Key = 0, V = 0 (Sec. 10.2.1.3.1) */
  memset(key, 0, 32);
  memset(V, 0, 16);
  drbg_update(entropy, key, V);
}

void orc_drbg_generate(uint8_t key[32], uint8_t V[16], size_t nbytes, uint8_t* out) {
  /* Sec. 10.2.1.5.1 with no additional input; nbytes <= 2^16 (2^19 bits) */
  uint8_t rk[240], blk[16], zero[48];
  orc_aes256_expand_key(key, rk);
  for (size_t off = 0; off < nbytes; off += 16) {
    v_increment(V);
    orc_aes256_encrypt(rk, V, blk);
    size_t m = nbytes - off < 16 ? nbytes - off : 16;
    memcpy(out + off, blk, m);
  }
  memset(zero, 0, sizeof(zero));
  drbg_update(zero, key, V);
}

/* Noise stream of (key, domain): a DRBG instantiated from the 48-byte entropy input      */
/* key (16) || domain (4, little endian) || 28 zero bytes, read in requests of 2^16 bytes;*/
/* word w is bytes 2w, 2w + 1 of the output (little endian).  Writes words 0 .. nwords-1.*/
void orc_drbg_words(const uint8_t key16[16], uint32_t domain, size_t nwords, uint16_t* out) {
  uint8_t entropy[48], key[32], V[16];
  memset(entropy, 0, sizeof(entropy));
  memcpy(entropy, key16, 16);
  for (int k = 0; k < 4; ++k) entropy[16 + k] = (uint8_t)(domain >> (8 * k));
  orc_drbg_instantiate(entropy, key, V);
  const size_t REQ = 65536;
  uint8_t* buf = (uint8_t*)malloc(REQ);
  size_t done = 0;
  while (done < nwords) {
    size_t want = (nwords - done) * 2 < REQ ? (nwords - done) * 2 : REQ;
    /* every request is a full 2^16 bytes (the stream does not depend on how much is read) */
    orc_drbg_generate(key, V, REQ, buf);
    for (size_t k = 0; k < want / 2; ++k) out[done + k] = (uint16_t)(buf[2 * k] | (buf[2 * k + 1] << 8));
    done += want / 2;
  }
  free(buf);
}
