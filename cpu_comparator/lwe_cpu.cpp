// All-cores CPU implementation of the matrix-form LWE KEM (see lwe_cpu.h): the CPU side of
// the paper's GPU-versus-multithreaded-CPU comparison (Sec. 4.1), on this project's scheme.
#include "lwe_cpu.h"

#include <immintrin.h>
#include <math.h>
#include <omp.h>
#include <string.h>

#include <vector>

namespace {

constexpr int NB = 8;   // nbar = mbar
constexpr int CB = 16;  // columns per packed block of the product

// ------------------------------------------------------------------------------------
// AES-128 with AES-NI; CTR blocks of (domain, b) = the big-endian 128-bit integer
// domain * 2^96 + b.
// ------------------------------------------------------------------------------------
struct Aes128 {
  __m128i rk[11];
};

__m128i expand_step(__m128i key, __m128i assist) {
  assist = _mm_shuffle_epi32(assist, 0xff);
  key = _mm_xor_si128(key, _mm_slli_si128(key, 4));
  key = _mm_xor_si128(key, _mm_slli_si128(key, 4));
  key = _mm_xor_si128(key, _mm_slli_si128(key, 4));
  return _mm_xor_si128(key, assist);
}

void aes_setup(Aes128& a, const uint8_t key[16]) {
  a.rk[0] = _mm_loadu_si128((const __m128i*)key);
#define LWC_STEP(i, rc) a.rk[i] = expand_step(a.rk[i - 1], _mm_aeskeygenassist_si128(a.rk[i - 1], rc))
  LWC_STEP(1, 0x01);
  LWC_STEP(2, 0x02);
  LWC_STEP(3, 0x04);
  LWC_STEP(4, 0x08);
  LWC_STEP(5, 0x10);
  LWC_STEP(6, 0x20);
  LWC_STEP(7, 0x40);
  LWC_STEP(8, 0x80);
  LWC_STEP(9, 0x1b);
  LWC_STEP(10, 0x36);
#undef LWC_STEP
}

__m128i ctr_block(uint32_t domain, uint64_t b) {
  uint8_t c[16] = {0};
  c[0] = (uint8_t)(domain >> 24);
  c[1] = (uint8_t)(domain >> 16);
  c[2] = (uint8_t)(domain >> 8);
  c[3] = (uint8_t)domain;
  for (int k = 0; k < 8; ++k) c[15 - k] = (uint8_t)(b >> (8 * k));
  return _mm_loadu_si128((const __m128i*)c);
}

// nblocks keystream blocks from block b0 of (key, domain), eight in flight
void keystream(const Aes128& a, uint32_t domain, uint64_t b0, size_t nblocks, uint8_t* out) {
  size_t k = 0;
  for (; k + 8 <= nblocks; k += 8) {
    __m128i x[8];
    for (int j = 0; j < 8; ++j) x[j] = _mm_xor_si128(ctr_block(domain, b0 + k + j), a.rk[0]);
    for (int r = 1; r < 10; ++r)
      for (int j = 0; j < 8; ++j) x[j] = _mm_aesenc_si128(x[j], a.rk[r]);
    for (int j = 0; j < 8; ++j) _mm_storeu_si128((__m128i*)(out + 16 * (k + j)), _mm_aesenclast_si128(x[j], a.rk[10]));
  }
  for (; k < nblocks; ++k) {
    __m128i x = _mm_xor_si128(ctr_block(domain, b0 + k), a.rk[0]);
    for (int r = 1; r < 10; ++r) x = _mm_aesenc_si128(x, a.rk[r]);
    _mm_storeu_si128((__m128i*)(out + 16 * k), _mm_aesenclast_si128(x, a.rk[10]));
  }
}

// ------------------------------------------------------------------------------------
// SHA3-256 (FIPS 202): Keccak-f[1600] on 64-bit lanes, rate 136 bytes, suffix 01, pad10*1.
// ------------------------------------------------------------------------------------
const uint64_t RC[24] = {
    0x0000000000000001ull, 0x0000000000008082ull, 0x800000000000808aull, 0x8000000080008000ull,
    0x000000000000808bull, 0x0000000080000001ull, 0x8000000080008081ull, 0x8000000000008009ull,
    0x000000000000008aull, 0x0000000000000088ull, 0x0000000080008009ull, 0x000000008000000aull,
    0x000000008000808bull, 0x800000000000008bull, 0x8000000000008089ull, 0x8000000000008003ull,
    0x8000000000008002ull, 0x8000000000000080ull, 0x000000000000800aull, 0x800000008000000aull,
    0x8000000080008081ull, 0x8000000000008080ull, 0x0000000080000001ull, 0x8000000080008008ull};
// rotation offset of lane x + 5y
const int ROT[25] = {0, 1, 62, 28, 27, 36, 44, 6, 55, 20, 3, 10, 43, 25, 39, 41, 45, 15, 21, 8, 18, 2, 61, 56, 14};

inline uint64_t rol(uint64_t v, int r) { return r ? (v << r) | (v >> (64 - r)) : v; }

void keccak(uint64_t a[25]) {
  for (int round = 0; round < 24; ++round) {
    uint64_t c[5], b[25];
    for (int x = 0; x < 5; ++x) c[x] = a[x] ^ a[x + 5] ^ a[x + 10] ^ a[x + 15] ^ a[x + 20];
    for (int x = 0; x < 5; ++x) {
      const uint64_t d = c[(x + 4) % 5] ^ rol(c[(x + 1) % 5], 1);
      for (int y = 0; y < 5; ++y) a[x + 5 * y] ^= d;
    }
    for (int x = 0; x < 5; ++x)
      for (int y = 0; y < 5; ++y) b[y + 5 * ((2 * x + 3 * y) % 5)] = rol(a[x + 5 * y], ROT[x + 5 * y]);
    for (int y = 0; y < 5; ++y)
      for (int x = 0; x < 5; ++x) a[x + 5 * y] = b[x + 5 * y] ^ (~b[(x + 1) % 5 + 5 * y] & b[(x + 2) % 5 + 5 * y]);
    a[0] ^= RC[round];
  }
}

// SHA3-256 of the concatenation of two byte strings
void sha3(const uint8_t* p0, size_t l0, const uint8_t* p1, size_t l1, uint8_t out[32]) {
  uint64_t a[25] = {0};
  uint8_t blk[136];
  size_t fill = 0;
  auto absorb = [&](const uint8_t* p, size_t l) {
    while (l) {
      if (fill == 0 && l >= 136) {
        for (int w = 0; w < 17; ++w) {
          uint64_t v;
          memcpy(&v, p + 8 * w, 8);
          a[w] ^= v;
        }
        keccak(a);
        p += 136;
        l -= 136;
        continue;
      }
      const size_t take = 136 - fill < l ? 136 - fill : l;
      memcpy(blk + fill, p, take);
      fill += take;
      p += take;
      l -= take;
      if (fill == 136) {
        for (int w = 0; w < 17; ++w) {
          uint64_t v;
          memcpy(&v, blk + 8 * w, 8);
          a[w] ^= v;
        }
        keccak(a);
        fill = 0;
      }
    }
  };
  absorb(p0, l0);
  if (l1) absorb(p1, l1);
  memset(blk + fill, 0, 136 - fill);
  blk[fill] ^= 0x06;
  blk[135] ^= 0x80;
  for (int w = 0; w < 17; ++w) {
    uint64_t v;
    memcpy(&v, blk + 8 * w, 8);
    a[w] ^= v;
  }
  keccak(a);
  memcpy(out, a, 32);
}

// ------------------------------------------------------------------------------------
// CDF sampler: T[k] = floor(2^15 P(|x| <= k) + 1/2) - 1 (k < K), T[K] = 2^15 - 1; a word u
// gives |e| = #{k < K : (u >> 1) > T[k]} and the sign of bit 0.
// ------------------------------------------------------------------------------------
void cdf(const lwc_params* p, uint16_t T[16]) {
  double acc[16];
  double s = 1.0;
  acc[0] = s;
  for (int x = 1; x <= p->K; ++x) {
    s += 2.0 * exp(-(double)x * x / (2.0 * p->sigma * p->sigma));
    acc[x] = s;
  }
  for (int k = 0; k < p->K; ++k) T[k] = (uint16_t)(floor(32768.0 * (acc[k] / acc[p->K]) + 0.5) - 1.0);
  T[p->K] = 32767;
}

inline int16_t sample(uint16_t u, const uint16_t* T, int K) {
  const int r = u >> 1;
  int e = 0;
  for (int k = 0; k < K; ++k) e += r > T[k];
  return (int16_t)((u & 1) ? -e : e);
}

// count samples of stream (key, domain) starting at word 0
void sample_stream(const Aes128& a, uint32_t domain, size_t count, const uint16_t* T, int K, int16_t* out) {
  std::vector<uint8_t> ks((count + 7) / 8 * 16);
  keystream(a, domain, 0, (count + 7) / 8, ks.data());
  for (size_t w = 0; w < count; ++w) out[w] = sample((uint16_t)(ks[2 * w] | (ks[2 * w + 1] << 8)), T, K);
}

// ------------------------------------------------------------------------------------
// Products mod 2^32 (reduced mod q by the caller): C[r][j] = sum_k X[r][k] Y[k][j] with X
// int16 [rows][n] and Y packed per 16-column block as [k / 2][16 columns][2] int16, so one
// _mm256_madd_epi16 multiplies a broadcast pair (X[r][k], X[r][k+1]) with eight columns.
// ------------------------------------------------------------------------------------
struct Packed {
  int n, ncols, nblk;
  std::vector<int16_t, std::allocator<int16_t>> y;  // [nblk][n/2][CB][2]
  const int16_t* block(int b) const { return y.data() + (size_t)b * (n / 2) * CB * 2; }
};

// 4 rows x 16 columns over the whole contraction
inline void micro(const int16_t* const xs[4], const int16_t* yb, int n, int32_t out[4][CB]) {
  __m256i acc[8];
  for (int k = 0; k < 8; ++k) acc[k] = _mm256_setzero_si256();
  for (int ip = 0; ip < n / 2; ++ip) {
    const __m256i y0 = _mm256_loadu_si256((const __m256i*)(yb + (size_t)ip * 32));
    const __m256i y1 = _mm256_loadu_si256((const __m256i*)(yb + (size_t)ip * 32 + 16));
    for (int r = 0; r < 4; ++r) {
      int32_t pair;
      memcpy(&pair, xs[r] + 2 * ip, 4);
      const __m256i sv = _mm256_set1_epi32(pair);
      acc[2 * r] = _mm256_add_epi32(acc[2 * r], _mm256_madd_epi16(sv, y0));
      acc[2 * r + 1] = _mm256_add_epi32(acc[2 * r + 1], _mm256_madd_epi16(sv, y1));
    }
  }
  for (int r = 0; r < 4; ++r) {
    _mm256_storeu_si256((__m256i*)out[r], acc[2 * r]);
    _mm256_storeu_si256((__m256i*)(out[r] + 8), acc[2 * r + 1]);
  }
}

// Runs the product over every (4-row group, column block) and hands each 4 x 16 tile to
// `epi(row0, col0, tile)`; rows past `rows` are computed from a zero row and skipped.
template <class Epi>
void product(const int16_t* X, int rows, const Packed& P, Epi epi) {
  const int groups = (rows + 3) / 4;
  const std::vector<int16_t> zero(P.n, 0);
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
  for (int b = 0; b < P.nblk; ++b)
    for (int g = 0; g < groups; ++g) {
      const int16_t* xs[4];
      for (int r = 0; r < 4; ++r) {
        const int row = 4 * g + r;
        xs[r] = row < rows ? X + (size_t)row * P.n : zero.data();
      }
      int32_t tile[4][CB];
      micro(xs, P.block(b), P.n, tile);
      epi(4 * g, b * CB, tile);
    }
}

// A[i][j] = keystream word (j n + i) of seedA, domain 0, masked to logq bits: all n^2 words.
std::vector<uint16_t> expand_A(const lwc_params* p, const uint8_t seedA[16]) {
  const size_t n = (size_t)p->n, words = n * n, blocks = words / 8;
  std::vector<uint16_t> A(words);
  Aes128 a;
  aes_setup(a, seedA);
  const uint16_t mask = (uint16_t)((1u << p->logq) - 1u);
#pragma omp parallel for schedule(static)
  for (long c = 0; c < (long)((blocks + 1023) / 1024); ++c) {
    const size_t b0 = (size_t)c * 1024, nb = blocks - b0 < 1024 ? blocks - b0 : 1024;
    keystream(a, 0, b0, nb, (uint8_t*)(A.data() + 8 * b0));
    for (size_t w = 8 * b0; w < 8 * (b0 + nb); ++w) A[w] &= mask;
  }
  return A;
}

// Y for encryption: Y[k][j] = A[k][j] (= word j n + k) for j < n, B[k][j - n] = Bt[j - n][k] after.
Packed pack_encrypt(const lwc_params* p, const std::vector<uint16_t>& A, const uint16_t* Bt) {
  Packed P;
  P.n = p->n;
  P.ncols = p->n + NB;
  P.nblk = (P.ncols + CB - 1) / CB;
  P.y.assign((size_t)P.nblk * (P.n / 2) * CB * 2, 0);
  const size_t n = (size_t)p->n;
#pragma omp parallel for schedule(static)
  for (int b = 0; b < P.nblk; ++b) {
    int16_t* yb = P.y.data() + (size_t)b * (n / 2) * CB * 2;
    for (int c = 0; c < CB; ++c) {
      const size_t j = (size_t)b * CB + c;
      if (j >= (size_t)P.ncols) continue;
      const uint16_t* col = j < n ? A.data() + j * n : Bt + (j - n) * n;
      for (size_t k = 0; k < n; ++k) yb[((k >> 1) * CB + c) * 2 + (k & 1)] = (int16_t)col[k];
    }
  }
  return P;
}

// Y for key generation: Y[k][i] = A[i][k] (= word k n + i), contracting over A's column index.
Packed pack_keygen(const lwc_params* p, const std::vector<uint16_t>& A) {
  Packed P;
  P.n = p->n;
  P.ncols = p->n;
  P.nblk = (P.ncols + CB - 1) / CB;
  P.y.assign((size_t)P.nblk * (P.n / 2) * CB * 2, 0);
  const size_t n = (size_t)p->n;
#pragma omp parallel for schedule(static)
  for (int b = 0; b < P.nblk; ++b) {
    int16_t* yb = P.y.data() + (size_t)b * (n / 2) * CB * 2;
    for (size_t k = 0; k < n; ++k)
      for (int c = 0; c < CB; ++c) {
        const size_t i = (size_t)b * CB + c;
        if (i < n) yb[((k >> 1) * CB + c) * 2 + (k & 1)] = (int16_t)A[k * n + i];
      }
  }
  return P;
}

inline void put16(uint8_t* d, uint16_t v) {
  d[0] = (uint8_t)v;
  d[1] = (uint8_t)(v >> 8);
}
inline uint16_t get16(const uint8_t* s) { return (uint16_t)(s[0] | (s[1] << 8)); }

uint32_t encode(const lwc_params* p, const uint8_t* mu, int coeff) {
  uint32_t k = 0;
  for (int t = 0; t < p->B; ++t) {
    const int pos = coeff * p->B + t;
    k |= (uint32_t)((mu[pos >> 3] >> (pos & 7)) & 1) << t;
  }
  return k << (p->logq - p->B);
}

// Encrypt count messages (coins[count][16]) under pk; writes ct records, or with cmp set
// flags[i] = 1 where the result differs from the received record.
void encrypt(const lwc_params* p, size_t count, const uint8_t* pk, const uint8_t* coins, const uint8_t* mu,
             size_t mb, uint8_t* ct, const uint8_t* cmp, uint8_t* flags) {
  const size_t n = (size_t)p->n, rows = count * NB, ctb = lwc_ct_bytes(p);
  const uint32_t mask = (1u << p->logq) - 1u;
  uint16_t T[16];
  cdf(p, T);
  std::vector<int16_t> S(rows * n), E(rows * n), E2(count * 64);
#pragma omp parallel for schedule(dynamic, 4)
  for (long i = 0; i < (long)count; ++i) {
    Aes128 a;
    aes_setup(a, coins + 16 * i);
    sample_stream(a, 1, NB * n, T, p->K, S.data() + (size_t)i * NB * n);
    sample_stream(a, 2, NB * n, T, p->K, E.data() + (size_t)i * NB * n);
    sample_stream(a, 3, 64, T, p->K, E2.data() + (size_t)i * 64);
  }
  std::vector<uint16_t> Bt(NB * n);
  for (size_t k = 0; k < NB * n; ++k) Bt[k] = get16(pk + 16 + 2 * k);
  const std::vector<uint16_t> A = expand_A(p, pk);
  const Packed P = pack_encrypt(p, A, Bt.data());
  product(S.data(), (int)rows, P, [&](int row0, int col0, int32_t tile[4][CB]) {
    for (int r = 0; r < 4; ++r) {
      const size_t row = (size_t)row0 + r;
      if (row >= rows) break;
      const size_t inst = row / NB, rr = row % NB;
      uint8_t diff = 0;
      for (int c = 0; c < CB; ++c) {
        const size_t j = (size_t)col0 + c;
        if (j >= n + NB) break;
        uint32_t v;
        size_t off;
        if (j < n) {
          v = ((uint32_t)tile[r][c] + (uint32_t)(int32_t)E[row * n + j]) & mask;
          off = 2 * (rr * n + j);
        } else {
          const size_t cc = j - n;
          v = ((uint32_t)tile[r][c] + (uint32_t)(int32_t)E2[inst * 64 + rr * NB + cc] +
               encode(p, mu + inst * mb, (int)(rr * NB + cc))) & mask;
          off = 2 * (NB * n + rr * NB + cc);
        }
        if (cmp)
          diff |= (uint8_t)(get16(cmp + inst * ctb + off) != (uint16_t)v);
        else
          put16(ct + inst * ctb + off, (uint16_t)v);
      }
      if (diff) __atomic_store_n(flags + inst, (uint8_t)1, __ATOMIC_RELAXED);
    }
  });
}

}  // namespace

extern "C" {

int lwc_threads(void) { return omp_get_max_threads(); }
size_t lwc_pk_bytes(const lwc_params* p) { return 16 + (size_t)NB * p->n * 2; }
size_t lwc_sk_bytes(const lwc_params* p) { return (size_t)NB * p->n * 2 + lwc_pk_bytes(p) + 64; }
size_t lwc_ct_bytes(const lwc_params* p) { return (size_t)NB * p->n * 2 + NB * NB * 2; }
size_t lwc_mu_bytes(const lwc_params* p) { return (size_t)NB * NB * p->B / 8; }

int lwc_keygen_batch(const lwc_params* p, size_t count, const uint8_t* seedA, const uint8_t* seedSK,
                     const uint8_t* z, uint8_t* pk, uint8_t* sk) {
  const size_t n = (size_t)p->n, pkb = lwc_pk_bytes(p), skb = lwc_sk_bytes(p);
  const uint32_t mask = (1u << p->logq) - 1u;
  uint16_t T[16];
  cdf(p, T);
  for (size_t i = 0; i < count; ++i) {
    std::vector<int16_t> St(NB * n), Et(NB * n);
    Aes128 a;
    aes_setup(a, seedSK + 16 * i);
    sample_stream(a, 1, NB * n, T, p->K, St.data());
    sample_stream(a, 2, NB * n, T, p->K, Et.data());
    const std::vector<uint16_t> A = expand_A(p, seedA + 16 * i);
    const Packed P = pack_keygen(p, A);
    uint8_t* rec = pk + i * pkb;
    memcpy(rec, seedA + 16 * i, 16);
    // B^T[c][col] = sum_k S^T[c][k] A[col][k] + E^T[c][col]
    product(St.data(), NB, P, [&](int row0, int col0, int32_t tile[4][CB]) {
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < CB; ++c) {
          const size_t row = (size_t)row0 + r, col = (size_t)col0 + c;
          if (row >= (size_t)NB || col >= n) continue;
          put16(rec + 16 + 2 * (row * n + col), (uint16_t)(((uint32_t)tile[r][c] + (uint32_t)(int32_t)Et[row * n + col]) & mask));
        }
    });
    uint8_t* s = sk + i * skb;
    for (size_t k = 0; k < NB * n; ++k) put16(s + 2 * k, (uint16_t)St[k]);
    memcpy(s + 2 * NB * n, rec, pkb);
    sha3(rec, pkb, nullptr, 0, s + 2 * NB * n + pkb);
    memcpy(s + 2 * NB * n + pkb + 32, z + 32 * i, 32);
  }
  return 0;
}

int lwc_encaps_batch(const lwc_params* p, size_t count, const uint8_t* pk, const uint8_t* mu, uint8_t* ct,
                     uint8_t* ss) {
  const size_t mb = lwc_mu_bytes(p), ctb = lwc_ct_bytes(p);
  uint8_t pkh[32];
  sha3(pk, lwc_pk_bytes(p), nullptr, 0, pkh);
  std::vector<uint8_t> coins(count * 16), kp(count * 32);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < (long)count; ++i) {
    uint8_t pre[33], h[32];
    pre[0] = 1;
    memcpy(pre + 1, pkh, 32);
    sha3(pre, 33, mu + i * mb, mb, h);
    memcpy(coins.data() + 16 * i, h, 16);
    sha3(pkh, 32, mu + i * mb, mb, kp.data() + 32 * i);
  }
  encrypt(p, count, pk, coins.data(), mu, mb, ct, nullptr, nullptr);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < (long)count; ++i) {
    uint8_t h[32];
    sha3(ct + i * ctb, ctb, nullptr, 0, h);
    sha3(kp.data() + 32 * i, 32, h, 32, ss + 32 * i);
  }
  return 0;
}

int lwc_decaps_batch(const lwc_params* p, size_t count, const uint8_t* sk, const uint8_t* ct, uint8_t* ss) {
  const size_t n = (size_t)p->n, mb = lwc_mu_bytes(p), ctb = lwc_ct_bytes(p), pkb = lwc_pk_bytes(p);
  const uint8_t* pk = sk + 2 * NB * n;
  const uint8_t* pkh = pk + pkb;
  const uint8_t* z = pkh + 32;
  const uint32_t mask = (1u << p->logq) - 1u;
  std::vector<int16_t> St(NB * n);
  for (size_t k = 0; k < NB * n; ++k) St[k] = (int16_t)get16(sk + 2 * k);
  std::vector<uint8_t> mu(count * mb), coins(count * 16), kp(count * 32), flags(count, 0);
  // mu' = decode(V - B' S), coins' and K'' per instance
#pragma omp parallel for schedule(static)
  for (long i = 0; i < (long)count; ++i) {
    const uint8_t* rec = ct + i * ctb;
    uint8_t* m = mu.data() + i * mb;
    memset(m, 0, mb);
    for (int r = 0; r < NB; ++r)
      for (int c = 0; c < NB; ++c) {
        uint32_t acc = get16(rec + 2 * (NB * n + r * NB + c));
        for (size_t j = 0; j < n; ++j) acc -= (uint32_t)get16(rec + 2 * (r * n + j)) * (uint32_t)(int32_t)St[c * n + j];
        const uint32_t M = acc & mask;
        const int sh = p->logq - p->B;
        const uint32_t k = ((M + (1u << (sh - 1))) & mask) >> sh;
        for (int t = 0; t < p->B; ++t) {
          const int pos = (r * NB + c) * p->B + t;
          m[pos >> 3] |= (uint8_t)(((k >> t) & 1) << (pos & 7));
        }
      }
    uint8_t pre[33], h[32];
    pre[0] = 1;
    memcpy(pre + 1, pkh, 32);
    sha3(pre, 33, m, mb, h);
    memcpy(coins.data() + 16 * i, h, 16);
    sha3(pkh, 32, m, mb, kp.data() + 32 * i);
  }
  encrypt(p, count, pk, coins.data(), mu.data(), mb, nullptr, ct, flags.data());
#pragma omp parallel for schedule(static)
  for (long i = 0; i < (long)count; ++i) {
    uint8_t pre[64];
    const uint8_t keep = (uint8_t)(flags[i] ? 0x00 : 0xff);
    for (int k = 0; k < 32; ++k) pre[k] = (uint8_t)((kp[32 * i + k] & keep) | (z[k] & (uint8_t)~keep));
    sha3(ct + i * ctb, ctb, nullptr, 0, pre + 32);
    sha3(pre, 64, nullptr, 0, ss + 32 * i);
  }
  return 0;
}

}  // extern "C"
