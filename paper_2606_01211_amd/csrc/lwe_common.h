// Definitions shared by the host side and the HIP kernels of liblwe_hip.
//
// Matrix form of the plain-LWE KEM (paper Sec. 2.1, Alg. 1-5) with nbar = mbar = 8 and
// q = 2^logq.  Everything here is integer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define LWE_HD __host__ __device__ __forceinline__

namespace lwe {

constexpr int NBAR = 8;
constexpr int MBAR = 8;
constexpr int MAX_K = 15;        // largest CDF support handled by the sampler
constexpr int SHA3_RATE = 136;   // SHA3-256 rate in bytes

constexpr int PB_BITS = 256;      // the paper's sets: one encryption per message bit
constexpr int DRBG_REQ_BLOCKS = 4096;  // AES blocks per CTR_DRBG Generate request (2^19 bits)

// One registered parameter set.  T[0..K] is the 16-bit CDF table of the error
// distribution; the sampler compares 15 keystream bits against T[0..K-1].
struct Params {
  int n, logq, B, K;
  double sigma;
  uint16_t T[MAX_K + 1];
  size_t pk_bytes, sk_bytes, ct_bytes, mu_bytes;
  int ldx;   // row stride in bytes of the int8 operand matrices (n rounded up to 64)
  // 0: matrix form (nbar = mbar = 8, q = 2^logq, CDF noise from AES-128-CTR).
  // 1: the paper's own sets (Table 1): nbar = 1, mbar = 256 (one encryption per message bit,
  //    one bit per coefficient), prime q, s binomial(eta), e / r / e1 Gaussian (CDF table),
  //    e2 uniform on [-ku, ku], all noise from the AES-256 CTR_DRBG.
  int paper;
  uint32_t q;       // modulus
  int nbar, mbar;   // rows of S^T (columns of B), rows of B' per instance
  int coef_bytes;   // bytes per serialised coefficient: 2, or 4 when q > 2^16
  int eta, ku;      // paper sets: binomial parameter of s, bound of e2
};

// ------------------------------------------------------------------------------------
// Keccak-f[1600] and the SHA3-256 sponge (FIPS 202).  Lane (x, y) is a[x + 5y].
// The round constants and rotation offsets are the published FIPS 202 values.
// ------------------------------------------------------------------------------------
LWE_HD uint64_t rotl64(uint64_t v, int r) { return (v << r) | (v >> (64 - r)); }

LWE_HD uint64_t keccak_rc(int round) {
  constexpr uint64_t rc[24] = {
      0x0000000000000001ull, 0x0000000000008082ull, 0x800000000000808Aull,
      0x8000000080008000ull, 0x000000000000808Bull, 0x0000000080000001ull,
      0x8000000080008081ull, 0x8000000000008009ull, 0x000000000000008Aull,
      0x0000000000000088ull, 0x0000000080008009ull, 0x000000008000000Aull,
      0x000000008000808Bull, 0x800000000000008Bull, 0x8000000000008089ull,
      0x8000000000008003ull, 0x8000000000008002ull, 0x8000000000000080ull,
      0x000000000000800Aull, 0x800000008000000Aull, 0x8000000080008081ull,
      0x8000000000008080ull, 0x0000000080000001ull, 0x8000000080008008ull};
  return rc[round];
}

// rho offset of lane (x, y), indexed x + 5y
LWE_HD int keccak_rho(int lane) {
  constexpr int r[25] = {0,  1,  62, 28, 27, 36, 44, 6,  55, 20, 3,  10, 43,
                         25, 39, 41, 45, 15, 21, 8,  18, 2,  61, 56, 14};
  return r[lane];
}

LWE_HD void keccak_f1600(uint64_t a[25]) {
#pragma unroll 1
  for (int round = 0; round < 24; ++round) {
    uint64_t c[5];
#pragma unroll
    for (int x = 0; x < 5; ++x) c[x] = a[x] ^ a[x + 5] ^ a[x + 10] ^ a[x + 15] ^ a[x + 20];
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      uint64_t d = c[(x + 4) % 5] ^ rotl64(c[(x + 1) % 5], 1);
#pragma unroll
      for (int y = 0; y < 5; ++y) a[x + 5 * y] ^= d;
    }
    // rho then pi: lane (x, y) moves to (y, 2x + 3y)
    uint64_t b[25];
#pragma unroll
    for (int x = 0; x < 5; ++x)
#pragma unroll
      for (int y = 0; y < 5; ++y) {
        const int r = keccak_rho(x + 5 * y);
        const uint64_t v = a[x + 5 * y];
        b[y + 5 * ((2 * x + 3 * y) % 5)] = r ? rotl64(v, r) : v;
      }
    // chi along rows
#pragma unroll
    for (int y = 0; y < 5; ++y)
#pragma unroll
      for (int x = 0; x < 5; ++x)
        a[x + 5 * y] = b[x + 5 * y] ^ (~b[(x + 1) % 5 + 5 * y] & b[(x + 2) % 5 + 5 * y]);
    a[0] ^= keccak_rc(round);
  }
}

// XOR `len` (< rate) bytes of a final partial block plus the SHA3 padding into the state.
LWE_HD void sha3_absorb_last(uint64_t a[25], const uint8_t* p, size_t len) {
  uint8_t blk[SHA3_RATE];
  for (int k = 0; k < SHA3_RATE; ++k) blk[k] = 0;
  for (size_t k = 0; k < len; ++k) blk[k] = p[k];
  blk[len] ^= 0x06;
  blk[SHA3_RATE - 1] ^= 0x80;
  for (int w = 0; w < SHA3_RATE / 8; ++w) {
    uint64_t v = 0;
    for (int k = 0; k < 8; ++k) v |= (uint64_t)blk[8 * w + k] << (8 * k);
    a[w] ^= v;
  }
  keccak_f1600(a);
}

LWE_HD void sha3_absorb_full(uint64_t a[25], const uint8_t* p) {
  for (int w = 0; w < SHA3_RATE / 8; ++w) {
    uint64_t v = 0;
    for (int k = 0; k < 8; ++k) v |= (uint64_t)p[8 * w + k] << (8 * k);
    a[w] ^= v;
  }
  keccak_f1600(a);
}

LWE_HD void sha3_squeeze32(const uint64_t a[25], uint8_t out[32]) {
  for (int k = 0; k < 32; ++k) out[k] = (uint8_t)(a[k / 8] >> (8 * (k % 8)));
}

// SHA3-256 of the concatenation of up to three byte strings.
LWE_HD void sha3_256_3(const uint8_t* p0, size_t l0, const uint8_t* p1, size_t l1,
                       const uint8_t* p2, size_t l2, uint8_t out[32]) {
  uint64_t a[25];
  for (int k = 0; k < 25; ++k) a[k] = 0;
  uint8_t blk[SHA3_RATE];
  size_t fill = 0;
  const uint8_t* parts[3] = {p0, p1, p2};
  size_t lens[3] = {l0, l1, l2};
  for (int part = 0; part < 3; ++part) {
    const uint8_t* p = parts[part];
    size_t l = lens[part];
    while (l > 0) {
      if (fill == 0 && l >= SHA3_RATE) {
        sha3_absorb_full(a, p);
        p += SHA3_RATE;
        l -= SHA3_RATE;
        continue;
      }
      size_t take = SHA3_RATE - fill < l ? SHA3_RATE - fill : l;
      for (size_t k = 0; k < take; ++k) blk[fill + k] = p[k];
      fill += take;
      p += take;
      l -= take;
      if (fill == SHA3_RATE) {
        sha3_absorb_full(a, blk);
        fill = 0;
      }
    }
  }
  sha3_absorb_last(a, blk, fill);
  sha3_squeeze32(a, out);
}

LWE_HD void sha3_256(const uint8_t* p, size_t len, uint8_t out[32]) {
  sha3_256_3(p, len, nullptr, 0, nullptr, 0, out);
}

// ------------------------------------------------------------------------------------
// AES-128.  The state and round keys are four little-endian 32-bit words per block
// (word c holds bytes 4c .. 4c+3, i.e. column c of the FIPS-197 state).
// ------------------------------------------------------------------------------------
LWE_HD uint8_t gf_mul2(uint8_t b) { return (uint8_t)((b << 1) ^ ((b >> 7) * 0x1b)); }

// Key expansion (FIPS-197 Sec. 5.2) using an S-box table `sb` (256 entries).
LWE_HD void aes128_key_schedule(const uint8_t key[16], const uint8_t* sb, uint32_t rk[44]) {
  for (int w = 0; w < 4; ++w)
    rk[w] = (uint32_t)key[4 * w] | ((uint32_t)key[4 * w + 1] << 8) |
            ((uint32_t)key[4 * w + 2] << 16) | ((uint32_t)key[4 * w + 3] << 24);
  uint8_t rcon = 1;
  for (int w = 4; w < 44; ++w) {
    uint32_t t = rk[w - 1];
    if ((w & 3) == 0) {
      // RotWord then SubWord, little-endian: bytes (b1, b2, b3, b0)
      t = (uint32_t)sb[(t >> 8) & 0xff] | ((uint32_t)sb[(t >> 16) & 0xff] << 8) |
          ((uint32_t)sb[(t >> 24) & 0xff] << 16) | ((uint32_t)sb[t & 0xff] << 24);
      t ^= rcon;
      rcon = gf_mul2(rcon);
    }
    rk[w] = rk[w - 4] ^ t;
  }
}

LWE_HD uint32_t bswap32(uint32_t v) {
  return (v >> 24) | ((v >> 8) & 0xff00u) | ((v << 8) & 0xff0000u) | (v << 24);
}

}  // namespace lwe
