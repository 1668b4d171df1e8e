// HIP kernels (gfx950) of the plain-LWE KEM hot path.
//
//  * AES-128-CTR with T-tables in LDS: the seed expansion sample(rho) of Alg. 1 that yields
//    the public matrix A, and the device-side noise source of Sec. 3.3.  A is regenerated
//    tile by tile inside the products (Sec. 3.5) and never written to HBM (an unfused
//    variant, kept for comparison, expands it once per call and reads it back).
//  * CDF-table sampling of the secrets and errors (Alg. 1-2).
//  * The mod-2^16 products B^T = S^T A^T + E^T, B' = S' A + E', V = S' B + E'' + enc(mu)
//    (Alg. 1-2) and M = V - B' S (Alg. 3) on int8 MFMA: each 16-bit operand is split into two
//    signed 8-bit limbs x = lo + 256 hi (mod 2^16), both limbs are multiplied against the
//    small int8 matrix with int32 accumulation, and lo + 256 hi is reduced mod 2^logq.
//  * SHA3-256 sponges for the Fujisaki-Okamoto transform (Alg. 4-5).
#include <type_traits>

#include "lwe_internal.h"

namespace lwe {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned short v2u16 __attribute__((ext_vector_type(2)));

// ======================================================================================
// AES-128 with T-tables in LDS.  T[0..255] = T0, T[256..] = T0 rotated by 8, 16, 24.
// ======================================================================================
__device__ __forceinline__ uint32_t rotl32(uint32_t v, int r) { return (v << r) | (v >> (32 - r)); }

__device__ __forceinline__ void load_tables(uint32_t* T, const uint32_t* __restrict__ T0) {
  for (int i = threadIdx.x; i < 256; i += blockDim.x) {
    const uint32_t v = T0[i];
    T[i] = v;
    T[256 + i] = rotl32(v, 8);
    T[512 + i] = rotl32(v, 16);
    T[768 + i] = rotl32(v, 24);
  }
}

// three-input XOR in one v_bitop3 (truth table 0x96)
__device__ __forceinline__ uint32_t x3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Byte address of T-table entry (byte BYTE of x): one SDWA shift selects the byte and
// scales it by four, where the plain form takes an extract and a shift-add.
template <int BYTE>
__device__ __forceinline__ uint32_t tab_addr(uint32_t x) {
  uint32_t r;
  if constexpr (BYTE == 0)
    asm("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
        : "=v"(r) : "v"(x));
  else if constexpr (BYTE == 1)
    asm("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
        : "=v"(r) : "v"(x));
  else if constexpr (BYTE == 2)
    asm("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2"
        : "=v"(r) : "v"(x));
  else
    asm("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3"
        : "=v"(r) : "v"(x));
  return r;
}

// Entry of table TAB (0..3, the byte rotations of T0) at byte address `addr`; the table
// offset folds into the LDS instruction's immediate.
template <int TAB>
__device__ __forceinline__ uint32_t tab(const uint32_t* __restrict__ T, uint32_t addr) {
  return *(const uint32_t*)((const char*)T + addr + 1024 * TAB);
}

// Encrypts the CTR counter block of domain `dom` (as its little-endian word) and block
// index b: the 128-bit big-endian integer dom * 2^96 + b, with round keys rk[0..43]
// (FIPS-197 key expansion) and the T-tables in LDS.  Per round and column: four table
// lookups (one shifted-byte address each) folded with the round key by two 3-input XORs.
// o[] receives the keystream block as four little-endian words.
template <class RK>
__device__ __forceinline__ void aes_ctr_block(const uint32_t* __restrict__ T, const RK& rk,
                                              uint32_t dom_le, uint64_t b, uint32_t o[4]) {
  uint32_t s0 = dom_le ^ rk[0];
  uint32_t s1 = rk[1];
  uint32_t s2 = bswap32((uint32_t)(b >> 32)) ^ rk[2];
  uint32_t s3 = bswap32((uint32_t)b) ^ rk[3];
#pragma unroll
  for (int r = 1; r < 10; ++r) {
    const uint32_t t0 = x3(x3(tab<0>(T, tab_addr<0>(s0)), tab<1>(T, tab_addr<1>(s1)), tab<2>(T, tab_addr<2>(s2))),
                           tab<3>(T, tab_addr<3>(s3)), rk[4 * r]);
    const uint32_t t1 = x3(x3(tab<0>(T, tab_addr<0>(s1)), tab<1>(T, tab_addr<1>(s2)), tab<2>(T, tab_addr<2>(s3))),
                           tab<3>(T, tab_addr<3>(s0)), rk[4 * r + 1]);
    const uint32_t t2 = x3(x3(tab<0>(T, tab_addr<0>(s2)), tab<1>(T, tab_addr<1>(s3)), tab<2>(T, tab_addr<2>(s0))),
                           tab<3>(T, tab_addr<3>(s1)), rk[4 * r + 2]);
    const uint32_t t3 = x3(x3(tab<0>(T, tab_addr<0>(s3)), tab<1>(T, tab_addr<1>(s0)), tab<2>(T, tab_addr<2>(s1))),
                           tab<3>(T, tab_addr<3>(s2)), rk[4 * r + 3]);
    s0 = t0;
    s1 = t1;
    s2 = t2;
    s3 = t3;
  }
  // Final round (no MixColumns): the S-box value of x sits in byte 0 of T2[x], byte 1 of
  // T3[x], byte 2 of T0[x] and byte 3 of T1[x].
  o[0] = ((tab<2>(T, tab_addr<0>(s0)) & 0xffu) | (tab<3>(T, tab_addr<1>(s1)) & 0xff00u) |
          (tab<0>(T, tab_addr<2>(s2)) & 0xff0000u) | (tab<1>(T, tab_addr<3>(s3)) & 0xff000000u)) ^
         rk[40];
  o[1] = ((tab<2>(T, tab_addr<0>(s1)) & 0xffu) | (tab<3>(T, tab_addr<1>(s2)) & 0xff00u) |
          (tab<0>(T, tab_addr<2>(s3)) & 0xff0000u) | (tab<1>(T, tab_addr<3>(s0)) & 0xff000000u)) ^
         rk[41];
  o[2] = ((tab<2>(T, tab_addr<0>(s2)) & 0xffu) | (tab<3>(T, tab_addr<1>(s3)) & 0xff00u) |
          (tab<0>(T, tab_addr<2>(s0)) & 0xff0000u) | (tab<1>(T, tab_addr<3>(s1)) & 0xff000000u)) ^
         rk[42];
  o[3] = ((tab<2>(T, tab_addr<0>(s3)) & 0xffu) | (tab<3>(T, tab_addr<1>(s0)) & 0xff00u) |
          (tab<0>(T, tab_addr<2>(s1)) & 0xff0000u) | (tab<1>(T, tab_addr<3>(s2)) & 0xff000000u)) ^
         rk[43];
}

// Round keys are read once into registers before the kernel stores anything, so they stay
// in scalar registers instead of being re-loaded (as possibly clobbered memory) per block.
struct RoundKeys {
  uint32_t w[44];
  __device__ __forceinline__ uint32_t operator[](int i) const { return w[i]; }
};
__device__ __forceinline__ RoundKeys load_rk(const uint32_t* __restrict__ rk) {
  RoundKeys r;
#pragma unroll
  for (int i = 0; i < 44; ++i) r.w[i] = rk[i];
  return r;
}

// ======================================================================================
// AES with lane-replicated T-tables (conflict-free LDS lookups).  32 copies of T0 and of T2
// (T2 = T0 rotated by 16): word e*64 + c holds T0[e] and word e*64 + 32 + c holds T2[e], for
// copy c = lane & 31, so the 32 lanes of a half-wave always read 32 different banks.  The
// byte address of a lookup, state byte * 256 + copy offset, is one v_perm_b32.  T1 and T3
// are T0 and T2 rotated by 8, so each column XORs its T1 and T3 terms first and rotates once:
//   t_j = T0[s_j.b0] ^ T2[s_j+2.b2] ^ rotl8(T0[s_j+1.b1] ^ T2[s_j+3.b3] ^ rotr8(rk)).
// 64 KB of LDS.
// ======================================================================================
constexpr int TR_WORDS = 256 * 64;

__device__ __forceinline__ void load_tables_rep(uint32_t* TR, const uint32_t* __restrict__ T0) {
  for (int i = threadIdx.x; i < TR_WORDS; i += blockDim.x) {
    const uint32_t v = T0[i >> 6];
    TR[i] = (i & 32) ? rotl32(v, 16) : v;
  }
}

// Entry of the replicated table for byte BYTE of x; `off` = copy offset (+128 for T2).
template <int BYTE>
__device__ __forceinline__ uint32_t rep_look(const uint32_t* __restrict__ TR, uint32_t x, uint32_t off) {
  // byte 1 of the address <- byte BYTE of x, byte 0 <- byte 0 of off, bytes 2, 3 <- 0
  const uint32_t addr = __builtin_amdgcn_perm(x, off, 0x0c0c0000u | ((4u + BYTE) << 8));
  return *(const uint32_t*)((const char*)TR + addr);
}

// One CTR keystream block (same definition as aes_ctr_block).  rkr[r] = rotr8 of round key
// word 4 + r (rounds 1-9), so that the round key folds into the rotated half.
template <class RK>
__device__ __forceinline__ void aes_ctr_block_rep(const uint32_t* __restrict__ TR, uint32_t off0,
                                                  uint32_t off2, const RK& rk, const uint32_t* rkr,
                                                  uint32_t dom_le, uint64_t b, uint32_t o[4]) {
  uint32_t s[4];
  s[0] = dom_le ^ rk[0];
  s[1] = rk[1];
  s[2] = bswap32((uint32_t)(b >> 32)) ^ rk[2];
  s[3] = bswap32((uint32_t)b) ^ rk[3];
#pragma unroll
  for (int r = 1; r < 10; ++r) {
    uint32_t t[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t a0 = rep_look<0>(TR, s[j], off0);
      const uint32_t a1 = rep_look<1>(TR, s[(j + 1) & 3], off0);
      const uint32_t a2 = rep_look<2>(TR, s[(j + 2) & 3], off2);
      const uint32_t a3 = rep_look<3>(TR, s[(j + 3) & 3], off2);
      t[j] = x3(a0, a2, rotl32(x3(a1, a3, rkr[4 * (r - 1) + j]), 8));
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = t[j];
  }
  // Final round: S(x) is byte 2 of T0[x].
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t a0 = rep_look<0>(TR, s[j], off0);
    const uint32_t a1 = rep_look<1>(TR, s[(j + 1) & 3], off0);
    const uint32_t a2 = rep_look<2>(TR, s[(j + 2) & 3], off0);
    const uint32_t a3 = rep_look<3>(TR, s[(j + 3) & 3], off0);
    const uint32_t lo = __builtin_amdgcn_perm(a1, a0, 0x0c0c0602u);  // S(a0), S(a1) in bytes 0, 1
    const uint32_t hi = __builtin_amdgcn_perm(a3, a2, 0x06020c0cu);  // S(a2), S(a3) in bytes 2, 3
    o[j] = x3(lo, hi, rk[40 + j]);
  }
}

// Counter blocks whose domain word and high counter word (zero: block indices below 2^32) are
// the same for a whole wave differ only in state word 3 after the initial round-key XOR, so 12
// of round 1's 16 lookups are the same for every block.  aes_round1_fixed_rep computes them once
// (per wave and key), folded the way each column needs them:
//   column 0: fx[0] ^ rotl8(fx[1] ^ T2[s3.b3]),  column 1: fx[2] ^ T2[s3.b2],
//   column 2: fx[3] ^ rotl8(fx[4] ^ T0[s3.b1]),  column 3: fx[5] ^ T0[s3.b0];
// aes_ctr_block_rep_fixed then runs one block from them (same result as aes_ctr_block_rep).
template <class RK>
__device__ __forceinline__ void aes_round1_fixed_rep(const uint32_t* __restrict__ TR, uint32_t off0, uint32_t off2,
                                                     const RK& rk, const uint32_t* rkr, uint32_t dom_le,
                                                     uint32_t fx[6]) {
  const uint32_t s0 = dom_le ^ rk[0], s1 = rk[1], s2 = rk[2];
  fx[0] = rep_look<0>(TR, s0, off0) ^ rep_look<2>(TR, s2, off2);
  fx[1] = rep_look<1>(TR, s1, off0) ^ rkr[0];
  fx[2] = rep_look<0>(TR, s1, off0) ^ rotl32(x3(rep_look<1>(TR, s2, off0), rep_look<3>(TR, s0, off2), rkr[1]), 8);
  fx[3] = rep_look<0>(TR, s2, off0) ^ rep_look<2>(TR, s0, off2);
  fx[4] = rep_look<3>(TR, s1, off2) ^ rkr[2];
  fx[5] = rep_look<2>(TR, s1, off2) ^ rotl32(x3(rep_look<1>(TR, s0, off0), rep_look<3>(TR, s2, off2), rkr[3]), 8);
}

template <class RK>
__device__ __forceinline__ void aes_ctr_block_rep_fixed(const uint32_t* __restrict__ TR, uint32_t off0,
                                                        uint32_t off2, const RK& rk, const uint32_t* rkr,
                                                        const uint32_t fx[6], uint32_t b_lo, uint32_t o[4]) {
  const uint32_t s3 = bswap32(b_lo) ^ rk[3];
  uint32_t s[4];
  s[0] = fx[0] ^ rotl32(fx[1] ^ rep_look<3>(TR, s3, off2), 8);
  s[1] = fx[2] ^ rep_look<2>(TR, s3, off2);
  s[2] = fx[3] ^ rotl32(fx[4] ^ rep_look<1>(TR, s3, off0), 8);
  s[3] = fx[5] ^ rep_look<0>(TR, s3, off0);
#pragma unroll
  for (int r = 2; r < 10; ++r) {
    uint32_t t[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t a0 = rep_look<0>(TR, s[j], off0);
      const uint32_t a1 = rep_look<1>(TR, s[(j + 1) & 3], off0);
      const uint32_t a2 = rep_look<2>(TR, s[(j + 2) & 3], off2);
      const uint32_t a3 = rep_look<3>(TR, s[(j + 3) & 3], off2);
      t[j] = x3(a0, a2, rotl32(x3(a1, a3, rkr[4 * (r - 1) + j]), 8));
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = t[j];
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t a0 = rep_look<0>(TR, s[j], off0);
    const uint32_t a1 = rep_look<1>(TR, s[(j + 1) & 3], off0);
    const uint32_t a2 = rep_look<2>(TR, s[(j + 2) & 3], off0);
    const uint32_t a3 = rep_look<3>(TR, s[(j + 3) & 3], off0);
    const uint32_t lo = __builtin_amdgcn_perm(a1, a0, 0x0c0c0602u);
    const uint32_t hi = __builtin_amdgcn_perm(a3, a2, 0x06020c0cu);
    o[j] = x3(lo, hi, rk[40 + j]);
  }
}

// ======================================================================================
// Limb split: a 16-bit value x (already reduced mod q) equals lo + 256 hi (mod 2^16) with
// lo = sext8(x & 0xff) and hi = sext8(((x + 0x80) >> 8) & 0xff).  The int8 byte of lo is the
// low byte of x itself.
// ======================================================================================
__device__ __forceinline__ uint32_t pk_add_u16(uint32_t a, uint32_t b) {
  v2u16 va = __builtin_bit_cast(v2u16, a), vb = __builtin_bit_cast(v2u16, b);
  return __builtin_bit_cast(uint32_t, va + vb);
}

// two words holding four uint16 values -> four lo bytes and four hi bytes
__device__ __forceinline__ void limbs4(uint32_t a, uint32_t b, uint32_t& lo, uint32_t& hi) {
  lo = __builtin_amdgcn_perm(b, a, 0x06040200u);
  const uint32_t a2 = pk_add_u16(a, 0x00800080u), b2 = pk_add_u16(b, 0x00800080u);
  hi = __builtin_amdgcn_perm(b2, a2, 0x07050301u);
}

// |e| = #{k < K : (u >> 1) > T[k]}, sign from bit 0.  KT > 0: support fixed at compile time;
// KT == 0: K is a (uniform) run-time value.  Every entry is compared: no early exit.
template <int KT>
__device__ __forceinline__ uint32_t sample_one_t(uint32_t u, const uint16_t* T, int K) {
  const uint32_t r = u >> 1;
  int e = 0;
  if constexpr (KT > 0) {
#pragma unroll
    for (int k = 0; k < KT; ++k) e += (r > (uint32_t)T[k]) ? 1 : 0;
  } else {
    for (int k = 0; k < K; ++k) e += (r > (uint32_t)T[k]) ? 1 : 0;
  }
  return (uint32_t)(uint8_t)(int8_t)((u & 1) ? -e : e);
}

__device__ __forceinline__ uint32_t sample_one(uint32_t u, const uint16_t* T, int K) {
  return sample_one_t<0>(u, T, K);
}

// Two samples at once from one keystream word pair w = u0 | u1 << 16, in packed 16-bit
// arithmetic: r > T[k] exactly when T[k] - r (both < 2^15) has bit 15 set.  T2[k] holds T[k]
// in both halves.  Returns the two signed samples as int16 halves (two's complement).
template <int KT>
__device__ __forceinline__ uint32_t sample_pair(uint32_t w, const uint32_t* T2, int K) {
  const v2u16 u = __builtin_bit_cast(v2u16, w);
  const v2u16 r = u >> (v2u16){1, 1};
  v2u16 e = {0, 0};
  if constexpr (KT > 0) {
#pragma unroll
    for (int k = 0; k < KT; ++k) e += (__builtin_bit_cast(v2u16, T2[k]) - r) >> (v2u16){15, 15};
  } else {
    for (int k = 0; k < K; ++k) e += (__builtin_bit_cast(v2u16, T2[k]) - r) >> (v2u16){15, 15};
  }
  const v2u16 m = (v2u16){0, 0} - (u & (v2u16){1, 1});  // 0xffff where the sign bit is set
  return __builtin_bit_cast(uint32_t, (v2u16)((e ^ m) - m));
}

// ======================================================================================
// Small utility kernels
// ======================================================================================
__global__ void k_fill_u32(uint32_t* p, size_t count, uint32_t v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

// Copies a row-major [rows][n] int8 matrix into the layout the products read: row-major with
// row stride ldx, or MFMA fragment order (frag_offset); columns n .. ldx-1 become zero.  One
// thread per destination byte of the `rows` rows.
__global__ void k_pack_x(const int8_t* __restrict__ src, int rows, int n, int ldx, int frag,
                         int8_t* __restrict__ dst) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)rows * ldx) return;
  const int row = (int)(t / ldx), k = (int)(t - (size_t)row * ldx);
  const int8_t v = k < n ? src[(size_t)row * n + k] : (int8_t)0;
  dst[frag ? frag_offset(row, k, ldx >> 6) : (size_t)row * ldx + k] = v;
}

// FIPS-197 key expansion, one key per thread; the S-box comes from byte 1 of T0.
__global__ void k_expand_keys(const uint8_t* __restrict__ keys, size_t key_stride, int count,
                              const uint32_t* __restrict__ T0, uint32_t* __restrict__ rk_out) {
  __shared__ uint8_t sb[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) sb[i] = (uint8_t)(T0[i] >> 8);
  __syncthreads();
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  uint8_t key[16];
  for (int b = 0; b < 16; ++b) key[b] = keys[(size_t)k * key_stride + b];
  uint32_t rk[44];
  aes128_key_schedule(key, sb, rk);
  for (int w = 0; w < 44; ++w) rk_out[(size_t)k * 44 + w] = rk[w];
}

__global__ void k_keystream(const uint32_t* __restrict__ rk, const uint32_t* __restrict__ T0,
                            uint32_t dom_le, uint64_t block0, size_t nblocks, uint8_t* out) {
  __shared__ uint32_t T[1024];
  load_tables(T, T0);
  __syncthreads();
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nblocks) return;
  const RoundKeys rkv = load_rk(rk);
  uint32_t o[4];
  aes_ctr_block(T, rkv, dom_le, block0 + t, o);
  uint4 v = make_uint4(o[0], o[1], o[2], o[3]);
  *(uint4*)(out + 16 * t) = v;
}

// A[i][j] = keystream word (j n + i) of domain 0 under seedA, masked to logq bits: AES block
// b holds column b / (n/8), rows 8 (b mod n/8) .. +7, so block b lands at out + 8 (b - b0).
// Persistent waves over units of 64 * EXPAND_ILP consecutive blocks, replicated tables.
constexpr int EXPAND_ILP = 4, EXPAND_WAVES = 8;
__global__ void __launch_bounds__(64 * EXPAND_WAVES) k_expand_A(uint32_t qmask2, const uint32_t* __restrict__ rk,
                                                               const uint32_t* __restrict__ T0, uint64_t b0,
                                                               size_t nblocks, uint16_t* out) {
  __shared__ uint32_t TR[TR_WORDS];
  load_tables_rep(TR, T0);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint32_t off0 = (uint32_t)(lane & 31) << 2, off2 = off0 + 128;
  const RoundKeys rkv = load_rk(rk);
  uint32_t rkr[36];
#pragma unroll
  for (int i = 0; i < 36; ++i) rkr[i] = rotl32(rkv[4 + i], 24);
  const size_t per_unit = 64 * EXPAND_ILP;
  const size_t n_units = (nblocks + per_unit - 1) / per_unit;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const size_t nwaves = (size_t)gridDim.x * EXPAND_WAVES;
  for (size_t u = (size_t)blockIdx.x * EXPAND_WAVES + wave; u < n_units; u += nwaves) {
    uint32_t o[EXPAND_ILP][4];
#pragma unroll
    for (int j = 0; j < EXPAND_ILP; ++j) {
      const size_t t = u * per_unit + j * 64 + lane;
      aes_ctr_block_rep(TR, off0, off2, rkv, rkr, 0u, b0 + (t < nblocks ? t : nblocks - 1), o[j]);
    }
#pragma unroll
    for (int j = 0; j < EXPAND_ILP; ++j) {
      const size_t t = u * per_unit + j * 64 + lane;
      if (t < nblocks)
        *(uint4*)(out + 8 * t) = make_uint4(o[j][0] & qmask2, o[j][1] & qmask2, o[j][2] & qmask2, o[j][3] & qmask2);
    }
  }
}

struct SampTable {
  uint16_t T[MAX_K + 1];
};

__global__ void k_sample_stream(SampTable st, int K, const uint32_t* __restrict__ rk,
                                const uint32_t* __restrict__ T0, uint32_t dom_le, uint64_t word0,
                                size_t count, int16_t* out) {
  __shared__ uint32_t T[1024];
  load_tables(T, T0);
  __syncthreads();
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const uint64_t w = word0 + t;
  const RoundKeys rkv = load_rk(rk);
  uint32_t o[4];
  aes_ctr_block(T, rkv, dom_le, w / 8, o);
  const uint32_t u = (o[(w % 8) >> 1] >> (16 * (w & 1))) & 0xffffu;
  out[t] = (int16_t)(int8_t)(uint8_t)sample_one(u, st.T, K);
}

// ======================================================================================
// Sampling of the secrets and errors of one KeyGen (S^T, E^T) or Encrypt (S', E', E'') per
// instance.  Keystream domains: 1 -> segment 0, 2 -> segment 1, 3 -> segment 2.  Every AES
// block gives 8 consecutive samples of one matrix row.
// ======================================================================================
// compute units of the current device (set by init_kernels; sizes persistent grids)
static int g_num_cus = 256;

constexpr int SAMPLE_ILP = 4;   // AES blocks per lane per unit
constexpr int SAMPLE_WAVES = 8; // waves per workgroup

// Samples and stores the eight values of AES block lb of segment seg of instance inst.
// Segments 0 and 1 are 8 x n matrices filled row by row, n/8 blocks per row: row = lb / nb
// is taken as mulhi(2 lb, magic) with magic = floor(2^32 / (2 nb)) + 1, exact because
// 2 lb < 2^16 and 2 nb <= 8192.  Row-major offsets reduce to 8 lb from the instance's base.
template <int KT>
__device__ __forceinline__ void sample_store(const SampleArgs& a, int inst, int seg, uint32_t lb,
                                             uint32_t nb, uint32_t magic, const uint32_t o[4]) {
  uint32_t h[4];  // samples 2k, 2k+1 as int16 halves
#pragma unroll
  for (int q = 0; q < 4; ++q) h[q] = sample_pair<KT>(o[q], a.T2, a.K);
  const uint32_t p0 = __builtin_amdgcn_perm(h[1], h[0], 0x06040200u);  // low bytes = int8 samples
  const uint32_t p1 = __builtin_amdgcn_perm(h[3], h[2], 0x06040200u);
  const uint2 v = make_uint2(p0, p1);
  if (seg == 0) {
    int8_t* dst;
    if (a.x_frag) {
      // frag_offset(8 inst + row, col, ldx / 64) with the instance's rows 8 (inst & 1) .. +7
      // of 16-row group inst >> 1; eight consecutive columns stay inside one 16-byte slot
      const uint32_t row = __umulhi(2u * lb, magic), col = 8u * (lb - row * nb);
      const uint32_t r16 = ((uint32_t)(inst & 1) << 3) | row;
      dst = a.X + (size_t)(inst >> 1) * (size_t)(a.ldx >> 6) * 1024u +
            (((col >> 6) * 64u + (r16 | (((col & 63u) >> 4) << 4))) * 16u + (col & 15u));
    } else if (a.ldx == a.n) {
      dst = a.X + (size_t)inst * 8 * a.n + 8u * lb;
    } else {
      const uint32_t row = __umulhi(2u * lb, magic), col = 8u * (lb - row * nb);
      dst = a.X + ((size_t)inst * 8 + row) * a.ldx + col;
    }
    *(uint2*)dst = v;
    if (a.X16)  // int16 copy, row-major 8 x n: byte offset 2 (row n + col) = 16 lb
      *(uint4*)(a.X16 + (size_t)inst * a.x16_stride + 16u * lb) = make_uint4(h[0], h[1], h[2], h[3]);
  } else if (seg == 1) {
    *(uint2*)(a.E + (size_t)inst * 8 * a.n + 8u * lb) = v;
  } else {
    *(uint2*)(a.E2 + (size_t)inst * 64 + 8u * lb) = v;
  }
}

template <int KT>
__global__ void __launch_bounds__(64 * SAMPLE_WAVES) k_sample(SampleArgs a, int count) {
  __shared__ uint32_t TR[TR_WORDS];
  load_tables_rep(TR, a.T0);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint32_t off0 = (uint32_t)(lane & 31) << 2, off2 = off0 + 128;
  const int n = a.n;
  const uint32_t nb = (uint32_t)n >> 3, magic = 0xffffffffu / (2u * nb) + 1u;
  // Segment 0 in fragment order is walked slot by slot, so that 16 consecutive lanes fill one
  // whole 128-byte line of the fragment (an instance's 8 rows x 16 columns of one step) and a
  // store never leaves a line partly written: slot ((s * 4 + c) * 8 + r) * 2 + h is the block of
  // row r, columns 64 s + 16 c + 8 h .. +7.  Slots past column n (the last step of an n that is
  // not a multiple of 64) have no block.  Row-major segments are walked block by block.
  const int p0 = a.x_frag ? 64 * ((n + 63) >> 6) : n;  // segment 0's slots
  const int total = p0 + n + (a.nseg == 3 ? 8 : 0);   // slots per instance
  // block index within its segment of slot t, and whether the slot has a block
  auto block_of = [&](int t, int seg, bool& has) __attribute__((always_inline)) -> uint32_t {
    has = true;
    if (seg == 1) return (uint32_t)(t - p0);
    if (seg == 2) return (uint32_t)(t - p0 - n);
    if (!a.x_frag) return (uint32_t)t;
    const uint32_t col = 64u * (uint32_t)(t >> 6) + 16u * ((uint32_t)(t >> 4) & 3u) + 8u * ((uint32_t)t & 1u);
    has = col < (uint32_t)n;
    return ((uint32_t)(t >> 1) & 7u) * nb + (col >> 3);
  };
  auto seg_of = [&](int t) __attribute__((always_inline)) { return t < p0 ? 0 : (t < p0 + n ? 1 : 2); };
  // this lane's block and first column within a 64-slot step of segment 0's fragment order
  const uint32_t lane_blk = (((uint32_t)lane >> 1) & 7u) * nb + (((uint32_t)lane >> 4) & 3u) * 2u + ((uint32_t)lane & 1u);
  const uint32_t lane_col = (((uint32_t)lane >> 4) & 3u) * 16u + ((uint32_t)lane & 1u) * 8u;
  // Work unit = 64 * SAMPLE_ILP consecutive blocks of one instance, taken by one wave, so
  // that the instance's round keys are wave-uniform (scalar registers).
  const int per_unit = 64 * SAMPLE_ILP;
  const int units_per_inst = (total + per_unit - 1) / per_unit;
  const int n_units = units_per_inst * count;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nwaves = gridDim.x * SAMPLE_WAVES;
  for (int u = blockIdx.x * SAMPLE_WAVES + wave; u < n_units; u += nwaves) {
    const int inst = u / units_per_inst, chunk = u - inst * units_per_inst;
    const RoundKeys rk = load_rk(a.rk + (size_t)inst * 44);
    uint32_t rkr[36];
#pragma unroll
    for (int i = 0; i < 36; ++i) rkr[i] = rotl32(rk[4 + i], 24);
    if (chunk == 0 && a.ldx > n) {  // zero the padding columns of segment 0
      const int pad = a.ldx - n;
      for (int idx = lane; idx < 8 * pad; idx += 64) {
        const int row = inst * 8 + idx / pad, k = n + idx % pad;
        a.X[a.x_frag ? frag_offset(row, k, a.ldx >> 6) : (size_t)row * a.ldx + k] = 0;
      }
    }
    uint32_t o[SAMPLE_ILP][4];
    const int t_first = chunk * per_unit, t_last = min(t_first + per_unit - 1, total - 1);
    const int seg_first = seg_of(t_first), seg_last = seg_of(t_last);
    if (seg_first == seg_last) {
      // A unit inside one segment (the usual case) has a wave-uniform domain word: round 1's
      // fixed lookups are done once for its blocks, and the segment's stores are uniform.  In
      // segment 0's fragment order a unit starts on a 64-slot step, so slot t_first + 64 j + lane
      // is lane_blk + 8 (step) with a wave-uniform step (all of the unit's slots exist there).
      const bool fragw = seg_first == 0 && a.x_frag;
      const int seg_base = seg_first == 0 ? 0 : (seg_first == 1 ? p0 : p0 + n);
      uint32_t fx[6];
      aes_round1_fixed_rep(TR, off0, off2, rk, rkr, bswap32((uint32_t)(seg_first + 1)), fx);
#pragma unroll
      for (int j = 0; j < SAMPLE_ILP; ++j) {
        const int t = t_first + j * 64 + lane;
        const uint32_t lb = fragw ? lane_blk + 8u * (uint32_t)((t_first >> 6) + j)
                                  : (uint32_t)((t <= t_last ? t : t_last) - seg_base);
        aes_ctr_block_rep_fixed(TR, off0, off2, rk, rkr, fx, lb, o[j]);
      }
#pragma unroll
      for (int j = 0; j < SAMPLE_ILP; ++j) {
        const int t = t_first + j * 64 + lane;
        if (fragw) {
          if (lane_col + 64u * (uint32_t)((t_first >> 6) + j) < (uint32_t)n)
            sample_store<KT>(a, inst, 0, lane_blk + 8u * (uint32_t)((t_first >> 6) + j), nb, magic, o[j]);
        } else if (t <= t_last) {
          sample_store<KT>(a, inst, seg_first, (uint32_t)(t - seg_base), nb, magic, o[j]);
        }
      }
    } else {
      // a unit across segments (at most two per instance): one block at a time
#pragma unroll 1
      for (int j = 0; j < SAMPLE_ILP; ++j) {
        const int t = t_first + j * 64 + lane;
        const int tc = t < total ? t : total - 1;
        const int seg = seg_of(tc);
        bool has;
        const uint32_t lb = block_of(tc, seg, has);
        aes_ctr_block_rep(TR, off0, off2, rk, rkr, bswap32((uint32_t)(seg + 1)), (uint64_t)lb, o[0]);
        if (has && t < total) sample_store<KT>(a, inst, seg, lb, nb, magic, o[0]);
      }
    }
  }
}

// ======================================================================================
// Product epilogue: reduce D mod q, add the error (and for V the encoded message), then
// store, compare with a received ciphertext, or accumulate a split-K partial.
// ======================================================================================
__device__ __forceinline__ uint32_t encode_coeff(const uint8_t* mu, int mu_bytes, int B, int logq,
                                                 int coeff) {
  const int bit = coeff * B, byte = bit >> 3, sh = bit & 7;
  uint32_t v = mu[byte];
  if (byte + 1 < mu_bytes) v |= (uint32_t)mu[byte + 1] << 8;
  return ((v >> sh) & ((1u << B) - 1u)) << (logq - B);
}

// value of output element (row, col) of the encryption / keygen layouts, and its byte
// offset inside the record
__device__ __forceinline__ void epi_value(const ProdArgs& a, int row, int col, uint32_t D,
                                          uint32_t& val, size_t& off) {
  const int inst = row >> 3, r = row & 7, n = a.n;
  const uint32_t qmask = (1u << a.logq) - 1u;
  if (col < n) {
    val = (D + (uint32_t)(int32_t)a.E[(size_t)row * n + col]) & qmask;
    off = a.out_off + 2 * ((size_t)r * n + col);
  } else {
    const int c = col - n;
    const int mb = 8 * a.B;
    val = (D + (uint32_t)(int32_t)a.E2[(size_t)inst * 64 + r * 8 + c] +
           encode_coeff(a.mu + (size_t)inst * a.mu_stride, mb, a.B, a.logq, r * 8 + c)) &
          qmask;
    off = 2 * ((size_t)8 * n + r * 8 + c);
  }
}

// Finalises one element; returns 1 if (compare mode) it differs from the received ct.
__device__ __forceinline__ uint32_t epi_store(const ProdArgs& a, int row, int col, uint32_t D) {
  uint32_t val;
  size_t off;
  epi_value(a, row, col, D, val, off);
  const int inst = row >> 3;
  if (a.mode == PM_COMPARE) {
    const uint16_t got = *(const uint16_t*)(a.cmp + (size_t)inst * a.cmp_stride + off);
    return got != (uint16_t)val ? 1u : 0u;
  }
  *(uint16_t*)(a.out + (size_t)inst * a.out_stride + off) = (uint16_t)val;
  return 0u;
}

// Compare mode: lanes 0-31 of a 16-row MFMA tile hold rows 0-7 (one instance) and lanes
// 32-63 rows 8-15 (the next one).  One atomic per instance and tile, whatever the data.
__device__ __forceinline__ void flag_tile(const ProdArgs& a, int row_base, uint32_t mism) {
  const uint64_t bal = __ballot(mism != 0);
  const int lane = threadIdx.x & 63;
  // OR-ing a zero changes nothing: only a mismatch issues an atomic
  if (lane == 0 && row_base < a.M && (bal & 0xffffffffull)) atomicOr(&a.flags[row_base >> 3], 1u);
  if (lane == 32 && row_base + 8 < a.M && (bal >> 32)) atomicOr(&a.flags[(row_base >> 3) + 1], 1u);
}

// ---- the paper's sets (prime q) ----
// x mod q for x < 2^64 (a multiple of q added first keeps negative sums non-negative)
__device__ __forceinline__ uint32_t mod_q64(long long x, uint32_t q) {
  long long r = x % (long long)q;
  return (uint32_t)(r < 0 ? r + (long long)q : r);
}

// A[i][j] = word mod q for the two 16-bit words of w (both halves; none for q > 2^16)
__device__ __forceinline__ uint32_t reduce_pair_q(uint32_t w, uint32_t q, uint32_t magic) {
  if (!magic) return w;
  const uint32_t x0 = w & 0xffffu, x1 = w >> 16;
  const uint32_t r0 = x0 - q * __umulhi(x0, magic), r1 = x1 - q * __umulhi(x1, magic);
  return r0 | (r1 << 16);
}

// Offset limbs of four values x < 2^16 held as 16-bit halves of a and b: the int8 bytes
// lo - 128 and hi - 128 (the bytes of x with the top bit flipped).
__device__ __forceinline__ void limbs4_offset(uint32_t a, uint32_t b, uint32_t& lo, uint32_t& hi) {
  lo = __builtin_amdgcn_perm(b, a, 0x06040200u) ^ 0x80808080u;
  hi = __builtin_amdgcn_perm(b, a, 0x07050301u) ^ 0x80808080u;
}

// Finalises element (row, col) of a paper-set product: D holds sums of limb partials already
// reduced mod q; adds the limb offsets' correction, the error and reduces mod q; stores the
// coefficient (keygen: t at out_off of the pk record; encryption: u_r[col] of the ct record),
// or in compare mode returns 1 if it differs from the received one.
__device__ __forceinline__ uint32_t epi_store_prime(const ProdArgs& a, int row, int col, uint32_t D) {
  const int inst = row / a.rows_per_inst, r = row - inst * a.rows_per_inst;
  const long long v = (long long)D + 32896LL * a.rowsum[row] + (long long)a.E[(size_t)row * a.n + col];
  const uint32_t val = mod_q64(v, a.qp);
  const size_t off = a.out_off + (size_t)a.coef_bytes * ((size_t)r * a.n + col);
  if (a.mode == PM_COMPARE) {
    const uint8_t* src = a.cmp + (size_t)inst * a.cmp_stride + off;
    const uint32_t got = a.coef_bytes == 4 ? *(const uint32_t*)src : (uint32_t)*(const uint16_t*)src;
    return got != val ? 1u : 0u;
  }
  uint8_t* dst = a.out + (size_t)inst * a.out_stride + off;
  if (a.coef_bytes == 4)
    *(uint32_t*)dst = val;
  else
    *(uint16_t*)dst = (uint16_t)val;
  return 0u;
}

// ======================================================================================
// Product, streaming form (small row counts: plain encryption, all key generations).
// Each wave generates its own A fragments per 64-row contraction step and multiplies them
// at once; waves of a workgroup split the K chunk and are reduced through LDS.
//   grid.x = n_jt * n_kc, grid.y = row tiles (or instances when per_inst_A)
// ======================================================================================
// MAT: read A from the expanded copy a.Amat instead of regenerating it (unfused variant).
// PRIME: the paper's sets (A mod a prime q, offset limbs, exact reduction mod q).
template <int CG, int RG, bool TRANS, bool MAT, bool PRIME = false>
__global__ void __launch_bounds__(1024) k_prod_stream(ProdArgs a, int ks_per_wave) {
  // Lane-replicated T-tables in static LDS (64 KB, conflict-free lookups; none in the unfused
  // variant); the reduction / transpose scratch in dynamic LDS.
  __shared__ uint32_t TR[MAT ? 1 : TR_WORDS];
  extern __shared__ uint32_t smem[];
  const int W = blockDim.x >> 6;
  uint32_t* red = smem;                                         // [W][RG][CG][4][64]
  uint8_t* tr = (uint8_t*)(red + (size_t)W * RG * CG * 256);    // TRANS: [W][2][CG][16][64]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int jt = blockIdx.x % a.n_jt, kc = blockIdx.x / a.n_jt, mt = blockIdx.y;
  const RoundKeys rk = load_rk(a.rkA + (a.per_inst_A ? (size_t)mt * 44 : 0));
  uint32_t rkr[36];  // rotr8 of round-key words 4 .. 39 (replicated-table AES)
#pragma unroll
  for (int i = 0; i < 36; ++i) rkr[i] = rotl32(rk[4 + i], 24);
  const uint32_t off0 = (uint32_t)(lane & 31) << 2, off2 = off0 + 128;
  const int n = a.n;
  const int m_begin = mt * a.m_tile, m_end = min(a.M, m_begin + a.m_tile);
  const int nn0 = jt * 16 * CG;
  const uint32_t qmask2 = ((1u << a.logq) - 1u) * 0x10001u;
  const int k_chunk0 = kc * a.kc_len;

  if constexpr (!MAT) load_tables_rep(TR, a.T0);
  __syncthreads();
  // domain 0 and block indices below 2^32 (n <= 32768): round 1's fixed part once per workgroup
  uint32_t fx[6];
  if constexpr (!MAT) aes_round1_fixed_rep(TR, off0, off2, rk, rkr, 0u, fx);

  v4i acc[RG][CG][2];
#pragma unroll
  for (int rg = 0; rg < RG; ++rg)
#pragma unroll
    for (int cg = 0; cg < CG; ++cg) acc[rg][cg][0] = acc[rg][cg][1] = v4i{0, 0, 0, 0};

  for (int st = 0; st < ks_per_wave; ++st) {
    const int kbase = k_chunk0 + (wave * ks_per_wave + st) * 64;
    const bool kvalid = kbase < n && (wave * ks_per_wave + st) * 64 < a.kc_len;
    v4i xf[RG];
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) {
      const int row = m_begin + rg * 16 + (lane & 15);
      const int k = kbase + 16 * (lane >> 4);
      if (kvalid && row < m_end)
        xf[rg] = *(const v4i*)(a.X + (size_t)row * a.ldx + k);
      else
        xf[rg] = v4i{0, 0, 0, 0};
    }
    v4i yf[CG][2];
    if constexpr (!TRANS) {
#pragma unroll
      for (int cg = 0; cg < CG; ++cg) {
        const int col = nn0 + cg * 16 + (lane & 15);
        const int k = kbase + 16 * (lane >> 4);
        uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (kvalid && k < n) {
          if (col < n) {
            if constexpr (MAT) {
              const uint16_t* src = a.Amat + (size_t)col * n + k;
              const uint4 v0 = *(const uint4*)src;
              w[0] = v0.x; w[1] = v0.y; w[2] = v0.z; w[3] = v0.w;
              if (k + 8 < n) {
                const uint4 v1 = *(const uint4*)(src + 8);
                w[4] = v1.x; w[5] = v1.y; w[6] = v1.z; w[7] = v1.w;
              }
            } else {
              const uint32_t b = (uint32_t)(((uint64_t)col * n + k) >> 3);
              aes_ctr_block_rep_fixed(TR, off0, off2, rk, rkr, fx, b, w);
              if (k + 8 < n) aes_ctr_block_rep_fixed(TR, off0, off2, rk, rkr, fx, b + 1, w + 4);
            }
          } else if (col < n + 8 && a.Bt) {
            const uint4 v0 = *(const uint4*)(a.Bt + 2 * ((size_t)(col - n) * n + k));
            w[0] = v0.x; w[1] = v0.y; w[2] = v0.z; w[3] = v0.w;
            if (k + 8 < n) {
              const uint4 v1 = *(const uint4*)(a.Bt + 2 * ((size_t)(col - n) * n + k + 8));
              w[4] = v1.x; w[5] = v1.y; w[6] = v1.z; w[7] = v1.w;
            }
          }
        }
        uint32_t lo[4], hi[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if constexpr (PRIME)
            limbs4_offset(reduce_pair_q(w[2 * q], a.qp, a.qp_magic), reduce_pair_q(w[2 * q + 1], a.qp, a.qp_magic),
                          lo[q], hi[q]);
          else
            limbs4(w[2 * q] & qmask2, w[2 * q + 1] & qmask2, lo[q], hi[q]);
        }
        yf[cg][0] = v4i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3]};
        yf[cg][1] = v4i{(int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
      }
    } else {
      // lane l owns column j = kbase + l of A and 16 consecutive rows per column group;
      // the 64 x 16 tile is transposed through this wave's LDS slice.
      uint8_t* my = tr + (size_t)wave * 2 * CG * 1024;
      const int j = kbase + lane;
#pragma unroll
      for (int cg = 0; cg < CG; ++cg) {
        const int i0 = nn0 + cg * 16;
        uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (kvalid && j < n && i0 < n) {
          if constexpr (MAT) {
            const uint16_t* src = a.Amat + (size_t)j * n + i0;
            const uint4 v0 = *(const uint4*)src;
            w[0] = v0.x; w[1] = v0.y; w[2] = v0.z; w[3] = v0.w;
            if (i0 + 8 < n) {
              const uint4 v1 = *(const uint4*)(src + 8);
              w[4] = v1.x; w[5] = v1.y; w[6] = v1.z; w[7] = v1.w;
            }
          } else {
            const uint32_t b = (uint32_t)(((uint64_t)j * n + i0) >> 3);
            aes_ctr_block_rep_fixed(TR, off0, off2, rk, rkr, fx, b, w);
            if (i0 + 8 < n) aes_ctr_block_rep_fixed(TR, off0, off2, rk, rkr, fx, b + 1, w + 4);
          }
        }
        uint32_t lo[4], hi[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if constexpr (PRIME)
            limbs4_offset(reduce_pair_q(w[2 * q], a.qp, a.qp_magic), reduce_pair_q(w[2 * q + 1], a.qp, a.qp_magic),
                          lo[q], hi[q]);
          else
            limbs4(w[2 * q] & qmask2, w[2 * q + 1] & qmask2, lo[q], hi[q]);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          my[(0 * CG + cg) * 1024 + r * 64 + lane] = (uint8_t)(lo[r >> 2] >> (8 * (r & 3)));
          my[(1 * CG + cg) * 1024 + r * 64 + lane] = (uint8_t)(hi[r >> 2] >> (8 * (r & 3)));
        }
      }
      __syncthreads();
#pragma unroll
      for (int cg = 0; cg < CG; ++cg)
#pragma unroll
        for (int limb = 0; limb < 2; ++limb)
          yf[cg][limb] = *(const v4i*)(my + (limb * CG + cg) * 1024 + (lane & 15) * 64 +
                                       16 * (lane >> 4));
      __syncthreads();
    }
#pragma unroll
    for (int rg = 0; rg < RG; ++rg)
#pragma unroll
      for (int cg = 0; cg < CG; ++cg)
#pragma unroll
        for (int limb = 0; limb < 2; ++limb)
          acc[rg][cg][limb] =
              __builtin_amdgcn_mfma_i32_16x16x64_i8(xf[rg], yf[cg][limb], acc[rg][cg][limb], 0, 0, 0);
  }

  // recombine limbs; reduce the waves' partial sums through LDS
  uint32_t D[RG][CG][4];
#pragma unroll
  for (int rg = 0; rg < RG; ++rg)
#pragma unroll
    for (int cg = 0; cg < CG; ++cg)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if constexpr (PRIME)
          D[rg][cg][i] = mod_q64((long long)acc[rg][cg][0][i] + 256LL * acc[rg][cg][1][i], a.qp);
        else
          D[rg][cg][i] = (uint32_t)acc[rg][cg][0][i] + ((uint32_t)acc[rg][cg][1][i] << 8);
      }
  if (W > 1) {
#pragma unroll
    for (int rg = 0; rg < RG; ++rg)
#pragma unroll
      for (int cg = 0; cg < CG; ++cg)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          red[(((size_t)wave * RG + rg) * CG + cg) * 256 + i * 64 + lane] = D[rg][cg][i];
    __syncthreads();
    if (wave != 0) return;
    for (int w = 1; w < W; ++w)
#pragma unroll
      for (int rg = 0; rg < RG; ++rg)
#pragma unroll
        for (int cg = 0; cg < CG; ++cg)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            D[rg][cg][i] += red[(((size_t)w * RG + rg) * CG + cg) * 256 + i * 64 + lane];
  }
#pragma unroll
  for (int rg = 0; rg < RG; ++rg) {
    uint32_t mism = 0;
    const int row_base = m_begin + rg * 16;
#pragma unroll
    for (int cg = 0; cg < CG; ++cg)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = row_base + 4 * (lane >> 4) + i;
        const int col = nn0 + cg * 16 + (lane & 15);
        if (row >= m_end || col >= a.ncols) continue;
        if (a.n_kc > 1)
          atomicAdd((uint32_t*)&a.acc32[(size_t)row * a.acc_ld + col], D[rg][cg][i]);
        else if constexpr (PRIME)
          mism |= epi_store_prime(a, row, col, D[rg][cg][i]);
        else
          mism |= epi_store(a, row, col, D[rg][cg][i]);
      }
    if (a.mode == PM_COMPARE && a.n_kc == 1) {
      if constexpr (PRIME) {
        // rows_per_inst (256) is a multiple of 16: the tile's rows belong to one instance
        if (__ballot(mism != 0) && (threadIdx.x & 63) == 0 && row_base < m_end)
          atomicOr(&a.flags[row_base / a.rows_per_inst], 1u);
      } else {
        flag_tile(a, row_base, mism);
      }
    }
  }
}

// ======================================================================================
// Product, strip form (large row counts: batched encryption against one public key).
// The workgroup regenerates a strip of A (all contraction rows of the K chunk x 16*CG
// columns) into LDS once, already split into limbs and laid out as MFMA fragments, and
// then streams every row tile of its row chunk through it.  The MFMA computes the
// transposed tile (A strip as the first operand), so each lane ends up holding four
// consecutive columns of one output row: the epilogue reads E' four bytes, and stores or
// compares the result eight bytes at a time after a lane transpose.
//   LDS: the strip, [ksteps][CG][limb][64 lanes][16 bytes] (dynamic), and the AES table
//   copies (64 KB, beside it or inside its space during the regeneration, see TAB below).
// Workgroup ids are remapped so that each XCD (ids congruent mod 8) processes a
// contiguous range of tiles, i.e. the same row chunks share that XCD's L2.
// ======================================================================================
constexpr int STRIP_WAVES = 8;

// UNR: contraction steps per unrolled loop body, and the depth of the X register ring (X
// fragments are requested UNR - 1 steps ahead; the strip is padded to a multiple of UNR).
// TAB: where the strip comes from.  0: the expanded copy a.Amat (unfused variant; the loop
// and epilogue are the same).  3 and 4: AES with the 64 KB conflict-free T0/T2 copies (one
// address per byte move, one rotation per column), 3 with the copies in static LDS beside the
// strip, 4 (strips too large to sit beside the copies, so larger than 96 KB) with the copies
// in the first 64 KB of the strip's own space: the blocks that land elsewhere are written first;
// those of the first 64 KB are held in registers (eight per thread) until every lookup is
// done, then written over the copies.
template <int CG, int RG, bool CMP, int UNR, int TAB>
__global__ void __launch_bounds__(64 * STRIP_WAVES) k_prod_strip(ProdArgs a) {
  constexpr bool MAT = TAB == 0;
  // strip-fragment ring depth: the phases of one loop body must fill whole ring turns
  constexpr int YD = (UNR * CG) % 3 == 0 ? 3 : 2;
  static_assert((UNR * CG) % YD == 0, "strip fragment ring does not tile the loop body");
  // static: a compile-time address for the table lookups
  static_assert(TAB == 0 || TAB == 3 || TAB == 4, "strip table mode");
  __shared__ uint32_t T[TAB == 3 ? TR_WORDS : 1];
  extern __shared__ uint32_t smem[];
  // the T0/T2 copies: static (TAB 3) or in the strip's space (TAB 4)
  uint32_t* const TRt = TAB == 4 ? smem : T;
  uint8_t* strip = (uint8_t*)smem;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int total = a.n_jt * a.n_kc * a.n_mt;
  const int per = (total + 7) / 8;
  const int v = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (v >= total) return;
  const int jt = v % a.n_jt;
  const int kc = (v / a.n_jt) % a.n_kc;
  const int mt = v / (a.n_jt * a.n_kc);
  const int n = a.n;
  const int nn0 = jt * 16 * CG;
  const int k0 = kc * a.kc_len;
  const int k_len = min(a.kc_len, n - k0);
  const int ksteps = (k_len + 63) >> 6;
  // The contraction loop runs UNR steps per iteration; the strip is padded with zero rows of
  // A up to that multiple (a zero strip row adds nothing to any product).
  const int kst = strip_steps(k_len, UNR);
  const uint32_t qmask = (1u << a.logq) - 1u;
  const uint32_t qmask2 = qmask * 0x10001u;
  const RoundKeys rk = load_rk(a.rkA);
  uint32_t rkr[36];  // rotr8 of round-key words 4 .. 39 (conflict-free table AES)
#pragma unroll
  for (int i = 0; i < 36; ++i) rkr[i] = rotl32(rk[4 + i], 24);
  const uint32_t qoff = (uint32_t)(lane & 31) << 2;

  if constexpr (!MAT) load_tables_rep(TRt, a.T0);
  __syncthreads();
  // domain 0 and block indices below 2^32 (n <= 32768): round 1's fixed part once per workgroup
  uint32_t fx[6];
  if constexpr (!MAT) aes_round1_fixed_rep(TRt, qoff, qoff + 128, rk, rkr, 0u, fx);

  // ---- regenerate (or, unfused, copy) the strip ----
  // Item t = one AES block = 8 consecutive contraction rows of one column.  Items are
  // numbered so that consecutive lanes fill consecutive 16-byte fragment slots (conflict-free
  // LDS stores): t = (((s * CG + cg) * 4 + g) * 2 + h) * 16 + c16, where the block covers rows
  // s*64 + g*16 + h*8 .. +7 of column 16*cg + c16 and lands in fragment lane g*16 + c16,
  // bytes h*8 .. +7.  Four blocks per thread and iteration, computed without branches (an
  // entry outside A is overwritten afterwards), so that the AES chains interleave.
  const int items = 16 * CG * kst * 8;
  struct Item {
    int col_local, kb;
  };
  auto item = [&](int t) __attribute__((always_inline)) {
    const int c16 = t & 15, h = (t >> 4) & 1, g = (t >> 5) & 3, rest = t >> 7;
    return Item{(rest % CG) * 16 + c16, (rest / CG) * 8 + g * 2 + h};
  };
  auto put = [&](int t, const uint32_t (&w)[4]) __attribute__((always_inline)) {
    uint32_t lo0, hi0, lo1, hi1;
    limbs4(w[0] & qmask2, w[1] & qmask2, lo0, hi0);
    limbs4(w[2] & qmask2, w[3] & qmask2, lo1, hi1);
    // fragment (s, cg, limb) base + lane slot: the same numbering as t without its h bit
    const int c16 = t & 15, h = (t >> 4) & 1, g = (t >> 5) & 3, rest = t >> 7;
    uint8_t* base = strip + ((size_t)(rest * 2) * 64 + g * 16 + c16) * 16 + h * 8;
    *(uint2*)base = make_uint2(lo0, lo1);
    *(uint2*)(base + 64 * 16) = make_uint2(hi0, hi1);
  };
  // entries outside A: zero padding rows, and the public-key columns (B^T) when present
  auto fixup = [&](const Item& it, uint32_t (&w)[4]) __attribute__((always_inline)) {
    const int k = k0 + 8 * it.kb, col = nn0 + it.col_local;
    if (k >= k0 + k_len || col >= n) {
      w[0] = w[1] = w[2] = w[3] = 0;
      if (k < k0 + k_len && col < n + 8 && a.Bt) {
        const uint4 bv = *(const uint4*)(a.Bt + 2 * ((size_t)(col - n) * n + k));
        w[0] = bv.x; w[1] = bv.y; w[2] = bv.z; w[3] = bv.w;
      }
    }
  };
  auto gen = [&](int t, uint32_t (&w)[4]) __attribute__((always_inline)) {
    const Item it = item(t);
    const int c = nn0 + it.col_local, k = k0 + 8 * it.kb;
    if constexpr (MAT) {
      // entries outside A read a valid one; fixup overwrites them below
      const int cc = c < n ? c : 0, kk = k < k0 + k_len ? k : k0;
      const uint4 v = *(const uint4*)(a.Amat + (size_t)cc * n + kk);
      w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    } else {
      aes_ctr_block_rep_fixed(TRt, qoff, qoff + 128, rk, rkr, fx, (uint32_t)(((uint64_t)c * n + k) >> 3), w);
    }
  };
  // TAB 4: items below HELD land in the table copies' 64 KB (128 items per 2 KB fragment pair)
  constexpr int HELD = TAB == 4 ? TR_WORDS * 4 / 2048 * 128 : 0;
  constexpr int ILP = 4;
  for (int t0 = HELD + threadIdx.x; t0 < items; t0 += ILP * blockDim.x) {
    int tt[ILP];
    uint32_t w[ILP][4];
#pragma unroll
    for (int j = 0; j < ILP; ++j) {
      const int t = t0 + j * blockDim.x;
      tt[j] = t < items ? t : t0;  // past the end: recompute t0, stored once
      gen(tt[j], w[j]);
    }
#pragma unroll
    for (int j = 0; j < ILP; ++j) {
      fixup(item(tt[j]), w[j]);
      if (j == 0 || tt[j] != t0) put(tt[j], w[j]);
    }
  }
  if constexpr (TAB == 4) {
    // the launch guarantees items >= HELD (a strip of at least 64 KB)
    constexpr int PER = HELD / (64 * STRIP_WAVES);
    static_assert(HELD % (64 * STRIP_WAVES) == 0, "held items per thread");
    uint32_t wh[PER][4];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int t = threadIdx.x + j * 64 * STRIP_WAVES;
      gen(t, wh[j]);
      fixup(item(t), wh[j]);
    }
    __syncthreads();  // every lookup into the copies is done
#pragma unroll
    for (int j = 0; j < PER; ++j) put(threadIdx.x + j * 64 * STRIP_WAVES, wh[j]);
  }
  __syncthreads();

  // ---- stream the row tiles ----
  // Each wave takes row blocks wave, wave + STRIP_WAVES, ...  Its loads form one continuous
  // software pipeline over (row block, step): X fragments three steps deep (global loads
  // issued two steps ahead, running into the next row block at the end of a block), strip
  // fragments three deep (LDS reads one step ahead, wrapping to step 0).  The rings are
  // indexed with compile-time slots in a three-step unrolled body (the strip is padded to a
  // multiple of three steps), so no register moves tie a wait on a fresh load to the current
  // step.  Rows past the chunk end read row m_begin instead (their results are never
  // stored), and X loads past the last real step re-read it (they meet zero strip rows), so
  // every operand load is unconditional and in bounds.  S' is in fragment order
  // (frag_offset): a wave's fragment of one 16-row group and step is 1 KB contiguous.
  const int m_begin = mt * a.m_tile, m_end = min(a.M, m_begin + a.m_tile);
  const int rows = m_end - m_begin;
  const int nrb = (rows + 16 * RG - 1) / (16 * RG);
  if (wave >= nrb) return;
  const int klast = ksteps - 1;
  // Fast tiles: the whole strip lies in B' (columns < n) and the contraction is not split,
  // so the epilogue is E' add, mask and one 8-byte store (or compare) per tile.  The other
  // workgroups (the strip holding V's columns, split-K) take the general epilogue.
  const bool fast = a.n_kc == 1 && nn0 + 16 * CG <= n;
  const int xsteps = a.ldx >> 6;
  auto row_offs = [&](int rb, size_t (&o)[RG]) __attribute__((always_inline)) {
    const int rbase = m_begin + rb * 16 * RG;
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) {
      const int g0 = rbase + rg * 16;  // groups past the chunk end read the chunk's first one
      o[rg] = ((size_t)((g0 < m_end ? g0 : m_begin) >> 4) * xsteps + (k0 >> 6)) * 1024;
    }
  };
  size_t xp[RG];  // current row block
  size_t xq[RG];  // next row block of this wave (the current one if there is none)
  row_offs(wave, xp);
  row_offs(wave + STRIP_WAVES < nrb ? wave + STRIP_WAVES : wave, xq);
  const int lane16 = 16 * lane;

  v4i xb[UNR][RG];  // X ring: slot = step mod UNR
  v4i yb[YD][2];    // strip fragment ring: slot = phase mod YD, a phase being one (step, cg)
  auto load_xs = [&](v4i (&dst)[RG], const size_t (&o)[RG], int s) __attribute__((always_inline)) {
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) dst[rg] = *(const v4i*)(a.X + (o[rg] + 1024 * (size_t)s) + lane16);
  };
  auto load_y = [&](v4i (&dst)[2], int s, int cg) __attribute__((always_inline)) {
    dst[0] = *(const v4i*)(strip + ((size_t)((s * CG + cg) * 2) * 64 + lane) * 16);
    dst[1] = *(const v4i*)(strip + ((size_t)((s * CG + cg) * 2 + 1) * 64 + lane) * 16);
  };
  v4i acc[RG][CG][2];
#pragma unroll
  for (int i = 0; i + 1 < UNR; ++i) load_xs(xb[i], xp, min(i, klast));
  load_y(yb[0], 0, 0);
  // UNR steps per iteration.  At each step the X fragments of step + UNR - 1 are requested
  // (from the next row block past the last step); at each phase the strip fragments of the
  // next phase (wrapping from the last step to step 0, the strip being the same for every
  // row block).  Scheduling barriers keep every request ahead of the MFMAs that hide it; the
  // scheduler would otherwise sink the loads next to their first use.
  auto body = [&](int s, auto last_tag) __attribute__((always_inline)) {
    constexpr bool LAST = decltype(last_tag)::value;
#pragma unroll
    for (int i = 0; i < UNR; ++i) {
      const int t = s + i, t2 = t + UNR - 1;
      if (!LAST || i == 0)
        load_xs(xb[(i + UNR - 1) % UNR], xp, min(t2, klast));
      else
        load_xs(xb[(i + UNR - 1) % UNR], xq, min(i - 1, klast));
#pragma unroll
      for (int cg = 0; cg < CG; ++cg) {
        const int ph = i * CG + cg;
        if (cg + 1 < CG)
          load_y(yb[(ph + 1) % YD], t, cg + 1);
        else
          load_y(yb[(ph + 1) % YD], (!LAST || i + 1 < UNR) ? t + 1 : 0, 0);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
          acc[rg][cg][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(yb[ph % YD][0], xb[i][rg], acc[rg][cg][0], 0, 0, 0);
          acc[rg][cg][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(yb[ph % YD][1], xb[i][rg], acc[rg][cg][1], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };

  // One pass over this wave's row blocks; FAST selects the epilogue (uniform per workgroup).
  auto run = [&](auto fast_tag) __attribute__((always_inline)) {
    constexpr bool FAST = decltype(fast_tag)::value;
    for (int rb = wave; rb < nrb; rb += STRIP_WAVES) {
      const int rbase = m_begin + rb * 16 * RG;
#pragma unroll
      for (int rg = 0; rg < RG; ++rg)
#pragma unroll
        for (int cg = 0; cg < CG; ++cg) acc[rg][cg][0] = acc[rg][cg][1] = v4i{0, 0, 0, 0};
      // Fast epilogue operands (E' words, and in compare mode the received ciphertext
      // words), loaded now so that their latency hides behind the contraction.  The loads
      // are unconditional (rows past the chunk end read row m_begin): no branch around them
      // keeps the wait before their use exact.  E' comes in the MFMA result layout (lane
      // (r, g) = (lane & 15, lane >> 4): row r, columns 4g .. 4g+3); the ciphertext words in
      // the transposed one that the epilogue stores and compares in (lane 4r + g).
      uint32_t epre[RG][CG];
      uint2 cpre[RG][CG];
      if constexpr (FAST) {
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
          const int row0 = rbase + rg * 16 + (lane & 15);
          const int row = row0 < m_end ? row0 : m_begin;
          const int rowt0 = rbase + rg * 16 + (lane >> 2);
          const int rowt = rowt0 < m_end ? rowt0 : m_begin;
#pragma unroll
          for (int cg = 0; cg < CG; ++cg) {
            const int col0 = nn0 + cg * 16 + 4 * (lane >> 4);
            epre[rg][cg] = *(const uint32_t*)(a.E + (size_t)row * n + col0);
            if constexpr (CMP) {
              const int colt = nn0 + cg * 16 + 4 * (lane & 3);
              cpre[rg][cg] = *(const uint2*)(a.cmp + (size_t)(rowt >> 3) * a.cmp_stride + a.out_off +
                                             2 * ((size_t)(rowt & 7) * n + colt));
            }
          }
        }
      }
      for (int s = 0; s + UNR < kst; s += UNR) body(s, std::false_type{});
      body(kst - UNR, std::true_type{});
#pragma unroll
      for (int rg = 0; rg < RG; ++rg) xp[rg] = xq[rg];
      {
        const int nb = rb + 2 * STRIP_WAVES;
        row_offs(nb < nrb ? nb : (rb + STRIP_WAVES < nrb ? rb + STRIP_WAVES : rb), xq);
      }

      // epilogue: lane holds columns 4*(lane>>4) .. +3 of row (lane & 15) of each 16x16 tile
#pragma unroll
      for (int rg = 0; rg < RG; ++rg) {
        const int row = rbase + rg * 16 + (lane & 15);
        const bool rvalid = row < m_end;
        const int inst = row >> 3, r = row & 7;
        uint32_t mism = 0;
#pragma unroll
        for (int cg = 0; cg < CG; ++cg) {
          const int col0 = nn0 + cg * 16 + 4 * (lane >> 4);
          uint32_t D[4];
#pragma unroll
          for (int i = 0; i < 4; ++i)
            D[i] = (uint32_t)acc[rg][cg][0][i] + ((uint32_t)acc[rg][cg][1][i] << 8);
          if constexpr (FAST) {
            const uint32_t e4 = epre[rg][cg];
            uint32_t v4[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) v4[i] = (D[i] + (uint32_t)(int32_t)(int8_t)(e4 >> (8 * i))) & qmask;
            const uint2 packed = make_uint2(v4[0] | (v4[1] << 16), v4[2] | (v4[3] << 16));
            // Lane (r, g) holds columns 4g .. 4g+3 of tile row r.  Transpose the 16 x 4 lane
            // grid so that lane 4r + g holds them: four consecutive lanes then cover one row's
            // 32 contiguous bytes, and a store or load touches 16 segments instead of 64.
            const int src = (((lane & 3) << 4) | (lane >> 2)) << 2;
            const uint2 sw = make_uint2((uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)packed.x),
                                        (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)packed.y));
            const int row2 = rbase + rg * 16 + (lane >> 2), col2 = nn0 + cg * 16 + 4 * (lane & 3);
            if constexpr (CMP) {
              mism |= row2 < m_end ? (cpre[rg][cg].x ^ sw.x) | (cpre[rg][cg].y ^ sw.y) : 0u;
            } else if (row2 < m_end) {
              *(uint2*)(a.out + (size_t)(row2 >> 3) * a.out_stride + a.out_off +
                        2 * ((size_t)(row2 & 7) * n + col2)) = sw;
            }
          } else {
            if (!rvalid) continue;
            if (a.n_kc > 1) {
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (col0 + i < a.ncols) atomicAdd((uint32_t*)&a.acc32[(size_t)row * a.acc_ld + col0 + i], D[i]);
            } else if (col0 + 4 <= n) {
              // a B' (or B^T) tile of the edge strip: as in the fast path
              const uint32_t e4 = *(const uint32_t*)(a.E + (size_t)row * n + col0);
              uint32_t v4[4];
#pragma unroll
              for (int i = 0; i < 4; ++i) v4[i] = (D[i] + (uint32_t)(int32_t)(int8_t)(e4 >> (8 * i))) & qmask;
              const uint2 packed = make_uint2(v4[0] | (v4[1] << 16), v4[2] | (v4[3] << 16));
              const size_t off = a.out_off + 2 * ((size_t)r * n + col0);
              if constexpr (CMP) {
                const uint2 got = *(const uint2*)(a.cmp + (size_t)inst * a.cmp_stride + off);
                mism |= (got.x ^ packed.x) | (got.y ^ packed.y);
              } else {
                *(uint2*)(a.out + (size_t)inst * a.out_stride + off) = packed;
              }
            } else if (col0 + 4 <= a.ncols) {
              // Four V coefficients c0 .. c0+3 of row r: V = D + E'' + enc(mu).  (n is a
              // multiple of 8, so a tile never straddles column n; columns past ncols are
              // padding.)
              const int c0 = col0 - n, coeff = r * 8 + c0;
              const uint32_t e4 = *(const uint32_t*)(a.E2 + (size_t)inst * 64 + coeff);
              const uint8_t* mu = a.mu + (size_t)inst * a.mu_stride;
              const int mb = 8 * a.B, bit = coeff * a.B, byte = bit >> 3, sh = bit & 7;
              uint32_t win = 0;  // message bits from bit `bit` on (at most 4B + 7 <= 31 bits used)
#pragma unroll
              for (int kb = 0; kb < 4; ++kb)
                if (byte + kb < mb) win |= (uint32_t)mu[byte + kb] << (8 * kb);
              win >>= sh;
              const uint32_t kmask = (1u << a.B) - 1u;
              uint32_t v4[4];
#pragma unroll
              for (int i = 0; i < 4; ++i)
                v4[i] = (D[i] + (uint32_t)(int32_t)(int8_t)(e4 >> (8 * i)) +
                         (((win >> (i * a.B)) & kmask) << (a.logq - a.B))) & qmask;
              const uint2 packed = make_uint2(v4[0] | (v4[1] << 16), v4[2] | (v4[3] << 16));
              const size_t off = 2 * ((size_t)8 * n + coeff);
              if constexpr (CMP) {
                const uint2 got = *(const uint2*)(a.cmp + (size_t)inst * a.cmp_stride + off);
                mism |= (got.x ^ packed.x) | (got.y ^ packed.y);
              } else {
                *(uint2*)(a.out + (size_t)inst * a.out_stride + off) = packed;
              }
            }
          }
        }
        if (CMP && a.n_kc == 1) {
          // Rows 0-7 of the tile are one instance, rows 8-15 the next: the lanes with
          // (lane & 15) < 8 and the others in the result layout, lanes 0-31 and 32-63 in the
          // transposed one (fast path).
          const uint64_t bal = __ballot(mism != 0);
          const uint64_t lo = FAST ? 0x00000000FFFFFFFFull : 0x00FF00FF00FF00FFull;
          const int row_base = rbase + rg * 16;
          // Only a mismatch issues an atomic (OR-ing a zero changes nothing).  An atomic
          // in every block would hold the next block's first wait on the X loads for its
          // round trip, vector memory operations completing in order.
          if (lane == 0 && row_base < a.M && (bal & lo)) atomicOr(&a.flags[row_base >> 3], 1u);
          if (lane == 8 && row_base + 8 < a.M && (bal & ~lo)) atomicOr(&a.flags[(row_base >> 3) + 1], 1u);
        }
      }
    }
  };
  if (fast)
    run(std::true_type{});
  else
    run(std::false_type{});
}

// Completes split-K products: acc32 holds the full D for every (row, col).
__global__ void k_finalize(ProdArgs a) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)a.M * a.ncols;
  const bool valid = t < total;
  const int row = valid ? (int)(t / a.ncols) : 0, col = valid ? (int)(t % a.ncols) : 0;
  uint32_t mism = 0;
  if (a.qp) {
    // the paper's sets: one flag update per differing element (rows_per_inst rows per instance)
    if (valid) mism = epi_store_prime(a, row, col, (uint32_t)a.acc32[(size_t)row * a.acc_ld + col]);
    if (a.mode == PM_COMPARE && mism) atomicOr(&a.flags[row / a.rows_per_inst], 1u);
    return;
  }
  if (valid) mism = epi_store(a, row, col, (uint32_t)a.acc32[(size_t)row * a.acc_ld + col]);
  if (a.mode == PM_COMPARE) {
    // a wave covers at most two instances (ncols >= 16 and 8 rows per instance)
    const int lane = threadIdx.x & 63;
    const int inst = valid ? row >> 3 : -1;
    const int inst0 = __shfl(inst, 0);
    const uint64_t b0 = __ballot(mism != 0 && inst == inst0);
    const uint64_t b1 = __ballot(mism != 0 && inst != inst0);
    int inst_last = inst;
    for (int off = 32; off > 0; off >>= 1) inst_last = max(inst_last, __shfl_xor(inst_last, off));
    if (lane == 0 && inst0 >= 0 && b0) atomicOr(&a.flags[inst0], 1u);
    if (lane == 0 && inst_last != inst0 && inst_last >= 0 && b1) atomicOr(&a.flags[inst_last], 1u);
  }
}

// ======================================================================================
// Decryption M = V - B' S (mod q) and decoding (Alg. 3, generalised to B bits per
// coefficient: nearest multiple of q / 2^B, halves rounded up).
// One workgroup (4 waves splitting the contraction) per 16 rows = 2 ciphertexts.
// ======================================================================================
__global__ void __launch_bounds__(256) k_decrypt(DecArgs a) {
  __shared__ uint32_t red[4][4][64];
  __shared__ uint8_t dec[16][8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = a.n;
  const int inst0 = 2 * blockIdx.x;
  const int m = lane & 15, g = lane >> 4;
  const int inst = inst0 + (m >> 3), r = m & 7;
  const bool rv = inst < a.count;
  const int c = lane & 15;
  const int ksteps = (n + 63) >> 6;
  v4i acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  for (int s = wave; s < ksteps; s += 4) {
    const int k = s * 64 + 16 * g;
    uint32_t bw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t sw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (rv && k < n) {
      const uint8_t* p = a.ct + (size_t)inst * a.ct_stride + 2 * ((size_t)r * n + k);
      const uint4 v0 = *(const uint4*)p;
      bw[0] = v0.x; bw[1] = v0.y; bw[2] = v0.z; bw[3] = v0.w;
      if (k + 8 < n) {
        const uint4 v1 = *(const uint4*)(p + 16);
        bw[4] = v1.x; bw[5] = v1.y; bw[6] = v1.z; bw[7] = v1.w;
      }
    }
    if (c < 8 && k < n) {
      const uint8_t* p = a.St16 + 2 * ((size_t)c * n + k);
      const uint4 v0 = *(const uint4*)p;
      sw[0] = v0.x; sw[1] = v0.y; sw[2] = v0.z; sw[3] = v0.w;
      if (k + 8 < n) {
        const uint4 v1 = *(const uint4*)(p + 16);
        sw[4] = v1.x; sw[5] = v1.y; sw[6] = v1.z; sw[7] = v1.w;
      }
    }
    uint32_t xlo[4], xhi[4], y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      limbs4(bw[2 * q], bw[2 * q + 1], xlo[q], xhi[q]);
      y[q] = __builtin_amdgcn_perm(sw[2 * q + 1], sw[2 * q], 0x06040200u);  // int16 -> int8
    }
    const v4i yf = {(int)y[0], (int)y[1], (int)y[2], (int)y[3]};
    acc0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(v4i{(int)xlo[0], (int)xlo[1], (int)xlo[2], (int)xlo[3]},
                                                 yf, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(v4i{(int)xhi[0], (int)xhi[1], (int)xhi[2], (int)xhi[3]},
                                                 yf, acc1, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) red[wave][i][lane] = (uint32_t)acc0[i] + ((uint32_t)acc1[i] << 8);
  __syncthreads();
  if (wave == 0) {
    const uint32_t qmask = (1u << a.logq) - 1u;
    const int sh = a.logq - a.B;
    const uint32_t half = 1u << (sh - 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t D = red[0][i][lane] + red[1][i][lane] + red[2][i][lane] + red[3][i][lane];
      const int row = 4 * g + i;  // row within the 16-row tile
      const int ins = inst0 + (row >> 3), rr = row & 7;
      if (c < 8 && ins < a.count) {
        const uint16_t V =
            *(const uint16_t*)(a.ct + (size_t)ins * a.ct_stride + 2 * ((size_t)8 * n + rr * 8 + c));
        const uint32_t Mv = ((uint32_t)V - D) & qmask;
        dec[row][c] = (uint8_t)(((Mv + half) & qmask) >> sh);
      }
    }
  }
  __syncthreads();
  // assemble message bytes: bit p of the message is bit p % B of coefficient p / B
  const int mb = a.mu_bytes;
  if ((int)threadIdx.x < 2 * mb) {
    const int which = threadIdx.x / mb, byte = threadIdx.x % mb;
    const int ins = inst0 + which;
    if (ins < a.count) {
      uint32_t v = 0;
      for (int b = 0; b < 8; ++b) {
        const int p = 8 * byte + b, coeff = p / a.B, bit = p % a.B;
        v |= (uint32_t)((dec[which * 8 + coeff / 8][coeff % 8] >> bit) & 1u) << b;
      }
      a.mu_out[(size_t)ins * mb + byte] = (uint8_t)v;
    }
  }
}

// ======================================================================================
// SHA3-256 sponges.
// ======================================================================================
// Keccak-f[1600] on 32-bit halves: lane (x, y) is (hi[x + 5y], lo[x + 5y]).  Written with the
// gfx950 three-input bit operations: a 3-way XOR (LUT 0x96) and chi's a ^ (~b & c) (LUT 0xD2),
// and 64-bit rotations as two funnel shifts (v_alignbit).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t chi3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xD2);
}
// rotate the 64-bit value (hi, lo) left by r, 0 < r < 64, r != 32
__device__ __forceinline__ void rotl64_32(uint32_t hi, uint32_t lo, int r, uint32_t& oh, uint32_t& ol) {
  if (r < 32) {
    oh = __builtin_amdgcn_alignbit(hi, lo, 32 - r);
    ol = __builtin_amdgcn_alignbit(lo, hi, 32 - r);
  } else {
    oh = __builtin_amdgcn_alignbit(lo, hi, 64 - r);
    ol = __builtin_amdgcn_alignbit(hi, lo, 64 - r);
  }
}

__device__ __forceinline__ void keccak_f1600_dev(uint32_t lo[25], uint32_t hi[25]) {
#pragma unroll
  for (int round = 0; round < 24; ++round) {
    uint32_t cl[5], ch[5];
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      cl[x] = xor3(xor3(lo[x], lo[x + 5], lo[x + 10]), lo[x + 15], lo[x + 20]);
      ch[x] = xor3(xor3(hi[x], hi[x + 5], hi[x + 10]), hi[x + 15], hi[x + 20]);
    }
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      uint32_t rh, rl;
      rotl64_32(ch[(x + 1) % 5], cl[(x + 1) % 5], 1, rh, rl);
#pragma unroll
      for (int y = 0; y < 5; ++y) {
        lo[x + 5 * y] = xor3(lo[x + 5 * y], cl[(x + 4) % 5], rl);
        hi[x + 5 * y] = xor3(hi[x + 5 * y], ch[(x + 4) % 5], rh);
      }
    }
    uint32_t bl[25], bh[25];
#pragma unroll
    for (int x = 0; x < 5; ++x)
#pragma unroll
      for (int y = 0; y < 5; ++y) {
        const int r = keccak_rho(x + 5 * y), d = y + 5 * ((2 * x + 3 * y) % 5);
        if (r == 0) {
          bl[d] = lo[x + 5 * y];
          bh[d] = hi[x + 5 * y];
        } else {
          rotl64_32(hi[x + 5 * y], lo[x + 5 * y], r, bh[d], bl[d]);
        }
      }
#pragma unroll
    for (int y = 0; y < 5; ++y)
#pragma unroll
      for (int x = 0; x < 5; ++x) {
        lo[x + 5 * y] = chi3(bl[x + 5 * y], bl[(x + 1) % 5 + 5 * y], bl[(x + 2) % 5 + 5 * y]);
        hi[x + 5 * y] = chi3(bh[x + 5 * y], bh[(x + 1) % 5 + 5 * y], bh[(x + 2) % 5 + 5 * y]);
      }
    const uint64_t rc = keccak_rc(round);
    lo[0] ^= (uint32_t)rc;
    hi[0] ^= (uint32_t)(rc >> 32);
  }
}

// SHA3-256 (FIPS 202: rate 136 bytes, domain bits 01, pad10*1) of a message of compile-time
// length LEN < 136, i.e. one rate block: msg[] is indexed with constants only, so the block,
// the state and the digest stay in registers.  Returns the digest as eight little-endian words.
template <int LEN>
__device__ __forceinline__ void sha3_256_block(const uint8_t (&msg)[LEN], uint32_t d[8]) {
  static_assert(LEN < 136, "one rate block");
  uint32_t lo[25], hi[25];
#pragma unroll
  for (int w = 0; w < 25; ++w) lo[w] = hi[w] = 0;
  auto put = [&](int k, uint32_t v) __attribute__((always_inline)) {
    uint32_t& word = ((k >> 2) & 1) ? hi[k >> 3] : lo[k >> 3];
    word ^= v << (8 * (k & 3));
  };
#pragma unroll
  for (int k = 0; k < LEN; ++k) put(k, msg[k]);
  put(LEN, 0x06u);
  put(135, 0x80u);
  keccak_f1600_dev(lo, hi);
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    d[2 * w] = lo[w];
    d[2 * w + 1] = hi[w];
  }
}

// coins = H(0x01 || H(pk) || mu)[0:16] and K' = H(H(pk) || mu) for one instance per thread,
// for a message of MU bytes (each hash is a single rate block).  coins and kprime are the
// library's own aligned buffers.
template <int MU>
__global__ void __launch_bounds__(64) k_fo_coins_t(int count, const uint8_t* __restrict__ pkh,
                                                   const uint8_t* __restrict__ mu, size_t mu_stride,
                                                   uint8_t* coins, uint8_t* kprime) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint8_t m1[1 + 32 + MU], m2[32 + MU];
  m1[0] = 1;
#pragma unroll
  for (int k = 0; k < 32; ++k) m1[1 + k] = m2[k] = pkh[k];
  const uint8_t* mi = mu + (size_t)i * mu_stride;
#pragma unroll
  for (int k = 0; k < MU; ++k) m1[33 + k] = m2[32 + k] = mi[k];
  uint32_t d[8];
  sha3_256_block(m1, d);
  *(uint4*)(coins + (size_t)i * 16) = make_uint4(d[0], d[1], d[2], d[3]);
  sha3_256_block(m2, d);
  *(uint4*)(kprime + (size_t)i * 32) = make_uint4(d[0], d[1], d[2], d[3]);
  *(uint4*)(kprime + (size_t)i * 32 + 16) = make_uint4(d[4], d[5], d[6], d[7]);
}

// ---------------------------------------------------------------------------------------
// Two-lane bit-interleaved Keccak-f[1600].  A pair of adjacent lanes holds one state: lane
// parity 0 keeps the even bits of every 64-bit lane word, parity 1 the odd bits, each as a
// 32-bit word.  XOR, AND and chi act on the halves independently; a 64-bit rotation by
// 2k rotates both halves by k, and a rotation by 2k+1 swaps the halves between the two
// lanes (one DPP move) with rotations by k+1 (even half) and k (odd half).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t swap_pair(uint32_t v) {
  // quad_perm [1, 0, 3, 2]: exchange with the adjacent lane
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t rot32(uint32_t v, uint32_t s) { return __builtin_amdgcn_alignbit(v, v, s); }

// even / odd halves of the round constants
__device__ __forceinline__ uint32_t keccak_rc_half(int round, int parity) {
  constexpr uint32_t rce[24] = {0x00000001u, 0x00000000u, 0x00000000u, 0x00000000u, 0x00000001u, 0x00000001u,
                                0x00000001u, 0x00000001u, 0x00000000u, 0x00000000u, 0x00000001u, 0x00000000u,
                                0x00000001u, 0x00000001u, 0x00000001u, 0x00000001u, 0x00000000u, 0x00000000u,
                                0x00000000u, 0x00000000u, 0x00000001u, 0x00000000u, 0x00000001u, 0x00000000u};
  constexpr uint32_t rco[24] = {0x00000000u, 0x00000089u, 0x8000008bu, 0x80008080u, 0x0000008bu, 0x00008000u,
                                0x80008088u, 0x80000082u, 0x0000000bu, 0x0000000au, 0x00008082u, 0x00008003u,
                                0x0000808bu, 0x8000000bu, 0x8000008au, 0x80000081u, 0x80000081u, 0x80000008u,
                                0x00000083u, 0x80008003u, 0x80008088u, 0x80000088u, 0x00008000u, 0x80008082u};
  return parity ? rco[round] : rce[round];
}

__device__ __forceinline__ void keccak_f1600_pair(uint32_t s[25], uint32_t p) {
  // rotation of the partner's C[x+1] by 1 (even half) or 0.  Passed through a move the compiler
  // cannot see into: knowing it is 0 or 31, it would turn each variable rotation into a constant
  // one plus a select (two instructions instead of one).
  uint32_t sh1;
  asm volatile("v_mov_b32 %0, %1" : "=v"(sh1) : "v"(p ? 0u : 31u));
  // Twelve rounds per iteration: few register moves for pi at the back edge (its position
  // cycle has length 24), and a body small enough to stay within 128 registers.
#pragma unroll 12
  for (int round = 0; round < 24; ++round) {
    uint32_t c[5];
#pragma unroll
    for (int x = 0; x < 5; ++x) c[x] = xor3(xor3(s[x], s[x + 5], s[x + 10]), s[x + 15], s[x + 20]);
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      const uint32_t rc = rot32(swap_pair(c[(x + 1) % 5]), sh1);
#pragma unroll
      for (int y = 0; y < 5; ++y) s[x + 5 * y] = xor3(s[x + 5 * y], c[(x + 4) % 5], rc);
    }
    uint32_t b[25];
#pragma unroll
    for (int x = 0; x < 5; ++x)
#pragma unroll
      for (int y = 0; y < 5; ++y) {
        const int r = keccak_rho(x + 5 * y), d = y + 5 * ((2 * x + 3 * y) % 5);
        const uint32_t v = s[x + 5 * y];
        if ((r & 1) == 0) {
          const int kk = r >> 1;
          b[d] = kk ? rot32(v, (uint32_t)(32 - kk)) : v;
        } else {
          const int kk = r >> 1;  // even half rotates by kk + 1, odd half by kk
          b[d] = rot32(swap_pair(v), (uint32_t)(31 - kk) + p);
        }
      }
#pragma unroll
    for (int y = 0; y < 5; ++y)
#pragma unroll
      for (int x = 0; x < 5; ++x)
        s[x + 5 * y] = chi3(b[x + 5 * y], b[(x + 1) % 5 + 5 * y], b[(x + 2) % 5 + 5 * y]);
    s[0] ^= keccak_rc_half(round, (int)p);
  }
}

// bit_permute_step of the even/odd separation network
__device__ __forceinline__ uint32_t perm_step(uint32_t x, uint32_t m, int sh) {
  const uint32_t t = __builtin_amdgcn_bitop3_b32(x >> sh, x, m, 0x28);  // ((x >> sh) ^ x) & m
  return xor3(x, t, t << sh);
}
// 32-bit word -> even bits in the low half, odd bits in the high half
__device__ __forceinline__ uint32_t unshuffle32(uint32_t x) {
  x = perm_step(x, 0x22222222u, 1);
  x = perm_step(x, 0x0c0c0c0cu, 2);
  x = perm_step(x, 0x00f000f0u, 4);
  return perm_step(x, 0x0000ff00u, 8);
}
__device__ __forceinline__ uint32_t shuffle32(uint32_t x) {
  x = perm_step(x, 0x0000ff00u, 8);
  x = perm_step(x, 0x00f000f0u, 4);
  x = perm_step(x, 0x0c0c0c0cu, 2);
  return perm_step(x, 0x22222222u, 1);
}
// Lane p holds 32-bit half p of a 64-bit message word; returns its interleaved half.
__device__ __forceinline__ uint32_t interleave_in(uint32_t w, uint32_t sel) {
  const uint32_t u = unshuffle32(w);
  const uint32_t v = swap_pair(u);
  // parity 0: (u & 0xffff) | (v << 16); parity 1: (v >> 16) | (u & 0xffff0000)
  return __builtin_amdgcn_perm(sel ? u : v, sel ? v : u, sel ? 0x07060302u : 0x05040100u);
}

// SHA3-256 of count records of len bytes, one record per pair of lanes.  Full 136-byte
// blocks are read as 4-byte words (when aligned) and the next block is fetched while the
// current one is permuted; the final block and the padding are assembled byte by byte.
// Up to 256 VGPRs (two waves per SIMD): the build gives it 217 and no scratch.  A tighter
// limit (128, four waves per SIMD, to leave room beside other streams' product and sampler
// workgroups) spilled the state to scratch, 20 times the digests' bytes in writes per launch.
// ALIGNED: every record starts at a 4-byte boundary (whole-word loads).
template <bool ALIGNED>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_hash_records(int count, const uint8_t* __restrict__ in, size_t stride, size_t len, uint8_t* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t p = (uint32_t)(t & 1);
  const int rec_raw = t >> 1;
  const bool valid = rec_raw < count;
  const int rec = valid ? rec_raw : count - 1;  // idle pairs shadow the last record (no store)
  const uint8_t* base = in + (size_t)rec * stride;
  uint32_t s[25];
#pragma unroll
  for (int k = 0; k < 25; ++k) s[k] = 0;
  const size_t nfull = len / SHA3_RATE;  // full rate blocks; block nfull is the padded last one
  // Raw message words of block b for this lane (bytes 8w + 4p .. 8w + 4p + 3 of the block).
  // The last block carries the remaining bytes, the domain bits 01 and pad10*1; with aligned
  // records only the word holding the end of the message is assembled byte by byte.  No lane
  // exchange happens in here (the branches may differ between the lanes of a pair).
  auto load_block = [&](size_t b, uint32_t (&m)[17]) {
    const size_t off = b * SHA3_RATE;
    if (ALIGNED && b < nfull) {  // a full block: one base address, immediate offsets
      const uint32_t* q = (const uint32_t*)(base + off) + p;
#pragma unroll
      for (int w = 0; w < 17; ++w) m[w] = q[2 * w];
      return;
    }
    const bool last = b == nfull;
    const int rem = last ? (int)(len - off) : SHA3_RATE;
#pragma unroll
    for (int w = 0; w < 17; ++w) {
      const int pos0 = 8 * w + 4 * (int)p;
      uint32_t v = 0;
      if (ALIGNED && pos0 + 4 <= rem) {
        v = *(const uint32_t*)(base + off + pos0);
      } else if (pos0 < rem) {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
          if (pos0 + kb < rem) v |= (uint32_t)base[off + pos0 + kb] << (8 * kb);
      }
      if (last) {
        if (rem >= pos0 && rem < pos0 + 4) v ^= 0x06u << (8 * (rem - pos0));
        if (pos0 + 3 == SHA3_RATE - 1) v ^= 0x80u << 24;
      }
      m[w] = v;
    }
  };
  // One absorption loop (one inlined copy of the permutation); the next block is fetched
  // while the current one is permuted.
  uint32_t cur[17];
  load_block(0, cur);
  for (size_t b = 0; b <= nfull; ++b) {
    uint32_t nxt[17];
    if (b < nfull) {
      load_block(b + 1, nxt);
    } else {
#pragma unroll
      for (int w = 0; w < 17; ++w) nxt[w] = 0;
    }
#pragma unroll
    for (int w = 0; w < 17; ++w) s[w] ^= interleave_in(cur[w], p);
    keccak_f1600_pair(s, p);
#pragma unroll
    for (int w = 0; w < 17; ++w) cur[w] = nxt[w];
  }
  // digest: words 0..3 re-interleaved by the even lane
  uint32_t d[8];
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    // the exchange runs on every lane (a DPP read from a lane masked off by a branch would
    // not see the partner); only the selection depends on the parity
    const uint32_t sw = swap_pair(s[w]);
    const uint32_t e = p ? sw : s[w];
    const uint32_t o = p ? s[w] : sw;
    d[2 * w] = shuffle32((e & 0xffffu) | (o << 16));
    d[2 * w + 1] = shuffle32((e >> 16) | (o & 0xffff0000u));
  }
  if (!valid || p) return;
  uint8_t* dst = out + (size_t)rec * 32;
  if ((((uintptr_t)dst) & 15) == 0) {
    *(uint4*)dst = make_uint4(d[0], d[1], d[2], d[3]);
    *(uint4*)(dst + 16) = make_uint4(d[4], d[5], d[6], d[7]);
  } else {
#pragma unroll
    for (int kb = 0; kb < 32; ++kb) dst[kb] = (uint8_t)(d[kb / 4] >> (8 * (kb % 4)));
  }
}

// SHA3-256 of count records, one record per thread: the state as 25 (lo, hi) word pairs, no
// lane exchange and no bit interleaving.  About a fifth fewer instructions per record than the
// two-lane kernel, but a wave carries 64 records, so a launch is one chain 1.6 times as long:
// the layout for many independent streams in flight, where the chip's work matters more than
// one call's latency.
template <bool ALIGNED>
__global__ void __launch_bounds__(64) k_hash_records_one(int count, const uint8_t* __restrict__ in, size_t stride,
                                                      size_t len, uint8_t* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < count;
  const int rec = valid ? t : count - 1;
  const uint8_t* base = in + (size_t)rec * stride;
  uint32_t lo[25], hi[25];
#pragma unroll
  for (int k = 0; k < 25; ++k) lo[k] = hi[k] = 0;
  const size_t nfull = len / SHA3_RATE;
  auto load_block = [&](size_t b, uint32_t (&m)[34]) {
    const size_t off = b * SHA3_RATE;
    if (ALIGNED && b < nfull) {
      const uint32_t* q = (const uint32_t*)(base + off);
#pragma unroll
      for (int w = 0; w < 34; ++w) m[w] = q[w];
      return;
    }
    const bool last = b == nfull;
    const int rem = last ? (int)(len - off) : SHA3_RATE;
#pragma unroll
    for (int w = 0; w < 34; ++w) {
      const int pos0 = 4 * w;
      uint32_t v = 0;
      if (ALIGNED && pos0 + 4 <= rem) {
        v = *(const uint32_t*)(base + off + pos0);
      } else if (pos0 < rem) {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
          if (pos0 + kb < rem) v |= (uint32_t)base[off + pos0 + kb] << (8 * kb);
      }
      if (last) {
        if (rem >= pos0 && rem < pos0 + 4) v ^= 0x06u << (8 * (rem - pos0));
        if (pos0 + 3 == SHA3_RATE - 1) v ^= 0x80u << 24;
      }
      m[w] = v;
    }
  };
  uint32_t cur[34];
  load_block(0, cur);
  for (size_t b = 0; b <= nfull; ++b) {
    uint32_t nxt[34];
    if (b < nfull) {
      load_block(b + 1, nxt);
    } else {
#pragma unroll
      for (int w = 0; w < 34; ++w) nxt[w] = 0;
    }
#pragma unroll
    for (int w = 0; w < 17; ++w) {
      lo[w] ^= cur[2 * w];
      hi[w] ^= cur[2 * w + 1];
    }
    keccak_f1600_dev(lo, hi);
#pragma unroll
    for (int w = 0; w < 34; ++w) cur[w] = nxt[w];
  }
  if (!valid) return;
  uint8_t* dst = out + (size_t)rec * 32;
  const uint32_t d[8] = {lo[0], hi[0], lo[1], hi[1], lo[2], hi[2], lo[3], hi[3]};
  if ((((uintptr_t)dst) & 15) == 0) {
    *(uint4*)dst = make_uint4(d[0], d[1], d[2], d[3]);
    *(uint4*)(dst + 16) = make_uint4(d[4], d[5], d[6], d[7]);
  } else {
#pragma unroll
    for (int kb = 0; kb < 32; ++kb) dst[kb] = (uint8_t)(d[kb / 4] >> (8 * (kb % 4)));
  }
}

// ss = H(pre || H(ct)) with pre = K' (accepted) or z (rejected), selected without branches; the
// 64-byte message is one rate block kept in registers.  kprime and hct are the library's
// 16-byte aligned buffers; z and ss may be any byte address (SS_ALIGNED: ss is 16-byte aligned).
template <bool SS_ALIGNED>
__global__ void __launch_bounds__(64) k_final_ss_t(int count, const uint32_t* __restrict__ flags,
                                                   const uint8_t* __restrict__ kprime,
                                                   const uint8_t* __restrict__ z,
                                                   const uint8_t* __restrict__ hct, uint8_t* ss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint8_t rej = flags ? (uint8_t)(0u - (uint32_t)(flags[i] != 0)) : 0;
  uint8_t buf[64];
  const uint4 k0 = *(const uint4*)(kprime + (size_t)i * 32), k1 = *(const uint4*)(kprime + (size_t)i * 32 + 16);
  const uint4 h0 = *(const uint4*)(hct + (size_t)i * 32), h1 = *(const uint4*)(hct + (size_t)i * 32 + 16);
  const uint32_t kw[8] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
  const uint32_t hw[8] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w};
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const uint8_t zk = z ? z[k] : 0;
    const uint8_t kk = (uint8_t)(kw[k >> 2] >> (8 * (k & 3)));
    buf[k] = (uint8_t)((kk & (uint8_t)~rej) | (zk & rej));
    buf[32 + k] = (uint8_t)(hw[k >> 2] >> (8 * (k & 3)));
  }
  uint32_t d[8];
  sha3_256_block(buf, d);
  uint8_t* o = ss + (size_t)i * 32;
  if constexpr (SS_ALIGNED) {
    *(uint4*)o = make_uint4(d[0], d[1], d[2], d[3]);
    *(uint4*)(o + 16) = make_uint4(d[4], d[5], d[6], d[7]);
  } else {
#pragma unroll
    for (int k = 0; k < 32; ++k) o[k] = (uint8_t)(d[k >> 2] >> (8 * (k & 3)));
  }
}

// ======================================================================================
// Launchers
// ======================================================================================
static inline unsigned nblk(size_t work, unsigned threads) {
  return (unsigned)((work + threads - 1) / threads);
}

hipError_t launch_fill_u32(uint32_t* p, size_t count, uint32_t v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  unsigned blocks = nblk(count, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t launch_expand_keys(const uint8_t* keys, size_t key_stride, int count, const uint32_t* T0,
                              uint32_t* rk_out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand_keys, dim3(nblk(count, 64)), dim3(64), 0, s, keys, key_stride, count,
                     T0, rk_out);
  return hipGetLastError();
}

hipError_t launch_keystream(const uint32_t* rk, const uint32_t* T0, uint32_t domain, uint64_t block0,
                            size_t nblocks, uint8_t* out, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_keystream, dim3(nblk(nblocks, 256)), dim3(256), 0, s, rk, T0, bswap32(domain),
                     block0, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_expand_A(const Params& p, const uint32_t* rk, const uint32_t* T0, uint32_t col0,
                           uint32_t ncols, uint16_t* out, hipStream_t s) {
  const size_t bpc = (size_t)p.n / 8, nblocks = (size_t)ncols * bpc;
  if (nblocks == 0) return hipSuccess;
  const uint32_t qmask2 = ((1u << p.logq) - 1u) * 0x10001u;
  // two workgroups (64 KB of tables each) per CU at most
  const size_t units = (nblocks + 64 * EXPAND_ILP - 1) / (64 * EXPAND_ILP);
  const unsigned grid = (unsigned)std::min<size_t>((units + EXPAND_WAVES - 1) / EXPAND_WAVES, 2 * (size_t)g_num_cus);
  hipLaunchKernelGGL(k_expand_A, dim3(grid), dim3(64 * EXPAND_WAVES), 0, s, qmask2, rk, T0, (uint64_t)col0 * bpc,
                     nblocks, out);
  return hipGetLastError();
}

hipError_t launch_pack_x(const int8_t* src, int rows, int n, int ldx, int frag, int8_t* dst, hipStream_t s) {
  const size_t total = (size_t)rows * ldx;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_x, dim3(nblk(total, 256)), dim3(256), 0, s, src, rows, n, ldx, frag, dst);
  return hipGetLastError();
}

hipError_t launch_sample_stream(const Params& p, const uint32_t* rk, const uint32_t* T0, uint32_t domain,
                                uint64_t word0, size_t count, int16_t* out, hipStream_t s) {
  if (count == 0) return hipSuccess;
  SampTable st;
  for (int k = 0; k <= MAX_K; ++k) st.T[k] = p.T[k];
  hipLaunchKernelGGL(k_sample_stream, dim3(nblk(count, 256)), dim3(256), 0, s, st, p.K, rk, T0,
                     bswap32(domain), word0, count, out);
  return hipGetLastError();
}

hipError_t launch_sample(const SampleArgs& a, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  // persistent waves: at most two workgroups (64 KB of tables each) per CU
  const int p0 = a.x_frag ? 64 * ((a.n + 63) >> 6) : a.n;  // segment 0's slots, as in k_sample
  const int total = p0 + a.n + (a.nseg == 3 ? 8 : 0);
  const long long units = (long long)((total + 64 * SAMPLE_ILP - 1) / (64 * SAMPLE_ILP)) * count;
  const unsigned grid = (unsigned)std::min<long long>((units + SAMPLE_WAVES - 1) / SAMPLE_WAVES, 2 * g_num_cus);
  switch (a.K) {
    case 6: hipLaunchKernelGGL(k_sample<6>, dim3(grid), dim3(64 * SAMPLE_WAVES), 0, s, a, count); break;
    case 10: hipLaunchKernelGGL(k_sample<10>, dim3(grid), dim3(64 * SAMPLE_WAVES), 0, s, a, count); break;
    case 12: hipLaunchKernelGGL(k_sample<12>, dim3(grid), dim3(64 * SAMPLE_WAVES), 0, s, a, count); break;
    default: hipLaunchKernelGGL(k_sample<0>, dim3(grid), dim3(64 * SAMPLE_WAVES), 0, s, a, count); break;
  }
  return hipGetLastError();
}

// dynamic LDS limit of the streaming product (the 64 KB of replicated T-tables are static)
constexpr size_t STREAM_DYN_LDS = 160 * 1024 - TR_WORDS * 4;

template <int CG, int RG, bool TRANS>
static hipError_t launch_stream_t(const ProdArgs& a, int waves, int n_row_tiles, int ks, hipStream_t s) {
  // dynamic LDS only (the T-tables are static)
  const size_t lds = (size_t)waves * RG * CG * 256 * 4 + (TRANS ? (size_t)waves * 2 * CG * 1024 : 0);
  if (lds > STREAM_DYN_LDS) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(a.n_jt * a.n_kc), (unsigned)n_row_tiles);
  if (a.qp) {
    if (a.Amat) return hipErrorInvalidValue;  // the paper's sets regenerate A (fused) only
    hipLaunchKernelGGL((k_prod_stream<CG, RG, TRANS, false, true>), grid, dim3(64 * waves), lds, s, a, ks);
  } else if (a.Amat) {
    hipLaunchKernelGGL((k_prod_stream<CG, RG, TRANS, true>), grid, dim3(64 * waves), lds, s, a, ks);
  } else {
    hipLaunchKernelGGL((k_prod_stream<CG, RG, TRANS, false>), grid, dim3(64 * waves), lds, s, a, ks);
  }
  return hipGetLastError();
}

hipError_t launch_product_stream(const ProdArgs& a, int cg, int rg, int waves, bool trans, int n_row_tiles,
                                 int ks, hipStream_t s) {
#define LWE_STREAM_CASE(CG_, RG_)                                                  \
  if (cg == CG_ && rg == RG_)                                                      \
    return trans ? launch_stream_t<CG_, RG_, true>(a, waves, n_row_tiles, ks, s)   \
                 : launch_stream_t<CG_, RG_, false>(a, waves, n_row_tiles, ks, s);
  LWE_STREAM_CASE(1, 1)
  LWE_STREAM_CASE(1, 2)
  LWE_STREAM_CASE(1, 4)
#undef LWE_STREAM_CASE
  return hipErrorInvalidValue;
}

size_t product_strip_lds_bytes(int cg, int kc_len, int unr) {
  return 4096 + (size_t)strip_steps(kc_len, unr) * 64 * 16 * cg * 2;
}

// Loop unroll (X ring depth) of the strip kernel.  Deeper rings (unrolls of 4, 5 and 7, which
// avoid padding at n = 976, 640 and 1344) measured slower on MI355X: at n = 1344 x 4096 the
// (3, 2) tile took 220 us with a 7-deep ring against 204 us with a 3-deep one (more registers,
// no longer room for a hash wave beside the workgroup), so only three is built.
int product_strip_unroll(int, int, int) { return 3; }

template <int CG, int RG, int UNR>
static hipError_t launch_strip_t(const ProdArgs& a, hipStream_t s) {
  const size_t lds = product_strip_lds_bytes(CG, a.kc_len, UNR) - 4096;  // the strip alone
  // the table copies beside the strip when both fit, else inside the strip's space (which is
  // then at least 96 KB, more than the copies' 64 KB)
  const int tab = a.Amat ? 0 : lds + TR_WORDS * 4 <= 160 * 1024 ? 3 : 4;
  if (tab == 4 && lds < TR_WORDS * 4) return hipErrorInvalidValue;
  // compare mode reads the received ciphertexts instead of writing them
  const bool cmp = a.mode == PM_COMPARE;
  auto kern = tab == 0 ? (cmp ? k_prod_strip<CG, RG, true, UNR, 0> : k_prod_strip<CG, RG, false, UNR, 0>)
            : tab == 3 ? (cmp ? k_prod_strip<CG, RG, true, UNR, 3> : k_prod_strip<CG, RG, false, UNR, 3>)
                       : (cmp ? k_prod_strip<CG, RG, true, UNR, 4> : k_prod_strip<CG, RG, false, UNR, 4>);
  const int total = a.n_jt * a.n_kc * a.n_mt;
  const unsigned grid = (unsigned)(8 * ((total + 7) / 8));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * STRIP_WAVES), lds, s, a);
  return hipGetLastError();
}

// (CG, RG) shapes the library builds
#define LWE_STRIP_SHAPES(X) X(1, 2) X(1, 4) X(2, 2) X(2, 4) X(3, 2) X(3, 4)

bool product_strip_shape_ok(int cg, int rg) {
#define LWE_SHAPE_OK(CG_, RG_) if (cg == CG_ && rg == RG_) return true;
  LWE_STRIP_SHAPES(LWE_SHAPE_OK)
#undef LWE_SHAPE_OK
  return false;
}

hipError_t launch_product_strip(const ProdArgs& a, int cg, int rg, int unr, hipStream_t s) {
  if (unr != 3) return hipErrorInvalidValue;
#define LWE_STRIP_CASE(CG_, RG_) \
  if (cg == CG_ && rg == RG_) return launch_strip_t<CG_, RG_, 3>(a, s);
  LWE_STRIP_SHAPES(LWE_STRIP_CASE)
#undef LWE_STRIP_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_finalize(const ProdArgs& a, hipStream_t s) {
  const size_t total = (size_t)a.M * a.ncols;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(nblk(total, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_decrypt(const DecArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_decrypt, dim3((unsigned)((a.count + 1) / 2)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fo_coins(int count, const uint8_t* pkh, const uint8_t* mu, size_t mu_stride, int mu_bytes,
                           uint8_t* coins, uint8_t* kprime, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const dim3 g(nblk(count, 64)), b(64);
  switch (mu_bytes) {  // 8 B bytes for B message bits per coefficient
#define LWE_FO_CASE(MU_) \
  case MU_: hipLaunchKernelGGL(k_fo_coins_t<MU_>, g, b, 0, s, count, pkh, mu, mu_stride, coins, kprime); break;
    LWE_FO_CASE(8) LWE_FO_CASE(16) LWE_FO_CASE(24) LWE_FO_CASE(32) LWE_FO_CASE(40) LWE_FO_CASE(48) LWE_FO_CASE(56)
    LWE_FO_CASE(64)
#undef LWE_FO_CASE
    default:  // the registry allows 1 to 8 message bits per coefficient
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_hash_records(int count, const uint8_t* in, size_t stride, size_t len, uint8_t* out,
                               int lanes, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (lanes != 1 && lanes != 2) return hipErrorInvalidValue;
  const bool aligned = (((uintptr_t)in | stride) & 3) == 0;
  if (lanes == 1) {
    if (aligned)
      hipLaunchKernelGGL(k_hash_records_one<true>, dim3(nblk((size_t)count, 64)), dim3(64), 0, s, count, in, stride,
                         len, out);
    else
      hipLaunchKernelGGL(k_hash_records_one<false>, dim3(nblk((size_t)count, 64)), dim3(64), 0, s, count, in,
                         stride, len, out);
  } else if (aligned) {
    hipLaunchKernelGGL(k_hash_records<true>, dim3(nblk(2 * (size_t)count, 64)), dim3(64), 0, s, count, in, stride,
                       len, out);
  } else {
    hipLaunchKernelGGL(k_hash_records<false>, dim3(nblk(2 * (size_t)count, 64)), dim3(64), 0, s, count, in, stride,
                       len, out);
  }
  return hipGetLastError();
}

hipError_t launch_final_ss(int count, const uint32_t* flags, const uint8_t* kprime, const uint8_t* z,
                           const uint8_t* hct, uint8_t* ss, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if ((((uintptr_t)kprime | (uintptr_t)hct) & 15) != 0) return hipErrorInvalidValue;  // own buffers only
  if ((((uintptr_t)ss) & 15) == 0) {
    hipLaunchKernelGGL(k_final_ss_t<true>, dim3(nblk(count, 64)), dim3(64), 0, s, count, flags, kprime, z, hct, ss);
  } else {
    hipLaunchKernelGGL(k_final_ss_t<false>, dim3(nblk(count, 64)), dim3(64), 0, s, count, flags, kprime, z, hct, ss);
  }
  return hipGetLastError();
}

template <int CG, int RG, int UNR>
static hipError_t allow_lds_strip_u() {
  const void* kerns[6] = {(const void*)k_prod_strip<CG, RG, false, UNR, 0>,
                          (const void*)k_prod_strip<CG, RG, true, UNR, 0>,
                          (const void*)k_prod_strip<CG, RG, false, UNR, 3>,
                          (const void*)k_prod_strip<CG, RG, true, UNR, 3>,
                          (const void*)k_prod_strip<CG, RG, false, UNR, 4>,
                          (const void*)k_prod_strip<CG, RG, true, UNR, 4>};
  for (int i = 0; i < 6; ++i) {
    const int dyn = 160 * 1024 - (i == 2 || i == 3 ? TR_WORDS * 4 : 0);
    hipError_t e = hipFuncSetAttribute(kerns[i], hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
template <int CG, int RG, bool TR>
static hipError_t allow_lds_stream() {
  hipError_t e = hipFuncSetAttribute((const void*)k_prod_stream<CG, RG, TR, false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)STREAM_DYN_LDS);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_prod_stream<CG, RG, TR, false, true>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)STREAM_DYN_LDS);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_prod_stream<CG, RG, TR, true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)STREAM_DYN_LDS);
}

hipError_t init_kernels() {
  hipError_t e = hipSuccess, r;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      g_num_cus = cus;
  }
#define LWE_TRY(x) \
  if ((r = (x)) != hipSuccess) e = r;
#define LWE_ALLOW_STRIP(CG_, RG_) LWE_TRY((allow_lds_strip_u<CG_, RG_, 3>()))
  LWE_STRIP_SHAPES(LWE_ALLOW_STRIP)
#undef LWE_ALLOW_STRIP
  LWE_TRY((allow_lds_stream<1, 1, false>()))
  LWE_TRY((allow_lds_stream<1, 2, false>()))
  LWE_TRY((allow_lds_stream<1, 4, false>()))
  LWE_TRY((allow_lds_stream<1, 1, true>()))
  LWE_TRY((allow_lds_stream<1, 2, true>()))
  LWE_TRY((allow_lds_stream<1, 4, true>()))
#undef LWE_TRY
  return e;
}

}  // namespace lwe
