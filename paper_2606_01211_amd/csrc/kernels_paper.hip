// HIP kernels (gfx950) of the paper's own parameter sets (Table 1): one encryption per message
// bit, prime q.
//
//  * The noise source: an AES-256 CTR_DRBG without derivation function (SP 800-90A 10.2.1),
//    the generator the paper runs on the device (Sec. 3.3).  Generate requests are 2^19 bits
//    (4096 blocks) each, and every request ends with an Update that re-keys the generator, so
//    the chain of (Key, V) over the requests is sequential: k_drbg_chain walks it once per
//    (instance, stream), one thread each, and stores every request's expanded key and V;
//    k_pb_sample then computes all output blocks of all requests in parallel.
//  * The samplers of Alg. 1-2 with Table 1's distributions: centred binomial (eta) for s, the
//    discrete Gaussian of sigma through the 16-bit CDF table for e, r, e1, centred uniform on
//    [-k, k] for e2.
//  * v_r = t^T r_r + e2_r + m_r round(q/2) (Alg. 2) and the row sums of the secret operands
//    (the correction term of the product's offset limbs), one wave per row.
//  * Decryption (Alg. 3): mu_r = v_r - s^T u_r mod q, decoded by the q/4 and 3q/4 thresholds.
// The products u_r = A^T r_r + e1_r and t = A s + e run in the prime mode of the streaming
// product kernel (A regenerated from AES-128-CTR, int8 limbs on MFMA).
#include <algorithm>

#include "lwe_internal.h"

namespace lwe {
namespace {

__device__ __forceinline__ uint32_t rotl8x(uint32_t v, int r) { return (v << r) | (v >> (32 - r)); }

// T-tables T0..T3 (T0 rotated by 0, 8, 16, 24) and the S-box in LDS.
struct AesTables {
  uint32_t T[1024];
  uint8_t sbox[256];
};

__device__ __forceinline__ void load_aes_tables(AesTables& t, const uint32_t* __restrict__ T0) {
  for (int i = threadIdx.x; i < 256; i += blockDim.x) {
    const uint32_t v = T0[i];
    t.T[i] = v;
    t.T[256 + i] = rotl8x(v, 8);
    t.T[512 + i] = rotl8x(v, 16);
    t.T[768 + i] = rotl8x(v, 24);
    t.sbox[i] = (uint8_t)(v >> 8);
  }
}

// AES-256 key expansion (FIPS-197 Sec. 5.2, Nk = 8): key and round keys as little-endian
// words (word c of a block holds bytes 4c .. 4c+3).
__device__ void aes256_expand(const AesTables& t, const uint32_t key[8], uint32_t rk[60]) {
  for (int w = 0; w < 8; ++w) rk[w] = key[w];
  uint32_t rcon = 1;
  for (int w = 8; w < 60; ++w) {
    uint32_t x = rk[w - 1];
    if ((w & 7) == 0) {
      // RotWord then SubWord: bytes (b1, b2, b3, b0)
      x = (uint32_t)t.sbox[(x >> 8) & 0xff] | ((uint32_t)t.sbox[(x >> 16) & 0xff] << 8) |
          ((uint32_t)t.sbox[x >> 24] << 16) | ((uint32_t)t.sbox[x & 0xff] << 24);
      x ^= rcon;
      rcon = (rcon << 1) ^ ((rcon >> 7) * 0x11bu);
    } else if ((w & 7) == 4) {
      x = (uint32_t)t.sbox[x & 0xff] | ((uint32_t)t.sbox[(x >> 8) & 0xff] << 8) |
          ((uint32_t)t.sbox[(x >> 16) & 0xff] << 16) | ((uint32_t)t.sbox[x >> 24] << 24);
    }
    rk[w] = rk[w - 8] ^ x;
  }
}

// One AES-256 block: s[] in, o[] out, little-endian column words.
__device__ __forceinline__ void aes256_block(const uint32_t* __restrict__ T, const uint32_t* rk, const uint32_t s_in[4],
                                             uint32_t o[4]) {
  uint32_t s0 = s_in[0] ^ rk[0], s1 = s_in[1] ^ rk[1], s2 = s_in[2] ^ rk[2], s3 = s_in[3] ^ rk[3];
#pragma unroll
  for (int r = 1; r < 14; ++r) {
    const uint32_t t0 = T[s0 & 0xff] ^ T[256 + ((s1 >> 8) & 0xff)] ^ T[512 + ((s2 >> 16) & 0xff)] ^ T[768 + (s3 >> 24)] ^ rk[4 * r];
    const uint32_t t1 = T[s1 & 0xff] ^ T[256 + ((s2 >> 8) & 0xff)] ^ T[512 + ((s3 >> 16) & 0xff)] ^ T[768 + (s0 >> 24)] ^ rk[4 * r + 1];
    const uint32_t t2 = T[s2 & 0xff] ^ T[256 + ((s3 >> 8) & 0xff)] ^ T[512 + ((s0 >> 16) & 0xff)] ^ T[768 + (s1 >> 24)] ^ rk[4 * r + 2];
    const uint32_t t3 = T[s3 & 0xff] ^ T[256 + ((s0 >> 8) & 0xff)] ^ T[512 + ((s1 >> 16) & 0xff)] ^ T[768 + (s2 >> 24)] ^ rk[4 * r + 3];
    s0 = t0;
    s1 = t1;
    s2 = t2;
    s3 = t3;
  }
  // final round: S-box values are byte 0 of T2, byte 1 of T3, byte 2 of T0, byte 3 of T1
  auto fin = [&](uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t k) {
    return ((T[512 + (a & 0xff)] & 0xffu) | (T[768 + ((b >> 8) & 0xff)] & 0xff00u) |
            (T[(c >> 16) & 0xff] & 0xff0000u) | (T[256 + (d >> 24)] & 0xff000000u)) ^ k;
  };
  o[0] = fin(s0, s1, s2, s3, rk[56]);
  o[1] = fin(s1, s2, s3, s0, rk[57]);
  o[2] = fin(s2, s3, s0, s1, rk[58]);
  o[3] = fin(s3, s0, s1, s2, rk[59]);
}

__device__ __forceinline__ uint32_t bswap(uint32_t v) {
  return (v >> 24) | ((v >> 8) & 0xff00u) | ((v << 8) & 0xff0000u) | (v << 24);
}

// V as four big-endian 32-bit limbs (v[0] most significant); V + add (mod 2^128)
__device__ __forceinline__ void v_add(uint32_t v[4], uint32_t add) {
  uint64_t c = (uint64_t)v[3] + add;
  v[3] = (uint32_t)c;
  for (int k = 2; k >= 0; --k) {
    c = (uint64_t)v[k] + (c >> 32);
    v[k] = (uint32_t)c;
  }
}

// the AES input block of counter V as little-endian column words
__device__ __forceinline__ void v_block(const uint32_t v[4], uint32_t blk[4]) {
  for (int c = 0; c < 4; ++c) blk[c] = bswap(v[c]);
}

// CTR_DRBG_Update (SP 800-90A 10.2.1.2) with the key already expanded into rk: three blocks of
// V+1, V+2, V+3 XOR provided (12 words), then Key = words 0..7, V = bytes 32..47.
__device__ void drbg_update(const uint32_t* T, const uint32_t rk[60], const uint32_t provided[12], uint32_t key[8],
                            uint32_t v[4]) {
  uint32_t tmp[12];
  for (int b = 0; b < 3; ++b) {
    v_add(v, 1);
    uint32_t blk[4];
    v_block(v, blk);
    aes256_block(T, rk, blk, tmp + 4 * b);
  }
  for (int k = 0; k < 12; ++k) tmp[k] ^= provided[k];
  for (int k = 0; k < 8; ++k) key[k] = tmp[k];
  for (int c = 0; c < 4; ++c) v[c] = bswap(tmp[8 + c]);
}

}  // namespace

// ======================================================================================
// DRBG request chains.  Thread (inst, seg) instantiates the generator of (keys[inst],
// domains[seg]) -- entropy input key (16 bytes) || domain (4 bytes, little endian) || 28 zero
// bytes, no personalization -- and walks requests[seg] Generate requests of 4096 blocks,
// storing for request r its 60 round-key words and its V (4 big-endian limbs) at
// chain[((inst * nseg + seg) * rmax + r) * 64].
// ======================================================================================
__global__ void __launch_bounds__(64) k_drbg_chain(const uint8_t* __restrict__ keys, size_t key_stride, int count,
                                                   PbChainArgs a, const uint32_t* __restrict__ T0,
                                                   uint32_t* __restrict__ chain) {
  __shared__ AesTables tabs;
  load_aes_tables(tabs, T0);
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count * a.nseg) return;
  const int inst = t / a.nseg, seg = t - inst * a.nseg;
  uint32_t ent[12];
  const uint8_t* k16 = keys + (size_t)inst * key_stride;
  for (int w = 0; w < 4; ++w)
    ent[w] = (uint32_t)k16[4 * w] | ((uint32_t)k16[4 * w + 1] << 8) | ((uint32_t)k16[4 * w + 2] << 16) |
             ((uint32_t)k16[4 * w + 3] << 24);
  ent[4] = a.domain[seg];
  for (int w = 5; w < 12; ++w) ent[w] = 0;
  uint32_t key[8] = {0, 0, 0, 0, 0, 0, 0, 0}, v[4] = {0, 0, 0, 0}, rk[60];
  aes256_expand(tabs, key, rk);
  drbg_update(tabs.T, rk, ent, key, v);  // Instantiate
  const uint32_t zero[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  uint32_t* out = chain + ((size_t)(inst * a.nseg + seg) * a.rmax) * 64;
  for (int r = 0; r < a.requests[seg]; ++r) {
    aes256_expand(tabs, key, rk);
    for (int w = 0; w < 60; ++w) out[(size_t)r * 64 + w] = rk[w];
    for (int c = 0; c < 4; ++c) out[(size_t)r * 64 + 60 + c] = v[c];
    v_add(v, DRBG_REQ_BLOCKS);          // the request's output blocks use V+1 .. V+4096
    drbg_update(tabs.T, rk, zero, key, v);  // Update with no additional input
  }
}

// ======================================================================================
// Samplers.  Thread = one output block (8 noise words) of one segment of one instance:
// block b of a stream lies in request b / 4096 at counter V_r + 1 + (b mod 4096).  Word w of
// the segment goes to row w / rowlen, column w mod rowlen of its destination; 8 consecutive
// words share a row (rowlen is a multiple of 8), so each block is one 8-byte store.
// ======================================================================================
__device__ __forceinline__ int pb_sample_word(uint32_t u, int dist, const PbSampleArgs& a) {
  if (dist == 0) {  // centred binomial: bit count of the low eta bits minus the next eta
    const uint32_t m = (1u << a.eta) - 1u;
    return __popc(u & m) - __popc((u >> a.eta) & m);
  }
  if (dist == 1) {  // CDF table: |e| = #{k < K : (u >> 1) > T[k]}, sign = bit 0
    const uint32_t r = u >> 1;
    int e = 0;
    for (int k = 0; k < a.K; ++k) e += r > (uint32_t)a.T[k] ? 1 : 0;
    return (u & 1) ? -e : e;
  }
  return (int)((u * (uint32_t)(2 * a.ku + 1)) >> 16) - a.ku;  // centred uniform on [-ku, ku]
}

__global__ void __launch_bounds__(256) k_pb_sample(PbSampleArgs a, const uint32_t* __restrict__ T0,
                                                   const uint32_t* __restrict__ chain) {
  __shared__ uint32_t T[1024];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) {
    const uint32_t v = T0[i];
    T[i] = v;
    T[256 + i] = rotl8x(v, 8);
    T[512 + i] = rotl8x(v, 16);
    T[768 + i] = rotl8x(v, 24);
  }
  __syncthreads();
  const size_t per_inst = (size_t)a.blocks[0] + a.blocks[1] + a.blocks[2];
  const size_t total = per_inst * a.count;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int inst = (int)(t / per_inst);
    size_t b = t - (size_t)inst * per_inst;
    int seg = 0;
    while (seg < 2 && b >= (size_t)a.blocks[seg]) b -= a.blocks[seg++];
    const uint32_t r = (uint32_t)(b / DRBG_REQ_BLOCKS), i = (uint32_t)(b % DRBG_REQ_BLOCKS);
    const uint32_t* req = chain + ((size_t)(inst * a.nseg + seg) * a.rmax + r) * 64;
    uint32_t rk[60];
#pragma unroll
    for (int w = 0; w < 60; ++w) rk[w] = req[w];
    uint32_t v[4] = {req[60], req[61], req[62], req[63]};
    v_add(v, i + 1);
    uint32_t blk[4], o[4];
    v_block(v, blk);
    aes256_block(T, rk, blk, o);
    // words 8b .. 8b+7 of the segment: row, column of word 8b
    const size_t w0 = 8 * b;
    const size_t row = w0 / a.rowlen[seg], col = w0 - row * a.rowlen[seg];
    int smp[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) smp[k] = pb_sample_word((o[k >> 1] >> (16 * (k & 1))) & 0xffffu, a.dist[seg], a);
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lo |= (uint32_t)(uint8_t)(int8_t)smp[k] << (8 * k);
      hi |= (uint32_t)(uint8_t)(int8_t)smp[4 + k] << (8 * k);
    }
    int8_t* dst = a.dst8[seg] + (size_t)inst * a.inst_stride8[seg] + row * a.ld8[seg] + col;
    *(uint2*)dst = make_uint2(lo, hi);
    if (seg == 0 && a.dst16) {
      uint16_t* d16 = (uint16_t*)(a.dst16 + (size_t)inst * a.dst16_stride) + w0;
      *(uint4*)d16 = make_uint4(((uint32_t)(uint16_t)smp[0]) | ((uint32_t)(uint16_t)smp[1] << 16),
                                ((uint32_t)(uint16_t)smp[2]) | ((uint32_t)(uint16_t)smp[3] << 16),
                                ((uint32_t)(uint16_t)smp[4]) | ((uint32_t)(uint16_t)smp[5] << 16),
                                ((uint32_t)(uint16_t)smp[6]) | ((uint32_t)(uint16_t)smp[7] << 16));
    }
  }
}

// ======================================================================================
// Row sums of X (the offset-limb correction of the product) and, for encryption, v_r of
// every bit: one wave per row of X.
// ======================================================================================
__device__ __forceinline__ long long wave_sum64(long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    const int lo = __shfl_xor((int)(uint32_t)v, off), hi = __shfl_xor((int)(v >> 32), off);
    v += (long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
  }
  return v;
}

__global__ void __launch_bounds__(256) k_pb_rows(PbRowsArgs a) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= a.rows) return;
  const int8_t* x = a.X + (size_t)row * a.ldx;
  const int inst = row / a.rows_per_inst, r = row - inst * a.rows_per_inst;
  int sum = 0;
  long long dot = 0;
  for (int i = lane * 4; i < a.n; i += 256) {
    const uint32_t xw = *(const uint32_t*)(x + i);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int xv = (int)(int8_t)(xw >> (8 * k));
      sum += xv;
      if (a.mode) {
        const uint8_t* tp = a.t + (size_t)a.coef_bytes * (i + k);
        const uint32_t tv = a.coef_bytes == 4 ? *(const uint32_t*)tp : (uint32_t)*(const uint16_t*)tp;
        dot += (long long)xv * tv;
      }
    }
  }
  sum = (int)wave_sum64(sum);
  if (a.mode) dot = wave_sum64(dot);
  if (lane != 0) return;
  a.rowsum[row] = sum;
  if (!a.mode) return;
  const int bit = (a.mu[(size_t)inst * a.mu_stride + (r >> 3)] >> (r & 7)) & 1;
  const long long v = dot + a.e2[(size_t)inst * a.rows_per_inst + r] + (bit ? (long long)((a.q + 1) / 2) : 0);
  long long red = v % (long long)a.q;
  const uint32_t val = (uint32_t)(red < 0 ? red + a.q : red);
  const size_t off = a.v_off + (size_t)a.coef_bytes * r;
  if (a.mode == 2) {
    const uint8_t* src = a.cmp + (size_t)inst * a.cmp_stride + off;
    const uint32_t got = a.coef_bytes == 4 ? *(const uint32_t*)src : (uint32_t)*(const uint16_t*)src;
    if (got != val) atomicOr(&a.flags[inst], 1u);
  } else {
    uint8_t* dst = a.out + (size_t)inst * a.out_stride + off;
    if (a.coef_bytes == 4)
      *(uint32_t*)dst = val;
    else
      *(uint16_t*)dst = (uint16_t)val;
  }
}

// ======================================================================================
// Decryption (Alg. 3): mu_r = v_r - s^T u_r mod q; bit r = 0 when 4 mu_r <= q or
// 4 mu_r >= 3q, else 1.  A workgroup of 8 waves decodes the 8 bits of one message byte.
// ======================================================================================
__global__ void __launch_bounds__(512) k_pb_decrypt(PbDecArgs a) {
  __shared__ uint32_t bits[8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int inst = blockIdx.x / (PB_BITS / 8), byte = blockIdx.x % (PB_BITS / 8);
  const int r = 8 * byte + wave;
  const uint8_t* rec = a.ct + (size_t)inst * a.ct_stride;
  const uint8_t* u = rec + (size_t)a.coef_bytes * r * a.n;
  const int16_t* s = (const int16_t*)a.sk;
  long long dot = 0;
  for (int j = lane; j < a.n; j += 64) {
    const uint32_t uv = a.coef_bytes == 4 ? ((const uint32_t*)u)[j] : (uint32_t)((const uint16_t*)u)[j];
    dot += (long long)uv * s[j];
  }
  dot = wave_sum64(dot);
  if (lane == 0) {
    const uint8_t* vp = rec + (size_t)a.coef_bytes * ((size_t)PB_BITS * a.n + r);
    const uint32_t v = a.coef_bytes == 4 ? *(const uint32_t*)vp : (uint32_t)*(const uint16_t*)vp;
    long long m = ((long long)v - dot) % (long long)a.q;
    if (m < 0) m += a.q;
    const long long m4 = 4 * m;
    bits[wave] = (m4 <= (long long)a.q || m4 >= 3LL * a.q) ? 0u : 1u;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t b = 0;
    for (int k = 0; k < 8; ++k) b |= bits[k] << k;
    a.mu_out[(size_t)inst * (PB_BITS / 8) + byte] = (uint8_t)b;
  }
}

// ---- launchers ----
static inline unsigned nblocks_of(size_t work, unsigned threads) {
  return (unsigned)((work + threads - 1) / threads);
}

hipError_t launch_drbg_chain(const uint8_t* keys, size_t key_stride, int count, const PbChainArgs& a,
                             const uint32_t* T0, uint32_t* chain, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_drbg_chain, dim3(nblocks_of((size_t)count * a.nseg, 64)), dim3(64), 0, s, keys, key_stride,
                     count, a, T0, chain);
  return hipGetLastError();
}

hipError_t launch_pb_sample(const PbSampleArgs& a, const uint32_t* T0, const uint32_t* chain, hipStream_t s) {
  const size_t total = ((size_t)a.blocks[0] + a.blocks[1] + a.blocks[2]) * a.count;
  if (total == 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<size_t>(nblocks_of(total, 256), 65536);
  hipLaunchKernelGGL(k_pb_sample, dim3(grid), dim3(256), 0, s, a, T0, chain);
  return hipGetLastError();
}

hipError_t launch_pb_rows(const PbRowsArgs& a, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pb_rows, dim3(nblocks_of((size_t)a.rows, 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pb_decrypt(const PbDecArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pb_decrypt, dim3((unsigned)(a.count * (PB_BITS / 8))), dim3(512), 0, s, a);
  return hipGetLastError();
}

}  // namespace lwe
