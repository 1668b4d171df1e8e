// Internal declarations of liblwe_hip: parameter registry, kernel argument blocks and
// kernel launchers.  Not part of the public ABI (include/lwe.h is).
#pragma once

#include "../../include/lwe.h"
#include "lwe_common.h"

namespace lwe {

// ---- registry (params.cpp) ----
bool build_cdf(int K, double sigma, uint16_t* T);
void finish_params(Params& p);
const Params* get_params(int pid);
int find_param(uint32_t n);
int find_param_paper(uint32_t n);
int register_param(uint32_t n, uint32_t logq, uint32_t B, uint32_t K, double sigma);
const uint32_t* aes_T0();
const uint8_t* aes_sbox();

// ---- kernel argument blocks (kernels.hip) ----
enum ProdMode : int { PM_KEYGEN = 0, PM_ENCRYPT = 1, PM_COMPARE = 2 };

// Product D = X * Y over the contraction index k, where X is an int8 matrix with M rows
// (S^T stacks for keygen, S' stacks for encryption) and Y is A (encryption) or A^T
// (keygen) regenerated from AES-128-CTR, extended for encryption by the 8 columns of
// B = (B^T)^T so that V = S' B is computed by the same contraction.
// Byte offset of S' element (row, k) in MFMA fragment order, the layout the strip product
// reads: 16-row groups, then 64-column contraction steps, then the 64 lanes of the operand
// fragment (lane = row % 16 + 16 * (k % 64 / 16)), 16 bytes each.  steps = ldx / 64.
LWE_HD size_t frag_offset(int row, int k, int steps) {
  const int lane = (row & 15) | (((k & 63) >> 4) << 4);
  return (((size_t)(row >> 4) * steps + (k >> 6)) * 64 + lane) * 16 + (k & 15);
}

struct ProdArgs {
  const uint32_t* rkA;   // round keys of seedA: 44 words, or [inst][44] if per_inst_A
  const uint32_t* T0;    // AES T-table (256 words, global)
  const int8_t* X;       // [M][ldx] int8, zero padded beyond n; the strip product reads it in
                         // fragment order (frag_offset), rows rounded up to 16
  int ldx;
  int M;                 // valid rows (8 per instance)
  int n, logq, B;
  int ncols;             // n (keygen) or n + 8 (encryption: A | B)
  const uint8_t* Bt;     // encryption: B^T (8 x n uint16) of the shared public key
  int kc_len;            // contraction rows per K chunk (multiple of 64)
  int n_kc;              // number of K chunks; > 1 accumulates partials into acc32
  int n_jt;              // column tiles
  int m_tile;            // rows per row tile (multiple of 16)
  int n_mt;              // row tiles
  int per_inst_A;        // keygen batches: every instance has its own A (row tile = instance)
  int32_t* acc32;        // split-K accumulator [M][acc_ld], zeroed before the launch
  int acc_ld;
  int mode;              // ProdMode
  const int8_t* E;       // keygen E^T / encryption E': [M][n] int8
  const int8_t* E2;      // encryption E'': [count][64] int8
  const uint8_t* mu;     // encryption messages [count][mu_stride]
  size_t mu_stride;
  uint8_t* out;          // keygen: pk records, encryption: ct records
  size_t out_stride, out_off;
  const uint8_t* cmp;    // compare: received ct records
  size_t cmp_stride;
  uint32_t* flags;       // compare: per instance, nonzero if any coefficient differs
  // Unfused variant: A already expanded into device memory, column-major [n][n] uint16
  // (A[i][j] at Amat[j * n + i], masked to logq bits); null when the product regenerates A.
  const uint16_t* Amat;
  // The paper's sets (prime q; qp == 0 for the power-of-two sets).  A[i][j] = word mod qp, split
  // into offset limbs x = (lo - 128) + 256 (hi - 128) + 32896 with lo, hi the bytes of x, so
  // the epilogue adds 32896 * rowsum[row] (the row sums of X) and reduces mod qp exactly.
  uint32_t qp;
  uint32_t qp_magic;     // floor(2^32 / qp) + 1 for qp < 2^16 (16-bit words reduced), else 0
  const int32_t* rowsum; // [M]
  int rows_per_inst;     // output rows per instance (nbar for keygen, mbar for encryption)
  int coef_bytes;        // bytes per stored coefficient
};

struct SampleArgs {
  const uint32_t* rk;    // [count][44]
  const uint32_t* T0;
  int n, K, ldx;
  int nseg;              // 2 (keygen: S^T, E^T) or 3 (encryption: S', E', E'')
  uint32_t T2[MAX_K];    // CDF entries T[0..K-1], each replicated in both 16-bit halves
  int8_t* X;             // segment 0 (domain 1): [count*8][ldx] row-major, or in MFMA fragment
                         // order when x_frag is set (see frag_offset)
  int x_frag;
  uint8_t* X16;          // optional int16 copy of segment 0 (secret key bytes), may be null
  size_t x16_stride;
  int8_t* E;             // segment 1 (domain 2): [count*8][n]
  int8_t* E2;            // segment 2 (domain 3): [count][64]
};

struct DecArgs {
  const uint8_t* ct;     // [count][ct_stride]
  size_t ct_stride;
  const uint8_t* St16;   // S^T int16 (8 x n), shared
  int n, logq, B, count;
  int mu_bytes;
  uint8_t* mu_out;       // [count][mu_bytes]
};

// ---- the paper's sets (kernels_paper.hip) ----
struct PbChainArgs {
  int nseg, rmax;         // noise streams per instance; request slots per stream in `chain`
  uint32_t domain[3];     // domain number of each stream
  int requests[3];        // Generate requests (4096 blocks each) per stream
};

struct PbSampleArgs {
  int count, nseg, rmax;
  uint32_t blocks[3];     // output blocks (8 words) per stream and instance
  int dist[3];            // 0 binomial(eta), 1 CDF table, 2 uniform on [-ku, ku]
  int rowlen[3];          // words per destination row (a multiple of 8)
  int8_t* dst8[3];        // destination of stream s: instance i, row r, column c at
  size_t inst_stride8[3]; //   dst8[s] + i * inst_stride8[s] + r * ld8[s] + c
  int ld8[3];
  uint8_t* dst16;         // optional int16 copy of stream 0 (sk records), may be null
  size_t dst16_stride;
  int eta, ku, K;
  uint16_t T[MAX_K + 1];  // CDF table
};

struct PbRowsArgs {
  const int8_t* X;        // [rows][ldx]
  int ldx, n, rows, rows_per_inst;
  int32_t* rowsum;        // [rows]
  int mode;               // 0 row sums only; 1 and v_r stored; 2 and v_r compared
  const uint8_t* t;       // t coefficients of the public key (coef_bytes each)
  int coef_bytes;
  const int8_t* e2;       // [count][rows_per_inst]
  const uint8_t* mu;      // [count][mu_stride]
  size_t mu_stride;
  uint32_t q;
  uint8_t* out;           // ct records: v_r at out + inst * out_stride + v_off + r * coef_bytes
  size_t out_stride, v_off;
  const uint8_t* cmp;     // compare mode: received ct records
  size_t cmp_stride;
  uint32_t* flags;        // compare mode: per instance, nonzero if any coefficient differs
};

struct PbDecArgs {
  const uint8_t* ct;      // [count][ct_stride]: u_0..u_255 then v
  size_t ct_stride;
  const uint8_t* sk;      // s as n int16 at the start of the secret key
  int n;
  uint32_t q;
  int coef_bytes, count;
  uint8_t* mu_out;        // [count][32]
};

hipError_t launch_drbg_chain(const uint8_t* keys, size_t key_stride, int count, const PbChainArgs& a,
                             const uint32_t* T0, uint32_t* chain, hipStream_t s);
hipError_t launch_pb_sample(const PbSampleArgs& a, const uint32_t* T0, const uint32_t* chain, hipStream_t s);
hipError_t launch_pb_rows(const PbRowsArgs& a, hipStream_t s);
hipError_t launch_pb_decrypt(const PbDecArgs& a, hipStream_t s);

// ---- launchers (kernels.hip); all return hipError_t of the launch ----
hipError_t launch_fill_u32(uint32_t* p, size_t count, uint32_t v, hipStream_t s);
hipError_t launch_expand_keys(const uint8_t* keys, size_t key_stride, int count,
                              const uint32_t* T0, uint32_t* rk_out, hipStream_t s);
hipError_t launch_keystream(const uint32_t* rk, const uint32_t* T0, uint32_t domain,
                            uint64_t block0, size_t nblocks, uint8_t* out, hipStream_t s);
hipError_t launch_expand_A(const Params& p, const uint32_t* rk, const uint32_t* T0,
                           uint32_t col0, uint32_t ncols, uint16_t* out, hipStream_t s);
hipError_t launch_sample_stream(const Params& p, const uint32_t* rk, const uint32_t* T0,
                                uint32_t domain, uint64_t word0, size_t count, int16_t* out,
                                hipStream_t s);
hipError_t launch_sample(const SampleArgs& a, int count, hipStream_t s);
hipError_t launch_pack_x(const int8_t* src, int rows, int n, int ldx, int frag, int8_t* dst, hipStream_t s);
hipError_t launch_product_stream(const ProdArgs& a, int cg, int rg, int waves, bool trans,
                                 int n_row_tiles, int ksteps_per_wave, hipStream_t s);
hipError_t launch_product_strip(const ProdArgs& a, int cg, int rg, int unr, hipStream_t s);
size_t product_strip_lds_bytes(int cg, int kc_len, int unr);
int product_strip_unroll(int cg, int rg, int kc_len);
bool product_strip_shape_ok(int cg, int rg);
// 64-deep contraction steps of a strip over kc_len rows, padded to the kernel's unroll.
LWE_HD int strip_steps(int kc_len, int unr) { return ((kc_len + 63) / 64 + unr - 1) / unr * unr; }
hipError_t launch_finalize(const ProdArgs& a, hipStream_t s);
hipError_t launch_decrypt(const DecArgs& a, hipStream_t s);
hipError_t launch_fo_coins(int count, const uint8_t* pkh, const uint8_t* mu, size_t mu_stride,
                           int mu_bytes, uint8_t* coins, uint8_t* kprime, hipStream_t s);
// lanes: 2 = two lanes per record (k_hash_records), 1 = one record per thread
hipError_t launch_hash_records(int count, const uint8_t* in, size_t stride, size_t len,
                               uint8_t* out, int lanes, hipStream_t s);
hipError_t launch_final_ss(int count, const uint32_t* flags, const uint8_t* kprime,
                           const uint8_t* z, const uint8_t* hct, uint8_t* ss, hipStream_t s);
hipError_t init_kernels();

}  // namespace lwe
