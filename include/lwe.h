/*
 * lwe.h -- C ABI of the MI355X plain-LWE KEM library (liblwe_hip.so).
 *
 * The scheme is the plain-LWE key encapsulation mechanism of Liberati et al.,
 * "GPU Acceleration of Learning With Errors KEMs Using OpenACC for Post-Quantum
 * Cryptography": the LWE relation b = A s + e mod q (Sec. 2.1, eq. (1)), the PKE
 * algorithms KeyGen / Encrypt / Decrypt (Alg. 1-3) and the KEM Encaps / Decaps built on
 * them with the Fujisaki-Okamoto transform and implicit rejection (Alg. 4-5, Sec. 2.1).
 * It is used here in matrix form with nbar = mbar = 8 and q = 2^logq:
 *
 *   KeyGen (Alg. 1)  A = AES-128-CTR(seedA) (n x n, never stored; regenerated on demand
 *                    as in Sec. 3.5), S^T, E^T from a 16-bit CDF table (seedSK),
 *                    B^T = S^T A^T + E^T mod q
 *   Encrypt (Alg. 2) S', E', E'' from the CDF table (coins),
 *                    B' = S' A + E' mod q,  V = S' B + E'' + encode(mu) mod q
 *   Decrypt (Alg. 3) M = V - B' S mod q,  mu = decode(M)
 *   Encaps (Alg. 4)  coins = H(0x01 || H(pk) || mu)[0:16], K' = H(H(pk) || mu),
 *                    ct = Encrypt(pk, mu; coins), K = H(K' || H(ct))
 *   Decaps (Alg. 5)  mu' = Decrypt(sk, ct), re-encrypt, K = H(K'' || H(ct)) if the
 *                    ciphertexts agree else H(z || H(ct)), in constant time.
 *   H = SHA3-256.
 *
 * Byte formats (all integers little-endian, no bit packing):
 *   pk = seedA[16] || B^T (8 x n uint16)
 *   sk = S^T (8 x n int16) || pk || H(pk)[32] || z[32]
 *   ct = B' (8 x n uint16, row major) || V (8 x 8 uint16)
 *   mu = 64*B bits (B bits per coefficient), ss = 32 bytes.
 *
 * Conventions for every entry point:
 *   - Buffers may be host or device memory (detected per pointer); device buffers must be
 *     on the context's device.  All buffers are owned by the caller; the library keeps no
 *     reference after the call returns.
 *   - hip_stream == NULL runs the call synchronously on the context's own stream.  Otherwise
 *     device work is queued on that stream (a hipStream_t).  Calls whose outputs include
 *     host memory synchronise the stream before returning, and so do Encaps and Decaps of
 *     batches up to the host-hashing size (16 unless tuned: lwe_tuning.host_hash_max), which
 *     hash on the host between device phases.  Every other call on device buffers returns
 *     once its work is queued: KeyGen's public-key hashes and Encaps' H(pk) are computed on
 *     the host by functions queued on the stream (hipLaunchHostFunc), in stream order, so
 *     such calls can also be captured into a HIP graph and replayed.  A captured graph uses
 *     the context's working buffers as they were at capture: replay it only while no call
 *     on that context needs larger ones (a larger batch or set grows, and so moves, them),
 *     and not after lwe_ctx_trim.  Device outputs are valid once the stream has been
 *     synchronised.
 *   - The return value is an lwe_status.  On error, outputs are unspecified.
 *   - A context is not thread-safe: use one context per host thread.  Calls on one context
 *     execute on the device in the order they are made, whatever streams they are given: a
 *     call on a stream other than the previous call's first waits (hipStreamWaitEvent) for
 *     the previous call's work, because calls reuse the context's device buffers.
 *   - Decaps of a malformed or tampered ciphertext is NOT an error: it returns LWE_OK and
 *     the implicit-rejection key H(z || H(ct)).
 */
#ifndef LWE_H
#define LWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lwe_ctx lwe_ctx;

typedef enum {
  LWE_OK = 0,
  LWE_EINVAL = -1,       /* bad argument: unknown parameter id, NULL pointer, bad size */
  LWE_ENOMEM = -2,       /* device allocation failed or would exceed the context budget */
  LWE_EDEVICE = -3,      /* a HIP runtime call failed */
  LWE_EUNSUPPORTED = -4  /* valid request that the library does not implement */
} lwe_status;

/* Parameter set description.  Two families:
 *  - matrix form (paper == 0; lwe_param_id): nbar = mbar = 8, q = 2^logq, B message bits
 *    per coefficient, every secret and error from the 16-bit CDF table, noise from
 *    AES-128-CTR;
 *  - the paper's own sets (paper == 1; lwe_param_id_paper), Table 1: one encryption per
 *    message bit (nbar = 1, mbar = 256, B = 1; Sec. 2.3, 3.2), prime q, s from the centred
 *    binomial distribution (eta), e / r / e1 from the CDF table of sigma, e2 uniform on
 *    [-k, k], all noise from an AES-256 CTR_DRBG (Sec. 3.3), decoding by Alg. 3's
 *    thresholds q/4 and 3q/4.  Coefficients are serialised in coef_bytes bytes. */
typedef struct {
  uint32_t n;      /* lattice dimension (multiple of 8) */
  uint32_t logq;   /* matrix form: q = 2^logq, 2 < logq <= 16; paper sets: bits of q */
  uint32_t B;      /* message bits per coefficient (mbar*nbar*B-bit messages) */
  uint32_t K;      /* error support [-K, K] of the CDF table */
  double sigma;    /* width of the discrete Gaussian the 16-bit CDF table approximates */
  size_t pk_bytes, sk_bytes, ct_bytes, mu_bytes;
  uint32_t paper;  /* 0 matrix form, 1 the paper's own set */
  uint32_t q;      /* modulus */
  uint32_t nbar, mbar, coef_bytes;
  uint32_t eta, k; /* paper sets: binomial parameter of s, bound of e2 (0 otherwise) */
} lwe_param_info;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the device memory the
 * context may hold, lwe_ctx_device_bytes (0 = no limit; otherwise at least 1024, the AES
 * table every context keeps); requests that need more fail with LWE_ENOMEM.  Returns
 * LWE_EDEVICE if the device cannot be used. */
int lwe_ctx_create(lwe_ctx** out, int device, size_t hbm_budget_bytes);
void lwe_ctx_destroy(lwe_ctx* ctx);
/* Device memory currently held by the context, in bytes: its 1 KB AES table plus the
 * working buffers, which grow to the largest request seen and are kept for reuse. */
size_t lwe_ctx_device_bytes(const lwe_ctx* ctx);
/* Changes the budget of lwe_ctx_create for later calls (0 = no limit, else >= 1024).  Memory
 * already held is not released (see lwe_ctx_trim).  LWE_EINVAL for a NULL context or a
 * budget below 1024. */
int lwe_ctx_set_budget(lwe_ctx* ctx, size_t hbm_budget_bytes);
/* Releases every working buffer of the context (lwe_ctx_device_bytes drops to 1024).  The
 * release is ordered after the context's queued work; later calls allocate again. */
int lwe_ctx_trim(lwe_ctx* ctx);
/* Device bytes (lwe_ctx_device_bytes) that one call of `op` (0 KeyGen, 1 Encaps, 2 Decaps,
 * batched or not) on `count` instances of set pid holds at most when made on a freshly
 * trimmed context with the context's tuning, host or device buffers alike: the admission
 * figure of a server that bounds device memory.  0 for invalid arguments. */
size_t lwe_ctx_call_bytes(lwe_ctx* ctx, int pid, int op, size_t count);
/* The context's own HIP stream (a hipStream_t; owned by the context, valid until
 * lwe_ctx_destroy).  Calls given a NULL stream run on it and return once it has finished;
 * a caller may also pass it explicitly to run asynchronously, so that each context's work
 * uses only the context's streams (this one and, see lwe_ctx_set_side_stream, the internal
 * one that overlaps the decapsulation hash), which keeps HIP's stream-to-hardware-queue
 * mapping predictable when several contexts run concurrently.  NULL for a NULL context. */
void* lwe_ctx_stream(lwe_ctx* ctx);
/* Whether lwe_decaps_batch hashes the received ciphertexts (the H(ct) of the FO transform,
 * Alg. 5) on the context's second stream, concurrently with the decryption and
 * re-encryption (enable = 1, the default), or first on the call's own stream (0).  The
 * second stream shortens one call; with 0 a context uses a single stream, and so a single
 * HIP hardware queue, which lets more contexts run concurrently before queues are shared.
 * The second stream is created by the first call that needs it.  Results are identical
 * either way.  Returns LWE_EINVAL for a NULL context or an enable other than 0 or 1. */
int lwe_ctx_set_side_stream(lwe_ctx* ctx, int enable);
/* Layout of the batched SHA3-256 (FIPS 202) hashing of records in KeyGen, Encaps and Decaps
 * (H(pk), H(ct) of the FO transform, Alg. 4-5): lanes = 2 (the default) hashes each record on
 * two lanes, each holding one bit-interleaved half of the state, which halves one call's hash
 * latency; lanes = 1 hashes one record per thread, about a fifth less work per record at 1.6
 * times the latency, which suits many contexts running at once.  Digests are identical either
 * way.  Returns LWE_EINVAL for a NULL context or lanes other than 1 or 2. */
int lwe_ctx_set_hash_lanes(lwe_ctx* ctx, int lanes);
const char* lwe_strerror(int status);

/* Parameter registry: id of the matrix-form set for lattice dimension n, or a negative
 * lwe_status. */
int lwe_param_id(uint32_t n);
/* Id of the paper's own set for n (Table 1: n = 512, 1024, 2048, 4096, 8192, 16384, 32768),
 * or a negative lwe_status.  Every KEM entry point (and lwe_ctx_call_bytes) accepts these
 * ids; the test hooks and lwe_decaps_batch_noalloc take matrix-form ids only
 * (LWE_EUNSUPPORTED otherwise). */
int lwe_param_id_paper(uint32_t n);
/* Registers an additional parameter set (for experiments and tests; not security-vetted).
 * Requires n % 8 == 0, 8 <= n <= 32768, 3 <= logq <= 16, 1 <= B <= 8 with B < logq,
 * 1 <= K <= 15, sigma > 0, and a strictly increasing CDF table.  Returns the new id,
 * or the id of an identical existing set, or a negative lwe_status. */
int lwe_param_register(uint32_t n, uint32_t logq, uint32_t B, uint32_t K, double sigma);
int lwe_param_get(int pid, lwe_param_info* out);
size_t lwe_pk_bytes(int pid);
size_t lwe_sk_bytes(int pid);
size_t lwe_ct_bytes(int pid);
size_t lwe_mu_bytes(int pid); /* shared secrets are always 32 bytes */
/* The 16-bit CDF table of set pid: T[0..K] (K+1 entries) copied to host memory. */
int lwe_cdf_table(int pid, uint16_t* T_out, size_t capacity);

/* ---- KEM, derandomised: outputs are deterministic functions of the inputs ---- */

/* KeyGen (Alg. 1) with explicit seeds.  seedA[16], seedSK[16], z[32]; pk/sk sized per pid. */
int lwe_keygen(lwe_ctx* ctx, int pid, const uint8_t* seedA, const uint8_t* seedSK,
               const uint8_t* z, uint8_t* pk, uint8_t* sk, void* hip_stream);
/* Encaps (Alg. 4) with explicit message mu (lwe_mu_bytes(pid) bytes). */
int lwe_encaps(lwe_ctx* ctx, int pid, const uint8_t* pk, const uint8_t* mu, uint8_t* ct,
               uint8_t* ss, void* hip_stream);
/* Decaps (Alg. 5), constant time with implicit rejection. */
int lwe_decaps(lwe_ctx* ctx, int pid, const uint8_t* sk, const uint8_t* ct, uint8_t* ss,
               void* hip_stream);

/* ---- randomised: seeds and messages drawn from the operating system (getrandom(2)) ----
 * KeyGen draws seedA, seedSK (16 bytes each) and z (32 bytes) per instance (Alg. 1 takes a
 * fresh seed); Encaps draws the message mu (Alg. 4 starts by sampling mu uniformly).  The
 * outputs are then those of lwe_keygen_batch / lwe_encaps_batch for the drawn inputs; the
 * host copies of the drawn bytes are overwritten before the call returns.  count == 0 is a
 * no-op; 1 <= count <= 65535.  LWE_EDEVICE if the random source fails. */
int lwe_keygen_rand(lwe_ctx* ctx, int pid, size_t count, uint8_t* pk, uint8_t* sk, void* hip_stream);
int lwe_encaps_rand(lwe_ctx* ctx, int pid, size_t count, const uint8_t* pk, uint8_t* ct, uint8_t* ss,
                    void* hip_stream);

/* ---- batched variants: `count` independent instances, arrays are [count][bytes] ----
 * Each instance's output is identical to what the single-instance call returns for the
 * same inputs.  encaps/decaps batches share one pk / one sk; keygen batches take count
 * seed triples.  1 <= count <= 65535 (count == 0 is a no-op returning LWE_OK). */
int lwe_keygen_batch(lwe_ctx* ctx, int pid, size_t count, const uint8_t* seedA,
                     const uint8_t* seedSK, const uint8_t* z, uint8_t* pk, uint8_t* sk,
                     void* hip_stream);
int lwe_encaps_batch(lwe_ctx* ctx, int pid, size_t count, const uint8_t* pk, const uint8_t* mu,
                     uint8_t* ct, uint8_t* ss, void* hip_stream);
int lwe_decaps_batch(lwe_ctx* ctx, int pid, size_t count, const uint8_t* sk, const uint8_t* ct,
                     uint8_t* ss, void* hip_stream);

/* ---- test hooks (stable names, unstable semantics; for parity tests only) ---- */

/* Columns col0 .. col0+ncols-1 of A for seedA: out[c*n + i] = A[i][col0 + c] (uint16),
 * generated by the same device code the products use (Alg. 1, sample(rho)). */
int lwe_test_expand_A(lwe_ctx* ctx, int pid, const uint8_t* seedA, uint32_t col0,
                      uint32_t ncols, uint16_t* out, void* hip_stream);
/* Raw AES-128-CTR keystream: nblocks 16-byte blocks of domain `domain` from block0. */
int lwe_test_keystream(lwe_ctx* ctx, const uint8_t* key, uint32_t domain, uint64_t block0,
                       size_t nblocks, uint8_t* out, void* hip_stream);
/* count samples of the CDF sampler of set pid from keystream words word0.. of (key, domain),
 * as int16. */
int lwe_test_sample(lwe_ctx* ctx, int pid, const uint8_t* key, uint32_t domain, uint64_t word0,
                    size_t count, int16_t* out, void* hip_stream);
/* The batched sampler kernel of KeyGen (mode 0: S^T from domain 1, E^T from domain 2) or of
 * Encrypt (mode 1: S' from domain 1, E' from domain 2, E'' from domain 3), Alg. 1-2, for
 * count instances whose AES-128 keys are keys[count][16] (seedSK or coins).  Outputs, with
 * ldx = n rounded up to a multiple of 64:
 *   X_out  the int8 operand matrix of segment 0 as the products read it: layout 0 is
 *          row-major [count*8][ldx]; layout 1 is MFMA fragment order over
 *          ceil(count*8/16)*16 rows (16-row groups, then 64-column steps, then 64 lanes of 16
 *          bytes; lane = row % 16 + 16 * (col % 64 / 16)); columns n .. ldx-1 are zero, and
 *          bytes of rows past count*8 are left as 0x5a;
 *   E_out  [count*8][n] int8 (segment 1);
 *   E2_out [count][64] int8 (segment 2), mode 1 only (NULL in mode 0);
 *   X16_out optional in mode 0 (NULL in mode 1): [count][8*n] int16, segment 0 as stored in sk. */
int lwe_test_sample_batch(lwe_ctx* ctx, int pid, size_t count, int mode, int layout, const uint8_t* keys,
                          int8_t* X_out, int8_t* E_out, int8_t* E2_out, uint8_t* X16_out, void* hip_stream);
/* The encryption product with injected operands (Alg. 2 without the sampler): for count
 * instances, B' = S A + E mod q and V = S B + E2 + encode(mu) mod q, where A comes from seedA
 * (regenerated inside the product kernel the batch size selects), B = (B^T)^T with
 * Bt = 8 x n uint16, S and E are [count*8][n] int8, E2 is [count][64] int8 and mu is
 * [count][mu_bytes]; ct receives [count][ct_bytes] records (B' then V).  With S = unit rows and
 * E = 0, B' row r is row r's selected row of A. */
int lwe_test_product(lwe_ctx* ctx, int pid, size_t count, const uint8_t* seedA, const uint8_t* Bt,
                     const int8_t* S, const int8_t* E, const int8_t* E2, const uint8_t* mu, uint8_t* ct,
                     void* hip_stream);
/* PKE encryption with explicit coins (no hashing): ct = Encrypt(pk, mu; coins). */
int lwe_test_encrypt(lwe_ctx* ctx, int pid, size_t count, const uint8_t* pk,
                     const uint8_t* coins /* [count][16] */, const uint8_t* mu, uint8_t* ct,
                     void* hip_stream);
/* PKE decryption without re-encryption: mu = Decrypt(sk, ct) for count ciphertexts. */
int lwe_test_decrypt(lwe_ctx* ctx, int pid, size_t count, const uint8_t* sk, const uint8_t* ct,
                     uint8_t* mu, void* hip_stream);
/* SHA3-256 of count messages of len bytes each ([count][len] -> [count][32]), computed
 * by the device sponge. */
int lwe_test_sha3(lwe_ctx* ctx, size_t count, size_t len, const uint8_t* in, uint8_t* out,
                  void* hip_stream);

/* Kernel timing for measurement.  While enabled, every kernel the context launches is
 * bracketed by a pair of HIP events on the stream it runs on.  lwe_prof_read synchronises
 * the recorded events and returns, for one kernel name ("sample", "prod_strip" (encryption),
 * "prod_strip_cmp" (the re-encryption and compare of a decapsulation),
 * "prod_stream", "finalize", "decrypt", "fo_coins", "expand_keys", "hash_records" (either
 * layout of lwe_ctx_set_hash_lanes), "final_ss", "fill", "keystream", "sample_stream",
 * "expand_A"; for the paper's sets "drbg_chain", "pb_sample", "pb_rows", "pb_decrypt"), the
 * number of launches and their summed device time since the last reset. */
int lwe_prof_enable(lwe_ctx* ctx, int on);
int lwe_prof_reset(lwe_ctx* ctx);
int lwe_prof_read(lwe_ctx* ctx, const char* kernel, uint64_t* launches, double* total_ms);

/* Tuning knobs of the batched product kernel (the tile autotuner of the Python package,
 * paper_2606_01211_amd.tune, writes them).  Zero leaves a knob at its built-in default.
 * lwe_set_tuning returns LWE_EINVAL for a (col_groups, row_groups) pair that the library does
 * not build, or an a_source other than 0 or 1. */
typedef struct {
  uint32_t col_groups;   /* 16-column groups per workgroup strip */
  uint32_t row_groups;   /* 16-row groups per wave in the streaming loop; built
                            (col_groups, row_groups) pairs: (1, 2|4), (2, 2|4), (3, 2|4) */
  uint32_t m_chunks;     /* row chunks sharing one regenerated strip of A */
  uint32_t host_hash_max;/* batches up to this size hash on the host */
  uint32_t a_source;     /* 0: every product regenerates A from its seed inside the kernel
                            (fused; the default).  1: each call first expands A once into
                            device memory (n * n * 2 bytes held by the context) and the
                            product reads it back (unfused; key-generation batches of more
                            than one instance stay fused).  Results are identical. */
} lwe_tuning;
int lwe_set_tuning(lwe_ctx* ctx, int pid, const lwe_tuning* t);
int lwe_get_tuning(lwe_ctx* ctx, int pid, lwe_tuning* t);

/* Decapsulation that allocates nothing, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * It computes exactly what lwe_decaps_batch computes (the same kernels), on the current
 * device, with the working memory (decrypted messages, coins, round keys, S', E', E'',
 * compare flags, ciphertext hashes, split-K accumulator) taken from one static device array
 * of LWE_NOALLOC_SCRATCH_BYTES per device, which the library holds until the process ends.
 *   sk, ct, ss: device pointers only (LWE_EINVAL otherwise); layouts as lwe_decaps_batch.
 *   hip_stream: the stream the work is queued on; NULL = the null stream, synchronous.
 * Returns LWE_ENOMEM, before launching anything, when count instances need more than the
 * array holds (at n = 1344 about 1,500 instances).  The first call on a device sets the
 * array up there (symbol lookup and a 1 KB table copy).  Every call on a device shares its
 * array, whose contents the next call overwrites: calls that overlap on one device (other
 * streams, other threads) race and must be ordered by the caller. */
#define LWE_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int lwe_decaps_batch_noalloc(int pid, size_t count, const uint8_t* sk, const uint8_t* ct, uint8_t* ss,
                             void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LWE_H */
