/*
 * Plain CPU oracle for the LWE KEM hot path (TEST INFRASTRUCTURE ONLY).
 *
 * This library is the slow, obviously-correct reference that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the product never links it, and it shares no
 * code, header, table or constant generator with the GPU path.
 *
 * Scheme (paper: Sec. 2.1 eq. (1); Alg. 1-5), matrix form with nbar = mbar = 8:
 *   KeyGen : A <- AES-128-CTR(seedA);  S^T, E^T <- CDF sampler(seedSK)
 *            B^T = S^T A^T + E^T  mod q               (Alg. 1, t = A s + e)
 *   Encrypt: S', E', E'' <- CDF sampler(coins)
 *            B' = S' A + E'        mod q               (Alg. 2, u = A^T r + e1)
 *            V  = S' B + E'' + enc(mu) mod q           (Alg. 2, v = t^T r + e2 + m)
 *   Decrypt: M  = V - B' S          mod q, mu' = dec(M) (Alg. 3)
 *   Encaps / Decaps: Fujisaki-Okamoto with implicit rejection (Alg. 4, 5).
 * All integers; q = 2^logq.
 */
#ifndef LWE_ORACLE_H
#define LWE_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NBAR 8
#define ORC_MBAR 8

typedef struct {
  int n;        /* lattice dimension, multiple of 8 */
  int logq;     /* q = 2^logq */
  int B;        /* message bits per coefficient */
  int K;        /* CDF support [-K, K] */
  double sigma; /* width of the centred discrete Gaussian the table approximates */
} orc_params;

/* Registry of the named parameter sets; returns 0 on success, -1 if n unknown. */
int orc_params_for(int n, orc_params* out);

/* byte sizes of the serialised objects */
size_t orc_pk_bytes(const orc_params* p);
size_t orc_sk_bytes(const orc_params* p);
size_t orc_ct_bytes(const orc_params* p);
size_t orc_mu_bytes(const orc_params* p);

/* ---- AES-128 (FIPS-197) ---- */
void orc_aes128_expand_key(const uint8_t key[16], uint8_t rk[176]);
void orc_aes128_encrypt(const uint8_t rk[176], const uint8_t in[16], uint8_t out[16]);

/* ---- CTR keystream (SP 800-38A incrementing function over all 128 bits) ----
 * Counter block for domain d and block index b is the big-endian 128-bit
 * integer d*2^96 + b.  Word w of the keystream is KS[2w] + 256*KS[2w+1]. */
void orc_ctr_blocks(const uint8_t key[16], uint32_t domain, uint64_t block0, size_t nblocks,
                    uint8_t* out);
void orc_ctr_words(const uint8_t key[16], uint32_t domain, uint64_t word0, size_t nwords,
                   uint16_t* out);

/* ---- SHA3-256 (FIPS 202) ---- */
void orc_sha3_256(const uint8_t* in, size_t len, uint8_t out[32]);

/* ---- CDF table and sampler ---- */
/* Fills T[0..K]; returns 0, or -1 if the table is not strictly increasing. */
int orc_cdf_table(int K, double sigma, uint16_t* T);
int orc_sample_word(uint16_t u, const uint16_t* T, int K);
/* count samples from keystream words word0.. of (key, domain) */
void orc_sample_stream(const orc_params* p, const uint8_t key[16], uint32_t domain, uint64_t word0,
                       size_t count, int16_t* out);

/* ---- building blocks ---- */
/* columns col0..col0+ncols-1 of A, each of n entries: out[c*n + i] = A[i][col0+c] */
void orc_expand_A_cols(const orc_params* p, const uint8_t seedA[16], int col0, int ncols,
                       uint16_t* out);
/* encode / decode of one coefficient value */
uint16_t orc_encode_coeff(const orc_params* p, const uint8_t* mu, int coeff);
int orc_decode_value(const orc_params* p, uint16_t x);

/* PKE layer with explicit randomness. Bt is nbar x n (uint16, q-reduced). */
void orc_pke_keygen(const orc_params* p, const uint8_t seedA[16], const uint8_t seedSK[16],
                    int16_t* St /* nbar x n */, uint16_t* Bt /* nbar x n */);
void orc_pke_encrypt(const orc_params* p, const uint8_t seedA[16], const uint16_t* Bt,
                     const uint8_t coins[16], const uint8_t* mu, uint16_t* Bp /* mbar x n */,
                     uint16_t* V /* mbar x nbar */);
void orc_pke_decrypt_M(const orc_params* p, const int16_t* St, const uint16_t* Bp, const uint16_t* V,
                       uint16_t* M /* mbar x nbar */);
void orc_pke_decode(const orc_params* p, const uint16_t* M, uint8_t* mu_out);

/* Single entries computed straight from the definitions, for sampled checks at large n. */
uint16_t orc_A_entry(const orc_params* p, const uint8_t seedA[16], long i, long j);
uint16_t orc_Bt_entry(const orc_params* p, const uint8_t seedA[16], const uint8_t seedSK[16], int c,
                      long i);
uint16_t orc_Bp_entry(const orc_params* p, const uint8_t seedA[16], const uint8_t coins[16], int r,
                      long j);

/* V = S' B + E'' + enc(mu) mod q alone (needs no A), for sampled checks at large n. */
void orc_pke_V(const orc_params* p, const uint16_t* Bt, const uint8_t coins[16], const uint8_t* mu,
               uint16_t* V /* mbar x nbar */);

/* Exact noise N = S'E - E'S + E'' of one encryption, as signed integers (not reduced);
 * returns max |N|. */
long orc_noise_max(const orc_params* p, const uint8_t seedSK[16], const uint8_t coins[16]);

/* ---- KEM (Alg. 4 / Alg. 5 with the FO transform) ---- */
void orc_kem_keygen(const orc_params* p, const uint8_t seedA[16], const uint8_t seedSK[16],
                    const uint8_t z[32], uint8_t* pk, uint8_t* sk);
void orc_kem_encaps(const orc_params* p, const uint8_t* pk, const uint8_t* mu, uint8_t* ct,
                    uint8_t ss[32]);
/* returns 1 if the re-encryption matched (accepted), 0 if implicitly rejected */
int orc_kem_decaps(const orc_params* p, const uint8_t* sk, const uint8_t* ct, uint8_t ss[32]);
/* coins and K' derived from (pkh, mu) */
void orc_fo_coins(const orc_params* p, const uint8_t pkh[32], const uint8_t* mu, uint8_t coins[16],
                  uint8_t kprime[32]);

/* number of OpenMP threads the oracle uses (1 if built without OpenMP) */
int orc_threads(void);

/* ---- AES-256 (FIPS-197, Nk = 8, Nr = 14) ---- */
void orc_aes256_expand_key(const uint8_t key[32], uint8_t rk[240]);
void orc_aes256_encrypt(const uint8_t rk[240], const uint8_t in[16], uint8_t out[16]);

/* ---- CTR_DRBG, AES-256, no derivation function (SP 800-90A Rev. 1, Sec. 10.2.1) ---- */
void orc_drbg_instantiate(const uint8_t entropy[48], uint8_t key[32], uint8_t V[16]);
/* one Generate request of nbytes (<= 65536) without additional input */
void orc_drbg_generate(uint8_t key[32], uint8_t V[16], size_t nbytes, uint8_t* out);
/* Noise words 0 .. nwords-1 of (key, domain): a DRBG instantiated from key (16 bytes) ||
 * domain (4 bytes, little endian) || 28 zero bytes and read in requests of 65536 bytes;
 * word w = bytes 2w, 2w+1 of the output, little endian. */
void orc_drbg_words(const uint8_t key16[16], uint32_t domain, size_t nwords, uint16_t* out);

/* ======================================================================================
 * The paper's own parameterisation (lwe_oracle_pb.c): one encryption per message bit
 * (256 of them: nbar = 1, mbar = 256, one bit per coefficient), prime q from Table 1,
 * s from the centred binomial distribution (eta), e, r, e1 from the discrete Gaussian of
 * sigma (CDF table), e2 from the centred uniform distribution on [-k, k], all noise from
 * the AES-256 CTR_DRBG above; A from AES-128-CTR(seedA) reduced mod q.
 * ====================================================================================== */
#define ORC_PB_BITS 256
enum { ORC_PB_BINOMIAL = 0, ORC_PB_GAUSSIAN = 1, ORC_PB_UNIFORM = 2 };

typedef struct {
  int n;        /* lattice dimension */
  int q;        /* prime modulus */
  double sigma; /* Gaussian width of e, r, e1 */
  int K;        /* support [-K, K] of the Gaussian's CDF table */
  int k;        /* e2 uniform on [-k, k] */
  int eta;      /* s binomial with parameter eta */
} orc_pb_params;

int orc_pb_params_for(int n, orc_pb_params* out); /* Table 1 rows n = 512 .. 32768 */
int orc_pb_support(double sigma);                  /* largest K with a strictly increasing table */
size_t orc_pb_coef_bytes(const orc_pb_params* p);  /* 2 if q < 2^16, else 4 */
size_t orc_pb_pk_bytes(const orc_pb_params* p);
size_t orc_pb_sk_bytes(const orc_pb_params* p);
size_t orc_pb_ct_bytes(const orc_pb_params* p);
int orc_pb_binomial(uint16_t w, int eta);
int orc_pb_uniform(uint16_t w, int k);
/* count samples of distribution dist (ORC_PB_*) from the noise words of (key, domain) */
void orc_pb_noise(const orc_pb_params* p, const uint8_t key[16], uint32_t domain, int dist, size_t count,
                  int16_t* out);
void orc_pb_expand_A_cols(const orc_pb_params* p, const uint8_t seedA[16], int col0, int ncols, uint32_t* out);
void orc_pb_pke_keygen(const orc_pb_params* p, const uint8_t seedA[16], const uint8_t seedSK[16], int16_t* s,
                       uint32_t* t);
void orc_pb_pke_encrypt(const orc_pb_params* p, const uint8_t seedA[16], const uint32_t* t, const uint8_t coins[16],
                        const uint8_t* mu, uint32_t* U /* 256 x n */, uint32_t* v /* 256 */);
int orc_pb_decode(int q, uint32_t x);
void orc_pb_pke_decrypt(const orc_pb_params* p, const int16_t* s, const uint32_t* U, const uint32_t* v,
                        uint8_t* mu);
long orc_pb_noise_max(const orc_pb_params* p, const uint8_t seedSK[16], const uint8_t coins[16]);
uint32_t orc_pb_t_entry(const orc_pb_params* p, const uint8_t seedA[16], const uint8_t seedSK[16], long i);
uint32_t orc_pb_u_entry(const orc_pb_params* p, const uint8_t seedA[16], const uint8_t coins[16], int r, long j);
void orc_pb_kem_keygen(const orc_pb_params* p, const uint8_t seedA[16], const uint8_t seedSK[16],
                       const uint8_t z[32], uint8_t* pk, uint8_t* sk);
void orc_pb_kem_encaps(const orc_pb_params* p, const uint8_t* pk, const uint8_t mu[32], uint8_t* ct,
                       uint8_t ss[32]);
int orc_pb_kem_decaps(const orc_pb_params* p, const uint8_t* sk, const uint8_t* ct, uint8_t ss[32]);

#ifdef __cplusplus
}
#endif
#endif
