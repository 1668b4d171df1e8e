/*
 * All-cores CPU implementation of the matrix-form LWE KEM, for comparison with the GPU
 * library (the paper compares its GPU code with a multithreaded OpenMP CPU version using
 * every core of the host, Sec. 4.1).
 *
 * Same scheme and byte formats as the GPU library and the oracle (nbar = mbar = 8,
 * q = 2^logq, AES-128-CTR seed expansion and noise, 16-bit CDF sampler, SHA3-256 FO
 * transform), written for speed on x86-64 hosts: AES-NI counter mode, an AVX2 int16
 * multiply-add micro-kernel for the products (arithmetic mod 2^32, reduced mod q at the
 * end), OpenMP over tiles and instances.  It shares no code with the oracle or the GPU
 * library; only the benchmark and the tests load it, and the GPU product path never calls it.
 */
#ifndef LWE_CPU_H
#define LWE_CPU_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int n;        /* multiple of 8 */
  int logq;     /* q = 2^logq, logq <= 16 */
  int B;        /* message bits per coefficient */
  int K;        /* CDF support [-K, K], K <= 15 */
  double sigma; /* width of the discrete Gaussian of the CDF table */
} lwc_params;

int lwc_threads(void);
size_t lwc_pk_bytes(const lwc_params* p);
size_t lwc_sk_bytes(const lwc_params* p);
size_t lwc_ct_bytes(const lwc_params* p);
size_t lwc_mu_bytes(const lwc_params* p);

/* KeyGen of count key pairs (seedA[count][16], seedSK[count][16], z[count][32]). */
int lwc_keygen_batch(const lwc_params* p, size_t count, const uint8_t* seedA, const uint8_t* seedSK,
                     const uint8_t* z, uint8_t* pk, uint8_t* sk);
/* Encaps of count messages mu[count][mu_bytes] under one public key. */
int lwc_encaps_batch(const lwc_params* p, size_t count, const uint8_t* pk, const uint8_t* mu, uint8_t* ct,
                     uint8_t* ss);
/* Decaps of count ciphertexts ct[count][ct_bytes] under one secret key. */
int lwc_decaps_batch(const lwc_params* p, size_t count, const uint8_t* sk, const uint8_t* ct, uint8_t* ss);

#ifdef __cplusplus
}
#endif
#endif
