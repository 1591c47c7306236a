/*
 * zinc.h -- C ABI of the MI355X (gfx950) library for batched CKKS encryption:
 * vanilla public-key encryption and Zinc encryption, from
 * "At Least Factor-of-Two Optimization for RWLE-Based Homomorphic Encryption"
 * (arXiv 2408.07304).
 *
 * The scheme follows the paper's statement of the problem: a homomorphic
 * scheme Pi = (Gen, Enc, Dec, +, x) and its Zinc extension (Gen, Enc_z, Dec)
 * (Security section).  Enc is Eq. 8 (vanilla CKKS encryption with the public
 * key of Eq. 7), Enc_z is Algorithm 1 (cached Enc(0) plus the plaintext plus
 * fresh Gaussian noise), Dec is [c1 + c2 sk]_q.  Encoding and decoding are the
 * CKKS canonical embedding, which the paper takes from the CKKS paper.
 *
 * Data conventions (all sizes in elements):
 *   N        ring degree, 2^log_n with 12 <= log_n <= 15.
 *   M        moduli in the chain; the last one is the special prime, present in
 *            the secret and public keys and absent from plaintexts and
 *            ciphertexts.  L = M - 1 data limbs.
 *   residues uint64, canonical in [0, q_l).
 *   slots    double [batch][n_slots], n_slots <= N/2, real values; missing
 *            slots up to N/2 are zero.
 *   plaintext uint64 [batch][L][N], coefficient domain, limb-major.
 *   ciphertext uint64 [batch][2][L][N] = (c1, c2), NTT domain, each limb in
 *            bit-reversed evaluation order: c[k] = sum_i a_i psi^((2 brv(k)+1) i)
 *            with psi the smallest primitive 2N-th root of unity mod q_l.
 *   ct_ids   uint64 [batch]: every random coefficient of ciphertext b is a
 *            function of (seed, ct_ids[b], tag, limb, index) only, so equal
 *            identifiers give bit-identical ciphertexts in any batch, plan or
 *            serving mix.  Identifiers must be < 2^63; ZINC_KEY_ID and
 *            ZINC_ZERO_ID are reserved for the keys and the cached Enc(0).
 *
 * Memory ownership: pointers named d_* are device memory owned by the caller
 * (contiguous, 8-byte aligned); the library never frees them and keeps no
 * pointer to them after a call returns, except inside a plan or a server
 * (see zinc_plan_create and zinc_server_create).  The library owns its tables, keys and the Zinc cache.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue
 * work and return; argument and state errors are reported synchronously.  A
 * device fault surfaces at the caller's next synchronisation.  Range
 * violations found on the device (a slot value whose scaled magnitude reaches
 * 2^62, a decoded coefficient outside the limb-0 lift range) set a sticky flag
 * read by zinc_device_errors.  So does a direct encryption call given a
 * reserved identifier (>= 2^63): that ciphertext is not written.
 *
 * Threads: a context is read-only after zinc_precompute; encryption calls on
 * one context may run concurrently on different streams (the batch codec's
 * first call for a plaintext modulus builds its tables under a lock).
 * zinc_keygen, zinc_precompute, zinc_set_bgv, zinc_set_tuning and
 * zinc_autotune need exclusive use of the context.
 *
 * Every call returns a zinc_status; zinc_last_error() gives a message for the
 * calling thread's most recent failure.
 */
#ifndef ZINC_H
#define ZINC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int zinc_status;
#define ZINC_OK 0
#define ZINC_E_INVAL (-1)   /* null pointer, zero or oversized count, bad enum value   */
#define ZINC_E_PARAM (-2)   /* invalid parameter set (ring degree, moduli, scale)      */
#define ZINC_E_STATE (-3)   /* call out of order (encrypt before keygen/precompute)    */
#define ZINC_E_NOMEM (-4)   /* device allocation failed                                */
#define ZINC_E_HIP   (-5)   /* HIP runtime error (launch, copy, device)                */
#define ZINC_E_RANGE (-6)   /* n_slots > N/2, scale too large for the moduli           */

#define ZINC_KEY_ID  0xFFFFFFFFFFFFFFFFull
#define ZINC_ZERO_ID 0xFFFFFFFFFFFFFFFEull
#define ZINC_MAX_MODULI 32

#define ZINC_SCHEME_VANILLA    0
#define ZINC_SCHEME_ZINC       1
#define ZINC_SCHEME_VANILLA_SP 2   /* zinc_encrypt_slots only: see zinc_encrypt_vanilla_sp */

/* Message describing the calling thread's last failed call ("" if none). */
const char* zinc_last_error(void);

typedef struct zinc_ctx zinc_ctx;
typedef struct zinc_plan zinc_plan;
typedef struct zinc_server zinc_server;

/* Parameter set (Polynomials and Distributions; System Implementation).
 *   log_n      ring degree N = 2^log_n, 12..15.
 *   n_moduli   M, 2..ZINC_MAX_MODULI; the last modulus is the special prime.
 *   bit_sizes  [M] bit sizes, 20..60, used when moduli == NULL: for each size,
 *              in order, the largest prime q < 2^b with q = 1 mod 2N not
 *              already chosen.
 *   moduli     [M] explicit primes (each = 1 mod 2N, < 2^60, distinct) or NULL.
 *   scale      Delta, > 0; Delta * 2^62 limits the slot magnitude.
 *   sigma      standard deviation of chi; only 3.2 (the paper's value) is
 *              accepted, as the sampler's cumulative table is built for it.
 *   seed       64-bit key of the counter-based generator (Philox4x32-10). */
typedef struct zinc_params {
    uint32_t log_n;
    uint32_t n_moduli;
    const uint32_t* bit_sizes;
    const uint64_t* moduli;
    double scale;
    double sigma;
    uint64_t seed;
} zinc_params;

typedef struct zinc_info {
    uint32_t n;                 /* N                                          */
    uint32_t log_n;
    uint32_t n_moduli;          /* M                                          */
    uint32_t limbs;             /* L = M - 1                                  */
    uint64_t moduli[ZINC_MAX_MODULI];
    uint64_t psi[ZINC_MAX_MODULI];   /* smallest primitive 2N-th roots        */
    double scale;
    uint64_t seed;
    uint64_t cdt[38];           /* cumulative table of chi (see zinc_keygen)  */
    size_t plaintext_bytes;     /* L*N*8 per plaintext                        */
    size_t ciphertext_bytes;    /* 2*L*N*8 per ciphertext                     */
    int keyed;                  /* zinc_keygen done                           */
    int precomputed;            /* zinc_precompute done                       */
    uint32_t ntt_fp64_mask;     /* bit l set: limb l's forward NTT runs in exact
                                   FP64 arithmetic (moduli below 2^50), else in
                                   64-bit integer (Shoup) arithmetic          */
    uint32_t tile[2];           /* coefficients per thread of the fused kernel
                                   for vanilla [0] and Zinc [1] (see zinc_tuning) */
    uint32_t reg_epilogue;      /* see zinc_tuning                            */
    uint64_t bgv_t;             /* BGV plaintext modulus t (zinc_set_bgv), 0
                                   for a CKKS/BFV context                     */
} zinc_info;

/* Create a context on the current HIP device: validate the parameters, derive
 * the moduli and roots, build the twiddle, FFT and sampler tables and upload
 * them (synchronously).  ZINC_E_PARAM on invalid parameters. */
zinc_status zinc_ctx_create(const zinc_params* p, zinc_ctx** out);
/* Free everything the context owns (synchronises the device first). */
zinc_status zinc_ctx_destroy(zinc_ctx* ctx);
zinc_status zinc_ctx_info(const zinc_ctx* ctx, zinc_info* out);

/* Gen (Eq. 7): s <- R_2 (uniform ternary), a <- R_q (uniform, drawn directly in
 * the NTT domain), e <- chi; pk1 = [-a s + e]_q, pk2 = a, over all M moduli.
 * chi is the discrete Gaussian of standard deviation 3.2 on [-19, 19],
 * sampled by inverting a 38-entry cumulative table with one 64-bit uniform.
 * Keys stay on the device.  Synchronous with respect to `stream`'s completion
 * only when the caller synchronises. */
zinc_status zinc_keygen(zinc_ctx* ctx, void* stream);

/* Zinc precomputation (Scheme Description, "Precomputation"): cache a single
 * Enc(0), a vanilla encryption of the zero plaintext under ZINC_ZERO_ID.
 * ZINC_E_STATE before zinc_keygen. */
zinc_status zinc_precompute(zinc_ctx* ctx, void* stream);

/* CKKS encoding (canonical embedding; the paper defers to the CKKS paper):
 * slot j <-> root zeta^(5^j mod 2N), zeta = exp(i pi/N);
 * m_i = round_half_even((2 Delta / N) Re sum_j z_j zeta^(-i 5^j)), reduced per
 * data limb.  d_slots [batch][n_slots] -> d_pt [batch][L][N].
 * ZINC_E_RANGE if n_slots > N/2. */
zinc_status zinc_encode(zinc_ctx* ctx, const double* d_slots, uint32_t n_slots, uint32_t batch,
                        uint64_t* d_pt, void* stream);

/* Vanilla encryption, Eq. 8 with pk2 in c2 (as the correctness proof of
 * Theorem 1 uses it): u <- R_2, e1, e2 <- chi;
 * c1 = [pk1 u + e1 + m]_q, c2 = [pk2 u + e2]_q.
 * d_pt [batch][L][N] -> d_ct [batch][2][L][N].  ZINC_E_STATE before keygen. */
zinc_status zinc_encrypt_vanilla(zinc_ctx* ctx, const uint64_t* d_pt, uint32_t batch,
                                 const uint64_t* d_ct_ids, uint64_t* d_ct, void* stream);

/* Zinc encryption, Algorithm 1: c = zero + m; e1', e2' <- chi;
 * c' = ([c1 + e1']_q, [c2 + e2']_q), with `zero` the cached Enc(0).
 * d_pt [batch][L][N] -> d_ct [batch][2][L][N].  ZINC_E_STATE before precompute. */
zinc_status zinc_encrypt(zinc_ctx* ctx, const uint64_t* d_pt, uint32_t batch,
                         const uint64_t* d_ct_ids, uint64_t* d_ct, void* stream);

/* Encode and encrypt in one fused launch (scheme = ZINC_SCHEME_VANILLA,
 * ZINC_SCHEME_ZINC or ZINC_SCHEME_VANILLA_SP): the result is bit-identical to
 * zinc_encode followed by zinc_encrypt_vanilla / zinc_encrypt /
 * zinc_encrypt_vanilla_sp.  d_slots [batch][n_slots]. */
zinc_status zinc_encrypt_slots(zinc_ctx* ctx, int scheme, const double* d_slots, uint32_t n_slots,
                               uint32_t batch, const uint64_t* d_ct_ids, uint64_t* d_ct,
                               void* stream);

/* Decryption Dec(c) = [c1 + c2 sk]_q (the equation after Algorithm 1), back to
 * the coefficient domain: d_ct [batch][2][L][N] -> d_pt [batch][L][N]. */
zinc_status zinc_decrypt(zinc_ctx* ctx, const uint64_t* d_ct, uint32_t batch, uint64_t* d_pt,
                         void* stream);

/* CKKS decoding: centred lift of limb 0 (valid while every coefficient is
 * below q_0/2 in magnitude; violations set the device error flag), then
 * z_j = Re m(zeta^(5^j)) / Delta.  d_pt [batch][L][N] -> d_slots [batch][N/2]. */
zinc_status zinc_decode(zinc_ctx* ctx, const uint64_t* d_pt, uint32_t batch, double* d_slots,
                        void* stream);

/* Vanilla encryption the way a library with a special prime computes it (the
 * paper's CPU baseline, SEAL, ends its chain in such a prime p, the context's
 * last modulus): Eq. 8's encryption of zero over all M moduli,
 * a_j = pk_j u + e_j, divided by p with rounding (coefficient-wise
 * round(a_j / p), which leaves the L data limbs), then the message added to
 * c1.  Same layouts as zinc_encrypt_vanilla; costlier (the special limb's
 * transforms and two inverse transforms); every ring degree.
 * zinc_encrypt_slots with ZINC_SCHEME_VANILLA_SP is the fused form.
 * Scratch of batch * 3 * N * 8 bytes is allocated and freed in `stream`'s
 * order (hipMallocAsync). */
zinc_status zinc_encrypt_vanilla_sp(zinc_ctx* ctx, const uint64_t* d_pt, uint32_t batch,
                                    const uint64_t* d_ct_ids, uint64_t* d_ct, void* stream);

/* zinc_encrypt_vanilla_sp without allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops that
 * forbid it): same arguments and results, but the per-ciphertext scratch
 * (3 * N int64) lives in a 64 MiB static device array of the library, one
 * per GPU, held until the process ends.  So a call takes at most
 * 64 MiB / (24 N) ciphertexts (682, 341, 170 and 85 at N = 4096 ... 32768;
 * ZINC_E_RANGE above).  Calls on one GPU share that array: calls that
 * overlap in time on one GPU (different streams, threads) race and must be
 * serialised by the caller.  The scratch needs no clearing (each ciphertext's
 * rows are written before they are read).  The context's device must be
 * current (ZINC_E_HIP otherwise).  Calls no allocating routine. */
zinc_status zinc_encrypt_vanilla_sp_noalloc(zinc_ctx* ctx, const uint64_t* d_pt, uint32_t batch,
                                            const uint64_t* d_ct_ids, uint64_t* d_ct, void* stream);

/* BFV on the same contexts (Scheme Flexibility section, Eq. 12): the message
 * is scaled by Delta = floor(Q / t), Q the product of the data moduli, and the
 * rest of the encryption is unchanged, so zinc_encrypt (Zinc) and
 * zinc_encrypt_vanilla (Eq. 8) encrypt BFV plaintexts as they are.
 * Plaintexts: integer polynomials with coefficients in Z_t, one per ring
 * coefficient (slot vectors go through zinc_batch_encode first), int64 [batch][N],
 * any representative (reduced mod t by the encoding).
 * zinc_bfv_encode: d_m -> d_pt [batch][L][N] = Delta * m mod q_l.
 * zinc_bfv_decode: decrypted residues d_pt [batch][L][N] (zinc_decrypt) ->
 * d_m = round(t x / Q) mod t, centred in (-t/2, t/2], x the residues'
 * CRT value (RNS scale-and-round; correct while the noise is below Delta/2).
 * t in [2, 2^32) and below every data modulus (ZINC_E_INVAL otherwise). */
zinc_status zinc_bfv_encode(zinc_ctx* ctx, uint64_t t, const int64_t* d_m, uint32_t batch, uint64_t* d_pt,
                            void* stream);
zinc_status zinc_bfv_decode(zinc_ctx* ctx, uint64_t t, const uint64_t* d_pt, uint32_t batch, int64_t* d_m,
                            void* stream);

/* BGV on the same contexts (Scheme Flexibility section, Eq. 13): every
 * Gaussian error (the key's e, Enc's e1 and e2, Zinc's fresh e1' and e2') is
 * multiplied by the plaintext modulus t, and the message enters unscaled.
 * zinc_set_bgv(ctx, t) puts the context in BGV form for the next zinc_keygen
 * and clears its keys and cached Enc(0) (keyed = precomputed = 0); t = 1
 * returns it to the CKKS/BFV form.  t in [2, 2^32) and below every data
 * modulus (ZINC_E_INVAL); every ring degree.  A BGV context encrypts
 * residue plaintexts through zinc_encrypt (Zinc, Algorithm 1 with t-scaled
 * errors) and zinc_encrypt_vanilla (Eq. 8 with t-scaled errors) and decrypts
 * through zinc_decrypt; zinc_encrypt_slots, zinc_encrypt_vanilla_sp, the BFV
 * codec, plans, servers and zinc_autotune reject it (ZINC_E_STATE).
 * zinc_bgv_encode: int64 d_m [batch][N], any representative ->
 * d_pt [batch][L][N] = m mod t (in [0, t)) on every limb.
 * zinc_bgv_decode: decrypted residues d_pt [batch][L][N] -> d_m = the centred
 * CRT value of the residues (in (-Q/2, Q/2]) mod t, centred in (-t/2, t/2]
 * (correct while the noise t (e u + e1 + e2 s) stays below Q/2).
 * Both: ZINC_E_STATE on a context not in BGV form. */
zinc_status zinc_set_bgv(zinc_ctx* ctx, uint64_t t);
zinc_status zinc_bgv_encode(zinc_ctx* ctx, const int64_t* d_m, uint32_t batch, uint64_t* d_pt, void* stream);
zinc_status zinc_bgv_decode(zinc_ctx* ctx, const uint64_t* d_pt, uint32_t batch, int64_t* d_m, void* stream);

/* Batch (slot) encoding of BFV and BGV plaintexts.  The paper takes encodings
 * from those schemes' own papers (Scheme Flexibility section); this is the
 * standard batch encoding for a prime t = 1 (mod 2N): slot j of a plaintext m
 * in Z_t[X]/(X^N + 1) is m(zeta^(e_j)) mod t, where zeta is the smallest
 * primitive 2N-th root of unity mod t, e_i = 3^i and e_(N/2 + i) = -3^i
 * (mod 2N) for i < N/2.  So X -> X^3 rotates each half of the slots by one
 * and X -> X^-1 swaps the halves, and products of plaintexts are slot-wise.
 * zinc_batch_encode: int64 slot values d_slots [batch][N] (any
 * representatives) -> the coefficients d_m [batch][N] in [0, t), ready for
 * zinc_bfv_encode or zinc_bgv_encode.
 * zinc_batch_decode: int64 coefficients d_m [batch][N] (any representatives,
 * e.g. zinc_bfv_decode's or zinc_bgv_decode's output) -> slot values
 * d_slots [batch][N] in (-t/2, t/2].
 * Input and output may be the same buffer.  t prime, t < 2^31, t = 1 mod 2N
 * (ZINC_E_INVAL otherwise).  The first call for a given t builds its tables
 * (20 N bytes of device memory, kept until zinc_ctx_destroy) with a
 * synchronous upload; later calls only launch. */
zinc_status zinc_batch_encode(zinc_ctx* ctx, uint64_t t, const int64_t* d_slots, uint32_t batch, int64_t* d_m,
                              void* stream);
zinc_status zinc_batch_decode(zinc_ctx* ctx, uint64_t t, const int64_t* d_m, uint32_t batch, int64_t* d_slots,
                              void* stream);

/* The element-wise step of Zinc encryption alone (Algorithm 1's additions, in
 * the NTT domain where the cached Enc(0) is kept), for callers that compute
 * the transforms themselves: d_ct = d_hat + Enc(0) component-wise mod q_l,
 * with d_hat [batch][2][L][N] = (NTT(m + e1'), NTT(e2')) as canonical residues.
 * d_ct may be d_hat (in place).  ZINC_E_STATE before zinc_precompute. */
zinc_status zinc_elementwise_zinc(zinc_ctx* ctx, const uint64_t* d_hat, uint32_t batch, uint64_t* d_ct,
                                  void* stream);

/* The element-wise step of vanilla encryption alone (Eq. 8 in the NTT domain):
 * c1 = pk1 * u_hat + hat1, c2 = pk2 * u_hat + hat2 mod q_l, with
 * d_uhat [batch][L][N] = NTT(u) and d_hat [batch][2][L][N] =
 * (NTT(m + e1), NTT(e2)), canonical residues.  d_ct may be d_hat; d_uhat must
 * not overlap d_ct.  ZINC_E_STATE before zinc_keygen. */
zinc_status zinc_elementwise_vanilla(zinc_ctx* ctx, const uint64_t* d_uhat, const uint64_t* d_hat,
                                     uint32_t batch, uint64_t* d_ct, void* stream);

/* Homomorphic addition (Eq. 2): out = a + b component-wise mod q_l.
 * All three are [batch][2][L][N]; out may alias a or b. */
zinc_status zinc_add(zinc_ctx* ctx, const uint64_t* d_a, const uint64_t* d_b, uint32_t batch,
                     uint64_t* d_out, void* stream);

/* Read and clear the context's sticky device error flags (synchronises the
 * device): bit 0 = slot magnitude out of range in encode, bit 1 = coefficient
 * outside the limb-0 lift range in decode, bit 2 = an encryption call
 * (zinc_encrypt, zinc_encrypt_vanilla, zinc_encrypt_vanilla_sp,
 * zinc_encrypt_slots) was given an identifier >= 2^63; the ciphertexts with
 * such identifiers were left unwritten, since the reserved ones select the
 * randomness of the keys and of the cached Enc(0). */
zinc_status zinc_device_errors(zinc_ctx* ctx, uint32_t* flags);

/* ---- mixed-shape batches (one persistent launch over several contexts) ----
 * An item names a context (index into ctxs), the float64 offset of its slot
 * vector (N/2 values of its ring degree) in the slot buffer, the uint64 offset
 * of its ciphertext ([2][L][N] of its context) in the ciphertext buffer, and its
 * ct_id.  zinc_plan_create copies the items to the device and sorts them by
 * cost; the plan keeps pointers to the contexts, which must outlive it.
 * zinc_plan_launch encrypts every item in one persistent launch on `stream`;
 * n_slot_words and n_ct_words are the lengths of d_slots (float64 words) and
 * d_ct (uint64 words), and a buffer that ends before some item's slots or
 * ciphertext is rejected (ZINC_E_INVAL) before anything is launched.  Launch:
 * the first call records the launch sequence as a HIP graph (on a private
 * stream, so any caller stream works, the null stream included), later calls
 * with the same buffers replay it, and new buffers are recorded again.  The
 * buffers must stay valid until the launch completes; launches of one plan
 * must not overlap (they share the plan's work counter). */
typedef struct zinc_item {
    uint32_t ctx_idx;
    uint32_t reserved;
    uint64_t slot_off;
    uint64_t ct_off;
    uint64_t ct_id;
} zinc_item;

zinc_status zinc_plan_create(zinc_ctx* const* ctxs, uint32_t n_ctx, const zinc_item* items,
                             uint32_t n_items, int scheme, zinc_plan** out);
zinc_status zinc_plan_launch(zinc_plan* plan, const double* d_slots, uint64_t n_slot_words, uint64_t* d_ct,
                             uint64_t n_ct_words, void* stream);
zinc_status zinc_plan_destroy(zinc_plan* plan);

/* ---- serving: admission, continuous batching, latency ---------------------
 * A server holds resident contexts (keys, tables and, for Zinc, the cached
 * Enc(0)) and encrypts requests of 1..max_batch plaintexts of one context as
 * they are submitted.  Each call of zinc_server_progress makes one scheduling
 * pass without blocking:
 *   1. reap: batches whose completion event has fired complete their
 *      requests and return their output bytes to the budget;
 *   2. admit: waiting requests, in submission order, are admitted while their
 *      ciphertext bytes (n_pt * 2 * L * N * 8) fit in the free part of the
 *      HBM budget (first fit over an arena of hbm_budget bytes; the first
 *      request that does not fit blocks the ones behind it);
 *   3. launch: every idle stream (of n_streams) takes admitted requests from
 *      the front, up to max_batch plaintexts, as one batch: a persistent
 *      launch of the mixed-shape kernel over all their plaintexts, whatever
 *      their contexts, followed by a completion event.
 * Plaintext k of a request reads the N/2 slots at d_slots + slot_off + k*N/2,
 * gets ct_id + k, and writes its ciphertext at ct_off + k*2*L*N of the output
 * base: d_ct if the configuration gives one, otherwise the server's own arena
 * (hbm_budget bytes allocated at creation).  In the arena, a completed
 * request's ciphertexts are either discarded at once (retain_outputs = 0,
 * which suits load generation) or kept (retain_outputs = 1) until the caller,
 * having read them through zinc_server_output, calls zinc_server_release;
 * kept outputs hold their share of the budget, so admission waits for
 * releases.  A request whose slots (or, with d_ct, ciphertexts) would reach
 * beyond slots_len (ct_len) is refused at submission.  Outputs are
 * bit-identical to separate launches with the same ct_ids.
 * The server's streams are its own (non-blocking, default priority): inputs
 * must be complete on the device before their requests are submitted.  Times
 * are nanoseconds of the host's monotonic clock since zinc_server_create.
 * A server is used from one thread at a time. */

typedef struct zinc_server_config {
    int scheme;               /* ZINC_SCHEME_VANILLA or ZINC_SCHEME_ZINC              */
    uint32_t n_streams;       /* concurrent batches, 1..16                            */
    uint32_t max_batch;       /* plaintexts per launch, 1..65536                      */
    uint32_t retain_outputs;  /* 1: arena outputs kept until zinc_server_release
                                 (needs d_ct NULL); 0: discarded on completion        */
    uint64_t hbm_budget;      /* bytes of ciphertext admitted at once; 0: half of the
                                 device's free memory at creation                     */
    const double* d_slots;    /* base of every request's slots                        */
    uint64_t* d_ct;           /* base of every request's output, or NULL (arena)      */
    uint64_t slots_len;       /* float64 words of d_slots (> 0)                       */
    uint64_t ct_len;          /* uint64 words of d_ct (> 0 when d_ct is given)        */
} zinc_server_config;

typedef struct zinc_request {
    uint32_t ctx_idx;         /* context (index into the server's contexts)           */
    uint32_t n_pt;            /* plaintexts, 1..max_batch                             */
    uint64_t slot_off;        /* float64 offset of plaintext 0's slots in d_slots     */
    uint64_t ct_off;          /* uint64 offset of ciphertext 0 in d_ct (unused with
                                 the arena)                                           */
    uint64_t ct_id;           /* ct_id of plaintext 0; ct_id + n_pt <= 2^63           */
} zinc_request;

typedef struct zinc_request_times {
    uint64_t submit_ns;       /* submission (for a trace replay: scheduled arrival)   */
    uint64_t admit_ns;        /* its output bytes were granted                        */
    uint64_t launch_ns;       /* its batch was enqueued                               */
    uint64_t done_ns;         /* its batch's completion was observed                  */
    uint32_t batch;           /* sequence number of its batch                         */
    uint32_t stream;          /* stream index that ran the batch                      */
    uint64_t dev_start_ns;    /* device interval of its batch: HIP timing events      */
    uint64_t dev_end_ns;      /* before and after the launch, in nanoseconds since a
                                 reference event recorded at zinc_server_create      */
} zinc_request_times;

/* The server keeps pointers to the contexts, which must outlive it; every
 * context needs keys, and for the Zinc scheme its cached Enc(0). */
zinc_status zinc_server_create(zinc_ctx* const* ctxs, uint32_t n_ctx, const zinc_server_config* cfg,
                               zinc_server** out);
/* Queue a request (host only, no device work).  ZINC_E_RANGE if its output
 * alone exceeds hbm_budget or n_pt exceeds max_batch.  *ticket numbers
 * requests 0, 1, 2, ... in submission order. */
zinc_status zinc_server_submit(zinc_server* srv, const zinc_request* req, uint64_t* ticket);
/* One scheduling pass (reap, admit, launch); *n_done (may be NULL) gets the
 * number of requests completed by this pass. */
zinc_status zinc_server_progress(zinc_server* srv, uint32_t* n_done);
/* *done = 1 and *times filled once the request has completed, else *done = 0. */
zinc_status zinc_server_query(zinc_server* srv, uint64_t ticket, int* done, zinc_request_times* times);
/* Retained outputs (retain_outputs = 1): *d_out = the device address of a
 * completed request's ciphertexts, n_pt * 2 * L * N uint64 words in the
 * server's arena, valid until zinc_server_release(srv, ticket).  ZINC_E_STATE
 * if the server does not retain outputs, or the request has not completed or
 * was already released. */
zinc_status zinc_server_output(zinc_server* srv, uint64_t ticket, uint64_t** d_out);
/* The same output copied (device to device, asynchronously on `stream`) into
 * caller memory d_dst of dst_words uint64 words (ZINC_E_INVAL if shorter). */
zinc_status zinc_server_read_output(zinc_server* srv, uint64_t ticket, uint64_t* d_dst, uint64_t dst_words,
                                    void* stream);
zinc_status zinc_server_release(zinc_server* srv, uint64_t ticket);
/* Progress until every submitted request has completed.  With retained
 * outputs, ZINC_E_STATE if waiting requests can only be admitted after some
 * outputs are released. */
zinc_status zinc_server_drain(zinc_server* srv);
/* Waits for the server's streams, then frees its resources. */
zinc_status zinc_server_destroy(zinc_server* srv);

/* Open-loop replay of an arrival trace: creates a server, submits request r
 * when the clock reaches arrival_ns[r] (nanoseconds after the replay starts,
 * non-decreasing), runs zinc_server_progress in between, drains, and writes
 * per-request times (relative to the replay start, submit_ns = the scheduled
 * arrival) to times[n_req].  retain_outputs must be 0. */
zinc_status zinc_serve_trace(zinc_ctx* const* ctxs, uint32_t n_ctx, const zinc_server_config* cfg,
                             const zinc_request* reqs, const uint64_t* arrival_ns, uint32_t n_req,
                             zinc_request_times* times);

/* ---- tuning ----------------------------------------------------------------
 * Three per-context choices change speed, never results: every combination
 * gives bit-identical ciphertexts.
 *   tile[s]        coefficients per thread of the fused encode + encrypt kernel
 *                  that zinc_encrypt_slots runs for scheme s (0 vanilla,
 *                  1 Zinc): 16 (default, every N), 8 (N = 4096 and 8192) or 32
 *                  (N <= 16384).  N = 32768 has the single value 16.
 *   reg_epilogue   bit s set: scheme s stores each transform straight from the
 *                  registers of its last pass (runs of consecutive
 *                  coefficients per thread) instead of through LDS in natural
 *                  order; N <= 16384, with 8 or 16 coefficients per thread.
 *   ntt_fp64_mask  limbs whose forward NTT runs in exact FP64 arithmetic
 *                  instead of 64-bit integer arithmetic; only limbs with a
 *                  modulus below 2^50 may be set (default: all of those).
 * Both need exclusive use of the context (no kernel of it in flight); the
 * arithmetic choice also applies to plans and servers using the context. */
typedef struct zinc_tuning {
    uint32_t tile[2];
    uint32_t ntt_fp64_mask;
    uint32_t reg_epilogue;
} zinc_tuning;

typedef struct zinc_tune_result {
    zinc_tuning chosen;
    uint32_t from_cache;        /* 1: applied from the cache file, nothing timed */
    uint32_t n_timed;           /* configurations timed                        */
    double best_ms[2];          /* one batch, chosen configuration, per scheme  */
    double default_ms[2];       /* one batch, default configuration (0: scheme
                                   not timed)                                  */
} zinc_tune_result;

/* ZINC_E_INVAL for a form the ring degree does not have or a mask bit on a
 * limb whose modulus is 2^50 or more. */
zinc_status zinc_set_tuning(zinc_ctx* ctx, const zinc_tuning* t);
zinc_status zinc_get_tuning(const zinc_ctx* ctx, zinc_tuning* t);
/* Time every combination of forms and arithmetic on `batch` (1..65536)
 * plaintexts of N/2 slots uniform on [-1, 1) (a fixed pseudo-random sequence)
 * with zinc_encrypt_slots (vanilla, and Zinc when
 * precomputed), on a private stream with HIP events (after 200 ms of
 * untimed launches; each candidate's best, over two sweeps, median of 9 runs
 * after 2 warm-up runs), and keep the fastest; candidates are tried default form
 * first, and a later one is kept only if more than 1% faster, so that
 * near-ties resolve the same way each time.  cache_path (may be NULL) names a
 * text file of earlier results keyed by device architecture, CU count, ring
 * degree, moduli and batch: a matching entry is applied without timing, and a
 * new result is added to the file.  Synchronous; needs keys
 * (ZINC_E_STATE before zinc_keygen). */
zinc_status zinc_autotune(zinc_ctx* ctx, uint32_t batch, const char* cache_path, zinc_tune_result* out);

/* ---- kernel-level entry points (parity testing of single steps) ---------- */

/* In-place forward / inverse negacyclic NTT of d_poly [n_polys][N] modulo the
 * context's modulus `limb` (0..M-1), in the order described above. */
zinc_status zinc_ntt_forward(zinc_ctx* ctx, uint32_t limb, uint64_t* d_poly, uint32_t n_polys,
                             void* stream);
zinc_status zinc_ntt_inverse(zinc_ctx* ctx, uint32_t limb, uint64_t* d_poly, uint32_t n_polys,
                             void* stream);

/* Draw the samplers' output for `batch` identifiers: kind 0 = R_2 ternary,
 * kind 1 = chi, as int64 [batch][N]; kind 2 = R_q uniform for modulus `limb`,
 * as uint64 [batch][N].  `tag` is the stream tag (1..255). */
zinc_status zinc_sample(zinc_ctx* ctx, int kind, uint32_t tag, uint32_t limb,
                        const uint64_t* d_ct_ids, uint32_t batch, void* d_out, void* stream);

/* Measurement aid: the device's peak rate of the forward transform's
 * butterfly, the roofline denominator of the fused encryption kernels (an
 * encryption's cost is its transforms, Theoretical Analysis section).  A
 * full-occupancy grid keeps 16 residues per thread in registers and runs
 * rounds of four radix-2 stages with the library's own butterfly: arith 0 =
 * 64-bit Shoup with the lazy reduction every fourth stage (moduli in
 * [2^20, 2^60)), arith 1 = exact FP64 (moduli in [2^20, 2^50)); twiddles are
 * wave-uniform, nothing touches memory until a final checksum.  Synchronous:
 * 200 ms of untimed launches, then `reps` (1..1000) launches timed with HIP
 * events; *bfly_per_s = butterflies per second of the median launch. */
zinc_status zinc_butterfly_rate(int arith, uint64_t q, uint32_t reps, double* bfly_per_s);

/* Copy the device-resident keys and cache (device-to-device, on `stream`):
 * secret key s_hat [M][N], public key [2][M][N], cached Enc(0) [2][L][N]. */
zinc_status zinc_export_keys(zinc_ctx* ctx, uint64_t* d_sk, uint64_t* d_pk, uint64_t* d_zero,
                             void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ZINC_H */
