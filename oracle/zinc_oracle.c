/*
 * zinc_oracle.c -- plain, slow, obviously-correct CPU oracle for batched CKKS
 * encryption ("vanilla", Eq. 8) and Zinc encryption (Algorithm 1) of
 * "At Least Factor-of-Two Optimization for RWLE-Based Homomorphic Encryption"
 * (arXiv 2408.07304).
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  Only tests/, the package smoke check and
 * the CPU-baseline leg of bench.py may load it.  The GPU library shares no code,
 * header, table or constant with it.
 *
 * Conventions (readings of the paper where it is silent are marked [S]):
 *   - Ring Z_q[X]/(X^N+1), RNS over primes q_0..q_{M-1}; the last prime is the
 *     special prime: present in sk/pk (M limbs), absent from ciphertexts and
 *     plaintexts (L = M-1 limbs).  [S]
 *   - Arithmetic mod q uses unsigned __int128 products and '%'.
 *   - NTT ("DFT" of the Evaluation section): a_hat[k] = sum_i a_i psi^((2 brv(k)+1) i)
 *     with psi the smallest primitive 2N-th root of unity mod q.  [S]
 *   - Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = seed,
 *     counter = (block, tag | limb<<8, ct_id lo, ct_id hi).  [S]
 *   - Ternary R_2: x = floor(3 w / 2^32) - 1 from one 32-bit word; coefficient
 *     k uses word k/(N/4) of block k mod N/4.  [S]
 *   - chi (sigma = 3.2, Polynomials and Distributions): discrete Gaussian on
 *     [-19, 19] by cumulative-table inversion of one 64-bit uniform (half
 *     k/(N/2) of block k mod N/2); the table is an input (computed by the
 *     Python side of the oracle).  [S]
 *   - Encoding: canonical embedding with slot j <-> root zeta^(5^j mod 2N),
 *     zeta = exp(i pi / N), real slots, round half to even.  [S]
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef unsigned __int128 u128;

#define ORACLE_KEY_ID  0xFFFFFFFFFFFFFFFFull
#define ORACLE_ZERO_ID 0xFFFFFFFFFFFFFFFEull

enum { TAG_SK = 1, TAG_A = 2, TAG_EPK = 3, TAG_U = 4, TAG_E1 = 5, TAG_E2 = 6,
       TAG_E1Z = 7, TAG_E2Z = 8 };

/* ------------------------------------------------------------------------ */
/* modular arithmetic (Polynomials and Distributions: [.]_q)                 */
/* ------------------------------------------------------------------------ */

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a * b) % q);
}

static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a + b) % q);
}

static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a + q - (b % q)) % q);
}

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulmod(r, b, q);
        b = mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}

/* residue of a signed integer */
static uint64_t smod(int64_t x, uint64_t q) {
    if (x >= 0) return (uint64_t)x % q;
    uint64_t r = ((uint64_t)(-(x + 1)) % q);   /* -(x+1) >= 0, avoids INT64_MIN overflow */
    /* x = -(r' + 1) with r' = -(x+1); x mod q = q - 1 - (r' mod q) */
    return q - 1 - r;
}

uint64_t oracle_mulmod(uint64_t a, uint64_t b, uint64_t q) { return mulmod(a, b, q); }
uint64_t oracle_powmod(uint64_t b, uint64_t e, uint64_t q) { return powmod(b, e, q); }

/* Deterministic Miller-Rabin: with the first twelve primes as bases the test
 * is exact for every n < 3.3e24 (Sorenson and Webster, "Strong pseudoprimes to
 * twelve prime bases", Math. Comp. 2017), hence for every 64-bit n. */
int oracle_is_prime(uint64_t n) {
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        uint64_t x = powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int witness = 1;
        for (int r = 1; r < s; r++) {
            x = mulmod(x, x, n);
            if (x == n - 1) { witness = 0; break; }
        }
        if (witness) return 0;
    }
    return 1;
}

/* Moduli [S]: for each requested bit size b, in order, the largest prime
 * q < 2^b with q = 1 (mod 2N) not already chosen.  Returns 0 on success. */
int oracle_choose_moduli(uint32_t log_n, uint32_t count, const uint32_t* bits, uint64_t* out) {
    uint64_t two_n = 2ull << log_n;
    for (uint32_t i = 0; i < count; i++) {
        if (bits[i] < log_n + 2 || bits[i] > 62) return -1;
        uint64_t top = 1ull << bits[i];
        /* largest value < 2^b that is = 1 mod 2N */
        uint64_t c = ((top - 1) / two_n) * two_n + 1;
        if (c >= top) c -= two_n;
        int found = 0;
        while (c > two_n) {
            if (oracle_is_prime(c)) {
                int used = 0;
                for (uint32_t j = 0; j < i; j++) if (out[j] == c) used = 1;
                if (!used) { out[i] = c; found = 1; break; }
            }
            c -= two_n;
        }
        if (!found) return -2;
    }
    return 0;
}

/* psi [S]: the smallest primitive 2N-th root of unity mod q.  With g the
 * smallest quadratic non-residue, psi0 = g^((q-1)/2N) has order exactly 2N
 * (Euler's criterion gives psi0^N = -1); the primitive 2N-th roots are the odd
 * powers of psi0. */
uint64_t oracle_find_psi(uint64_t q, uint32_t log_n) {
    uint64_t n = 1ull << log_n, two_n = 2 * n;
    if ((q - 1) % two_n != 0) return 0;
    uint64_t g = 2;
    while (powmod(g, (q - 1) / 2, q) != q - 1) g++;
    uint64_t psi0 = powmod(g, (q - 1) / two_n, q);
    uint64_t psi0_sq = mulmod(psi0, psi0, q);
    uint64_t cur = psi0, best = psi0;
    for (uint64_t k = 1; k < n; k++) {
        cur = mulmod(cur, psi0_sq, q);
        if (cur < best) best = cur;
    }
    return best;
}

static uint32_t bitrev(uint32_t x, uint32_t bits) {
    uint32_t r = 0;
    for (uint32_t i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

/* Forward negacyclic NTT, textbook in-place Cooley-Tukey over a table of psi
 * powers in bit-reversed order.  Input: coefficients in natural order.
 * Output: a_hat[k] = sum_i a_i psi^((2 brv(k)+1) i), canonical in [0, q). */
void oracle_ntt_forward(uint64_t* a, uint32_t log_n, uint64_t q, uint64_t psi) {
    uint32_t n = 1u << log_n;
    uint64_t* tab = (uint64_t*)malloc(sizeof(uint64_t) * n);
    for (uint32_t k = 0; k < n; k++) tab[k] = powmod(psi, bitrev(k, log_n), q);
    uint32_t t = n;
    for (uint32_t m = 1; m < n; m <<= 1) {
        t >>= 1;
        for (uint32_t i = 0; i < m; i++) {
            uint64_t w = tab[m + i];
            for (uint32_t j = 2 * i * t; j < 2 * i * t + t; j++) {
                uint64_t u = a[j] % q;
                uint64_t v = mulmod(a[j + t], w, q);
                a[j] = addmod(u, v, q);
                a[j + t] = submod(u, v, q);
            }
        }
    }
    free(tab);
}

/* Inverse of oracle_ntt_forward: Gentleman-Sande with psi^-1 powers in
 * bit-reversed order, then multiplication by N^-1. */
void oracle_ntt_inverse(uint64_t* a, uint32_t log_n, uint64_t q, uint64_t psi) {
    uint32_t n = 1u << log_n;
    uint64_t psi_inv = powmod(psi, q - 2, q);
    uint64_t* tab = (uint64_t*)malloc(sizeof(uint64_t) * n);
    for (uint32_t k = 0; k < n; k++) tab[k] = powmod(psi_inv, bitrev(k, log_n), q);
    uint32_t t = 1;
    for (uint32_t m = n; m > 1; m >>= 1) {
        uint32_t h = m >> 1;
        for (uint32_t i = 0; i < h; i++) {
            uint64_t w = tab[h + i];
            for (uint32_t j = 2 * i * t; j < 2 * i * t + t; j++) {
                uint64_t u = a[j] % q, v = a[j + t] % q;
                a[j] = addmod(u, v, q);
                a[j + t] = mulmod(submod(u, v, q), w, q);
            }
        }
        t <<= 1;
    }
    uint64_t n_inv = powmod(n % q, q - 2, q);
    for (uint32_t j = 0; j < n; j++) a[j] = mulmod(a[j], n_inv, q);
    free(tab);
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 Philox round  */
/* with the multipliers and Weyl key increments given in that paper.          */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_block(uint64_t seed, uint64_t ct_id, uint32_t tag, uint32_t limb,
                         uint32_t block, uint32_t out[4]) {
    uint32_t ctr[4] = {block, (tag & 0xFFu) | ((limb & 0xFFu) << 8), (uint32_t)ct_id,
                       (uint32_t)(ct_id >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* R_2 (ternary, uniform on {-1,0,1}; Polynomials and Distributions).
 * n is a multiple of 4; coefficient k takes word k / (n/4) of block k mod (n/4). */
void oracle_sample_ternary(uint64_t seed, uint64_t ct_id, uint32_t tag, uint32_t n, int64_t* out) {
    uint32_t quarter = n / 4;
    for (uint32_t k = 0; k < n; k++) {
        uint32_t w[4];
        philox_block(seed, ct_id, tag, 0, k % quarter, w);
        uint64_t v = ((uint64_t)3 * w[k / quarter]) >> 32;
        out[k] = (int64_t)v - 1;
    }
}

/* chi: discrete Gaussian on [-19, 19]; x = -19 + #{i : U >= T[i]}.
 * n is even; coefficient k takes the 64-bit half k / (n/2) of block k mod (n/2). */
void oracle_sample_gaussian(uint64_t seed, uint64_t ct_id, uint32_t tag, uint32_t n,
                            const uint64_t cdt[38], int64_t* out) {
    uint32_t half = n / 2;
    for (uint32_t k = 0; k < n; k++) {
        uint32_t w[4];
        philox_block(seed, ct_id, tag, 0, k % half, w);
        uint32_t h = 2 * (k / half);
        uint64_t u = (uint64_t)w[h] | ((uint64_t)w[h + 1] << 32);
        int64_t cnt = 0;
        for (int i = 0; i < 38; i++) cnt += (u >= cdt[i]) ? 1 : 0;
        out[k] = cnt - 19;
    }
}

/* R_q (uniform, Polynomials and Distributions), drawn per limb from a 128-bit
 * uniform reduced mod q. */
void oracle_sample_uniform(uint64_t seed, uint64_t ct_id, uint32_t tag, uint32_t limb, uint32_t n,
                           uint64_t q, uint64_t* out) {
    for (uint32_t k = 0; k < n; k++) {
        uint32_t w[4];
        philox_block(seed, ct_id, tag, limb, k, w);
        u128 v = (u128)w[0] | ((u128)w[1] << 32) | ((u128)w[2] << 64) | ((u128)w[3] << 96);
        out[k] = (uint64_t)(v % q);
    }
}

/* ------------------------------------------------------------------------ */
/* the scheme                                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t log_n;
    uint32_t n_moduli;       /* M: data limbs plus the special prime */
    uint64_t seed;
    double scale;            /* Delta */
    uint64_t q[32];
    uint64_t psi[32];
    uint64_t cdt[38];
    uint64_t noise_t;        /* BGV (Eq. 13): every error polynomial is scaled by t;
                                1 for CKKS and BFV */
} oracle_params;

/* residue of a Gaussian error coefficient as the scheme uses it: x, or t x
 * for BGV (Eq. 13 scales the errors of the key, of Enc and of Zinc's e') */
static uint64_t noise_mod(const oracle_params* p, int64_t x, uint64_t q) {
    return smod(x * (int64_t)(p->noise_t ? p->noise_t : 1), q);
}

/* Gen (Eq. 7): s <- R_2, a <- R_q, e <- chi;  pk1 = [-a s + e]_q, pk2 = a.
 * Outputs: s_hat [M][N] (NTT domain), pk [2][M][N] (NTT domain). */
void oracle_keygen(const oracle_params* p, uint64_t* s_hat, uint64_t* pk) {
    uint32_t n = 1u << p->log_n, M = p->n_moduli;
    int64_t* s = (int64_t*)malloc(sizeof(int64_t) * n);
    int64_t* e = (int64_t*)malloc(sizeof(int64_t) * n);
    uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * n);
    oracle_sample_ternary(p->seed, ORACLE_KEY_ID, TAG_SK, n, s);
    oracle_sample_gaussian(p->seed, ORACLE_KEY_ID, TAG_EPK, n, p->cdt, e);
    for (uint32_t l = 0; l < M; l++) {
        uint64_t q = p->q[l];
        uint64_t* sh = s_hat + (size_t)l * n;
        uint64_t* pk1 = pk + (size_t)l * n;
        uint64_t* pk2 = pk + ((size_t)M + l) * n;
        for (uint32_t k = 0; k < n; k++) sh[k] = smod(s[k], q);
        oracle_ntt_forward(sh, p->log_n, q, p->psi[l]);
        oracle_sample_uniform(p->seed, ORACLE_KEY_ID, TAG_A, l, n, q, pk2);  /* a, NTT domain */
        for (uint32_t k = 0; k < n; k++) tmp[k] = noise_mod(p, e[k], q);
        oracle_ntt_forward(tmp, p->log_n, q, p->psi[l]);
        for (uint32_t k = 0; k < n; k++)
            pk1[k] = addmod(submod(0, mulmod(pk2[k], sh[k], q), q), tmp[k], q);
    }
    free(s); free(e); free(tmp);
}

/* Vanilla encryption (Eq. 8, reading pk_2 in c_2 as the correctness proof does):
 * c1 = [pk1 u + e1 + m]_q, c2 = [pk2 u + e2]_q over the L data limbs.
 * pt [L][N] coefficient-domain residues; pk [2][M][N]; ct [2][L][N] NTT domain. */
void oracle_encrypt_vanilla(const oracle_params* p, const uint64_t* pk, const uint64_t* pt,
                            uint64_t ct_id, uint64_t* ct) {
    uint32_t n = 1u << p->log_n, M = p->n_moduli, L = M - 1;
    int64_t* u = (int64_t*)malloc(sizeof(int64_t) * n);
    int64_t* e1 = (int64_t*)malloc(sizeof(int64_t) * n);
    int64_t* e2 = (int64_t*)malloc(sizeof(int64_t) * n);
    uint64_t* uh = (uint64_t*)malloc(sizeof(uint64_t) * n);
    oracle_sample_ternary(p->seed, ct_id, TAG_U, n, u);
    oracle_sample_gaussian(p->seed, ct_id, TAG_E1, n, p->cdt, e1);
    oracle_sample_gaussian(p->seed, ct_id, TAG_E2, n, p->cdt, e2);
    for (uint32_t l = 0; l < L; l++) {
        uint64_t q = p->q[l];
        const uint64_t* pk1 = pk + (size_t)l * n;
        const uint64_t* pk2 = pk + ((size_t)M + l) * n;
        uint64_t* c1 = ct + (size_t)l * n;
        uint64_t* c2 = ct + ((size_t)L + l) * n;
        for (uint32_t k = 0; k < n; k++) uh[k] = smod(u[k], q);
        oracle_ntt_forward(uh, p->log_n, q, p->psi[l]);
        for (uint32_t k = 0; k < n; k++) c1[k] = addmod(pt[(size_t)l * n + k], noise_mod(p, e1[k], q), q);
        oracle_ntt_forward(c1, p->log_n, q, p->psi[l]);
        for (uint32_t k = 0; k < n; k++) c2[k] = noise_mod(p, e2[k], q);
        oracle_ntt_forward(c2, p->log_n, q, p->psi[l]);
        for (uint32_t k = 0; k < n; k++) {
            c1[k] = addmod(mulmod(pk1[k], uh[k], q), c1[k], q);
            c2[k] = addmod(mulmod(pk2[k], uh[k], q), c2[k], q);
        }
    }
    free(u); free(e1); free(e2); free(uh);
}

/* Vanilla encryption as a library with a special prime computes it (the
 * paper's CPU baseline is SEAL, whose chain ends in such a prime p = q_{M-1};
 * Eq. 8 read over the whole chain): the public-key encryption of zero over all
 * M limbs, a_j = pk_j u + e_j (j = 1, 2), is divided by p with rounding,
 * a_j' = round(a_j / p) coefficient-wise, which leaves the L data limbs, and
 * then the message is added: c1 = a1' + m, c2 = a2'.  Rounding in RNS: with
 * r = a_j mod p (coefficients in [0, p)), h = (p - 1) / 2 and
 * t = (r + h) mod p, round(a_j / p) = (a_j + h - t) / p, an exact division,
 * so limb l gets (a_j + (h - t)) p^-1 mod q_l.
 * pk [2][M][N]; pt [L][N] coefficient domain; ct [2][L][N] NTT domain. */
void oracle_encrypt_vanilla_sp(const oracle_params* p, const uint64_t* pk, const uint64_t* pt,
                               uint64_t ct_id, uint64_t* ct) {
    uint32_t n = 1u << p->log_n, M = p->n_moduli, L = M - 1;
    uint64_t qp = p->q[L], h = (qp - 1) / 2;
    int64_t* u = (int64_t*)malloc(sizeof(int64_t) * n);
    int64_t* e[2];
    e[0] = (int64_t*)malloc(sizeof(int64_t) * n);
    e[1] = (int64_t*)malloc(sizeof(int64_t) * n);
    uint64_t* a = (uint64_t*)malloc(sizeof(uint64_t) * 2 * (size_t)M * n);   /* [2][M][N] */
    uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * n);
    int64_t* d = (int64_t*)malloc(sizeof(int64_t) * n);
    oracle_sample_ternary(p->seed, ct_id, TAG_U, n, u);
    oracle_sample_gaussian(p->seed, ct_id, TAG_E1, n, p->cdt, e[0]);
    oracle_sample_gaussian(p->seed, ct_id, TAG_E2, n, p->cdt, e[1]);
    /* encryption of zero over the whole chain, NTT domain */
    for (uint32_t l = 0; l < M; l++) {
        uint64_t q = p->q[l];
        uint64_t* uh = tmp;
        for (uint32_t k = 0; k < n; k++) uh[k] = smod(u[k], q);
        oracle_ntt_forward(uh, p->log_n, q, p->psi[l]);
        for (int j = 0; j < 2; j++) {
            uint64_t* aj = a + ((size_t)j * M + l) * n;
            const uint64_t* pkj = pk + ((size_t)j * M + l) * n;
            for (uint32_t k = 0; k < n; k++) aj[k] = noise_mod(p, e[j][k], q);
            oracle_ntt_forward(aj, p->log_n, q, p->psi[l]);
            for (uint32_t k = 0; k < n; k++) aj[k] = addmod(mulmod(pkj[k], uh[k], q), aj[k], q);
        }
    }
    /* division by p with rounding, then the message */
    for (int j = 0; j < 2; j++) {
        memcpy(tmp, a + ((size_t)j * M + L) * n, sizeof(uint64_t) * n);
        oracle_ntt_inverse(tmp, p->log_n, qp, p->psi[L]);                  /* r = a_j mod p */
        for (uint32_t k = 0; k < n; k++) {
            uint64_t t = addmod(tmp[k], h, qp);
            d[k] = (int64_t)h - (int64_t)t;                                   /* h - t */
        }
        for (uint32_t l = 0; l < L; l++) {
            uint64_t q = p->q[l], pinv = powmod(qp % q, q - 2, q);
            for (uint32_t k = 0; k < n; k++) tmp[k] = smod(d[k], q);
            oracle_ntt_forward(tmp, p->log_n, q, p->psi[l]);
            uint64_t* out = ct + ((size_t)j * L + l) * n;
            const uint64_t* aj = a + ((size_t)j * M + l) * n;
            for (uint32_t k = 0; k < n; k++) out[k] = mulmod(addmod(aj[k], tmp[k], q), pinv, q);
            if (j == 0) {
                memcpy(tmp, pt + (size_t)l * n, sizeof(uint64_t) * n);
                oracle_ntt_forward(tmp, p->log_n, q, p->psi[l]);
                for (uint32_t k = 0; k < n; k++) out[k] = addmod(out[k], tmp[k], q);
            }
        }
    }
    free(u); free(e[0]); free(e[1]); free(a); free(tmp); free(d);
}

/* Zinc precomputation: the cached Enc(0) is a vanilla encryption of the zero
 * plaintext under the reserved identifier ZERO_ID. */
void oracle_zinc_precompute(const oracle_params* p, const uint64_t* pk, uint64_t* zero) {
    uint32_t n = 1u << p->log_n, L = p->n_moduli - 1;
    uint64_t* pt = (uint64_t*)calloc((size_t)L * n, sizeof(uint64_t));
    oracle_encrypt_vanilla(p, pk, pt, ORACLE_ZERO_ID, zero);
    free(pt);
}

/* Zinc encryption (Algorithm 1): c = zero + m; e1', e2' <- chi;
 * c' = ([c1 + e1']_q, [c2 + e2']_q).  All three additions are carried out in
 * the NTT domain in which the cached zero is stored. */
void oracle_encrypt_zinc(const oracle_params* p, const uint64_t* zero, const uint64_t* pt,
                         uint64_t ct_id, uint64_t* ct) {
    uint32_t n = 1u << p->log_n, L = p->n_moduli - 1;
    int64_t* e1 = (int64_t*)malloc(sizeof(int64_t) * n);
    int64_t* e2 = (int64_t*)malloc(sizeof(int64_t) * n);
    uint64_t* mh = (uint64_t*)malloc(sizeof(uint64_t) * n);
    uint64_t* eh = (uint64_t*)malloc(sizeof(uint64_t) * n);
    oracle_sample_gaussian(p->seed, ct_id, TAG_E1Z, n, p->cdt, e1);
    oracle_sample_gaussian(p->seed, ct_id, TAG_E2Z, n, p->cdt, e2);
    for (uint32_t l = 0; l < L; l++) {
        uint64_t q = p->q[l];
        const uint64_t* z1 = zero + (size_t)l * n;
        const uint64_t* z2 = zero + ((size_t)L + l) * n;
        uint64_t* c1 = ct + (size_t)l * n;
        uint64_t* c2 = ct + ((size_t)L + l) * n;
        /* step 1: c = zero + m */
        memcpy(mh, pt + (size_t)l * n, sizeof(uint64_t) * n);
        oracle_ntt_forward(mh, p->log_n, q, p->psi[l]);
        for (uint32_t k = 0; k < n; k++) { c1[k] = addmod(z1[k], mh[k], q); c2[k] = z2[k]; }
        /* steps 2-3: add fresh e1', e2' */
        for (uint32_t k = 0; k < n; k++) eh[k] = noise_mod(p, e1[k], q);
        oracle_ntt_forward(eh, p->log_n, q, p->psi[l]);
        for (uint32_t k = 0; k < n; k++) c1[k] = addmod(c1[k], eh[k], q);
        for (uint32_t k = 0; k < n; k++) eh[k] = noise_mod(p, e2[k], q);
        oracle_ntt_forward(eh, p->log_n, q, p->psi[l]);
        for (uint32_t k = 0; k < n; k++) c2[k] = addmod(c2[k], eh[k], q);
    }
    free(e1); free(e2); free(mh); free(eh);
}

/* The element-wise step of Zinc encryption on its own (Algorithm 1, steps 1
 * and 3, in the NTT domain where the cached zero is kept): given
 * hat = (NTT(m + e1'), NTT(e2')) as [2][L][N] residues, ct = [zero + hat]_q. */
void oracle_elementwise_zinc(const oracle_params* p, const uint64_t* zero, const uint64_t* hat, uint64_t* ct) {
    uint32_t n = 1u << p->log_n, L = p->n_moduli - 1;
    for (uint32_t j = 0; j < 2; j++)
        for (uint32_t l = 0; l < L; l++) {
            size_t o = ((size_t)j * L + l) * n;
            for (uint32_t k = 0; k < n; k++) ct[o + k] = addmod(zero[o + k], hat[o + k], p->q[l]);
        }
}

/* The element-wise step of vanilla encryption on its own (Eq. 8 in the NTT
 * domain): given u_hat = NTT(u) [L][N] and hat = (NTT(m + e1), NTT(e2)) as
 * [2][L][N], c1 = [pk1 u_hat + hat1]_q and c2 = [pk2 u_hat + hat2]_q over the
 * L data limbs (pk [2][M][N]). */
void oracle_elementwise_vanilla(const oracle_params* p, const uint64_t* pk, const uint64_t* uhat,
                                const uint64_t* hat, uint64_t* ct) {
    uint32_t n = 1u << p->log_n, M = p->n_moduli, L = M - 1;
    for (uint32_t l = 0; l < L; l++) {
        uint64_t q = p->q[l];
        const uint64_t* pk1 = pk + (size_t)l * n;
        const uint64_t* pk2 = pk + ((size_t)M + l) * n;
        const uint64_t* u = uhat + (size_t)l * n;
        for (uint32_t k = 0; k < n; k++) {
            ct[(size_t)l * n + k] = addmod(mulmod(pk1[k], u[k], q), hat[(size_t)l * n + k], q);
            ct[((size_t)L + l) * n + k] = addmod(mulmod(pk2[k], u[k], q), hat[((size_t)L + l) * n + k], q);
        }
    }
}

/* Decryption (Dec(c) = [c1 + c2 sk]_q): p = INTT(c1 + c2 s_hat) per data limb. */
void oracle_decrypt(const oracle_params* p, const uint64_t* s_hat, const uint64_t* ct, uint64_t* pt) {
    uint32_t n = 1u << p->log_n, L = p->n_moduli - 1;
    for (uint32_t l = 0; l < L; l++) {
        uint64_t q = p->q[l];
        const uint64_t* c1 = ct + (size_t)l * n;
        const uint64_t* c2 = ct + ((size_t)L + l) * n;
        uint64_t* o = pt + (size_t)l * n;
        for (uint32_t k = 0; k < n; k++) o[k] = addmod(c1[k], mulmod(c2[k], s_hat[(size_t)l * n + k], q), q);
        oracle_ntt_inverse(o, p->log_n, q, p->psi[l]);
    }
}

/* Homomorphic addition of two ciphertexts (Eq. 2): component-wise mod q. */
void oracle_add(const oracle_params* p, const uint64_t* a, const uint64_t* b, uint64_t* out) {
    uint32_t n = 1u << p->log_n, L = p->n_moduli - 1;
    for (uint32_t l = 0; l < 2 * L; l++)
        for (uint32_t k = 0; k < n; k++)
            out[(size_t)l * n + k] = addmod(a[(size_t)l * n + k], b[(size_t)l * n + k], p->q[l % L]);
}

/* ------------------------------------------------------------------------ */
/* CKKS encoding / decoding by the canonical-embedding definition             */
/* ------------------------------------------------------------------------ */

/* slot exponent r_j = 5^j mod 2N */
static void slot_exponents(uint32_t log_n, uint64_t* r) {
    uint64_t two_n = 2ull << log_n, half = 1ull << (log_n - 1), g = 1;
    for (uint64_t j = 0; j < half; j++) { r[j] = g; g = (g * 5) % two_n; }
}

/* Encode: x_i = (2 Delta / N) * sum_j z_j cos(pi * (i r_j mod 2N) / N), the
 * real polynomial whose value at zeta^(r_j) is Delta z_j (and at the conjugate
 * root, Delta conj(z_j)).  Slots beyond n_slots are zero.  Extended-precision
 * accumulation; m_i = x_i rounded half to even; frac_out[i] = x_i - m_i. */
void oracle_encode(const oracle_params* p, const double* z, uint32_t n_slots,
                   int64_t* m_out, double* frac_out) {
    uint32_t n = 1u << p->log_n, half = n / 2;
    uint64_t two_n = 2ull * n;
    uint64_t* r = (uint64_t*)malloc(sizeof(uint64_t) * half);
    long double* c = (long double*)malloc(sizeof(long double) * two_n);
    slot_exponents(p->log_n, r);
    const long double pi = 3.14159265358979323846264338327950288L;
    for (uint64_t k = 0; k < two_n; k++) c[k] = cosl(pi * (long double)k / (long double)n);
    long double f = 2.0L * (long double)p->scale / (long double)n;
    for (uint32_t i = 0; i < n; i++) {
        long double acc = 0.0L;
        for (uint32_t j = 0; j < n_slots && j < half; j++)
            acc += (long double)z[j] * c[((uint64_t)i * r[j]) % two_n];
        long double x = f * acc;
        long double mr = rintl(x);
        m_out[i] = (int64_t)mr;
        if (frac_out) frac_out[i] = (double)(x - mr);
    }
    free(r); free(c);
}

/* Decode: z_j = Re m(zeta^(r_j)) / Delta = sum_i m_i cos(pi (i r_j mod 2N) / N) / Delta
 * for a centred integer polynomial m (real parts; the imaginary parts are
 * zero for real-slot encodings). */
void oracle_decode(const oracle_params* p, const int64_t* m, double* z_out) {
    uint32_t n = 1u << p->log_n, half = n / 2;
    uint64_t two_n = 2ull * n;
    uint64_t* r = (uint64_t*)malloc(sizeof(uint64_t) * half);
    long double* c = (long double*)malloc(sizeof(long double) * two_n);
    slot_exponents(p->log_n, r);
    const long double pi = 3.14159265358979323846264338327950288L;
    for (uint64_t k = 0; k < two_n; k++) c[k] = cosl(pi * (long double)k / (long double)n);
    for (uint32_t j = 0; j < half; j++) {
        long double acc = 0.0L;
        for (uint32_t i = 0; i < n; i++) acc += (long double)m[i] * c[((uint64_t)i * r[j]) % two_n];
        z_out[j] = (double)(acc / (long double)p->scale);
    }
    free(r); free(c);
}

/* Plaintext polynomial from a signed integer polynomial: residues per data limb. */
void oracle_to_rns(const oracle_params* p, const int64_t* m, uint32_t n_limbs, uint64_t* pt) {
    uint32_t n = 1u << p->log_n;
    for (uint32_t l = 0; l < n_limbs; l++)
        for (uint32_t k = 0; k < n; k++) pt[(size_t)l * n + k] = smod(m[k], p->q[l]);
}

/* Whole path for one plaintext vector: encode, residues, encrypt (scheme 0 =
 * vanilla with pk, scheme 1 = Zinc with the cached zero). */
void oracle_encrypt_slots(const oracle_params* p, int scheme, const uint64_t* pk_or_zero,
                          const double* z, uint32_t n_slots, uint64_t ct_id, uint64_t* ct) {
    uint32_t n = 1u << p->log_n, L = p->n_moduli - 1;
    int64_t* m = (int64_t*)malloc(sizeof(int64_t) * n);
    uint64_t* pt = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)L * n);
    oracle_encode(p, z, n_slots, m, NULL);
    oracle_to_rns(p, m, L, pt);
    if (scheme == 0) oracle_encrypt_vanilla(p, pk_or_zero, pt, ct_id, ct);
    else if (scheme == 2) oracle_encrypt_vanilla_sp(p, pk_or_zero, pt, ct_id, ct);
    else oracle_encrypt_zinc(p, pk_or_zero, pt, ct_id, ct);
    free(m); free(pt);
}
