// Host-side number theory and table construction for the parameter sets:
// the moduli rule, the 2N-th roots of unity, Shoup companions and the
// cumulative table of the discrete Gaussian chi (Polynomials and
// Distributions: sigma = 3.2).
#include <cstring>

#include "zinc_internal.h"

namespace zinc {

typedef unsigned __int128 u128;

uint64_t mulmod_host(uint64_t a, uint64_t b, uint64_t q) {
    return static_cast<uint64_t>(static_cast<u128>(a) * b % q);
}

uint64_t powmod_host(uint64_t b, uint64_t e, uint64_t q) {
    uint64_t acc = 1 % q, base = b % q;
    for (; e; e >>= 1) {
        if (e & 1) acc = mulmod_host(acc, base, q);
        base = mulmod_host(base, base, q);
    }
    return acc;
}

// Strong-probable-prime test to the seven bases found by J. Sinclair, which
// together admit no composite below 2^64 (a deterministic test for uint64).
bool is_prime(uint64_t n) {
    if (n < 4) return n >= 2;
    if ((n & 1) == 0) return false;
    for (uint64_t p : {3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull})
        if (n % p == 0) return n == p;
    uint64_t odd = n - 1;
    unsigned twos = __builtin_ctzll(odd);
    odd >>= twos;
    static const uint64_t kBases[7] = {2, 325, 9375, 28178, 450775, 9780504, 1795265022};
    for (uint64_t a : kBases) {
        uint64_t b = a % n;
        if (b == 0) continue;
        uint64_t x = powmod_host(b, odd, n);
        if (x == 1 || x == n - 1) continue;
        bool composite = true;
        for (unsigned i = 1; i < twos && composite; ++i) {
            x = mulmod_host(x, x, n);
            if (x == n - 1) composite = false;
        }
        if (composite) return false;
    }
    return true;
}

// For every requested bit size b (in order): the largest prime q < 2^b with
// q = 1 (mod 2N) that is not already in the chain.
bool choose_moduli(uint32_t log_n, uint32_t count, const uint32_t* bits, uint64_t* out) {
    const uint64_t step = 2ull << log_n;
    for (uint32_t i = 0; i < count; ++i) {
        const uint64_t limit = 1ull << bits[i];
        uint64_t cand = (limit - 1) - ((limit - 1) % step) + 1;  // largest value = 1 mod 2N, <= 2^b
        if (cand >= limit) cand -= step;
        bool ok = false;
        for (; cand > step; cand -= step) {
            if (!is_prime(cand)) continue;
            bool dup = false;
            for (uint32_t j = 0; j < i; ++j) dup |= (out[j] == cand);
            if (dup) continue;
            out[i] = cand;
            ok = true;
            break;
        }
        if (!ok) return false;
    }
    return true;
}

// The smallest primitive 2N-th root of unity modulo q.  An element x has order
// exactly 2N iff x^N = -1.  Starting from any such root r, every primitive
// 2N-th root is r^(2k+1); the minimum over k is returned.
uint64_t smallest_psi(uint64_t q, uint32_t log_n) {
    const uint64_t n = 1ull << log_n;
    if ((q - 1) % (2 * n) != 0) return 0;
    uint64_t r = 0;
    for (uint64_t g = 2; g < q; ++g) {
        uint64_t cand = powmod_host(g, (q - 1) / (2 * n), q);
        if (powmod_host(cand, n, q) == q - 1) { r = cand; break; }
    }
    if (r == 0) return 0;
    const uint64_t r2 = mulmod_host(r, r, q);
    uint64_t best = r, cur = r;
    for (uint64_t k = 1; k < n; ++k) {
        cur = mulmod_host(cur, r2, q);
        if (cur < best) best = cur;
    }
    return best;
}

// floor(w * 2^64 / q) for w < q: the Shoup companion of w.
uint64_t shoup_companion(uint64_t w, uint64_t q) {
    return static_cast<uint64_t>((static_cast<u128>(w) << 64) / q);
}

// exp(-t) for 0 <= t < 64 in binary128: Taylor series of exp(-t / 2^10) to
// 24 terms, then ten squarings.  Relative error below 1e-30.
static __float128 exp_neg_q(__float128 t) {
    __float128 a = -t / 1024;
    __float128 term = 1, sum = 1;
    for (int k = 1; k < 24; ++k) {
        term = term * a / k;
        sum += term;
    }
    for (int i = 0; i < 10; ++i) sum = sum * sum;
    return sum;
}

// Cumulative table of chi: rho(x) = exp(-x^2 / (2 sigma^2)) on |x| <= 19,
// T[i] = floor(2^64 * sum_{x <= -19 + i} rho(x) / sum_x rho(x)), i < 38.
// A 64-bit uniform U maps to x = -19 + #{i : U >= T[i]}.
void gaussian_cdt(double sigma, uint64_t out[kCdtLen]) {
    // sigma is taken as the decimal the caller meant (3.2), not its binary
    // double, so that the table is the one of the real number 3.2.
    __float128 s = static_cast<__float128>(static_cast<long long>(sigma * 1000000.0 + 0.5)) / 1000000;
    __float128 rho[2 * kTail + 1];
    __float128 total = 0;
    for (int x = -kTail; x <= kTail; ++x) {
        __float128 xf = x;
        rho[x + kTail] = exp_neg_q(xf * xf / (2 * s * s));
    }
    // sum from the tails inward, the smaller terms first
    for (int i = 0; i <= kTail - 1; ++i) total += rho[i] + rho[2 * kTail - i];
    total += rho[kTail];
    __float128 two64 = 18446744073709551616.0Q;
    __float128 acc = 0;
    for (int i = 0; i < kCdtLen; ++i) {
        acc += rho[i];
        __float128 v = two64 * acc / total;
        out[i] = static_cast<uint64_t>(v);
    }
}

// First-level table of the chi sampler.  For a 64-bit uniform U in bucket
// b = U >> 56 the count #{i : U >= T[i]} is lo_b + #{i : b 2^56 < T[i] <= U},
// lo_b = #{i : T[i] <= b 2^56}.  Entry b: bits [0, 56) the low bits of the
// bucket's one interior threshold (0 if it has none), bits [56, 62) the base
// count (lo_b, or lo_b - 1 without an interior threshold, so that the one
// comparison U >= (b << 56 | low bits) always adds 1), bit 63 set when the
// bucket holds two or more interior thresholds (the device then searches the
// whole table).
void gaussian_buckets(const uint64_t cdt[kCdtLen], uint64_t out[kCdtBuckets]) {
    for (int b = 0; b < kCdtBuckets; ++b) {
        const uint64_t start = (uint64_t)b << kCdtShift;
        uint64_t lo = 0, inner = 0, thr = 0;
        for (int i = 0; i < kCdtLen; ++i) {
            if (cdt[i] <= start) ++lo;
            else if ((cdt[i] >> kCdtShift) == (uint64_t)b) { ++inner; thr = cdt[i]; }
        }
        if (inner == 1) out[b] = (lo << 56) | (thr & kCdtLowMask);
        else if (inner == 0 && lo > 0) out[b] = (lo - 1) << 56;
        else out[b] = 1ull << 63;
    }
}

}  // namespace zinc
