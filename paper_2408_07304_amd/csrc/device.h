// Device building blocks for gfx950: 64-bit modular arithmetic (Shoup),
// Philox4x32-10, the three samplers, the register/LDS negacyclic NTT and the
// FP64 FFT of the CKKS canonical embedding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "zinc_internal.h"

namespace zinc {

typedef uint64_t u64;

// ---------------------------------------------------------------------------
// modular arithmetic.  All moduli are below 2^60, so values up to 4q fit in
// 64 bits with room for Harvey's lazy reduction.
// ---------------------------------------------------------------------------

// y * w mod q in [0, 2q), for any y < 2^64, w < q, wp = floor(w 2^64 / q).
__device__ __forceinline__ u64 shoup_lazy(u64 y, u64 w, u64 wp, u64 q) {
    // high word of y wp from 32-bit pieces: each partial sum fits in 64 bits
    const uint32_t yl = (uint32_t)y, yh = (uint32_t)(y >> 32), pl = (uint32_t)wp, ph = (uint32_t)(wp >> 32);
    const u64 m1 = (u64)yl * ph + __umulhi(yl, pl);
    const u64 m2 = (u64)yh * pl + (uint32_t)m1;
    const u64 hi = (u64)yh * ph + (m1 >> 32) + (m2 >> 32);
    return y * w - hi * q;
}

__device__ __forceinline__ u64 csub(u64 x, u64 m) { return x >= m ? x - m : x; }

__device__ __forceinline__ u64 addmod(u64 a, u64 b, u64 q) { return csub(a + b, q); }

// residue of a signed 64-bit integer with |x| < 2^63
__device__ __forceinline__ u64 reduce_signed(long long x, const LimbConst& lc) {
    const u64 a = x < 0 ? (u64)(-x) : (u64)x;
    u64 r = csub(a - __umul64hi(a, lc.bar) * lc.q, lc.q);
    return (x < 0 && r != 0) ? lc.q - r : r;
}

// reduce_signed with a cheap path for |x| < q (q < 2^62), the usual size of
// an encoded message coefficient plus noise
__device__ __forceinline__ u64 reduce_signed_near(long long x, const LimbConst& lc) {
    const long long q = (long long)lc.q;
    if (x > -q && x < q) return (u64)(x < 0 ? x + q : x);
    return reduce_signed(x, lc);
}

// residue of a small signed integer (|x| < q)
__device__ __forceinline__ u64 small_mod(int x, u64 q) {
    return x < 0 ? q - (u64)(unsigned)(-x) : (u64)(unsigned)x;
}

// Cooley-Tukey butterfly with lazy reduction (moduli below 2^60, so 16 q fits
// in 64 bits): the Shoup product t = y w mod q lies in [0, 2q) for any 64-bit
// y, so (a + t, a - t + 2q) exceed the bound of a by at most 2q.  RED: first
// bring x from [0, 16q) into [0, 8q); otherwise a = x.  ntt_fwd places the
// reductions so that no value reaches 16q (see fwd_reduce).
template <bool RED>
__device__ __forceinline__ void ct_bfly(u64& x, u64& y, u64 w, u64 wp, u64 q, u64 q2, u64 q8) {
    const u64 a = RED ? csub(x, q8) : x;
    const u64 t = shoup_lazy(y, w, wp, q);
    x = a + t;
    y = a - t + q2;
}

// Stage j (0-based) of an integer forward transform whose inputs lie in
// [0, 4q): without reductions the bound after j stages is (4 + 2j) q, so the
// first reduction is due at stage 6 (bound 16q) and then every fourth stage
// (8q + 4 * 2q).  Outputs lie in [0, 16q).
__host__ __device__ constexpr bool fwd_reduce(int j) { return j >= 6 && (j - 6) % 4 == 0; }

// [0, 16q) -> [0, q)
__device__ __forceinline__ u64 canon16(u64 x, u64 q) {
    return csub(csub(csub(csub(x, q << 3), q << 2), q << 1), q);
}

// Gentleman-Sande butterfly: x, y in [0, 2q) -> (x + y, (x - y) w) in [0, 2q).
__device__ __forceinline__ void gs_bfly(u64& x, u64& y, u64 w, u64 wp, u64 q, u64 q2) {
    const u64 a = csub(x + y, q2);
    const u64 d = x - y + q2;
    y = shoup_lazy(d, w, wp, q);
    x = a;
}

// remainder of (hi 2^64 + lo) by q (hi < q): restoring long division.  Slow;
// used only at key generation.
__device__ __forceinline__ u64 mod128(u64 hi, u64 lo, u64 q) {
    u64 r = hi;
    for (int i = 63; i >= 0; --i) {
        const u64 top = r >> 63;
        r = (r << 1) | ((lo >> i) & 1);
        if (top || r >= q) r -= q;
    }
    return r;
}

// floor(w 2^64 / q) for w < q (Shoup companion), by long division.
__device__ __forceinline__ u64 shoup_companion_dev(u64 w, u64 q) {
    u64 r = w, quo = 0;
    for (int i = 63; i >= 0; --i) {
        const u64 top = r >> 63;
        r <<= 1;
        quo <<= 1;
        if (top || r >= q) { r -= q; quo |= 1; }
    }
    return quo;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter (c0, c1, c2, c3),
// key (k0, k1); ten rounds, Weyl key schedule.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                     uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product each (a single v_mad_u64_u32) and
        // one three-input XOR each (v_bitop3_b32, truth table 0x96)
        const u64 p0 = (u64)0xD2511F53u * c0, p1 = (u64)0xCD9E8D57u * c2;
        c0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        c1 = (uint32_t)p1;
        c2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ U4 draw(u64 seed, u64 ct_id, uint32_t tag, uint32_t limb, uint32_t block) {
    return philox(block, (tag & 0xFFu) | ((limb & 0xFFu) << 8), (uint32_t)ct_id,
                  (uint32_t)(ct_id >> 32), (uint32_t)seed, (uint32_t)(seed >> 32));
}

// chi: x = -19 + #{i < 38 : U >= T[i]}, the count by a branch-free binary
// search over the table padded to 64 entries with 2^64-1 (tab in LDS,
// ascending).  After the six steps pos is the number of entries <= u, except
// that it stops at 63; the pads can only be <= u when u = 2^64-1, where every
// real threshold is counted, so the count of real thresholds is min(pos, 38).
__device__ __forceinline__ int gauss_bsearch(u64 u, const u64* tab) {
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t step = 32; step >= 1; step >>= 1) pos += (u >= tab[pos + step - 1]) ? step : 0u;
    return (int)(pos < (uint32_t)kCdtLen ? pos : (uint32_t)kCdtLen) - kTail;
}

// The same value with one lookup in the bucket table that follows the
// thresholds in tab (built by the host's gaussian_buckets): within bucket
// b = u >> 54 (1024 buckets) all but the two tail buckets hold at most one
// threshold above the bucket's start, which is compared in full 64 bits; the
// tail buckets, flagged in bit 63, fall back to the search.  An entry holds
// the count of thresholds at or below the bucket's start in bits 56..61 and
// the inner threshold's low 54 bits.  With 1024 buckets a wave of 64 lanes
// takes the fallback on about 12 % of its draws (256 buckets: 40 %).
__device__ __forceinline__ int gauss_sample(u64 u, const u64* tab) {
    const u64 e = tab[kCdtPad + (uint32_t)(u >> kCdtShift)];
    const u64 thr = (u & ~kCdtLowMask) | (e & kCdtLowMask);
    int x = (int)((e >> 56) & 63u) + (u >= thr ? 1 : 0) - kTail;
    if (e >> 63) x = gauss_bsearch(u, tab);
    return x;
}

// Copy the sampler's table (kCdtTab words) to LDS; blockDim.x threads.
__device__ __forceinline__ void load_cdt(u64* tab, const u64* __restrict__ cdt, uint32_t t) {
    for (uint32_t i = t; i < (uint32_t)kCdtTab; i += blockDim.x) tab[i] = cdt[i];
    __syncthreads();
}

// R_2: x = floor(3 w / 2^32) - 1
__device__ __forceinline__ int ternary_from(uint32_t w) { return (int)__umulhi(w, 3u) - 1; }

// ---------------------------------------------------------------------------
// NTT geometry: N = 2^LOGN coefficients over T = 2^LOGT threads, R = N/T per
// thread in registers.  The log N stages are split into NPASS passes of at
// most LOGR stages; pass p acts on index bits [LO(p), H(p)).  In pass p,
// thread t holds the R indices formed by putting the pass's active bits (the
// low K(p) bits of the register number c) at [LO, H) and the remaining bits --
// first the thread id, then the high bits of c -- at the other positions,
// lowest first.  Passes are joined by exchanges through LDS.
// ---------------------------------------------------------------------------
template <int LOGN_, int LOGT_>
struct Geom {
    static constexpr int LOGN = LOGN_, LOGT = LOGT_;
    static constexpr int N = 1 << LOGN, T = 1 << LOGT;
    static constexpr int LOGR = LOGN - LOGT, R = 1 << LOGR;
    static constexpr int NPASS = (LOGN + LOGR - 1) / LOGR;
    static constexpr int H_ = N / 2;
    __host__ __device__ static constexpr int K(int p) { return LOGN / NPASS + (p < LOGN % NPASS ? 1 : 0); }
    __host__ __device__ static constexpr int H(int p) { return p == 0 ? LOGN : H(p - 1) - K(p - 1); }
    __host__ __device__ static constexpr int LO(int p) { return H(p) - K(p); }
    __host__ __device__ static constexpr uint32_t spread(int p, uint32_t na) {
        return (na & ((1u << LO(p)) - 1u)) | ((na >> LO(p)) << H(p));
    }
    __host__ __device__ static constexpr uint32_t cpart(int p, int c) {
        return ((uint32_t)(c & ((1 << K(p)) - 1)) << LO(p)) |
               spread(p, (uint32_t)(c >> K(p)) << LOGT);
    }
    __device__ static __forceinline__ uint32_t tpart(int p, uint32_t t) { return spread(p, t); }
    static_assert(LOGR >= 2, "at least 4 coefficients per thread");
    static_assert(LOGN / NPASS + (LOGN % NPASS ? 1 : 0) <= LOGR, "pass wider than a thread's registers");
};

// LDS layout: one 8-byte pad word after every 16 words.  pad() is additive
// over index parts with disjoint bits, so a thread's per-register addresses are
// its base address plus compile-time offsets (instruction immediates), and the
// strided access patterns of the passes spread over all banks.
__host__ __device__ constexpr uint32_t pad(uint32_t i) { return i + (i >> 4); }
template <int N>
struct LdsWords { static constexpr int value = N + N / 16; };

// An integer the compiler cannot see through: address arithmetic derived from
// it is recomputed inside each transform instead of being hoisted out of the
// per-limb loop and held in registers across it, and loads through different
// instances are not merged.
__device__ __forceinline__ uint32_t opaque_tid(uint32_t t) {
    asm volatile("" : "+v"(t));
    return t;
}
__device__ __forceinline__ uint32_t opaque_s(uint32_t x) {   // x must be wave-uniform
    x = (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
    asm volatile("" : "+s"(x));
    return x;
}

// The part of thread t's index that selects twiddles in pass P.  Twiddle
// indices drop every index bit below the butterfly's bit, so when the pass's
// active bits lie above the 64 lane bits (LO >= 6) the twiddles are uniform
// across the wavefront: the index is then taken from the first lane, which puts
// it in scalar registers (and, with uniform_tw, the loads on the scalar path).
template <class G, int P>
__device__ __forceinline__ uint32_t tw_tpart(uint32_t t) {
    constexpr int LO = G::LO(P), HH = G::H(P);
    if constexpr (P == 0) {
        return 0u;
    } else if constexpr (LO >= 6) {
        return (uint32_t)__builtin_amdgcn_readfirstlane((int)(t >> LO)) << HH;
    } else {
        return G::tpart(P, t);
    }
}

// Twiddle index of the butterfly on local bit b of register c in pass P.
// For a whole transform (smul = 1) it is 2^s + g for stage s and group g.  A
// transform of 2N coefficients whose first stage has been applied splits into
// two independent N-point transforms (the halves h = 0, 1); their stage s and
// group g use index (2 + h) 2^s + g of the 2N-point table (smul = 2 + h).
template <class G, int P>
__device__ __forceinline__ uint32_t tw_index(uint32_t tp, int c, int b, uint32_t smul) {
    constexpr int LO = G::LO(P), HH = G::H(P), K = G::K(P);
    const int s = G::LOGN - HH + (K - 1 - b);          // stage within this transform
    return (smul << s) + ((tp | G::cpart(P, c)) >> (LO + b + 1));
}

// An exchange between the layouts of passes P1 and P2 stays inside each
// wavefront when the wave-number bits of the thread id (those above its 64
// lanes) sit on the same index bits in both layouts: every wave then owns the
// same indices, hence the same LDS words, before and after.  The LDS executes
// a wave's instructions in order, so such an exchange needs no workgroup
// barrier, only a compiler barrier that keeps the wave's reads after its
// writes.
template <class G>
__host__ __device__ constexpr bool wave_local(int p1, int p2) {
    for (int b = 6; b < G::LOGT; ++b)
        if (G::spread(p1, 1u << b) != G::spread(p2, 1u << b)) return false;
    return true;
}

// Compiler barrier for LDS accesses exchanged within one wavefront.
__device__ __forceinline__ void wave_lds_fence() { asm volatile("" ::: "memory"); }

template <class G, int P, class T>
__device__ __forceinline__ void lds_put(T* lds, const T (&v)[G::R], uint32_t t) {
    T* base = lds + pad(G::tpart(P, t));
#pragma unroll
    for (int c = 0; c < G::R; ++c) base[pad(G::cpart(P, c))] = v[c];
}

template <class G, int P, class T>
__device__ __forceinline__ void lds_get(const T* lds, T (&v)[G::R], uint32_t t) {
    const T* base = lds + pad(G::tpart(P, t));
#pragma unroll
    for (int c = 0; c < G::R; ++c) v[c] = base[pad(G::cpart(P, c))];
}

// v from the layout of pass P1 to that of pass P2 through LDS: within each
// wavefront when the layouts allow it (wave_local), else with workgroup
// barriers before the writes (earlier readers of the words are done) and
// after them.
template <class G, int P1, int P2, class T>
__device__ __forceinline__ void exchange(T* lds, T (&v)[G::R], uint32_t t) {
    // A forward transform's first exchange follows LDS use of the caller (often
    // reads in natural order, across waves): it must take barriers.  With
    // K(0) + K(1) above log R it always does.
    static_assert(!(P1 == 0 && P2 == 1) || !wave_local<G>(0, 1), "first exchange must take barriers");
    if constexpr (wave_local<G>(P1, P2)) {
        wave_lds_fence();
        lds_put<G, P1>(lds, v, t);
        wave_lds_fence();
    } else {
        __syncthreads();
        lds_put<G, P1>(lds, v, t);
        __syncthreads();
    }
    lds_get<G, P2>(lds, v, t);
}


// A twiddle and its companion (Shoup factor, or w/q) are adjacent in the
// tables at an even index: one 16-byte load.
typedef u64 u64x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u64x2 load_pair(const u64* p) { return *reinterpret_cast<const u64x2*>(p); }
__device__ __forceinline__ f64x2 load_pair(const double* p) { return *reinterpret_cast<const f64x2*>(p); }

// Passes whose twiddle index is the same in every lane (see tw_tpart).  With
// 16 or more coefficients per thread their twiddles are read through the
// constant address space (the tables are never written while a kernel runs),
// which lets the compiler use scalar loads and keeps them off the vector
// memory path (vanilla at N = 8192: 2 % faster).  With 8 per thread the
// scalar loads, which share a wait counter with the LDS exchanges, measured
// slightly slower, so those geometries keep vector loads.
template <class G, int P>
__device__ __forceinline__ constexpr bool uniform_tw() { return G::R >= 16 && (P == 0 || G::LO(P) >= 6); }
__device__ __forceinline__ u64x2 load_pair_uniform(const u64* p) {
    return *(const __attribute__((address_space(4))) u64x2*)(p);
}
__device__ __forceinline__ f64x2 load_pair_uniform(const double* p) {
    return *(const __attribute__((address_space(4))) f64x2*)(p);
}
template <class G, int P, class T>
__device__ __forceinline__ auto load_tw(const T* p) {
    if constexpr (uniform_tw<G, P>()) return load_pair_uniform(p);
    else return load_pair(p);
}

// The twiddles of the first stage of forward pass P, requested ahead of the
// exchange into the pass's layout so that their latency overlaps the LDS
// round trip (and, on the FP64 path, the optional reduction's branch, behind
// which no load of the pass could otherwise start).  w[c] is set for the
// registers c that start a butterfly of that stage; registers sharing a
// twiddle share one load.  Only for 16 coefficients per thread in workgroups
// of at most 512 threads: measured 2 % faster at N = 8192; with 1024 threads
// (N = 16384) the registers held across the exchange spill, and with 8 per
// thread it gains nothing.
template <class G>
__host__ __device__ constexpr bool preload_tw() { return G::R == 16 && G::T <= 512; }
template <class G, int P, class T>
struct FirstTw {
    typename std::conditional<std::is_same<T, double>::value, f64x2, u64x2>::type w[G::R];
};
template <class G, int P, class T>
__device__ __forceinline__ FirstTw<G, P, T> first_tw(const T* __restrict__ tw, uint32_t toff, uint32_t smul,
                                                      uint32_t t) {
    constexpr int b = G::K(P) - 1;
    const uint32_t tp = tw_tpart<G, P>(t);
    FirstTw<G, P, T> r;
#pragma unroll
    for (int c = 0; c < G::R; ++c)
        if (!(c & (1 << b))) r.w[c] = load_tw<G, P>(tw + toff + 2 * tw_index<G, P>(tp, c, b, smul));
    return r;
}

// ---- integer path (any modulus below 2^60): Shoup butterflies, lazy bounds ----

template <class G, int P>
__device__ __forceinline__ void fwd_pass(u64 (&v)[G::R], uint32_t t, const u64* __restrict__ tw,
                                         uint32_t toff, uint32_t smul, u64 q, u64 q2,
                                         const FirstTw<G, P, u64>* w0 = nullptr) {
    constexpr int K = G::K(P);
    const uint32_t tp = tw_tpart<G, P>(t);
    const u64 q8 = q << 3;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int b = K - 1 - i;
        constexpr int J0 = G::LOGN - G::H(P);            // stages before this pass
#pragma unroll
        for (int c = 0; c < G::R; ++c) {
            if (c & (1 << b)) continue;
            const uint32_t ti = toff + 2 * tw_index<G, P>(tp, c, b, smul);
            const u64x2 w = w0 && i == 0 ? w0->w[c] : load_tw<G, P>(tw + ti);
            if (fwd_reduce(J0 + i)) ct_bfly<true>(v[c], v[c | (1 << b)], w.x, w.y, q, q2, q8);
            else ct_bfly<false>(v[c], v[c | (1 << b)], w.x, w.y, q, q2, q8);
        }
    }
}

template <class G, int P>
__device__ __forceinline__ void inv_pass(u64 (&v)[G::R], uint32_t t, const u64* __restrict__ itw,
                                         uint32_t toff, uint32_t smul, u64 q, u64 q2) {
    constexpr int K = G::K(P);
    const uint32_t tp = tw_tpart<G, P>(t);
#pragma unroll
    for (int b = 0; b < K; ++b) {
#pragma unroll
        for (int c = 0; c < G::R; ++c) {
            if (c & (1 << b)) continue;
            const uint32_t ti = toff + 2 * tw_index<G, P>(tp, c, b, smul);
            const u64x2 w = load_tw<G, P>(itw + ti);
            gs_bfly(v[c], v[c | (1 << b)], w.x, w.y, q, q2);
        }
    }
}

template <class G, int P>
__device__ __forceinline__ void fwd_rest(u64 (&v)[G::R], u64* lds, const u64* __restrict__ tw, uint32_t toff,
                                         uint32_t smul, u64 q, u64 q2, uint32_t t) {
    if constexpr (P < G::NPASS) {
        if constexpr (preload_tw<G>()) {
            const auto w0 = first_tw<G, P>(tw, toff, smul, t);
            exchange<G, P - 1, P>(lds, v, t);
            fwd_pass<G, P>(v, t, tw, toff, smul, q, q2, &w0);
        } else {
            exchange<G, P - 1, P>(lds, v, t);
            fwd_pass<G, P>(v, t, tw, toff, smul, q, q2);
        }
        fwd_rest<G, P + 1>(v, lds, tw, toff, smul, q, q2, t);
    }
}

// Forward NTT modulo q of limb `limb`: v in pass-0 layout with values in
// [0, 4q) -> v in the last pass's layout with values in [0, 16q) (canon16).  tw is the
// [M][NT][2] table of (psi^brv(k), Shoup companion) of NT-point transforms
// (NT = G::N, or 2 G::N for a half of a split transform, smul = 2 + half);
// lds the padded exchange buffer.
template <class G>
__device__ __forceinline__ void ntt_fwd(u64 (&v)[G::R], u64* lds, const u64* __restrict__ tw, uint32_t limb,
                                        u64 q, u64 q2, uint32_t t_, uint32_t smul = 1, uint32_t nt = G::N) {
    const uint32_t toff = opaque_s(limb * 2u * nt);
    const uint32_t t = opaque_tid(t_);
    fwd_pass<G, 0>(v, t, tw, toff, smul, q, q2);
    fwd_rest<G, 1>(v, lds, tw, toff, smul, q, q2, t);
}

template <class G, int P>
__device__ __forceinline__ void inv_rest(u64 (&v)[G::R], u64* lds, const u64* __restrict__ itw, uint32_t toff,
                                         uint32_t smul, u64 q, u64 q2, uint32_t t) {
    if constexpr (P >= 0) {
        exchange<G, P + 1, P>(lds, v, t);
        inv_pass<G, P>(v, t, itw, toff, smul, q, q2);
        inv_rest<G, P - 1>(v, lds, itw, toff, smul, q, q2, t);
    }
}

// Inverse NTT without the N^-1 factor: v in the last pass's layout with values
// in [0, 2q) -> v in pass-0 layout with values in [0, 2q).  Table indexing as
// for ntt_fwd.
template <class G>
__device__ __forceinline__ void ntt_inv(u64 (&v)[G::R], u64* lds, const u64* __restrict__ itw, uint32_t limb,
                                        u64 q, u64 q2, uint32_t t_, uint32_t smul = 1, uint32_t nt = G::N) {
    constexpr int PL = G::NPASS - 1;
    const uint32_t toff = opaque_s(limb * 2u * nt);
    const uint32_t t = opaque_tid(t_);
    inv_pass<G, PL>(v, t, itw, toff, smul, q, q2);
    inv_rest<G, PL - 1>(v, lds, itw, toff, smul, q, q2, t);
}

// Write v (last forward pass layout) to LDS so that lds[pad(i)] is coefficient i,
// then a workgroup barrier: readers of the natural order span all waves.  Called
// straight after ntt_fwd / ntt_fwd_fp, whose last LDS accesses were each wave's
// reads of its own indices of the last pass -- the very words it now writes --
// while the other waves can still be reading only their own, disjoint, words.
// So no barrier is needed before the writes, only a compiler barrier that keeps
// them after those reads (a single-pass transform has no exchange and keeps the
// barrier).
template <class G, class T>
__device__ __forceinline__ void to_natural(T* lds, const T (&v)[G::R], uint32_t t_) {
    const uint32_t t = opaque_tid(t_);
    if constexpr (G::NPASS > 1) wave_lds_fence();
    else __syncthreads();
    lds_put<G, G::NPASS - 1>(lds, v, t);
    __syncthreads();
}

// The same writes with no barrier after them, for readers that take only their
// own wave's words (wave_pair_index): in the last pass a wave holds whole blocks
// of 64 * 2^K consecutive coefficients.  A later writer of other words must
// still take a workgroup barrier first, as a forward transform's first
// exchange and the encoder do.
template <class G, class T>
__device__ __forceinline__ void to_natural_wave(T* lds, const T (&v)[G::R], uint32_t t_) {
    static_assert(G::NPASS > 1, "follows the transform's last exchange");
    const uint32_t t = opaque_tid(t_);
    wave_lds_fence();
    lds_put<G, G::NPASS - 1>(lds, v, t);
    wave_lds_fence();
}

// Coefficient index of the i-th pair (i < R/2) that thread t takes after
// to_natural_wave: the pairs of each of its wave's blocks go to consecutive
// lanes, so each read, load and store of a pair by the wave covers 128
// consecutive coefficients.
template <class G>
__host__ __device__ __forceinline__ uint32_t wave_pair_index(uint32_t t, int i) {
    constexpr int PL = G::NPASS - 1, K = G::K(PL);
    static_assert(G::LO(PL) == 0 && K >= 1 && G::LOGT >= 6, "last pass covers bit 0");
    const uint32_t h = (uint32_t)i >> (K - 1), j = (uint32_t)i & ((1u << (K - 1)) - 1u);
    return (h << (G::LOGT + K)) | ((t >> 6) << (6 + K)) | (j << 7) | ((t & 63u) << 1);
}

// ---- FP64 path (moduli below 2^50): exact integer arithmetic in doubles ----
//
// MI355X issues FP64 FMA at the full VALU rate, so for moduli below 2^50 the
// butterfly runs on doubles holding exact signed integers.  With w < q and the
// rounded quotient wq = fl(w/q), for |y| < 2^53:
//   k = rint(y * wq), h = fl(y w), l = fma(y, w, -h) = y w - h exactly,
//   r = fma(-k, q, h) = h - k q exactly (|h - k q| < 2^53), t = r + l exactly,
// so t = y w - k q with |t| <= q (1/2 + |y| 2^-52), and x +- t is exact while
// it stays below 2^53.  A stage therefore raises a bound B on |x|, |y| to
// B + q (1/2 + B 2^-52).  Moduli below 2^47 are not reduced inside the
// transform: from inputs up to 2q + 64 (a residue, the cached Enc(0)'s
// coefficient and an error) every value stays below 2^52 over 15 stages.
// Moduli in [2^47, 2^50) are rounded into [-q/2 - 1, q/2 + 1] at the start
// of every pass but the first; with first-pass inputs up to q + 64 the
// values stay below 2^53 (the worst case, a five-stage first pass near
// q = 2^50, reaches about 2^52.4).  A CPU test propagates these bounds for
// every thread geometry.

#pragma clang fp contract(off)
__device__ __forceinline__ double fp_mulmod(double y, double w, double wq, double q) {
    const double k = __builtin_rint(y * wq);
    const double h = y * w;
    const double l = __builtin_fma(y, w, -h);
    const double r = __builtin_fma(-k, q, h);
    return r + l;
}

__device__ __forceinline__ void ct_bfly_fp(double& x, double& y, double w, double wq, double q) {
    const double t = fp_mulmod(y, w, wq, q);
    const double a = x;
    x = a + t;
    y = a - t;
}

// x - round(x / q) q, exact for |x| < 2^53: result in [-q/2 - 1, q/2 + 1].
__device__ __forceinline__ double fp_round_reduce(double x, double q, double qinv) {
    return __builtin_fma(-__builtin_rint(x * qinv), q, x);
}

// exact integer in (-2^52, 2^52) -> canonical residue in [0, q) as uint64
// (x * qinv is within 1.01/q of x/q, so the rounded quotient leaves |r| <=
// q/2 + 1, and one correction of the negative side gives [0, q).)
__device__ __forceinline__ u64 fp_canon(double x, double q, double qinv) {
    double r = __builtin_fma(-__builtin_rint(x * qinv), q, x);
    r = r < 0.0 ? r + q : r;
    return (u64)__double_as_longlong(r + 0x1p52) - 0x4330000000000000ull;
}

// uint64 below 2^52 -> double, exactly
__device__ __forceinline__ double u64_to_fp(u64 x) {
    return __longlong_as_double((long long)(x | 0x4330000000000000ull)) - 0x1p52;
}
#pragma clang fp contract(on)

template <class G, int P>
__device__ __forceinline__ void fwd_pass_fp(double (&v)[G::R], uint32_t t, const double* __restrict__ tw,
                                            uint32_t toff, uint32_t smul, double q, double qinv, bool reduce,
                                            const FirstTw<G, P, double>* w0 = nullptr) {
    constexpr int K = G::K(P);
    const uint32_t tp = tw_tpart<G, P>(t);
    if (reduce) {
#pragma unroll
        for (int c = 0; c < G::R; ++c) v[c] = fp_round_reduce(v[c], q, qinv);
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int b = K - 1 - i;
#pragma unroll
        for (int c = 0; c < G::R; ++c) {
            if (c & (1 << b)) continue;
            const uint32_t ti = toff + 2 * tw_index<G, P>(tp, c, b, smul);
            const f64x2 w = w0 && i == 0 ? w0->w[c] : load_tw<G, P>(tw + ti);
            ct_bfly_fp(v[c], v[c | (1 << b)], w.x, w.y, q);
        }
    }
}

template <class G, int P>
__device__ __forceinline__ void fwd_rest_fp(double (&v)[G::R], double* lds, const double* __restrict__ tw,
                                            uint32_t toff, uint32_t smul, double q, double qinv, bool reduce,
                                            uint32_t t) {
    if constexpr (P < G::NPASS) {
        if constexpr (preload_tw<G>()) {
            const auto w0 = first_tw<G, P>(tw, toff, smul, t);
            exchange<G, P - 1, P>(lds, v, t);
            fwd_pass_fp<G, P>(v, t, tw, toff, smul, q, qinv, reduce, &w0);
        } else {
            exchange<G, P - 1, P>(lds, v, t);
            fwd_pass_fp<G, P>(v, t, tw, toff, smul, q, qinv, reduce);
        }
        fwd_rest_fp<G, P + 1>(v, lds, tw, toff, smul, q, qinv, reduce, t);
    }
}

// Forward NTT in FP64: v in pass-0 layout, exact integers with |v| <= q ->
// v in the last pass's layout, exact integers congruent to the transform, with
// magnitude below 2^52.  tw_fp is the [M][NT][2] table of (psi^brv(k), its
// quotient by q) as doubles; table indexing as for ntt_fwd.
template <class G>
__device__ __forceinline__ void ntt_fwd_fp(double (&v)[G::R], double* lds, const double* __restrict__ tw,
                                           uint32_t limb, double q, double qinv, bool reduce, uint32_t t_,
                                           uint32_t smul = 1, uint32_t nt = G::N) {
    const uint32_t toff = opaque_s(limb * 2u * nt);
    const uint32_t t = opaque_tid(t_);
    fwd_pass_fp<G, 0>(v, t, tw, toff, smul, q, qinv, false);
    fwd_rest_fp<G, 1>(v, lds, tw, toff, smul, q, qinv, reduce, t);
}

// ---------------------------------------------------------------------------
// samplers in pass-0 layout.  Coefficient k of an N-draw of chi uses half
// k / (N/2) of Philox block k mod N/2; of R_2, word k / (N/4) of block
// k mod N/4.  In pass-0 layout the top two index bits are the top two active
// bits of the register number, so a thread owns every coefficient of the
// blocks it draws.
// ---------------------------------------------------------------------------
template <int R>
struct Packed8 {
    uint32_t w[R / 4];
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int i = 0; i < R / 4; ++i) w[i] = 0;
    }
    __device__ __forceinline__ void set(int c, int x) { w[c >> 2] |= ((uint32_t)(x & 0xFF)) << (8 * (c & 3)); }
    __device__ __forceinline__ int get(int c) const { return (int)(int8_t)(uint8_t)(w[c >> 2] >> (8 * (c & 3))); }
    // A copy whose words the compiler cannot see through, so that values
    // derived from the samples (conversions, residues) are computed where they
    // are used, not hoisted out of the per-limb loop and kept live.
    __device__ __forceinline__ Packed8 fresh() const {
        Packed8 r = *this;
#pragma unroll
        for (int i = 0; i < R / 4; ++i) asm volatile("" : "+v"(r.w[i]));
        return r;
    }
};

template <class G>
__device__ __forceinline__ void sample_gauss_p0(Packed8<G::R>& out, const DevParams& p, const u64* tab,
                                                u64 ct_id, uint32_t tag, uint32_t t) {
    constexpr int TOP = 1 << (G::K(0) - 1);
    const uint32_t tp = G::tpart(0, t);
    out.clear();
#pragma unroll
    for (int c = 0; c < G::R; ++c) {
        if (c & TOP) continue;
        const uint32_t k = tp | G::cpart(0, c);   // < N/2
        const U4 r = draw(p.seed, ct_id, tag, 0, k);
        out.set(c, gauss_sample((u64)r.x | ((u64)r.y << 32), tab));
        out.set(c | TOP, gauss_sample((u64)r.z | ((u64)r.w << 32), tab));
    }
}

template <class G>
__device__ __forceinline__ void sample_ternary_p0(Packed8<G::R>& out, const DevParams& p, u64 ct_id,
                                                  uint32_t tag, uint32_t t) {
    constexpr int SH = G::K(0) - 2;
    constexpr int TOP2 = 3 << SH;
    const uint32_t tp = G::tpart(0, t);
    out.clear();
#pragma unroll
    for (int c = 0; c < G::R; ++c) {
        if (c & TOP2) continue;
        const uint32_t k = tp | G::cpart(0, c);   // < N/4
        const U4 r = draw(p.seed, ct_id, tag, 0, k);
        out.set(c, ternary_from(r.x));
        out.set(c | (1 << SH), ternary_from(r.y));
        out.set(c | (2 << SH), ternary_from(r.z));
        out.set(c | (3 << SH), ternary_from(r.w));
    }
}

// ---------------------------------------------------------------------------
// FP64 FFT for the canonical embedding: radix-2 decimation in time over
// H = N/2 points held in LDS, input in bit-reversed order, output natural.
// sign = -1: F[i] = sum_k A[k] exp(-2 pi i k i / H); sign = +1: conjugate roots.
// ---------------------------------------------------------------------------
struct C2 {
    double x, y;
};

__device__ __forceinline__ C2 cmul(C2 a, C2 b) { return C2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// fft_tw holds exp(-2 pi i k / 2^LOGTAB) for k < 2^(LOGTAB-1); an FFT of
// 2^LOGH <= 2^LOGTAB points reads it with stride 2^(LOGTAB-LOGH).
template <int LOGH, int T, int SIGN, int LOGTAB = LOGH>
__device__ __forceinline__ void fft_dit(C2* A, const double* __restrict__ fft_tw, uint32_t t) {
    constexpr int H = 1 << LOGH;
#pragma unroll 1
    for (int s = 1; s <= LOGH; ++s) {
        const int half = 1 << (s - 1);
        for (int b = t; b < H / 2; b += T) {
            const int pos = b & (half - 1);
            const int i0 = ((b >> (s - 1)) << s) + pos, i1 = i0 + half;
            const int ti = pos << (LOGTAB - s);
            C2 w{fft_tw[2 * ti], fft_tw[2 * ti + 1]};
            if (SIGN > 0) w.y = -w.y;
            const C2 a = A[i0], bw = cmul(A[i1], w);
            A[i0] = C2{a.x + bw.x, a.y + bw.y};
            A[i1] = C2{a.x - bw.x, a.y - bw.y};
        }
        __syncthreads();
    }
}

// The same transform with its stages grouped into passes of LOGR = LOGH -
// log2(T) stages held in registers.  In pass p, bits [B, B + K) of an index
// (B = p LOGR, K = min(LOGR, LOGH - B)) come from a thread's register number
// and the other bits from its thread index (then its remaining register bits):
// every thread loads its 2^LOGR points, applies the pass's stages and stores
// them back to the same places, so one barrier per pass suffices (none between
// passes that keep each wave on its own words, see fft_wave_local).  Every
// butterfly performs the operations of fft_dit on the same values, so the
// result equals fft_dit's bit for bit, for any T.  A is indexed through padc().
// PARTIAL: the workgroup has more than T threads; all of them reach the
// barriers and only threads t < T work.
__host__ __device__ constexpr uint32_t padc(uint32_t i) { return i + (i >> 4); }
__host__ __device__ constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// Index bits of register e of thread t in pass P of fft_reg_pass.
template <int LOGH, int LOGT, int P>
struct FftPass {
    static constexpr int LOGR = LOGH - LOGT, R = 1 << LOGR;
    static constexpr int B = P * LOGR, K = (LOGH - B < LOGR) ? LOGH - B : LOGR;
    __host__ __device__ static __forceinline__ uint32_t idx(uint32_t t, int e) {
        const uint32_t c = (uint32_t)e & ((1u << K) - 1u), rest = t | ((uint32_t)(e >> K) << LOGT);
        return (rest & ((1u << B) - 1u)) | (c << B) | ((rest >> B) << (B + K));
    }
};

// Passes P and P + 1 touch the same words in each wavefront when every wave bit
// of the thread index (those above its 64 lanes) sits on the same index bit in
// both: a thread bit b lands on bit b below a pass's base B, else on b + K.
// Between such passes a wave reads back only its own stores, which the LDS
// executes in order, so no workgroup barrier is needed (as for wave_local).
template <int LOGH, int LOGT, int P>
__host__ __device__ constexpr bool fft_wave_local() {
    using F0 = FftPass<LOGH, LOGT, P>;
    using F1 = FftPass<LOGH, LOGT, P + 1>;
    for (int b = 6; b < LOGT; ++b)
        if ((b < F0::B ? b : b + F0::K) != (b < F1::B ? b : b + F1::K)) return false;
    return true;
}

// The twiddles of pass P, w[k][e] for stage k and the registers e that start
// a butterfly; they depend on the thread index only, so they are requested
// before the barrier that ends the previous pass and arrive while it waits.
template <int LOGH, int LOGT, int SIGN, int LOGTAB, int P>
struct FftTw {
    using F = FftPass<LOGH, LOGT, P>;
    C2 w[F::K > 0 ? F::K : 1][F::R];
};
template <int LOGH, int LOGT, int SIGN, int LOGTAB, int P>
__device__ __forceinline__ FftTw<LOGH, LOGT, SIGN, LOGTAB, P> fft_pass_tw(const double* __restrict__ fft_tw,
                                                                          uint32_t t) {
    using F = FftPass<LOGH, LOGT, P>;
    FftTw<LOGH, LOGT, SIGN, LOGTAB, P> r;
#pragma unroll
    for (int k = 0; k < F::K; ++k) {
        const int s = F::B + k + 1;
        const uint32_t half = 1u << (s - 1);
#pragma unroll
        for (int e = 0; e < F::R; ++e) {
            if (e & (1 << k)) continue;
            const uint32_t ti = (F::idx(t, e) & (half - 1u)) << (LOGTAB - s);   // < 2^(LOGTAB-1) for any t
            const f64x2 w = load_pair(fft_tw + 2 * ti);
            r.w[k][e] = C2{w.x, SIGN > 0 ? -w.y : w.y};
        }
    }
    return r;
}

template <int LOGH, int LOGT, int SIGN, int LOGTAB, int P, bool PARTIAL>
__device__ __forceinline__ void fft_reg_pass(C2* A, const double* __restrict__ fft_tw, uint32_t t,
                                             const FftTw<LOGH, LOGT, SIGN, LOGTAB, P>& tw) {
    using F = FftPass<LOGH, LOGT, P>;
    constexpr int R = F::R, K = F::K;
    if constexpr (F::B < LOGH) {
        const bool active = !PARTIAL || t < (1u << LOGT);
        if (active) {
            C2 v[R];
#pragma unroll
            for (int e = 0; e < R; ++e) v[e] = A[padc(F::idx(t, e))];
#pragma unroll
            for (int k = 0; k < K; ++k) {
#pragma unroll
                for (int e = 0; e < R; ++e) {
                    if (e & (1 << k)) continue;
                    const C2 a = v[e], bw = cmul(v[e | (1 << k)], tw.w[k][e]);
                    v[e] = C2{a.x + bw.x, a.y + bw.y};
                    v[e | (1 << k)] = C2{a.x - bw.x, a.y - bw.y};
                }
            }
#pragma unroll
            for (int e = 0; e < R; ++e) A[padc(F::idx(t, e))] = v[e];
        }
        FftTw<LOGH, LOGT, SIGN, LOGTAB, P + 1> next;
        if constexpr (F::B + F::LOGR < LOGH)
            if (active) next = fft_pass_tw<LOGH, LOGT, SIGN, LOGTAB, P + 1>(fft_tw, t);
        // the last pass's stores are read by every thread: a barrier
        if constexpr (F::B + F::LOGR < LOGH && fft_wave_local<LOGH, LOGT, P>()) wave_lds_fence();
        else __syncthreads();
        fft_reg_pass<LOGH, LOGT, SIGN, LOGTAB, P + 1, PARTIAL>(A, fft_tw, t, next);
    }
}

template <int LOGH, int T, int SIGN, int LOGTAB = LOGH, bool PARTIAL = false>
__device__ __forceinline__ void fft_dit_reg(C2* A, const double* __restrict__ fft_tw, uint32_t t) {
    static_assert((1 << ilog2(T)) == T && ilog2(T) < LOGH, "T must be a power of two below 2^LOGH");
    constexpr int LOGT = ilog2(T);
    FftTw<LOGH, LOGT, SIGN, LOGTAB, 0> tw0;
    if (!PARTIAL || t < (1u << LOGT)) tw0 = fft_pass_tw<LOGH, LOGT, SIGN, LOGTAB, 0>(fft_tw, t);
    fft_reg_pass<LOGH, LOGT, SIGN, LOGTAB, 0, PARTIAL>(A, fft_tw, t, tw0);
}

// CKKS encoding of one slot vector into the integer coefficients m held in
// pass-0 layout: place Delta z_j at position (5^j mod 2N - 1)/4 of a real
// N/2-point vector Z, transform, twist by zeta^-i and scale by 2/N;
// coefficient i < N/2 is the real part of entry i, coefficient i + N/2 its
// imaginary part; round half to even.  Z is real, so the transform runs on
// Y[k] = Z[2k] + i Z[2k+1] (Q = N/4 points) and is unscrambled: with Yf its
// transform, E[m] = (Yf[m] + conj Yf[Q-m]) / 2, O[m] = (Yf[m] - conj Yf[Q-m]) / 2i
// and F[m] = E[m mod Q] + exp(-2 pi i m / (N/2)) O[m mod Q].  The Q-point
// transform runs on Q/8 threads (8 points each, fewer passes); the others wait
// at its barriers.  A thread's registers c and c | TOP hold coefficients i and
// i + N/2, which come from the same entry F[i].  Uses lds (LdsWords<N> words)
// as the padded complex work array.
template <class G>
__device__ __forceinline__ void encode_p0(long long (&m)[G::R], u64* lds, const DevParams& p,
                                          const double* __restrict__ z, uint32_t n_slots, uint32_t t) {
    constexpr int H = G::N / 2, Q = H / 2, LOGH = G::LOGN - 1, LOGQ = LOGH - 1;
    constexpr int TF = Q / 8 < G::T ? Q / 8 : G::T;
    double* Ad = reinterpret_cast<double*>(lds);
    C2* A = reinterpret_cast<C2*>(lds);
    __syncthreads();
    for (uint32_t j = t; j < (uint32_t)H; j += G::T) {
        const double val = j < n_slots ? p.scale * z[j] : 0.0;
        const uint32_t bk = p.slot_pos[j];               // brv_{log H}(k_j)
        Ad[2 * padc(bk & (Q - 1)) + (bk >> (LOGH - 1))] = val;   // Y[k_j / 2] gets Z[k_j] in Re or Im
    }
    __syncthreads();
    fft_dit_reg<LOGQ, TF, -1, LOGH, (TF < G::T)>(A, p.fft_tw, t);
    const double f = 2.0 / (double)G::N;
    constexpr int TOP = 1 << (G::K(0) - 1);
    const uint32_t tp = G::tpart(0, t);
    bool bad = false;
    auto to_int = [&](double x) -> long long {
        x = __builtin_rint(x);
        // an integer below 2^51: adding 1.5 * 2^52 is exact and leaves it in
        // the low mantissa bits, read off with one 64-bit subtraction
        if (__builtin_fabs(x) < 0x1p51) return __double_as_longlong(x + 0x1.8p52) - 0x4338000000000000ll;
        if (!(__builtin_fabs(x) < 4611686018427387904.0)) {   // 2^62 (also catches NaN)
            bad = true;
            return 0;
        }
        return (long long)x;
    };
#pragma unroll
    for (int c = 0; c < G::R; ++c) {
        if (c & TOP) continue;
        const uint32_t i = tp | G::cpart(0, c);         // < H
        const uint32_t m1 = i & (Q - 1), m2 = (Q - m1) & (Q - 1);
        const C2 y1 = A[padc(m1)], y2 = A[padc(m2)];
        const C2 ev{0.5 * (y1.x + y2.x), 0.5 * (y1.y - y2.y)};     // (Y1 + conj Y2) / 2
        const C2 od{0.5 * (y1.y + y2.y), -0.5 * (y1.x - y2.x)};    // (Y1 - conj Y2) / 2i
        C2 w{p.fft_tw[2 * (i & (H / 2 - 1))], p.fft_tw[2 * (i & (H / 2 - 1)) + 1]};
        if (i >= (uint32_t)(H / 2)) {
            w.x = -w.x;
            w.y = -w.y;
        }
        const C2 o = cmul(w, od);
        const C2 F{ev.x + o.x, ev.y + o.y};
        const C2 r = cmul(F, C2{p.twist[2 * i], p.twist[2 * i + 1]});
        m[c] = to_int(r.x * f);
        m[c | TOP] = to_int(r.y * f);
    }
    if (bad) atomicOr(p.err, 1u);
}

// Encoding of slot vectors with at most kSparseSlots values, for the encoding
// kernels: entry i of the N/2-point transform of the real vector Z (Delta z_j
// at position k_j) is F[i] = sum_j Delta z_j exp(-2 pi i k_j i / (N/2)),
// evaluated term by term from the root table (exp(-2 pi i x / (N/2)) for
// x < N/4, the negation of the entry x - N/4 above; k_j from slot_pos, which
// holds brv(k_j)); no LDS, no barriers.  Measured on 1024 rows: one value
// 23 % (N = 8192) and 8 % (N = 32768, where writing the residues dominates)
// faster than the transform, three values 9 % and 2 %; with four values the
// transform was as fast.  The fused encryption kernels keep the transform for
// every vector: there the encoding is a small share of the launch, and the
// extra code cost registers (scratch spills in the split and plan kernels).
constexpr uint32_t kSparseSlots = 3;
template <int LOGH>
__device__ __forceinline__ C2 sparse_transform(const DevParams& p, const double* __restrict__ z, uint32_t n_slots,
                                               uint32_t i) {
    constexpr uint32_t H = 1u << LOGH;
    C2 F{0.0, 0.0};
#pragma unroll
    for (uint32_t j = 0; j < kSparseSlots; ++j) {
        if (j >= n_slots) break;
        const double a = p.scale * z[j];
        const uint32_t k = __brev(p.slot_pos[j]) >> (32 - LOGH);
        const uint32_t x = (k * i) & (H - 1), xs = x & (H / 2 - 1);
        const f64x2 w = load_pair(p.fft_tw + 2 * xs);
        const double sg = x >= H / 2 ? -a : a;
        F.x += sg * w.x;
        F.y += sg * w.y;
    }
    return F;
}

// Coefficients i and i + N/2 of the encoding from entry F[i] of the
// transform: twist by zeta^-i, scale by 2/N, round half to even; false when
// a value is out of range (|x| >= 2^62 or NaN), which then encodes as 0.
__device__ __forceinline__ bool encode_pair(const DevParams& p, uint32_t i, C2 F, double f, long long& lo,
                                            long long& hi) {
    const C2 r = cmul(F, C2{p.twist[2 * i], p.twist[2 * i + 1]});
    const double xl = __builtin_rint(r.x * f), xh = __builtin_rint(r.y * f);
    const bool okl = __builtin_fabs(xl) < 4611686018427387904.0, okh = __builtin_fabs(xh) < 4611686018427387904.0;
    lo = okl ? (long long)xl : 0;
    hi = okh ? (long long)xh : 0;
    return okl && okh;
}

// encode_p0's result for a vector of at most kSparseSlots values.
template <class G>
__device__ __forceinline__ void encode_sparse_p0(long long (&m)[G::R], const DevParams& p,
                                                 const double* __restrict__ z, uint32_t n_slots, uint32_t t) {
    constexpr int LOGH = G::LOGN - 1;
    constexpr int TOP = 1 << (G::K(0) - 1);
    const double f = 2.0 / (double)G::N;
    const uint32_t tp = G::tpart(0, t);
    bool bad = false;
#pragma unroll
    for (int c = 0; c < G::R; ++c) {
        if (c & TOP) continue;
        const uint32_t i = tp | G::cpart(0, c);         // < N/2
        bad |= !encode_pair(p, i, sparse_transform<LOGH>(p, z, n_slots, i), f, m[c], m[c | TOP]);
    }
    if (bad) atomicOr(p.err, 1u);
}

}  // namespace zinc
