// Device helpers and the per-ciphertext encryption body for ring degree
// N = 32768 (split transforms; see kernels_split.hip).
#pragma once

#include <type_traits>

#include "kernels_common.h"

namespace zinc {

namespace split {

using GS = Geom<14, 10>;                 // geometry of one half
constexpr int NF = 32768;                // full ring degree
constexpr int NH = GS::N;                // 16384
constexpr int RS = GS::R;                // 16 coefficients per thread and half
constexpr int TS = GS::T;                // 1024 threads

// Thread t holds, for register c, the coefficients jp(c) and jp(c) + N/2, with
// jp(c) its pass-0 position in the half geometry.
__device__ __forceinline__ uint32_t jp(uint32_t tp0, int c) { return tp0 | GS::cpart(0, c); }

// Samples of one draw for both halves: lo[c] is coefficient jp(c), hi[c] is
// jp(c) + N/2 (the two 64-bit halves of Philox block jp(c)).
struct Pair8 {
    Packed8<RS> lo, hi;
    __device__ __forceinline__ Pair8 fresh() const { return Pair8{lo.fresh(), hi.fresh()}; }
};

__device__ __forceinline__ void sample_gauss_split(Pair8& o, const DevParams& p, const u64* tab, u64 ct_id,
                                                   uint32_t tag, uint32_t t) {
    const uint32_t tp0 = GS::tpart(0, t);
    o.lo.clear();
    o.hi.clear();
#pragma unroll
    for (int c = 0; c < RS; ++c) {
        const U4 r = draw(p.seed, ct_id, tag, 0, jp(tp0, c));
        o.lo.set(c, gauss_sample((u64)r.x | ((u64)r.y << 32), tab));
        o.hi.set(c, gauss_sample((u64)r.z | ((u64)r.w << 32), tab));
    }
}

// Ternary: coefficient k uses word k / (N/4) of block k mod N/4; block jp(c)
// (c with the top active bit clear) feeds jp(c), jp(c) + N/4, jp(c) + N/2 and
// jp(c) + 3N/4, i.e. registers c and c | TOP of both halves.
__device__ __forceinline__ void sample_ternary_split(Pair8& o, const DevParams& p, u64 ct_id, uint32_t tag,
                                                     uint32_t t) {
    constexpr int TOP = 1 << (GS::K(0) - 1);
    const uint32_t tp0 = GS::tpart(0, t);
    o.lo.clear();
    o.hi.clear();
#pragma unroll
    for (int c = 0; c < RS; ++c) {
        if (c & TOP) continue;
        const U4 r = draw(p.seed, ct_id, tag, 0, jp(tp0, c));
        o.lo.set(c, ternary_from(r.x));
        o.lo.set(c | TOP, ternary_from(r.y));
        o.hi.set(c, ternary_from(r.z));
        o.hi.set(c | TOP, ternary_from(r.w));
    }
}

// CKKS encoding for N = 32768 into m_lo[c] = m_{jp(c)}, m_hi[c] = m_{jp(c)+N/2}.
// The N/2 slot values sit at positions k_j of a real vector Z of N/2 points;
// Y[k] = Z[2k] + i Z[2k+1] (N/4 points) is transformed in LDS and unscrambled:
// with Yf its FFT and Q = N/4, E[m] = (Yf[m] + conj Yf[Q-m]) / 2,
// O[m] = (Yf[m] - conj Yf[Q-m]) / 2i, F[m] = E[m mod Q] + exp(-2 pi i m / (N/2)) O[m mod Q].
// Coefficient i < N/2 is Re, coefficient i + N/2 is Im, of (2/N) F[i] zeta^-i.
__device__ __forceinline__ void encode_split(long long (&mlo)[RS], long long (&mhi)[RS], u64* lds,
                                             const DevParams& p, const double* __restrict__ z, uint32_t n_slots,
                                             uint32_t t) {
    constexpr int H = NF / 2, Q = H / 2, LOGH = 14, LOGQ = 13;
    double* Ad = reinterpret_cast<double*>(lds);
    C2* A = reinterpret_cast<C2*>(lds);
    __syncthreads();
    for (uint32_t j = t; j < (uint32_t)H; j += TS) {
        const double val = j < n_slots ? p.scale * z[j] : 0.0;
        const uint32_t bk = p.slot_pos[j];               // brv_{log H}(k_j)
        Ad[2 * padc(bk & (Q - 1)) + (bk >> (LOGH - 1))] = val;   // Y[k_j / 2] gets Z[k_j] in Re or Im
    }
    __syncthreads();
    fft_dit_reg<LOGQ, TS, -1, LOGH>(A, p.fft_tw, t);
    const double f = 2.0 / (double)NF;
    const uint32_t tp0 = GS::tpart(0, t);
    bool bad = false;
#pragma unroll
    for (int c = 0; c < RS; ++c) {
        const uint32_t i = jp(tp0, c);                   // < H
        const uint32_t m1 = i & (Q - 1), m2 = (Q - m1) & (Q - 1);
        const C2 y1 = A[padc(m1)], y2 = A[padc(m2)];
        const C2 ev{0.5 * (y1.x + y2.x), 0.5 * (y1.y - y2.y)};     // (Y1 + conj Y2) / 2
        const C2 od{0.5 * (y1.y + y2.y), -0.5 * (y1.x - y2.x)};    // (Y1 - conj Y2) / 2i
        C2 w{p.fft_tw[2 * (i & (H / 2 - 1))], p.fft_tw[2 * (i & (H / 2 - 1)) + 1]};
        if (i >= (uint32_t)(H / 2)) { w.x = -w.x; w.y = -w.y; }
        const C2 o = cmul(w, od);
        const C2 F{ev.x + o.x, ev.y + o.y};
        const C2 r = cmul(F, C2{p.twist[2 * i], p.twist[2 * i + 1]});
        double xl = __builtin_rint(r.x * f), xh = __builtin_rint(r.y * f);
        if (!(__builtin_fabs(xl) < 4611686018427387904.0)) { bad = true; xl = 0.0; }
        if (!(__builtin_fabs(xh) < 4611686018427387904.0)) { bad = true; xh = 0.0; }
        mlo[c] = (long long)xl;
        mhi[c] = (long long)xh;
    }
    if (bad) atomicOr(p.err, 1u);
}

// encode_split's result for a vector of at most kSparseSlots values (the
// direct sum of encode_sparse_p0), for the encoding kernel.
__device__ __forceinline__ void encode_sparse_split(long long (&mlo)[RS], long long (&mhi)[RS], const DevParams& p,
                                                    const double* __restrict__ z, uint32_t n_slots, uint32_t t) {
    const double f = 2.0 / (double)NF;
    const uint32_t tp0 = GS::tpart(0, t);
    bool bad = false;
#pragma unroll
    for (int c = 0; c < RS; ++c) {
        const uint32_t i = jp(tp0, c);                   // < N/2
        bad |= !encode_pair(p, i, sparse_transform<14>(p, z, n_slots, i), f, mlo[c], mhi[c]);
    }
    if (bad) atomicOr(p.err, 1u);
}

// One modulus of a split transform.
struct SplitLimb {
    const u64* tw;
    const double* tw_fp;
    u64 q, q2, w0, w0s;                  // w0 = psi^brv(1) (stage 0), Shoup companion
    double qd, qinv, w0d, w0q;
    uint32_t mode, limb;
    u64* lds;
    uint32_t t;

    __device__ __forceinline__ SplitLimb(const DevParams& p, const LimbConst& lc, uint32_t l, u64* lds_, uint32_t t_)
        : tw(p.tw), tw_fp(p.tw_fp), q(lc.q), q2(lc.q2), qd(lc.qd), qinv(lc.qinv), mode(lc.fp), limb(l), lds(lds_),
          t(t_) {
        const size_t o = ((size_t)l * NF + 1) * 2;
        w0 = p.tw[o];
        w0s = p.tw[o + 1];
        w0d = p.tw_fp[o];
        w0q = p.tw_fp[o + 1];
    }
    __device__ __forceinline__ bool fp() const { return mode != 0; }

    // stage 0 on one pair, output of half h (raw 64-bit pattern): integer path
    // inputs in [0, 4q), outputs in [0, 4q); FP path inputs |x| <= q.
    __device__ __forceinline__ u64 stage0(u64 xl, u64 xh, int h) const {
        if (fp()) {
            const double a = __longlong_as_double((long long)xl), b = __longlong_as_double((long long)xh);
            const double tt = fp_mulmod(b, w0d, w0q, qd);
            double r = h ? a - tt : a + tt;
            if (mode == 2) r = fp_round_reduce(r, qd, qinv);
            return (u64)__double_as_longlong(r);
        }
        const u64 a = csub(xl, q2), tt = shoup_lazy(xh, w0, w0s, q);
        return h ? a - tt + q2 : a + tt;
    }

    // half-h transform of the pass-0 values in(c) (raw patterns); leaves the
    // result in LDS in natural order of the half.  WAVE: each wave then reads
    // back only its own blocks (wave_pair_index), with no workgroup barrier.
    // hook() runs after the last pass, before the write-back (early loads of
    // epilogue operands go there).
    template <bool WAVE = false, class In, class Hook>
    __device__ __forceinline__ void run_half(int h, In in, Hook hook) const {
        if (fp()) {
            double v[RS];
#pragma unroll
            for (int c = 0; c < RS; ++c) v[c] = __longlong_as_double((long long)in(c));
            double* ld = reinterpret_cast<double*>(lds);
            ntt_fwd_fp<GS>(v, ld, tw_fp, limb, qd, qinv, mode == 2, t, 2u + (uint32_t)h, NF);
            hook();
            if constexpr (WAVE) to_natural_wave<GS>(ld, v, t);
            else to_natural<GS>(ld, v, t);
        } else {
            u64 v[RS];
#pragma unroll
            for (int c = 0; c < RS; ++c) v[c] = in(c);
            ntt_fwd<GS>(v, lds, tw, limb, q, q2, t, 2u + (uint32_t)h, NF);
            hook();
            if constexpr (WAVE) to_natural_wave<GS>(lds, v, t);
            else to_natural<GS>(lds, v, t);
        }
    }
    template <bool WAVE = false, class In>
    __device__ __forceinline__ void run_half(int h, In in) const {
        run_half<WAVE>(h, in, []() {});
    }

    __device__ __forceinline__ u64 canon(uint32_t k) const {
        if (fp()) return fp_canon(reinterpret_cast<const double*>(lds)[pad(k)], qd, qinv);
        return canon16(lds[pad(k)], q);
    }

    __device__ __forceinline__ u64 mul(u64 a, u64 b, u64 b_sh) const {
        if (fp()) {
            const double bd = u64_to_fp(b);
            const double r = fp_mulmod(u64_to_fp(a), bd, bd * qinv, qd);
            return (u64)__double_as_longlong((r < 0.0 ? r + qd : r) + 0x1p52) - 0x4330000000000000ull;
        }
        return csub(shoup_lazy(a, b, b_sh, q), q);
    }

    // raw input patterns
    __device__ __forceinline__ u64 small(int x) const {
        return fp() ? (u64)__double_as_longlong((double)x) : small_mod(x, q);
    }
    __device__ __forceinline__ u64 residue(u64 r) const {   // canonical or [0, 2q) residue
        return fp() ? (u64)__double_as_longlong(u64_to_fp(r)) : r;
    }
    // a Gaussian error as the scheme adds it: x, or t x under BGV (Eq. 13)
    template <bool BGV>
    __device__ __forceinline__ u64 noise(int x, u64 nt, const LimbConst& lc) const {
        if constexpr (!BGV) return small(x);
        else return fp() ? (u64)__double_as_longlong(noise_rf<true>(x, nt, lc)) : noise_ri<true>(x, nt, lc);
    }
};

// ---------------------------------------------------------------------------
// inverse transform, N = 32768: both half inverses, then the pairing stage
// (Gentleman-Sande with psi^-brv(1)) and N^-1.  xin(k) gives input k in
// [0, 2q); out(k, v) receives canonical outputs.  With a stash (N/2 words,
// which may be the input or output buffer) the half-0 result waits there, at
// the positions jp(c) this thread writes last, instead of in registers.
// ---------------------------------------------------------------------------
template <class In, class Out>
__device__ __forceinline__ void intt_split(const DevParams& p, const LimbConst& lc, uint32_t l, u64* lds,
                                           uint32_t t, In xin, Out out, u64* stash = nullptr) {
    constexpr int PL = GS::NPASS - 1;
    const u64 q = lc.q, q2 = lc.q2;
    u64 lo[RS];
    const uint32_t tps = GS::tpart(0, t);
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
        __syncthreads();
        {
            const uint32_t tt = opaque_tid(t);
#pragma unroll
            for (int i = 0; i < RS; ++i) lds[pad(tt + TS * i)] = xin((uint32_t)h * NH + tt + TS * i);
        }
        __syncthreads();
        u64 v[RS];
        lds_get<GS, PL>(lds, v, t);
        ntt_inv<GS>(v, lds, p.itw, l, q, q2, t, 2u + (uint32_t)h, NF);
        if (h == 0) {
#pragma unroll
            for (int c = 0; c < RS; ++c) {
                if (stash) stash[jp(tps, c)] = v[c];
                else lo[c] = v[c];
            }
        } else {
            const size_t o = ((size_t)l * NF + 1) * 2;
            const u64 iw = p.itw[o], iws = p.itw[o + 1];
            const uint32_t tp0 = GS::tpart(0, t);
#pragma unroll
            for (int c = 0; c < RS; ++c) {
                u64 x = stash ? stash[jp(tps, c)] : lo[c], y = v[c];
                gs_bfly(x, y, iw, iws, q, q2);
                out(jp(tp0, c), csub(shoup_lazy(x, lc.ninv, lc.ninv_sh, q), q));
                out(NH + jp(tp0, c), csub(shoup_lazy(y, lc.ninv, lc.ninv_sh, q), q));
            }
        }
    }
}

}  // namespace split

// ---------------------------------------------------------------------------
// encryption, N = 32768.  Stashes: the encoded message (int64) in the c1 slot
// of the last limb (m_lo at jp, m_hi at jp + N/2); the half-1 input of every
// message transform in the upper half of its own destination slot; vanilla's
// NTT(u) in the c2 slot of the current limb.  Each thread reads back only what
// it wrote, before any thread overwrites it.
// ---------------------------------------------------------------------------
// Encrypt one ciphertext of ring degree 32768 with all TS threads of the
// workgroup; lds holds LdsWords<NH> words, tab the chi table.  BGV = true
// (integer plaintexts only): every Gaussian error is scaled by the plaintext
// modulus p.noise_t (Eq. 13); the ternary u is not.  Only data limbs
// [l0, min(l1, L)) are computed (the noise and the message are the
// ciphertext's own whatever the range, so separate ranges of one ciphertext
// may run in separate workgroups); the stash is the c1 slot of the range's
// last limb.
template <int SCHEME, bool FROM_SLOTS, bool BGV = false>
__device__ __forceinline__ void encrypt_item_split(const DevParams& p, const double* slots, uint32_t n_slots,
                                                   const u64* pt, u64 ct_id, u64* ct, u64* lds, const u64* tab,
                                                   uint32_t t, uint32_t l0 = 0, uint32_t l1 = ~0u) {
    using namespace split;
    static_assert(!(FROM_SLOTS && BGV), "BGV encrypts integer plaintexts");
    const uint32_t L = p.L, le = l1 < L ? l1 : L;
    long long* stash = reinterpret_cast<long long*>(ct + (size_t)(le - 1) * NF);

    if constexpr (FROM_SLOTS) {
        long long mlo[RS], mhi[RS];
        encode_split(mlo, mhi, lds, p, slots, n_slots, t);
        const uint32_t tp0 = GS::tpart(0, t);
#pragma unroll
        for (int c = 0; c < RS; ++c) {
            stash[jp(tp0, c)] = mlo[c];
            stash[NH + jp(tp0, c)] = mhi[c];
        }
    }

    // message transform of limb l into dst (natural order) with epilogue
    // epi(k, value_k, value_k+1, pre(k)) on pairs (k even: one 16-byte access;
    // a wave covers whole lines); pre(k), an operand of the epilogue, is loaded
    // after the last pass so that its latency overlaps the write-back (one
    // workgroup per CU: no other workgroup hides it).  Vanilla's epilogues take each wave's own blocks of
    // the last pass (wave_pair_index, no barrier after the write-back: 2 %
    // faster); Zinc's, which load the cached Enc(0) in the epilogue, measured
    // 1 % slower that way (each moment's accesses of the workgroup are spread
    // over 4 KiB blocks), so they take consecutive pairs across the waves.
    constexpr bool WAVE = SCHEME != ZINC_SCHEME_ZINC;
    auto pair_index = [](uint32_t tt, int i) -> uint32_t {
        if constexpr (WAVE) return wave_pair_index<GS>(tt, i);
        else return 2 * (tt + TS * i);
    };
    auto message_ntt = [&](const SplitLimb& sl, const LimbConst& lc, uint32_t l, const Packed8<RS>& elo,
                           const Packed8<RS>& ehi, u64* dst, auto&& pre, auto&& epi) {
        decltype(pre(0u)) pv[RS / 2];
        auto fetch = [&](uint32_t base) {
            return [&, base]() {
                const uint32_t tt = opaque_tid(t);
#pragma unroll
                for (int i = 0; i < RS / 2; ++i) pv[i] = pre(base + pair_index(tt, i));
            };
        };
        const uint32_t tp0 = GS::tpart(0, opaque_tid(t));
        u64 u[RS];
#pragma unroll
        for (int c = 0; c < RS; ++c) {
            const uint32_t k = jp(tp0, c);
            u64 xl, xh;
            if constexpr (FROM_SLOTS) {
                xl = sl.residue(reduce_signed_near(stash[k] + elo.get(c), lc));
                xh = sl.residue(reduce_signed_near(stash[NH + k] + ehi.get(c), lc));
            } else {
                const u64* ptl = pt + (size_t)l * NF;
                xl = sl.residue(csub(ptl[k] + noise_ri<BGV>(elo.get(c), p.noise_t, lc), lc.q));
                xh = sl.residue(csub(ptl[NH + k] + noise_ri<BGV>(ehi.get(c), p.noise_t, lc), lc.q));
            }
            u[c] = sl.stage0(xl, xh, 0);
            dst[NH + k] = sl.stage0(xl, xh, 1);          // half-1 input, read back below
        }
        sl.template run_half<WAVE>(0, [&](int c) { return u[c]; }, fetch(0));
        {
            const uint32_t tt = opaque_tid(t);
#pragma unroll
            for (int i = 0; i < RS / 2; ++i) {
                const uint32_t k = pair_index(tt, i);
                epi(k, sl.canon(k), sl.canon(k + 1), pv[i]);
            }
        }
        const uint32_t tp1 = GS::tpart(0, opaque_tid(t));
        sl.template run_half<WAVE>(1, [&](int c) { return dst[NH + jp(tp1, c)]; }, fetch(NH));
        {
            const uint32_t tt = opaque_tid(t);
#pragma unroll
            for (int i = 0; i < RS / 2; ++i) {
                const uint32_t k = pair_index(tt, i);
                epi(NH + k, sl.canon(k), sl.canon(k + 1), pv[i]);
            }
        }
    };
    // transform of a small-coefficient polynomial (samples), both halves; an
    // error polynomial (ERR true) is scaled by t under BGV
    auto small_ntt = [&](const SplitLimb& sl, const LimbConst& lc, const Pair8& e, auto err, auto&& pre,
                         auto&& epi) {
        constexpr bool S = decltype(err)::value && BGV;
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            const Pair8 el = e.fresh();
            decltype(pre(0u)) pv[RS / 2];
            sl.template run_half<WAVE>(h, [&](int c) {
                return sl.stage0(sl.noise<S>(el.lo.get(c), p.noise_t, lc), sl.noise<S>(el.hi.get(c), p.noise_t, lc), h);
            }, [&]() {
                const uint32_t tt = opaque_tid(t);
#pragma unroll
                for (int i = 0; i < RS / 2; ++i) pv[i] = pre((uint32_t)h * NH + pair_index(tt, i));
            });
            const uint32_t tt = opaque_tid(t);
#pragma unroll
            for (int i = 0; i < RS / 2; ++i) {
                const uint32_t k = pair_index(tt, i);
                epi((uint32_t)h * NH + k, sl.canon(k), sl.canon(k + 1), pv[i]);
            }
        }
    };

    auto no_pre = [](uint32_t) { return 0; };     // vanilla: operands loaded in the epilogue

    if constexpr (SCHEME == ZINC_SCHEME_ZINC) {
        Pair8 e1, e2;
        sample_gauss_split(e1, p, tab, ct_id, TAG_E1Z, t);
        sample_gauss_split(e2, p, tab, ct_id, TAG_E2Z, t);
#pragma unroll 1
        for (uint32_t l = l0; l < le; ++l) {
            const LimbConst lc = p.limbs[l];
            const SplitLimb sl(p, lc, l, lds, t);
            u64* c1 = ct + (size_t)l * NF;
            u64* c2 = ct + (size_t)(L + l) * NF;
            const u64* z1 = p.zero + (size_t)l * NF;
            const u64* z2 = p.zero + (size_t)(L + l) * NF;
            const Pair8 e1l = e1.fresh();
            message_ntt(sl, lc, l, e1l.lo, e1l.hi, c1, [&](uint32_t k) { return load_pair(z1 + k); },
                        [&](uint32_t k, u64 a, u64 b, u64x2 z) {
                            store_pair_final(c1 + k, addmod(a, z.x, lc.q), addmod(b, z.y, lc.q));
                        });
            small_ntt(sl, lc, e2, std::true_type{}, [&](uint32_t k) { return load_pair(z2 + k); },
                      [&](uint32_t k, u64 a, u64 b, u64x2 z) {
                          store_pair_final(c2 + k, addmod(a, z.x, lc.q), addmod(b, z.y, lc.q));
                      });
        }
    } else {
        Pair8 u, e1, e2;
        sample_ternary_split(u, p, ct_id, TAG_U, t);
        sample_gauss_split(e1, p, tab, ct_id, TAG_E1, t);
        sample_gauss_split(e2, p, tab, ct_id, TAG_E2, t);
        const uint32_t M = p.M;
#pragma unroll 1
        for (uint32_t l = l0; l < le; ++l) {
            const LimbConst lc = p.limbs[l];
            const SplitLimb sl(p, lc, l, lds, t);
            u64* c1 = ct + (size_t)l * NF;
            u64* c2 = ct + (size_t)(L + l) * NF;
            const u64* pk1 = p.pk + (size_t)l * NF;
            const u64* pk1s = p.pk_sh + (size_t)l * NF;
            const u64* pk2 = p.pk + (size_t)(M + l) * NF;
            const u64* pk2s = p.pk_sh + (size_t)(M + l) * NF;
            small_ntt(sl, lc, u, std::false_type{}, no_pre,
                      [&](uint32_t k, u64 a, u64 b, int) { store_pair(c2 + k, a, b); });   // u_hat
            const Pair8 e1l = e1.fresh();
            message_ntt(sl, lc, l, e1l.lo, e1l.hi, c1, no_pre, [&](uint32_t k, u64 a, u64 b, int) {
                const u64x2 u2 = load_pair(c2 + k), w = load_pair(pk1 + k), ws = load_pair(pk1s + k);
                store_pair_final(c1 + k, addmod(a, sl.mul(u2.x, w.x, ws.x), lc.q),
                                 addmod(b, sl.mul(u2.y, w.y, ws.y), lc.q));
            });
            small_ntt(sl, lc, e2, std::true_type{}, no_pre, [&](uint32_t k, u64 a, u64 b, int) {
                const u64x2 u2 = load_pair(c2 + k), w = load_pair(pk2 + k), ws = load_pair(pk2s + k);
                store_pair_final(c2 + k, addmod(a, sl.mul(u2.x, w.x, ws.x), lc.q),
                                 addmod(b, sl.mul(u2.y, w.y, ws.y), lc.q));
            });
        }
    }
}

}  // namespace zinc
