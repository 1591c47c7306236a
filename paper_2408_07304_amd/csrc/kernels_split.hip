// Kernels for ring degree N = 32768.  A polynomial of 32768 uint64 words does
// not fit the 160 KiB LDS of a CU, so every transform is split: its first
// stage pairs coefficients j and j + N/2, which one thread holds in registers,
// and after it the two halves are independent 16384-point transforms run one
// after the other through the same LDS exchange buffer (twiddle index base
// (2 + h) 2^s for half h, see tw_index).  The inverse runs the two half
// transforms first and the pairing stage last.  CKKS encoding uses the
// real-input FFT identity so that its N/4-point complex FFT fits LDS;
// decoding combines two N/4-point FFTs in the last radix-2 stage.
#include "kernels_common.h"

namespace zinc {

namespace {

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
        o.lo.set(c, gauss_bsearch((u64)r.x | ((u64)r.y << 32), tab));
        o.hi.set(c, gauss_bsearch((u64)r.z | ((u64)r.w << 32), tab));
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
        Ad[2 * (bk & (Q - 1)) + (bk >> (LOGH - 1))] = val;   // Y[k_j / 2] gets Z[k_j] in Re or Im
    }
    __syncthreads();
    fft_dit<LOGQ, TS, -1, LOGH>(A, p.fft_tw, t);
    const double f = 2.0 / (double)NF;
    const uint32_t tp0 = GS::tpart(0, t);
    bool bad = false;
#pragma unroll
    for (int c = 0; c < RS; ++c) {
        const uint32_t i = jp(tp0, c);                   // < H
        const uint32_t m1 = i & (Q - 1), m2 = (Q - m1) & (Q - 1);
        const C2 y1 = A[m1], y2 = A[m2];
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
    // result in LDS in natural order of the half
    template <class In>
    __device__ __forceinline__ void run_half(int h, In in) const {
        if (fp()) {
            double v[RS];
#pragma unroll
            for (int c = 0; c < RS; ++c) v[c] = __longlong_as_double((long long)in(c));
            double* ld = reinterpret_cast<double*>(lds);
            ntt_fwd_fp<GS>(v, ld, tw_fp, limb, qd, qinv, mode == 2, t, 2u + (uint32_t)h, NF);
            to_natural<GS>(ld, v, t);
        } else {
            u64 v[RS];
#pragma unroll
            for (int c = 0; c < RS; ++c) v[c] = in(c);
            ntt_fwd<GS>(v, lds, tw, limb, q, q2, t, 2u + (uint32_t)h, NF);
            to_natural<GS>(lds, v, t);
        }
    }

    __device__ __forceinline__ u64 canon(uint32_t k) const {
        if (fp()) return fp_canon(reinterpret_cast<const double*>(lds)[pad(k)], qd, qinv);
        return canon4(lds[pad(k)], q, q2);
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
};

}  // namespace

// ---------------------------------------------------------------------------
// encryption, N = 32768.  Stashes: the encoded message (int64) in the c1 slot
// of the last limb (m_lo at jp, m_hi at jp + N/2); the half-1 input of every
// message transform in the upper half of its own destination slot; vanilla's
// NTT(u) in the c2 slot of the current limb.  Each thread reads back only what
// it wrote, before any thread overwrites it.
// ---------------------------------------------------------------------------
template <int SCHEME, bool FROM_SLOTS>
__global__ void __launch_bounds__(TS) __attribute__((amdgpu_waves_per_eu(4)))
k_encrypt_split(DevParams p, EncArgs a) {
    __shared__ u64 lds[LdsWords<NH>::value];
    __shared__ u64 tab[kCdtPad];
    const uint32_t t = threadIdx.x, b = blockIdx.x;
    const u64 ct_id = a.ct_ids[b];
    load_cdt(tab, p.cdt, t);
    const uint32_t L = p.L;
    u64* ct = a.ct + (size_t)b * 2 * L * NF;
    long long* stash = reinterpret_cast<long long*>(ct + (size_t)(L - 1) * NF);
    const u64* pt = a.pt + (size_t)b * L * NF;

    if constexpr (FROM_SLOTS) {
        long long mlo[RS], mhi[RS];
        encode_split(mlo, mhi, lds, p, a.slots + (size_t)b * a.n_slots, a.n_slots, t);
        const uint32_t tp0 = GS::tpart(0, t);
#pragma unroll
        for (int c = 0; c < RS; ++c) {
            stash[jp(tp0, c)] = mlo[c];
            stash[NH + jp(tp0, c)] = mhi[c];
        }
    }

    // message transform of limb l into dst (natural order) with epilogue fn(k, value)
    auto message_ntt = [&](const SplitLimb& sl, const LimbConst& lc, uint32_t l, const Packed8<RS>& elo,
                           const Packed8<RS>& ehi, u64* dst, auto&& epi) {
        const uint32_t tp0 = GS::tpart(0, opaque_tid(t));
        u64 u[RS];
#pragma unroll
        for (int c = 0; c < RS; ++c) {
            const uint32_t k = jp(tp0, c);
            u64 xl, xh;
            if constexpr (FROM_SLOTS) {
                xl = sl.residue(reduce_signed(stash[k] + elo.get(c), lc));
                xh = sl.residue(reduce_signed(stash[NH + k] + ehi.get(c), lc));
            } else {
                const u64* ptl = pt + (size_t)l * NF;
                xl = sl.residue(csub(ptl[k] + small_mod(elo.get(c), lc.q), lc.q));
                xh = sl.residue(csub(ptl[NH + k] + small_mod(ehi.get(c), lc.q), lc.q));
            }
            u[c] = sl.stage0(xl, xh, 0);
            dst[NH + k] = sl.stage0(xl, xh, 1);          // half-1 input, read back below
        }
        sl.run_half(0, [&](int c) { return u[c]; });
        {
            const uint32_t tt = opaque_tid(t);
#pragma unroll
            for (int i = 0; i < RS; ++i) epi(tt + TS * i, sl.canon(tt + TS * i));
        }
        const uint32_t tp1 = GS::tpart(0, opaque_tid(t));
        sl.run_half(1, [&](int c) { return dst[NH + jp(tp1, c)]; });
        {
            const uint32_t tt = opaque_tid(t);
#pragma unroll
            for (int i = 0; i < RS; ++i) epi(NH + tt + TS * i, sl.canon(tt + TS * i));
        }
    };
    // transform of a small-coefficient polynomial (samples), both halves
    auto small_ntt = [&](const SplitLimb& sl, const Pair8& e, auto&& epi) {
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            const Pair8 el = e.fresh();
            sl.run_half(h, [&](int c) { return sl.stage0(sl.small(el.lo.get(c)), sl.small(el.hi.get(c)), h); });
            const uint32_t tt = opaque_tid(t);
#pragma unroll
            for (int i = 0; i < RS; ++i) epi((uint32_t)h * NH + tt + TS * i, sl.canon(tt + TS * i));
        }
    };

    if constexpr (SCHEME == ZINC_SCHEME_ZINC) {
        Pair8 e1, e2;
        sample_gauss_split(e1, p, tab, ct_id, TAG_E1Z, t);
        sample_gauss_split(e2, p, tab, ct_id, TAG_E2Z, t);
#pragma unroll 1
        for (uint32_t l = 0; l < L; ++l) {
            const LimbConst lc = p.limbs[l];
            const SplitLimb sl(p, lc, l, lds, t);
            u64* c1 = ct + (size_t)l * NF;
            u64* c2 = ct + (size_t)(L + l) * NF;
            const u64* z1 = p.zero + (size_t)l * NF;
            const u64* z2 = p.zero + (size_t)(L + l) * NF;
            const Pair8 e1l = e1.fresh();
            message_ntt(sl, lc, l, e1l.lo, e1l.hi, c1, [&](uint32_t k, u64 v) { c1[k] = addmod(v, z1[k], lc.q); });
            small_ntt(sl, e2, [&](uint32_t k, u64 v) { c2[k] = addmod(v, z2[k], lc.q); });
        }
    } else {
        Pair8 u, e1, e2;
        sample_ternary_split(u, p, ct_id, TAG_U, t);
        sample_gauss_split(e1, p, tab, ct_id, TAG_E1, t);
        sample_gauss_split(e2, p, tab, ct_id, TAG_E2, t);
        const uint32_t M = p.M;
#pragma unroll 1
        for (uint32_t l = 0; l < L; ++l) {
            const LimbConst lc = p.limbs[l];
            const SplitLimb sl(p, lc, l, lds, t);
            u64* c1 = ct + (size_t)l * NF;
            u64* c2 = ct + (size_t)(L + l) * NF;
            const u64* pk1 = p.pk + (size_t)l * NF;
            const u64* pk1s = p.pk_sh + (size_t)l * NF;
            const u64* pk2 = p.pk + (size_t)(M + l) * NF;
            const u64* pk2s = p.pk_sh + (size_t)(M + l) * NF;
            small_ntt(sl, u, [&](uint32_t k, u64 v) { c2[k] = v; });                       // u_hat
            const Pair8 e1l = e1.fresh();
            message_ntt(sl, lc, l, e1l.lo, e1l.hi, c1,
                        [&](uint32_t k, u64 v) { c1[k] = addmod(v, sl.mul(c2[k], pk1[k], pk1s[k]), lc.q); });
            small_ntt(sl, e2, [&](uint32_t k, u64 v) { c2[k] = addmod(v, sl.mul(c2[k], pk2[k], pk2s[k]), lc.q); });
        }
    }
}

// ---------------------------------------------------------------------------
// key generation, N = 32768 (integer arithmetic), one workgroup per modulus
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(TS) k_keygen_split(DevParams p, u64* sk, u64* sk_sh, u64* pk, u64* pk_sh) {
    __shared__ u64 lds[LdsWords<NH>::value];
    __shared__ u64 tab[kCdtPad];
    const uint32_t t = threadIdx.x, l = blockIdx.x;
    load_cdt(tab, p.cdt, t);
    LimbConst lc = p.limbs[l];
    lc.fp = 0;
    const SplitLimb sl(p, lc, l, lds, t);
    const uint32_t M = p.M;
    Pair8 s, e;
    sample_ternary_split(s, p, ZINC_KEY_ID, TAG_SK, t);
    sample_gauss_split(e, p, tab, ZINC_KEY_ID, TAG_EPK, t);
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
        const Pair8 sh_ = s.fresh();
        sl.run_half(h, [&](int c) { return sl.stage0(small_mod(sh_.lo.get(c), lc.q), small_mod(sh_.hi.get(c), lc.q), h); });
        const uint32_t tt = opaque_tid(t);
#pragma unroll
        for (int i = 0; i < RS; ++i) {
            const uint32_t k = (uint32_t)h * NH + tt + TS * i;
            const u64 v = sl.canon(tt + TS * i);
            sk[(size_t)l * NF + k] = v;
            sk_sh[(size_t)l * NF + k] = shoup_companion_dev(v, lc.q);
        }
        const Pair8 eh_ = e.fresh();
        sl.run_half(h, [&](int c) { return sl.stage0(small_mod(eh_.lo.get(c), lc.q), small_mod(eh_.hi.get(c), lc.q), h); });
        const uint32_t t2 = opaque_tid(t);
#pragma unroll
        for (int i = 0; i < RS; ++i) {
            const uint32_t k = (uint32_t)h * NH + t2 + TS * i;
            const u64 ehat = sl.canon(t2 + TS * i);
            const u64 shat = sk[(size_t)l * NF + k], shs = sk_sh[(size_t)l * NF + k];
            const U4 r = draw(p.seed, ZINC_KEY_ID, TAG_A, l, k);
            const u64 hi = ((u64)r.w << 32) | r.z, lo = ((u64)r.y << 32) | r.x;
            const u64 ah = mod128(mod128(0, hi, lc.q), lo, lc.q);
            const u64 as = csub(shoup_lazy(ah, shat, shs, lc.q), lc.q);
            const u64 p1 = addmod(as ? lc.q - as : 0, ehat, lc.q);
            pk[(size_t)l * NF + k] = p1;
            pk[(size_t)(M + l) * NF + k] = ah;
            pk_sh[(size_t)l * NF + k] = shoup_companion_dev(p1, lc.q);
            pk_sh[(size_t)(M + l) * NF + k] = shoup_companion_dev(ah, lc.q);
        }
    }
}

// ---------------------------------------------------------------------------
// inverse transform, N = 32768: both half inverses, then the pairing stage
// (Gentleman-Sande with psi^-brv(1)) and N^-1.  xin(k) gives input k in
// [0, 2q); out(k, v) receives canonical outputs.
// ---------------------------------------------------------------------------
template <class In, class Out>
__device__ __forceinline__ void intt_split(const DevParams& p, const LimbConst& lc, uint32_t l, u64* lds,
                                           uint32_t t, In xin, Out out) {
    constexpr int PL = GS::NPASS - 1;
    const u64 q = lc.q, q2 = lc.q2;
    u64 lo[RS];
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
            for (int c = 0; c < RS; ++c) lo[c] = v[c];
        } else {
            const size_t o = ((size_t)l * NF + 1) * 2;
            const u64 iw = p.itw[o], iws = p.itw[o + 1];
            const uint32_t tp0 = GS::tpart(0, t);
#pragma unroll
            for (int c = 0; c < RS; ++c) {
                u64 x = lo[c], y = v[c];
                gs_bfly(x, y, iw, iws, q, q2);
                out(jp(tp0, c), csub(shoup_lazy(x, lc.ninv, lc.ninv_sh, q), q));
                out(NH + jp(tp0, c), csub(shoup_lazy(y, lc.ninv, lc.ninv_sh, q), q));
            }
        }
    }
}

__global__ void __launch_bounds__(TS) k_decrypt_split(DevParams p, const u64* ct, u64* pt) {
    __shared__ u64 lds[LdsWords<NH>::value];
    const uint32_t t = threadIdx.x, l = blockIdx.x, b = blockIdx.y, L = p.L;
    const LimbConst lc = p.limbs[l];
    const u64* c1 = ct + ((size_t)b * 2 * L + l) * NF;
    const u64* c2 = ct + ((size_t)b * 2 * L + L + l) * NF;
    const u64* s = p.sk + (size_t)l * NF;
    const u64* ss = p.sk_sh + (size_t)l * NF;
    u64* o = pt + ((size_t)b * L + l) * NF;
    intt_split(p, lc, l, lds, t,
               [&](uint32_t k) { return csub(c1[k] + csub(shoup_lazy(c2[k], s[k], ss[k], lc.q), lc.q), lc.q2); },
               [&](uint32_t k, u64 v) { o[k] = v; });
}

template <bool INV>
__global__ void __launch_bounds__(TS) k_ntt_split(DevParams p, uint32_t limb, u64* poly) {
    __shared__ u64 lds[LdsWords<NH>::value];
    const uint32_t t = threadIdx.x;
    u64* x = poly + (size_t)blockIdx.x * NF;
    const LimbConst lc = p.limbs[limb];
    if constexpr (!INV) {
        const SplitLimb sl(p, lc, limb, lds, t);
        const uint32_t tp0 = GS::tpart(0, t);
        u64 u[RS];
#pragma unroll
        for (int c = 0; c < RS; ++c) {
            const uint32_t k = jp(tp0, c);
            const u64 xl = sl.residue(x[k]), xh = sl.residue(x[NH + k]);
            u[c] = sl.stage0(xl, xh, 0);
            x[NH + k] = sl.stage0(xl, xh, 1);
        }
        sl.run_half(0, [&](int c) { return u[c]; });
#pragma unroll
        for (int i = 0; i < RS; ++i) x[t + TS * i] = sl.canon(t + TS * i);
        const uint32_t tp1 = GS::tpart(0, opaque_tid(t));
        sl.run_half(1, [&](int c) { return x[NH + jp(tp1, c)]; });
#pragma unroll
        for (int i = 0; i < RS; ++i) x[NH + t + TS * i] = sl.canon(t + TS * i);
    } else {
        // in place: every input is read (both halves, at the start of each half)
        // before the pairing stage writes any output
        intt_split(p, lc, limb, lds, t, [&](uint32_t k) { return x[k]; }, [&](uint32_t k, u64 v) { x[k] = v; });
    }
}

__global__ void __launch_bounds__(TS) k_encode_split(DevParams p, const double* slots, uint32_t n_slots, u64* pt) {
    __shared__ u64 lds[LdsWords<NH>::value];
    const uint32_t t = threadIdx.x, b = blockIdx.x;
    long long mlo[RS], mhi[RS];
    encode_split(mlo, mhi, lds, p, slots + (size_t)b * n_slots, n_slots, t);
    const uint32_t tp0 = GS::tpart(0, t);
    for (uint32_t l = 0; l < p.L; ++l) {
        const LimbConst lc = p.limbs[l];
        u64* o = pt + ((size_t)b * p.L + l) * NF;
#pragma unroll
        for (int c = 0; c < RS; ++c) {
            o[jp(tp0, c)] = reduce_signed(mlo[c], lc);
            o[NH + jp(tp0, c)] = reduce_signed(mhi[c], lc);
        }
    }
}

// Decoding, N = 32768: y_i = (m_i + i m_{i+N/2}) zeta^i (i < N/2); the even- and
// odd-indexed halves are transformed separately (N/4 points each, roots
// exp(+2 pi i / (N/4))), E kept in registers, then F[k] = E[k] + w^k O[k],
// F[k + N/4] = E[k] - w^k O[k] with w = exp(+2 pi i / (N/2)); z_j = Re F[k_j] / Delta.
__global__ void __launch_bounds__(TS) k_decode_split(DevParams p, const u64* pt, double* slots) {
    constexpr int H = NF / 2, Q = H / 2, LOGH = 14, LOGQ = 13, PER = Q / TS;
    __shared__ u64 lds[LdsWords<NH>::value];
    C2* A = reinterpret_cast<C2*>(lds);
    double* Rd = reinterpret_cast<double*>(lds);
    const uint32_t t = threadIdx.x, b = blockIdx.x, L = p.L;
    const LimbConst l0 = p.limbs[0];
    const u64* x0 = pt + (size_t)b * L * NF;
    bool bad = false;
    C2 E[PER];
#pragma unroll 1
    for (int par = 0; par < 2; ++par) {
        __syncthreads();
        for (uint32_t k2 = t; k2 < (uint32_t)Q; k2 += TS) {
            const uint32_t i = 2 * k2 + par;
            long long v[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t k = i + h * H;
                const u64 r = x0[k];
                v[h] = r > l0.half ? (long long)r - (long long)l0.q : (long long)r;
                if (L > 1) bad |= reduce_signed(v[h], p.limbs[1]) != x0[(size_t)NF + k];
            }
            const C2 y = cmul(C2{(double)v[0], (double)v[1]}, C2{p.twist[2 * i], -p.twist[2 * i + 1]});
            A[__brev(k2) >> (32 - LOGQ)] = y;
        }
        __syncthreads();
        fft_dit<LOGQ, TS, +1, LOGH>(A, p.fft_tw, t);
        if (par == 0) {
#pragma unroll
            for (int r = 0; r < PER; ++r) E[r] = A[t + TS * r];
        }
    }
    if (bad) atomicOr(p.err, 2u);
    double re_lo[PER], re_hi[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const uint32_t k = t + TS * r;
        const C2 w{p.fft_tw[2 * k], -p.fft_tw[2 * k + 1]};        // exp(+2 pi i k / H)
        const C2 o = cmul(w, A[k]);
        re_lo[r] = E[r].x + o.x;
        re_hi[r] = E[r].x - o.x;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        Rd[t + TS * r] = re_lo[r];
        Rd[Q + t + TS * r] = re_hi[r];
    }
    __syncthreads();
    const double inv = 1.0 / p.scale;
    for (uint32_t j = t; j < (uint32_t)H; j += TS) {
        const uint32_t kj = __brev(p.slot_pos[j]) >> (32 - LOGH);
        slots[(size_t)b * H + j] = Rd[kj] * inv;
    }
}

// ---------------------------------------------------------------------------
// launchers (N = 32768)
// ---------------------------------------------------------------------------
hipError_t launch_split_keygen(const DevParams& p, uint64_t* sk, uint64_t* sk_sh, uint64_t* pk, uint64_t* pk_sh,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_keygen_split, dim3(p.M), dim3(TS), 0, s, p, (u64*)sk, (u64*)sk_sh, (u64*)pk, (u64*)pk_sh);
    return hipGetLastError();
}

hipError_t launch_split_encrypt(const DevParams& p, int scheme, bool from_slots, const double* slots,
                                uint32_t n_slots, const uint64_t* pt, uint32_t batch, const uint64_t* ct_ids,
                                uint64_t* ct, hipStream_t s) {
    EncArgs a{slots, n_slots, (const u64*)pt, (const u64*)ct_ids, (u64*)ct};
    if (scheme == ZINC_SCHEME_ZINC) {
        if (from_slots) hipLaunchKernelGGL((k_encrypt_split<ZINC_SCHEME_ZINC, true>), dim3(batch), dim3(TS), 0, s, p, a);
        else hipLaunchKernelGGL((k_encrypt_split<ZINC_SCHEME_ZINC, false>), dim3(batch), dim3(TS), 0, s, p, a);
    } else {
        if (from_slots) hipLaunchKernelGGL((k_encrypt_split<ZINC_SCHEME_VANILLA, true>), dim3(batch), dim3(TS), 0, s, p, a);
        else hipLaunchKernelGGL((k_encrypt_split<ZINC_SCHEME_VANILLA, false>), dim3(batch), dim3(TS), 0, s, p, a);
    }
    return hipGetLastError();
}

hipError_t launch_split_encode(const DevParams& p, const double* slots, uint32_t n_slots, uint32_t batch,
                               uint64_t* pt, hipStream_t s) {
    hipLaunchKernelGGL(k_encode_split, dim3(batch), dim3(TS), 0, s, p, slots, n_slots, (u64*)pt);
    return hipGetLastError();
}

hipError_t launch_split_decrypt(const DevParams& p, const uint64_t* ct, uint32_t batch, uint64_t* pt,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_decrypt_split, dim3(p.L, batch), dim3(TS), 0, s, p, (const u64*)ct, (u64*)pt);
    return hipGetLastError();
}

hipError_t launch_split_decode(const DevParams& p, const uint64_t* pt, uint32_t batch, double* slots,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_decode_split, dim3(batch), dim3(TS), 0, s, p, (const u64*)pt, slots);
    return hipGetLastError();
}

hipError_t launch_split_ntt(const DevParams& p, bool inverse, uint32_t limb, uint64_t* poly, uint32_t n_polys,
                            hipStream_t s) {
    if (inverse) hipLaunchKernelGGL((k_ntt_split<true>), dim3(n_polys), dim3(TS), 0, s, p, limb, (u64*)poly);
    else hipLaunchKernelGGL((k_ntt_split<false>), dim3(n_polys), dim3(TS), 0, s, p, limb, (u64*)poly);
    return hipGetLastError();
}

}  // namespace zinc
