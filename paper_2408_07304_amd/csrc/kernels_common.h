// Helpers shared by the encryption kernels of every ring degree.
#pragma once

#include "device.h"

namespace zinc {

// coefficients per thread (R) = 16 for every supported ring degree
template <int LOGN>
struct Cfg;
template <>
struct Cfg<12> { using G = Geom<12, 8>; };
template <>
struct Cfg<13> { using G = Geom<13, 9>; };
template <>
struct Cfg<14> { using G = Geom<14, 10>; };

// How a kernel of ring degree 2^LOGN receives its parameters: by value below
// 16384 (the hardware preloads the first words of the argument, which saves
// latency on short workgroups), else as a pointer to the context's device copy
// (DevParams::self), read field by field with scalar loads, which leaves the
// registers to the transform (by value the largest kernels spill).
template <int LOGN>
struct ParamArg {
    using type = DevParams;
    __host__ __device__ static type of(const DevParams& p) { return p; }
};
template <>
struct ParamArg<14> {
    using type = const DevParams* __restrict__;
    __host__ __device__ static const DevParams* of(const DevParams& p) { return p.self; }
};
__device__ __forceinline__ const DevParams& deref(const DevParams& p) { return p; }
__device__ __forceinline__ const DevParams& deref(const DevParams* p) { return *p; }

struct EncArgs {
    const double* slots;     // [batch][n_slots] (FROM_SLOTS)
    uint32_t n_slots;
    const u64* pt;           // [batch][L][N]   (!FROM_SLOTS)
    const u64* ct_ids;       // [batch]
    u64* ct;                 // [batch][2][L][N]
    uint32_t reserved_ok;    // 1 only for the cached Enc(0), which uses ZINC_ZERO_ID
};

// Identifiers of 2^63 and above are reserved for the keys and the cached
// Enc(0), whose randomness they select.  A direct encryption call naming one
// writes nothing for that ciphertext and sets bit 2 of the error flags.  The
// id is the same for every thread of the workgroup, so the whole group leaves
// before its first barrier.
__device__ __forceinline__ bool reserved_id(const DevParams& p, const EncArgs& a, u64 id, uint32_t t) {
    if (a.reserved_ok || (id >> 63) == 0) return false;
    if (t == 0) atomicOr(p.err, 4u);
    return true;
}

// Per-limb view of the arithmetic: the forward NTT runs either on uint64
// residues (Shoup, any modulus) or on doubles holding exact integers (moduli
// below 2^50); after to_natural() the transform's coefficient k is read back as
// a canonical residue with canon(k).
template <class G>
struct LimbNtt {
    const u64* tw;
    const double* tw_fp;
    u64 q, q2;
    double qd, qinv;
    uint32_t mode;
    uint32_t limb;
    u64* lds;
    uint32_t t;

    __device__ __forceinline__ LimbNtt(const DevParams& p, const LimbConst& lc, uint32_t l, u64* lds_, uint32_t t_)
        : tw(p.tw), tw_fp(p.tw_fp), q(lc.q), q2(lc.q2), qd(lc.qd), qinv(lc.qinv), mode(lc.fp), limb(l),
          lds(lds_), t(t_) {}

    __device__ __forceinline__ bool fp() const { return mode != 0; }

    // Transform the pass-0 inputs given by in(c) (integer path: a residue in
    // [0, 2q); FP path: an exact integer of magnitude at most q, as double).
    // hook() runs after the last pass, before the exchange into natural
    // order (early loads of epilogue operands go there).  WAVE: each wave then
    // reads back only its own blocks (wave_pair_index), with no workgroup
    // barrier; else any thread may read any coefficient.
    template <bool WAVE = false, class InInt, class InFp, class Hook>
    __device__ __forceinline__ void run(InInt in_int, InFp in_fp, Hook hook) const {
        if (fp()) {
            double v[G::R];
#pragma unroll
            for (int c = 0; c < G::R; ++c) v[c] = in_fp(c);
            double* ld = reinterpret_cast<double*>(lds);
            ntt_fwd_fp<G>(v, ld, tw_fp, limb, qd, qinv, mode == 2, t);
            hook();
            if constexpr (WAVE) to_natural_wave<G>(ld, v, t);
            else to_natural<G>(ld, v, t);
        } else {
            u64 v[G::R];
#pragma unroll
            for (int c = 0; c < G::R; ++c) v[c] = in_int(c);
            ntt_fwd<G>(v, lds, tw, limb, q, q2, t);
            hook();
            if constexpr (WAVE) to_natural_wave<G>(lds, v, t);
            else to_natural<G>(lds, v, t);
        }
    }
    template <class InInt, class InFp>
    __device__ __forceinline__ void run(InInt in_int, InFp in_fp) const {
        run(in_int, in_fp, []() {});
    }

    // The same transform, leaving canonical residues in registers: res[c] is
    // coefficient out_index<G>(t, c).  The last pass covers the lowest index
    // bits, so a thread holds runs of consecutive coefficients and stores from
    // registers stay coalesced with no LDS round trip.
    template <class InInt, class InFp>
    __device__ __forceinline__ void run_regs(InInt in_int, InFp in_fp, u64 (&res)[G::R]) const {
        if (fp()) {
            double v[G::R];
#pragma unroll
            for (int c = 0; c < G::R; ++c) v[c] = in_fp(c);
            ntt_fwd_fp<G>(v, reinterpret_cast<double*>(lds), tw_fp, limb, qd, qinv, mode == 2, t);
#pragma unroll
            for (int c = 0; c < G::R; ++c) res[c] = fp_canon(v[c], qd, qinv);
        } else {
            u64 v[G::R];
#pragma unroll
            for (int c = 0; c < G::R; ++c) v[c] = in_int(c);
            ntt_fwd<G>(v, lds, tw, limb, q, q2, t);
#pragma unroll
            for (int c = 0; c < G::R; ++c) res[c] = canon16(v[c], q);
        }
    }

    // canonical residue of transform coefficient k (after run())
    __device__ __forceinline__ u64 canon(uint32_t k) const {
        if (fp()) return fp_canon(reinterpret_cast<const double*>(lds)[pad(k)], qd, qinv);
        return canon16(lds[pad(k)], q);
    }

    // a * b mod q for canonical residues a, b (the pk * u_hat product)
    __device__ __forceinline__ u64 mul(u64 a, u64 b, u64 b_sh) const {
        if (fp()) {
            const double bd = u64_to_fp(b);
            const double r = fp_mulmod(u64_to_fp(a), bd, bd * qinv, qd);   // |r| < q
            return (u64)__double_as_longlong((r < 0.0 ? r + qd : r) + 0x1p52) - 0x4330000000000000ull;
        }
        return csub(shoup_lazy(a, b, b_sh, q), q);
    }
};

// Coefficient index held in register c after the last pass of a transform.
// The last pass covers index bits from 0, so registers c and c + 1 (c even)
// hold coefficients k and k + 1 with k even: one 16-byte access.
template <class G>
__device__ __forceinline__ uint32_t out_index(uint32_t t, int c) {
    static_assert(G::LO(G::NPASS - 1) == 0 && G::K(G::NPASS - 1) >= 1, "last pass covers bit 0");
    return G::tpart(G::NPASS - 1, t) | G::cpart(G::NPASS - 1, c);
}

__device__ __forceinline__ void store_pair(u64* p, u64 a, u64 b) {
    *reinterpret_cast<u64x2*>(p) = u64x2{a, b};
}
// Final ciphertext words, which no later step of the launch reads: written
// non-temporally so that they stream to HBM instead of displacing the
// twiddles, keys and cached Enc(0) in L2.
__device__ __forceinline__ void store_pair_final(u64* p, u64 a, u64 b) {
    __builtin_nontemporal_store(u64x2{a, b}, reinterpret_cast<u64x2*>(p));
}

// Transform one polynomial of a limb and hand every coefficient pair the
// thread owns to epi(k, v_k, v_k+1, pre(k)) (k even, canonical values; pre(k)
// an operand of the epilogue loaded for that pair).  REG = false: back to
// natural order through LDS within each wave, so that each store instruction
// of a wave covers 128 consecutive coefficients; pre(k) is issued after the
// last pass, so its latency overlaps that exchange.  A thread takes the same
// pairs in every transform of a given geometry.  REG = true: straight from the
// registers of the last pass, whose runs of consecutive coefficients give
// 2^K-strided accesses but no LDS round trip.  Which is faster depends on the
// ring degree and the scheme (autotuned).
template <bool REG, class G, class InInt, class InFp, class Pre, class Epi>
__device__ __forceinline__ void transform_store_pre(const LimbNtt<G>& nt, uint32_t t, InInt in_int, InFp in_fp,
                                                    Pre pre, Epi epi) {
    if constexpr (REG) {
        u64 r[G::R];
        nt.run_regs(in_int, in_fp, r);
        const uint32_t tt = opaque_tid(t);
#pragma unroll
        for (int c = 0; c < G::R; c += 2) {
            const uint32_t k = out_index<G>(tt, c);
            epi(k, r[c], r[c + 1], pre(k));
        }
    } else {
        decltype(pre(0u)) pv[G::R / 2];
        nt.template run<true>(in_int, in_fp, [&]() {
            const uint32_t tt = opaque_tid(t);
#pragma unroll
            for (int i = 0; i < G::R / 2; ++i) pv[i] = pre(wave_pair_index<G>(tt, i));
        });
        const uint32_t tt = opaque_tid(t);
#pragma unroll
        for (int i = 0; i < G::R / 2; ++i) {
            const uint32_t k = wave_pair_index<G>(tt, i);
            epi(k, nt.canon(k), nt.canon(k + 1), pv[i]);
        }
    }
}

template <bool REG, class G, class InInt, class InFp, class Epi>
__device__ __forceinline__ void transform_store(const LimbNtt<G>& nt, uint32_t t, InInt in_int, InFp in_fp,
                                                Epi epi) {
    transform_store_pre<REG>(nt, t, in_int, in_fp, [](uint32_t) { return 0; },
                             [&](uint32_t k, u64 a, u64 b, int) { epi(k, a, b); });
}

// A Gaussian error coefficient x as the scheme adds it, for the integer and the
// FP64 transforms: x itself, or t x under BGV (Eq. 13 scales every error by
// the plaintext modulus t).  |x| < 64 and t < 2^32, so t x is below 2^38 and
// exact in a double.
template <bool BGV>
__device__ __forceinline__ u64 noise_ri(int x, u64 t, const LimbConst& lc) {     // [0, q)
    if constexpr (BGV) return reduce_signed((long long)x * (long long)t, lc);
    else return small_mod(x, lc.q);
}
template <bool BGV>
__device__ __forceinline__ double noise_rf(int x, u64 t, const LimbConst& lc) {  // |value| <= q/2 + 64
    if constexpr (BGV) return fp_round_reduce((double)x * (double)t, lc.qd, lc.qinv);
    else return (double)x;
}

// Pass-0 message input of limb l: (m + e) with m read back from the stash
// (encoded slots) or from the caller's plaintext residues.  BGV (plaintext
// residues only): the error is t e.
template <class G, bool FROM_SLOTS, bool BGV = false>
struct MessageIn {
    const long long* stash;
    const u64* pt;
    Packed8<G::R> e;
    LimbConst lc;
    uint32_t tp0;
    u64 noise_t;
    static_assert(!(FROM_SLOTS && BGV), "BGV encrypts integer plaintexts");
    __device__ __forceinline__ u64 ri(int c) const {       // residue in [0, 2q)
        const uint32_t k = tp0 | G::cpart(0, c);
        if constexpr (FROM_SLOTS) return reduce_signed_near(stash[k] + e.get(c), lc);
        else return pt[k] + noise_ri<BGV>(e.get(c), noise_t, lc);
    }
    __device__ __forceinline__ double rf(int c) const {    // |value| <= q
        const uint32_t k = tp0 | G::cpart(0, c);
        if constexpr (FROM_SLOTS) {
            // below 2^52 the integer converts exactly and one rounded quotient
            // brings it into [-q, q]; larger messages take the integer route
            const long long x = stash[k] + e.get(c);
            if (x > -(1ll << 52) && x < (1ll << 52)) return fp_round_reduce((double)x, lc.qd, lc.qinv);
            return u64_to_fp(reduce_signed(x, lc));
        } else if constexpr (BGV) {
            // pt < 2^50 on FP64 limbs and |t e| < 2^38: the sum is exact
            return fp_round_reduce(u64_to_fp(pt[k]) + (double)e.get(c) * (double)noise_t, lc.qd, lc.qinv);
        } else {
            return u64_to_fp(pt[k]) + (double)e.get(c);
        }
    }
};

// One workgroup per ciphertext.  The encoded message (FROM_SLOTS) is stashed
// as int64 in the ciphertext's own c1 slot of the last limb, in pass-0 layout;
// each thread reads back only what it wrote, and the slot is overwritten only
// by that limb's c1 epilogue, after the last read.  Vanilla keeps NTT(u) of the
// current limb in that limb's c2 slot the same way until c2 is stored.
//
// Encrypt one ciphertext with the threads t in [0, G::T) of a group whose
// barriers every thread of the workgroup reaches (the whole workgroup, or one
// of several equal groups running the same ring degree in lockstep).  lds is
// the group's exchange buffer (LdsWords<N> words), tab the chi table in LDS.
// G is the thread geometry: any Geom<LOGN, LOGT> with at least 4 coefficients
// per thread (the default is Cfg<LOGN>::G, 16 per thread).
//
// BGV = true (integer plaintexts only): every Gaussian error is scaled by the
// plaintext modulus p.noise_t (Eq. 13).
//
// Only data limbs [l0, l1) are encrypted (all of them by default): a small
// batch spreads each ciphertext's limbs over several workgroups, each of which
// draws the same noise (counter-based) and encodes the same message, and
// stashes the message in the c1 slot of its own last limb.
template <class G, int SCHEME, bool FROM_SLOTS, bool REG_EPI = false, bool BGV = false>
__device__ __forceinline__ void encrypt_item_g(const DevParams& p, const double* slots, uint32_t n_slots,
                                               const u64* pt, u64 ct_id, u64* ct, u64* lds, const u64* tab,
                                               uint32_t t, uint32_t l0 = 0, uint32_t l1 = ~0u) {
    constexpr int R = G::R, N = G::N;
    const uint32_t L = p.L;
    if (l1 > L) l1 = L;
    long long* stash = reinterpret_cast<long long*>(ct + (size_t)(l1 - 1) * N);
    // final ciphertext words: non-temporal from the natural-order epilogue,
    // whose wave writes whole lines; the register epilogue's strided 16-byte
    // writes measured far slower non-temporal, so they stay ordinary stores
    auto final_store = [](u64* q, u64 a, u64 b) {
        if constexpr (REG_EPI) store_pair(q, a, b);
        else store_pair_final(q, a, b);
    };

    if constexpr (FROM_SLOTS) {
        long long m[R];
        encode_p0<G>(m, lds, p, slots, n_slots, t);
        const uint32_t tp0 = G::tpart(0, t);
#pragma unroll
        for (int c = 0; c < R; ++c) stash[tp0 | G::cpart(0, c)] = m[c];
    }

    if constexpr (SCHEME == ZINC_SCHEME_ZINC) {
        Packed8<R> e1, e2;
        sample_gauss_p0<G>(e1, p, tab, ct_id, TAG_E1Z, t);
        sample_gauss_p0<G>(e2, p, tab, ct_id, TAG_E2Z, t);
#pragma unroll 1
        for (uint32_t l = l0; l < l1; ++l) {
            const LimbConst lc = p.limbs[l];
            const LimbNtt<G> nt{p, lc, l, lds, t};
            const MessageIn<G, FROM_SLOTS, BGV> msg{stash, pt + (size_t)l * N, e1.fresh(), lc,
                                                    G::tpart(0, opaque_tid(t)), p.noise_t};
            // c1 = zero1 + NTT(m + e1')
            const u64* z1 = p.zero + (size_t)l * N;
            u64* c1 = ct + (size_t)l * N;
            transform_store_pre<REG_EPI>(nt, t, [&](int c) { return msg.ri(c); }, [&](int c) { return msg.rf(c); },
                                         [&](uint32_t k) { return load_pair(z1 + k); },
                                         [&](uint32_t k, u64 a, u64 b, u64x2 z) {
                                             final_store(c1 + k, addmod(a, z.x, lc.q), addmod(b, z.y, lc.q));
                                         });
            // c2 = zero2 + NTT(e2')
            const Packed8<R> e2l = e2.fresh();
            const u64* z2 = p.zero + (size_t)(L + l) * N;
            u64* c2 = ct + (size_t)(L + l) * N;
            transform_store_pre<REG_EPI>(nt, t, [&](int c) { return noise_ri<BGV>(e2l.get(c), p.noise_t, lc); },
                                         [&](int c) { return noise_rf<BGV>(e2l.get(c), p.noise_t, lc); },
                                         [&](uint32_t k) { return load_pair(z2 + k); },
                                         [&](uint32_t k, u64 a, u64 b, u64x2 z) {
                                             final_store(c2 + k, addmod(a, z.x, lc.q), addmod(b, z.y, lc.q));
                                         });
        }
    } else {
        Packed8<R> u, e1, e2;
        sample_ternary_p0<G>(u, p, ct_id, TAG_U, t);
        sample_gauss_p0<G>(e1, p, tab, ct_id, TAG_E1, t);
        sample_gauss_p0<G>(e2, p, tab, ct_id, TAG_E2, t);
        const uint32_t M = p.M;
#pragma unroll 1
        for (uint32_t l = l0; l < l1; ++l) {
            const LimbConst lc = p.limbs[l];
            const LimbNtt<G> nt{p, lc, l, lds, t};
            u64* c1 = ct + (size_t)l * N;
            u64* c2 = ct + (size_t)(L + l) * N;
            // u_hat -> the c2 slot of this limb, at the positions this thread stores
            const Packed8<R> ul = u.fresh();
            transform_store<REG_EPI>(nt, t, [&](int c) { return small_mod(ul.get(c), lc.q); },
                                     [&](int c) { return (double)ul.get(c); },
                                     [&](uint32_t k, u64 a, u64 b) { store_pair(c2 + k, a, b); });
            // c1 = pk1 u_hat + NTT(m + e1)
            const MessageIn<G, FROM_SLOTS, BGV> msg{stash, pt + (size_t)l * N, e1.fresh(), lc,
                                                    G::tpart(0, opaque_tid(t)), p.noise_t};
            const u64* pk1 = p.pk + (size_t)l * N;
            const u64* pk1s = p.pk_sh + (size_t)l * N;
            transform_store<REG_EPI>(nt, t, [&](int c) { return msg.ri(c); }, [&](int c) { return msg.rf(c); },
                                     [&](uint32_t k, u64 a, u64 b) {
                                         const u64x2 u2 = load_pair(c2 + k), w = load_pair(pk1 + k),
                                                     ws = load_pair(pk1s + k);
                                         final_store(c1 + k, addmod(a, nt.mul(u2.x, w.x, ws.x), lc.q),
                                                     addmod(b, nt.mul(u2.y, w.y, ws.y), lc.q));
                                     });
            // c2 = pk2 u_hat + NTT(e2)
            const Packed8<R> e2l = e2.fresh();
            const u64* pk2 = p.pk + (size_t)(M + l) * N;
            const u64* pk2s = p.pk_sh + (size_t)(M + l) * N;
            transform_store<REG_EPI>(nt, t, [&](int c) { return noise_ri<BGV>(e2l.get(c), p.noise_t, lc); },
                                     [&](int c) { return noise_rf<BGV>(e2l.get(c), p.noise_t, lc); },
                                     [&](uint32_t k, u64 a, u64 b) {
                                         const u64x2 u2 = load_pair(c2 + k), w = load_pair(pk2 + k),
                                                     ws = load_pair(pk2s + k);
                                         final_store(c2 + k, addmod(a, nt.mul(u2.x, w.x, ws.x), lc.q),
                                                     addmod(b, nt.mul(u2.y, w.y, ws.y), lc.q));
                                     });
        }
    }
}

template <int LOGN, int SCHEME, bool FROM_SLOTS, bool BGV = false>
__device__ __forceinline__ void encrypt_item(const DevParams& p, const double* slots, uint32_t n_slots,
                                             const u64* pt, u64 ct_id, u64* ct, u64* lds, const u64* tab,
                                             uint32_t t, uint32_t l0 = 0, uint32_t l1 = ~0u) {
    encrypt_item_g<typename Cfg<LOGN>::G, SCHEME, FROM_SLOTS, false, BGV>(p, slots, n_slots, pt, ct_id, ct, lds,
                                                                          tab, t, l0, l1);
}

// Data limbs of workgroup y of gridDim.y that share one ciphertext.
__device__ __forceinline__ uint32_t limb_group_start(uint32_t L, uint32_t y) { return y * L / gridDim.y; }

}  // namespace zinc
