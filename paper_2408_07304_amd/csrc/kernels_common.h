// Helpers shared by the encryption kernels of every ring degree.
#pragma once

#include "device.h"

namespace zinc {

struct EncArgs {
    const double* slots;     // [batch][n_slots] (FROM_SLOTS)
    uint32_t n_slots;
    const u64* pt;           // [batch][L][N]   (!FROM_SLOTS)
    const u64* ct_ids;       // [batch]
    u64* ct;                 // [batch][2][L][N]
};

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
    template <class InInt, class InFp>
    __device__ __forceinline__ void run(InInt in_int, InFp in_fp) const {
        if (fp()) {
            double v[G::R];
#pragma unroll
            for (int c = 0; c < G::R; ++c) v[c] = in_fp(c);
            double* ld = reinterpret_cast<double*>(lds);
            ntt_fwd_fp<G>(v, ld, tw_fp, limb, qd, qinv, mode == 2, t);
            to_natural<G>(ld, v, t);
        } else {
            u64 v[G::R];
#pragma unroll
            for (int c = 0; c < G::R; ++c) v[c] = in_int(c);
            ntt_fwd<G>(v, lds, tw, limb, q, q2, t);
            to_natural<G>(lds, v, t);
        }
    }

    // canonical residue of transform coefficient k (after run())
    __device__ __forceinline__ u64 canon(uint32_t k) const {
        if (fp()) return fp_canon(reinterpret_cast<const double*>(lds)[pad(k)], qd, qinv);
        return canon4(lds[pad(k)], q, q2);
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

// Pass-0 message input of limb l: (m + e) with m read back from the stash
// (encoded slots) or from the caller's plaintext residues.
template <class G, bool FROM_SLOTS>
struct MessageIn {
    const long long* stash;
    const u64* pt;
    Packed8<G::R> e;
    LimbConst lc;
    uint32_t tp0;
    __device__ __forceinline__ u64 ri(int c) const {       // residue in [0, 2q)
        const uint32_t k = tp0 | G::cpart(0, c);
        if constexpr (FROM_SLOTS) return reduce_signed(stash[k] + e.get(c), lc);
        else return pt[k] + small_mod(e.get(c), lc.q);
    }
    __device__ __forceinline__ double rf(int c) const {    // |value| <= q
        const uint32_t k = tp0 | G::cpart(0, c);
        if constexpr (FROM_SLOTS) return u64_to_fp(reduce_signed(stash[k] + e.get(c), lc));
        else return u64_to_fp(pt[k]) + (double)e.get(c);
    }
};

}  // namespace zinc
