// Special-prime vanilla encryption for ring degree N = 32768: the computation
// of k_encrypt_sp (Eq. 8's encryption of zero over all M moduli, division by
// the special prime p with rounding, then the message), with every transform
// split after its first stage as in kernels_split.hip.
//
// Rounding in RNS, as for the smaller rings: r = a_j mod p, h = (p - 1)/2,
// D_j = h - ((r + h) mod p) and round(a_j / p) = (a_j + D_j) / p, so data
// limb l of component j is pk_j p^-1 * NTT(u) + NTT((e_j + D_j) p^-1), plus
// NTT(m) in c1.
//
// One workgroup of TS threads per ciphertext.  Per-ciphertext scratch ws
// [3][N] int64: the encoded message (slot path), D_1, D_2.  On the special
// limb, NTT(u) mod p waits in the D_2 row and a_1 = NTT(e_1) + pk_1 NTT(u) in
// the D_1 row, in natural order at the indices the inverse transform's first
// step reads with the same thread; a_2 replaces NTT(u) element by element;
// each inverse transform then writes D_j over a_j in place (it reads all of
// its input before any thread writes output, and parks its half-0 result in
// the first half of the same row).  D_j and the message are read
// back on the data limbs by the thread that wrote them.  The second half's
// input of the c1 transform waits in the upper half of c1, as in the CKKS
// kernels; that of the c2 transform, (e_2 + D_2) p^-1, is recomputed, since
// c2 already holds NTT(u).  Every transform takes the
// integer (Shoup) path, exact for any modulus, as key generation does.
#include "split_common.h"

namespace zinc {

namespace {

using namespace split;

template <bool FROM_SLOTS>
__global__ void __launch_bounds__(TS) __attribute__((amdgpu_waves_per_eu(4)))
k_encrypt_sp_split(DevParams p, EncArgs a, long long* ws_all) {
    __shared__ u64 lds[LdsWords<NH>::value];
    __shared__ u64 tab[kCdtTab];
    const uint32_t t = threadIdx.x, b = blockIdx.x;
    const u64 ct_id = a.ct_ids[b];
    if (reserved_id(p, a, ct_id, t)) return;
    load_cdt(tab, p.cdt, t);
    const uint32_t L = p.L, M = p.M;
    long long* wm = ws_all + (size_t)b * 3 * NF;
    long long* wd1 = wm + NF;
    long long* wd2 = wm + 2 * NF;
    u64* ct = a.ct + (size_t)b * 2 * L * NF;
    const u64* pt = FROM_SLOTS ? nullptr : a.pt + (size_t)b * L * NF;

    if constexpr (FROM_SLOTS) {
        long long mlo[RS], mhi[RS];
        encode_split(mlo, mhi, lds, p, a.slots + (size_t)b * a.n_slots, a.n_slots, t);
        const uint32_t tp0 = GS::tpart(0, t);
#pragma unroll
        for (int c = 0; c < RS; ++c) {
            wm[jp(tp0, c)] = mlo[c];
            wm[NH + jp(tp0, c)] = mhi[c];
        }
    }
    Pair8 u, e1, e2;
    sample_ternary_split(u, p, ct_id, TAG_U, t);
    sample_gauss_split(e1, p, tab, ct_id, TAG_E1, t);
    sample_gauss_split(e2, p, tab, ct_id, TAG_E2, t);

    // forward transform of a small-coefficient polynomial, both halves, with
    // epilogue epi(h, k) reading output k of half h from LDS
    auto small_fwd = [&](const SplitLimb& sl, const Pair8& e, auto&& epi) {
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            const Pair8 el = e.fresh();
            sl.run_half(h, [&](int c) { return sl.stage0(sl.small(el.lo.get(c)), sl.small(el.hi.get(c)), h); });
            epi(h);
        }
    };

    // ---- the special limb: the rounding offsets D_1, D_2 ----
    {
        LimbConst lc = p.limbs[L];
        lc.fp = 0;
        const SplitLimb sl(p, lc, L, lds, t);
        u64* ua = reinterpret_cast<u64*>(wd2);     // NTT(u) mod p, then a_2
        small_fwd(sl, u, [&](int h) {
            const uint32_t tt = opaque_tid(t);
#pragma unroll
            for (int i = 0; i < RS; ++i) ua[(uint32_t)h * NH + tt + TS * i] = sl.canon(tt + TS * i);
        });
#pragma unroll 1
        for (int j = 0; j < 2; ++j) {
            const u64* pkj = p.pk + ((size_t)j * M + L) * NF;
            const u64* pkjs = p.pk_sh + ((size_t)j * M + L) * NF;
            long long* wd = j == 0 ? wd1 : wd2;
            u64* aj = reinterpret_cast<u64*>(wd);
            small_fwd(sl, j == 0 ? e1 : e2, [&](int h) {
                const uint32_t tt = opaque_tid(t);
#pragma unroll
                for (int i = 0; i < RS; ++i) {
                    const uint32_t k = tt + TS * i, kk = (uint32_t)h * NH + k;
                    aj[kk] = addmod(sl.canon(k), sl.mul(ua[kk], pkj[kk], pkjs[kk]), lc.q);   // a_j mod p
                }
            });
            intt_split(p, lc, L, lds, t, [&](uint32_t k) { return aj[k]; }, [&](uint32_t k, u64 x) {
                wd[k] = (long long)lc.half - (long long)addmod(x, lc.half, lc.q);
            }, aj);
        }
    }

    // ---- the data limbs ----
#pragma unroll 1
    for (uint32_t l = 0; l < L; ++l) {
        LimbConst lc = p.limbs[l];
        lc.fp = 0;
        const SplitLimb sl(p, lc, l, lds, t);
        u64* c1 = ct + (size_t)l * NF;
        u64* c2 = ct + (size_t)(L + l) * NF;
        small_fwd(sl, u, [&](int h) {            // NTT(u) -> c2, at the pairs this thread stores below
            const uint32_t tt = opaque_tid(t);
#pragma unroll
            for (int i = 0; i < RS / 2; ++i) {
                const uint32_t k = 2 * (tt + TS * i);
                store_pair(c2 + (uint32_t)h * NH + k, sl.canon(k), sl.canon(k + 1));
            }
        });
        // canonical inputs (e_1 + D_1) p^-1 + m and (e_2 + D_2) p^-1 at coefficient k
        auto in1 = [&](uint32_t k, int e) {
            const u64 y = csub(shoup_lazy(reduce_signed(e + wd1[k], lc), lc.pinv, lc.pinv_sh, lc.q), lc.q);
            u64 mm;
            if constexpr (FROM_SLOTS) mm = reduce_signed(wm[k], lc);
            else mm = pt[(size_t)l * NF + k];
            return addmod(y, mm, lc.q);
        };
        auto in2 = [&](uint32_t k, int e) {
            return csub(shoup_lazy(reduce_signed(e + wd2[k], lc), lc.pinv, lc.pinv_sh, lc.q), lc.q);
        };
        // dst = NTT(input) + pkp * NTT(u), both halves.  STASH: the second
        // half's stage-0 output waits in the upper half of dst (read back by the
        // thread that wrote it before any thread stores there); otherwise the
        // input is recomputed for the second half.
        auto enc_ntt = [&](const Pair8& e, auto&& in, const u64* w, const u64* ws, u64* dst, auto stash) {
            constexpr bool STASH = decltype(stash)::value;
#pragma unroll 1
            for (int h = 0; h < 2; ++h) {
                const Pair8 el = e.fresh();
                const uint32_t tp0 = GS::tpart(0, opaque_tid(t));
                if (STASH && h == 1) {
                    sl.run_half(1, [&](int c) { return dst[NH + jp(tp0, c)]; });
                } else {
                    sl.run_half(h, [&](int c) {
                        const uint32_t k = jp(tp0, c);
                        const u64 xl = sl.residue(in(k, el.lo.get(c))), xh = sl.residue(in(NH + k, el.hi.get(c)));
                        if constexpr (STASH) dst[NH + k] = sl.stage0(xl, xh, 1);
                        return sl.stage0(xl, xh, h);
                    });
                }
                const uint32_t tt = opaque_tid(t);
#pragma unroll
                for (int i = 0; i < RS / 2; ++i) {
                    const uint32_t k = 2 * (tt + TS * i), kk = (uint32_t)h * NH + k;
                    const u64x2 u2 = load_pair(c2 + kk), ww = load_pair(w + kk), wws = load_pair(ws + kk);
                    store_pair_final(dst + kk, addmod(sl.canon(k), sl.mul(u2.x, ww.x, wws.x), lc.q),
                                     addmod(sl.canon(k + 1), sl.mul(u2.y, ww.y, wws.y), lc.q));
                }
            }
        };
        enc_ntt(e1, in1, p.pkp + (size_t)l * NF, p.pkp_sh + (size_t)l * NF, c1, std::true_type{});
        enc_ntt(e2, in2, p.pkp + (size_t)(L + l) * NF, p.pkp_sh + (size_t)(L + l) * NF, c2, std::false_type{});
    }
}

}  // namespace

hipError_t launch_split_encrypt_sp(const DevParams& p, bool from_slots, const double* slots, uint32_t n_slots,
                                   const uint64_t* pt, uint32_t batch, const uint64_t* ct_ids, uint64_t* ct,
                                   int64_t* ws, hipStream_t s) {
    const EncArgs a{slots, n_slots, (const u64*)pt, (const u64*)ct_ids, (u64*)ct};
    long long* w = reinterpret_cast<long long*>(ws);
    if (from_slots) hipLaunchKernelGGL((k_encrypt_sp_split<true>), dim3(batch), dim3(TS), 0, s, p, a, w);
    else hipLaunchKernelGGL((k_encrypt_sp_split<false>), dim3(batch), dim3(TS), 0, s, p, a, w);
    return hipGetLastError();
}

}  // namespace zinc
