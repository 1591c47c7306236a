// Vanilla encryption the way a library with a special prime p = q_{M-1}
// computes it: Eq. 8's encryption of zero over all M moduli, a_j = pk_j u + e_j,
// divided by p with rounding down to the L data limbs, then the message added.
//
// Rounding in RNS: with r = a_j mod p (coefficients in [0, p)), h = (p - 1)/2
// and t = (r + h) mod p, round(a_j / p) = (a_j + h - t) / p exactly, so limb l
// is (a_j + (h - t)) p^-1 mod q_l.  By linearity of the transform, on a data
// limb this is pk_j p^-1 * NTT(u) + NTT((e_j + h - t) p^-1) (+ NTT(m) in
// c1): the same three forward transforms per data limb as Eq. 8, with
// pk_j p^-1 precomputed at key generation and the offsets D_j = h - t (small
// integers, |D_j| <= p/2) computed once on the special limb: three forward
// transforms and two inverse transforms there.
//
// One workgroup per ciphertext.  Per-ciphertext scratch ws [3][N] int64:
// the encoded message, D_1, D_2 (pass-0 layout, each thread reads back what
// it wrote).  NTT(u) mod p waits in the D_2 row (in the last pass's layout)
// until D_2 overwrites it after the inverse transform's first barrier.
#include <mutex>

#include "kernels_common.h"

namespace zinc {

namespace {

template <int LOGN, bool FROM_SLOTS>
__global__ void __launch_bounds__(Cfg<LOGN>::G::T) __attribute__((amdgpu_waves_per_eu(4)))
k_encrypt_sp(DevParams p, EncArgs a, long long* ws_all) {
    using G = typename Cfg<LOGN>::G;
    constexpr int R = G::R, N = G::N;
    __shared__ u64 lds[LdsWords<N>::value];
    __shared__ u64 tab[kCdtTab];
    const uint32_t t = threadIdx.x, b = blockIdx.x;
    const u64 ct_id = a.ct_ids[b];
    if (reserved_id(p, a, ct_id, t)) return;
    load_cdt(tab, p.cdt, t);
    const uint32_t L = p.L, M = p.M;
    long long* wm = ws_all + (size_t)b * 3 * N;
    long long* wd1 = wm + N;
    long long* wd2 = wm + 2 * N;
    u64* ct = a.ct + (size_t)b * 2 * L * N;
    const u64* pt = FROM_SLOTS ? nullptr : a.pt + (size_t)b * L * N;

    if constexpr (FROM_SLOTS) {
        long long m[R];
        encode_p0<G>(m, lds, p, a.slots + (size_t)b * a.n_slots, a.n_slots, t);
        const uint32_t tp0 = G::tpart(0, t);
#pragma unroll
        for (int c = 0; c < R; ++c) wm[tp0 | G::cpart(0, c)] = m[c];
    }
    Packed8<R> u, e1, e2;
    sample_ternary_p0<G>(u, p, ct_id, TAG_U, t);
    sample_gauss_p0<G>(e1, p, tab, ct_id, TAG_E1, t);
    sample_gauss_p0<G>(e2, p, tab, ct_id, TAG_E2, t);

    // ---- the special limb: the rounding offsets D_1, D_2 ----
    {
        const LimbConst lc = p.limbs[L];
        const LimbNtt<G> nt{p, lc, L, lds, t};
        u64 r[R];
        const Packed8<R> ul = u.fresh();
        nt.run_regs([&](int c) { return small_mod(ul.get(c), lc.q); }, [&](int c) { return (double)ul.get(c); }, r);
        {
            const uint32_t tt = opaque_tid(t);
#pragma unroll
            for (int c = 0; c < R; ++c) wd2[out_index<G>(tt, c)] = (long long)r[c];   // NTT(u) mod p
        }
#pragma unroll 1
        for (int j = 0; j < 2; ++j) {
            const Packed8<R> ej = (j == 0 ? e1 : e2).fresh();
            nt.run_regs([&](int c) { return small_mod(ej.get(c), lc.q); }, [&](int c) { return (double)ej.get(c); },
                        r);
            const u64* pkj = p.pk + ((size_t)j * M + L) * N;
            const u64* pkjs = p.pk_sh + ((size_t)j * M + L) * N;
            {
                const uint32_t tt = opaque_tid(t);
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    const uint32_t k = out_index<G>(tt, c);
                    r[c] = addmod(r[c], nt.mul((u64)wd2[k], pkj[k], pkjs[k]), lc.q);       // a_j mod p
                }
            }
            ntt_inv<G>(r, lds, p.itw, L, lc.q, lc.q2, t);       // -> pass-0 layout, N^-1 pending
            const uint32_t tp0 = G::tpart(0, opaque_tid(t));
            long long* wd = j == 0 ? wd1 : wd2;
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const u64 x = csub(shoup_lazy(r[c], lc.ninv, lc.ninv_sh, lc.q), lc.q);   // a_j mod p, in [0, p)
                const u64 tr = addmod(x, lc.half, lc.q);
                wd[tp0 | G::cpart(0, c)] = (long long)lc.half - (long long)tr;
            }
        }
    }

    // ---- the data limbs ----
#pragma unroll 1
    for (uint32_t l = 0; l < L; ++l) {
        const LimbConst lc = p.limbs[l];
        const LimbNtt<G> nt{p, lc, l, lds, t};
        u64* c1 = ct + (size_t)l * N;
        u64* c2 = ct + (size_t)(L + l) * N;
        // NTT(u) -> the c2 slot of this limb, at the positions this thread stores
        const Packed8<R> ul = u.fresh();
        transform_store<false>(nt, t, [&](int c) { return small_mod(ul.get(c), lc.q); },
                               [&](int c) { return (double)ul.get(c); },
                               [&](uint32_t k, u64 x, u64 y) { store_pair(c2 + k, x, y); });
        // inputs (e_1 + D_1) p^-1 + m and (e_2 + D_2) p^-1, canonical
        const uint32_t tp0 = G::tpart(0, opaque_tid(t));
        const Packed8<R> e1l = e1.fresh();
        auto in1 = [&](int c) {
            const uint32_t k = tp0 | G::cpart(0, c);
            const u64 y = csub(shoup_lazy(reduce_signed(e1l.get(c) + wd1[k], lc), lc.pinv, lc.pinv_sh, lc.q), lc.q);
            u64 mm;
            if constexpr (FROM_SLOTS) mm = reduce_signed(wm[k], lc);
            else mm = pt[(size_t)l * N + k];
            return addmod(y, mm, lc.q);
        };
        const u64* w1 = p.pkp + (size_t)l * N;
        const u64* w1s = p.pkp_sh + (size_t)l * N;
        transform_store<false>(nt, t, in1, [&](int c) { return u64_to_fp(in1(c)); },
                               [&](uint32_t k, u64 x, u64 y) {
                                   const u64x2 u2 = load_pair(c2 + k), w = load_pair(w1 + k), ws = load_pair(w1s + k);
                                   store_pair_final(c1 + k, addmod(x, nt.mul(u2.x, w.x, ws.x), lc.q),
                                                    addmod(y, nt.mul(u2.y, w.y, ws.y), lc.q));
                               });
        const Packed8<R> e2l = e2.fresh();
        auto in2 = [&](int c) {
            const uint32_t k = tp0 | G::cpart(0, c);
            return csub(shoup_lazy(reduce_signed(e2l.get(c) + wd2[k], lc), lc.pinv, lc.pinv_sh, lc.q), lc.q);
        };
        const u64* w2 = p.pkp + (size_t)(L + l) * N;
        const u64* w2s = p.pkp_sh + (size_t)(L + l) * N;
        transform_store<false>(nt, t, in2, [&](int c) { return u64_to_fp(in2(c)); },
                               [&](uint32_t k, u64 x, u64 y) {
                                   const u64x2 u2 = load_pair(c2 + k), w = load_pair(w2 + k), ws = load_pair(w2s + k);
                                   store_pair_final(c2 + k, addmod(x, nt.mul(u2.x, w.x, ws.x), lc.q),
                                                    addmod(y, nt.mul(u2.y, w.y, ws.y), lc.q));
                               });
    }
}

// pkp_j[l] = pk_j[l] p^-1 mod q_l on the data limbs, with Shoup companions.
__global__ void __launch_bounds__(256) k_scale_pk(DevParams p, u64* pkp, u64* pkp_sh) {
    const uint32_t n = p.n, L = p.L, M = p.M;
    const size_t total = (size_t)2 * L * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t row = (uint32_t)(i / n), j = row / L, l = row % L;
        const LimbConst lc = p.limbs[l];
        const u64 w = p.pk[((size_t)j * M + l) * n + i % n];
        const u64 v = csub(shoup_lazy(w, lc.pinv, lc.pinv_sh, lc.q), lc.q);
        pkp[i] = v;
        pkp_sh[i] = shoup_companion_dev(v, lc.q);
    }
}

}  // namespace

hipError_t launch_scale_pk(const DevParams& p, uint64_t* pkp, uint64_t* pkp_sh, hipStream_t s) {
    const uint32_t blocks = (uint32_t)(((size_t)2 * p.L * p.n + 255) / 256);
    hipLaunchKernelGGL(k_scale_pk, dim3(blocks), dim3(256), 0, s, p, (u64*)pkp, (u64*)pkp_sh);
    return hipGetLastError();
}

hipError_t launch_encrypt_sp(const DevParams& p, bool from_slots, const double* slots, uint32_t n_slots,
                             const uint64_t* pt, uint32_t batch, const uint64_t* ct_ids, uint64_t* ct, int64_t* ws,
                             hipStream_t s) {
    const EncArgs a{slots, n_slots, (const u64*)pt, (const u64*)ct_ids, (u64*)ct};
    long long* w = reinterpret_cast<long long*>(ws);
#define F(LN)                                                                                              \
    case LN:                                                                                               \
        if (from_slots)                                                                                    \
            hipLaunchKernelGGL((k_encrypt_sp<LN, true>), dim3(batch), dim3(Cfg<LN>::G::T), 0, s, p, a, w); \
        else                                                                                               \
            hipLaunchKernelGGL((k_encrypt_sp<LN, false>), dim3(batch), dim3(Cfg<LN>::G::T), 0, s, p, a, w); \
        break;
    switch (p.log_n) {
        case 15: return launch_split_encrypt_sp(p, from_slots, slots, n_slots, pt, batch, ct_ids, ct, ws, s);
        F(12)
        F(13)
        F(14)
        default: return hipErrorInvalidValue;
    }
#undef F
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point (zinc_encrypt_vanilla_sp_noalloc):
// a file-scope device array, one copy per GPU at its own address, held until
// the process ends and shared by every call on that GPU.  On the host the
// array's name only stands in for the device symbol, so host code uses the
// address hipGetSymbolAddress gives for the current device, never the name.
// ---------------------------------------------------------------------------
static __device__ __align__(256) long long scratch[kSpScratchBytes / sizeof(long long)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
long long* g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t sp_scratch(int device, long long** out) {
    *out = nullptr;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device || device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[device] = static_cast<long long*>(p);
    }
    *out = g_scratch[device];
    return hipSuccess;
}

}  // namespace zinc
