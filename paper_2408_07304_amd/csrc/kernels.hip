// HIP kernels for gfx950: key generation (Eq. 7), vanilla encryption (Eq. 8),
// Zinc encryption (Algorithm 1), CKKS encode/decode, decryption, homomorphic
// addition (Eq. 2), and the kernel-level NTT and sampler entry points.
//
// One workgroup owns one ciphertext: it draws the ciphertext's noise once
// into registers, encodes its slot vector once (FP64 FFT in LDS), and then
// runs every limb's NTTs through one LDS exchange buffer, adding the cached
// Enc(0) (Zinc) or pk * NTT(u) (vanilla) in the coalesced store epilogue.
#include "kernels_common.h"

namespace zinc {

// ---------------------------------------------------------------------------
// encryption
// ---------------------------------------------------------------------------
// SPLIT: the workgroups y = 0 .. gridDim.y - 1 of ciphertext b share its data
// limbs (small batches, limb_groups); otherwise one workgroup does all of them
// (a separate instantiation, so that the usual form keeps its code).
template <int LOGN, int SCHEME, bool FROM_SLOTS, bool BGV = false, bool SPLIT = false>
__global__ void __launch_bounds__(Cfg<LOGN>::G::T) __attribute__((amdgpu_waves_per_eu(4)))
k_encrypt(typename ParamArg<LOGN>::type pa, EncArgs a) {
    const DevParams& p = deref(pa);
    using G = typename Cfg<LOGN>::G;
    constexpr int N = G::N;
    __shared__ u64 lds[LdsWords<N>::value];
    __shared__ u64 tab[kCdtTab];
    const uint32_t t = threadIdx.x;
    const uint32_t b = blockIdx.x;
    const u64 id = a.ct_ids[b];
    if (reserved_id(p, a, id, t)) return;
    load_cdt(tab, p.cdt, t);
    const uint32_t L = p.L;
    encrypt_item<LOGN, SCHEME, FROM_SLOTS, BGV>(p, a.slots + (size_t)b * a.n_slots, a.n_slots,
                                          a.pt + (size_t)b * L * N, id, a.ct + (size_t)b * 2 * L * N,
                                          lds, tab, t, SPLIT ? limb_group_start(L, blockIdx.y) : 0u,
                                          SPLIT ? limb_group_start(L, blockIdx.y + 1) : ~0u);
}

// ---------------------------------------------------------------------------
// key generation: one workgroup per modulus (all M of them)
// ---------------------------------------------------------------------------
template <int LOGN>
__global__ void __launch_bounds__(Cfg<LOGN>::G::T) k_keygen(DevParams p, u64* sk, u64* sk_sh, u64* pk,
                                                              u64* pk_sh) {
    using G = typename Cfg<LOGN>::G;
    constexpr int R = G::R, N = G::N;
    __shared__ u64 lds[LdsWords<N>::value];
    __shared__ u64 tab[kCdtTab];
    const uint32_t t = threadIdx.x;
    const uint32_t l = blockIdx.x;
    load_cdt(tab, p.cdt, t);
    const LimbConst lc = p.limbs[l];
    const u64 q = lc.q, q2 = lc.q2;
    const uint32_t M = p.M;

    Packed8<R> s, e;
    sample_ternary_p0<G>(s, p, ZINC_KEY_ID, TAG_SK, t);
    sample_gauss_p0<G>(e, p, tab, ZINC_KEY_ID, TAG_EPK, t);
    u64 v[R];
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = small_mod(s.get(c), q);
    ntt_fwd<G>(v, lds, p.tw, l, q, q2, t);
    to_natural<G>(lds, v, t);
    u64 sh[R], shs[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t k = t + G::T * i;
        sh[i] = canon16(lds[pad(k)], q);
        shs[i] = shoup_companion_dev(sh[i], q);
        sk[(size_t)l * N + k] = sh[i];
        sk_sh[(size_t)l * N + k] = shs[i];
    }
    const u64 et = p.noise_t > 1 ? p.noise_t : 0;      // BGV: the error is t e (Eq. 13)
#pragma unroll
    for (int c = 0; c < R; ++c)
        v[c] = et ? reduce_signed((long long)e.get(c) * (long long)et, lc) : small_mod(e.get(c), q);
    ntt_fwd<G>(v, lds, p.tw, l, q, q2, t);
    to_natural<G>(lds, v, t);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t k = t + G::T * i;
        const u64 eh = canon16(lds[pad(k)], q);
        // a <- R_q, drawn directly in the NTT domain: 128 uniform bits mod q
        const U4 r = draw(p.seed, ZINC_KEY_ID, TAG_A, l, k);
        const u64 hi = ((u64)r.w << 32) | r.z, lo = ((u64)r.y << 32) | r.x;
        const u64 ah = mod128(mod128(0, hi, q), lo, q);
        const u64 as = csub(shoup_lazy(ah, sh[i], shs[i], q), q);      // a * s
        const u64 p1 = addmod(as ? q - as : 0, eh, q);                   // -a s + e
        pk[(size_t)l * N + k] = p1;
        pk[(size_t)(M + l) * N + k] = ah;
        pk_sh[(size_t)l * N + k] = shoup_companion_dev(p1, q);
        pk_sh[(size_t)(M + l) * N + k] = shoup_companion_dev(ah, q);
    }
}

// ---------------------------------------------------------------------------
// encode: slots -> residues of the integer coefficients, per data limb
// ---------------------------------------------------------------------------
template <int LOGN>
__global__ void __launch_bounds__(Cfg<LOGN>::G::T) k_encode(DevParams p, const double* slots,
                                                              uint32_t n_slots, u64* pt) {
    using G = typename Cfg<LOGN>::G;
    constexpr int R = G::R, N = G::N;
    __shared__ u64 lds[LdsWords<N>::value];
    const uint32_t t = threadIdx.x, b = blockIdx.x;
    long long m[R];
    // n_slots is the same in every workgroup: no barrier is skipped by some threads only
    if (n_slots <= kSparseSlots) encode_sparse_p0<G>(m, p, slots + (size_t)b * n_slots, n_slots, t);
    else encode_p0<G>(m, lds, p, slots + (size_t)b * n_slots, n_slots, t);
    const uint32_t tp0 = G::tpart(0, t);
    for (uint32_t l = 0; l < p.L; ++l) {
        const LimbConst lc = p.limbs[l];
        u64* out = pt + ((size_t)b * p.L + l) * N;
#pragma unroll
        for (int c = 0; c < R; ++c) out[tp0 | G::cpart(0, c)] = reduce_signed(m[c], lc);
    }
}

// ---------------------------------------------------------------------------
// decrypt: p = INTT(c1 + c2 s_hat), one workgroup per (limb, ciphertext)
// ---------------------------------------------------------------------------
template <int LOGN>
__global__ void __launch_bounds__(Cfg<LOGN>::G::T) k_decrypt(DevParams p, const u64* ct, u64* pt) {
    using G = typename Cfg<LOGN>::G;
    constexpr int R = G::R, N = G::N, PL = G::NPASS - 1;
    __shared__ u64 lds[LdsWords<N>::value];
    const uint32_t t = threadIdx.x, l = blockIdx.x, b = blockIdx.y, L = p.L;
    const LimbConst lc = p.limbs[l];
    const u64 q = lc.q, q2 = lc.q2;
    const u64* c1 = ct + ((size_t)b * 2 * L + l) * N;
    const u64* c2 = ct + ((size_t)b * 2 * L + L + l) * N;
    const u64* s = p.sk + (size_t)l * N;
    const u64* ss = p.sk_sh + (size_t)l * N;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t k = t + G::T * i;
        lds[pad(k)] = csub(c1[k] + csub(shoup_lazy(c2[k], s[k], ss[k], q), q), q2);   // [0, 2q)
    }
    __syncthreads();
    u64 v[R];
    lds_get<G, PL>(lds, v, t);
    ntt_inv<G>(v, lds, p.itw, l, q, q2, t);
    u64* out = pt + ((size_t)b * L + l) * N;
    const uint32_t tp0 = G::tpart(0, t);
#pragma unroll
    for (int c = 0; c < R; ++c) out[tp0 | G::cpart(0, c)] = csub(shoup_lazy(v[c], lc.ninv, lc.ninv_sh, q), q);
}

// ---------------------------------------------------------------------------
// decode: centred lift of limb 0, FP64 FFT, z_j = Re m(zeta^(5^j)) / Delta
// ---------------------------------------------------------------------------
template <int LOGN>
__global__ void __launch_bounds__(Cfg<LOGN>::G::T) k_decode(DevParams p, const u64* pt, double* slots) {
    using G = typename Cfg<LOGN>::G;
    constexpr int N = G::N, H = N / 2, LOGH = LOGN - 1, T = G::T;
    __shared__ u64 lds[LdsWords<N>::value];
    C2* A = reinterpret_cast<C2*>(lds);
    const uint32_t t = threadIdx.x, b = blockIdx.x, L = p.L;
    const LimbConst l0 = p.limbs[0];
    const u64* x0 = pt + (size_t)b * L * N;
    bool bad = false;
    for (uint32_t i = t; i < (uint32_t)H; i += T) {
        long long v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t k = i + h * H;
            const u64 r = x0[k];
            v[h] = r > l0.half ? (long long)r - (long long)l0.q : (long long)r;
            if (L > 1) {
                const LimbConst l1 = p.limbs[1];
                bad |= reduce_signed(v[h], l1) != x0[(size_t)N + k];
            }
        }
        // y_i = (m_i + i m_{i+H}) zeta^i, scattered to bit-reversed position
        const C2 y = cmul(C2{(double)v[0], (double)v[1]}, C2{p.twist[2 * i], -p.twist[2 * i + 1]});
        A[__brev(i) >> (32 - LOGH)] = y;
    }
    if (bad) atomicOr(p.err, 2u);
    __syncthreads();
    fft_dit<LOGH, T, +1>(A, p.fft_tw, t);
    const double inv = 1.0 / p.scale;
    for (uint32_t j = t; j < (uint32_t)H; j += T) {
        const uint32_t kj = __brev(p.slot_pos[j]) >> (32 - LOGH);
        slots[(size_t)b * H + j] = A[kj].x * inv;
    }
}

// ---------------------------------------------------------------------------
// homomorphic addition (Eq. 2), streaming
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_add(DevParams p, const u64* __restrict__ a, const u64* __restrict__ b,
                                             u64* __restrict__ out, size_t n_pairs) {
    const uint32_t log_n = p.log_n, L = p.L;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pairs;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t e = 2 * i;
        const uint32_t limb = (uint32_t)((e >> log_n) % L);
        const u64 q = p.limbs[limb].q;
        const ulonglong2 x = reinterpret_cast<const ulonglong2*>(a)[i];
        const ulonglong2 y = reinterpret_cast<const ulonglong2*>(b)[i];
        reinterpret_cast<ulonglong2*>(out)[i] = make_ulonglong2(addmod(x.x, y.x, q), addmod(x.y, y.y, q));
    }
}

// ---------------------------------------------------------------------------
// kernel-level entry points: standalone NTT and samplers
// ---------------------------------------------------------------------------
template <int LOGN, bool INV>
__global__ void __launch_bounds__(Cfg<LOGN>::G::T) k_ntt(DevParams p, uint32_t limb, u64* poly) {
    using G = typename Cfg<LOGN>::G;
    constexpr int R = G::R, N = G::N, PL = G::NPASS - 1;
    __shared__ u64 lds[LdsWords<N>::value];
    const uint32_t t = threadIdx.x;
    u64* x = poly + (size_t)blockIdx.x * N;
    const LimbConst lc = p.limbs[limb];
    const u64 q = lc.q, q2 = lc.q2;
    const uint32_t tp0 = G::tpart(0, t);
    if constexpr (!INV) {
        // the same per-modulus arithmetic as the encryption kernels
        const LimbNtt<G> nt{p, lc, limb, lds, t};
        nt.run([&](int c) { return x[tp0 | G::cpart(0, c)]; }, [&](int c) { return u64_to_fp(x[tp0 | G::cpart(0, c)]); });
#pragma unroll
        for (int i = 0; i < R; ++i) x[t + G::T * i] = nt.canon(t + G::T * i);
    } else {
        u64 v[R];
#pragma unroll
        for (int i = 0; i < R; ++i) lds[pad(t + G::T * i)] = x[t + G::T * i];
        __syncthreads();
        lds_get<G, PL>(lds, v, t);
        ntt_inv<G>(v, lds, p.itw, limb, q, q2, t);
#pragma unroll
        for (int c = 0; c < R; ++c) x[tp0 | G::cpart(0, c)] = csub(shoup_lazy(v[c], lc.ninv, lc.ninv_sh, q), q);
    }
}

__global__ void __launch_bounds__(256) k_sample(DevParams p, int kind, uint32_t tag, uint32_t limb,
                                                const u64* ct_ids, void* out) {
    __shared__ u64 tab[kCdtTab];
    load_cdt(tab, p.cdt, threadIdx.x);
    const uint32_t n = p.n, b = blockIdx.y;
    const u64 id = ct_ids[b];
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        if (kind == 0) {
            const U4 r = draw(p.seed, id, tag, 0, k % (n / 4));
            const uint32_t w[4] = {r.x, r.y, r.z, r.w};
            reinterpret_cast<long long*>(out)[(size_t)b * n + k] = ternary_from(w[k / (n / 4)]);
        } else if (kind == 1) {
            const U4 r = draw(p.seed, id, tag, 0, k % (n / 2));
            const u64 uu = (k / (n / 2)) ? ((u64)r.z | ((u64)r.w << 32)) : ((u64)r.x | ((u64)r.y << 32));
            reinterpret_cast<long long*>(out)[(size_t)b * n + k] = gauss_sample(uu, tab);
        } else {
            const u64 q = p.limbs[limb].q;
            const U4 r = draw(p.seed, id, tag, limb, k);
            const u64 hi = ((u64)r.w << 32) | r.z, lo = ((u64)r.y << 32) | r.x;
            reinterpret_cast<u64*>(out)[(size_t)b * n + k] = mod128(mod128(0, hi, q), lo, q);
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define ZINC_DISPATCH_LOGN(logn, F) \
    switch (logn) {                 \
        case 12: F(12); break;      \
        case 13: F(13); break;      \
        case 14: F(14); break;      \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_keygen(const DevParams& p, uint64_t* sk, uint64_t* sk_sh, uint64_t* pk,
                         uint64_t* pk_sh, hipStream_t s) {
    if (p.log_n == 15) return launch_split_keygen(p, sk, sk_sh, pk, pk_sh, s);
#define F(LN) hipLaunchKernelGGL(k_keygen<LN>, dim3(p.M), dim3(Cfg<LN>::G::T), 0, s, p, \
                                 (u64*)sk, (u64*)sk_sh, (u64*)pk, (u64*)pk_sh)
    ZINC_DISPATCH_LOGN(p.log_n, F)
#undef F
    return hipGetLastError();
}

hipError_t launch_encrypt_pt(const DevParams& p, int scheme, const uint64_t* pt, uint32_t batch,
                             const uint64_t* ct_ids, uint64_t* ct, hipStream_t s, bool reserved_ok) {
    if (p.log_n == 15)
        return launch_split_encrypt(p, scheme, false, nullptr, 0, pt, batch, ct_ids, ct, s, reserved_ok);
    EncArgs a{nullptr, 0, (const u64*)pt, (const u64*)ct_ids, (u64*)ct, reserved_ok ? 1u : 0u};
    const bool bgv = p.noise_t > 1;
    const uint32_t S = limb_groups(p, batch);
#define G_(LN, SCH, B)                                                                                       \
    do {                                                                                                     \
        if (S > 1)                                                                                           \
            hipLaunchKernelGGL((k_encrypt<LN, SCH, false, B, true>), dim3(batch, S), dim3(Cfg<LN>::G::T), 0, \
                               s, ParamArg<LN>::of(p), a);                                                   \
        else                                                                                                 \
            hipLaunchKernelGGL((k_encrypt<LN, SCH, false, B>), dim3(batch), dim3(Cfg<LN>::G::T), 0, s,       \
                               ParamArg<LN>::of(p), a);                                                      \
    } while (0)
#define F(LN)                                        \
    if (scheme == ZINC_SCHEME_ZINC) {                \
        if (bgv) G_(LN, ZINC_SCHEME_ZINC, true);     \
        else G_(LN, ZINC_SCHEME_ZINC, false);        \
    } else {                                         \
        if (bgv) G_(LN, ZINC_SCHEME_VANILLA, true);  \
        else G_(LN, ZINC_SCHEME_VANILLA, false);     \
    }
    ZINC_DISPATCH_LOGN(p.log_n, F)
#undef F
#undef G_
    return hipGetLastError();
}

hipError_t launch_encrypt_slots(const DevParams& p, int scheme, const double* slots, uint32_t n_slots,
                                uint32_t batch, const uint64_t* ct_ids, uint64_t* ct, hipStream_t s) {
    if (p.log_n == 15)
        return launch_split_encrypt(p, scheme, true, slots, n_slots, nullptr, batch, ct_ids, ct, s);
    EncArgs a{slots, n_slots, nullptr, (const u64*)ct_ids, (u64*)ct};
    const uint32_t S = limb_groups(p, batch);
#define H_(LN, SCH, SP) \
    hipLaunchKernelGGL((k_encrypt<LN, SCH, true, false, SP>), dim3(batch, S), dim3(Cfg<LN>::G::T), 0, s, \
                       ParamArg<LN>::of(p), a)
#define F(LN)                                                        \
    if (scheme == ZINC_SCHEME_ZINC) {                                \
        if (S > 1) H_(LN, ZINC_SCHEME_ZINC, true);                   \
        else H_(LN, ZINC_SCHEME_ZINC, false);                        \
    } else {                                                         \
        if (S > 1) H_(LN, ZINC_SCHEME_VANILLA, true);                \
        else H_(LN, ZINC_SCHEME_VANILLA, false);                     \
    }
    ZINC_DISPATCH_LOGN(p.log_n, F)
#undef F
#undef H_
    return hipGetLastError();
}

hipError_t launch_encode(const DevParams& p, const double* slots, uint32_t n_slots, uint32_t batch,
                         uint64_t* pt, hipStream_t s) {
    if (p.log_n == 15) return launch_split_encode(p, slots, n_slots, batch, pt, s);
#define F(LN) hipLaunchKernelGGL(k_encode<LN>, dim3(batch), dim3(Cfg<LN>::G::T), 0, s, p, slots, n_slots, \
                                 (u64*)pt)
    ZINC_DISPATCH_LOGN(p.log_n, F)
#undef F
    return hipGetLastError();
}

hipError_t launch_decrypt(const DevParams& p, const uint64_t* ct, uint32_t batch, uint64_t* pt,
                          hipStream_t s) {
    if (p.log_n == 15) return launch_split_decrypt(p, ct, batch, pt, s);
#define F(LN) hipLaunchKernelGGL(k_decrypt<LN>, dim3(p.L, batch), dim3(Cfg<LN>::G::T), 0, s, p, \
                                 (const u64*)ct, (u64*)pt)
    ZINC_DISPATCH_LOGN(p.log_n, F)
#undef F
    return hipGetLastError();
}

hipError_t launch_decode(const DevParams& p, const uint64_t* pt, uint32_t batch, double* slots,
                         hipStream_t s) {
    if (p.log_n == 15) return launch_split_decode(p, pt, batch, slots, s);
#define F(LN) hipLaunchKernelGGL(k_decode<LN>, dim3(batch), dim3(Cfg<LN>::G::T), 0, s, p, (const u64*)pt, slots)
    ZINC_DISPATCH_LOGN(p.log_n, F)
#undef F
    return hipGetLastError();
}

hipError_t launch_add(const DevParams& p, const uint64_t* a, const uint64_t* b, uint32_t batch,
                      uint64_t* out, hipStream_t s) {
    const size_t words = (size_t)batch * 2 * p.L * p.n;
    const size_t pairs = words / 2;
    size_t blocks = (pairs + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add, dim3((unsigned)blocks), dim3(256), 0, s, p, (const u64*)a, (const u64*)b,
                       (u64*)out, pairs);
    return hipGetLastError();
}

hipError_t launch_ntt(const DevParams& p, bool inverse, uint32_t limb, uint64_t* poly, uint32_t n_polys,
                      hipStream_t s) {
    if (p.log_n == 15) return launch_split_ntt(p, inverse, limb, poly, n_polys, s);
#define F(LN)                                                                                          \
    if (inverse)                                                                                       \
        hipLaunchKernelGGL((k_ntt<LN, true>), dim3(n_polys), dim3(Cfg<LN>::G::T), 0, s, p, limb, (u64*)poly); \
    else                                                                                               \
        hipLaunchKernelGGL((k_ntt<LN, false>), dim3(n_polys), dim3(Cfg<LN>::G::T), 0, s, p, limb, (u64*)poly)
    ZINC_DISPATCH_LOGN(p.log_n, F)
#undef F
    return hipGetLastError();
}

hipError_t launch_sample(const DevParams& p, int kind, uint32_t tag, uint32_t limb, const uint64_t* ct_ids,
                         uint32_t batch, void* out, hipStream_t s) {
    const unsigned gx = (p.n + 255) / 256;
    hipLaunchKernelGGL(k_sample, dim3(gx, batch), dim3(256), 0, s, p, kind, tag, limb, (const u64*)ct_ids, out);
    return hipGetLastError();
}

}  // namespace zinc
