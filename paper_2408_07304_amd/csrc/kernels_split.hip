// Kernels for ring degree N = 32768.  A polynomial of 32768 uint64 words does
// not fit the 160 KiB LDS of a CU, so every transform is split: its first
// stage pairs coefficients j and j + N/2, which one thread holds in registers,
// and after it the two halves are independent 16384-point transforms run one
// after the other through the same LDS exchange buffer (twiddle index base
// (2 + h) 2^s for half h, see tw_index).  The inverse runs the two half
// transforms first and the pairing stage last.  CKKS encoding uses the
// real-input FFT identity so that its N/4-point complex FFT fits LDS;
// decoding combines two N/4-point FFTs in the last radix-2 stage.
#include "split_common.h"

namespace zinc {

using namespace split;

template <int SCHEME, bool FROM_SLOTS, bool BGV = false>
__global__ void __launch_bounds__(TS) __attribute__((amdgpu_waves_per_eu(4)))
k_encrypt_split(const DevParams* __restrict__ pp, EncArgs a) {
    const DevParams& p = *pp;   // see ParamArg
    __shared__ u64 lds[LdsWords<NH>::value];
    __shared__ u64 tab[kCdtTab];
    const uint32_t t = threadIdx.x, b = blockIdx.x;
    const u64 id = a.ct_ids[b];
    if (reserved_id(p, a, id, t)) return;
    load_cdt(tab, p.cdt, t);
    const uint32_t L = p.L;
    encrypt_item_split<SCHEME, FROM_SLOTS, BGV>(p, a.slots + (size_t)b * a.n_slots, a.n_slots, a.pt + (size_t)b * L * NF,
                                           id, a.ct + (size_t)b * 2 * L * NF, lds, tab, t);
}

// ---------------------------------------------------------------------------
// key generation, N = 32768 (integer arithmetic), one workgroup per modulus;
// under BGV the key error is t e (Eq. 13)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(TS) k_keygen_split(const DevParams* __restrict__ pp, u64* sk, u64* sk_sh, u64* pk, u64* pk_sh) {
    const DevParams& p = *pp;   // see ParamArg
    __shared__ u64 lds[LdsWords<NH>::value];
    __shared__ u64 tab[kCdtTab];
    const uint32_t t = threadIdx.x, l = blockIdx.x;
    load_cdt(tab, p.cdt, t);
    LimbConst lc = p.limbs[l];
    lc.fp = 0;
    const SplitLimb sl(p, lc, l, lds, t);
    const uint32_t M = p.M;
    const u64 et = p.noise_t > 1 ? p.noise_t : 0;
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
        auto err = [&](int x) { return et ? reduce_signed((long long)x * (long long)et, lc) : small_mod(x, lc.q); };
        sl.run_half(h, [&](int c) { return sl.stage0(err(eh_.lo.get(c)), err(eh_.hi.get(c)), h); });
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

__global__ void __launch_bounds__(TS) k_decrypt_split(const DevParams* __restrict__ pp, const u64* ct, u64* pt) {
    const DevParams& p = *pp;   // see ParamArg
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
__global__ void __launch_bounds__(TS) k_ntt_split(const DevParams* __restrict__ pp, uint32_t limb, u64* poly) {
    const DevParams& p = *pp;   // see ParamArg
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

__global__ void __launch_bounds__(TS) k_encode_split(const DevParams* __restrict__ pp, const double* slots, uint32_t n_slots, u64* pt) {
    const DevParams& p = *pp;   // see ParamArg
    __shared__ u64 lds[LdsWords<NH>::value];
    const uint32_t t = threadIdx.x, b = blockIdx.x;
    long long mlo[RS], mhi[RS];
    // n_slots is the same in every workgroup: no barrier is skipped by some threads only
    if (n_slots <= kSparseSlots) encode_sparse_split(mlo, mhi, p, slots + (size_t)b * n_slots, n_slots, t);
    else encode_split(mlo, mhi, lds, p, slots + (size_t)b * n_slots, n_slots, t);
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
__global__ void __launch_bounds__(TS) k_decode_split(const DevParams* __restrict__ pp, const u64* pt, double* slots) {
    const DevParams& p = *pp;   // see ParamArg
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
    hipLaunchKernelGGL(k_keygen_split, dim3(p.M), dim3(TS), 0, s, p.self, (u64*)sk, (u64*)sk_sh, (u64*)pk, (u64*)pk_sh);
    return hipGetLastError();
}

hipError_t launch_split_encrypt(const DevParams& p, int scheme, bool from_slots, const double* slots,
                                uint32_t n_slots, const uint64_t* pt, uint32_t batch, const uint64_t* ct_ids,
                                uint64_t* ct, hipStream_t s, bool reserved_ok) {
    EncArgs a{slots, n_slots, (const u64*)pt, (const u64*)ct_ids, (u64*)ct, reserved_ok ? 1u : 0u};
    if (p.noise_t > 1) {            // BGV: integer plaintexts only
        if (from_slots) return hipErrorInvalidValue;
        if (scheme == ZINC_SCHEME_ZINC)
            hipLaunchKernelGGL((k_encrypt_split<ZINC_SCHEME_ZINC, false, true>), dim3(batch), dim3(TS), 0, s, p.self, a);
        else hipLaunchKernelGGL((k_encrypt_split<ZINC_SCHEME_VANILLA, false, true>), dim3(batch), dim3(TS), 0, s, p.self, a);
    } else if (scheme == ZINC_SCHEME_ZINC) {
        if (from_slots) hipLaunchKernelGGL((k_encrypt_split<ZINC_SCHEME_ZINC, true>), dim3(batch), dim3(TS), 0, s, p.self, a);
        else hipLaunchKernelGGL((k_encrypt_split<ZINC_SCHEME_ZINC, false>), dim3(batch), dim3(TS), 0, s, p.self, a);
    } else {
        if (from_slots) hipLaunchKernelGGL((k_encrypt_split<ZINC_SCHEME_VANILLA, true>), dim3(batch), dim3(TS), 0, s, p.self, a);
        else hipLaunchKernelGGL((k_encrypt_split<ZINC_SCHEME_VANILLA, false>), dim3(batch), dim3(TS), 0, s, p.self, a);
    }
    return hipGetLastError();
}

hipError_t launch_split_encode(const DevParams& p, const double* slots, uint32_t n_slots, uint32_t batch,
                               uint64_t* pt, hipStream_t s) {
    hipLaunchKernelGGL(k_encode_split, dim3(batch), dim3(TS), 0, s, p.self, slots, n_slots, (u64*)pt);
    return hipGetLastError();
}

hipError_t launch_split_decrypt(const DevParams& p, const uint64_t* ct, uint32_t batch, uint64_t* pt,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_decrypt_split, dim3(p.L, batch), dim3(TS), 0, s, p.self, (const u64*)ct, (u64*)pt);
    return hipGetLastError();
}

hipError_t launch_split_decode(const DevParams& p, const uint64_t* pt, uint32_t batch, double* slots,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_decode_split, dim3(batch), dim3(TS), 0, s, p.self, (const u64*)pt, slots);
    return hipGetLastError();
}

hipError_t launch_split_ntt(const DevParams& p, bool inverse, uint32_t limb, uint64_t* poly, uint32_t n_polys,
                            hipStream_t s) {
    if (inverse) hipLaunchKernelGGL((k_ntt_split<true>), dim3(n_polys), dim3(TS), 0, s, p.self, limb, (u64*)poly);
    else hipLaunchKernelGGL((k_ntt_split<false>), dim3(n_polys), dim3(TS), 0, s, p.self, limb, (u64*)poly);
    return hipGetLastError();
}

}  // namespace zinc
