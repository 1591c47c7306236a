// BFV on the same contexts (Scheme Flexibility section, Eq. 12): integer
// plaintexts m in Z_t (one coefficient per slot of the ring, no batching)
// scaled by Delta = floor(Q / t), Q the product of the data moduli.  The
// ciphertexts are those of zinc_encrypt / zinc_encrypt_vanilla applied to the
// scaled plaintext, so Zinc needs no change for BFV.
//
// Decoding follows the RNS scale-and-round of Halevi, Polyakov and Shoup
// (CT-RSA 2019): with x = sum_l c_l Qt_l (Q/q_l) mod Q, Qt_l = (Q/q_l)^-1 mod
// q_l, t x / Q = sum_l c_l t Qt_l / q_l - t k for an integer k.  Writing
// t Qt_l = w_l q_l + b_l (w_l, b_l integers, b_l < q_l), each term
// c_l (w_l + b_l / q_l) has the integer part c_l w_l + floor(c_l b_l / q_l)
// (taken mod t) and the exact fraction ((c_l b_l) mod q_l) / q_l, which is
// summed in FP64.  m = round(t x / Q) mod t, centred to (-t/2, t/2].
//
// BGV (Eq. 13) encodes m as m mod t itself (the BFV encoder with Delta = 1)
// and decodes the centred value of x mod Q, reduced mod t: with
// y_l = c_l Qt_l mod q_l, x = sum_l y_l (Q/q_l) - k Q, and the centred lift
// takes k = round(sum_l y_l / q_l) (an FP64 sum; its rounding error, about
// L 2^-53, matters only for |x| within that fraction of Q/2, far outside any
// decryptable noise).  Then x mod t = sum_l (y_l mod t)((Q/q_l) mod t)
// - k (Q mod t), all mod t.
#include "device.h"

namespace zinc {

namespace {

__global__ void __launch_bounds__(256) k_bfv_encode(DevParams p, BfvConsts k, const long long* m, uint32_t batch,
                                                    u64* pt) {
    const uint32_t n = p.n, L = p.L;
    const size_t total = (size_t)batch * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const size_t b = i / n, c = i % n;
        long long x = m[i] % (long long)k.t;           // the representative in [0, t), below every q_l
        if (x < 0) x += (long long)k.t;
        for (uint32_t l = 0; l < L; ++l) {
            const LimbConst lc = p.limbs[l];
            pt[(b * L + l) * n + c] = csub(shoup_lazy((u64)x, k.delta[l], k.delta_sh[l], lc.q), lc.q);
        }
    }
}

__global__ void __launch_bounds__(256) k_bfv_decode(DevParams p, BfvConsts k, const u64* pt, uint32_t batch,
                                                    long long* m) {
    const uint32_t n = p.n, L = p.L;
    const u64 t = k.t;
    const size_t total = (size_t)batch * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const size_t b = i / n, c = i % n;
        u64 whole = 0;           // integer part, mod t
        double frac = 0.0;       // sum of the exact fractions, in [0, L)
        for (uint32_t l = 0; l < L; ++l) {
            const LimbConst lc = p.limbs[l];
            const u64 x = pt[(b * L + l) * n + c];
            // x b_l = quo q_l + rem with rem in [0, q_l): Shoup quotient, corrected once
            u64 quo = __umul64hi(x, k.b_sh[l]);
            u64 rem = x * k.b[l] - quo * lc.q;
            if (rem >= lc.q) {
                rem -= lc.q;
                ++quo;
            }
            whole = (whole + (x % t) * k.w_mod_t[l] % t + quo % t) % t;
            frac += (double)rem / (double)lc.q;
        }
        const u64 r = (whole + (u64)__builtin_rint(frac)) % t;
        m[i] = r > t / 2 ? (long long)r - (long long)t : (long long)r;
    }
}

__global__ void __launch_bounds__(256) k_bgv_decode(DevParams p, BgvConsts k, const u64* pt, uint32_t batch,
                                                    long long* m) {
    const uint32_t n = p.n, L = p.L;
    const u64 t = k.t;
    const size_t total = (size_t)batch * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const size_t b = i / n, c = i % n;
        u64 acc = 0;            // sum of (y_l mod t)((Q/q_l) mod t), each term reduced mod t
        double frac = 0.0;      // sum of y_l / q_l, in [0, L)
        for (uint32_t l = 0; l < L; ++l) {
            const LimbConst lc = p.limbs[l];
            const u64 y = csub(shoup_lazy(pt[(b * L + l) * n + c], k.qt[l], k.qt_sh[l], lc.q), lc.q);
            acc += (y % t) * k.qhat_mod_t[l] % t;
            frac += (double)y / (double)lc.q;
        }
        const u64 kq = (u64)__builtin_rint(frac) * k.q_mod_t % t;     // k <= L, k (Q mod t) < 2^37
        const u64 r = (acc % t + t - kq) % t;
        m[i] = r > t / 2 ? (long long)r - (long long)t : (long long)r;
    }
}

uint32_t blocks_for(size_t total) {
    const size_t b = (total + 255) / 256;
    return (uint32_t)(b < 65535 * 16 ? b : 65535 * 16);
}

}  // namespace

hipError_t launch_bfv_encode(const DevParams& p, const BfvConsts& k, const int64_t* m, uint32_t batch, uint64_t* pt,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_bfv_encode, dim3(blocks_for((size_t)batch * p.n)), dim3(256), 0, s, p, k,
                       (const long long*)m, batch, (u64*)pt);
    return hipGetLastError();
}

hipError_t launch_bfv_decode(const DevParams& p, const BfvConsts& k, const uint64_t* pt, uint32_t batch, int64_t* m,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_bfv_decode, dim3(blocks_for((size_t)batch * p.n)), dim3(256), 0, s, p, k, (const u64*)pt,
                       batch, (long long*)m);
    return hipGetLastError();
}

hipError_t launch_bgv_decode(const DevParams& p, const BgvConsts& k, const uint64_t* pt, uint32_t batch, int64_t* m,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_bgv_decode, dim3(blocks_for((size_t)batch * p.n)), dim3(256), 0, s, p, k, (const u64*)pt,
                       batch, (long long*)m);
    return hipGetLastError();
}

}  // namespace zinc
