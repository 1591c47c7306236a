// The element-wise steps of encryption as streaming kernels of their own, for
// callers that compute the transforms separately: Zinc's additions of the
// cached Enc(0) (Algorithm 1, in the NTT domain) and vanilla's pk * u_hat
// products and additions (Eq. 8).  Both are bound by HBM bandwidth: every
// word is read and written once, with 16-byte accesses; the cached zero and the
// public key are shared by the whole batch and stay in L2.
#include "device.h"

namespace zinc {

namespace {

constexpr int kEwThreads = 256;
constexpr int kEwPairs = 2;          // 16-byte pairs per thread per row chunk

// The transform outputs and the ciphertexts are streamed once: non-temporal
// loads and stores (measured 3-6 % faster than cached ones); the shared
// Enc(0) and public key use ordinary loads so that they stay in L2.
__device__ __forceinline__ u64x2 ld2(const u64* p) { return load_pair(p); }
__device__ __forceinline__ u64x2 ld2_stream(const u64* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const u64x2*>(p));
}
__device__ __forceinline__ void st2(u64* p, u64x2 v) { __builtin_nontemporal_store(v, reinterpret_cast<u64x2*>(p)); }

// rows = batch * 2L polynomials of N words; row r is component (r / L) % 2 of
// limb r % L of ciphertext r / 2L.  Grid: x covers one row in chunks of
// kEwThreads * kEwPairs pairs, y strides over rows.
// Each thread reads its words before writing the same words, so ct may alias
// hat.
__global__ void __launch_bounds__(kEwThreads) k_ew_zinc(DevParams p, const u64* hat, uint32_t rows, u64* ct) {
    const uint32_t n = p.n, L = p.L;
    const uint32_t base = blockIdx.x * (kEwThreads * kEwPairs * 2) + threadIdx.x * 2;
    for (uint32_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const uint32_t l = r % L, j = (r / L) % 2;
        const u64 q = p.limbs[l].q;
        const u64* z = p.zero + ((size_t)j * L + l) * n;
        const u64* h = hat + (size_t)r * n;
        u64* o = ct + (size_t)r * n;
        u64x2 hv[kEwPairs], zv[kEwPairs];
#pragma unroll
        for (int i = 0; i < kEwPairs; ++i) {
            const uint32_t k = base + i * kEwThreads * 2;
            hv[i] = ld2_stream(h + k);
            zv[i] = ld2(z + k);
        }
#pragma unroll
        for (int i = 0; i < kEwPairs; ++i) {
            const uint32_t k = base + i * kEwThreads * 2;
            st2(o + k, u64x2{addmod(hv[i].x, zv[i].x, q), addmod(hv[i].y, zv[i].y, q)});
        }
    }
}

// rows = batch * L (ciphertext r / L, limb r % L): reads u_hat and both hat
// components of the limb, writes both components.
__global__ void __launch_bounds__(kEwThreads) k_ew_vanilla(DevParams p, const u64* uhat, const u64* hat,
                                                           uint32_t rows, u64* ct) {
    const uint32_t n = p.n, L = p.L, M = p.M;
    const uint32_t base = blockIdx.x * (kEwThreads * kEwPairs * 2) + threadIdx.x * 2;
    for (uint32_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const uint32_t b = r / L, l = r % L;
        const u64 q = p.limbs[l].q;
        const u64* u = uhat + (size_t)r * n;
        const size_t o1 = ((size_t)b * 2 * L + l) * n, o2 = o1 + (size_t)L * n;
        const u64 *pk1 = p.pk + (size_t)l * n, *pk1s = p.pk_sh + (size_t)l * n;
        const u64 *pk2 = p.pk + (size_t)(M + l) * n, *pk2s = p.pk_sh + (size_t)(M + l) * n;
#pragma unroll
        for (int i = 0; i < kEwPairs; ++i) {
            const uint32_t k = base + i * kEwThreads * 2;
            const u64x2 uv = ld2_stream(u + k), h1 = ld2_stream(hat + o1 + k), h2 = ld2_stream(hat + o2 + k);
            const u64x2 a1 = ld2(pk1 + k), s1 = ld2(pk1s + k), a2 = ld2(pk2 + k), s2 = ld2(pk2s + k);
            st2(ct + o1 + k, u64x2{addmod(csub(shoup_lazy(uv.x, a1.x, s1.x, q), q), h1.x, q),
                                     addmod(csub(shoup_lazy(uv.y, a1.y, s1.y, q), q), h1.y, q)});
            st2(ct + o2 + k, u64x2{addmod(csub(shoup_lazy(uv.x, a2.x, s2.x, q), q), h2.x, q),
                                     addmod(csub(shoup_lazy(uv.y, a2.y, s2.y, q), q), h2.y, q)});
        }
    }
}

dim3 ew_grid(uint32_t n, uint32_t rows) {
    const uint32_t per_block = kEwThreads * kEwPairs * 2;   // words
    return dim3(n / per_block, rows < 65535u ? rows : 65535u);
}

}  // namespace

hipError_t launch_elementwise_zinc(const DevParams& p, const uint64_t* hat, uint32_t batch, uint64_t* ct,
                                   hipStream_t s) {
    const uint32_t rows = batch * 2 * p.L;
    hipLaunchKernelGGL(k_ew_zinc, ew_grid(p.n, rows), dim3(kEwThreads), 0, s, p, (const u64*)hat, rows, (u64*)ct);
    return hipGetLastError();
}

hipError_t launch_elementwise_vanilla(const DevParams& p, const uint64_t* uhat, const uint64_t* hat, uint32_t batch,
                                      uint64_t* ct, hipStream_t s) {
    const uint32_t rows = batch * p.L;
    hipLaunchKernelGGL(k_ew_vanilla, ew_grid(p.n, rows), dim3(kEwThreads), 0, s, p, (const u64*)uhat,
                       (const u64*)hat, rows, (u64*)ct);
    return hipGetLastError();
}

}  // namespace zinc
