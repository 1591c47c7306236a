// Batch (slot) encoding of BFV and BGV plaintexts (the schemes of the Scheme
// Flexibility section take their encodings from their own papers).  For a
// prime t = 1 (mod 2N), Z_t[X]/(X^N + 1) is N copies of Z_t, one per odd
// power of a primitive 2N-th root zeta: slot j holds m(zeta^(e_j)), with
// e_i = 3^i and e_(N/2 + i) = -3^i (mod 2N) for i < N/2.
//
// The forward negacyclic transform below gives entry k = m(zeta^(2 brv(k)+1)),
// so slot j sits at entry pos[j] = brv((e_j - 1)/2) (a host table).  Encoding
// scatters the slots to those entries and runs the inverse transform; decoding
// runs the forward transform and gathers.  t < 2^31, so every residue is a
// 32-bit word and products use 32-bit Shoup arithmetic.  One workgroup per
// plaintext holds its N words in LDS (128 KiB at N = 32768); every input word
// is read before the first barrier and outputs are written after the last, so
// input and output may be the same buffer.
#include "device.h"

namespace zinc {

namespace {

constexpr int kBatchThreads = 1024;

// y w mod t for y < 2^32, w < t, ws = floor(w 2^32 / t): the estimate
// floor(y ws / 2^32) is the quotient or one below it, so y w - q t is in [0, 2t).
__device__ __forceinline__ uint32_t mul_t(uint32_t y, uint32_t w, uint32_t ws, uint32_t t) {
    const uint32_t r = y * w - __umulhi(y, ws) * t;
    return r >= t ? r - t : r;
}
__device__ __forceinline__ uint32_t add_t(uint32_t a, uint32_t b, uint32_t t) {   // a, b < t < 2^31
    const uint32_t r = a + b;
    return r >= t ? r - t : r;
}
__device__ __forceinline__ uint32_t sub_t(uint32_t a, uint32_t b, uint32_t t) {
    return a >= b ? a - b : a + (t - b);
}
__device__ __forceinline__ uint32_t mod_t(long long x, uint32_t t) {
    const long long r = x % (long long)t;
    return (uint32_t)(r < 0 ? r + (long long)t : r);
}

// Cooley-Tukey, natural order in, entry k = a(zeta^(2 brv(k)+1)) out; stage
// with m blocks uses tw[m + i] = zeta^brv(m + i) for block i.
template <uint32_t N>
__device__ __forceinline__ void fwd_t(uint32_t* a, const BatchArgs& g, uint32_t tid) {
    const uint32_t t = g.t;
    for (uint32_t m = 1, gap = N / 2, sh = __builtin_ctz(N / 2); m < N; m <<= 1, gap >>= 1, --sh) {
        for (uint32_t b = tid; b < N / 2; b += kBatchThreads) {
            const uint32_t i = b >> sh, j = 2 * i * gap + (b & (gap - 1));
            const uint32_t w = g.tw[2 * (m + i)], ws = g.tw[2 * (m + i) + 1];
            const uint32_t x = a[j], y = mul_t(a[j + gap], w, ws, t);
            a[j] = add_t(x, y, t);
            a[j + gap] = sub_t(x, y, t);
        }
        __syncthreads();
    }
}

// Gentleman-Sande with itw[m + i] = zeta^-brv(m + i), stages in reverse:
// undoes fwd_t up to the factor N, which the caller removes.
template <uint32_t N>
__device__ __forceinline__ void inv_t(uint32_t* a, const BatchArgs& g, uint32_t tid) {
    const uint32_t t = g.t;
    for (uint32_t m = N / 2, gap = 1, sh = 0; m >= 1; m >>= 1, gap <<= 1, ++sh) {
        for (uint32_t b = tid; b < N / 2; b += kBatchThreads) {
            const uint32_t i = b >> sh, j = 2 * i * gap + (b & (gap - 1));
            const uint32_t w = g.itw[2 * (m + i)], ws = g.itw[2 * (m + i) + 1];
            const uint32_t x = a[j], y = a[j + gap];
            a[j] = add_t(x, y, t);
            a[j + gap] = mul_t(sub_t(x, y, t), w, ws, t);
        }
        __syncthreads();
    }
}

template <int LOGN>
__global__ void __launch_bounds__(kBatchThreads) k_batch_encode(BatchArgs g, const long long* slots, long long* m) {
    constexpr uint32_t N = 1u << LOGN;
    __shared__ uint32_t a[N];
    const uint32_t tid = threadIdx.x;
    const size_t base = (size_t)blockIdx.x * N;
    for (uint32_t j = tid; j < N; j += kBatchThreads) a[g.pos[j]] = mod_t(slots[base + j], g.t);
    __syncthreads();
    inv_t<N>(a, g, tid);
    for (uint32_t i = tid; i < N; i += kBatchThreads) m[base + i] = (long long)mul_t(a[i], g.ninv, g.ninv_sh, g.t);
}

template <int LOGN>
__global__ void __launch_bounds__(kBatchThreads) k_batch_decode(BatchArgs g, const long long* m, long long* slots) {
    constexpr uint32_t N = 1u << LOGN;
    __shared__ uint32_t a[N];
    const uint32_t tid = threadIdx.x, t = g.t;
    const size_t base = (size_t)blockIdx.x * N;
    for (uint32_t i = tid; i < N; i += kBatchThreads) a[i] = mod_t(m[base + i], t);
    __syncthreads();
    fwd_t<N>(a, g, tid);
    for (uint32_t j = tid; j < N; j += kBatchThreads) {
        const uint32_t r = a[g.pos[j]];
        slots[base + j] = r > t / 2 ? (long long)r - (long long)t : (long long)r;
    }
}

}  // namespace

hipError_t launch_batch_codec(const BatchArgs& g, uint32_t log_n, bool decode, const int64_t* in, uint32_t batch,
                              int64_t* out, hipStream_t s) {
    const long long* x = (const long long*)in;
    long long* y = (long long*)out;
#define F(LN)                                                                                      \
    case LN:                                                                                       \
        if (decode)                                                                                \
            hipLaunchKernelGGL(k_batch_decode<LN>, dim3(batch), dim3(kBatchThreads), 0, s, g, x, y); \
        else                                                                                       \
            hipLaunchKernelGGL(k_batch_encode<LN>, dim3(batch), dim3(kBatchThreads), 0, s, g, x, y); \
        break;
    switch (log_n) {
        F(12)
        F(13)
        F(14)
        F(15)
        default: return hipErrorInvalidValue;
    }
#undef F
    return hipGetLastError();
}

}  // namespace zinc
