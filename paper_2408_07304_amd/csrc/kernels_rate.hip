// Peak rate of the forward NTT's butterfly on this device: the roofline
// denominator of the fused encryption kernels, which are bound by VALU issue
// (the paper's Theoretical Analysis section puts an encryption's cost in its
// transforms).  Every thread of a full-occupancy grid keeps 16 residues in
// registers and runs rounds of four radix-2 stages over them with the
// kernels' own butterflies -- ct_bfly (64-bit Shoup, with the lazy reduction
// every fourth stage that ntt_fwd schedules) or ct_bfly_fp (exact FP64) --
// with wave-uniform twiddles in scalar registers and no memory traffic, so
// the measured rate is what the arithmetic alone allows.
#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "device.h"

namespace zinc {

namespace {

constexpr int kRateThreads = 256;
constexpr int kRateVals = 16;            // residues per thread
constexpr int kRateStages = 4;           // stages per round
constexpr int kRateBflyPerRound = kRateVals / 2 * kRateStages;

struct RateArgs {
    u64 w[8], wp[8];                     // twiddles and Shoup companions (integer)
    double fw[8], fwq[8];                // twiddles and fl(w / q) (FP64)
    u64 q;
    double qd;
};

template <bool FP>
__global__ void __launch_bounds__(kRateThreads) k_bfly_rate(RateArgs a, uint32_t rounds, u64* sink) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (FP) {
        double v[kRateVals];
#pragma unroll
        for (int c = 0; c < kRateVals; ++c) v[c] = (double)((tid * 2654435761u + 977u * c) % 1000003u);
#pragma unroll 1
        for (uint32_t r = 0; r < rounds; ++r) {
#pragma unroll
            for (int s = 0; s < kRateStages; ++s) {
                const int b = kRateStages - 1 - s;
#pragma unroll
                for (int c = 0; c < kRateVals; ++c) {
                    if (c & (1 << b)) continue;
                    const int k = 2 * s + ((c >> (b + 1)) & 1);
                    ct_bfly_fp(v[c], v[c | (1 << b)], a.fw[k], a.fwq[k], a.qd);
                }
            }
        }
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kRateVals; ++c) acc += v[c];
        sink[tid] = (u64)__double_as_longlong(acc);
    } else {
        const u64 q = a.q, q2 = 2 * q, q8 = q << 3;
        u64 v[kRateVals];
#pragma unroll
        for (int c = 0; c < kRateVals; ++c) v[c] = ((u64)tid * 0x9E3779B97F4A7C15ull + 977ull * c) % q;
        // values stay below 16q: the first stage of each round reduces x from
        // [0, 16q) into [0, 8q) and each stage adds at most 2q
#pragma unroll 1
        for (uint32_t r = 0; r < rounds; ++r) {
#pragma unroll
            for (int s = 0; s < kRateStages; ++s) {
                const int b = kRateStages - 1 - s;
#pragma unroll
                for (int c = 0; c < kRateVals; ++c) {
                    if (c & (1 << b)) continue;
                    const int k = 2 * s + ((c >> (b + 1)) & 1);
                    if (s == 0) ct_bfly<true>(v[c], v[c | (1 << b)], a.w[k], a.wp[k], q, q2, q8);
                    else ct_bfly<false>(v[c], v[c | (1 << b)], a.w[k], a.wp[k], q, q2, q8);
                }
            }
        }
        u64 acc = 0;
#pragma unroll
        for (int c = 0; c < kRateVals; ++c) acc ^= v[c];
        sink[tid] = acc;
    }
}

zinc_status rate_fail(zinc_status code, const std::string& msg) {
    set_error(msg);
    return code;
}

}  // namespace

}  // namespace zinc

using namespace zinc;

extern "C" zinc_status zinc_butterfly_rate(int arith, uint64_t q, uint32_t reps, double* bfly_per_s) {
    if (!bfly_per_s) return rate_fail(ZINC_E_INVAL, "zinc_butterfly_rate: null output");
    *bfly_per_s = 0.0;
    if (arith != 0 && arith != 1) return rate_fail(ZINC_E_INVAL, "zinc_butterfly_rate: arith must be 0 (integer) or 1 (FP64)");
    if (reps < 1 || reps > 1000) return rate_fail(ZINC_E_INVAL, "zinc_butterfly_rate: reps must be in [1, 1000]");
    const uint64_t qmax = arith ? (1ull << 50) : (1ull << 60);
    if ((q & 1) == 0 || q < (1ull << 20) || q >= qmax)
        return rate_fail(ZINC_E_INVAL, "zinc_butterfly_rate: q must be odd, in [2^20, 2^60) (integer) or [2^20, 2^50) (FP64)");
    RateArgs a{};
    for (int k = 0; k < 8; ++k) {
        const uint64_t w = (q / 3 + 104729ull * (uint64_t)(k + 1)) % q;
        a.w[k] = w;
        a.wp[k] = shoup_companion(w, q);
        a.fw[k] = (double)w;
        a.fwq[k] = (double)((long double)w / (long double)q);
    }
    a.q = q;
    a.qd = (double)q;
    const uint32_t grid = (uint32_t)device_cu_count() * 8;     // 32 waves per CU
    const uint32_t rounds = 256;
    const double bfly = (double)grid * kRateThreads * rounds * kRateBflyPerRound;

    u64* sink = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&sink, (size_t)grid * kRateThreads * sizeof(u64));
    if (e != hipSuccess) return rate_fail(ZINC_E_NOMEM, "zinc_butterfly_rate: sink allocation failed");
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto launch = [&]() {
        if (arith) hipLaunchKernelGGL(k_bfly_rate<true>, dim3(grid), dim3(kRateThreads), 0, s, a, rounds, sink);
        else hipLaunchKernelGGL(k_bfly_rate<false>, dim3(grid), dim3(kRateThreads), 0, s, a, rounds, sink);
        return hipGetLastError();
    };
    // untimed launches for 200 ms first, so that the timed ones see the
    // clocks a sustained workload runs at
    const auto t0 = std::chrono::steady_clock::now();
    while (e == hipSuccess && std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(200)) {
        for (int i = 0; i < 8 && e == hipSuccess; ++i) e = launch();
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    std::vector<float> ms;
    for (uint32_t r = 0; r < reps && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        ms.push_back(t);
    }
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(sink);
    if (e != hipSuccess) return rate_fail(ZINC_E_HIP, std::string("zinc_butterfly_rate: ") + hipGetErrorString(e));
    std::sort(ms.begin(), ms.end());
    const double med = ms[ms.size() / 2];
    if (!(med > 0.0)) return rate_fail(ZINC_E_HIP, "zinc_butterfly_rate: zero launch time");
    *bfly_per_s = bfly / (med * 1e-3);
    return ZINC_OK;
}
