// Persistent kernel of a mixed-shape plan: every workgroup (1024 threads, one
// per CU) repeatedly takes the next unit of work from a device counter and
// encrypts it.  A unit is 4, 2, 1 or 1 ciphertexts of one context of ring
// degree 4096, 8192, 16384 or 32768: the 1024 threads split into that many
// groups of N/16 threads which run the same code in lockstep (their barriers
// coincide), each group with its own slice of the 136 KiB LDS buffer.  A
// ring-degree-32768 unit may cover a group of the ciphertext's limbs only.
// Units are ordered by decreasing cost, so the largest ones start first.
#pragma once
#include "split_common.h"

namespace zinc {

namespace {  // each including translation unit has its own copy

constexpr int kPlanThreads = 1024;
constexpr int kPlanLds = LdsWords<16384>::value;     // = 4 x LdsWords<4096> = 2 x LdsWords<8192>
static_assert(4 * LdsWords<4096>::value == kPlanLds && 2 * LdsWords<8192>::value == kPlanLds, "LDS slices");

template <int LOGN, int SCHEME>
__device__ __forceinline__ void run_group(const DevParams& p, const PlanItem* __restrict__ items, const PlanUnit& un,
                                          const double* slots, u64* ct, u64* dummy, u64* lds, const u64* tab,
                                          uint32_t t) {
    constexpr int T = 1 << (LOGN - 4), N = 1 << LOGN;
    // groups are whole wavefronts, so the group index is wave-uniform
    const uint32_t g = (uint32_t)__builtin_amdgcn_readfirstlane((int)(t / T)), tt = t % T;
    const PlanItem it = items[un.first + g];
    u64* out = (it.dummy ? dummy : ct) + it.ct_off;
    encrypt_item<LOGN, SCHEME, true>(p, slots + it.slot_off, N / 2, nullptr, it.ct_id, out,
                                     lds + (size_t)g * LdsWords<N>::value, tab, tt);
}

template <int SCHEME>
__global__ void __launch_bounds__(kPlanThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_plan(const DevParams* __restrict__ ctxs, const PlanItem* __restrict__ items, const PlanUnit* __restrict__ units,
       uint32_t n_units, uint32_t* counter, const double* __restrict__ slots, u64* ct, u64* dummy) {
    __shared__ u64 lds[kPlanLds];
    __shared__ u64 tab[kCdtTab];
    __shared__ uint32_t s_unit;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_unit = atomicAdd(counter, 1u);
        __syncthreads();
        // the same value in every lane: taken from the first lane so that the
        // unit and its context are read with scalar loads into scalar registers
        const uint32_t ui = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_unit);
        if (ui >= n_units) break;                     // every wave of the workgroup leaves here
        const PlanUnit un = units[ui];
        const DevParams& p = ctxs[un.ctx];   // fields read on demand (scalar loads)
        // The thread index as a value the compiler cannot see through, taken
        // afresh in every iteration: otherwise every address derived from it
        // alone is hoisted out of the work loop and held in registers across
        // all four ring degrees' code (hundreds of spilled registers).
        const uint32_t t = opaque_tid(threadIdx.x);
        load_cdt(tab, p.cdt, t);
        switch (un.log_n) {
            case 12: run_group<12, SCHEME>(p, items, un, slots, ct, dummy, lds, tab, t); break;
            case 13: run_group<13, SCHEME>(p, items, un, slots, ct, dummy, lds, tab, t); break;
            case 14: run_group<14, SCHEME>(p, items, un, slots, ct, dummy, lds, tab, t); break;
            default: {
                const PlanItem it = items[un.first];
                u64* out = (it.dummy ? dummy : ct) + it.ct_off;
                encrypt_item_split<SCHEME, true>(p, slots + it.slot_off, 32768 / 2, nullptr, it.ct_id, out, lds,
                                                 tab, t, un.l0, un.l1);
            }
        }
    }
}

__global__ void k_reset_counter(uint32_t* counter) { *counter = 0u; }

// Reset the work counter and run the persistent kernel of one scheme.
template <int SCHEME>
hipError_t launch_plan_scheme(const PlanDev& d, const double* slots, uint64_t* ct, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, d.counter);
    hipLaunchKernelGGL(k_plan<SCHEME>, dim3(d.grid), dim3(kPlanThreads), 0, s, d.ctxs, d.items, d.units, d.n_units,
                       d.counter, slots, (u64*)ct, (u64*)d.dummy);
    return hipGetLastError();
}

}  // namespace

}  // namespace zinc
