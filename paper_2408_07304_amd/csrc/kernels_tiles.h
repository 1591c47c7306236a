// Alternative forms of the fused encode + encrypt kernel, chosen per context by
// zinc_autotune: 8 or 32 coefficients per thread instead of 16, and stores
// straight from the last pass's registers instead of through LDS in natural
// order.  Fewer coefficients per thread give more waves per CU (latency
// hiding) at the cost of one more LDS exchange pass; more give one pass fewer
// at lower occupancy.  Results are bit-identical for every form.
#pragma once
#include "kernels_common.h"

namespace zinc {

namespace {  // each including translation unit has its own copy

// WPE: waves per SIMD that the register budget must allow (the LDS buffer of
// one ciphertext already bounds the workgroups per CU).
// SPLIT: as for k_encrypt, the workgroups along y share a ciphertext's limbs.
template <class G, int SCHEME, int WPE, bool REG, bool SPLIT>
__global__ void __launch_bounds__(G::T) __attribute__((amdgpu_waves_per_eu(WPE)))
k_encrypt_tile(typename ParamArg<G::LOGN>::type pa, EncArgs a) {
    const DevParams& p = deref(pa);
    constexpr int N = G::N;
    __shared__ u64 lds[LdsWords<N>::value];
    __shared__ u64 tab[kCdtTab];
    const uint32_t t = threadIdx.x;
    const uint32_t b = blockIdx.x;
    const u64 id = a.ct_ids[b];
    if (reserved_id(p, a, id, t)) return;
    load_cdt(tab, p.cdt, t);
    encrypt_item_g<G, SCHEME, true, REG>(p, a.slots + (size_t)b * a.n_slots, a.n_slots, nullptr, id,
                                         a.ct + (size_t)b * 2 * p.L * N, lds, tab, t,
                                         SPLIT ? limb_group_start(p.L, blockIdx.y) : 0u,
                                         SPLIT ? limb_group_start(p.L, blockIdx.y + 1) : ~0u);
}

template <class G, int SCHEME, int WPE, bool REG>
hipError_t launch_tile(const DevParams& p, const EncArgs& a, uint32_t batch, hipStream_t s) {
    const uint32_t S = limb_groups(p, batch);
    if (S > 1)
        hipLaunchKernelGGL((k_encrypt_tile<G, SCHEME, WPE, REG, true>), dim3(batch, S), dim3(G::T), 0, s,
                           ParamArg<G::LOGN>::of(p), a);
    else
        hipLaunchKernelGGL((k_encrypt_tile<G, SCHEME, WPE, REG, false>), dim3(batch), dim3(G::T), 0, s,
                           ParamArg<G::LOGN>::of(p), a);
    return hipGetLastError();
}

// tile: kTileR8, kTileR16 or kTileR32; reg: register epilogue.  The default
// form (16 per thread, natural-order stores) is k_encrypt.
template <int SCHEME>
hipError_t launch_tile_scheme(const DevParams& p, int tile, bool reg, const EncArgs& a, uint32_t batch,
                              hipStream_t s) {
    switch ((p.log_n * 4 + tile) * 2 + (reg ? 1 : 0)) {
        case (12 * 4 + kTileR8) * 2: return launch_tile<Geom<12, 9>, SCHEME, 8, false>(p, a, batch, s);
        case (12 * 4 + kTileR8) * 2 + 1: return launch_tile<Geom<12, 9>, SCHEME, 8, true>(p, a, batch, s);
        case (12 * 4 + kTileR16) * 2 + 1: return launch_tile<Geom<12, 8>, SCHEME, 4, true>(p, a, batch, s);
        case (12 * 4 + kTileR32) * 2: return launch_tile<Geom<12, 7>, SCHEME, 2, false>(p, a, batch, s);
        case (13 * 4 + kTileR8) * 2: return launch_tile<Geom<13, 10>, SCHEME, 8, false>(p, a, batch, s);
        case (13 * 4 + kTileR8) * 2 + 1: return launch_tile<Geom<13, 10>, SCHEME, 8, true>(p, a, batch, s);
        case (13 * 4 + kTileR16) * 2 + 1: return launch_tile<Geom<13, 9>, SCHEME, 4, true>(p, a, batch, s);
        case (13 * 4 + kTileR32) * 2: return launch_tile<Geom<13, 8>, SCHEME, 2, false>(p, a, batch, s);
        case (14 * 4 + kTileR16) * 2 + 1: return launch_tile<Geom<14, 10>, SCHEME, 4, true>(p, a, batch, s);
        case (14 * 4 + kTileR32) * 2: return launch_tile<Geom<14, 9>, SCHEME, 2, false>(p, a, batch, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

}  // namespace zinc
