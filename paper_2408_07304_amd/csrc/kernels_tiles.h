// Alternative thread geometries of the fused encode + encrypt kernel, chosen
// per context by zinc_autotune: 8 or 32 coefficients per thread instead of 16.
// Fewer coefficients per thread give more waves per CU (latency hiding) at the
// cost of one more LDS exchange pass; more give one pass fewer and fewer
// barriers at lower occupancy.  Results are bit-identical for every geometry.
#pragma once
#include "kernels_common.h"

namespace zinc {

namespace {  // each including translation unit has its own copy

// WPE: waves per SIMD that the register budget must allow (the LDS buffer of
// one ciphertext already bounds the workgroups per CU).
template <class G, int SCHEME, int WPE>
__global__ void __launch_bounds__(G::T) __attribute__((amdgpu_waves_per_eu(WPE)))
k_encrypt_tile(DevParams p, EncArgs a) {
    constexpr int N = G::N;
    __shared__ u64 lds[LdsWords<N>::value];
    __shared__ u64 tab[kCdtPad];
    const uint32_t t = threadIdx.x;
    const uint32_t b = blockIdx.x;
    load_cdt(tab, p.cdt, t);
    encrypt_item_g<G, SCHEME, true>(p, a.slots + (size_t)b * a.n_slots, a.n_slots, nullptr, a.ct_ids[b],
                                    a.ct + (size_t)b * 2 * p.L * N, lds, tab, t);
}

template <class G, int SCHEME, int WPE>
hipError_t launch_tile(const DevParams& p, const EncArgs& a, uint32_t batch, hipStream_t s) {
    hipLaunchKernelGGL((k_encrypt_tile<G, SCHEME, WPE>), dim3(batch), dim3(G::T), 0, s, p, a);
    return hipGetLastError();
}

// tile: kTileR8 or kTileR32
template <int SCHEME>
hipError_t launch_tile_scheme(const DevParams& p, int tile, const EncArgs& a, uint32_t batch, hipStream_t s) {
    switch (p.log_n * 4 + tile) {
        case 12 * 4 + kTileR8: return launch_tile<Geom<12, 9>, SCHEME, 8>(p, a, batch, s);
        case 12 * 4 + kTileR32: return launch_tile<Geom<12, 7>, SCHEME, 2>(p, a, batch, s);
        case 13 * 4 + kTileR8: return launch_tile<Geom<13, 10>, SCHEME, 8>(p, a, batch, s);
        case 13 * 4 + kTileR32: return launch_tile<Geom<13, 8>, SCHEME, 2>(p, a, batch, s);
        case 14 * 4 + kTileR32: return launch_tile<Geom<14, 9>, SCHEME, 2>(p, a, batch, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

}  // namespace zinc
