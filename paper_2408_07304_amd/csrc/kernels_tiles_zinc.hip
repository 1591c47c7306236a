// Alternative geometries of the fused kernel, Zinc scheme.
#include "kernels_tiles.h"

namespace zinc {

hipError_t launch_encrypt_slots_tile_zinc(const DevParams& p, int tile, bool reg, const double* slots,
                                          uint32_t n_slots, uint32_t batch, const uint64_t* ct_ids, uint64_t* ct,
                                          hipStream_t s) {
    const EncArgs a{slots, n_slots, nullptr, (const u64*)ct_ids, (u64*)ct};
    return launch_tile_scheme<ZINC_SCHEME_ZINC>(p, tile, reg, a, batch, s);
}

}  // namespace zinc
