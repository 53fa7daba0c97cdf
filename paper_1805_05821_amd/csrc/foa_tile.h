// Partial tile loads for the sweeps that prefetch only part of the next
// panel's tile (register budget): groups [G0, G1) of a panel's basis tile,
// one 16-byte non-temporal load per group and lane, into dst[D0 + g - G0].
#pragma once

#include "foa_device.h"

namespace foa {

template <typename TV, int G0, int G1, int D0, int D>
__device__ __forceinline__ void load_tile_groups(__amdgpu_buffer_rsrc_t rt, unsigned goff0, unsigned gbytes,
                                                 TV (&dst)[D][Vec<TV>::EPL]) {
#pragma unroll
  for (int g = G0; g < G1; ++g) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rt, (int)(goff0 + g * gbytes), 0, kTileLoad);
    unpack16<TV>(v, dst[D0 + g - G0]);
  }
}

}  // namespace foa
