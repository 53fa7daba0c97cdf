// Buffer-resource helpers shared by the kernels.  A raw buffer access whose
// offset is at or beyond the resource's num_records returns 0 (loads) or is
// dropped (stores): kernels mask dead columns, padded rows and idle lanes by
// pointing their offset at kOOR instead of branching, so the compiler can count
// outstanding memory operations exactly and keep prefetched data in flight.
#pragma once

#include <hip/hip_runtime.h>

namespace foa {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000;   // raw buffer, 32-bit data format (CDNA)
constexpr unsigned kOOR = 0x80000000u;   // offset beyond every range used with it
// Cache policy of the basis-tile loads: non-temporal (the "nt" bit).  A tile
// is streamed once per sweep and the basis is far larger than the caches; on
// MI355X this policy raises a read-mostly panel walk from about 6.3 to about
// 7.1 TB/s (measured with a stand-alone probe of the access pattern).
constexpr int kTileLoad = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kRsrcWord3);
}

}  // namespace foa
