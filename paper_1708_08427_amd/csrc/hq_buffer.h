// Raw buffer access for gfx950 kernels.
//
// A buffer resource covers at most 2 GiB from its base; a lane whose byte
// offset is kOOB (or beyond the resource's size) is switched off: its load
// returns 0 and its store is dropped.  Kernels use this to issue every memory
// instruction unconditionally, so that the compiler's wait counts cover
// exactly the loads a step needs and never the stores issued after them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hq {

using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr uint32_t kOOB = 0x80000000u;  // byte offset past the end of every buffer used this way

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

// The same for a base and size computed per wave: both are made uniform
// explicitly, so the resource lives in scalar registers.
__device__ __forceinline__ rsrc_t make_rsrc_uniform(const void *p, uint32_t bytes) {
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const uint32_t n = __builtin_amdgcn_readfirstlane(bytes);
    return make_rsrc(reinterpret_cast<const void *>(((uint64_t)hi << 32) | lo), n);
}

}  // namespace hq
