// Raw-buffer access for the HIP kernels (device code only).
//
// A buffer resource holds a base address and a size in bytes; each load or store takes a
// wave-uniform byte offset (an SGPR: field, row, plane) and a per-lane byte offset (one
// VGPR), so no 64-bit address arithmetic runs on the vector ALU.  The hardware range check
// makes an access whose lane offset is at or past the size read zero and write nothing;
// kBufferOff is such an offset, used to switch single lanes off without a branch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace iewpf {

// Word 3 of a gfx9-family raw buffer resource: 32-bit data format, no swizzle.
constexpr int kRawBufferWord3 = 0x00020000;
constexpr unsigned kBufferOff = 0x80000000u;

// bytes must stay below 2^31 (callers check their sizes on the host).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), static_cast<short>(0),
                                           static_cast<int>(bytes), kRawBufferWord3);
}
__device__ __forceinline__ float ld_buf(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(voff),
                                                              static_cast<int>(soff), 0));
}
__device__ __forceinline__ void st_buf(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, static_cast<int>(voff),
                                        static_cast<int>(soff), 0);
}

}  // namespace iewpf
