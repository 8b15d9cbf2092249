// bufio.h -- buffer loads and stores with a 32-bit per-lane byte offset and a
// uniform (scalar) one: gathers and row stores without 64-bit address
// arithmetic on the vector ALU.  Raw buffers, resource word 3 for gfx950.
#pragma once

#include <cstdint>

namespace cis {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float bf_floatx4 __attribute__((ext_vector_type(4)));
typedef double bf_double2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), short(0), int(bytes), 0x00020000);
}
__device__ __forceinline__ void buffer_ld(float &x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    x = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0));
}
__device__ __forceinline__ void buffer_ld(double &x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), 0);
    x = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(v[1]) << 32) | v[0]));
}
__device__ __forceinline__ uint32_t buffer_ld_u32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0);
}
// 16-byte forms
__device__ __forceinline__ void buffer_ld(bf_floatx4 &x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    x = __builtin_bit_cast(bf_floatx4, __builtin_amdgcn_raw_buffer_load_b128(r, int(voff), int(soff), 0));
}
__device__ __forceinline__ void buffer_ld(bf_double2 &x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    x = __builtin_bit_cast(bf_double2, __builtin_amdgcn_raw_buffer_load_b128(r, int(voff), int(soff), 0));
}
__device__ __forceinline__ void buffer_st(const bf_floatx4 &x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, x), r, int(voff), int(soff), 0);
}
__device__ __forceinline__ void buffer_st(const bf_double2 &x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, x), r, int(voff), int(soff), 0);
}
// streaming stores (non-temporal hint: data read once, much later)
__device__ __forceinline__ void buffer_st_nt(const bf_floatx4 &x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, x), r, int(voff), int(soff), 2);
}
__device__ __forceinline__ void buffer_st_nt(const bf_double2 &x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, x), r, int(voff), int(soff), 2);
}

}  // namespace cis
