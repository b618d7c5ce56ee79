// Raw buffer access on gfx950 (shared by the QR and GEMM kernels).
#pragma once
#include <hip/hip_runtime.h>

namespace sdc {

// Raw buffer access (gfx9 resource word 3 for untyped, unswizzled data):
// a load at a byte offset outside [0, bytes) returns zero and a store there
// is dropped, so padding rows and columns need no branches, and offsets are
// 32 bits.  The whole offset is passed as the per-lane offset (the range
// check applies to it; the scalar offset is left at zero).  kOob is an
// offset past every range used here, with room for the largest column step
// added to it (all ranges and steps are below 2^31 bytes).
constexpr unsigned kOob = 0x80000000u;
template <typename T> struct RawBuf {
    __amdgpu_buffer_rsrc_t r;
    __device__ RawBuf(const T* base, unsigned bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, (int)bytes, 0x00020000)) {}
    __device__ T load(unsigned off) const {
        if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
        else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
    __device__ void store(T x, unsigned off) const {
        if constexpr (sizeof(T) == 8) {
            typedef unsigned u2 __attribute__((ext_vector_type(2)));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, off, 0, 0);
        } else {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, off, 0, 0);
        }
    }
    // two adjacent FP32 elements in one 8-byte access (both in range or both
    // out of it: the callers pass kOob for a pair outside the data)
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __device__ f2 load2(unsigned off) const {
        static_assert(sizeof(T) == 4, "pairs of FP32 elements");
        return __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    }
    __device__ void store2(f2 x, unsigned off) const {
        static_assert(sizeof(T) == 4, "pairs of FP32 elements");
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, off, 0, 0);
    }
};

}  // namespace sdc
