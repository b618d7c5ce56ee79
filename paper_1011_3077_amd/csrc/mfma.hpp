// CDNA matrix-core wrappers: one 16x16x4 multiply-accumulate per wavefront.
//
// Operand layout of v_mfma_{f64_16x16x4f64, f32_16x16x4f32} (wave64), as
// measured on gfx950:
//   A (16 x 4):  lane l supplies A[l % 16][l / 16]
//   B (4 x 16):  lane l supplies B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[row(l / 16, v)][l % 16], v = 0..3, with
//                row(g, v) = g + 4 v for f64 and 4 g + v for f32.
#pragma once
#include <hip/hip_runtime.h>

namespace sdc {

template <typename T> struct Mfma;

template <> struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static constexpr int row(int g, int v) { return g + 4 * v; }
    __device__ static inline v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

template <> struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static constexpr int row(int g, int v) { return 4 * g + v; }
    __device__ static inline v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

}  // namespace sdc
