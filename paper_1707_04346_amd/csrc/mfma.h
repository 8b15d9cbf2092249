// mfma.h -- the 16x16x4 matrix-core products of the sigma kernels (FP32 and
// FP64 forms) and the accumulator layout they produce on gfx950.
//
// Operand layout of one 16x16x4 product D = A B + C (64 lanes):
//   A: lane l holds A[l % 16][l / 16];  B: lane l holds B[l / 16][l % 16];
//   D column = l % 16, row as given by out_row(l, r) for accumulator register r.
#pragma once

namespace cis {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef double double2_t __attribute__((ext_vector_type(2)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
    using acc_t = floatx4;
    using vec_t = floatx4;   // 16-byte load: 4 columns
    static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // accumulator register r of a lane holds output row 4*(lane/16) + r
    static __device__ __forceinline__ int out_row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mfma<double> {
    using acc_t = doublex4;
    using vec_t = double2_t;  // 16-byte load: 2 columns
    static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // the FP64 form spaces a lane's rows by 4: register r holds row lane/16 + 4*r
    static __device__ __forceinline__ int out_row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

}  // namespace cis
