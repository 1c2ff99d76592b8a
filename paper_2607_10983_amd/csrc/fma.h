// Point arithmetic with its rounding written out, shared by the kernels that
// must agree bitwise.
//
// fma_rn: fused multiply-add rounded once in the operands' own precision.  The
// generic __builtin_fma is the double one: on float operands it would compute
// in double and round twice (and run on the slower FP64 units).
// fw3: the one-dimensional full-weighting stencil 1/4, 1/2, 1/4 applied to
// (a, b, c), summed left to right with no contraction.
#pragma once
#include <hip/hip_runtime.h>

namespace mg {

__device__ __forceinline__ float fma_rn(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_rn(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ T fw3(T a, T b, T c) {
#pragma clang fp contract(off)
    return ((T(0.25) * a) + (T(0.5) * b)) + (T(0.25) * c);
}

}  // namespace mg
