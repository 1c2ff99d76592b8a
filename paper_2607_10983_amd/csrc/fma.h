// Fused multiply-add rounded once in the operands' own precision.  The
// generic __builtin_fma is the double one: on float operands it would
// compute in double and round twice (and run on the slower FP64 units).
#pragma once
#include <hip/hip_runtime.h>

namespace mg {

__device__ __forceinline__ float fma_rn(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_rn(double a, double b, double c) { return __builtin_fma(a, b, c); }

}  // namespace mg
