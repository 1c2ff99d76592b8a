// 19-point flux-form operator, row-wave kernels (var_row.hip) for levels with
// 64 <= n <= 1024.  Internal interface.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace mg {

bool var_row_kernels_apply(int n);
// number of per-block partial sums launch_var_outer_row writes
int var_row_blocks(int n);

// out = x + a (x - xprev) + c D^-1 (b - M x); x == nullptr: out = c D^-1 b
template <typename T, typename TC>
hipError_t launch_var_smooth_row(int n, double ih2, const TC* C, const T* x, const T* xprev, const T* b, T* out,
                                 double a, double c, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
// Two steps in one pass, only the second written:
//   y1 = x + a1 (x - xp) + c1 D^-1 (b - M x) (xp == nullptr: xp = 0),
//   y2 = y1 + a2 (y1 - x) + c2 D^-1 (b - M y1);
// y2 must differ from x and xp.  Float rows of up to 1 KB, n >= 128
// (var_pair_applies); hipErrorInvalidValue otherwise.
bool var_pair_applies(int n, size_t elem);
template <typename T, typename TC>
hipError_t launch_var_smooth_pair(int n, double ih2, const TC* C, const T* x, const T* xp, const T* b, T* y2,
                                  double a1, double c1, double a2, double c2, hipStream_t s, hipEvent_t ev0,
                                  hipEvent_t ev1);
// out = b - M x (b != nullptr) or out = M x
template <typename T, typename TC>
hipError_t launch_var_resid_row(int n, double ih2, const TC* C, const T* x, const T* b, T* out, hipStream_t s,
                                hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename TA, typename TR, typename TE, typename TC>
hipError_t launch_var_outer_row(int n, double ih2, const TC* C, const double* phi_in, const TE* e, double* phi_out,
                                const double* b, double bmean, TR* r, TR* x1, double c0, double* partials,
                                hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

}  // namespace mg
