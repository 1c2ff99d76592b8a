// Seven-point row-wave kernels (flat_row.hip): one wavefront per full x-row,
// used for levels with 64 <= n <= 1024.  Internal interface.
#pragma once
#include <hip/hip_runtime.h>

#include "sums.h"

namespace mg {

bool row_kernels_apply(int n);
// number of per-block partial sums the outer-residual kernel writes for an
// n^3 grid (double_arith: residual in double, otherwise float)
int row_outer_blocks(int n, bool double_arith);

template <typename T>
hipError_t launch_smooth_row(int n, double ih2, const T* x, const T* xprev, const T* b, T* out, double a,
                             double cd, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Step 1 of a pass from zero read from b alone: out = x1 + a1 x1 + cd1 (b - M x1)
// with x1 = cd0 * b formed on the fly in T (the bits of a single step from
// zero followed by a single step).  out must differ from b.
template <typename T>
hipError_t launch_smooth_fromb_row(int n, double ih2, const T* b, T* out, double a1, double cd1, double cd0,
                                   hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Post-smoothing on rows over 2 KB without two-step kernels
// (step_pro_applies): step 0 from x0 = x + P e formed on the fly (x_prev = 0,
// out = x1; x is not changed), and step 1 with x_prev = x0 = xold + P e
// formed pointwise (out may be xold).  e on the (n/2)^3 grid.
bool step_pro_applies(int n, size_t elem);
template <typename T>
hipError_t launch_smooth_pro_row(int n, double ih2, const T* x, const T* e, const T* b, T* out, double a0,
                                 double cd0, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename T>
hipError_t launch_smooth_prevp_row(int n, double ih2, const T* x1, const T* xold, const T* e, const T* b, T* out,
                                   double a1, double cd1, hipStream_t s, hipEvent_t ev0 = nullptr,
                                   hipEvent_t ev1 = nullptr);
// Step 2 of that pass: out = x + a2 (x - x1) + cd2 (b - M x) with x_prev
// x1 = cd0 * b formed from the b rows (not read).  out must differ from x and b.
template <typename T>
hipError_t launch_smooth_prevb_row(int n, double ih2, const T* x, const T* b, T* out, double a2, double cd2,
                                   double cd0, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Two consecutive smoothing steps in one pass (y2 and optionally y1 written;
// xp may be nullptr for x_prev = 0).  y2 and y1 must not alias x, xp or b.
// x0_mode == 1: the first three steps of a pass from zero instead; x and xp
// are not read, the first step x = cd0 * b is formed on the fly in T, and
// (a1, cd1) and (a2, cd2) are steps 1 and 2.
// x0_mode == 2: steps 2 and 3 of a pass from zero whose step 1 (x) came from
// launch_smooth_fromb_row: x_prev is the first step cd0 * b, formed on the fly
// (xp and y1 must be nullptr).
// sums (x0_mode 1 and 2 only): an extra block also finishes those partial
// sums (sums.h).
// ec != nullptr (x0_mode 0, no xp, pair_pro_applies): the pair starts from
// x0 = x + P ec, ec on the (n/2)^3 grid, formed on the fly; x is not changed.
// pair_kernels_apply tells whether n and the element size are supported.
bool pair_kernels_apply(int n, size_t elem);
bool pair_pro_applies(int n, size_t elem);
// Three steps in one pass from x with x_prev = 0 (the start of a smoothing
// pass that is not from zero): y3 after steps (a0, cd0), (a1, cd1), (a2, cd2).
// y3 must differ from x and b.
bool triple_kernels_apply(int n, size_t elem);
// The same pass starting from x0 = x + P e (e on the (n/2)^3 grid), x0 formed
// on the fly and never written: y3 after three steps from x0.  n >= 128.
bool triple_pro_applies(int n, size_t elem);
template <typename T>
hipError_t launch_prolong_triple_row(int n, double ih2, const T* x, const T* e, const T* b, T* y3, double a0,
                                     double cd0, double a1, double cd1, double a2, double cd2, hipStream_t s,
                                     hipEvent_t ev0, hipEvent_t ev1);
template <typename T>
hipError_t launch_smooth_triple_row(int n, double ih2, const T* x, const T* b, T* y3, double a0, double cd0,
                                    double a1, double cd1, double a2, double cd2, hipStream_t s, hipEvent_t ev0,
                                    hipEvent_t ev1);
template <typename T>
hipError_t launch_smooth_pair_row(int n, double ih2, const T* x, const T* xp, const T* b, T* y2, T* y1,
                                  double a1, double cd1, double a2, double cd2, hipStream_t s,
                                  hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, int x0_mode = 0,
                                  double cd0 = 0.0, const SumsJob* sums = nullptr, const T* ec = nullptr);
template <typename TA, typename TR, typename TE>
hipError_t launch_outer_row(int n, double ih2, const double* phi_in, const TE* e, double* phi_out, const double* b,
                            double bmean, TR* r, TR* x1, double cd0, double* partials, hipStream_t s,
                            hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename T>
hipError_t launch_rr_row(int n, double ih2, const T* x, const T* b, T* coarse, hipStream_t s,
                         hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename T>
hipError_t launch_prolong_row(int n, const T* e, T* x, hipStream_t s, hipEvent_t ev0 = nullptr,
                              hipEvent_t ev1 = nullptr);

}  // namespace mg
