// Fused level visits of the 32^3 and 64^3 seven-point levels with Chebyshev
// smoothing (visit.hip).  Internal interface.
#pragma once
#include <hip/hip_runtime.h>

namespace mg {

// Largest smoothing degree a fused visit handles (its plane stacks must fit LDS).
constexpr int kVisitMaxDegree = 4;

// True when the pre (post) visit of the level (n^3 points, n = 32 or 64,
// smoothing degree) can run fused.  The 64^3 pre visit's tile halo of four
// rows covers at most three steps.
bool visit_pre_applies(int n, int degree);
bool visit_post_applies(int n, int degree);

// Pre-smoothing from zero, residual and full weighting in one launch:
// xout (n^3) = `degree` steps from zero on b; coarse_b ((n/2)^3) = R(b - M xout).
// a[k], c[k]: the step coefficients of the level (x + a_k (x - x_prev) + c_k D^-1 (b - M x)).
hipError_t launch_visit_pre(int n, double ih2, const float* b, float* xout, float* coarse_b, const double* a,
                            const double* c, int degree, hipStream_t s);

// Prolongation and post-smoothing in one launch: xout = `degree` steps on
// xin + P e (e on the (n/2)^3 grid); xout must differ from xin.
hipError_t launch_visit_post(int n, double ih2, const float* xin, const float* e, const float* b, float* xout,
                             const double* a, const double* c, int degree, hipStream_t s);

}  // namespace mg
