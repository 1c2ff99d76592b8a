// Single-workgroup V-cycle tail (tail.hip): the levels of at most 16^3 points
// of a seven-point hierarchy, down to a coarsest level of at most 8^3 points,
// in one kernel launch.  Internal interface.
#pragma once
#include <hip/hip_runtime.h>

namespace mg {

constexpr int kTailMaxLevels = 4;
constexpr int kTailMaxSteps = 16;

struct TailSchedule {
    int steps;
    int cheb;  // 1: Chebyshev (uses the previous iterate), 0: Jacobi
    double a[kTailMaxLevels][kTailMaxSteps];
    double c[kTailMaxLevels][kTailMaxSteps];
};

// Only x0[0] and b[0] (the first tail level) are accessed in global memory:
// the tail reads b[0] and leaves the V-cycle result in x0[0].
template <typename T>
struct TailArgs {
    int nlev;                      // levels in the tail, the last one is the coarsest
    int n[kTailMaxLevels];
    int lg[kTailMaxLevels];
    double ih2[kTailMaxLevels];
    T* x0[kTailMaxLevels];
    T* x1[kTailMaxLevels];
    T* b[kTailMaxLevels];
    TailSchedule sched;
    const double* Q;               // coarsest separable basis (nc x nc)
    const double* lam1;            // its 1-D eigenvalues
};

template <typename T>
hipError_t launch_tail(const TailArgs<T>& args, hipStream_t s);

}  // namespace mg
