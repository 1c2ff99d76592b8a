// mg_geometry_bwd_noalloc: the reverse mode of the moving-mesh geometry
// without any device allocation.  mg_geometry_bwd allocates a 6 n^3 double
// temporary (the per-cell cotangent of the triad) for each call; this variant
// keeps that temporary in a fixed, library-owned device array and walks the
// grid in z slabs that fit it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"
#include "mg.h"

using namespace mg;

namespace {

// 48 MiB of doubles per GPU, held until the process ends.  A slab of P planes
// of an n^3 grid needs 6 P n^2 doubles; P >= 3 (one output plane and its two
// neighbours) bounds n by 512.
constexpr size_t kScratchDoubles = (size_t)48 * 1024 * 1024 / sizeof(double);
static_assert(kScratchDoubles == (size_t)MG_NOALLOC_SCRATCH_BYTES / sizeof(double), "header and library agree");

__device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` per device, looked up once per device with that
// device current.  In host code the array's name is only a stand-in symbol.
constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mutex;

hipError_t scratch_of_current_device(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = static_cast<double*>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" mg_status mg_geometry_bwd_noalloc(int n, double h, const double* psi, const double* Cbar,
                                             const double* sqrtgbar, double* psibar, void* stream) {
    if (n < 4 || n > MG_NOALLOC_MAX_N || (n & (n - 1)) != 0 || !(h > 0) || !psi || !Cbar || !psibar)
        return MG_ERR_INVALID;
    double* Jbar = nullptr;
    if (scratch_of_current_device(&Jbar) != hipSuccess) {
        (void)hipGetLastError();
        return MG_ERR_HIP;
    }
    const double ih2 = 1.0 / (h * h);
    hipStream_t s = (hipStream_t)stream;
    const size_t plane = 6 * (size_t)n * n;  // doubles of one Jbar plane
    const int fit = (int)(kScratchDoubles / plane);
    hipError_t e = hipSuccess;
    if (fit >= n) {  // the whole grid at once, as mg_geometry_bwd does
        e = launch_geometry_bwd_cell(n, ih2, psi, Cbar, sqrtgbar, Jbar, s);
        if (e == hipSuccess) e = launch_hessian_adjoint(n, ih2, Jbar, psibar, s);
    } else {
        // slabs of `out` output planes with their two neighbour planes; the
        // next slab's cell kernel follows this slab's adjoint on the stream
        const int out = fit - 2;
        for (int z0 = 0; z0 < n && e == hipSuccess; z0 += out) {
            const int count = n - z0 < out ? n - z0 : out;
            e = launch_geometry_bwd_cell(n, ih2, psi, Cbar, sqrtgbar, Jbar, s, z0 - 1, count + 2);
            if (e == hipSuccess) e = launch_hessian_adjoint(n, ih2, Jbar, psibar, s, z0 - 1, count + 2, z0, count);
        }
    }
    return e == hipSuccess ? MG_OK : MG_ERR_HIP;
}
