// Initial guesses for the next solve and the force readout after a solve.
//
// combine3: the predictors of successive solves are linear combinations of
// earlier solutions (recycling, growth scaling, linear and quadratic
// extrapolation), one streaming pass of 8 bytes per term plus 8 written.
//
// accel: the acceleration -s J^-1 grad phi with the fourth-order central
// difference (u_{-2} - 8 u_{-1} + 8 u_{+1} - u_{+2}) / (12 h) along each axis
// and J = I + Hess psi from the same second-order stencils as the geometry.
// One pass reads phi (and psi) once from HBM; the +-2 neighbours come from
// the caches.
#include "kernels.h"
#include "stencil.h"

namespace mg {
namespace {

__global__ void k_combine3(size_t count, double c1, const double* phi1, double c2, const double* phi2,
                           double c3, const double* phi3, double* out) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        double v = c1 * phi1[i];
        if (c2 != 0.0) v += c2 * phi2[i];
        if (c3 != 0.0) v += c3 * phi3[i];
        out[i] = v;
    }
}

__device__ __forceinline__ double d4(const double* __restrict__ u, const Grid& g, int x, int y, int z, int dx,
                                     int dy, int dz, double i12h) {
    return (u[g(x - 2 * dx, y - 2 * dy, z - 2 * dz)] - 8.0 * u[g(x - dx, y - dy, z - dz)] +
            8.0 * u[g(x + dx, y + dy, z + dz)] - u[g(x + 2 * dx, y + 2 * dy, z + 2 * dz)]) *
           i12h;
}

template <typename TO, bool CURV>
__global__ __launch_bounds__(kThreads) void k_accel(int n, double ih2, double i12h, const double* __restrict__ phi,
                                                    const double* __restrict__ psi, double scale,
                                                    TO* __restrict__ a, int nz) {
    const Grid g{n, n - 1};
    const size_t N = (size_t)n * n * n;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    for (int z = z0; z < z0 + nz; ++z) {
        const size_t i = g(x, y, z);
        double gx = d4(phi, g, x, y, z, 1, 0, 0, i12h);
        double gy = d4(phi, g, x, y, z, 0, 1, 0, i12h);
        double gz = d4(phi, g, x, y, z, 0, 0, 1, i12h);
        if constexpr (CURV) {
            double H[6];
            hess_at(psi, g, x, y, z, ih2, H);
            H[0] += 1.0; H[1] += 1.0; H[2] += 1.0;
            Sym3 J, K;
            sym_from6(H, J);
            (void)inv3(J, K);
            const double ax = K.m[0][0] * gx + K.m[0][1] * gy + K.m[0][2] * gz;
            const double ay = K.m[1][0] * gx + K.m[1][1] * gy + K.m[1][2] * gz;
            const double az = K.m[2][0] * gx + K.m[2][1] * gy + K.m[2][2] * gz;
            gx = ax; gy = ay; gz = az;
        }
        a[i] = (TO)(-scale * gx);
        a[N + i] = (TO)(-scale * gy);
        a[2 * N + i] = (TO)(-scale * gz);
    }
}

}  // namespace

hipError_t launch_combine3(size_t count, double c1, const double* phi1, double c2, const double* phi2,
                           double c3, const double* phi3, double* out, hipStream_t s) {
    size_t blocks = (count + kThreads - 1) / kThreads;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_combine3, dim3((unsigned)blocks), dim3(kThreads), 0, s, count, c1, phi1, c2, phi2, c3,
                       phi3, out);
    return hipGetLastError();
}

template <typename TO>
hipError_t launch_accel(int n, double h, const double* phi, const double* psi, double scale, TO* a,
                        hipStream_t s) {
    const Shape sh = stencil_shape(n);
    const double ih2 = 1.0 / (h * h), i12h = 1.0 / (12.0 * h);
    if (psi)
        hipLaunchKernelGGL((k_accel<TO, true>), sh.grid, sh.block, 0, s, n, ih2, i12h, phi, psi, scale, a, sh.nz);
    else
        hipLaunchKernelGGL((k_accel<TO, false>), sh.grid, sh.block, 0, s, n, ih2, i12h, phi, psi, scale, a, sh.nz);
    return hipGetLastError();
}

template hipError_t launch_accel<float>(int, double, const double*, const double*, double, float*, hipStream_t);
template hipError_t launch_accel<double>(int, double, const double*, const double*, double, double*, hipStream_t);

}  // namespace mg
