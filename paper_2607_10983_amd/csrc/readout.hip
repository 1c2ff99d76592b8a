// Initial guesses for the next solve and the force readout after a solve.
//
// combine3: the predictors of successive solves are linear combinations of
// earlier solutions (recycling, growth scaling, linear and quadratic
// extrapolation), one streaming pass of 8 bytes per term plus 8 written.
//
// accel: the acceleration -s J^-1 grad phi with the fourth-order central
// difference (u_{-2} - 8 u_{-1} + 8 u_{+1} - u_{+2}) / (12 h) along each axis
// and J = I + Hess psi from the same second-order stencils as the geometry.
// One pass reads phi (and psi) once from HBM.  Levels of 64 .. 1024 points
// per side use a row-wave kernel: one wavefront per x-row (lane l holds VEC =
// n/64 consecutive points), the x-neighbours from rotating cross-lane moves,
// the z-neighbours from a register queue of the wave's own rows as it
// marches a chunk of planes, the y-neighbour rows from the caches (they are
// the adjacent waves' rows).  Other sizes use one thread per (x, y) column.
#include "kernels.h"
#include "row.h"
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

// ---- row-wave force readout ------------------------------------------------------
constexpr int kAccelWaves = 4;

// u shifted by -2, -1, +1, +2 in x along a row held VEC per lane.
template <int VEC>
__device__ __forceinline__ void xshifts(const double (&u)[VEC], double (&m2)[VEC], double (&m1)[VEC],
                                        double (&p1)[VEC], double (&p2)[VEC]) {
    if constexpr (VEC == 1) {
        m1[0] = lane_rot(u[0], -1);
        m2[0] = lane_rot(m1[0], -1);
        p1[0] = lane_rot(u[0], 1);
        p2[0] = lane_rot(p1[0], 1);
    } else {
        const double l1 = lane_rot(u[VEC - 1], -1), l2 = lane_rot(u[VEC - 2], -1);
        const double r1 = lane_rot(u[0], 1), r2 = lane_rot(u[1], 1);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            m1[e] = e >= 1 ? u[e - 1] : l1;
            m2[e] = e >= 2 ? u[e - 2] : (e == 1 ? l1 : l2);
            p1[e] = e + 1 < VEC ? u[e + 1] : r1;
            p2[e] = e + 2 < VEC ? u[e + 2] : (e + 1 < VEC ? r1 : r2);
        }
    }
}

// u shifted by -1 and +1 in x.
template <int VEC>
__device__ __forceinline__ void xshift1(const double (&u)[VEC], double (&m1)[VEC], double (&p1)[VEC]) {
    const double l1 = lane_rot(u[VEC - 1], -1), r1 = lane_rot(u[0], 1);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        m1[e] = e >= 1 ? u[e - 1] : l1;
        p1[e] = e + 1 < VEC ? u[e + 1] : r1;
    }
}

template <typename TO, int VEC, bool CURV>
__global__ __launch_bounds__(64 * kAccelWaves) void k_accel_row(int n, double ih2, double i12h,
                                                                const double* __restrict__ phi,
                                                                const double* __restrict__ psi, double scale,
                                                                TO* __restrict__ a, int nz, int nyb) {
    constexpr int NR = 64 * VEC;
    const RowGrid g{NR, NR - 1};
    const size_t N = (size_t)NR * NR * NR;
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int y = yb * kAccelWaves + wave_id();
    const int z0 = zc * nz;
    const size_t off = (size_t)(threadIdx.x & 63) * VEC;
    // phi rows of this wave at planes z-2 .. z+2, psi rows at z-1 .. z+1
    double q0[VEC], q1[VEC], q2[VEC], q3[VEC], q4[VEC];
    double s0[VEC], s1[VEC], s2[VEC];
    ldrow<double, VEC>(q0, phi + g.row(y, z0 - 2) + off);
    ldrow<double, VEC>(q1, phi + g.row(y, z0 - 1) + off);
    ldrow<double, VEC>(q2, phi + g.row(y, z0) + off);
    ldrow<double, VEC>(q3, phi + g.row(y, z0 + 1) + off);
    if constexpr (CURV) {
        ldrow<double, VEC>(s0, psi + g.row(y, z0 - 1) + off);
        ldrow<double, VEC>(s1, psi + g.row(y, z0) + off);
    }
    for (int k = 0; k < nz; ++k) {
        const int z = z0 + k;
        double ym2[VEC], ym1[VEC], yp1[VEC], yp2[VEC];
        ldrow<double, VEC>(q4, phi + g.row(y, z + 2) + off);
        ldrow<double, VEC>(ym2, phi + g.row(y - 2, z) + off);
        ldrow<double, VEC>(ym1, phi + g.row(y - 1, z) + off);
        ldrow<double, VEC>(yp1, phi + g.row(y + 1, z) + off);
        ldrow<double, VEC>(yp2, phi + g.row(y + 2, z) + off);
        double m2[VEC], m1[VEC], p1[VEC], p2[VEC];
        xshifts<VEC>(q2, m2, m1, p1, p2);
        double gx[VEC], gy[VEC], gz[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            gx[e] = (m2[e] - 8.0 * m1[e] + 8.0 * p1[e] - p2[e]) * i12h;
            gy[e] = (ym2[e] - 8.0 * ym1[e] + 8.0 * yp1[e] - yp2[e]) * i12h;
            gz[e] = (q0[e] - 8.0 * q1[e] + 8.0 * q3[e] - q4[e]) * i12h;
        }
        if constexpr (CURV) {
            double tm[VEC], tp[VEC], um[VEC], up[VEC], wm[VEC], wp[VEC];
            ldrow<double, VEC>(s2, psi + g.row(y, z + 1) + off);
            ldrow<double, VEC>(tm, psi + g.row(y - 1, z) + off);
            ldrow<double, VEC>(tp, psi + g.row(y + 1, z) + off);
            ldrow<double, VEC>(um, psi + g.row(y - 1, z - 1) + off);
            ldrow<double, VEC>(up, psi + g.row(y + 1, z - 1) + off);
            ldrow<double, VEC>(wm, psi + g.row(y - 1, z + 1) + off);
            ldrow<double, VEC>(wp, psi + g.row(y + 1, z + 1) + off);
            double cm[VEC], cp[VEC], tmm[VEC], tmp[VEC], tpm[VEC], tpp[VEC], lm[VEC], lp[VEC], hm[VEC], hp[VEC];
            xshift1<VEC>(s1, cm, cp);
            xshift1<VEC>(tm, tmm, tmp);
            xshift1<VEC>(tp, tpm, tpp);
            xshift1<VEC>(s0, lm, lp);
            xshift1<VEC>(s2, hm, hp);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const double c = s1[e];
                double H[6];
                H[0] = (cp[e] - 2.0 * c + cm[e]) * ih2;
                H[1] = (tp[e] - 2.0 * c + tm[e]) * ih2;
                H[2] = (s2[e] - 2.0 * c + s0[e]) * ih2;
                H[3] = (tpp[e] - tmp[e] - tpm[e] + tmm[e]) * 0.25 * ih2;
                H[4] = (hp[e] - lp[e] - hm[e] + lm[e]) * 0.25 * ih2;
                H[5] = (wp[e] - up[e] - wm[e] + um[e]) * 0.25 * ih2;
                H[0] += 1.0; H[1] += 1.0; H[2] += 1.0;
                Sym3 J, K;
                sym_from6(H, J);
                (void)inv3(J, K);
                const double ax = K.m[0][0] * gx[e] + K.m[0][1] * gy[e] + K.m[0][2] * gz[e];
                const double ay = K.m[1][0] * gx[e] + K.m[1][1] * gy[e] + K.m[1][2] * gz[e];
                const double az = K.m[2][0] * gx[e] + K.m[2][1] * gy[e] + K.m[2][2] * gz[e];
                gx[e] = ax; gy[e] = ay; gz[e] = az;
            }
        }
        TO ox[VEC], oy[VEC], oz[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            ox[e] = (TO)(-scale * gx[e]);
            oy[e] = (TO)(-scale * gy[e]);
            oz[e] = (TO)(-scale * gz[e]);
        }
        const size_t r = g.row(y, z) + off;
        strow<TO, VEC>(a + r, ox);
        strow<TO, VEC>(a + N + r, oy);
        strow<TO, VEC>(a + 2 * N + r, oz);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            q0[e] = q1[e]; q1[e] = q2[e]; q2[e] = q3[e]; q3[e] = q4[e];
            if constexpr (CURV) { s0[e] = s1[e]; s1[e] = s2[e]; }
        }
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
    const double ih2 = 1.0 / (h * h), i12h = 1.0 / (12.0 * h);
    if (n >= 64 && n <= 1024) {
        // rows in blocks of kAccelWaves; z chunks of at least 8 planes, about 1024 blocks
        const int nyb = n / kAccelWaves;
        int nz = n;
        while (nz > 8 && nyb * (n / nz) < 1024) nz >>= 1;
        const dim3 grid(nyb * (n / nz)), block(64 * kAccelWaves);
#define MG_ACCEL(VEC)                                                                                            \
    do {                                                                                                         \
        if (psi) hipLaunchKernelGGL((k_accel_row<TO, VEC, true>), grid, block, 0, s, n, ih2, i12h, phi, psi,      \
                                    scale, a, nz, nyb);                                                          \
        else hipLaunchKernelGGL((k_accel_row<TO, VEC, false>), grid, block, 0, s, n, ih2, i12h, phi, psi, scale, \
                                a, nz, nyb);                                                                     \
    } while (0)
        switch (n) {
            case 64: MG_ACCEL(1); break;
            case 128: MG_ACCEL(2); break;
            case 256: MG_ACCEL(4); break;
            case 512: MG_ACCEL(8); break;
            case 1024: MG_ACCEL(16); break;
            default: return hipErrorInvalidValue;
        }
#undef MG_ACCEL
        return hipGetLastError();
    }
    const Shape sh = stencil_shape(n);
    if (psi)
        hipLaunchKernelGGL((k_accel<TO, true>), sh.grid, sh.block, 0, s, n, ih2, i12h, phi, psi, scale, a, sh.nz);
    else
        hipLaunchKernelGGL((k_accel<TO, false>), sh.grid, sh.block, 0, s, n, ih2, i12h, phi, psi, scale, a, sh.nz);
    return hipGetLastError();
}

template hipError_t launch_accel<float>(int, double, const double*, const double*, double, float*, hipStream_t);
template hipError_t launch_accel<double>(int, double, const double*, const double*, double, double*, hipStream_t);

}  // namespace mg
