// Fused level visits for the 32^3 and 64^3 levels of the seven-point hierarchy.
//
// On a 32^3 level every kernel of a V-cycle visit is far too small to fill the
// chip, and the visit costs its launch latencies (2v + 3 launches for v
// smoothing steps).  Here the visit takes two launches.  Each workgroup (1024
// threads, one per (x, y) point of a 32 x 32 plane) owns one coarse plane Z,
// i.e. fine planes 2Z and 2Z + 1, and recomputes what it needs of the
// neighbouring planes (a halo of v + 1 planes shrinking by one per step), all
// of it in LDS:
//
//   pre:  x_1 = c_0 D^-1 b (pointwise), v - 1 further steps, r = b - M x_v,
//         coarse rhs = R r; writes x_v on the owned planes and the coarse plane;
//   post: x_0 = x + P e, v steps; writes x_v on the owned planes.
//
// This is the paper's fused wide-halo level visit (one exchange per visit
// instead of one per step), used here to save launches instead of exchanges.
// Every point formula is the shared one of the unfused kernels (stencil.h), so
// the result is bitwise that of the separate smoothing, residual, restriction
// and prolongation kernels.
#include "visit.h"

#include "fma.h"
#include "stencil.h"

namespace mg {
namespace {

constexpr int kN = 32;                // points per side
constexpr int kP = kN * kN;           // points per plane = threads per workgroup
constexpr int kMaxDeg = kVisitMaxDegree;
constexpr int kPrePlanes = 2 * kMaxDeg + 3;   // planes of x_1 in the pre visit
// b and two iterate stacks of kPrePlanes planes, and the three residual planes
// of the pre visit: 144 KB of the 160 KB a gfx950 workgroup may use
constexpr int kLdsFloats = (3 * kPrePlanes + 3) * kP;

struct VisitCoef {
    float a[kMaxDeg], cd[kMaxDeg];  // step k: x + a_k (x - x_prev) + cd_k (b - M x)
};

__device__ __forceinline__ int wrap(int i) { return i & (kN - 1); }

// seven-point stencil at (x, y) of plane p of an LDS stack of planes
__device__ __forceinline__ float M_at(const float* st, int p, int x, int y, float ih2) {
    const float* c = st + p * kP;
    const float* m = c - kP;
    const float* q = c + kP;
    return flat7_pt<float>(c[y * kN + wrap(x - 1)], c[y * kN + wrap(x + 1)], c[wrap(y - 1) * kN + x],
                           c[wrap(y + 1) * kN + x], m[y * kN + x], q[y * kN + x], c[y * kN + x], ih2);
}

// Plane stacks: every stack holds the planes [lo, lo + NP) of a field.  Two
// iterate stacks alternate: a step reads x_{k-1} only at the point it writes,
// so x_{k+1} overwrites x_{k-1} in place.  V (the step count) is a template
// parameter so that every plane loop unrolls and the global loads of the
// staging loops are all in flight at once.
template <int V>
__global__ __launch_bounds__(kP) void k_visit_pre(const float* __restrict__ b, float* __restrict__ xout,
                                                  float* __restrict__ coarse_b, float ih2, VisitCoef coef) {
    constexpr int NP = 2 * V + 3;  // planes of x_1: z0 - 1 - V .. z0 + 1 + V
    __shared__ float lds[kLdsFloats];
    const int t = threadIdx.x;
    const int x = t & (kN - 1), y = t >> 5;
    const int Z = blockIdx.x;
    const int z0 = 2 * Z;
    const int lo = z0 - 1 - V;
    float* sb = lds;  // b on the x_1 planes
    float* buf[2] = {lds + NP * kP, lds + 2 * NP * kP};
    float* rs = lds + 3 * NP * kP;  // residual on planes z0 - 1 .. z0 + 1
    static_assert(3 * NP * kP + 3 * kP <= kLdsFloats, "pre visit stacks exceed LDS");
    // b and x_1 = c_0 D^-1 b on every plane of the stack
    float bv[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) bv[p] = b[(size_t)wrap(lo + p) * kP + t];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        sb[p * kP + t] = bv[p];
        buf[0][p * kP + t] = coef.cd[0] * bv[p];
    }
    __syncthreads();
    // step k makes x_{k+1} on planes lo + k .. z0 + 1 + V - k (one fewer per side each step)
    int cur = 0, prv = -1;
#pragma unroll
    for (int k = 1; k < V; ++k) {
        const int out = prv >= 0 ? prv : 1;
#pragma unroll
        for (int p = k; p <= NP - 1 - k; ++p) {
            const float xc = buf[cur][p * kP + t];
            const float xp = prv >= 0 ? buf[prv][p * kP + t] : 0.0f;
            const float Mx = M_at(buf[cur], p, x, y, ih2);
            buf[out][p * kP + t] = step_pt<float>(xc, xp, sb[p * kP + t], Mx, coef.a[k], coef.cd[k]);
        }
        __syncthreads();
        prv = cur;
        cur = out;
    }
    // residual on planes z0 - 1 .. z0 + 1 (stack planes V .. V + 2)
#pragma unroll
    for (int p = V; p <= V + 2; ++p) rs[(p - V) * kP + t] = sb[p * kP + t] - M_at(buf[cur], p, x, y, ih2);
    // the smoothed iterate on the owned planes
#pragma unroll
    for (int p = V + 1; p <= V + 2; ++p) xout[(size_t)(lo + p) * kP + t] = buf[cur][p * kP + t];
    __syncthreads();
    // full weighting onto coarse plane Z (16 x 16 points)
    if (t < kP / 4) {
        const int X = t & (kN / 2 - 1), Y = t >> 4;
        float vv[3][3][3];
#pragma unroll
        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
                    vv[dz][dy][dx] = rs[dz * kP + wrap(2 * Y + dy - 1) * kN + wrap(2 * X + dx - 1)];
        coarse_b[(size_t)Z * (kP / 4) + t] = fw_pt<float>(vv);
    }
}

template <int V>
__global__ __launch_bounds__(kP) void k_visit_post(const float* __restrict__ xin, const float* __restrict__ e,
                                                   const float* __restrict__ b, float* __restrict__ xout, float ih2,
                                                   VisitCoef coef) {
    constexpr int NP = 2 * V + 2;              // planes of x_0: z0 - V .. z0 + 1 + V
    constexpr int NC = 2 * ((V + 1) / 2) + 2;  // coarse planes the prolongation reads
    constexpr int nc = kN / 2, pc = nc * nc;
    __shared__ float lds[kLdsFloats];
    const int t = threadIdx.x;
    const int x = t & (kN - 1), y = t >> 5;
    const int Z = blockIdx.x;
    const int z0 = 2 * Z;
    const int lo = z0 - V;
    const int zlo = Z - (V + 1) / 2;  // first staged coarse plane
    float* sb = lds;
    float* buf[2] = {lds + NP * kP, lds + 2 * NP * kP};
    float* se = lds + 3 * NP * kP;  // coarse planes zlo .. zlo + NC - 1
    static_assert(3 * NP * kP + NC * pc <= kLdsFloats, "post visit stacks exceed LDS");
    float bv[NP], xv[NP], ev[(NC * pc + kP - 1) / kP];
#pragma unroll
    for (int j = 0; j < (NC * pc + kP - 1) / kP; ++j) {
        const int q = j * kP + t;
        ev[j] = q < NC * pc ? e[(size_t)((zlo + q / pc) & (nc - 1)) * pc + (q % pc)] : 0.0f;
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        bv[p] = b[(size_t)wrap(lo + p) * kP + t];
        xv[p] = xin[(size_t)wrap(lo + p) * kP + t];
    }
#pragma unroll
    for (int j = 0; j < (NC * pc + kP - 1) / kP; ++j)
        if (j * kP + t < NC * pc) se[j * kP + t] = ev[j];
    __syncthreads();
    // coarse value at periodic (X, Y, Zc); Zc is unwrapped, within the staged planes
    auto ec = [&](int X, int Y, int Zc) { return se[(Zc - zlo) * pc + (Y & (nc - 1)) * nc + (X & (nc - 1))]; };
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        sb[p * kP + t] = bv[p];
        buf[0][p * kP + t] = add_pt<float>(xv[p], prolong_pt<float>(ec, x, y, lo + p));
    }
    __syncthreads();
    int cur = 0, prv = -1;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const int out = prv >= 0 ? prv : 1;
#pragma unroll
        for (int p = k + 1; p <= NP - 2 - k; ++p) {
            const float xc = buf[cur][p * kP + t];
            const float xp = prv >= 0 ? buf[prv][p * kP + t] : 0.0f;
            const float Mx = M_at(buf[cur], p, x, y, ih2);
            buf[out][p * kP + t] = step_pt<float>(xc, xp, sb[p * kP + t], Mx, coef.a[k], coef.cd[k]);
        }
        __syncthreads();
        prv = cur;
        cur = out;
    }
#pragma unroll
    for (int p = V; p <= V + 1; ++p) xout[(size_t)(lo + p) * kP + t] = buf[cur][p * kP + t];
}

// step coefficients in the kernels' precision, c_k / D rounded as in the
// single-step launches
VisitCoef visit_coef(double ih2, const double* a, const double* c, int degree) {
    VisitCoef coef{};
    const double D = -6.0 * ih2;
    for (int k = 0; k < degree; ++k) {
        coef.a[k] = (float)a[k];
        coef.cd[k] = (float)(c[k] / D);
    }
    return coef;
}

// ---- the 64^3 level: tiles of 64 x 8 fine rows -------------------------------------
// A workgroup owns coarse plane Z and fine rows y0 .. y0+7 (y0 = 8 t, tile t
// of 8); it keeps the rows y0-4 .. y0+11 (16 x 64 = one point per thread) of
// every plane it needs, and the valid rows shrink by one per side per step
// like the planes.  Point formulas are those of the row kernels of this size:
// the stencil and step of flat7_row / cheb_step (same operation order), the
// restriction in y, then x, then z with fw3 rounding (k_rr_row), the
// prolongation in x, then y, then z (k_prolong_row for one point per lane).
constexpr int kN64 = 64, kTY = 8, kHY = 4, kTR = kTY + 2 * kHY;  // 16 tile rows
static_assert(kN64 * kTR == kP, "one tile point per thread");

__device__ __forceinline__ int wrap64(int i) { return i & (kN64 - 1); }

// seven-point stencil at (x, row r) of plane p of a tile stack (r +- 1 inside the tile)
__device__ __forceinline__ float M_tile(const float* st, int p, int x, int r, float ih2) {
    const float* c = st + p * kP;
    const float* m = c - kP;
    const float* q = c + kP;
    return flat7_pt<float>(c[r * kN64 + wrap64(x - 1)], c[r * kN64 + wrap64(x + 1)], c[(r - 1) * kN64 + x],
                           c[(r + 1) * kN64 + x], m[r * kN64 + x], q[r * kN64 + x], c[r * kN64 + x], ih2);
}

template <int V>
__global__ __launch_bounds__(kP) void k_visit64_pre(const float* __restrict__ b, float* __restrict__ xout,
                                                    float* __restrict__ coarse_b, float ih2, VisitCoef coef) {
    constexpr int NP = 2 * V + 3;  // planes z0 - 1 - V .. z0 + 1 + V
    __shared__ float lds[kLdsFloats];
    const int t = threadIdx.x;
    const int x = t & (kN64 - 1), r = t >> 6;
    const int Z = blockIdx.x >> 3, tile = blockIdx.x & 7;
    const int z0 = 2 * Z, y0 = kTY * tile;
    const int y = wrap64(y0 - kHY + r);
    const int lo = z0 - 1 - V;
    float* sb = lds;
    float* buf[2] = {lds + NP * kP, lds + 2 * NP * kP};
    float* rs = lds + 3 * NP * kP;  // residual on planes z0 - 1 .. z0 + 1
    static_assert(3 * NP * kP + 3 * kP <= kLdsFloats, "pre visit stacks exceed LDS");
    static_assert(V + 1 <= kHY, "the tile halo covers the steps, the residual and the restriction");
    float bv[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) bv[p] = b[((size_t)wrap64(lo + p) * kN64 + y) * kN64 + x];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        sb[p * kP + t] = bv[p];
        buf[0][p * kP + t] = coef.cd[0] * bv[p];
    }
    __syncthreads();
    int cur = 0, prv = -1;
#pragma unroll
    for (int k = 1; k < V; ++k) {  // x_{k+1} on rows k .. 15-k, planes k .. NP-1-k
        const int out = prv >= 0 ? prv : 1;
        if (r >= k && r <= kTR - 1 - k) {
#pragma unroll
            for (int p = k; p <= NP - 1 - k; ++p) {
                const float xc = buf[cur][p * kP + t];
                const float xp = prv >= 0 ? buf[prv][p * kP + t] : 0.0f;
                const float Mx = M_tile(buf[cur], p, x, r, ih2);
                buf[out][p * kP + t] = step_pt<float>(xc, xp, sb[p * kP + t], Mx, coef.a[k], coef.cd[k]);
            }
        }
        __syncthreads();
        prv = cur;
        cur = out;
    }
    // residual on rows 3 .. 11 (fine rows y0-1 .. y0+7), planes V .. V+2
    if (r >= kHY - 1 && r <= kHY + kTY - 1) {
#pragma unroll
        for (int p = V; p <= V + 2; ++p) rs[(p - V) * kP + t] = sb[p * kP + t] - M_tile(buf[cur], p, x, r, ih2);
    }
    // the smoothed iterate on the owned rows and planes
    if (r >= kHY && r < kHY + kTY) {
#pragma unroll
        for (int p = V + 1; p <= V + 2; ++p) xout[((size_t)(lo + p) * kN64 + y) * kN64 + x] = buf[cur][p * kP + t];
    }
    __syncthreads();
    // full weighting onto the tile's 4 coarse rows of coarse plane Z: y, then x, then z
    if (t < (kN64 / 2) * (kTY / 2)) {
        const int X = t & (kN64 / 2 - 1), Yl = t >> 5;
        const float* rr = rs;
        float sz[3];
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
            float sx[3];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int xx = wrap64(2 * X + dx - 1);
                const float* col = rr + dz * kP + xx;
                const int r0 = kHY - 1 + 2 * Yl;  // tile row of fine row 2Y - 1
                sx[dx] = fw3<float>(col[r0 * kN64], col[(r0 + 1) * kN64], col[(r0 + 2) * kN64]);
            }
            sz[dz] = fw3<float>(sx[0], sx[1], sx[2]);
        }
        const int Y = y0 / 2 + Yl;
        coarse_b[((size_t)Z * (kN64 / 2) + Y) * (kN64 / 2) + X] = fw3<float>(sz[0], sz[1], sz[2]);
    }
}

template <int V>
__global__ __launch_bounds__(kP) void k_visit64_post(const float* __restrict__ xin, const float* __restrict__ e,
                                                     const float* __restrict__ b, float* __restrict__ xout,
                                                     float ih2, VisitCoef coef) {
    constexpr int NP = 2 * V + 2;              // planes z0 - V .. z0 + 1 + V
    constexpr int NC = 2 * ((V + 1) / 2) + 2;  // coarse planes the prolongation reads
    constexpr int nc = kN64 / 2;
    constexpr int CR = kTR / 2 + 2;            // coarse rows staged: (y0-4)/2 - 1 .. (y0+11)/2 + 1
    __shared__ float lds[kLdsFloats];
    const int t = threadIdx.x;
    const int x = t & (kN64 - 1), r = t >> 6;
    const int Z = blockIdx.x >> 3, tile = blockIdx.x & 7;
    const int z0 = 2 * Z, y0 = kTY * tile;
    const int yu = y0 - kHY + r;  // unwrapped fine row (parity and coarse row as for the wrapped one)
    const int y = wrap64(yu);
    const int lo = z0 - V;
    const int zlo = Z - (V + 1) / 2, ylo = (y0 - kHY) / 2 - 1;  // first staged coarse plane / row
    float* sb = lds;
    float* buf[2] = {lds + NP * kP, lds + 2 * NP * kP};
    float* se = lds + 3 * NP * kP;  // coarse planes zlo .. zlo+NC-1, rows ylo .. ylo+CR-1
    static_assert(3 * NP * kP + NC * CR * nc <= kLdsFloats, "post visit stacks exceed LDS");
    static_assert(V <= kHY, "the tile halo covers the steps");
    constexpr int NE = (NC * CR * nc + kP - 1) / kP;
    float ev[NE], bv[NP], xv[NP];
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        const int q = j * kP + t;
        if (q < NC * CR * nc) {
            const int zc = q / (CR * nc), rc = (q / nc) % CR, xc = q % nc;
            ev[j] = e[((size_t)((zlo + zc) & (nc - 1)) * nc + ((ylo + rc) & (nc - 1))) * nc + xc];
        }
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const size_t gi = ((size_t)wrap64(lo + p) * kN64 + y) * kN64 + x;
        bv[p] = b[gi];
        xv[p] = xin[gi];
    }
#pragma unroll
    for (int j = 0; j < NE; ++j)
        if (j * kP + t < NC * CR * nc) se[j * kP + t] = ev[j];
    __syncthreads();
    // coarse value at (X, Y, Zc): Y, Zc unwrapped within the staged block, X periodic
    auto ec = [&](int X, int Y, int Zc) { return se[((Zc - zlo) * CR + (Y - ylo)) * nc + (X & (nc - 1))]; };
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        sb[p * kP + t] = bv[p];
        buf[0][p * kP + t] = add_pt<float>(xv[p], prolong_pt<float>(ec, x, yu, lo + p));
    }
    __syncthreads();
    int cur = 0, prv = -1;
#pragma unroll
    for (int k = 0; k < V; ++k) {  // x_{k+1} on rows k+1 .. 14-k, planes k+1 .. NP-2-k
        const int out = prv >= 0 ? prv : 1;
        if (r >= k + 1 && r <= kTR - 2 - k) {
#pragma unroll
            for (int p = k + 1; p <= NP - 2 - k; ++p) {
                const float xc = buf[cur][p * kP + t];
                const float xp = prv >= 0 ? buf[prv][p * kP + t] : 0.0f;
                const float Mx = M_tile(buf[cur], p, x, r, ih2);
                buf[out][p * kP + t] = step_pt<float>(xc, xp, sb[p * kP + t], Mx, coef.a[k], coef.cd[k]);
            }
        }
        __syncthreads();
        prv = cur;
        cur = out;
    }
    if (r >= kHY && r < kHY + kTY) {
#pragma unroll
        for (int p = V; p <= V + 1; ++p) xout[((size_t)(lo + p) * kN64 + y) * kN64 + x] = buf[cur][p * kP + t];
    }
}

}  // namespace

bool visit_pre_applies(int n, int degree) {
    return degree >= 1 && ((n == kN && degree <= kMaxDeg) || (n == kN64 && degree <= kHY - 1));
}
bool visit_post_applies(int n, int degree) {
    return degree >= 1 && ((n == kN && degree <= kMaxDeg) || (n == kN64 && degree <= kHY && degree <= kMaxDeg));
}

hipError_t launch_visit_pre(int n, double ih2, const float* b, float* xout, float* coarse_b, const double* a,
                            const double* c, int degree, hipStream_t s) {
    if (!visit_pre_applies(n, degree)) return hipErrorInvalidValue;
    const VisitCoef coef = visit_coef(ih2, a, c, degree);
    const float fih2 = (float)ih2;
    if (n == kN64) {
        const dim3 grid((kN64 / 2) * (kN64 / kTY)), block(kP);
        switch (degree) {
        case 1: hipLaunchKernelGGL(k_visit64_pre<1>, grid, block, 0, s, b, xout, coarse_b, fih2, coef); break;
        case 2: hipLaunchKernelGGL(k_visit64_pre<2>, grid, block, 0, s, b, xout, coarse_b, fih2, coef); break;
        default: hipLaunchKernelGGL(k_visit64_pre<3>, grid, block, 0, s, b, xout, coarse_b, fih2, coef); break;
        }
        return hipGetLastError();
    }
    const dim3 grid(kN / 2), block(kP);
    switch (degree) {
    case 1: hipLaunchKernelGGL(k_visit_pre<1>, grid, block, 0, s, b, xout, coarse_b, fih2, coef); break;
    case 2: hipLaunchKernelGGL(k_visit_pre<2>, grid, block, 0, s, b, xout, coarse_b, fih2, coef); break;
    case 3: hipLaunchKernelGGL(k_visit_pre<3>, grid, block, 0, s, b, xout, coarse_b, fih2, coef); break;
    default: hipLaunchKernelGGL(k_visit_pre<4>, grid, block, 0, s, b, xout, coarse_b, fih2, coef); break;
    }
    return hipGetLastError();
}

hipError_t launch_visit_post(int n, double ih2, const float* xin, const float* e, const float* b, float* xout,
                             const double* a, const double* c, int degree, hipStream_t s) {
    if (!visit_post_applies(n, degree) || xout == xin) return hipErrorInvalidValue;
    const VisitCoef coef = visit_coef(ih2, a, c, degree);
    const float fih2 = (float)ih2;
    if (n == kN64) {
        const dim3 grid((kN64 / 2) * (kN64 / kTY)), block(kP);
        switch (degree) {
        case 1: hipLaunchKernelGGL(k_visit64_post<1>, grid, block, 0, s, xin, e, b, xout, fih2, coef); break;
        case 2: hipLaunchKernelGGL(k_visit64_post<2>, grid, block, 0, s, xin, e, b, xout, fih2, coef); break;
        case 3: hipLaunchKernelGGL(k_visit64_post<3>, grid, block, 0, s, xin, e, b, xout, fih2, coef); break;
        default: hipLaunchKernelGGL(k_visit64_post<4>, grid, block, 0, s, xin, e, b, xout, fih2, coef); break;
        }
        return hipGetLastError();
    }
    const dim3 grid(kN / 2), block(kP);
    switch (degree) {
    case 1: hipLaunchKernelGGL(k_visit_post<1>, grid, block, 0, s, xin, e, b, xout, fih2, coef); break;
    case 2: hipLaunchKernelGGL(k_visit_post<2>, grid, block, 0, s, xin, e, b, xout, fih2, coef); break;
    case 3: hipLaunchKernelGGL(k_visit_post<3>, grid, block, 0, s, xin, e, b, xout, fih2, coef); break;
    default: hipLaunchKernelGGL(k_visit_post<4>, grid, block, 0, s, xin, e, b, xout, fih2, coef); break;
    }
    return hipGetLastError();
}

}  // namespace mg
