// Device building blocks shared by the generic stencil kernels: periodic
// indexing, fixed-order block reductions, field accessors, the seven-point and
// 19-point flux-form operators at one point, and the column launch shape.
#pragma once
#include <hip/hip_runtime.h>

#include "fma.h"

#include <cstddef>

namespace mg {
namespace {

constexpr int kThreads = 256;

struct Grid {
    int n, mask;
    __device__ __forceinline__ size_t operator()(int x, int y, int z) const {
        return ((size_t)(z & mask) * (size_t)n + (size_t)(y & mask)) * (size_t)n + (size_t)(x & mask);
    }
};

__device__ __forceinline__ int lin_tid() {
    return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
}
__device__ __forceinline__ int lin_bid() {
    return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

// Fixed-order LDS tree over a power-of-two block; result valid in every thread.
__device__ double block_sum(double v, double* sh) {
    const int tid = lin_tid();
    const int nt = blockDim.x * blockDim.y * blockDim.z;
    sh[tid] = v;
    __syncthreads();
    for (int s = nt >> 1; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}
__device__ double block_max(double v, double* sh) {
    const int tid = lin_tid();
    const int nt = blockDim.x * blockDim.y * blockDim.z;
    sh[tid] = v;
    __syncthreads();
    for (int s = nt >> 1; s > 0; s >>= 1) {
        if (tid < s) sh[tid] = fmax(sh[tid], sh[tid + s]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// ---- field accessors (value of the iterate at a linear index, in type T) ----
template <typename T, typename TU>
struct Plain {
    const TU* p;
    __device__ __forceinline__ T operator()(size_t i) const { return (T)p[i]; }
};
template <typename T, typename TE>
struct PlusE {  // phi + e, formed in double
    const double* p;
    const TE* e;
    __device__ __forceinline__ T operator()(size_t i) const { return (T)(p[i] + (double)e[i]); }
};

// ---- operators -------------------------------------------------------------------
// Seven-point Laplacian: (sum of the six neighbours - 6 u) / h^2.
template <typename T, typename F>
__device__ __forceinline__ T flat_Mu(const F& u, const Grid& g, int x, int y, int z, T uc, T ih2);

// ---- point formulas with their rounding written out ------------------------------
// Every seven-point kernel (row kernels, generic column kernels, fused level
// visits) evaluates the stencil, the smoothing step, full weighting and the
// prolongation through these, with no contraction left to the compiler, so
// that fused and unfused paths produce the same bits.

// (sum of the six neighbours - 6 c) / h^2
template <typename T>
__device__ __forceinline__ T flat7_pt(T xm, T xp, T ym, T yp, T zm, T zp, T c, T ih2) {
#pragma clang fp contract(off)
    const T s = ((xm + xp) + (ym + yp)) + (zm + zp);
    return fma_rn(T(-6), c, s) * ih2;
}

// one smoothing step x + a (x - xp) + cd (b - M x), cd = c / D
template <typename T>
__device__ __forceinline__ T step_pt(T x, T xp, T b, T Mx, T a, T cd) {
#pragma clang fp contract(off)
    return fma_rn(cd, b - Mx, fma_rn(a, x - xp, x));
}

// full weighting of the 27 fine values v[dz][dy][dx] (offsets -1, 0, 1)
template <typename T>
__device__ __forceinline__ T fw_pt(const T (&v)[3][3][3]) {
#pragma clang fp contract(off)
    const T w1[3] = {T(0.25), T(0.5), T(0.25)};
    T acc = T(0);
    for (int dz = 0; dz < 3; ++dz) {
        T accy = T(0);
        for (int dy = 0; dy < 3; ++dy) {
            T accx = T(0);
            for (int dx = 0; dx < 3; ++dx) accx += w1[dx] * v[dz][dy][dx];
            accy += w1[dy] * accx;
        }
        acc += w1[dz] * accy;
    }
    return acc;
}

// trilinear prolongation at fine point (x, y, z) of the coarse field read by
// ec(X, Y, Z) (periodic indices)
template <typename T, typename E>
__device__ __forceinline__ T prolong_pt(const E& ec, int x, int y, int z) {
#pragma clang fp contract(off)
    const int X = x >> 1, Y = y >> 1, Z = z >> 1;
    const int ox = x & 1, oy = y & 1, oz = z & 1;
    T vz[2];
    for (int kz = 0; kz <= oz; ++kz) {
        T vy[2];
        for (int ky = 0; ky <= oy; ++ky) {
            const T a0 = ec(X, Y + ky, Z + kz);
            vy[ky] = ox ? T(0.5) * (a0 + ec(X + 1, Y + ky, Z + kz)) : a0;
        }
        vz[kz] = oy ? T(0.5) * (vy[0] + vy[1]) : vy[0];
    }
    return oz ? T(0.5) * (vz[0] + vz[1]) : vz[0];
}

template <typename T>
__device__ __forceinline__ T add_pt(T x, T p) {
#pragma clang fp contract(off)
    return x + p;
}

template <typename T, typename F>
__device__ __forceinline__ T flat_Mu(const F& u, const Grid& g, int x, int y, int z, T uc, T ih2) {
    return flat7_pt<T>(u(g(x - 1, y, z)), u(g(x + 1, y, z)), u(g(x, y - 1, z)), u(g(x, y + 1, z)),
                       u(g(x, y, z - 1)), u(g(x, y, z + 1)), uc, ih2);
}

// Flux-form operator: face-averaged diagonal coefficients times compact
// normal differences, plus D0_a (C^{ab} D0_b u) for the six ordered pairs.
// Returns M u and the diagonal D (both scaled by 1/h^2).
template <typename T, typename TC, typename F>
__device__ __forceinline__ void var_Mu(const F& u, const TC* __restrict__ C, size_t N, const Grid& g,
                                       int x, int y, int z, T uc, T ih2, T& Mu, T& D) {
    const TC* Cxx = C;
    const TC* Cyy = C + N;
    const TC* Czz = C + 2 * N;
    const TC* Cxy = C + 3 * N;
    const TC* Cxz = C + 4 * N;
    const TC* Cyz = C + 5 * N;
    const size_t i0 = g(x, y, z);
    T acc, dsum;
    {
        const T c0 = (T)Cxx[i0];
        const T fp = T(0.5) * (c0 + (T)Cxx[g(x + 1, y, z)]);
        const T fm = T(0.5) * (c0 + (T)Cxx[g(x - 1, y, z)]);
        acc = fp * (u(g(x + 1, y, z)) - uc) - fm * (uc - u(g(x - 1, y, z)));
        dsum = fp + fm;
    }
    {
        const T c0 = (T)Cyy[i0];
        const T fp = T(0.5) * (c0 + (T)Cyy[g(x, y + 1, z)]);
        const T fm = T(0.5) * (c0 + (T)Cyy[g(x, y - 1, z)]);
        acc += fp * (u(g(x, y + 1, z)) - uc) - fm * (uc - u(g(x, y - 1, z)));
        dsum += fp + fm;
    }
    {
        const T c0 = (T)Czz[i0];
        const T fp = T(0.5) * (c0 + (T)Czz[g(x, y, z + 1)]);
        const T fm = T(0.5) * (c0 + (T)Czz[g(x, y, z - 1)]);
        acc += fp * (u(g(x, y, z + 1)) - uc) - fm * (uc - u(g(x, y, z - 1)));
        dsum += fp + fm;
    }
    T cross;
    {   // pairs (x,y) and (y,x)
        const T upp = u(g(x + 1, y + 1, z)), upm = u(g(x + 1, y - 1, z));
        const T ump = u(g(x - 1, y + 1, z)), umm = u(g(x - 1, y - 1, z));
        cross = (T)Cxy[g(x + 1, y, z)] * (upp - upm) - (T)Cxy[g(x - 1, y, z)] * (ump - umm);
        cross += (T)Cxy[g(x, y + 1, z)] * (upp - ump) - (T)Cxy[g(x, y - 1, z)] * (upm - umm);
    }
    {   // pairs (x,z) and (z,x)
        const T upp = u(g(x + 1, y, z + 1)), upm = u(g(x + 1, y, z - 1));
        const T ump = u(g(x - 1, y, z + 1)), umm = u(g(x - 1, y, z - 1));
        cross += (T)Cxz[g(x + 1, y, z)] * (upp - upm) - (T)Cxz[g(x - 1, y, z)] * (ump - umm);
        cross += (T)Cxz[g(x, y, z + 1)] * (upp - ump) - (T)Cxz[g(x, y, z - 1)] * (upm - umm);
    }
    {   // pairs (y,z) and (z,y)
        const T upp = u(g(x, y + 1, z + 1)), upm = u(g(x, y + 1, z - 1));
        const T ump = u(g(x, y - 1, z + 1)), umm = u(g(x, y - 1, z - 1));
        cross += (T)Cyz[g(x, y + 1, z)] * (upp - upm) - (T)Cyz[g(x, y - 1, z)] * (ump - umm);
        cross += (T)Cyz[g(x, y, z + 1)] * (upp - ump) - (T)Cyz[g(x, y, z - 1)] * (upm - umm);
    }
    Mu = (acc + T(0.25) * cross) * ih2;
    D = -dsum * ih2;
}

template <typename T, typename TC>
__device__ __forceinline__ T var_diag(const TC* __restrict__ C, size_t N, const Grid& g, int x, int y, int z,
                                      T ih2) {
    const size_t i0 = g(x, y, z);
    T d = T(0);
    for (int a = 0; a < 3; ++a) {
        const TC* c = C + a * N;
        const T c0 = (T)c[i0];
        const int dx = a == 0, dy = a == 1, dz = a == 2;
        d += T(0.5) * (c0 + (T)c[g(x + dx, y + dy, z + dz)]) + T(0.5) * (c0 + (T)c[g(x - dx, y - dy, z - dz)]);
    }
    return -d * ih2;
}

// ---- launch shape ------------------------------------------------------------------
struct Shape {
    dim3 grid, block;
    int nz;
};
inline Shape stencil_shape(int n) {
    const int bx = n < 64 ? n : 64;
    int by = kThreads / bx;
    if (by > n) by = n;
    size_t pts = (size_t)n * n * n;
    size_t want = pts / ((size_t)kThreads * 2048);
    int nz = 1;
    while ((size_t)nz * 2 <= want && nz < 32) nz *= 2;
    if (nz > n) nz = n;
    Shape s;
    s.block = dim3(bx, by, 1);
    s.grid = dim3(n / bx, n / by, n / nz);
    s.nz = nz;
    return s;
}

// ---- moving-mesh geometry at one point -----------------------------------------
// Second-order central Hessian of psi, components (xx, yy, zz, xy, xz, yz).
__device__ __forceinline__ void hess_at(const double* __restrict__ psi, const Grid& g, int x, int y, int z,
                                        double ih2, double H[6]) {
    const double c = psi[g(x, y, z)];
    H[0] = (psi[g(x + 1, y, z)] - 2.0 * c + psi[g(x - 1, y, z)]) * ih2;
    H[1] = (psi[g(x, y + 1, z)] - 2.0 * c + psi[g(x, y - 1, z)]) * ih2;
    H[2] = (psi[g(x, y, z + 1)] - 2.0 * c + psi[g(x, y, z - 1)]) * ih2;
    H[3] = (psi[g(x + 1, y + 1, z)] - psi[g(x + 1, y - 1, z)] - psi[g(x - 1, y + 1, z)] + psi[g(x - 1, y - 1, z)]) * 0.25 * ih2;
    H[4] = (psi[g(x + 1, y, z + 1)] - psi[g(x + 1, y, z - 1)] - psi[g(x - 1, y, z + 1)] + psi[g(x - 1, y, z - 1)]) * 0.25 * ih2;
    H[5] = (psi[g(x, y + 1, z + 1)] - psi[g(x, y + 1, z - 1)] - psi[g(x, y - 1, z + 1)] + psi[g(x, y - 1, z - 1)]) * 0.25 * ih2;
}

// Symmetric 3x3 (a,b,c,d,e,f) = (xx,yy,zz,xy,xz,yz): determinant and inverse.
struct Sym3 {
    double m[3][3];
};
__device__ __forceinline__ void sym_from6(const double s[6], Sym3& A) {
    A.m[0][0] = s[0]; A.m[1][1] = s[1]; A.m[2][2] = s[2];
    A.m[0][1] = A.m[1][0] = s[3];
    A.m[0][2] = A.m[2][0] = s[4];
    A.m[1][2] = A.m[2][1] = s[5];
}
__device__ __forceinline__ double inv3(const Sym3& J, Sym3& K) {
    const double (*m)[3] = J.m;
    const double c00 = m[1][1] * m[2][2] - m[1][2] * m[2][1];
    const double c01 = m[1][2] * m[2][0] - m[1][0] * m[2][2];
    const double c02 = m[1][0] * m[2][1] - m[1][1] * m[2][0];
    const double det = m[0][0] * c00 + m[0][1] * c01 + m[0][2] * c02;
    const double id = 1.0 / det;
    K.m[0][0] = c00 * id;
    K.m[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) * id;
    K.m[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) * id;
    K.m[1][0] = c01 * id;
    K.m[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) * id;
    K.m[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) * id;
    K.m[2][0] = c02 * id;
    K.m[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) * id;
    K.m[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) * id;
    return det;
}
__device__ __forceinline__ void mul3(const Sym3& A, const Sym3& B, Sym3& C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C.m[i][j] = A.m[i][0] * B.m[0][j] + A.m[i][1] * B.m[1][j] + A.m[i][2] * B.m[2][j];
}

}  // namespace
}  // namespace mg
