// Single-workgroup V-cycle tail for the seven-point hierarchy.
//
// Levels with at most 16^3 points are far too small to fill the chip; one
// kernel launch per smoothing step there costs more in launch latency than in
// work.  This kernel runs the whole remaining V-cycle from a small level down
// to the coarsest and back up inside ONE workgroup of 1024 threads: every
// smoothing step, residual, restriction, coarsest solve and prolongation is
// a phase of the same kernel, separated by workgroup barriers.  All tail
// level fields live in LDS (gfx950 gives a workgroup up to 160 KB: three
// fields of 16^3 + 8^3 + 4^3 points take 56 KB in float, 112 KB in double);
// only the first tail level's right-hand side is read from and its result
// written back to global memory.  The coarsest level's exact solve
// (separable real Fourier basis) also runs in LDS, in double.
#include "tail.h"

namespace mg {
namespace {

constexpr int kTailThreads = 1024;

constexpr int kMaxPts = 4;  // 16^3 points / 1024 threads

__device__ __forceinline__ void coords(int i, int n, int lg, int& x, int& y, int& z) {
    x = i & (n - 1);
    y = (i >> lg) & (n - 1);
    z = i >> (2 * lg);
}
__device__ __forceinline__ int at(int x, int y, int z, int n, int lg) {
    const int m = n - 1;
    return ((((z & m) << lg) | (y & m)) << lg) | (x & m);
}

template <typename T>
__device__ __forceinline__ T Mx_at(const T* u, int x, int y, int z, int n, int lg, T ih2) {
    const T c = u[at(x, y, z, n, lg)];
    T s = u[at(x - 1, y, z, n, lg)] + u[at(x + 1, y, z, n, lg)];
    s += u[at(x, y - 1, z, n, lg)] + u[at(x, y + 1, z, n, lg)];
    s += u[at(x, y, z - 1, n, lg)] + u[at(x, y, z + 1, n, lg)];
    return (s - T(6) * c) * ih2;
}

// Every phase computes the thread's (at most kMaxPts) points with all loads
// issued before any store, then stores them, then waits at the barrier.
template <typename T, typename F>
__device__ __forceinline__ void phase(int N, F f, T* out) {
    T v[kMaxPts];
#pragma unroll
    for (int k = 0; k < kMaxPts; ++k) {
        const int i = threadIdx.x + k * kTailThreads;
        if (i < N) v[k] = f(i);
    }
#pragma unroll
    for (int k = 0; k < kMaxPts; ++k) {
        const int i = threadIdx.x + k * kTailThreads;
        if (i < N) out[i] = v[k];
    }
    __syncthreads();
}

constexpr int kTailElems = 3 * (4096 + 512 + 64);  // x0, x1, b of 16^3, 8^3, 4^3

// LDS layout: level l's x0, x1, b follow those of levels 0..l-1.
template <typename T>
struct Fields {
    T* base;
    const TailArgs<T>* A;
    __device__ __forceinline__ T* lev(int l) const {
        int off = 0;
        for (int k = 0; k < l; ++k) off += 3 * A->n[k] * A->n[k] * A->n[k];
        return base + off;
    }
    __device__ __forceinline__ T* x(int l, int k) const {
        const int N = A->n[l] * A->n[l] * A->n[l];
        return lev(l) + k * N;
    }
    __device__ __forceinline__ T* b(int l) const { return x(l, 2); }
};

// One smoothing pass on tail level l (same buffer rotation as the multi-kernel path).
template <typename T>
__device__ int smooth_pass(const TailArgs<T>& A, const Fields<T>& F, int l, int cur, bool from_zero) {
    const int n = A.n[l], lg = A.lg[l], N = n * n * n;
    const T ih2 = (T)A.ih2[l];
    const T dinv = T(1) / (T(-6) * ih2);
    const T* b = F.b(l);
    int prev = -1;
    for (int k = 0; k < A.sched.steps; ++k) {
        const T a = (T)A.sched.a[l][k], c = (T)A.sched.c[l][k];
        if (k == 0 && from_zero) {
            phase<T>(N, [&](int i) { return c * dinv * b[i]; }, F.x(l, 0));
            cur = 0;
            prev = -1;
        } else {
            const bool use_prev = A.sched.cheb && prev >= 0;
            const int o = use_prev ? prev : 1 - cur;
            const T* xc = F.x(l, cur);
            const T* xp = use_prev ? F.x(l, prev) : nullptr;
            phase<T>(N, [&](int i) {
                int x, y, z;
                coords(i, n, lg, x, y, z);
                const T Mx = Mx_at(xc, x, y, z, n, lg, ih2);
                const T xi = xc[i];
                const T pv = use_prev ? xp[i] : T(0);
                return xi + a * (xi - pv) + c * dinv * (b[i] - Mx);
            }, F.x(l, o));
            prev = cur;
            cur = o;
        }
    }
    return cur;
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailArgs<T> A) {
    __shared__ T fields[kTailElems];
    __shared__ double sA[512];
    __shared__ double sB[512];
    __shared__ double q[64];
    __shared__ double lam[8];
    const Fields<T> F{fields, &A};
    unsigned curbits = 0;  // bit l: buffer holding level l's iterate (no private array)
    const int nl = A.nlev;
    const int tid = threadIdx.x;
    {   // right-hand side of the first tail level from global memory
        const int N0 = A.n[0] * A.n[0] * A.n[0];
        T* b0 = F.b(0);
        for (int i = tid; i < N0; i += kTailThreads) b0[i] = A.b[0][i];
        __syncthreads();
    }
    // ---------------- down leg
    for (int l = 0; l + 1 < nl; ++l) {
        const int n = A.n[l], lg = A.lg[l], N = n * n * n;
        const T ih2 = (T)A.ih2[l];
        const int cl = smooth_pass(A, F, l, 0, true);
        curbits = (curbits & ~(1u << l)) | ((unsigned)cl << l);
        // residual into the free buffer, then full weighting into the coarse rhs
        T* r = F.x(l, 1 - cl);
        const T* xc = F.x(l, cl);
        const T* b = F.b(l);
        phase<T>(N, [&](int i) {
            int x, y, z;
            coords(i, n, lg, x, y, z);
            return b[i] - Mx_at(xc, x, y, z, n, lg, ih2);
        }, r);
        const int nc = A.n[l + 1], lgc = A.lg[l + 1], Nc = nc * nc * nc;
        phase<T>(Nc, [&](int i) {
            int X, Y, Z;
            coords(i, nc, lgc, X, Y, Z);
            T acc = T(0);
            for (int dz = -1; dz <= 1; ++dz) {
                T ay = T(0);
                for (int dy = -1; dy <= 1; ++dy) {
                    const int fy = 2 * Y + dy, fz = 2 * Z + dz;
                    const T ax = T(0.25) * r[at(2 * X - 1, fy, fz, n, lg)] + T(0.5) * r[at(2 * X, fy, fz, n, lg)] +
                                 T(0.25) * r[at(2 * X + 1, fy, fz, n, lg)];
                    ay += (dy == 0 ? T(0.5) : T(0.25)) * ax;
                }
                acc += (dz == 0 ? T(0.5) : T(0.25)) * ay;
            }
            return acc;
        }, F.b(l + 1));
    }
    // ---------------- coarsest: exact zero-mean solve in double (separable basis)
    {
        const int l = nl - 1;
        const int nc = A.n[l];
        const int N = nc * nc * nc;
        for (int i = tid; i < nc * nc; i += kTailThreads) q[i] = A.Q[i];
        for (int i = tid; i < nc; i += kTailThreads) lam[i] = A.lam1[i];
        const T* bl = F.b(l);
        for (int i = tid; i < N; i += kTailThreads) sA[i] = (double)bl[i];
        __syncthreads();
        auto pass = [&](const double* src, double* dst, int axis, bool forward) {
            for (int i = tid; i < N; i += kTailThreads) {
                const int x = i % nc, y = (i / nc) % nc, z = i / (nc * nc);
                const int k = axis == 0 ? x : axis == 1 ? y : z;
                const int stride = axis == 0 ? 1 : axis == 1 ? nc : nc * nc;
                const int base = i - k * stride;
                double acc = 0.0;
                for (int j = 0; j < nc; ++j) acc += (forward ? q[j + nc * k] : q[k + nc * j]) * src[base + j * stride];
                dst[i] = acc;
            }
            __syncthreads();
        };
        pass(sA, sB, 0, true);
        pass(sB, sA, 1, true);
        pass(sA, sB, 2, true);
        for (int i = tid; i < N; i += kTailThreads) {
            const int x = i % nc, y = (i / nc) % nc, z = i / (nc * nc);
            sB[i] = (x == 0 && y == 0 && z == 0) ? 0.0 : sB[i] / (lam[x] + lam[y] + lam[z]);
        }
        __syncthreads();
        pass(sB, sA, 2, false);
        pass(sA, sB, 1, false);
        pass(sB, sA, 0, false);
        T* xl = F.x(l, 0);
        for (int i = tid; i < N; i += kTailThreads) xl[i] = (T)sA[i];
        curbits &= ~(1u << l);
        __syncthreads();
    }
    // ---------------- up leg
    for (int l = nl - 2; l >= 0; --l) {
        const int n = A.n[l], lg = A.lg[l], N = n * n * n;
        const int nc = A.n[l + 1], lgc = A.lg[l + 1];
        const T* e = F.x(l + 1, (curbits >> (l + 1)) & 1);
        const int cl = (curbits >> l) & 1;
        T* xv = F.x(l, cl);
        phase<T>(N, [&](int i) {
            int x, y, z;
            coords(i, n, lg, x, y, z);
            const int X = x >> 1, Y = y >> 1, Z = z >> 1, ox = x & 1, oy = y & 1, oz = z & 1;
            const T w = (ox ? T(0.5) : T(1)) * (oy ? T(0.5) : T(1)) * (oz ? T(0.5) : T(1));
            T v = T(0);
            for (int kz = 0; kz <= oz; ++kz)
                for (int ky = 0; ky <= oy; ++ky)
                    for (int kx = 0; kx <= ox; ++kx) v += w * e[at(X + kx, Y + ky, Z + kz, nc, lgc)];
            return xv[i] + v;
        }, xv);
        const int cn = smooth_pass(A, F, l, cl, false);
        curbits = (curbits & ~(1u << l)) | ((unsigned)cn << l);
    }
    {   // result of the first tail level to global memory (always its buffer x0)
        const int N0 = A.n[0] * A.n[0] * A.n[0];
        const T* x0 = F.x(0, curbits & 1);
        for (int i = tid; i < N0; i += kTailThreads) A.x0[0][i] = x0[i];
    }
}

}  // namespace

template <typename T>
hipError_t launch_tail(const TailArgs<T>& args, hipStream_t s) {
    if (args.nlev < 2 || args.nlev > kTailMaxLevels || args.n[0] > 16 || args.n[args.nlev - 1] > 8)
        return hipErrorInvalidValue;
    int elems = 0;
    for (int l = 0; l < args.nlev; ++l) elems += 3 * args.n[l] * args.n[l] * args.n[l];
    if (elems > kTailElems) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_tail<T>), dim3(1), dim3(kTailThreads), 0, s, args);
    return hipGetLastError();
}

template hipError_t launch_tail<float>(const TailArgs<float>&, hipStream_t);
template hipError_t launch_tail<double>(const TailArgs<double>&, hipStream_t);

}  // namespace mg
