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

// Level geometry as compile-time constants: the tail's levels have 16^3, 8^3
// or 4^3 points, and with the sizes fixed every neighbour index reduces to a
// few masks and the per-thread point loops unroll.
template <int N>
struct Geo {
    static constexpr int n = N;
    static constexpr int lg = N == 16 ? 4 : N == 8 ? 3 : 2;
    static constexpr int P = N * N * N;
    static constexpr int m = N - 1;
    static constexpr int pts = (P + kTailThreads - 1) / kTailThreads;  // points per thread
    static_assert(N == 4 || N == 8 || N == 16, "tail levels have 4^3, 8^3 or 16^3 points");
    __device__ static __forceinline__ void coords(int i, int& x, int& y, int& z) {
        x = i & m;
        y = (i >> lg) & m;
        z = i >> (2 * lg);
    }
    __device__ static __forceinline__ int at(int x, int y, int z) {
        return ((((z & m) << lg) | (y & m)) << lg) | (x & m);
    }
};

template <typename T, int N>
__device__ __forceinline__ T Mx_at(const T* u, int i, T ih2) {
    using G = Geo<N>;
    constexpr int mx = G::m, my = G::m << G::lg, pz = N * N;
    const T c = u[i];
    T s = u[(i & ~mx) | ((i - 1) & mx)] + u[(i & ~mx) | ((i + 1) & mx)];
    s += u[(i & ~my) | ((i - N) & my)] + u[(i & ~my) | ((i + N) & my)];
    s += u[(i - pz) & (G::P - 1)] + u[(i + pz) & (G::P - 1)];
    return (s - T(6) * c) * ih2;
}

// Every phase computes the thread's points with all loads issued before any
// store, then stores them, then waits at the barrier.
template <typename T, int P, typename F>
__device__ __forceinline__ void phase(F f, T* out) {
    constexpr int K = (P + kTailThreads - 1) / kTailThreads;
    T v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * kTailThreads;
        if (P % kTailThreads == 0 || i < P) v[k] = f(i);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * kTailThreads;
        if (P % kTailThreads == 0 || i < P) out[i] = v[k];
    }
    __syncthreads();
}

// 16^3 stencil phases: thread t owns the 4 consecutive x points 4t .. 4t+3
// (a quarter of an x row), so its own points and the y and z neighbour
// segments come with one 16-byte LDS access each, and only the two x
// neighbours beyond the segment are single loads: 7 LDS reads for 4 points
// instead of 28.  Same expression as Mx_at, point by point.
template <typename T>
__device__ __forceinline__ void seg4(T (&v)[4], const T* p) {
    if constexpr (sizeof(T) == 4) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
}
template <typename T>
__device__ __forceinline__ void put4(T* p, const T (&v)[4]) {
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
        *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
    }
}
// M u at the 4 points i0 .. i0+3 of a 16^3 level (i0 a multiple of 4); c = u there
template <typename T>
__device__ __forceinline__ void Mx16_seg(const T* u, int i0, T ih2, T (&c)[4], T (&Mx)[4]) {
    constexpr int N = 16, P = N * N * N, mx = N - 1, my = (N - 1) * N, pz = N * N;
    T ym[4], yp[4], zm[4], zp[4];
    seg4<T>(c, u + i0);
    seg4<T>(ym, u + ((i0 & ~my) | ((i0 - N) & my)));
    seg4<T>(yp, u + ((i0 & ~my) | ((i0 + N) & my)));
    seg4<T>(zm, u + ((i0 - pz) & (P - 1)));
    seg4<T>(zp, u + ((i0 + pz) & (P - 1)));
    const T lft = u[(i0 & ~mx) | ((i0 - 1) & mx)];
    const T rgt = u[(i0 & ~mx) | ((i0 + 4) & mx)];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const T l = e > 0 ? c[e - 1] : lft;
        const T r = e < 3 ? c[e + 1] : rgt;
        T s = l + r;
        s += ym[e] + yp[e];
        s += zm[e] + zp[e];
        Mx[e] = (s - T(6) * c[e]) * ih2;
    }
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

// One smoothing pass on tail level l of N^3 points (same buffer rotation as
// the multi-kernel path).
template <typename T, int N>
__device__ int smooth_pass(const TailArgs<T>& A, const Fields<T>& F, int l, int cur, bool from_zero) {
    constexpr int P = Geo<N>::P;
    const T ih2 = (T)A.ih2[l];
    const T dinv = T(1) / (T(-6) * ih2);
    const T* b = F.b(l);
    int prev = -1;
    for (int k = 0; k < A.sched.steps; ++k) {
        const T a = (T)A.sched.a[l][k], c = (T)A.sched.c[l][k];
        if (k == 0 && from_zero) {
            phase<T, P>([&](int i) { return c * dinv * b[i]; }, F.x(l, 0));
            cur = 0;
            prev = -1;
        } else {
            const bool use_prev = A.sched.cheb && prev >= 0;
            const int o = use_prev ? prev : 1 - cur;
            const T* xc = F.x(l, cur);
            const T* xp = use_prev ? F.x(l, prev) : nullptr;
            if constexpr (N == 16 && P == 4 * kTailThreads) {
                const int i0 = 4 * threadIdx.x;
                T xi[4], Mx[4], bb[4], pv[4] = {T(0), T(0), T(0), T(0)}, v[4];
                Mx16_seg<T>(xc, i0, ih2, xi, Mx);
                seg4<T>(bb, b + i0);
                if (use_prev) seg4<T>(pv, xp + i0);
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = xi[e] + a * (xi[e] - pv[e]) + c * dinv * (bb[e] - Mx[e]);
                put4<T>(F.x(l, o) + i0, v);
                __syncthreads();
            } else {
                phase<T, P>([&](int i) {
                    const T Mx = Mx_at<T, N>(xc, i, ih2);
                    const T xi = xc[i];
                    const T pv = use_prev ? xp[i] : T(0);
                    return xi + a * (xi - pv) + c * dinv * (b[i] - Mx);
                }, F.x(l, o));
            }
            prev = cur;
            cur = o;
        }
    }
    return cur;
}

// Down leg on level l (N^3 points): smoothing from zero, residual into the
// free buffer, full weighting into the coarse right-hand side.  Returns the
// buffer holding the smoothed iterate.
template <typename T, int N>
__device__ int down_level(const TailArgs<T>& A, const Fields<T>& F, int l) {
    using G = Geo<N>;
    using Gc = Geo<N / 2>;
    const T ih2 = (T)A.ih2[l];
    const int cl = smooth_pass<T, N>(A, F, l, 0, true);
    T* r = F.x(l, 1 - cl);
    const T* xc = F.x(l, cl);
    const T* b = F.b(l);
    if constexpr (N == 16 && G::P == 4 * kTailThreads) {
        const int i0 = 4 * threadIdx.x;
        T xi[4], Mx[4], bb[4], v[4];
        Mx16_seg<T>(xc, i0, ih2, xi, Mx);
        seg4<T>(bb, b + i0);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = bb[e] - Mx[e];
        put4<T>(r + i0, v);
        __syncthreads();
    } else {
        phase<T, G::P>([&](int i) { return b[i] - Mx_at<T, N>(xc, i, ih2); }, r);
    }
    phase<T, Gc::P>([&](int i) {
        int X, Y, Z;
        Gc::coords(i, X, Y, Z);
        T acc = T(0);
        for (int dz = -1; dz <= 1; ++dz) {
            T ay = T(0);
            for (int dy = -1; dy <= 1; ++dy) {
                const int fy = 2 * Y + dy, fz = 2 * Z + dz;
                const T ax = T(0.25) * r[G::at(2 * X - 1, fy, fz)] + T(0.5) * r[G::at(2 * X, fy, fz)] +
                             T(0.25) * r[G::at(2 * X + 1, fy, fz)];
                ay += (dy == 0 ? T(0.5) : T(0.25)) * ax;
            }
            acc += (dz == 0 ? T(0.5) : T(0.25)) * ay;
        }
        return acc;
    }, F.b(l + 1));
    return cl;
}

// Up leg on level l (N^3 points): x += P e, then post-smoothing.  Returns the
// buffer holding the result.
template <typename T, int N>
__device__ int up_level(const TailArgs<T>& A, const Fields<T>& F, int l, int cl, const T* e) {
    using G = Geo<N>;
    using Gc = Geo<N / 2>;
    T* xv = F.x(l, cl);
    phase<T, G::P>([&](int i) {
        int x, y, z;
        G::coords(i, x, y, z);
        const int X = x >> 1, Y = y >> 1, Z = z >> 1, ox = x & 1, oy = y & 1, oz = z & 1;
        const T w = (ox ? T(0.5) : T(1)) * (oy ? T(0.5) : T(1)) * (oz ? T(0.5) : T(1));
        T v = T(0);
        for (int kz = 0; kz <= oz; ++kz)
            for (int ky = 0; ky <= oy; ++ky)
                for (int kx = 0; kx <= ox; ++kx) v += w * e[Gc::at(X + kx, Y + ky, Z + kz)];
        return xv[i] + v;
    }, xv);
    return smooth_pass<T, N>(A, F, l, cl, false);
}

// Exact zero-mean solve on the coarsest level (NC^3 points) in double with the
// separable basis: three forward passes, the division by the eigenvalue sums,
// three backward passes.  The basis q and eigenvalues lam are in LDS.
template <typename T, int NC>
__device__ void coarsest(const T* bl, T* xl, double* sA, double* sB, const double* q, const double* lam) {
    constexpr int N = NC * NC * NC;
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += kTailThreads) sA[i] = (double)bl[i];
    __syncthreads();
    auto pass = [&](const double* src, double* dst, int axis, bool forward) {
        for (int i = tid; i < N; i += kTailThreads) {
            const int x = i % NC, y = (i / NC) % NC, z = i / (NC * NC);
            const int k = axis == 0 ? x : axis == 1 ? y : z;
            const int stride = axis == 0 ? 1 : axis == 1 ? NC : NC * NC;
            const int base = i - k * stride;
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) acc += (forward ? q[j + NC * k] : q[k + NC * j]) * src[base + j * stride];
            dst[i] = acc;
        }
        __syncthreads();
    };
    pass(sA, sB, 0, true);
    pass(sB, sA, 1, true);
    pass(sA, sB, 2, true);
    for (int i = tid; i < N; i += kTailThreads) {
        const int x = i % NC, y = (i / NC) % NC, z = i / (NC * NC);
        sB[i] = (x == 0 && y == 0 && z == 0) ? 0.0 : sB[i] / (lam[x] + lam[y] + lam[z]);
    }
    __syncthreads();
    pass(sB, sA, 2, false);
    pass(sA, sB, 1, false);
    pass(sB, sA, 0, false);
    for (int i = tid; i < N; i += kTailThreads) xl[i] = (T)sA[i];
    __syncthreads();
}

// The same solve on a 4^3 coarsest level by one wave: lane i owns point
// i = x + 4 y + 16 z and takes the other points of its line from their lanes
// by cross-lane moves, so the six passes need no workgroup barrier.  Same
// sums in the same order as the workgroup version.
template <typename T>
__device__ void coarsest4(const T* bl, T* xl, const double* q, const double* lam) {
    constexpr int NC = 4;
    if (threadIdx.x < 64) {
        const int i = threadIdx.x, x = i & 3, y = (i >> 2) & 3, z = i >> 4;
        auto pass = [&](double u, int axis, bool forward) {
            const int k = axis == 0 ? x : axis == 1 ? y : z;
            const int stride = axis == 0 ? 1 : axis == 1 ? NC : NC * NC;
            const int base = i - k * stride;
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j)
                acc += (forward ? q[j + NC * k] : q[k + NC * j]) * __shfl(u, base + j * stride, 64);
            return acc;
        };
        double v = (double)bl[i];
        v = pass(v, 0, true);
        v = pass(v, 1, true);
        v = pass(v, 2, true);
        v = (x == 0 && y == 0 && z == 0) ? 0.0 : v / (lam[x] + lam[y] + lam[z]);
        v = pass(v, 2, false);
        v = pass(v, 1, false);
        v = pass(v, 0, false);
        xl[i] = (T)v;
    }
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailArgs<T> A) {
    __shared__ __align__(16) T fields[kTailElems];
    __shared__ double sA[512];
    __shared__ double sB[512];
    __shared__ double q[64];
    __shared__ double lam[8];
    const Fields<T> F{fields, &A};
    unsigned curbits = 0;  // bit l: buffer holding level l's iterate (no private array)
    const int nl = A.nlev;
    const int tid = threadIdx.x;
    const int ncst = A.n[nl - 1];
    {   // right-hand side of the first tail level and the coarsest basis from
        // global memory, all loads in flight together
        const int N0 = A.n[0] * A.n[0] * A.n[0];
        T* b0 = F.b(0);
        for (int i = tid; i < N0; i += kTailThreads) b0[i] = A.b[0][i];
        if (tid < ncst * ncst) q[tid] = A.Q[tid];
        if (tid < ncst) lam[tid] = A.lam1[tid];
        __syncthreads();
    }
    // ---------------- down leg
    for (int l = 0; l + 1 < nl; ++l) {
        const int cl = A.n[l] == 16 ? down_level<T, 16>(A, F, l) : down_level<T, 8>(A, F, l);
        curbits = (curbits & ~(1u << l)) | ((unsigned)cl << l);
    }
    // ---------------- coarsest: exact zero-mean solve in double (separable basis)
    {
        const int l = nl - 1;
        if (ncst == 8) coarsest<T, 8>(F.b(l), F.x(l, 0), sA, sB, q, lam);
        else coarsest4<T>(F.b(l), F.x(l, 0), q, lam);
        curbits &= ~(1u << l);
    }
    // ---------------- up leg
    for (int l = nl - 2; l >= 0; --l) {
        const T* e = F.x(l + 1, (curbits >> (l + 1)) & 1);
        const int cl = (curbits >> l) & 1;
        const int cn = A.n[l] == 16 ? up_level<T, 16>(A, F, l, cl, e) : up_level<T, 8>(A, F, l, cl, e);
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
    // levels of 16^3 or 8^3 points down to a coarsest of 8^3 or 4^3, halving each time
    if (args.nlev < 2 || args.nlev > kTailMaxLevels) return hipErrorInvalidValue;
    for (int l = 0; l < args.nlev; ++l) {
        const int nl = args.n[l];
        const bool coarsest = l == args.nlev - 1;
        if (coarsest ? (nl != 8 && nl != 4) : (nl != 16 && nl != 8)) return hipErrorInvalidValue;
        if (l > 0 && nl * 2 != args.n[l - 1]) return hipErrorInvalidValue;
    }
    int elems = 0;
    for (int l = 0; l < args.nlev; ++l) elems += 3 * args.n[l] * args.n[l] * args.n[l];
    if (elems > kTailElems) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_tail<T>), dim3(1), dim3(kTailThreads), 0, s, args);
    return hipGetLastError();
}

template hipError_t launch_tail<float>(const TailArgs<float>&, hipStream_t);
template hipError_t launch_tail<double>(const TailArgs<double>&, hipStream_t);

}  // namespace mg
