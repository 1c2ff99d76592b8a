// Seven-point "row-wave" kernels for levels with 64 <= n <= 1024.
//
// One wavefront owns one whole x-row of the level: lane l holds the VEC = n/64
// contiguous elements [l*VEC, (l+1)*VEC) and moves them with 16-byte vector
// loads/stores, so a wave reads or writes n*sizeof(T) contiguous bytes per
// row.  Because the wave spans the full periodic row, the x-neighbours of a
// lane's first and last element come from the neighbouring lanes by rotating
// cross-lane moves (the wrap-around included) and no x-halo is ever loaded.
// The y-neighbour rows are the rows of the adjacent waves (served by L1/L2),
// and z-neighbours come from a register queue as the wave marches a chunk of
// planes.  Blocks of four
// waves are renumbered so that consecutive row blocks land on the same XCD
// and share their halo rows through that XCD's L2.
#include <type_traits>

#include "flat_row.h"

#include "fma.h"
#include "launch.h"
#include "row.h"
#include "sums.h"

#include <cstdint>
#include <type_traits>

namespace mg {
namespace {

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;

// Element i (0 <= i < 64 VEC) of a row copy written by lds_strow.
template <typename T, int VEC>
__device__ __forceinline__ T lds_elem(const T* row, int i) {
    constexpr int B = VEC * (int)sizeof(T);
    if constexpr (B <= 16) {
        return row[i];
    } else {
        constexpr int P = 16 / (int)sizeof(T);
        const int l = i / VEC, e = i - l * VEC;
        return row[((e / P) * 64 + l) * P + e % P];
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void copyrow(T (&d)[VEC], const T (&s)[VEC]) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) d[e] = s[e];
}

// M x on one row: c = centre row, ym/yp = rows y-1/y+1, zm/zp = planes z-1/z+1.
// The rounding of the stencil and of the smoothing step below is written out
// (no contraction left to the compiler), so every kernel that applies a step
// -- single or fused -- produces the same bits.
template <typename T, int VEC>
__device__ __forceinline__ void flat7_row(const T (&c)[VEC], const T (&ym)[VEC], const T (&yp)[VEC],
                                          const T (&zm)[VEC], const T (&zp)[VEC], T ih2, T (&Mx)[VEC]) {
#pragma clang fp contract(off)
    const T lft = lane_rot(c[VEC - 1], -1);
    const T rgt = lane_rot(c[0], 1);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const T l = e > 0 ? c[e - 1] : lft;
        const T r = e < VEC - 1 ? c[e + 1] : rgt;
        const T s = ((l + r) + (ym[e] + yp[e])) + (zm[e] + zp[e]);
        Mx[e] = fma_rn(T(-6), c[e], s) * ih2;
    }
}

// flat7_row for a row split into segments held by several waves: the
// x-neighbours beyond the segment (lane 0's left, lane 63's right) are the
// lane's halo value hx instead of the wrapped-around lanes of its own wave.
// Same arithmetic as flat7_row.
template <typename T, int VEC, int S>
__device__ __forceinline__ void flat7_row_seg(const T (&c)[VEC], const T (&ym)[VEC], const T (&yp)[VEC],
                                              const T (&zm)[VEC], const T (&zp)[VEC], T ih2, T (&Mx)[VEC], T hx) {
#pragma clang fp contract(off)
    T lft = lane_rot(c[VEC - 1], -1);
    T rgt = lane_rot(c[0], 1);
    if constexpr (S > 1) {
        const int lane = threadIdx.x & 63;
        if (lane == 0) lft = hx;
        if (lane == 63) rgt = hx;
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const T l = e > 0 ? c[e - 1] : lft;
        const T r = e < VEC - 1 ? c[e + 1] : rgt;
        const T s = ((l + r) + (ym[e] + yp[e])) + (zm[e] + zp[e]);
        Mx[e] = fma_rn(T(-6), c[e], s) * ih2;
    }
}

// Element of a full row (length S * 64 * VEC) that lane `lane` of the wave
// holding segment `seg` needs beyond its segment: the one before the segment
// for the lower half of the wave (lane 0 uses it), the one after it for the
// upper half (lane 63 uses it).  Periodic in x.
template <int VEC, int S>
__device__ __forceinline__ int seg_halo(int seg, int lane) {
    constexpr int NR = 64 * VEC, NF = NR * S;
    return lane < 32 ? (seg * NR - 1) & (NF - 1) : ((seg + 1) * NR) & (NF - 1);
}

// The coarse rows the trilinear prolongation of fine row (y, z) reads (VEC >= 2):
// (Y, Z), and (Y+1, Z), (Y, Z+1), (Y+1, Z+1) where y, z are odd; loaded raw so
// that a prefetch is not waited for until the values are combined.
// VEC == 1 (64^3): lane l holds fine x = l, i.e. coarse X = l / 2, and reads
// the coarse values X and X + 1 of each row itself.
template <typename T, int VEC>
struct CoarseRows {
    T t00[VEC / 2], t01[VEC / 2], t10[VEC / 2], t11[VEC / 2];
};
template <typename T>
struct CoarseRows<T, 1> {
    T a, a1, b0, b1, c0, c1, d0, d1;  // rows (Y, Z), (Y+1, Z), (Y, Z+1), (Y+1, Z+1) at X, X + 1
};
template <typename T, int VEC>
__device__ __forceinline__ void coarse_load(CoarseRows<T, VEC>& c, const T* e, const RowGrid& gc, int y, int z,
                                            int lane) {
    const int Y = y >> 1, Z = z >> 1, oy = y & 1, oz = z & 1;
    if constexpr (VEC == 1) {
        const int X = lane >> 1, ox = lane & 1, m = gc.mask;
        const T* r0 = e + gc.row(Y, Z);
        c.a = r0[X & m];
        if (ox) c.a1 = r0[(X + 1) & m];
        if (oy) {
            const T* r1 = e + gc.row(Y + 1, Z);
            c.b0 = r1[X & m];
            if (ox) c.b1 = r1[(X + 1) & m];
        }
        if (oz) {
            const T* r2 = e + gc.row(Y, Z + 1);
            c.c0 = r2[X & m];
            if (ox) c.c1 = r2[(X + 1) & m];
            if (oy) {
                const T* r3 = e + gc.row(Y + 1, Z + 1);
                c.d0 = r3[X & m];
                if (ox) c.d1 = r3[(X + 1) & m];
            }
        }
    } else {
        constexpr int CV = VEC / 2;
        const size_t off = (size_t)lane * CV;
        ldrow<T, CV>(c.t00, e + gc.row(Y, Z) + off);
        if (oy) ldrow<T, CV>(c.t01, e + gc.row(Y + 1, Z) + off);
        if (oz) ldrow<T, CV>(c.t10, e + gc.row(Y, Z + 1) + off);
        if (oy && oz) ldrow<T, CV>(c.t11, e + gc.row(Y + 1, Z + 1) + off);
    }
}
// xv += P e on fine row (y, z): interpolate in y, then z, then x (the x + 1
// coarse value from the next lane).  Rounding written out: every kernel that
// prolongs (the prolongation kernel, the fused post-smoothing pass) gets the
// same bits.
template <typename T, int VEC>
__device__ __forceinline__ void prolong_add(T (&xv)[VEC], const CoarseRows<T, VEC>& c, int y, int z) {
#pragma clang fp contract(off)
    const int oy = y & 1, oz = z & 1;
    if constexpr (VEC == 1) {  // interpolate in x, then y, then z
        const int ox = threadIdx.x & 1;
        T v = ox ? T(0.5) * (c.a + c.a1) : c.a;
        if (oy) v = T(0.5) * (v + (ox ? T(0.5) * (c.b0 + c.b1) : c.b0));
        if (oz) {
            T u = ox ? T(0.5) * (c.c0 + c.c1) : c.c0;
            if (oy) u = T(0.5) * (u + (ox ? T(0.5) * (c.d0 + c.d1) : c.d0));
            v = T(0.5) * (v + u);
        }
        xv[0] = xv[0] + v;
    } else {
        constexpr int CV = VEC / 2, CW = CV + 1;
        T w[CW];
        auto seg = [&](const T (&t)[CV], int q) { return q < CV ? t[q] : lane_rot(t[0], 1); };
#pragma unroll
        for (int q = 0; q < CW; ++q) {
            const T r00 = seg(c.t00, q);
            T a0 = r00;
            if (oy) a0 = T(0.5) * (r00 + seg(c.t01, q));
            if (oz) {
                const T r10 = seg(c.t10, q);
                const T a1 = oy ? T(0.5) * (r10 + seg(c.t11, q)) : r10;
                a0 = T(0.5) * (a0 + a1);
            }
            w[q] = a0;
        }
#pragma unroll
        for (int q = 0; q < CV; ++q) {
            xv[2 * q] = xv[2 * q] + w[q];
            xv[2 * q + 1] = xv[2 * q + 1] + T(0.5) * (w[q] + w[q + 1]);
        }
    }
}

// The coarse rows of fine row (y, z) for a row split into S segments of
// 64 VEC points, one per wave (VEC >= 2): the segment's VEC / 2 coarse values
// per lane of each row, and the first coarse value after the segment
// (periodic), which lane 63 needs where an unsplit row takes it from the
// next lane.
template <typename T, int VEC>
struct CoarseSeg {
    CoarseRows<T, VEC> r;
    T h00, h01, h10, h11;
};
template <typename T, int VEC>
__device__ __forceinline__ void coarse_load_seg(CoarseSeg<T, VEC>& c, const T* e, const RowGrid& gc, int y, int z,
                                                int seg, int lane) {
    constexpr int CV = VEC / 2, NC = 32 * VEC;  // coarse values per lane and per segment
    const int Y = y >> 1, Z = z >> 1, oy = y & 1, oz = z & 1;
    const size_t off = (size_t)seg * NC + (size_t)lane * CV;
    const int hx = ((seg + 1) * NC) & gc.mask;
    const T* r0 = e + gc.row(Y, Z);
    ldrow<T, CV>(c.r.t00, r0 + off);
    c.h00 = r0[hx];
    if (oy) {
        const T* r1 = e + gc.row(Y + 1, Z);
        ldrow<T, CV>(c.r.t01, r1 + off);
        c.h01 = r1[hx];
    }
    if (oz) {
        const T* r2 = e + gc.row(Y, Z + 1);
        ldrow<T, CV>(c.r.t10, r2 + off);
        c.h10 = r2[hx];
    }
    if (oy && oz) {
        const T* r3 = e + gc.row(Y + 1, Z + 1);
        ldrow<T, CV>(c.r.t11, r3 + off);
        c.h11 = r3[hx];
    }
}
// prolong_add for a segment: the same interpolation and rounding, with lane
// 63's coarse value after the segment taken from the halo.
template <typename T, int VEC>
__device__ __forceinline__ void prolong_add_seg(T (&xv)[VEC], const CoarseSeg<T, VEC>& c, int y, int z) {
#pragma clang fp contract(off)
    static_assert(VEC >= 2, "two fine points per lane at least");
    const int oy = y & 1, oz = z & 1;
    const bool last = (threadIdx.x & 63) == 63;
    constexpr int CV = VEC / 2, CW = CV + 1;
    T w[CW];
    auto seg = [&](const T (&t)[CV], T h, int q) {
        if (q < CV) return t[q];
        const T r = lane_rot(t[0], 1);
        return last ? h : r;
    };
#pragma unroll
    for (int q = 0; q < CW; ++q) {
        const T r00 = seg(c.r.t00, c.h00, q);
        T a0 = r00;
        if (oy) a0 = T(0.5) * (r00 + seg(c.r.t01, c.h01, q));
        if (oz) {
            const T r10 = seg(c.r.t10, c.h10, q);
            const T a1 = oy ? T(0.5) * (r10 + seg(c.r.t11, c.h11, q)) : r10;
            a0 = T(0.5) * (a0 + a1);
        }
        w[q] = a0;
    }
#pragma unroll
    for (int q = 0; q < CV; ++q) {
        xv[2 * q] = xv[2 * q] + w[q];
        xv[2 * q + 1] = xv[2 * q + 1] + T(0.5) * (w[q] + w[q + 1]);
    }
}

// One smoothing step at a point: x + a (x - xp) + cd (b - M x).
template <typename T>
__device__ __forceinline__ T cheb_step(T x, T xp, T b, T Mx, T a, T cd) {
#pragma clang fp contract(off)
    return fma_rn(cd, b - Mx, fma_rn(a, x - xp, x));
}

// The pointwise first step of a pass from zero, x = cd0 r (cd0 = c0 / D),
// formed in T; with FROMB false, r itself.
template <typename T, bool FROMB>
__device__ __forceinline__ T first_step(T r, T cd0) {
    if constexpr (FROMB) return cd0 * r;
    return r;
}

// =====================================================================================
// Chebyshev / Jacobi step: out = x + a (x - xprev) + cd (b - M x), cd = c / D
// =====================================================================================
// S > 1: each row split into S segments of 64 VEC elements, one per wave (a
// block of kWaves waves holds kWaves / S rows), so that rows of several KB
// keep a modest number of values per lane; the x-neighbours across segment
// ends come from one halo element loaded with each centre row.
// FROMB: the second step of a pass from zero, read from b alone: x holds the b
// rows, the iterate is the pointwise first step cd0 b formed from them, and
// x_prev = 0.  PREVB: the third step of such a pass, whose x_prev is that
// pointwise first step, formed from the b row instead of being read.
template <typename T, int VEC, bool HASX, bool PREV, int S = 1, bool FROMB = false, bool PREVB = false>
__global__ __launch_bounds__(kBlock) void k_smooth_row(int n, T ih2, const T* x, const T* xprev,
                                                       const T* __restrict__ b, T* out, T a, T cd, int nz,
                                                       int nyb, T cd0) {
    static_assert(kWaves % S == 0, "a block holds whole rows");
    static_assert(!FROMB || (HASX && !PREV), "a step from b has no x_prev");
    static_assert(!PREVB || (HASX && PREV && !FROMB), "PREVB forms x_prev from b");
    constexpr bool LDP = PREV && !PREVB;  // x_prev is loaded
    constexpr int NR = 64 * VEC;
    const RowGrid g{NR * S, NR * S - 1};
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int w = wave_id();
    const int y = yb * (kWaves / S) + w / S, seg = w % S;
    const int z0 = zc * nz;
    const int lane = threadIdx.x & 63;
    const size_t off = (size_t)seg * NR + (size_t)lane * VEC;
    const int hoff = S > 1 ? seg_halo<VEC, S>(seg, lane) : 0;
    if constexpr (!HASX) {
        for (int k = 0; k < nz; ++k) {
            const size_t r = g.row(y, z0 + k) + off;
            T bb[VEC], o[VEC];
            ldrow<T, VEC>(bb, b + r);
#pragma unroll
            for (int e = 0; e < VEC; ++e) o[e] = cd * bb[e];  // x = 0: the step is cd b
            strow<T, VEC>(out + r, o);
        }
        return;
    } else {
        T zm[VEC], c[VEC], zp[VEC], ym[VEC], yp[VEC], bb[VEC], pp[VEC];
        T hc = T(0), hp = T(0);  // x-halo of c and zp (S > 1)
        ldrow<T, VEC>(zm, x + g.row(y, z0 - 1) + off);
        ldrow<T, VEC>(c, x + g.row(y, z0) + off);
        ldrow<T, VEC>(zp, x + g.row(y, z0 + 1) + off);
        if constexpr (S > 1) {
            hc = x[g.row(y, z0) + hoff];
            hp = x[g.row(y, z0 + 1) + hoff];
        }
        ldrow<T, VEC>(ym, x + g.row(y - 1, z0) + off);
        ldrow<T, VEC>(yp, x + g.row(y + 1, z0) + off);
        if constexpr (!FROMB) ldrow<T, VEC>(bb, b + g.row(y, z0) + off);
        if constexpr (LDP) ldrow<T, VEC>(pp, xprev + g.row(y, z0) + off);
        for (int k = 0; k < nz; ++k) {
            const int z = z0 + k;
            // prefetch the next plane's operands before any store of this plane
            T zpp[VEC], ymn[VEC], ypn[VEC], bn[VEC], pn[VEC];
            T hpp = T(0);
            const bool more = k + 1 < nz;
            if (more) {
                ldrow<T, VEC>(zpp, x + g.row(y, z + 2) + off);
                if constexpr (S > 1) hpp = x[g.row(y, z + 2) + hoff];
                ldrow<T, VEC>(ymn, x + g.row(y - 1, z + 1) + off);
                ldrow<T, VEC>(ypn, x + g.row(y + 1, z + 1) + off);
                if constexpr (!FROMB) ldrow<T, VEC>(bn, b + g.row(y, z + 1) + off);
                if constexpr (LDP) ldrow<T, VEC>(pn, xprev + g.row(y, z + 1) + off);
            }
            T Mx[VEC], o[VEC];
            if constexpr (FROMB) {  // x = cd0 b on the row and its neighbours; b = the raw centre row
                T fc[VEC], fym[VEC], fyp[VEC], fzm[VEC], fzp[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    fc[e] = first_step<T, true>(c[e], cd0);
                    fym[e] = first_step<T, true>(ym[e], cd0);
                    fyp[e] = first_step<T, true>(yp[e], cd0);
                    fzm[e] = first_step<T, true>(zm[e], cd0);
                    fzp[e] = first_step<T, true>(zp[e], cd0);
                }
                flat7_row_seg<T, VEC, S>(fc, fym, fyp, fzm, fzp, ih2, Mx, first_step<T, true>(hc, cd0));
#pragma unroll
                for (int e = 0; e < VEC; ++e) o[e] = cheb_step<T>(fc[e], T(0), c[e], Mx[e], a, cd);
            } else {
                flat7_row_seg<T, VEC, S>(c, ym, yp, zm, zp, ih2, Mx, hc);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const T xpe = PREVB ? first_step<T, true>(bb[e], cd0) : PREV ? pp[e] : T(0);
                    o[e] = cheb_step<T>(c[e], xpe, bb[e], Mx[e], a, cd);
                }
            }
            strow<T, VEC>(out + g.row(y, z) + off, o);
            if (more) {
                copyrow(zm, c);
                copyrow(c, zp);
                copyrow(zp, zpp);
                hc = hp;
                hp = hpp;
                copyrow(ym, ymn);
                copyrow(yp, ypn);
                if constexpr (!FROMB) copyrow(bb, bn);
                if constexpr (LDP) copyrow(pp, pn);
            }
        }
    }
}

// =====================================================================================
// Outer defect correction: value = phi_in (+ e); r = (b - bmean) - M value
// =====================================================================================
template <typename TA, typename TR, typename TE, int VEC, bool UPDATE>
__device__ __forceinline__ void ld_value(TA (&v)[VEC], const double* phi, const TE* e, size_t r) {
    double p[VEC];
    ldrow<double, VEC>(p, phi + r);
    if constexpr (UPDATE) {
        TE q[VEC];
        ldrow<TE, VEC>(q, e + r);
#pragma unroll
        for (int k = 0; k < VEC; ++k) v[k] = (TA)(p[k] + (double)q[k]);
    } else {
#pragma unroll
        for (int k = 0; k < VEC; ++k) v[k] = (TA)p[k];
    }
}

// Per-block partial sums of the outer kernels, three arrays of gridDim.x:
// [0] sum (b - bmean)^2, [1] sum r^2, [2] sum phi (phi = the potential whose
// residual is formed, in double).
__device__ __forceinline__ void outer_partials(double* partials, double sb, double ss, double sp, double* sh,
                                               int waves) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        sb += __shfl_xor(sb, o, 64);
        ss += __shfl_xor(ss, o, 64);
        sp += __shfl_xor(sp, o, 64);
    }
    if (lane == 0) {
        sh[wave] = sb;
        sh[waves + wave] = ss;
        sh[2 * waves + wave] = sp;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int q = 0; q < waves; ++q) t += sh[threadIdx.x * waves + q];
        partials[threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// The potential (phi, or phi + e) at one element as TA: the x-halo of a split row.
template <typename TA, typename TE, bool UPDATE>
__device__ __forceinline__ TA ld_value1(const double* phi, const TE* e, size_t i) {
    if constexpr (UPDATE) return (TA)(phi[i] + (double)e[i]);
    return (TA)phi[i];
}

// S > 1: rows split into S segments, one per wave, as in k_smooth_row.
template <typename TA, typename TR, typename TE, int VEC, bool UPDATE, int S = 1>
__global__ __launch_bounds__(kBlock) void k_outer_row(int n, TA ih2, const double* __restrict__ phi_in,
                                                      const TE* __restrict__ e, double* __restrict__ phi_out,
                                                      const double* __restrict__ b, double bmean,
                                                      TR* __restrict__ r, TR* __restrict__ x1, TA cd0,
                                                      double* __restrict__ partials, int nz, int nyb) {
    static_assert(kWaves % S == 0, "a block holds whole rows");
    __shared__ double sh[3 * kWaves];
    constexpr int NR = 64 * VEC;
    const RowGrid g{NR * S, NR * S - 1};
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int wave = wave_id();
    const int y = yb * (kWaves / S) + wave / S, seg = wave % S;
    const int z0 = zc * nz;
    const int lane = threadIdx.x & 63;
    const size_t off = (size_t)seg * NR + (size_t)lane * VEC;
    const int hoff = S > 1 ? seg_halo<VEC, S>(seg, lane) : 0;
    TA zm[VEC], c[VEC], zp[VEC], ym[VEC], yp[VEC];
    TA hc = TA(0), hp = TA(0);  // x-halo of c and zp (S > 1)
    double bb[VEC];
    ld_value<TA, TR, TE, VEC, UPDATE>(zm, phi_in, e, g.row(y, z0 - 1) + off);
    ld_value<TA, TR, TE, VEC, UPDATE>(c, phi_in, e, g.row(y, z0) + off);
    ld_value<TA, TR, TE, VEC, UPDATE>(zp, phi_in, e, g.row(y, z0 + 1) + off);
    if constexpr (S > 1) {
        hc = ld_value1<TA, TE, UPDATE>(phi_in, e, g.row(y, z0) + hoff);
        hp = ld_value1<TA, TE, UPDATE>(phi_in, e, g.row(y, z0 + 1) + hoff);
    }
    ld_value<TA, TR, TE, VEC, UPDATE>(ym, phi_in, e, g.row(y - 1, z0) + off);
    ld_value<TA, TR, TE, VEC, UPDATE>(yp, phi_in, e, g.row(y + 1, z0) + off);
    ldrow<double, VEC>(bb, b + g.row(y, z0) + off);
    double ss = 0.0, sb = 0.0, sp = 0.0;
    for (int k = 0; k < nz; ++k) {
        const int z = z0 + k;
        TA zpp[VEC], ymn[VEC], ypn[VEC];
        TA hpp = TA(0);
        double bn[VEC];
        const bool more = k + 1 < nz;
        if (more) {
            ld_value<TA, TR, TE, VEC, UPDATE>(zpp, phi_in, e, g.row(y, z + 2) + off);
            if constexpr (S > 1) hpp = ld_value1<TA, TE, UPDATE>(phi_in, e, g.row(y, z + 2) + hoff);
            ld_value<TA, TR, TE, VEC, UPDATE>(ymn, phi_in, e, g.row(y - 1, z + 1) + off);
            ld_value<TA, TR, TE, VEC, UPDATE>(ypn, phi_in, e, g.row(y + 1, z + 1) + off);
            ldrow<double, VEC>(bn, b + g.row(y, z + 1) + off);
        }
        TA Mx[VEC];
        TR ro[VEC];
        flat7_row_seg<TA, VEC, S>(c, ym, yp, zm, zp, ih2, Mx, hc);
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            const double bq = bb[q] - bmean;
            const TA ri = (TA)bq - Mx[q];
            ro[q] = (TR)ri;
            ss += (double)ri * (double)ri;
            sb += bq * bq;
        }
        const size_t row = g.row(y, z) + off;
        strow<TR, VEC>(r + row, ro);
        if (x1) {
            TR xo[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) xo[q] = (TR)cd0 * ro[q];  // in the iterate's precision, as the first step from zero
            strow<TR, VEC>(x1 + row, xo);
        }
        if constexpr (UPDATE) {
            double po[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) po[q] = (double)c[q];
            // phi_out keeps the double sum phi + e (c holds it rounded to TA)
            if constexpr (sizeof(TA) != sizeof(double)) {
                double p[VEC];
                TE qv[VEC];
                ldrow<double, VEC>(p, phi_in + row);
                ldrow<TE, VEC>(qv, e + row);
#pragma unroll
                for (int q = 0; q < VEC; ++q) po[q] = p[q] + (double)qv[q];
            }
            strow<double, VEC>(phi_out + row, po);
#pragma unroll
            for (int q = 0; q < VEC; ++q) sp += po[q];
        } else if constexpr (sizeof(TA) == sizeof(double)) {
#pragma unroll
            for (int q = 0; q < VEC; ++q) sp += (double)c[q];
        } else {
            double p[VEC];
            ldrow<double, VEC>(p, phi_in + row);
#pragma unroll
            for (int q = 0; q < VEC; ++q) sp += p[q];
        }
        if (more) {
            copyrow(zm, c);
            copyrow(c, zp);
            copyrow(zp, zpp);
            hc = hp;
            hp = hpp;
            copyrow(ym, ymn);
            copyrow(yp, ypn);
            copyrow(bb, bn);
        }
    }
    // fixed-order block reduction: wave butterfly, then the wave sums in order
    outer_partials(partials, sb, ss, sp, sh, kWaves);
}

// =====================================================================================
// LDS row-sharing variants: a block of W waves owns W consecutive rows; each
// plane's rows (plus the two block-halo rows, loaded by the edge waves) are
// published in LDS (double-buffered by plane parity, one barrier per plane),
// so the y-neighbour rows come from LDS instead of L2/HBM.  Used where the
// 2 (W + 2) rows fit in 80 KB of LDS.
// =====================================================================================
// S > 1: W rows of S segments each (one wave per segment), for rows whose
// unsplit queues would not fit a wave's registers; each segment keeps its
// slice of the LDS rows, and the x-neighbours across segment ends come from
// one halo element loaded with each centre row, as in k_smooth_row.
// PRO: the first step of a post-smoothing pass from x0 = x + P e (ec: the
// coarse correction), x_prev = 0; x0 is formed row by row as the rows arrive
// and never written, and the x-halo of a segment comes from its neighbour's
// slot of the LDS row.  PREVP: the second step of that pass, x_prev = x0
// formed pointwise from the old iterate (xprev) and ec.  Both use the
// prolongation of k_prolong_row, same bits.
template <typename T, int VEC, int W, bool PREV, bool FROMB = false, bool PREVB = false, int S = 1, bool PRO = false,
          bool PREVP = false>
__global__ __launch_bounds__(64 * W * S) void k_smooth_lds(int n, T ih2, const T* x, const T* xprev,
                                                           const T* __restrict__ b, T* out, T a, T cd, int nz,
                                                           int nyb, T cd0, const T* __restrict__ ec) {
    static_assert(!(FROMB && PREV), "a step from b has no x_prev");
    static_assert(!PREVB || (PREV && !FROMB), "PREVB forms x_prev from b");
    static_assert(!PRO || (!PREV && !FROMB && VEC >= 2), "the prolongation starts a pass, x_prev = 0");
    static_assert(!PREVP || (PREV && !PREVB && VEC >= 2), "PREVP forms x_prev from x and e");
    constexpr bool LDP = PREV && !PREVB && !PREVP;  // x_prev is loaded as it is
    constexpr int NR = 64 * VEC, NF = NR * S;
    using Coarse = typename std::conditional<(S > 1), CoarseSeg<T, VEC>, CoarseRows<T, VEC>>::type;
    __shared__ T rows[2][W + 2][NF];
    const RowGrid g{NF, NF - 1};
    const RowGrid gc{NF / 2, NF / 2 - 1};  // PRO / PREVP: the coarse grid of ec
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int wv = wave_id();
    const int w = wv / S, seg = wv - w * S;
    const int y0 = yb * W;
    const int y = y0 + w;
    const int z0 = zc * nz;
    const int lane = threadIdx.x & 63;
    const size_t off = (size_t)seg * NR + (size_t)lane * VEC;
    const int hoff = S > 1 ? seg_halo<VEC, S>(seg, lane) : 0;
    const bool lo = w == 0, hi = w == W - 1;
    const int yh = lo ? y0 - 1 : y0 + W;  // halo row of the edge waves
    auto cload = [&](Coarse& cr, int yy, int zz) {
        if constexpr (S > 1) coarse_load_seg<T, VEC>(cr, ec, gc, yy, zz, seg, lane);
        else coarse_load<T, VEC>(cr, ec, gc, yy, zz, lane);
    };
    auto padd = [&](T (&v)[VEC], const Coarse& cr, int yy, int zz) {
        if constexpr (S > 1) prolong_add_seg<T, VEC>(v, cr, yy, zz);
        else prolong_add<T, VEC>(v, cr, yy, zz);
    };
    T zm[VEC], c[VEC], zp[VEC], bb[VEC], pp[VEC], h[VEC];
    T hc = T(0), hp = T(0);  // x-halo of c and zp (S > 1, not PRO)
    ldrow<T, VEC>(zm, x + g.row(y, z0 - 1) + off);
    ldrow<T, VEC>(c, x + g.row(y, z0) + off);
    ldrow<T, VEC>(zp, x + g.row(y, z0 + 1) + off);
    if constexpr (S > 1 && !PRO) {
        hc = x[g.row(y, z0) + hoff];
        hp = x[g.row(y, z0 + 1) + hoff];
    }
    if constexpr (!FROMB) ldrow<T, VEC>(bb, b + g.row(y, z0) + off);
    if constexpr (LDP || PREVP) ldrow<T, VEC>(pp, xprev + g.row(y, z0) + off);
    if (lo || hi) ldrow<T, VEC>(h, x + g.row(yh, z0) + off);
    if constexpr (PRO) {  // x0 = x + P e on the rows loaded so far
        Coarse cr;
        cload(cr, y, z0 - 1);
        padd(zm, cr, y, z0 - 1);
        cload(cr, y, z0);
        padd(c, cr, y, z0);
        cload(cr, y, z0 + 1);
        padd(zp, cr, y, z0 + 1);
        if (lo || hi) {
            cload(cr, yh, z0);
            padd(h, cr, yh, z0);
        }
    }
    if constexpr (PREVP) {
        Coarse cr;
        cload(cr, y, z0);
        padd(pp, cr, y, z0);
    }
    for (int k = 0; k < nz; ++k) {
        const int z = z0 + k;
        const int buf = k & 1;
        T zpp[VEC], bn[VEC], pn[VEC], hn[VEC];
        T hpp = T(0);
        Coarse cpp, chn, cpn;  // PRO: coarse rows of zpp and hn; PREVP: of pn
        const bool more = k + 1 < nz;
        if (more) {
            ldrow<T, VEC>(zpp, x + g.row(y, z + 2) + off);
            if constexpr (S > 1 && !PRO) hpp = x[g.row(y, z + 2) + hoff];
            if constexpr (!FROMB) ldrow<T, VEC>(bn, b + g.row(y, z + 1) + off);
            if constexpr (LDP || PREVP) ldrow<T, VEC>(pn, xprev + g.row(y, z + 1) + off);
            if (lo || hi) ldrow<T, VEC>(hn, x + g.row(yh, z + 1) + off);
            if constexpr (PRO) {
                cload(cpp, y, z + 2);
                if (lo || hi) cload(chn, yh, z + 1);
            }
            if constexpr (PREVP) cload(cpn, y, z + 1);
        }
        lds_strow<T, VEC>(rows[buf][w + 1] + seg * NR, lane, c);
        if (lo) lds_strow<T, VEC>(rows[buf][0] + seg * NR, lane, h);
        if (hi) lds_strow<T, VEC>(rows[buf][W + 1] + seg * NR, lane, h);
        __syncthreads();
        T ym[VEC], yp[VEC];
        lds_ldrow<T, VEC>(ym, rows[buf][w] + seg * NR, lane);
        lds_ldrow<T, VEC>(yp, rows[buf][w + 2] + seg * NR, lane);
        if constexpr (PRO && S > 1) {  // x0 beyond the segment: the neighbour segment's slot
            const T* row = rows[buf][w + 1];
            hc = lane < 32 ? lds_elem<T, VEC>(row + ((seg + S - 1) % S) * NR, NR - 1)
                           : lds_elem<T, VEC>(row + ((seg + 1) % S) * NR, 0);
        }
        T Mx[VEC], o[VEC];
        if constexpr (FROMB) {  // x = cd0 b on the row and its neighbours; b = the raw centre row
            T fc[VEC], fym[VEC], fyp[VEC], fzm[VEC], fzp[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                fc[e] = first_step<T, true>(c[e], cd0);
                fym[e] = first_step<T, true>(ym[e], cd0);
                fyp[e] = first_step<T, true>(yp[e], cd0);
                fzm[e] = first_step<T, true>(zm[e], cd0);
                fzp[e] = first_step<T, true>(zp[e], cd0);
            }
            flat7_row_seg<T, VEC, S>(fc, fym, fyp, fzm, fzp, ih2, Mx, first_step<T, true>(hc, cd0));
#pragma unroll
            for (int e = 0; e < VEC; ++e) o[e] = cheb_step<T>(fc[e], T(0), c[e], Mx[e], a, cd);
        } else {
            flat7_row_seg<T, VEC, S>(c, ym, yp, zm, zp, ih2, Mx, hc);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const T xpe = PREVB ? first_step<T, true>(bb[e], cd0) : PREV ? pp[e] : T(0);
                o[e] = cheb_step<T>(c[e], xpe, bb[e], Mx[e], a, cd);
            }
        }
        strow<T, VEC>(out + g.row(y, z) + off, o);
        if (more) {
            if constexpr (PRO) {
                padd(zpp, cpp, y, z + 2);
                if (lo || hi) padd(hn, chn, yh, z + 1);
            }
            if constexpr (PREVP) padd(pn, cpn, y, z + 1);
            copyrow(zm, c);
            copyrow(c, zp);
            copyrow(zp, zpp);
            hc = hp;
            hp = hpp;
            if constexpr (!FROMB) copyrow(bb, bn);
            if constexpr (LDP || PREVP) copyrow(pp, pn);
            if (lo || hi) copyrow(h, hn);
        }
    }
}

// =====================================================================================
// Two consecutive smoothing steps in one pass (temporal blocking in z):
//   y1 = x  + a1 (x  - xp) + cd1 (b - M x)       (xp = 0 when PREV1 is false)
//   y2 = y1 + a2 (y1 - x ) + cd2 (b - M y1)
// Only y2 (and, with Y1OUT, y1) is written.  A block of NW waves owns rows
// y0-1 .. y0+W (W = NW - 2 outputs): every wave forms y1 on its row one plane
// ahead of the second step, the x rows y +- 1 coming from the caches; the y1
// plane the second step needs is shared through LDS (double-buffered by plane
// parity, one barrier per plane), with the two edge waves supplying the halo
// rows.  A z chunk of nz output planes forms y1 on nz + 2 planes.  The
// arithmetic of each step is that of k_smooth_row, in the same order.
//
// FROMB: the first three steps of a pass from zero.  x is not read: it is
// the pointwise first step x = cd0 b (cd0 = c0 / D), formed from the b rows
// in T exactly as the single step from zero and the outer residual kernel
// form it, and xp = 0.  One pass then reads b and writes the third step.
// PREVB: the third and fourth steps of a pass from zero of degree 4, whose
// second step (x) a single-step launch formed from b alone.  x_prev is then
// the pointwise first step cd0 b, formed from the b rows in T like the
// above, instead of being written and read back.
// With a sums job (job.count > 0), one extra block (block 0, dispatched first) finishes the
// partial sums of the outer residual launch that produced b, instead of a
// launch of its own (FROMB and PREVB only).
// =====================================================================================
// S > 1: each row is split into S segments of 64 VEC elements, one per wave
// (S consecutive waves hold one row), so that long rows keep few values per
// lane; the x-neighbours across segment ends come from a halo element loaded
// with each row of the first step's z queue, and from the neighbouring
// segment's slot in LDS for the second step.
template <typename T, int VEC, int NW, bool PREV1, bool Y1OUT, bool FROMB = false, bool PF2 = false, int NZC = 0,
          int S = 1, bool PREVB = false>
__global__ __launch_bounds__(64 * NW) void k_smooth2_lds(int n, T ih2, const T* __restrict__ x,
                                                         const T* __restrict__ xp, const T* __restrict__ b,
                                                         T* __restrict__ y2, T* __restrict__ y1o, T a1, T cd1, T a2,
                                                         T cd2, int nz, int nyb, T cd0, SumsJob job) {
    static_assert(!(FROMB && PREV1), "a pass from zero has no x_prev");
    static_assert(!PREVB || PREV1, "PREVB forms x_prev from b");
    constexpr bool LDP = PREV1 && !PREVB;  // x_prev is loaded
    static_assert(S == 1 || VEC * sizeof(T) <= 16, "split rows keep the plain LDS row layout");
    static_assert(NW % S == 0, "a block holds whole rows");
    constexpr int NR = 64 * VEC;
    constexpr int W = NW / S - 2;
    __shared__ T rows[2][NW][NR];
    const RowGrid g{NR * S, NR * S - 1};
    int nb = gridDim.x, bid = blockIdx.x;
    if constexpr (FROMB || PREVB) {
        if (job.count > 0) {  // block 0 finishes the sums, dispatched first
            nb -= 1;
            bid -= 1;
            if (bid < 0) {
                __shared__ double sh[kSumLanes];
                finish_sums(job, sh);
                return;
            }
        }
    }
    const int lb = xcd_logical(bid, nb);
    const int yb = lb % nyb, zc = lb / nyb;
    const int w = wave_id();
    const int wr = w / S, seg = w - wr * S;  // row of the block and segment of the row
    const int lane = threadIdx.x & 63;
    const int y = yb * W - 1 + wr;  // rows outside [0, n) wrap for loads
    const bool outw = wr >= 1 && wr <= W && y < n;
    const int z0 = zc * nz;
    const size_t off = (size_t)seg * NR + (size_t)lane * VEC;
    const int hoff = S > 1 ? seg_halo<VEC, S>(seg, lane) : 0;
    // LDS slots of the same row's previous / next segment (second-step halo)
    const int wprev = wr * S + (seg + S - 1) % S, wnext = wr * S + (seg + 1) % S;
    // first step: x on this row at planes z1-1, z1, z1+1, rows y-1 / y+1 at z1, b and xp at z1
    // (FROMB: these hold the b rows, x is formed from them, and b1 / b2 are
    // the queue's own rows)
    T xm[VEC], xc[VEC], xq[VEC], ym[VEC], yp[VEC], b1[VEC], p1[VEC];
    // second step: y1 on this row at z2-1 and z2 (z2 = z1 - 1) and b at z2; its
    // x_prev is x at z2, i.e. xm
    T sm[VEC], sc[VEC], b2[VEC];
    // S > 1: x-halo elements of the centre rows xc, xq (and xa) of the first step
    T hc = T(0), hq = T(0), ha = T(0);
    const T* src = FROMB ? b : x;
    int z1 = z0 - 1;
    ldrow<T, VEC>(xm, src + g.row(y, z1 - 1) + off);
    ldrow<T, VEC>(xc, src + g.row(y, z1) + off);
    ldrow<T, VEC>(xq, src + g.row(y, z1 + 1) + off);
    if constexpr (S > 1) {
        hc = src[g.row(y, z1) + hoff];
        hq = src[g.row(y, z1 + 1) + hoff];
    }
    ldrow<T, VEC>(ym, src + g.row(y - 1, z1) + off);
    ldrow<T, VEC>(yp, src + g.row(y + 1, z1) + off);
    if constexpr (!FROMB) ldrow<T, VEC>(b1, b + g.row(y, z1) + off);
    if constexpr (LDP) ldrow<T, VEC>(p1, xp + g.row(y, z1) + off);
    // NZC > 0: the chunk height is a compile-time constant and the plane loop
    // unrolls completely, so the row queues are renamed instead of copied and
    // each prefetched row is waited for where it is first used, not at the end
    // of the iteration that issued it.
    const int steps = (NZC > 0 ? NZC : nz) + 2;
    // PF2: operands of the plane after next are loaded one iteration earlier
    // (a second register set), i.e. two planes ahead of their use
    T xa[VEC], yma[VEC], ypa[VEC], ba[VEC], pa[VEC];
    if constexpr (PF2) {
        ldrow<T, VEC>(xa, src + g.row(y, z1 + 2) + off);
        if constexpr (S > 1) ha = src[g.row(y, z1 + 2) + hoff];
        ldrow<T, VEC>(yma, src + g.row(y - 1, z1 + 1) + off);
        ldrow<T, VEC>(ypa, src + g.row(y + 1, z1 + 1) + off);
        if constexpr (!FROMB) ldrow<T, VEC>(ba, b + g.row(y, z1 + 1) + off);
        if constexpr (LDP) ldrow<T, VEC>(pa, xp + g.row(y, z1 + 1) + off);
    }
    auto plane = [&](const int j) {
        const bool more = j + 1 < steps;
        const int ahead = PF2 ? 1 : 0;  // the loads below are for plane z1 + 1 + ahead
        const bool load = j + 1 + ahead < steps;
        T xn[VEC], ymn[VEC], ypn[VEC], bn[VEC], pn[VEC];
        T hn = T(0);
        if (load) {
            ldrow<T, VEC>(xn, src + g.row(y, z1 + 2 + ahead) + off);
            if constexpr (S > 1) hn = src[g.row(y, z1 + 2 + ahead) + hoff];
            ldrow<T, VEC>(ymn, src + g.row(y - 1, z1 + 1 + ahead) + off);
            ldrow<T, VEC>(ypn, src + g.row(y + 1, z1 + 1 + ahead) + off);
            if constexpr (!FROMB) ldrow<T, VEC>(bn, b + g.row(y, z1 + 1 + ahead) + off);
            if constexpr (LDP) ldrow<T, VEC>(pn, xp + g.row(y, z1 + 1 + ahead) + off);
        }
        T M1[VEC], sp[VEC];
        if constexpr (FROMB) {
            T fc[VEC], fm[VEC], fq[VEC], fym[VEC], fyp[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                fc[e] = first_step<T, FROMB>(xc[e], cd0);
                fm[e] = first_step<T, FROMB>(xm[e], cd0);
                fq[e] = first_step<T, FROMB>(xq[e], cd0);
                fym[e] = first_step<T, FROMB>(ym[e], cd0);
                fyp[e] = first_step<T, FROMB>(yp[e], cd0);
            }
            flat7_row_seg<T, VEC, S>(fc, fym, fyp, fm, fq, ih2, M1, first_step<T, FROMB>(hc, cd0));
#pragma unroll
            for (int e = 0; e < VEC; ++e) sp[e] = cheb_step<T>(fc[e], T(0), xc[e], M1[e], a1, cd1);
        } else {
            flat7_row_seg<T, VEC, S>(xc, ym, yp, xm, xq, ih2, M1, hc);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const T xpe = PREVB ? first_step<T, true>(b1[e], cd0) : PREV1 ? p1[e] : T(0);
                sp[e] = cheb_step<T>(xc[e], xpe, b1[e], M1[e], a1, cd1);
            }
        }
        if constexpr (Y1OUT) {
            if (outw && j >= 1 && j <= nz) strow<T, VEC>(y1o + g.row(y, z1) + off, sp);
        }
        if (j >= 2) {
            const int buf = j & 1;
            lds_strow<T, VEC>(rows[buf][w], lane, sc);
            __syncthreads();
            if (outw) {
                T nm[VEC], np[VEC], M2[VEC], o[VEC];
                lds_ldrow<T, VEC>(nm, rows[buf][w - S], lane);
                lds_ldrow<T, VEC>(np, rows[buf][w + S], lane);
                T hs = T(0);
                if constexpr (S > 1) hs = lane < 32 ? rows[buf][wprev][NR - 1] : rows[buf][wnext][0];
                flat7_row_seg<T, VEC, S>(sc, nm, np, sm, sp, ih2, M2, hs);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    if constexpr (FROMB)  // x_prev = first step at z2, b at z2 = the raw queue row
                        o[e] = cheb_step<T>(sc[e], first_step<T, FROMB>(xm[e], cd0), xm[e], M2[e], a2, cd2);
                    else
                        o[e] = cheb_step<T>(sc[e], xm[e], b2[e], M2[e], a2, cd2);
                }
                strow<T, VEC>(y2 + g.row(y, z1 - 1) + off, o);
            }
        }
        copyrow(sm, sc);
        copyrow(sc, sp);
        if constexpr (!FROMB) copyrow(b2, b1);
        if (more) {
            copyrow(xm, xc);
            copyrow(xc, xq);
            hc = hq;
            if constexpr (PF2) {
                hq = ha;
                if (load) ha = hn;
                copyrow(xq, xa);
                copyrow(ym, yma);
                copyrow(yp, ypa);
                if constexpr (!FROMB) copyrow(b1, ba);
                if constexpr (LDP) copyrow(p1, pa);
                if (load) {
                    copyrow(xa, xn);
                    copyrow(yma, ymn);
                    copyrow(ypa, ypn);
                    if constexpr (!FROMB) copyrow(ba, bn);
                    if constexpr (LDP) copyrow(pa, pn);
                }
            } else {
                hq = hn;
                copyrow(xq, xn);
                copyrow(ym, ymn);
                copyrow(yp, ypn);
                if constexpr (!FROMB) copyrow(b1, bn);
                if constexpr (LDP) copyrow(p1, pn);
            }
        }
    };
    if constexpr (NZC > 0) {
#pragma unroll
        for (int j = 0; j < NZC + 2; ++j, ++z1) plane(j);
    } else {
        for (int j = 0; j < steps; ++j, ++z1) plane(j);
    }
}

// The same two steps with the x plane (FROMB: the b plane) shared through LDS
// as well: every wave loads only its own row of x (b, x_prev) and publishes
// it one plane ahead of its use, so the first step's y-neighbours (and, for
// split rows, its x-halo) come from LDS instead of the caches; only the two
// edge rows of the block load their outer neighbour row.  One barrier per
// plane for both planes; same arithmetic and bits as k_smooth2_lds.
// PRO: the pair starts a post-smoothing pass from x0 = x + P e (ec: the
// coarse correction on the (n/2)^3 grid), formed row by row as the x rows
// arrive and never written; the prolongation of k_prolong_row, same bits.
template <typename T, int VEC, int NW, bool PREV1, bool Y1OUT, bool FROMB, int NZC, int S, bool PREVB = false,
          bool PRO = false, bool PFA = false>
__global__ __launch_bounds__(64 * NW) void k_smooth2x_lds(int n, T ih2, const T* __restrict__ x,
                                                          const T* __restrict__ xp, const T* __restrict__ b,
                                                          T* __restrict__ y2, T* __restrict__ y1o, T a1, T cd1,
                                                          T a2, T cd2, int nyb, T cd0, SumsJob job,
                                                          const T* __restrict__ ec) {
    static_assert(!(FROMB && PREV1), "a pass from zero has no x_prev");
    static_assert(!PREVB || PREV1, "PREVB forms x_prev from b");
    static_assert(!PRO || (!FROMB && !PREV1 && VEC >= 2), "the prolongation starts a pass from x, x_prev = 0");
    constexpr bool LDP = PREV1 && !PREVB;  // x_prev is loaded
    static_assert(VEC * sizeof(T) <= 16, "plain LDS row layout");
    static_assert(NW % S == 0 && NW / S >= 3, "a block holds whole rows, at least one output row");
    constexpr int NR = 64 * VEC;
    constexpr int R = NW / S;  // rows of the block
    constexpr int W = R - 2;   // output rows
    __shared__ T xs[2][NW][NR];    // x (FROMB: b) rows of a plane, one plane ahead
    __shared__ T rows[2][NW][NR];  // first-step rows of a plane
    const RowGrid g{NR * S, NR * S - 1};
    const RowGrid gc{NR * S / 2, NR * S / 2 - 1};  // PRO: the coarse grid of ec
    int nb = gridDim.x, bid = blockIdx.x;
    if constexpr (FROMB || PREVB) {
        if (job.count > 0) {  // block 0 finishes the sums, dispatched first
            nb -= 1;
            bid -= 1;
            if (bid < 0) {
                __shared__ double sh[kSumLanes];
                finish_sums(job, sh);
                return;
            }
        }
    }
    const int lb = xcd_logical(bid, nb);
    const int yb = lb % nyb, zc = lb / nyb;
    const int w = wave_id();
    const int wr = w / S, seg = w - wr * S;
    const int lane = threadIdx.x & 63;
    const int y = yb * W - 1 + wr;  // rows outside [0, n) wrap for loads
    const bool outw = wr >= 1 && wr <= W && y < n;
    const bool lo = wr == 0, hi = wr == R - 1;
    const int yo = lo ? y - 1 : y + 1;  // outer neighbour row of an edge row
    const int z0 = zc * NZC;
    const size_t off = (size_t)seg * NR + (size_t)lane * VEC;
    const int wprev = wr * S + (seg + S - 1) % S, wnext = wr * S + (seg + 1) % S;
    const T* src = FROMB ? b : x;
    int z1 = z0 - 1;
    // first step at z1: this row at z1-1, z1, z1+1, the outer row (edges) at z1, b and xp at z1
    T xm[VEC], xc[VEC], xq[VEC], o1[VEC] = {}, b1[VEC], p1[VEC];
    // second step at z2 = z1 - 1: first-step rows at z2-1, z2; b at z2; x_prev = xm
    T sm[VEC] = {}, sc[VEC] = {}, b2[VEC] = {};
    ldrow<T, VEC>(xm, src + g.row(y, z1 - 1) + off);
    ldrow<T, VEC>(xc, src + g.row(y, z1) + off);
    ldrow<T, VEC>(xq, src + g.row(y, z1 + 1) + off);
    if (lo || hi) ldrow<T, VEC>(o1, src + g.row(yo, z1) + off);
    if constexpr (!FROMB) ldrow<T, VEC>(b1, b + g.row(y, z1) + off);
    if constexpr (LDP) ldrow<T, VEC>(p1, xp + g.row(y, z1) + off);
    if constexpr (PRO) {  // x0 = x + P e on the rows loaded so far
        CoarseSeg<T, VEC> c;
        coarse_load_seg<T, VEC>(c, ec, gc, y, z1 - 1, seg, lane);
        prolong_add_seg<T, VEC>(xm, c, y, z1 - 1);
        coarse_load_seg<T, VEC>(c, ec, gc, y, z1, seg, lane);
        prolong_add_seg<T, VEC>(xc, c, y, z1);
        coarse_load_seg<T, VEC>(c, ec, gc, y, z1 + 1, seg, lane);
        prolong_add_seg<T, VEC>(xq, c, y, z1 + 1);
        if (lo || hi) {
            coarse_load_seg<T, VEC>(c, ec, gc, yo, z1, seg, lane);
            prolong_add_seg<T, VEC>(o1, c, yo, z1);
        }
    }
    lds_strow<T, VEC>(xs[0][w], lane, xc);
    constexpr int steps = NZC + 2;
    // PFA: the rows of the next plane are loaded one iteration earlier into a
    // second register set (xa, oa, ba, pa), i.e. two planes ahead of their use
    constexpr int ahead = PFA ? 1 : 0;
    T xa[VEC], oa[VEC] = {}, ba[VEC], pa[VEC];
    CoarseSeg<T, VEC> ca, coa;
    if constexpr (PFA) {
        ldrow<T, VEC>(xa, src + g.row(y, z1 + 2) + off);
        if (lo || hi) ldrow<T, VEC>(oa, src + g.row(yo, z1 + 1) + off);
        if constexpr (PRO) {
            coarse_load_seg<T, VEC>(ca, ec, gc, y, z1 + 2, seg, lane);
            if (lo || hi) coarse_load_seg<T, VEC>(coa, ec, gc, yo, z1 + 1, seg, lane);
        }
        if constexpr (!FROMB) ldrow<T, VEC>(ba, b + g.row(y, z1 + 1) + off);
        if constexpr (LDP) ldrow<T, VEC>(pa, xp + g.row(y, z1 + 1) + off);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < steps; ++j, ++z1) {
        const bool more = j + 1 < steps;
        const bool load = j + 1 + ahead < steps;
        const int cb = j & 1;
        T xn[VEC], bn[VEC], pn[VEC], on[VEC];
        CoarseSeg<T, VEC> cn, con;  // PRO: coarse rows of xn and on
        if (load) {
            ldrow<T, VEC>(xn, src + g.row(y, z1 + 2 + ahead) + off);
            if (lo || hi) ldrow<T, VEC>(on, src + g.row(yo, z1 + 1 + ahead) + off);
            if constexpr (PRO) {
                coarse_load_seg<T, VEC>(cn, ec, gc, y, z1 + 2 + ahead, seg, lane);
                if (lo || hi) coarse_load_seg<T, VEC>(con, ec, gc, yo, z1 + 1 + ahead, seg, lane);
            }
            if constexpr (!FROMB) ldrow<T, VEC>(bn, b + g.row(y, z1 + 1 + ahead) + off);
            if constexpr (LDP) ldrow<T, VEC>(pn, xp + g.row(y, z1 + 1 + ahead) + off);
        }
        // first step at z1
        T ym[VEC], yp[VEC], M1[VEC], sp[VEC];
        if (lo) copyrow(ym, o1);
        else lds_ldrow<T, VEC>(ym, xs[cb][w - S], lane);
        if (hi) copyrow(yp, o1);
        else lds_ldrow<T, VEC>(yp, xs[cb][w + S], lane);
        T hx = T(0);
        if constexpr (S > 1) hx = lane < 32 ? xs[cb][wprev][NR - 1] : xs[cb][wnext][0];
        if constexpr (FROMB) {
            T fc[VEC], fm[VEC], fq[VEC], fym[VEC], fyp[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                fc[e] = first_step<T, FROMB>(xc[e], cd0);
                fm[e] = first_step<T, FROMB>(xm[e], cd0);
                fq[e] = first_step<T, FROMB>(xq[e], cd0);
                fym[e] = first_step<T, FROMB>(ym[e], cd0);
                fyp[e] = first_step<T, FROMB>(yp[e], cd0);
            }
            flat7_row_seg<T, VEC, S>(fc, fym, fyp, fm, fq, ih2, M1, first_step<T, FROMB>(hx, cd0));
#pragma unroll
            for (int e = 0; e < VEC; ++e) sp[e] = cheb_step<T>(fc[e], T(0), xc[e], M1[e], a1, cd1);
        } else {
            flat7_row_seg<T, VEC, S>(xc, ym, yp, xm, xq, ih2, M1, hx);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const T xpe = PREVB ? first_step<T, true>(b1[e], cd0) : PREV1 ? p1[e] : T(0);
                sp[e] = cheb_step<T>(xc[e], xpe, b1[e], M1[e], a1, cd1);
            }
        }
        if constexpr (Y1OUT) {
            if (outw && j >= 1 && j <= NZC) strow<T, VEC>(y1o + g.row(y, z1) + off, sp);
        }
        // publish x at z1+1 (used by the next plane's first step) and the first step at z1-1
        if (more) lds_strow<T, VEC>(xs[cb ^ 1][w], lane, xq);
        if (j >= 2) lds_strow<T, VEC>(rows[cb][w], lane, sc);
        __syncthreads();
        if (j >= 2 && outw) {  // second step at z1-1
            T nm[VEC], np[VEC], M2[VEC], o[VEC];
            lds_ldrow<T, VEC>(nm, rows[cb][w - S], lane);
            lds_ldrow<T, VEC>(np, rows[cb][w + S], lane);
            T hs = T(0);
            if constexpr (S > 1) hs = lane < 32 ? rows[cb][wprev][NR - 1] : rows[cb][wnext][0];
            flat7_row_seg<T, VEC, S>(sc, nm, np, sm, sp, ih2, M2, hs);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                if constexpr (FROMB)  // x_prev = first step at z2, b at z2 = the raw queue row
                    o[e] = cheb_step<T>(sc[e], first_step<T, FROMB>(xm[e], cd0), xm[e], M2[e], a2, cd2);
                else
                    o[e] = cheb_step<T>(sc[e], xm[e], b2[e], M2[e], a2, cd2);
            }
            strow<T, VEC>(y2 + g.row(y, z1 - 1) + off, o);
        }
        copyrow(sm, sc);
        copyrow(sc, sp);
        if constexpr (!FROMB) copyrow(b2, b1);
        if (more) {
            if constexpr (PFA) {
                if constexpr (PRO) {  // two iterations after their loads were issued
                    prolong_add_seg<T, VEC>(xa, ca, y, z1 + 2);
                    if (lo || hi) prolong_add_seg<T, VEC>(oa, coa, yo, z1 + 1);
                }
                copyrow(xm, xc);
                copyrow(xc, xq);
                copyrow(xq, xa);
                if (lo || hi) copyrow(o1, oa);
                if constexpr (!FROMB) copyrow(b1, ba);
                if constexpr (LDP) copyrow(p1, pa);
                if (load) {
                    copyrow(xa, xn);
                    if (lo || hi) copyrow(oa, on);
                    if constexpr (PRO) {
                        ca = cn;
                        coa = con;
                    }
                    if constexpr (!FROMB) copyrow(ba, bn);
                    if constexpr (LDP) copyrow(pa, pn);
                }
            } else {
                if constexpr (PRO) {  // a whole iteration after their loads were issued
                    prolong_add_seg<T, VEC>(xn, cn, y, z1 + 2);
                    if (lo || hi) prolong_add_seg<T, VEC>(on, con, yo, z1 + 1);
                }
                copyrow(xm, xc);
                copyrow(xc, xq);
                copyrow(xq, xn);
                if (lo || hi) copyrow(o1, on);
                if constexpr (!FROMB) copyrow(b1, bn);
                if constexpr (LDP) copyrow(p1, pn);
            }
        }
    }
}

// =====================================================================================
// Three consecutive smoothing steps in one pass, starting a pass from x
// (x_prev = 0, as in the first step of a post-smoothing pass):
//   y1 = x  + a0 x + cd0 (b - M x)
//   y2 = y1 + a1 (y1 - x ) + cd1 (b - M y1)
//   y3 = y2 + a2 (y2 - y1) + cd2 (b - M y2)
// Only y3 is written.  A block of NW waves owns rows y0-2 .. y0+W+1 (W = NW - 4
// outputs): every wave forms y1 on its row (x rows y +- 1 from the caches),
// waves 1 .. NW-2 form y2 one plane behind, waves 2 .. NW-3 form y3 one more
// plane behind.  The y1 and y2 planes are shared through LDS, double-buffered
// by iteration parity, one barrier per plane.  The arithmetic of each step is
// that of k_smooth_row, in the same order.  NZC: compile-time chunk height
// (the plane loop unrolls completely, see k_smooth2_lds).
// =====================================================================================
template <typename T, int VEC, int NW, int NZC>
__global__ __launch_bounds__(64 * NW) void k_smooth3_lds(int n, T ih2, const T* __restrict__ x,
                                                         const T* __restrict__ b, T* __restrict__ y3, T a0, T cd0,
                                                         T a1, T cd1, T a2, T cd2, int nyb) {
    constexpr int NR = 64 * VEC;
    constexpr int W = NW - 4;
    __shared__ T rows1[2][NW][NR];
    __shared__ T rows2[2][NW][NR];
    const RowGrid g{64 * VEC, 64 * VEC - 1};
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int w = wave_id();
    const int lane = threadIdx.x & 63;
    const int y = yb * W - 2 + w;  // rows outside [0, n) wrap for loads
    const bool st2 = w >= 1 && w <= NW - 2;
    const bool outw = w >= 2 && w <= NW - 3 && y < n;
    const int z0 = zc * NZC;
    const size_t off = (size_t)lane * VEC;
    // stage 1 at plane z1: x on this row at z1-1, z1, z1+1, rows y-1 / y+1 at z1, b at z1
    T xm[VEC], xc[VEC], xq[VEC], ym[VEC], yp[VEC], b1[VEC];
    // stage 2 at z1-1: y1 at z1-2, z1-1 (and z1 just formed), b at z1-1; x_prev = x at z1-1 = xm
    // stage 3 at z1-2: y2 at z1-3, z1-2 (and z1-1 just formed), b at z1-2; x_prev = y1 at z1-2 = s1m
    // (the queues start empty: their first planes are formed before they are read)
    T s1m[VEC] = {}, s1c[VEC] = {}, b2[VEC] = {};
    T s2m[VEC] = {}, s2c[VEC] = {}, b3[VEC] = {};
    int z1 = z0 - 2;
    ldrow<T, VEC>(xm, x + g.row(y, z1 - 1) + off);
    ldrow<T, VEC>(xc, x + g.row(y, z1) + off);
    ldrow<T, VEC>(xq, x + g.row(y, z1 + 1) + off);
    ldrow<T, VEC>(ym, x + g.row(y - 1, z1) + off);
    ldrow<T, VEC>(yp, x + g.row(y + 1, z1) + off);
    ldrow<T, VEC>(b1, b + g.row(y, z1) + off);
    constexpr int steps = NZC + 4;
#pragma unroll
    for (int j = 0; j < steps; ++j, ++z1) {
        const bool more = j + 1 < steps;
        T xn[VEC], ymn[VEC], ypn[VEC], bn[VEC];
        if (more) {
            ldrow<T, VEC>(xn, x + g.row(y, z1 + 2) + off);
            ldrow<T, VEC>(ymn, x + g.row(y - 1, z1 + 1) + off);
            ldrow<T, VEC>(ypn, x + g.row(y + 1, z1 + 1) + off);
            ldrow<T, VEC>(bn, b + g.row(y, z1 + 1) + off);
        }
        // stage 1: y1 at z1 (x_prev = 0)
        T M1[VEC], s1p[VEC];
        flat7_row<T, VEC>(xc, ym, yp, xm, xq, ih2, M1);
#pragma unroll
        for (int e = 0; e < VEC; ++e) s1p[e] = cheb_step<T>(xc[e], T(0), b1[e], M1[e], a0, cd0);
        T s2p[VEC] = {};
        if (j >= 2) {
            const int buf = j & 1;
            lds_strow<T, VEC>(rows1[buf][w], lane, s1c);                // y1 at z1-1
            if (j >= 3 && st2) lds_strow<T, VEC>(rows2[buf][w], lane, s2c);  // y2 at z1-2
            __syncthreads();
            if (st2) {  // stage 2: y2 at z1-1
                T nm[VEC], np[VEC], M2[VEC];
                lds_ldrow<T, VEC>(nm, rows1[buf][w - 1], lane);
                lds_ldrow<T, VEC>(np, rows1[buf][w + 1], lane);
                flat7_row<T, VEC>(s1c, nm, np, s1m, s1p, ih2, M2);
#pragma unroll
                for (int e = 0; e < VEC; ++e) s2p[e] = cheb_step<T>(s1c[e], xm[e], b2[e], M2[e], a1, cd1);
            }
            if (j >= 4 && outw) {  // stage 3: y3 at z1-2
                T nm[VEC], np[VEC], M3[VEC], o[VEC];
                lds_ldrow<T, VEC>(nm, rows2[buf][w - 1], lane);
                lds_ldrow<T, VEC>(np, rows2[buf][w + 1], lane);
                flat7_row<T, VEC>(s2c, nm, np, s2m, s2p, ih2, M3);
#pragma unroll
                for (int e = 0; e < VEC; ++e) o[e] = cheb_step<T>(s2c[e], s1m[e], b3[e], M3[e], a2, cd2);
                strow<T, VEC>(y3 + g.row(y, z1 - 2) + off, o);
            }
        }
        // rotate the queues
        copyrow(s2m, s2c);
        copyrow(s2c, s2p);
        copyrow(b3, b2);
        copyrow(s1m, s1c);
        copyrow(s1c, s1p);
        copyrow(b2, b1);
        if (more) {
            copyrow(xm, xc);
            copyrow(xc, xq);
            copyrow(xq, xn);
            copyrow(ym, ymn);
            copyrow(yp, ypn);
            copyrow(b1, bn);
        }
    }
}

// =====================================================================================
// The three-step pass fused with the prolongation before it: the pass starts
// from x0 = x + P e, formed row by row as x and the coarse rows arrive, never
// written.  Each wave forms x0 on its own row (z queue) and the two edge waves
// also on one halo row each; the x0 plane is shared through LDS like the y1
// and y2 planes, so stage 1 reads its y-neighbours there instead of from the
// caches.  Same three steps as k_smooth3_lds, same bits as prolongation
// followed by three single steps.
// =====================================================================================
template <typename T, int VEC, int NW, int NZC>
__global__ __launch_bounds__(64 * NW) void k_smooth3p_lds(int n, T ih2, const T* __restrict__ x,
                                                          const T* __restrict__ e, const T* __restrict__ b,
                                                          T* __restrict__ y3, T a0, T cd0, T a1, T cd1, T a2, T cd2,
                                                          int nyb) {
    constexpr int NR = 64 * VEC;
    constexpr int W = NW - 4;
    __shared__ T rows0[2][NW + 2][NR];  // x0: slot w + 1 = wave w's row, slots 0 / NW + 1 the halo rows
    __shared__ T rows1[2][NW][NR];
    __shared__ T rows2[2][NW][NR];
    const RowGrid g{64 * VEC, 64 * VEC - 1};
    const RowGrid gc{32 * VEC, 32 * VEC - 1};
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int w = wave_id();
    const int lane = threadIdx.x & 63;
    const int y = yb * W - 2 + w;  // rows outside [0, n) wrap for loads (parity and coarse row wrap alike)
    const bool lo = w == 0, hi = w == NW - 1;
    const int yh = lo ? y - 1 : y + 1;  // halo row of an edge wave
    const bool st2 = w >= 1 && w <= NW - 2;
    const bool outw = w >= 2 && w <= NW - 3 && y < n;
    const int z0 = zc * NZC;
    const size_t off = (size_t)lane * VEC;
    auto load_x0 = [&](T (&v)[VEC], int yy, int zz) {
        CoarseRows<T, VEC> c;
        ldrow<T, VEC>(v, x + g.row(yy, zz) + off);
        coarse_load<T, VEC>(c, e, gc, yy, zz, lane);
        prolong_add<T, VEC>(v, c, yy, zz);
    };
    // x0 on this row at z1-1, z1, z1+1 and on the halo row at z1; b at z1
    T xm[VEC], xc[VEC], xq[VEC], h[VEC] = {}, b1[VEC];
    T s1m[VEC] = {}, s1c[VEC] = {}, b2[VEC] = {};
    T s2m[VEC] = {}, s2c[VEC] = {}, b3[VEC] = {};
    int z1 = z0 - 2;
    load_x0(xm, y, z1 - 1);
    load_x0(xc, y, z1);
    load_x0(xq, y, z1 + 1);
    if (lo || hi) load_x0(h, yh, z1);
    ldrow<T, VEC>(b1, b + g.row(y, z1) + off);
    constexpr int steps = NZC + 4;
#pragma unroll
    for (int j = 0; j < steps; ++j, ++z1) {
        const bool more = j + 1 < steps;
        // raw operands of the next plane: this row at z1+2, the halo row at z1+1, b at z1+1
        T xr[VEC], hr[VEC], bn[VEC];
        CoarseRows<T, VEC> cr, chr;
        if (more) {
            ldrow<T, VEC>(xr, x + g.row(y, z1 + 2) + off);
            coarse_load<T, VEC>(cr, e, gc, y, z1 + 2, lane);
            if (lo || hi) {
                ldrow<T, VEC>(hr, x + g.row(yh, z1 + 1) + off);
                coarse_load<T, VEC>(chr, e, gc, yh, z1 + 1, lane);
            }
            ldrow<T, VEC>(bn, b + g.row(y, z1 + 1) + off);
        }
        const int buf = j & 1;
        lds_strow<T, VEC>(rows0[buf][w + 1], lane, xc);
        if (lo) lds_strow<T, VEC>(rows0[buf][0], lane, h);
        if (hi) lds_strow<T, VEC>(rows0[buf][NW + 1], lane, h);
        if (j >= 2) lds_strow<T, VEC>(rows1[buf][w], lane, s1c);                 // y1 at z1-1
        if (j >= 3 && st2) lds_strow<T, VEC>(rows2[buf][w], lane, s2c);          // y2 at z1-2
        __syncthreads();
        // stage 1: y1 at z1 (x_prev = 0)
        T s1p[VEC];
        {
            T ym[VEC], yp[VEC], M1[VEC];
            lds_ldrow<T, VEC>(ym, rows0[buf][w], lane);
            lds_ldrow<T, VEC>(yp, rows0[buf][w + 2], lane);
            flat7_row<T, VEC>(xc, ym, yp, xm, xq, ih2, M1);
#pragma unroll
            for (int q = 0; q < VEC; ++q) s1p[q] = cheb_step<T>(xc[q], T(0), b1[q], M1[q], a0, cd0);
        }
        T s2p[VEC] = {};
        if (j >= 2 && st2) {  // stage 2: y2 at z1-1, x_prev = x0 at z1-1
            T nm[VEC], np[VEC], M2[VEC];
            lds_ldrow<T, VEC>(nm, rows1[buf][w - 1], lane);
            lds_ldrow<T, VEC>(np, rows1[buf][w + 1], lane);
            flat7_row<T, VEC>(s1c, nm, np, s1m, s1p, ih2, M2);
#pragma unroll
            for (int q = 0; q < VEC; ++q) s2p[q] = cheb_step<T>(s1c[q], xm[q], b2[q], M2[q], a1, cd1);
        }
        if (j >= 4 && outw) {  // stage 3: y3 at z1-2, x_prev = y1 at z1-2
            T nm[VEC], np[VEC], M3[VEC], o[VEC];
            lds_ldrow<T, VEC>(nm, rows2[buf][w - 1], lane);
            lds_ldrow<T, VEC>(np, rows2[buf][w + 1], lane);
            flat7_row<T, VEC>(s2c, nm, np, s2m, s2p, ih2, M3);
#pragma unroll
            for (int q = 0; q < VEC; ++q) o[q] = cheb_step<T>(s2c[q], s1m[q], b3[q], M3[q], a2, cd2);
            strow<T, VEC>(y3 + g.row(y, z1 - 2) + off, o);
        }
        copyrow(s2m, s2c);
        copyrow(s2c, s2p);
        copyrow(b3, b2);
        copyrow(s1m, s1c);
        copyrow(s1c, s1p);
        copyrow(b2, b1);
        if (more) {
            copyrow(xm, xc);
            copyrow(xc, xq);
            prolong_add<T, VEC>(xr, cr, y, z1 + 2);
            copyrow(xq, xr);
            if (lo || hi) {
                prolong_add<T, VEC>(hr, chr, yh, z1 + 1);
                copyrow(h, hr);
            }
            copyrow(b1, bn);
        }
    }
}

// S > 1: rows split into S segments, one per wave (W rows of S waves), for
// rows whose unsplit queues would not fit a wave's registers; each segment
// keeps its own slice of the LDS rows, and the x-neighbours across segment
// ends come from one halo element loaded with each centre row.
template <typename TA, typename TR, typename TE, int VEC, int W, bool UPDATE, int S = 1>
__global__ __launch_bounds__(64 * W * S) void k_outer_lds(int n, TA ih2, const double* __restrict__ phi_in,
                                                          const TE* __restrict__ e, double* __restrict__ phi_out,
                                                          const double* __restrict__ b, double bmean,
                                                          TR* __restrict__ r, TR* __restrict__ x1, TA cd0,
                                                          double* __restrict__ partials, int nz, int nyb) {
    constexpr int NR = 64 * VEC, NF = NR * S;
    __shared__ TA rows[2][W + 2][NF];
    __shared__ double sh[3 * W * S];
    const RowGrid g{NF, NF - 1};
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int wv = wave_id();
    const int w = wv / S, seg = wv - w * S;
    const int y0 = yb * W;
    const int y = y0 + w;
    const int z0 = zc * nz;
    const int lane = threadIdx.x & 63;
    const size_t off = (size_t)seg * NR + (size_t)lane * VEC;
    const int hoff = S > 1 ? seg_halo<VEC, S>(seg, lane) : 0;
    const bool lo = w == 0, hi = w == W - 1;
    const int yh = lo ? y0 - 1 : y0 + W;
    TA zm[VEC], c[VEC], zp[VEC], h[VEC];
    TA hc = TA(0), hp = TA(0);  // x-halo of c and zp (S > 1)
    double bb[VEC];
    ld_value<TA, TR, TE, VEC, UPDATE>(zm, phi_in, e, g.row(y, z0 - 1) + off);
    ld_value<TA, TR, TE, VEC, UPDATE>(c, phi_in, e, g.row(y, z0) + off);
    ld_value<TA, TR, TE, VEC, UPDATE>(zp, phi_in, e, g.row(y, z0 + 1) + off);
    if constexpr (S > 1) {
        hc = ld_value1<TA, TE, UPDATE>(phi_in, e, g.row(y, z0) + hoff);
        hp = ld_value1<TA, TE, UPDATE>(phi_in, e, g.row(y, z0 + 1) + hoff);
    }
    ldrow<double, VEC>(bb, b + g.row(y, z0) + off);
    if (lo || hi) ld_value<TA, TR, TE, VEC, UPDATE>(h, phi_in, e, g.row(yh, z0) + off);
    double ss = 0.0, sb = 0.0, sp = 0.0;
    for (int k = 0; k < nz; ++k) {
        const int z = z0 + k;
        const int buf = k & 1;
        TA zpp[VEC], hn[VEC];
        TA hpp = TA(0);
        double bn[VEC];
        const bool more = k + 1 < nz;
        if (more) {
            ld_value<TA, TR, TE, VEC, UPDATE>(zpp, phi_in, e, g.row(y, z + 2) + off);
            if constexpr (S > 1) hpp = ld_value1<TA, TE, UPDATE>(phi_in, e, g.row(y, z + 2) + hoff);
            ldrow<double, VEC>(bn, b + g.row(y, z + 1) + off);
            if (lo || hi) ld_value<TA, TR, TE, VEC, UPDATE>(hn, phi_in, e, g.row(yh, z + 1) + off);
        }
        lds_strow<TA, VEC>(rows[buf][w + 1] + seg * NR, lane, c);
        if (lo) lds_strow<TA, VEC>(rows[buf][0] + seg * NR, lane, h);
        if (hi) lds_strow<TA, VEC>(rows[buf][W + 1] + seg * NR, lane, h);
        __syncthreads();
        TA ym[VEC], yp[VEC];
        lds_ldrow<TA, VEC>(ym, rows[buf][w] + seg * NR, lane);
        lds_ldrow<TA, VEC>(yp, rows[buf][w + 2] + seg * NR, lane);
        TA Mx[VEC];
        TR ro[VEC];
        flat7_row_seg<TA, VEC, S>(c, ym, yp, zm, zp, ih2, Mx, hc);
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            const double bq = bb[q] - bmean;
            const TA ri = (TA)bq - Mx[q];
            ro[q] = (TR)ri;
            ss += (double)ri * (double)ri;
            sb += bq * bq;
        }
        const size_t row = g.row(y, z) + off;
        strow<TR, VEC>(r + row, ro);
        if (x1) {
            TR xo[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) xo[q] = (TR)cd0 * ro[q];  // in the iterate's precision, as the first step from zero
            strow<TR, VEC>(x1 + row, xo);
        }
        if constexpr (UPDATE) {
            double po[VEC];
            if constexpr (sizeof(TA) == sizeof(double)) {
#pragma unroll
                for (int q = 0; q < VEC; ++q) po[q] = (double)c[q];
            } else {  // keep the double sum phi + e (c holds it rounded to TA)
                double p[VEC];
                TE qv[VEC];
                ldrow<double, VEC>(p, phi_in + row);
                ldrow<TE, VEC>(qv, e + row);
#pragma unroll
                for (int q = 0; q < VEC; ++q) po[q] = p[q] + (double)qv[q];
            }
            strow<double, VEC>(phi_out + row, po);
#pragma unroll
            for (int q = 0; q < VEC; ++q) sp += po[q];
        } else if constexpr (sizeof(TA) == sizeof(double)) {
#pragma unroll
            for (int q = 0; q < VEC; ++q) sp += (double)c[q];
        } else {
            double p[VEC];
            ldrow<double, VEC>(p, phi_in + row);
#pragma unroll
            for (int q = 0; q < VEC; ++q) sp += p[q];
        }
        if (more) {
            copyrow(zm, c);
            copyrow(c, zp);
            copyrow(zp, zpp);
            hc = hp;
            hp = hpp;
            copyrow(bb, bn);
            if (lo || hi) copyrow(h, hn);
        }
    }
    outer_partials(partials, sb, ss, sp, sh, W * S);
}

// =====================================================================================
// Residual + full-weighting restriction: one wave per coarse row Y, marching
// fine planes; fine rows 2Y-1, 2Y, 2Y+1 are formed, combined in y, then in x
// across lanes, then accumulated in z, each with fw3's rounding.
// =====================================================================================
// S > 1: each coarse row's fine rows split into S segments of 64 VEC
// elements, one wave each (a block of kWaves waves holds kWaves / S coarse
// rows).  The stencil's x-neighbours across segment ends come from halo
// elements loaded with each row, and the full weighting in x of a segment's
// first coarse point takes the previous segment's last fine value from LDS.
template <typename T, int VEC, int S = 1>
__global__ __launch_bounds__(kBlock) void k_rr_row(int n, T ih2, const T* __restrict__ x,
                                                   const T* __restrict__ b, T* __restrict__ coarse, int nzc,
                                                   int nyb) {
#pragma clang fp contract(off)  // full weighting in y, then x, then z, as fw3 rounds it
    static_assert(S == 1 || VEC >= 2, "split rows hold at least two fine points per lane");
    static_assert(kWaves % S == 0, "a block holds whole rows");
    constexpr int CV = VEC >= 2 ? VEC / 2 : 1;
    constexpr int NR = 64 * VEC;
    constexpr int nc = NR * S / 2;
    const RowGrid g{NR * S, NR * S - 1};
    const RowGrid gc{nc, nc - 1};
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int Y = yb * (kWaves / S) + w / S, seg = w % S;
    const int wprev = (w / S) * S + (seg + S - 1) % S;
    const int Z0 = zc * nzc;
    const int y1 = 2 * Y;
    const size_t off = (size_t)seg * NR + (size_t)lane * VEC;
    const int hoff = S > 1 ? seg_halo<VEC, S>(seg, lane) : 0;
    __shared__ T edge[2][kWaves];  // last fine value of each segment (S > 1)
    // x rows 2Y-2 .. 2Y+2 at plane z (index 0..4) and rows 2Y-1..2Y+1 at z-1, z+1
    T c0[VEC], c1[VEC], c2[VEC];     // rows 2Y-1, 2Y, 2Y+1 at plane z
    T m0[VEC], m1[VEC], m2[VEC];     // same rows at z-1
    T p0[VEC], p1[VEC], p2[VEC];     // same rows at z+1
    T hm[VEC], hp[VEC];              // rows 2Y-2, 2Y+2 at plane z
    T h0 = T(0), h1 = T(0), h2 = T(0);  // x-halo of c0, c1, c2 (S > 1)
    int z = 2 * Z0 - 1;
    ldrow<T, VEC>(m0, x + g.row(y1 - 1, z - 1) + off);
    ldrow<T, VEC>(m1, x + g.row(y1, z - 1) + off);
    ldrow<T, VEC>(m2, x + g.row(y1 + 1, z - 1) + off);
    ldrow<T, VEC>(c0, x + g.row(y1 - 1, z) + off);
    ldrow<T, VEC>(c1, x + g.row(y1, z) + off);
    ldrow<T, VEC>(c2, x + g.row(y1 + 1, z) + off);
    if constexpr (S > 1) {
        h0 = x[g.row(y1 - 1, z) + hoff];
        h1 = x[g.row(y1, z) + hoff];
        h2 = x[g.row(y1 + 1, z) + hoff];
    }
    T acc[CV];
    const int nf = 2 * nzc + 1;
    for (int k = 0; k < nf; ++k, ++z) {
        ldrow<T, VEC>(p0, x + g.row(y1 - 1, z + 1) + off);
        ldrow<T, VEC>(p1, x + g.row(y1, z + 1) + off);
        ldrow<T, VEC>(p2, x + g.row(y1 + 1, z + 1) + off);
        T q0 = T(0), q1 = T(0), q2 = T(0);
        if constexpr (S > 1) {
            q0 = x[g.row(y1 - 1, z + 1) + hoff];
            q1 = x[g.row(y1, z + 1) + hoff];
            q2 = x[g.row(y1 + 1, z + 1) + hoff];
        }
        ldrow<T, VEC>(hm, x + g.row(y1 - 2, z) + off);
        ldrow<T, VEC>(hp, x + g.row(y1 + 2, z) + off);
        T b0[VEC], b1[VEC], b2[VEC];
        ldrow<T, VEC>(b0, b + g.row(y1 - 1, z) + off);
        ldrow<T, VEC>(b1, b + g.row(y1, z) + off);
        ldrow<T, VEC>(b2, b + g.row(y1 + 1, z) + off);
        T M0[VEC], M1[VEC], M2[VEC], s[VEC];
        flat7_row_seg<T, VEC, S>(c0, hm, c1, m0, p0, ih2, M0, h0);
        flat7_row_seg<T, VEC, S>(c1, c0, c2, m1, p1, ih2, M1, h1);
        flat7_row_seg<T, VEC, S>(c2, c1, hp, m2, p2, ih2, M2, h2);
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            s[e] = fw3<T>(b0[e] - M0[e], b1[e] - M1[e], b2[e] - M2[e]);
        // x: coarse element q <-> fine 2q; needs fine 2q-1 (previous lane's last for q = 0)
        T sx[CV];
        if constexpr (VEC >= 2) {
            T lft = lane_rot(s[VEC - 1], -1);
            if constexpr (S > 1) {  // lane 0: the previous segment's last fine value
                if (lane == 63) edge[k & 1][w] = s[VEC - 1];
                __syncthreads();
                if (lane == 0) lft = edge[k & 1][wprev];
            }
#pragma unroll
            for (int q = 0; q < CV; ++q) {
                const T l = q > 0 ? s[2 * q - 1] : lft;
                sx[q] = fw3<T>(l, s[2 * q], s[2 * q + 1]);
            }
        } else {
            const T l = lane_rot(s[0], -1), r = lane_rot(s[0], 1);
            sx[0] = fw3<T>(l, s[0], r);
        }
        // z: odd fine plane 2Z-1 opens coarse plane Z, 2Z adds 1/2, 2Z+1 closes it
        const bool odd = (k & 1) == 0;  // k = 0 <-> z = 2 Z0 - 1
        if (k == 0) {
#pragma unroll
            for (int q = 0; q < CV; ++q) acc[q] = T(0.25) * sx[q];
        } else if (!odd) {
#pragma unroll
            for (int q = 0; q < CV; ++q) acc[q] += T(0.5) * sx[q];
        } else {
            const int Z = (z - 1) >> 1;
#pragma unroll
            for (int q = 0; q < CV; ++q) acc[q] += T(0.25) * sx[q];
            if constexpr (VEC >= 2) {
                strow<T, CV>(coarse + gc.row(Y, Z) + (size_t)seg * (NR / 2) + (size_t)lane * CV, acc);
            } else {
                if ((lane & 1) == 0) coarse[gc.row(Y, Z) + (lane >> 1)] = acc[0];
            }
#pragma unroll
            for (int q = 0; q < CV; ++q) acc[q] = T(0.25) * sx[q];
        }
        copyrow(m0, c0);
        copyrow(m1, c1);
        copyrow(m2, c2);
        copyrow(c0, p0);
        copyrow(c1, p1);
        copyrow(c2, p2);
        h0 = q0;
        h1 = q1;
        h2 = q2;
    }
}

// The same residual + restriction with the fine rows shared through LDS
// (VEC >= 2): a block of (W + 1) S waves owns coarse rows Y0 .. Y0+W-1.
// Wave w (row slot wr = w / S, segment w mod S of S) loads fine rows
// fa = 2Y-1 and fb = 2Y (Y = Y0 + wr; slot W: rows 2Y0+2W-1 and 2Y0+2W, slot
// 0 also row 2Y0-2) one plane ahead and publishes them, so each x and b row
// is read once per block and each residual row is formed once (k_rr_row
// forms rows 2Y+-1 twice and reads x rows 2.5 times).  Slot wr < W combines
// r(2Y-1), r(2Y) with r(2Y+1) of slot wr + 1 (through LDS); slot W only forms
// r(2Y0+2W-1).  Split rows (S > 1) take the stencil's x-halo from the
// neighbouring segment in LDS, and the full weighting in x of a segment's
// first coarse point re-forms the previous segment's last y-weighted value
// from the shared residual rows and the published last element of its
// r(2Y).  One barrier per plane: the x plane, the shared residual row and
// the edge values are double-buffered by plane parity.  Same point formulas
// and the same fw3 order as k_rr_row, same bits.
template <typename T, int VEC, int W, int S>
__global__ __launch_bounds__(64 * (W + 1) * S) void k_rr_lds(int n, T ih2, const T* __restrict__ x,
                                                             const T* __restrict__ b, T* __restrict__ coarse,
                                                             int nzc, int nyb) {
#pragma clang fp contract(off)  // full weighting in y, then x, then z, as fw3 rounds it
    static_assert(VEC >= 2, "two fine points per lane at least");
    constexpr int CV = VEC / 2;
    constexpr int NR = 64 * VEC;  // a segment
    constexpr int NF = NR * S;    // a fine row
    constexpr int nc = NF / 2;
    __shared__ T xs[2][2 * W + 3][NF];  // fine rows 2Y0-2 .. 2Y0+2W of a plane
    __shared__ T rs[2][W + 1][NF];      // r(2Y-1) of each row slot
    __shared__ T eb[2][W + 1][S];       // last element of each segment of r(2Y)
    const RowGrid g{NF, NF - 1};
    const RowGrid gc{nc, nc - 1};
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int wr = w / S, seg = w - wr * S;
    const int ps = (seg + S - 1) % S, ns = (seg + 1) % S;  // neighbouring segments (periodic)
    const bool comb = wr < W;
    const int Y = yb * W + wr;
    const int fa = 2 * Y - 1, fb = 2 * Y;  // rows outside [0, n) wrap in g.row
    const int ia = 2 * wr + 1, ib = 2 * wr + 2;  // their rows in xs
    const size_t off = (size_t)seg * NR + (size_t)lane * VEC;
    const int so = seg * NR;  // the segment in an LDS row
    const int Z0 = zc * nzc;
    const int nf = 2 * nzc + 1;
    int z = 2 * Z0 - 1;
    // x-halo of a row segment (lane 0: the previous segment's last element,
    // lane 63: the next segment's first)
    auto halo = [&](const T* row) -> T {
        if constexpr (S == 1) {
            return T(0);
        } else {
            return lane < 32 ? lds_elem<T, VEC>(row + ps * NR, NR - 1) : lds_elem<T, VEC>(row + ns * NR, 0);
        }
    };
    // x rows at z-1, z, z+1 and the prefetched z+2 (a: fa, b: fb); slot 0's row
    // 2Y0-2 at z+1 (tp, published next) and the prefetched one (tq)
    T am[VEC], ac[VEC], ap[VEC], an[VEC], bm[VEC], bc[VEC], bp[VEC], bn[VEC], tp[VEC] = {}, tq[VEC] = {};
    // b rows at z and the prefetched z+1
    T ga[VEC], gb[VEC], gan[VEC], gbn[VEC];
    ldrow<T, VEC>(am, x + g.row(fa, z - 1) + off);
    ldrow<T, VEC>(ac, x + g.row(fa, z) + off);
    ldrow<T, VEC>(ap, x + g.row(fa, z + 1) + off);
    ldrow<T, VEC>(bm, x + g.row(fb, z - 1) + off);
    ldrow<T, VEC>(bc, x + g.row(fb, z) + off);
    ldrow<T, VEC>(bp, x + g.row(fb, z + 1) + off);
    ldrow<T, VEC>(ga, b + g.row(fa, z) + off);
    if (comb) ldrow<T, VEC>(gb, b + g.row(fb, z) + off);
    if (wr == 0) {
        ldrow<T, VEC>(tq, x + g.row(fa - 1, z) + off);
        ldrow<T, VEC>(tp, x + g.row(fa - 1, z + 1) + off);
    }
    lds_strow<T, VEC>(xs[z & 1][ia] + so, lane, ac);
    lds_strow<T, VEC>(xs[z & 1][ib] + so, lane, bc);
    if (wr == 0) lds_strow<T, VEC>(xs[z & 1][0] + so, lane, tq);
    __syncthreads();
    T acc[CV];
    for (int k = 0; k < nf; ++k, ++z) {
        const bool more = k + 1 < nf;
        const int cb = z & 1;
        if (more) {  // the plane after next (x) and the next plane (b), one iteration early
            ldrow<T, VEC>(an, x + g.row(fa, z + 2) + off);
            ldrow<T, VEC>(bn, x + g.row(fb, z + 2) + off);
            ldrow<T, VEC>(gan, b + g.row(fa, z + 1) + off);
            if (comb) ldrow<T, VEC>(gbn, b + g.row(fb, z + 1) + off);
            if (wr == 0) ldrow<T, VEC>(tq, x + g.row(fa - 1, z + 2) + off);
            // publish plane z + 1 (its slot was last read before the previous barrier)
            lds_strow<T, VEC>(xs[cb ^ 1][ia] + so, lane, ap);
            lds_strow<T, VEC>(xs[cb ^ 1][ib] + so, lane, bp);
            if (wr == 0) lds_strow<T, VEC>(xs[cb ^ 1][0] + so, lane, tp);
        }
        // r(fa) = b - M x: y-neighbours row fa-1 (xs) and fb (own)
        T ym[VEC], Ma[VEC], ra[VEC];
        lds_ldrow<T, VEC>(ym, xs[cb][ia - 1] + so, lane);
        flat7_row_seg<T, VEC, S>(ac, ym, bc, am, ap, ih2, Ma, halo(xs[cb][ia]));
#pragma unroll
        for (int e = 0; e < VEC; ++e) ra[e] = ga[e] - Ma[e];
        lds_strow<T, VEC>(rs[cb][wr] + so, lane, ra);
        T rb[VEC];
        if (comb) {  // r(fb): y-neighbours fa (own) and fb+1 (xs)
            T yp[VEC], Mb[VEC];
            lds_ldrow<T, VEC>(yp, xs[cb][ib + 1] + so, lane);
            flat7_row_seg<T, VEC, S>(bc, ac, yp, bm, bp, ih2, Mb, halo(xs[cb][ib]));
#pragma unroll
            for (int e = 0; e < VEC; ++e) rb[e] = gb[e] - Mb[e];
            if constexpr (S > 1) {
                if (lane == 63) eb[cb][wr][seg] = rb[VEC - 1];
            }
        }
        __syncthreads();
        if (comb) {
            T rc[VEC], s[VEC];
            lds_ldrow<T, VEC>(rc, rs[cb][wr + 1] + so, lane);
#pragma unroll
            for (int e = 0; e < VEC; ++e) s[e] = fw3<T>(ra[e], rb[e], rc[e]);
            // x: coarse element q <-> fine 2q; needs fine 2q-1 (previous lane's last for q = 0;
            // for lane 0 of a split row, the previous segment's last, formed again from LDS)
            T lft = lane_rot(s[VEC - 1], -1);
            if constexpr (S > 1) {
                if (lane == 0)
                    lft = fw3<T>(lds_elem<T, VEC>(rs[cb][wr] + ps * NR, NR - 1), eb[cb][wr][ps],
                                 lds_elem<T, VEC>(rs[cb][wr + 1] + ps * NR, NR - 1));
            }
            T sx[CV];
#pragma unroll
            for (int q = 0; q < CV; ++q) {
                const T l = q > 0 ? s[2 * q - 1] : lft;
                sx[q] = fw3<T>(l, s[2 * q], s[2 * q + 1]);
            }
            // z: odd fine plane 2Z-1 opens coarse plane Z, 2Z adds 1/2, 2Z+1 closes it
            const bool odd = (k & 1) == 0;  // k = 0 <-> z = 2 Z0 - 1
            if (k == 0) {
#pragma unroll
                for (int q = 0; q < CV; ++q) acc[q] = T(0.25) * sx[q];
            } else if (!odd) {
#pragma unroll
                for (int q = 0; q < CV; ++q) acc[q] += T(0.5) * sx[q];
            } else {
                const int Zc = (z - 1) >> 1;
#pragma unroll
                for (int q = 0; q < CV; ++q) acc[q] += T(0.25) * sx[q];
                strow<T, CV>(coarse + gc.row(Y, Zc) + (size_t)seg * (NR / 2) + (size_t)lane * CV, acc);
#pragma unroll
                for (int q = 0; q < CV; ++q) acc[q] = T(0.25) * sx[q];
            }
        }
        if (more) {
            copyrow(am, ac);
            copyrow(ac, ap);
            copyrow(ap, an);
            copyrow(bm, bc);
            copyrow(bc, bp);
            copyrow(bp, bn);
            copyrow(ga, gan);
            if (comb) copyrow(gb, gbn);
            if (wr == 0) copyrow(tp, tq);
        }
    }
}

// =====================================================================================
// Trilinear prolongation + correction: x (fine row y, plane z) += P e
// =====================================================================================
template <typename T, int VEC>
__device__ __forceinline__ void coarse_seg(T (&v)[VEC / 2 + 1], const T* row, int lane) {
    constexpr int CV = VEC / 2;
    T t[CV];
    ldrow<T, CV>(t, row + (size_t)lane * CV);
#pragma unroll
    for (int q = 0; q < CV; ++q) v[q] = t[q];
    v[CV] = lane_rot(t[0], 1);
}

// S > 1: rows split into S segments, one per wave (rows over 2 KB), with the
// segment-aware coarse loads of the fused pair.  The next plane's x row and
// coarse rows are loaded before the current plane is combined and stored.
template <typename T, int VEC, int S = 1>
__global__ __launch_bounds__(kBlock) void k_prolong_row(int n, const T* __restrict__ e, T* __restrict__ x, int nz,
                                                        int nyb) {
    static_assert(kWaves % S == 0, "a block holds whole rows");
    static_assert(S == 1 || VEC >= 2, "split rows hold at least two fine points per lane");
    constexpr int NR = 64 * VEC, NF = NR * S, nc = NF / 2;
    using Coarse = typename std::conditional<(S > 1), CoarseSeg<T, VEC>, CoarseRows<T, VEC>>::type;
    const RowGrid g{NF, NF - 1};
    const RowGrid gc{nc, nc - 1};
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int y = yb * (kWaves / S) + w / S, seg = w % S;
    const int z0 = zc * nz;
    const size_t off = (size_t)seg * NR + (size_t)lane * VEC;
    auto load = [&](T (&xv)[VEC], Coarse& c, int z) {
        ldrow<T, VEC>(xv, x + g.row(y, z) + off);
        if constexpr (S > 1) coarse_load_seg<T, VEC>(c, e, gc, y, z, seg, lane);
        else coarse_load<T, VEC>(c, e, gc, y, z, lane);
    };
    T xv[VEC];
    Coarse c;
    load(xv, c, z0);
    for (int k = 0; k < nz; ++k) {
        const int z = z0 + k;
        T xn[VEC];
        Coarse cn;
        if (k + 1 < nz) load(xn, cn, z + 1);
        if constexpr (S > 1) prolong_add_seg<T, VEC>(xv, c, y, z);
        else prolong_add<T, VEC>(xv, c, y, z);
        strow<T, VEC>(x + g.row(y, z) + off, xv);
        copyrow(xv, xn);
        c = cn;
    }
}

// ---- launch shapes -------------------------------------------------------------------
// rows of the (n x n) plane grouped four per block; z split into chunks of nz
// planes so that about `target` blocks are launched.  Every launch shape is a
// function of n and the element size only, so two contexts in one process
// never see different shapes.
constexpr int kTargetBlocks = 8192;

// Kernels whose working set does not fit the Infinity Cache (the outer
// residual with its double fields, residual + restriction) take longer z
// chunks: each chunk re-reads the planes of its z-neighbour queue, and the
// counters showed 36% extra fetch at the short chunk length.
void shape(int rows, int planes, int min_nz, int& nz, int& nyb, int& blocks, int target = 0) {
    nyb = rows / kWaves;
    if (target == 0) target = kTargetBlocks;
    nz = planes;
    while (nz > min_nz && (long)nyb * (planes / nz) < target) nz >>= 1;
    blocks = nyb * (planes / nz);
}

constexpr int kLdsWaves = 8;
constexpr size_t kLdsBudget = 80 * 1024;
constexpr size_t kOuterSegLdsBudget = 96 * 1024;
template <typename T>
bool lds_rows_fit(int n) {
    return 2ull * (kLdsWaves + 2) * (size_t)n * sizeof(T) <= kLdsBudget;
}

}  // namespace

bool row_kernels_apply(int n) { return n >= 64 && n <= 1024 && (n & (n - 1)) == 0; }

// block count the residual + restriction kernel's chunks aim for on levels of
// 256^3 and more (256^3: 512 blocks 22.6 us, 1024 blocks 25.2 us, 256 blocks 28.9 us)
constexpr int kRrTarget = 512;

// Longest z chunks that still give one block of kLdsWaves waves per CU: the
// outer kernel is bound by its bytes, and a chunk re-reads its two halo planes
// (256^3: chunks of 32 planes 103.6 us against 107.8 us for 16; 16-wave
// blocks measured slower).
void outer_lds_shape(int n, int waves, int& nz, int& nyb, int& blocks) {
    nyb = n / waves;
    nz = n;
    while (nz > 16 && nyb * (n / nz) < 256) nz >>= 1;
    blocks = nyb * (n / nz);
}

// The outer residual runs in double (TA) for MG_FP64/MG_MIXED and float for
// MG_FP32; the block count must match what launch_outer_row uses.
// Segments per row of the kernels that keep their rows in registers without
// LDS (single step, outer residual): rows of more than 2 KB are split so that
// a lane holds at most 32 bytes (1024^3 double: 4 segments of 2 KB; a lane of
// an unsplit 8 KB row held 128 bytes, and these kernels ran one wave per SIMD).
constexpr size_t kRowSegBytes = 2048;
inline int row_segments(int n, size_t elem) {
    const size_t row = (size_t)n * elem;
    return row > kRowSegBytes ? (int)(row / kRowSegBytes) : 1;
}

// Rows of at least kOuterSegMinRow bytes (512^3 and 1024^3 double): blocks
// of 16 waves, 16 / S rows each split into S segments of 2 KB, the rows still
// shared through LDS (96 KB for 4 rows + 2 halo rows of 8 KB,
// double-buffered).  1024^3 outer residual against the row kernel without
// LDS: mixed 3.9 -> 5.4 TB/s, FP64 3.8 -> 5.3 TB/s (2 rows per block: 4.9);
// 512^3 against unsplit 4 KB rows in 8-wave blocks: 5.22 -> 5.41 TB/s mixed,
// 5.14 -> 5.38 TB/s FP64.
// Float arithmetic (the pure FP32 solver) keeps VEC = 8 per lane and needs
// more registers than 16-wave blocks leave (it spilled): blocks of 8 waves.
constexpr int outer_seg_waves(size_t elem) { return elem == sizeof(double) ? 16 : 8; }
constexpr size_t kOuterSegMinRow = 4096;
inline bool outer_seg_lds(int n, size_t elem) {
    const int S = row_segments(n, elem), waves = outer_seg_waves(elem);
    return S > 1 && (size_t)n * elem >= kOuterSegMinRow && waves % S == 0 &&
           2ull * (waves / S + 2) * n * elem <= kOuterSegLdsBudget;
}

int row_outer_blocks(int n, bool double_arith) {
    int nz, nyb, blocks;
    const size_t elem = double_arith ? sizeof(double) : sizeof(float);
    if (outer_seg_lds(n, elem)) {
        outer_lds_shape(n, outer_seg_waves(elem) / row_segments(n, elem), nz, nyb, blocks);
        return blocks;
    }
    if (double_arith ? lds_rows_fit<double>(n) : lds_rows_fit<float>(n)) {
        outer_lds_shape(n, kLdsWaves, nz, nyb, blocks);
        return blocks;
    }
    shape(n * row_segments(n, double_arith ? sizeof(double) : sizeof(float)), n, 16, nz, nyb, blocks, 1024);
    return blocks;
}

// Row kernel with S segments per row: VEC = n / (64 S) elements per lane.
#define DISPATCH_SEG(n, S, ...)                                                \
    switch ((n) / (64 * (S))) {                                                \
        case 4: { constexpr int VEC = 4; __VA_ARGS__; break; }                 \
        case 8: { constexpr int VEC = 8; __VA_ARGS__; break; }                 \
        default: return hipErrorInvalidValue;                                  \
    }

#define DISPATCH_VEC(n, ...)                                  \
    switch (n) {                                              \
        case 64: { constexpr int VEC = 1; __VA_ARGS__; break; }   \
        case 128: { constexpr int VEC = 2; __VA_ARGS__; break; }  \
        case 256: { constexpr int VEC = 4; __VA_ARGS__; break; }  \
        case 512: { constexpr int VEC = 8; __VA_ARGS__; break; }  \
        case 1024: { constexpr int VEC = 16; __VA_ARGS__; break; } \
        default: return hipErrorInvalidValue;                 \
    }

// Single steps on rows over 2 KB (1024^3 float, 512^3 and 1024^3 double):
// rows split into S segments of 2 KB, one wave each, in blocks of 16 waves
// (16 / S rows), the rows still shared through LDS; kStepSegTarget blocks per
// launch at least.  Against the segments without LDS (1024^3 double) or the
// unsplit LDS rows: 1024^3 double 3.9 -> 4.9 TB/s, 512^3 double 5.0 -> 5.3,
// 1024^3 float 5.05 -> 5.18 TB/s (blocks of 8 waves: 4.9, 5.2, 5.0 TB/s).
constexpr int kStepSegWaves = 16;
constexpr int kStepSegTarget = 1024;
constexpr size_t kStepSegLdsBudget = 96 * 1024;
inline bool step_seg_lds(int n, size_t elem) {
    const int S = row_segments(n, elem);
    return S > 1 && kStepSegWaves % S == 0 && 2ull * (kStepSegWaves / S + 2) * n * elem <= kStepSegLdsBudget;
}
// The first two post-smoothing steps with the prolongation formed on the fly
// (steps of the split LDS kernel with the coarse rows as well).  The step
// that prolongs fits 128 VGPRs and takes 16-wave blocks like the plain steps
// (1024^3 FP64 65.9 -> 65.2 ms per cycle against 8 waves); the step that
// forms x_prev = x + P e needs more and takes blocks of 8 waves (16 spilled).
constexpr int kStepProWaves = 16;
constexpr int kStepPrevpWaves = 8;
bool step_pro_applies(int n, size_t elem) {
    const int S = row_segments(n, elem);
    return step_seg_lds(n, elem) && kStepProWaves % S == 0 && kStepPrevpWaves % S == 0;
}

// Single smoothing step, in one of five modes: MODE_PLAIN (x, [x_prev], b),
// MODE_FROMB (step 1 of a pass from zero, from b alone: the iterate is the
// pointwise first step cd0 b, x_prev = 0), MODE_PREVB (step 2 of such a
// pass: x_prev is cd0 b, formed from the b rows), MODE_PRO (step 0 of a
// post-smoothing pass from x + P e, formed on the fly) and MODE_PREVP (step
// 1 of that pass: x_prev = x + P e formed pointwise from the old iterate).
enum StepMode { MODE_PLAIN, MODE_FROMB, MODE_PREVB, MODE_PRO, MODE_PREVP };
template <typename T, int MODE>
hipError_t launch_step_mode(int n, double ih2, const T* x, const T* xprev, const T* b, T* out, double a, double cd,
                            double cd0, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, const T* ec = nullptr) {
    constexpr bool FB = MODE == MODE_FROMB, PB = MODE == MODE_PREVB, PR = MODE == MODE_PRO,
                   PP = MODE == MODE_PREVP;
    int nz, nyb, blocks;
    // Rows over 2 KB with LDS room for 16 / S of them: split into 2 KB
    // segments, one wave each, the rows still shared through LDS.  The steps
    // that prolong on the fly hold the coarse rows as well: blocks of 8 waves.
    if (x != nullptr && step_seg_lds(n, sizeof(T))) {
        const int S = row_segments(n, sizeof(T));
        const int waves = PR ? kStepProWaves : PP ? kStepPrevpWaves : kStepSegWaves;
        nyb = n / (waves / S);
        nz = n;
        while (nz > 4 && nyb * (n / nz) < kStepSegTarget) nz >>= 1;
        blocks = nyb * (n / nz);
#define MG_STEP_SEGLDS(SS)                                                                                        \
    DISPATCH_SEG(n, SS, {                                                                                         \
        constexpr int Wr = (PR ? kStepProWaves : PP ? kStepPrevpWaves : kStepSegWaves) / SS;                      \
        if constexpr (2ull * (Wr + 2) * 64 * VEC * SS * sizeof(T) <= kStepSegLdsBudget) {                         \
            if constexpr (PR)                                                                                     \
                MG_LAUNCH((k_smooth_lds<T, VEC, Wr, false, false, false, SS, true>), dim3(blocks),                \
                          dim3(64 * Wr * SS), s, ev0, ev1, n, (T)ih2, x, xprev, b, out, (T)a, (T)cd, nz, nyb,     \
                          (T)cd0, ec);                                                                            \
            else if constexpr (PP)                                                                                \
                MG_LAUNCH((k_smooth_lds<T, VEC, Wr, true, false, false, SS, false, true>), dim3(blocks),          \
                          dim3(64 * Wr * SS), s, ev0, ev1, n, (T)ih2, x, xprev, b, out, (T)a, (T)cd, nz, nyb,     \
                          (T)cd0, ec);                                                                            \
            else if (xprev == nullptr && !PB)                                                                     \
                MG_LAUNCH((k_smooth_lds<T, VEC, Wr, false, FB, false, SS>), dim3(blocks), dim3(64 * Wr * SS), s,  \
                          ev0, ev1, n, (T)ih2, x, xprev, b, out, (T)a, (T)cd, nz, nyb, (T)cd0, ec);               \
            else if constexpr (!FB)                                                                               \
                MG_LAUNCH((k_smooth_lds<T, VEC, Wr, true, false, PB, SS>), dim3(blocks), dim3(64 * Wr * SS), s,   \
                          ev0, ev1, n, (T)ih2, x, xprev, b, out, (T)a, (T)cd, nz, nyb, (T)cd0, ec);               \
        } else {                                                                                                  \
            return hipErrorInvalidValue;                                                                          \
        }                                                                                                         \
    })
        switch (S) {
            case 2: MG_STEP_SEGLDS(2); break;
            case 4: MG_STEP_SEGLDS(4); break;
            default: return hipErrorInvalidValue;
        }
#undef MG_STEP_SEGLDS
        return hipGetLastError();
    }
    if constexpr (PR || PP) return hipErrorInvalidValue;  // split rows with LDS only
    // Row sharing through LDS pays where the level's fields exceed the 256 MB
    // Infinity Cache (n >= 512); below that the y-halo rows already hit in
    // cache and the per-plane barrier costs more than it saves (measured).
    if (x != nullptr && n >= 512 && lds_rows_fit<T>(n)) {
        constexpr int Wv = kLdsWaves;
        nyb = n / Wv;
        nz = n;
        while (nz > 4 && nyb * (n / nz) < 2048) nz >>= 1;
        blocks = nyb * (n / nz);
        DISPATCH_VEC(n, {
            if constexpr (2ull * (Wv + 2) * 64 * VEC * sizeof(T) <= kLdsBudget) {
                if (xprev == nullptr && !PB)
                    MG_LAUNCH((k_smooth_lds<T, VEC, Wv, false, FB>), dim3(blocks), dim3(64 * Wv), s, ev0, ev1, n,
                              (T)ih2, x, xprev, b, out, (T)a, (T)cd, nz, nyb, (T)cd0, ec);
                else if constexpr (!FB)
                    MG_LAUNCH((k_smooth_lds<T, VEC, Wv, true, false, PB>), dim3(blocks), dim3(64 * Wv), s, ev0,
                              ev1, n, (T)ih2, x, xprev, b, out, (T)a, (T)cd, nz, nyb, (T)cd0, ec);
            }
        })
        return hipGetLastError();
    }
    const int S = x != nullptr ? row_segments(n, sizeof(T)) : 1;
    if (S > 1) {
        shape(n * S, n, 4, nz, nyb, blocks);
#define MG_SMOOTH_SEG(SS)                                                                                       \
    DISPATCH_SEG(n, SS, {                                                                                       \
        if (xprev == nullptr && !PB)                                                                            \
            MG_LAUNCH((k_smooth_row<T, VEC, true, false, SS, FB>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n,  \
                      (T)ih2, x, xprev, b, out, (T)a, (T)cd, nz, nyb, (T)cd0);                                  \
        else if constexpr (!FB)                                                                                 \
            MG_LAUNCH((k_smooth_row<T, VEC, true, true, SS, false, PB>), dim3(blocks), dim3(kBlock), s, ev0,   \
                      ev1, n, (T)ih2, x, xprev, b, out, (T)a, (T)cd, nz, nyb, (T)cd0);                          \
    })
        switch (S) {
            case 2: MG_SMOOTH_SEG(2); break;
            case 4: MG_SMOOTH_SEG(4); break;
            default: return hipErrorInvalidValue;
        }
#undef MG_SMOOTH_SEG
        return hipGetLastError();
    }
    shape(n, n, 4, nz, nyb, blocks);
    DISPATCH_VEC(n, {
        if (x == nullptr) {
            if constexpr (MODE == MODE_PLAIN)
                MG_LAUNCH((k_smooth_row<T, VEC, false, false>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, (T)ih2,
                          x, xprev, b, out, (T)a, (T)cd, nz, nyb, (T)cd0);
        } else if (xprev == nullptr && !PB) {
            MG_LAUNCH((k_smooth_row<T, VEC, true, false, 1, FB>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n,
                      (T)ih2, x, xprev, b, out, (T)a, (T)cd, nz, nyb, (T)cd0);
        } else if constexpr (!FB) {
            MG_LAUNCH((k_smooth_row<T, VEC, true, true, 1, false, PB>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n,
                      (T)ih2, x, xprev, b, out, (T)a, (T)cd, nz, nyb, (T)cd0);
        }
    })
    return hipGetLastError();
}

template <typename T>
hipError_t launch_smooth_row(int n, double ih2, const T* x, const T* xprev, const T* b, T* out, double a,
                             double cd, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    return launch_step_mode<T, MODE_PLAIN>(n, ih2, x, xprev, b, out, a, cd, 0.0, s, ev0, ev1);
}

template <typename T>
hipError_t launch_smooth_fromb_row(int n, double ih2, const T* b, T* out, double a1, double cd1, double cd0,
                                   hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (b == nullptr || out == b) return hipErrorInvalidValue;
    return launch_step_mode<T, MODE_FROMB>(n, ih2, b, nullptr, b, out, a1, cd1, cd0, s, ev0, ev1);
}

template <typename T>
hipError_t launch_smooth_prevb_row(int n, double ih2, const T* x, const T* b, T* out, double a2, double cd2,
                                   double cd0, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (x == nullptr || b == nullptr || out == x || out == b) return hipErrorInvalidValue;
    return launch_step_mode<T, MODE_PREVB>(n, ih2, x, nullptr, b, out, a2, cd2, cd0, s, ev0, ev1);
}

// Step 0 of a post-smoothing pass from x0 = x + P e (x_prev = 0), x0 formed
// on the fly: out = x1.  Rows over 2 KB only (step_pro_applies).
template <typename T>
hipError_t launch_smooth_pro_row(int n, double ih2, const T* x, const T* e, const T* b, T* out, double a0,
                                 double cd0, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (!step_pro_applies(n, sizeof(T)) || !x || !e || !b || out == x || out == b) return hipErrorInvalidValue;
    return launch_step_mode<T, MODE_PRO>(n, ih2, x, nullptr, b, out, a0, cd0, 0.0, s, ev0, ev1, e);
}

// Step 1 of that pass: x_prev = x0 = xold + P e formed pointwise; out may be xold.
template <typename T>
hipError_t launch_smooth_prevp_row(int n, double ih2, const T* x1, const T* xold, const T* e, const T* b, T* out,
                                   double a1, double cd1, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (!step_pro_applies(n, sizeof(T)) || !x1 || !xold || !e || !b || out == x1 || out == b)
        return hipErrorInvalidValue;
    return launch_step_mode<T, MODE_PREVP>(n, ih2, x1, xold, b, out, a1, cd1, 0.0, s, ev0, ev1, e);
}

// Waves per block of the two-step kernel (W = waves - 2 output rows): 8
// (measured best of 8, 12 and 16 on the 256^3 sequence: 37.4 vs 37.7 vs
// 38.0 ms).  The pass from zero picks its own block by row size.
constexpr int kPairWavesDefault = 8;
constexpr size_t kPairLdsBudget = 64 * 1024;
constexpr int kPairUnrollNz = 8;  // chunk height of the fully unrolled two-step variant
// Prefetch depth of the two-step kernel: two planes ahead for 2 KB rows,
// whose blocks run one per CU (512^3 float 541 -> 498 us per launch); one
// plane for smaller rows, where the extra registers cost occupancy (256^3
// float 53 -> 61 us).  The pass from zero reads one field (b), so its
// unrolled variant prefetches two planes ahead at the same occupancy
// (256^3: 40.3 -> 37.7 us, 128^3: 9.5 -> 8.7 us per launch).

// Largest row (bytes) whose two-step kernel fits a wave's registers without
// spilling: 8-wave blocks leave a wave 256 VGPRs (float n <= 512, double
// n <= 256), 12- and 16-wave blocks 170 / 128 (float n <= 256, double n <= 128).
constexpr size_t pair_max_row_bytes(int waves) { return waves <= 8 ? 2048 : 1024; }

bool pair_kernels_apply(int n, size_t elem) {
    return row_kernels_apply(n) && (size_t)n * elem <= pair_max_row_bytes(kPairWavesDefault) &&
           2ull * kPairWavesDefault * (size_t)n * elem <= kPairLdsBudget;
}

// launch of one k_smooth2_lds variant inside launch_pair_nw (VEC from DISPATCH_VEC)
#define MG_PAIR1(PREV1, Y1OUT, FROMB, PF2, NZC, PREVB)                                                           \
    MG_LAUNCH((k_smooth2_lds<T, VEC, NW, PREV1, Y1OUT, FROMB, PF2, NZC, 1, PREVB>),                                 \
              dim3(blocks + ((FROMB || PREVB) ? extra : 0)), dim3(64 * NW), s, ev0, ev1, n, (T)ih2, x, xp, b, y2, \
              y1, (T)a1, (T)cd1, (T)a2, (T)cd2, nz, nyb, (T)cd0, (FROMB || PREVB) ? sums : SumsJob{})
#define MG_PAIRB(PREV1, Y1OUT, FROMB, PREVB)                                                     \
    do {                                                                                         \
        if (pf2) MG_PAIR1(PREV1, Y1OUT, FROMB, true, 0, PREVB);                                  \
        else if (nz == kPairUnrollNz) MG_PAIR1(PREV1, Y1OUT, FROMB, false, kPairUnrollNz, PREVB); \
        else MG_PAIR1(PREV1, Y1OUT, FROMB, false, 0, PREVB);                                     \
    } while (0)
#define MG_PAIR(PREV1, Y1OUT, FROMB) MG_PAIRB(PREV1, Y1OUT, FROMB, false)

template <typename T, int NW>
hipError_t launch_pair_nw(int n, double ih2, const T* x, const T* xp, const T* b, T* y2, T* y1, double a1, double cd1,
                          double a2, double cd2, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, int x0_mode,
                          double cd0, const SumsJob& sums) {
    const int extra = sums.count > 0 ? 1 : 0;  // the block that finishes the sums (pass from zero only)
    constexpr int W = NW - 2;
    const int nyb = (n + W - 1) / W;
    // about 1000 blocks, z chunks of at least 8 planes; 64^3: chunks of 4
    // planes (pass from zero 6.1 -> 5.0 us per launch)
    int nz = n;
    const int min_nz = n <= 64 ? 4 : 8;
    while (nz > min_nz && (long)nyb * (n / nz) < 1024) nz >>= 1;
    const int blocks = nyb * (n / nz);
    const bool pf2 = (size_t)n * sizeof(T) >= 2048;
    DISPATCH_VEC(n, {
        if constexpr (64 * VEC * sizeof(T) <= pair_max_row_bytes(NW) && 2ull * NW * 64 * VEC * sizeof(T) <= kPairLdsBudget) {
            if (x0_mode == 2) {
                MG_PAIRB(true, false, false, true);
            } else if (x0_mode != 0) {
                if (!pf2 && nz == kPairUnrollNz) {
                    if (y1 == nullptr) MG_PAIR1(false, false, true, true, kPairUnrollNz, false);
                    else MG_PAIR1(false, true, true, true, kPairUnrollNz, false);
                } else if (y1 == nullptr) MG_PAIR(false, false, true);
                else MG_PAIR(false, true, true);
            } else if (xp == nullptr && y1 == nullptr) {
                MG_PAIR(false, false, false);
            } else if (xp == nullptr) {
                MG_PAIR(false, true, false);
            } else if (y1 == nullptr) {
                MG_PAIR(true, false, false);
            } else {
                MG_PAIR(true, true, false);
            }
        } else {
            return hipErrorInvalidValue;  // row does not fit this block's register or LDS budget
        }
    })
    return hipGetLastError();
}
#undef MG_PAIR
#undef MG_PAIRB
#undef MG_PAIR1

// Rows longer than kPairSegBytes run the two-step kernels split into segments
// of that many bytes, one wave each, with the block shape of the 1 KB rows of
// 256^3 float (16 waves = 8 rows): a lane then holds 16 bytes of a row, and
// the register budget of 16-wave blocks holds the fully unrolled variants.
// A chunk of NZC output planes reads NZC + 4 planes of x and NZC + 2 of b and
// x_prev; chunks of 16 planes instead of 8 cut the fetch of the first step's
// z halo: 512^3 float pairs 4.45 -> 4.63 TB/s, 256^3 double 3.97 -> 4.31 TB/s
// (32 planes: 4.58 TB/s at 512^3), same bits.
constexpr size_t kPairSegBytes = 1024;
constexpr int kPairSegWaves = 16;  // block of the split two-step kernels
constexpr int kPairSegNz = 16;     // their (fully unrolled) chunk height
// rows loaded two planes ahead of their use (not with the prolongation in
// double, where the second register set spilled)
constexpr bool kPairXPf = true;
// x plane of the split two-step kernels shared through LDS (k_smooth2x_lds):
// 512^3 float pairs 4.07 -> 4.45 TB/s, 256^3 double 3.74 -> 3.98 TB/s, same
// bits.  Unsplit 1 KB rows keep k_smooth2_lds: the 256^3 float pass from zero
// measured 37.9 us there against 40.6 us in this kernel and block shape.
constexpr bool kPairXLds = true;
inline int pair_segments(int n, size_t elem) {
    const size_t row = (size_t)n * elem;
    return row > kPairSegBytes ? (int)(row / kPairSegBytes) : 1;
}

// The prolongation runs fused into the first pair of a post-smoothing pass on
// split rows (512^3 float, 256^3 double).
bool pair_pro_applies(int n, size_t elem) {
    return kPairXLds && pair_kernels_apply(n, elem) && pair_segments(n, elem) == 2;
}

#define MG_PAIRS(PREV1, Y1OUT, FROMB, PF2, PREVB, PRO)                                                             \
    do {                                                                                                         \
        constexpr bool JOB = FROMB || PREVB;                                                                     \
        if constexpr (kPairXLds)                                                                                 \
            MG_LAUNCH((k_smooth2x_lds<T, VEC, NW, PREV1, Y1OUT, FROMB, kPairSegNz, S, PREVB, PRO,                \
                                      kPairXPf && !(PRO && sizeof(T) == sizeof(double))>),                     \
                      dim3(blocks + (JOB ? extra : 0)), dim3(64 * NW), s, ev0, ev1, n, (T)ih2, x, xp, b, y2, y1,   \
                      (T)a1, (T)cd1, (T)a2, (T)cd2, nyb, (T)cd0, JOB ? sums : SumsJob{}, ec);                    \
        else                                                                                                     \
            MG_LAUNCH((k_smooth2_lds<T, VEC, NW, PREV1, Y1OUT, FROMB, PF2, kPairSegNz, S, PREVB>),               \
                      dim3(blocks + (JOB ? extra : 0)), dim3(64 * NW), s, ev0, ev1, n, (T)ih2, x, xp, b, y2, y1,   \
                      (T)a1, (T)cd1, (T)a2, (T)cd2, kPairSegNz, nyb, (T)cd0, JOB ? sums : SumsJob{});            \
    } while (0)
template <typename T, int NW, int S>
hipError_t launch_pair_seg(int n, double ih2, const T* x, const T* xp, const T* b, T* y2, T* y1, double a1,
                           double cd1, double a2, double cd2, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                           int x0_mode, double cd0, const SumsJob& sums, const T* ec) {
    constexpr int W = NW / S - 2;
    const int extra = sums.count > 0 ? 1 : 0;  // the block that finishes the sums (pass from zero only)
    const int nyb = (n + W - 1) / W;
    if (n % kPairSegNz != 0) return hipErrorInvalidValue;
    const int blocks = nyb * (n / kPairSegNz);
    const int vec = n / (64 * S);
    auto go = [&](auto vtag) -> hipError_t {
        constexpr int VEC = decltype(vtag)::value;
        if constexpr (VEC * sizeof(T) <= 16 && 2ull * NW * 64 * VEC * sizeof(T) <= kPairLdsBudget) {
            if (ec != nullptr) {
                if constexpr (VEC >= 2) {
                    if (y1 == nullptr) MG_PAIRS(false, false, false, false, false, true);
                    else MG_PAIRS(false, true, false, false, false, true);
                } else {
                    return hipErrorInvalidValue;
                }
            } else if (x0_mode == 2) {
                MG_PAIRS(true, false, false, false, true, false);
            } else if (x0_mode != 0) {
                if (y1 == nullptr) MG_PAIRS(false, false, true, true, false, false);
                else MG_PAIRS(false, true, true, true, false, false);
            } else if (xp == nullptr && y1 == nullptr) {
                MG_PAIRS(false, false, false, false, false, false);
            } else if (xp == nullptr) {
                MG_PAIRS(false, true, false, false, false, false);
            } else if (y1 == nullptr) {
                MG_PAIRS(true, false, false, false, false, false);
            } else {
                MG_PAIRS(true, true, false, false, false, false);
            }
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    };
    switch (vec) {
        case 2: return go(std::integral_constant<int, 2>{});
        case 4: return go(std::integral_constant<int, 4>{});
        default: return hipErrorInvalidValue;
    }
}
#undef MG_PAIRS

template <typename T>
hipError_t launch_smooth_pair_row(int n, double ih2, const T* x, const T* xp, const T* b, T* y2, T* y1,
                                  double a1, double cd1, double a2, double cd2, hipStream_t s, hipEvent_t ev0,
                                  hipEvent_t ev1, int x0_mode, double cd0, const SumsJob* sums_job, const T* ec) {
    if (!pair_kernels_apply(n, sizeof(T))) return hipErrorInvalidValue;
    if (ec != nullptr && (!pair_pro_applies(n, sizeof(T)) || x0_mode != 0 || xp != nullptr || x == nullptr))
        return hipErrorInvalidValue;
    const SumsJob sums = sums_job ? *sums_job : SumsJob{};
    if (x0_mode < 0 || x0_mode > 2) return hipErrorInvalidValue;
    if (sums.count > 0 && x0_mode == 0) return hipErrorInvalidValue;
    if (x0_mode != 1 && x == nullptr) return hipErrorInvalidValue;
    if (x0_mode != 0 && xp != nullptr) return hipErrorInvalidValue;
    if (x0_mode == 2 && y1 != nullptr) return hipErrorInvalidValue;
    switch (pair_segments(n, sizeof(T))) {
        case 1: break;
        case 2:
            return launch_pair_seg<T, kPairSegWaves, 2>(n, ih2, x, xp, b, y2, y1, a1, cd1, a2, cd2, s, ev0, ev1,
                                                        x0_mode, cd0, sums, ec);
        default: return hipErrorInvalidValue;
    }
    int waves = kPairWavesDefault;
    // The pass from zero (one field read) runs best in larger blocks where the
    // row fits their register budget: 256^3 16 waves 33.8 us (8: 35.4, 12: 38.3),
    // 128^3 12 waves 7.8 us (8: 8.6), 64^3 8 waves.
    if (x0_mode == 1) {
        const size_t row = (size_t)n * sizeof(T);
        waves = (n >= 256 && row <= pair_max_row_bytes(16)) ? 16 : (n >= 128 && row <= pair_max_row_bytes(12)) ? 12 : 8;
        if (2ull * waves * row > kPairLdsBudget) waves = 8;
    }
    if (waves == 8)
        return launch_pair_nw<T, 8>(n, ih2, x, xp, b, y2, y1, a1, cd1, a2, cd2, s, ev0, ev1, x0_mode, cd0, sums);
    if (waves == 12)
        return launch_pair_nw<T, 12>(n, ih2, x, xp, b, y2, y1, a1, cd1, a2, cd2, s, ev0, ev1, x0_mode, cd0, sums);
    return launch_pair_nw<T, 16>(n, ih2, x, xp, b, y2, y1, a1, cd1, a2, cd2, s, ev0, ev1, x0_mode, cd0, sums);
}

// Three-step kernel: 12 waves (8 output rows) per block, chunks of
// kTripleNz planes; rows of at most 1 KB (float n <= 256, double n <= 128).
constexpr int kTripleNz = 8;
// z chunk of the fused post-smoothing pass in 12-wave blocks from 256^3: 16
// planes.  Below 256^3 the chunk is kTripleNz.  A chunk forms step 0 on
// NZC + 4 planes for NZC outputs, and each plane costs a barrier round
// whatever its share of useful work: 256^3 with 12-wave blocks, 8 planes
// 56.1 us, 16 planes 48.5 us, 32 planes 47.5 us (32 planes gave fewer blocks
// than CUs at 128 rows of 8 and measured no better over the whole sequence).
constexpr int kTripleProNzLarge = 16;
// block of the three-step kernels: 8 waves at 64^3, 12 above (measured:
// 64^3 5.7 vs 6.4 us, 128^3 10.1 vs 10.8 us, 256^3 within 1%)
inline int triple_waves(int n) { return n <= 64 ? 8 : 12; }

bool triple_kernels_apply(int n, size_t elem) {
    return row_kernels_apply(n) && (size_t)n * elem <= 1024 && n % kTripleNz == 0;
}

template <typename T, int NW>
hipError_t launch_triple_nw(int n, double ih2, const T* x, const T* b, T* y3, double a0, double cd0, double a1,
                            double cd1, double a2, double cd2, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    constexpr int W = NW - 4;
    const int nyb = (n + W - 1) / W;
    const int blocks = nyb * (n / kTripleNz);
    DISPATCH_VEC(n, {
        if constexpr (64 * VEC * sizeof(T) <= 1024)
            MG_LAUNCH((k_smooth3_lds<T, VEC, NW, kTripleNz>), dim3(blocks), dim3(64 * NW), s, ev0, ev1, n, (T)ih2, x,
                      b, y3, (T)a0, (T)cd0, (T)a1, (T)cd1, (T)a2, (T)cd2, nyb);
    })
    return hipGetLastError();
}

template <typename T>
hipError_t launch_smooth_triple_row(int n, double ih2, const T* x, const T* b, T* y3, double a0, double cd0,
                                    double a1, double cd1, double a2, double cd2, hipStream_t s, hipEvent_t ev0,
                                    hipEvent_t ev1) {
    if (!triple_kernels_apply(n, sizeof(T)) || x == y3 || b == y3) return hipErrorInvalidValue;
    if (triple_waves(n) == 8)
        return launch_triple_nw<T, 8>(n, ih2, x, b, y3, a0, cd0, a1, cd1, a2, cd2, s, ev0, ev1);
    return launch_triple_nw<T, 12>(n, ih2, x, b, y3, a0, cd0, a1, cd1, a2, cd2, s, ev0, ev1);
}
template <typename T, int NW>
hipError_t launch_triple_pro_nw(int n, double ih2, const T* x, const T* e, const T* b, T* y3, double a0, double cd0,
                                double a1, double cd1, double a2, double cd2, hipStream_t s, hipEvent_t ev0,
                                hipEvent_t ev1) {
    constexpr int W = NW - 4;
    const int nyb = (n + W - 1) / W;
    int nzc = kTripleNz;
    if (NW == 12 && n >= 256) nzc = kTripleProNzLarge;
    if (n % nzc != 0) nzc = kTripleNz;
    const int blocks = nyb * (n / nzc);
#define MG_TRIPLE_PRO(NZC)                                                                                       \
    MG_LAUNCH((k_smooth3p_lds<T, VEC, NW, NZC>), dim3(blocks), dim3(64 * NW), s, ev0, ev1, n, (T)ih2, x, e, b, y3, \
              (T)a0, (T)cd0, (T)a1, (T)cd1, (T)a2, (T)cd2, nyb)
    DISPATCH_VEC(n, {
        if constexpr (64 * VEC * sizeof(T) <= 1024) {
            if constexpr (NW == 12) {
                if (nzc == kTripleProNzLarge) MG_TRIPLE_PRO(kTripleProNzLarge);
                else MG_TRIPLE_PRO(kTripleNz);
            } else {
                MG_TRIPLE_PRO(kTripleNz);
            }
        } else {
            return hipErrorInvalidValue;
        }
    })
#undef MG_TRIPLE_PRO
    return hipGetLastError();
}

// From 128^3: at 64^3 the fused pass (11.1 us) is no faster than the
// prolongation and the three-step pass apart (5.0 + 5.8 us).
bool triple_pro_applies(int n, size_t elem) { return n >= 128 && triple_kernels_apply(n, elem); }

template <typename T>
hipError_t launch_prolong_triple_row(int n, double ih2, const T* x, const T* e, const T* b, T* y3, double a0,
                                     double cd0, double a1, double cd1, double a2, double cd2, hipStream_t s,
                                     hipEvent_t ev0, hipEvent_t ev1) {
    if (!triple_pro_applies(n, sizeof(T)) || y3 == x || y3 == b || y3 == e) return hipErrorInvalidValue;
    if (triple_waves(n) == 8)
        return launch_triple_pro_nw<T, 8>(n, ih2, x, e, b, y3, a0, cd0, a1, cd1, a2, cd2, s, ev0, ev1);
    return launch_triple_pro_nw<T, 12>(n, ih2, x, e, b, y3, a0, cd0, a1, cd1, a2, cd2, s, ev0, ev1);
}
template hipError_t launch_prolong_triple_row<float>(int, double, const float*, const float*, const float*, float*,
                                                     double, double, double, double, double, double, hipStream_t,
                                                     hipEvent_t, hipEvent_t);
template hipError_t launch_prolong_triple_row<double>(int, double, const double*, const double*, const double*,
                                                      double*, double, double, double, double, double, double,
                                                      hipStream_t, hipEvent_t, hipEvent_t);

template hipError_t launch_smooth_triple_row<float>(int, double, const float*, const float*, float*, double, double,
                                                    double, double, double, double, hipStream_t, hipEvent_t,
                                                    hipEvent_t);
template hipError_t launch_smooth_triple_row<double>(int, double, const double*, const double*, double*, double,
                                                     double, double, double, double, double, hipStream_t,
                                                     hipEvent_t, hipEvent_t);

template <typename TA, typename TR, typename TE>
hipError_t launch_outer_row(int n, double ih2, const double* phi_in, const TE* e, double* phi_out, const double* b,
                            double bmean, TR* r, TR* x1, double cd0, double* partials, hipStream_t s,
                            hipEvent_t ev0, hipEvent_t ev1) {
    int nz, nyb, blocks;
    if (outer_seg_lds(n, sizeof(TA))) {
        outer_lds_shape(n, outer_seg_waves(sizeof(TA)) / row_segments(n, sizeof(TA)), nz, nyb, blocks);
#define MG_OUTER_SEGLDS(SS)                                                                                          \
    DISPATCH_SEG(n, SS, {                                                                                            \
        constexpr int Wr = outer_seg_waves(sizeof(TA)) / SS;                                                         \
        if constexpr (2ull * (Wr + 2) * 64 * VEC * SS * sizeof(TA) <= kOuterSegLdsBudget) {                          \
            if (e)                                                                                                   \
                MG_LAUNCH((k_outer_lds<TA, TR, TE, VEC, Wr, true, SS>), dim3(blocks), dim3(64 * Wr * SS), s, ev0,  \
                          ev1, n, (TA)ih2, phi_in, e, phi_out, b, bmean, r, x1, (TA)cd0, partials, nz, nyb);        \
            else                                                                                                     \
                MG_LAUNCH((k_outer_lds<TA, TR, TE, VEC, Wr, false, SS>), dim3(blocks), dim3(64 * Wr * SS), s, ev0, \
                          ev1, n, (TA)ih2, phi_in, e, phi_out, b, bmean, r, x1, (TA)cd0, partials, nz, nyb);        \
        } else {                                                                                                     \
            return hipErrorInvalidValue;                                                                             \
        }                                                                                                            \
    })
        switch (row_segments(n, sizeof(TA))) {
            case 2: MG_OUTER_SEGLDS(2); break;
            case 4: MG_OUTER_SEGLDS(4); break;
            default: return hipErrorInvalidValue;
        }
#undef MG_OUTER_SEGLDS
        return hipGetLastError();
    }
    if (lds_rows_fit<TA>(n)) {
        outer_lds_shape(n, kLdsWaves, nz, nyb, blocks);
#define MG_OUTER_LDS(Wv)                                                                                           \
    DISPATCH_VEC(n, {                                                                                              \
        if constexpr (2ull * (Wv + 2) * 64 * VEC * sizeof(TA) <= kLdsBudget) {                                     \
            if (e)                                                                                                 \
                MG_LAUNCH((k_outer_lds<TA, TR, TE, VEC, Wv, true>), dim3(blocks), dim3(64 * Wv), s, ev0, ev1, n, \
                                   (TA)ih2, phi_in, e, phi_out, b, bmean, r, x1, (TA)cd0, partials, nz, nyb);     \
            else                                                                                                   \
                MG_LAUNCH((k_outer_lds<TA, TR, TE, VEC, Wv, false>), dim3(blocks), dim3(64 * Wv), s, ev0, ev1, n, \
                                   (TA)ih2, phi_in, e, phi_out, b, bmean, r, x1, (TA)cd0, partials, nz, nyb);     \
        }                                                                                                          \
    })
        MG_OUTER_LDS(kLdsWaves)
#undef MG_OUTER_LDS
        return hipGetLastError();
    }
    const int S = row_segments(n, sizeof(TA));
    if (S > 1) {
        shape(n * S, n, 16, nz, nyb, blocks, 1024);
#define MG_OUTER_SEG(SS)                                                                                              \
    DISPATCH_SEG(n, SS, {                                                                                             \
        if (e)                                                                                                        \
            MG_LAUNCH((k_outer_row<TA, TR, TE, VEC, true, SS>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, (TA)ih2, \
                      phi_in, e, phi_out, b, bmean, r, x1, (TA)cd0, partials, nz, nyb);                              \
        else                                                                                                          \
            MG_LAUNCH((k_outer_row<TA, TR, TE, VEC, false, SS>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, (TA)ih2, \
                      phi_in, e, phi_out, b, bmean, r, x1, (TA)cd0, partials, nz, nyb);                               \
    })
        switch (S) {
            case 2: MG_OUTER_SEG(2); break;
            case 4: MG_OUTER_SEG(4); break;
            default: return hipErrorInvalidValue;
        }
#undef MG_OUTER_SEG
        return hipGetLastError();
    }
    shape(n, n, 16, nz, nyb, blocks, 1024);
    DISPATCH_VEC(n, {
        if (e)
            MG_LAUNCH((k_outer_row<TA, TR, TE, VEC, true>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, (TA)ih2,
                               phi_in, e, phi_out, b, bmean, r, x1, (TA)cd0, partials, nz, nyb);
        else
            MG_LAUNCH((k_outer_row<TA, TR, TE, VEC, false>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, (TA)ih2,
                               phi_in, e, phi_out, b, bmean, r, x1, (TA)cd0, partials, nz, nyb);
    })
    return hipGetLastError();
}

// Fine rows of 2 KB (512^3 float, 256^3 double) take the LDS kernel with 8
// coarse rows per block; rows of 4 KB (1024^3 float, 512^3 double) with 4
// coarse rows of two 2 KB segments (10 waves, 128 KB of LDS).
constexpr bool kRrLds = true;
constexpr size_t kRrLdsSegBytes = 2048;
inline int rr_lds_segments(int n, size_t elem) {
    const size_t row = (size_t)n * elem;
    return kRrLds && (row == kRrLdsSegBytes || row == 2 * kRrLdsSegBytes) ? (int)(row / kRrLdsSegBytes) : 0;
}
constexpr int rr_lds_rows(int S) { return S == 1 ? 8 : 4; }

template <typename T, int S>
hipError_t launch_rr_lds(int n, double ih2, const T* x, const T* b, T* coarse, hipStream_t s, hipEvent_t ev0,
                         hipEvent_t ev1) {
    constexpr int W = rr_lds_rows(S);
    const int nc = n / 2;
    const int nyb = nc / W;
    int nzc = nc;
    while (nzc > 4 && nyb * (nc / nzc) < kRrTarget) nzc >>= 1;
    const int blocks = nyb * (nc / nzc);
    DISPATCH_SEG(n, S, {
        if constexpr (64 * VEC * sizeof(T) == kRrLdsSegBytes) {
            MG_LAUNCH((k_rr_lds<T, VEC, W, S>), dim3(blocks), dim3(64 * (W + 1) * S), s, ev0, ev1, n, (T)ih2, x, b,
                      coarse, nzc, nyb);
        } else {
            return hipErrorInvalidValue;
        }
    })
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rr_row(int n, double ih2, const T* x, const T* b, T* coarse, hipStream_t s, hipEvent_t ev0,
                         hipEvent_t ev1) {
    const int nc = n / 2;
    int nzc, nyb, blocks;
    switch (rr_lds_segments(n, sizeof(T))) {
        case 1: return launch_rr_lds<T, 1>(n, ih2, x, b, coarse, s, ev0, ev1);
        case 2: return launch_rr_lds<T, 2>(n, ih2, x, b, coarse, s, ev0, ev1);
        default: break;
    }
    // small levels are latency chains: chunks of 2 coarse planes (128^3: 7.7 -> 5.7 us,
    // 64^3: 6.8 -> 4.8 us per launch)
    const int S = row_segments(n, sizeof(T));
    shape(nc * S, nc, n <= 128 ? 2 : 4, nzc, nyb, blocks, n >= 256 ? kRrTarget : 1024);
    if (S > 1) {
        switch (S) {
            case 2: DISPATCH_SEG(n, 2, { MG_LAUNCH((k_rr_row<T, VEC, 2>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n,
                                                   (T)ih2, x, b, coarse, nzc, nyb); }) break;
            case 4: DISPATCH_SEG(n, 4, { MG_LAUNCH((k_rr_row<T, VEC, 4>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n,
                                                   (T)ih2, x, b, coarse, nzc, nyb); }) break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    DISPATCH_VEC(n, {
        MG_LAUNCH((k_rr_row<T, VEC>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, (T)ih2, x, b, coarse, nzc, nyb);
    })
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_row(int n, const T* e, T* x, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    int nz, nyb, blocks;
    const int S = row_segments(n, sizeof(T));
    shape(n * S, n, 4, nz, nyb, blocks);
    switch (S) {
        case 1:
            DISPATCH_VEC(n, {
                MG_LAUNCH((k_prolong_row<T, VEC>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, e, x, nz, nyb);
            })
            break;
        case 2:
            DISPATCH_SEG(n, 2, {
                MG_LAUNCH((k_prolong_row<T, VEC, 2>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, e, x, nz, nyb);
            })
            break;
        case 4:
            DISPATCH_SEG(n, 4, {
                MG_LAUNCH((k_prolong_row<T, VEC, 4>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, e, x, nz, nyb);
            })
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_smooth_row<float>(int, double, const float*, const float*, const float*, float*, double,
                                             double, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_smooth_row<double>(int, double, const double*, const double*, const double*, double*,
                                              double, double, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_smooth_fromb_row<float>(int, double, const float*, float*, double, double, double,
                                                   hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_smooth_fromb_row<double>(int, double, const double*, double*, double, double, double,
                                                    hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_smooth_pro_row<float>(int, double, const float*, const float*, const float*, float*,
                                                 double, double, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_smooth_pro_row<double>(int, double, const double*, const double*, const double*, double*,
                                                  double, double, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_smooth_prevp_row<float>(int, double, const float*, const float*, const float*,
                                                   const float*, float*, double, double, hipStream_t, hipEvent_t,
                                                   hipEvent_t);
template hipError_t launch_smooth_prevp_row<double>(int, double, const double*, const double*, const double*,
                                                    const double*, double*, double, double, hipStream_t, hipEvent_t,
                                                    hipEvent_t);
template hipError_t launch_smooth_prevb_row<float>(int, double, const float*, const float*, float*, double, double,
                                                   double, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_smooth_prevb_row<double>(int, double, const double*, const double*, double*, double,
                                                    double, double, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_smooth_pair_row<float>(int, double, const float*, const float*, const float*, float*,
                                                  float*, double, double, double, double, hipStream_t, hipEvent_t,
                                                  hipEvent_t, int, double, const SumsJob*, const float*);
template hipError_t launch_smooth_pair_row<double>(int, double, const double*, const double*, const double*,
                                                   double*, double*, double, double, double, double, hipStream_t,
                                                   hipEvent_t, hipEvent_t, int, double, const SumsJob*, const double*);
template hipError_t launch_rr_row<float>(int, double, const float*, const float*, float*, hipStream_t, hipEvent_t,
                                         hipEvent_t);
template hipError_t launch_rr_row<double>(int, double, const double*, const double*, double*, hipStream_t, hipEvent_t,
                                          hipEvent_t);
template hipError_t launch_prolong_row<float>(int, const float*, float*, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_prolong_row<double>(int, const double*, double*, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_outer_row<double, double, double>(int, double, const double*, const double*, double*,
                                                             const double*, double, double*, double*, double,
                                                             double*, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_outer_row<double, float, float>(int, double, const double*, const float*, double*,
                                                           const double*, double, float*, float*, double, double*,
                                                           hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_outer_row<float, float, float>(int, double, const double*, const float*, double*,
                                                          const double*, double, float*, float*, double, double*,
                                                          hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace mg
