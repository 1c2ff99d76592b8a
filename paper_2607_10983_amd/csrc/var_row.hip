// 19-point flux-form operator, row-wave kernels for 64 <= n <= 1024.
//
// Same organisation as the seven-point row kernels: one wavefront owns one
// whole x-row (lane l holds VEC = n/64 contiguous elements), x-shifted values
// of any row come from rotating cross-lane moves (periodic wrap included),
// and the wave marches a chunk of z-planes keeping the 3 x 3 (y, z) block of
// iterate rows around its row in registers.  The coefficient components that
// couple z (C^{zz}, C^{xz}, C^{yz}) ride in the same kind of z queue for the
// wave's own row, so each of their rows is read once per pass; C^{xx},
// C^{yy}, C^{xy} and the y-neighbour rows of C^{yy}, C^{xy}, C^{yz} are read
// per plane (the y-neighbour rows are re-reads of the adjacent waves' rows).
// Where the queue would cost occupancy (rows of more than 16 bytes per lane in
// the smoothing kernel, VEC > 4 elsewhere) the z rows are re-read instead.
// The operator (Sec. 4.3.1, cross terms read as averaged fluxes):
//   M u = sum_a [f_a+ (u_{+a} - u) - f_a- (u - u_{-a})] / h^2
//       + 1/(4 h^2) sum_{a != b} [C^{ab}_{+a} (u_{+a+b} - u_{+a-b}) - C^{ab}_{-a} (u_{-a+b} - u_{-a-b})]
// with f_a+- the mean of C^{aa} over the two cells of the face, and
// D = -sum_a (f_a+ + f_a-) / h^2 its diagonal.
#include "var_row.h"

#include "launch.h"
#include "row.h"

namespace mg {
namespace {

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
constexpr bool kVarLds = true;  // smoothing steps and the residual share the iterate's rows through LDS (n >= 128)
// The LDS kernels load the plane's C rows (CRows) before its barrier, so their
// latency overlaps the wait, at the cost of registers live across it (float
// smoothing step 3 instead of 4 waves per SIMD).  256^3 moving mesh: single
// step 131 -> 127 us mixed, 319 -> 308 us FP64; float residual 77 -> 76 us.
constexpr bool kVarCrowsEarly = true;

// coefficient row in compute precision T
template <typename T, typename TC, int VEC>
__device__ __forceinline__ void ldcrow(T (&v)[VEC], const TC* p) {
    TC t[VEC];
    ldrow<TC, VEC>(t, p);
#pragma unroll
    for (int e = 0; e < VEC; ++e) v[e] = (T)t[e];
}

// Row shifted by +1 / -1 in x: element e of the result is row[e + 1] / row[e - 1].
template <typename T, int VEC>
__device__ __forceinline__ void shifts(const T (&r)[VEC], T (&p)[VEC], T (&m)[VEC]) {
    const T first_next = lane_rot(r[0], 1);
    const T last_prev = lane_rot(r[VEC - 1], -1);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        p[e] = e < VEC - 1 ? r[e + 1] : first_next;
        m[e] = e > 0 ? r[e - 1] : last_prev;
    }
}

// z queue of the own row's C^{zz}, C^{xz}, C^{yz} at planes z-1, z, z+1 (index 0, 1, 2)
template <typename T, int VEC>
struct CQueue {
    T zz[3][VEC], xz[3][VEC], yz[3][VEC];
};
template <bool ZQ, typename T, typename TC, int VEC>
__device__ __forceinline__ void cq_load(CQueue<T, VEC>& q, int slot, const TC* __restrict__ C, size_t N,
                                        const RowGrid& g, int y, int z, size_t off) {
    if constexpr (!ZQ) return;
    const size_t r = g.row(y, z) + off;
    ldcrow<T, TC, VEC>(q.zz[slot], C + 2 * N + r);
    ldcrow<T, TC, VEC>(q.xz[slot], C + 4 * N + r);
    ldcrow<T, TC, VEC>(q.yz[slot], C + 5 * N + r);
}
template <bool ZQ, typename T, int VEC>
__device__ __forceinline__ void cq_shift(CQueue<T, VEC>& q) {
    if constexpr (!ZQ) return;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        q.zz[0][e] = q.zz[1][e];
        q.zz[1][e] = q.zz[2][e];
        q.xz[0][e] = q.xz[1][e];
        q.xz[1][e] = q.xz[2][e];
        q.yz[0][e] = q.yz[1][e];
        q.yz[1][e] = q.yz[2][e];
    }
}

// The rows of C in the plane of row (y, z) that the 19-point formula reads
// besides the z queue: C^{xx} at y; C^{yy} and C^{xy} at y, y + 1, y - 1;
// C^{yz} at y + 1, y - 1 (converted to T).  Loaded ahead of the plane's
// barrier, their latency overlaps the wait.
template <typename T, int VEC>
struct CRows {
    T xx[VEC], yy[VEC], yyp[VEC], yym[VEC], xy[VEC], xyp[VEC], xym[VEC], yzp[VEC], yzm[VEC];
};
template <typename T, typename TC, int VEC>
__device__ __forceinline__ void cr_load(CRows<T, VEC>& c, const TC* __restrict__ C, size_t N, const RowGrid& g,
                                        int y, int z, size_t off) {
    const size_t r0 = g.row(y, z) + off, rp = g.row(y + 1, z) + off, rm = g.row(y - 1, z) + off;
    ldcrow<T, TC, VEC>(c.xx, C + r0);
    ldcrow<T, TC, VEC>(c.yy, C + N + r0);
    ldcrow<T, TC, VEC>(c.yyp, C + N + rp);
    ldcrow<T, TC, VEC>(c.yym, C + N + rm);
    ldcrow<T, TC, VEC>(c.xy, C + 3 * N + r0);
    ldcrow<T, TC, VEC>(c.xyp, C + 3 * N + rp);
    ldcrow<T, TC, VEC>(c.xym, C + 3 * N + rm);
    ldcrow<T, TC, VEC>(c.yzp, C + 5 * N + rp);
    ldcrow<T, TC, VEC>(c.yzm, C + 5 * N + rm);
}

// U[dy + 1][dz + 1] = iterate rows (y + dy, z + dz), q the z queue of the row
// (unused without ZQ), cr the plane's other C rows; returns M u and D of row (y, z).
template <bool ZQ, typename T, typename TC, int VEC>
__device__ __forceinline__ void var19_row_c(const T (&U)[3][3][VEC], const CQueue<T, VEC>& q,
                                            const CRows<T, VEC>& cr, const TC* __restrict__ C, size_t N,
                                            const RowGrid& g, int y, int z, size_t off, T ih2, T (&Mu)[VEC],
                                            T (&D)[VEC]) {
    const TC* Czz = C + 2 * N;
    const TC* Cxz = C + 4 * N;
    const TC* Cyz = C + 5 * N;
    const size_t r0 = g.row(y, z) + off;
    // z rows of C^{zz}, C^{xz}, C^{yz}: from the queue, or re-read
    T lzz[3][VEC], lxz[3][VEC], lyz[3][VEC];
    if constexpr (!ZQ) {
        ldcrow<T, TC, VEC>(lzz[1], Czz + r0);
        ldcrow<T, TC, VEC>(lzz[2], Czz + g.row(y, z + 1) + off);
        ldcrow<T, TC, VEC>(lzz[0], Czz + g.row(y, z - 1) + off);
        ldcrow<T, TC, VEC>(lxz[1], Cxz + r0);
        ldcrow<T, TC, VEC>(lxz[2], Cxz + g.row(y, z + 1) + off);
        ldcrow<T, TC, VEC>(lxz[0], Cxz + g.row(y, z - 1) + off);
        ldcrow<T, TC, VEC>(lyz[2], Cyz + g.row(y, z + 1) + off);
        ldcrow<T, TC, VEC>(lyz[0], Cyz + g.row(y, z - 1) + off);
    }
    const T(&zz)[3][VEC] = ZQ ? q.zz : lzz;
    const T(&xz)[3][VEC] = ZQ ? q.xz : lxz;
    const T(&yz)[3][VEC] = ZQ ? q.yz : lyz;
    T acc[VEC], dsum[VEC], cross[VEC];
    T up[VEC], um[VEC];
    shifts<T, VEC>(U[1][1], up, um);
    {   // x faces
        const T(&c)[VEC] = cr.xx;
        T cp[VEC], cm[VEC];
        shifts<T, VEC>(c, cp, cm);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const T uc = U[1][1][e];
            const T fp = T(0.5) * (c[e] + cp[e]), fm = T(0.5) * (c[e] + cm[e]);
            acc[e] = fp * (up[e] - uc) - fm * (uc - um[e]);
            dsum[e] = fp + fm;
        }
    }
    {   // y faces
        const T(&c)[VEC] = cr.yy;
        const T(&cp)[VEC] = cr.yyp;
        const T(&cm)[VEC] = cr.yym;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const T uc = U[1][1][e];
            const T fp = T(0.5) * (c[e] + cp[e]), fm = T(0.5) * (c[e] + cm[e]);
            acc[e] += fp * (U[2][1][e] - uc) - fm * (uc - U[0][1][e]);
            dsum[e] += fp + fm;
        }
    }
    {   // z faces
        const T(&c)[VEC] = zz[1];
        const T(&cp)[VEC] = zz[2];
        const T(&cm)[VEC] = zz[0];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const T uc = U[1][1][e];
            const T fp = T(0.5) * (c[e] + cp[e]), fm = T(0.5) * (c[e] + cm[e]);
            acc[e] += fp * (U[1][2][e] - uc) - fm * (uc - U[1][0][e]);
            dsum[e] += fp + fm;
        }
    }
    {   // pairs (x,y) and (y,x): C^{xy} at x+-1 (row y) and at y+-1
        const T(&c)[VEC] = cr.xy;
        T cxp[VEC], cxm[VEC];
        shifts<T, VEC>(c, cxp, cxm);
        const T(&cyp)[VEC] = cr.xyp;
        const T(&cym)[VEC] = cr.xym;
        T ypp[VEC], ypm[VEC], ymp[VEC], ymm[VEC];  // u(y+1, x+-1), u(y-1, x+-1)
        shifts<T, VEC>(U[2][1], ypp, ypm);
        shifts<T, VEC>(U[0][1], ymp, ymm);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            // upp = u(x+1,y+1), upm = u(x+1,y-1), ump = u(x-1,y+1), umm = u(x-1,y-1)
            const T upp = ypp[e], upm = ymp[e], ump = ypm[e], umm = ymm[e];
            cross[e] = cxp[e] * (upp - upm) - cxm[e] * (ump - umm) + cyp[e] * (upp - ump) - cym[e] * (upm - umm);
        }
    }
    {   // pairs (x,z) and (z,x)
        T cxp[VEC], cxm[VEC];
        shifts<T, VEC>(xz[1], cxp, cxm);
        const T(&czp)[VEC] = xz[2];
        const T(&czm)[VEC] = xz[0];
        T zpp[VEC], zpm[VEC], zmp[VEC], zmm[VEC];  // u(z+1, x+-1), u(z-1, x+-1)
        shifts<T, VEC>(U[1][2], zpp, zpm);
        shifts<T, VEC>(U[1][0], zmp, zmm);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const T upp = zpp[e], upm = zmp[e], ump = zpm[e], umm = zmm[e];
            cross[e] += cxp[e] * (upp - upm) - cxm[e] * (ump - umm) + czp[e] * (upp - ump) - czm[e] * (upm - umm);
        }
    }
    {   // pairs (y,z) and (z,y)
        const T(&cyp)[VEC] = cr.yzp;
        const T(&cym)[VEC] = cr.yzm;
        const T(&czp)[VEC] = yz[2];
        const T(&czm)[VEC] = yz[0];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            // upp = u(y+1,z+1), upm = u(y+1,z-1), ump = u(y-1,z+1), umm = u(y-1,z-1)
            const T upp = U[2][2][e], upm = U[2][0][e], ump = U[0][2][e], umm = U[0][0][e];
            cross[e] += cyp[e] * (upp - upm) - cym[e] * (ump - umm) + czp[e] * (upp - ump) - czm[e] * (upm - umm);
        }
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        Mu[e] = (acc[e] + T(0.25) * cross[e]) * ih2;
        D[e] = -dsum[e] * ih2;
    }
}

// The same with the plane's C rows loaded here.
template <bool ZQ, typename T, typename TC, int VEC>
__device__ __forceinline__ void var19_row(const T (&U)[3][3][VEC], const CQueue<T, VEC>& q,
                                          const TC* __restrict__ C, size_t N, const RowGrid& g, int y, int z,
                                          size_t off, T ih2, T (&Mu)[VEC], T (&D)[VEC]) {
    CRows<T, VEC> cr;
    cr_load<T, TC, VEC>(cr, C, N, g, y, z, off);
    var19_row_c<ZQ, T, TC, VEC>(U, q, cr, C, N, g, y, z, off, ih2, Mu, D);
}

// diagonal only (first smoothing step from zero)
template <typename T, typename TC, int VEC>
__device__ __forceinline__ void var19_diag(const TC* __restrict__ C, size_t N, const RowGrid& g, int y, int z,
                                           size_t off, T ih2, T (&D)[VEC]) {
    const size_t r0 = g.row(y, z) + off;
    T c[VEC], cp[VEC], cm[VEC], d[VEC];
    ldcrow<T, TC, VEC>(c, C + r0);
    shifts<T, VEC>(c, cp, cm);
#pragma unroll
    for (int e = 0; e < VEC; ++e) d[e] = T(0.5) * (c[e] + cp[e]) + T(0.5) * (c[e] + cm[e]);
    ldcrow<T, TC, VEC>(c, C + N + r0);
    ldcrow<T, TC, VEC>(cp, C + N + g.row(y + 1, z) + off);
    ldcrow<T, TC, VEC>(cm, C + N + g.row(y - 1, z) + off);
#pragma unroll
    for (int e = 0; e < VEC; ++e) d[e] += T(0.5) * (c[e] + cp[e]) + T(0.5) * (c[e] + cm[e]);
    ldcrow<T, TC, VEC>(c, C + 2 * N + r0);
    ldcrow<T, TC, VEC>(cp, C + 2 * N + g.row(y, z + 1) + off);
    ldcrow<T, TC, VEC>(cm, C + 2 * N + g.row(y, z - 1) + off);
#pragma unroll
    for (int e = 0; e < VEC; ++e) D[e] = -(d[e] + T(0.5) * (c[e] + cp[e]) + T(0.5) * (c[e] + cm[e])) * ih2;
}

// value accessor of the iterate rows: plain field, or phi + e formed in double
template <typename T, typename TU, int VEC>
struct PlainRows {
    const TU* u;
    __device__ __forceinline__ void load(T (&v)[VEC], size_t r) const {
        TU t[VEC];
        ldrow<TU, VEC>(t, u + r);
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = (T)t[e];
    }
};
template <typename T, typename TE, int VEC>
struct SumRows {
    const double* p;
    const TE* e;
    __device__ __forceinline__ void load(T (&v)[VEC], size_t r) const {
        double a[VEC];
        TE b[VEC];
        ldrow<double, VEC>(a, p + r);
        ldrow<TE, VEC>(b, e + r);
#pragma unroll
        for (int k = 0; k < VEC; ++k) v[k] = (T)(a[k] + (double)b[k]);
    }
};

template <typename T, int VEC, typename Src>
__device__ __forceinline__ void load_plane3(T (&U)[3][3][VEC], int dz, const Src& src, const RowGrid& g, int y, int z,
                                            size_t off) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) src.load(U[dy][dz], g.row(y + dy - 1, z) + off);
}

template <typename T, int VEC>
__device__ __forceinline__ void shift_queue(T (&U)[3][3][VEC]) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            U[dy][0][e] = U[dy][1][e];
            U[dy][1][e] = U[dy][2][e];
        }
}

// Iterate rows of a block of W waves (rows y0 .. y0+W-1) through a ring of
// four LDS planes: every wave loads only its own row (the edge waves also the
// block's halo row), publishes it one plane ahead of its use, and takes the
// rows y +- 1 at z-1, z, z+1 from the ring.  One barrier per plane (by the
// kernel, between ring_publish and ring_gather): a slot is written two
// iterations after it was last read.
template <typename T, int VEC, int W>
struct Ring {
    T (*r)[W + 2][64 * VEC];  // the kernel's __shared__ T [4][W + 2][64 VEC]
    int w, hs, lane;          // own ring row w + 1; the edge wave's halo ring row hs
    bool edge;
    __device__ __forceinline__ T* row(int z, int i) const { return r[z & 3][i]; }
};
// prologue: U[1][0..2] = own row at z0-1, z0, z0+1; planes z0-1, z0 published;
// hr = the halo row at z0+1
template <typename T, int VEC, int W, typename Src>
__device__ __forceinline__ void ring_start(const Ring<T, VEC, W>& rg, T (&U)[3][3][VEC], T (&hr)[VEC], const Src& src,
                                           const RowGrid& g, int y, int yh, int z0, size_t off) {
    src.load(U[1][0], g.row(y, z0 - 1) + off);
    src.load(U[1][1], g.row(y, z0) + off);
    src.load(U[1][2], g.row(y, z0 + 1) + off);
    lds_strow<T, VEC>(rg.row(z0 - 1, rg.w + 1), rg.lane, U[1][0]);
    lds_strow<T, VEC>(rg.row(z0, rg.w + 1), rg.lane, U[1][1]);
    if (rg.edge) {
        src.load(hr, g.row(yh, z0 - 1) + off);
        lds_strow<T, VEC>(rg.row(z0 - 1, rg.hs), rg.lane, hr);
        src.load(hr, g.row(yh, z0) + off);
        lds_strow<T, VEC>(rg.row(z0, rg.hs), rg.lane, hr);
        src.load(hr, g.row(yh, z0 + 1) + off);
    }
}
// publish plane z + 1 (own row U[1][2], halo row hr)
template <typename T, int VEC, int W>
__device__ __forceinline__ void ring_publish(const Ring<T, VEC, W>& rg, const T (&U)[3][3][VEC], const T (&hr)[VEC],
                                             int z) {
    lds_strow<T, VEC>(rg.row(z + 1, rg.w + 1), rg.lane, U[1][2]);
    if (rg.edge) lds_strow<T, VEC>(rg.row(z + 1, rg.hs), rg.lane, hr);
}
// after the barrier: the rows y -+ 1 at z-1, z, z+1
template <typename T, int VEC, int W>
__device__ __forceinline__ void ring_gather(const Ring<T, VEC, W>& rg, T (&U)[3][3][VEC], int z) {
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
        lds_ldrow<T, VEC>(U[0][dz], rg.row(z - 1 + dz, rg.w), rg.lane);
        lds_ldrow<T, VEC>(U[2][dz], rg.row(z - 1 + dz, rg.w + 2), rg.lane);
    }
}
// advance the own queue and the halo row by one plane (xn, hn: plane z + 2)
template <typename T, int VEC, int W>
__device__ __forceinline__ void ring_shift(const Ring<T, VEC, W>& rg, T (&U)[3][3][VEC], T (&hr)[VEC],
                                           const T (&xn)[VEC], const T (&hn)[VEC]) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        U[1][0][e] = U[1][1][e];
        U[1][1][e] = U[1][2][e];
        U[1][2][e] = xn[e];
        if (rg.edge) hr[e] = hn[e];
    }
}

// =====================================================================================
// smoothing step: out = x + a (x - xprev) + c D^-1 (b - M x)
// =====================================================================================
template <typename T, typename TC, int VEC, bool HASX, bool PREV, bool ZQ = (VEC * sizeof(T) <= 16)>
__global__ __launch_bounds__(kBlock) void k_var_smooth_row(int n, T ih2, const TC* __restrict__ C, const T* x,
                                                           const T* xprev, const T* __restrict__ b, T* out, T a, T c,
                                                           int nz, int nyb) {
    const RowGrid g{64 * VEC, 64 * VEC - 1};
    constexpr size_t N = (size_t)(64 * VEC) * (64 * VEC) * (64 * VEC);
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int y = yb * kWaves + wave_id();
    const int z0 = zc * nz;
    const size_t off = (size_t)(threadIdx.x & 63) * VEC;
    if constexpr (!HASX) {
        for (int k = 0; k < nz; ++k) {
            const int z = z0 + k;
            T D[VEC], bb[VEC], o[VEC];
            var19_diag<T, TC, VEC>(C, N, g, y, z, off, ih2, D);
            ldrow<T, VEC>(bb, b + g.row(y, z) + off);
#pragma unroll
            for (int e = 0; e < VEC; ++e) o[e] = c * bb[e] / D[e];
            strow<T, VEC>(out + g.row(y, z) + off, o);
        }
    } else {
        const PlainRows<T, T, VEC> src{x};
        T U[3][3][VEC];
        CQueue<T, VEC> q;
        load_plane3<T, VEC>(U, 0, src, g, y, z0 - 1, off);
        load_plane3<T, VEC>(U, 1, src, g, y, z0, off);
        cq_load<ZQ, T, TC, VEC>(q, 0, C, N, g, y, z0 - 1, off);
        cq_load<ZQ, T, TC, VEC>(q, 1, C, N, g, y, z0, off);
        for (int k = 0; k < nz; ++k) {
            const int z = z0 + k;
            load_plane3<T, VEC>(U, 2, src, g, y, z + 1, off);
            cq_load<ZQ, T, TC, VEC>(q, 2, C, N, g, y, z + 1, off);
            T bb[VEC], pp[VEC], Mu[VEC], D[VEC], o[VEC];
            const size_t r = g.row(y, z) + off;
            ldrow<T, VEC>(bb, b + r);
            if constexpr (PREV) ldrow<T, VEC>(pp, xprev + r);
            var19_row<ZQ, T, TC, VEC>(U, q, C, N, g, y, z, off, ih2, Mu, D);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const T xc = U[1][1][e];
                const T xp = PREV ? pp[e] : T(0);
                o[e] = xc + a * (xc - xp) + c * (bb[e] - Mu[e]) / D[e];
            }
            strow<T, VEC>(out + r, o);
            shift_queue<T, VEC>(U);
            cq_shift<ZQ, T, VEC>(q);
        }
    }
}

// The same step with the y-neighbour rows of the iterate shared through LDS
// (Ring): a block of W waves owns rows y0 .. y0+W-1.  Same arithmetic as
// k_var_smooth_row (var19_row on the same 3 x 3 rows), same bits.
template <typename T, typename TC, int VEC, int W, bool PREV, bool ZQ>
__global__ __launch_bounds__(64 * W) void k_var_smooth_lds(int n, T ih2, const TC* __restrict__ C, const T* x,
                                                           const T* xprev, const T* __restrict__ b, T* out, T a,
                                                           T c, int nz, int nyb) {
    constexpr int NR = 64 * VEC;
    constexpr size_t N = (size_t)NR * NR * NR;
    __shared__ T ring[4][W + 2][NR];
    const RowGrid g{NR, NR - 1};
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int w = wave_id();
    const int y0 = yb * W, y = y0 + w;
    const int z0 = zc * nz;
    const int lane = threadIdx.x & 63;
    const size_t off = (size_t)lane * VEC;
    const bool lo = w == 0, hi = w == W - 1;
    const int yh = lo ? y0 - 1 : y0 + W;  // halo row of the edge waves
    const Ring<T, VEC, W> rg{ring, w, lo ? 0 : W + 1, lane, lo || hi};
    const PlainRows<T, T, VEC> src{x};
    T U[3][3][VEC], hr[VEC], xn[VEC], hn[VEC];
    ring_start<T, VEC, W>(rg, U, hr, src, g, y, yh, z0, off);
    CQueue<T, VEC> q;
    cq_load<ZQ, T, TC, VEC>(q, 0, C, N, g, y, z0 - 1, off);
    cq_load<ZQ, T, TC, VEC>(q, 1, C, N, g, y, z0, off);
    for (int k = 0; k < nz; ++k) {
        const int z = z0 + k;
        const bool more = k + 1 < nz;
        if (more) {  // the plane after next, one iteration early
            src.load(xn, g.row(y, z + 2) + off);
            if (rg.edge) src.load(hn, g.row(yh, z + 2) + off);
        }
        ring_publish<T, VEC, W>(rg, U, hr, z);
        cq_load<ZQ, T, TC, VEC>(q, 2, C, N, g, y, z + 1, off);
        CRows<T, VEC> cr;
        if constexpr (kVarCrowsEarly) cr_load<T, TC, VEC>(cr, C, N, g, y, z, off);
        T bb[VEC], pp[VEC], Mu[VEC], D[VEC], o[VEC];
        const size_t r = g.row(y, z) + off;
        ldrow<T, VEC>(bb, b + r);
        if constexpr (PREV) ldrow<T, VEC>(pp, xprev + r);
        __syncthreads();
        ring_gather<T, VEC, W>(rg, U, z);
        if constexpr (!kVarCrowsEarly) cr_load<T, TC, VEC>(cr, C, N, g, y, z, off);
        var19_row_c<ZQ, T, TC, VEC>(U, q, cr, C, N, g, y, z, off, ih2, Mu, D);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const T xc = U[1][1][e];
            const T xp = PREV ? pp[e] : T(0);
            o[e] = xc + a * (xc - xp) + c * (bb[e] - Mu[e]) / D[e];
        }
        strow<T, VEC>(out + r, o);
        if (more) ring_shift<T, VEC, W>(rg, U, hr, xn, hn);
        cq_shift<ZQ, T, VEC>(q);
    }
}

// Two consecutive smoothing steps in one pass:
//   y1 = x  + a1 (x - xp) + c1 D^-1 (b - M x)    (xp = 0 without PREV1)
//   y2 = y1 + a2 (y1 - x) + c2 D^-1 (b - M y1)
// Only y2 is written, and C is read once for both steps.  A block of NW waves
// owns rows y0-1 .. y0+W (W = NW - 2 outputs): every wave forms y1 on its row
// (x rows through Ring) one plane ahead of the second step and publishes it
// into a second ring of four planes, from which waves 1 .. W gather the 3 x 3
// (y, z) neighbourhood of their y1 row; the two edge waves only supply the
// halo rows of y1.  The second step's z rows of C^{zz}, C^{xz}, C^{yz} come
// from the first step's queue one plane earlier.  Two barriers per plane.
// Each step is the arithmetic of k_var_smooth_row, so the result is bitwise
// that of two single steps.
template <typename T, typename TC, int VEC, int NW, bool PREV1, bool ZQ>
__global__ __launch_bounds__(64 * NW) void k_var_smooth2_lds(int n, T ih2, const TC* __restrict__ C,
                                                             const T* __restrict__ x, const T* __restrict__ xp,
                                                             const T* __restrict__ b, T* __restrict__ y2, T a1,
                                                             T c1, T a2, T c2, int nz, int nyb) {
    constexpr int NR = 64 * VEC;
    constexpr size_t N = (size_t)NR * NR * NR;
    constexpr int W = NW - 2;
    __shared__ T ring[4][NW + 2][NR];  // x rows y0-2 .. y0+W+1
    __shared__ T yr[4][NW][NR];        // y1 rows y0-1 .. y0+W
    const RowGrid g{NR, NR - 1};
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int w = wave_id();
    const int yr0 = yb * W - 1, y = yr0 + w;  // rows outside [0, n) wrap in g.row
    const int z0 = zc * nz;
    const int lane = threadIdx.x & 63;
    const size_t off = (size_t)lane * VEC;
    const bool lo = w == 0, hi = w == NW - 1, outw = !lo && !hi && y < n;  // the last block is ragged
    const int yh = lo ? yr0 - 1 : yr0 + NW;
    const Ring<T, VEC, NW> rg{ring, w, lo ? 0 : NW + 1, lane, lo || hi};
    const PlainRows<T, T, VEC> src{x};
    T U[3][3][VEC], hr[VEC], xn[VEC], hn[VEC];
    int z1 = z0 - 1;  // plane of the first step; the second step is at z1 - 1
    ring_start<T, VEC, NW>(rg, U, hr, src, g, y, yh, z1, off);
    CQueue<T, VEC> q;     // planes z1-1, z1, z1+1
    CQueue<T, VEC> q2{};  // planes z1-2, z1-1, z1 (the second step's)
    cq_load<ZQ, T, TC, VEC>(q, 0, C, N, g, y, z1 - 1, off);
    cq_load<ZQ, T, TC, VEC>(q, 1, C, N, g, y, z1, off);
    T bo[VEC] = {};  // b at z1 - 1
    for (int j = 0; j < nz + 2; ++j, ++z1) {
        const bool more = j + 1 < nz + 2;
        if (more) {  // the plane after next, one iteration early
            src.load(xn, g.row(y, z1 + 2) + off);
            if (rg.edge) src.load(hn, g.row(yh, z1 + 2) + off);
        }
        ring_publish<T, VEC, NW>(rg, U, hr, z1);
        cq_load<ZQ, T, TC, VEC>(q, 2, C, N, g, y, z1 + 1, off);
        T bb[VEC], pp[VEC], Mu[VEC], D[VEC], o[VEC];
        const size_t r = g.row(y, z1) + off;
        ldrow<T, VEC>(bb, b + r);
        if constexpr (PREV1) ldrow<T, VEC>(pp, xp + r);
        __syncthreads();
        ring_gather<T, VEC, NW>(rg, U, z1);
        var19_row<ZQ, T, TC, VEC>(U, q, C, N, g, y, z1, off, ih2, Mu, D);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const T xc = U[1][1][e];
            const T xpe = PREV1 ? pp[e] : T(0);
            o[e] = xc + a1 * (xc - xpe) + c1 * (bb[e] - Mu[e]) / D[e];
        }
        lds_strow<T, VEC>(yr[z1 & 3][w], lane, o);
        if constexpr (ZQ) {  // the second step's queue: planes z1-2 (kept), z1-1, z1
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                q2.zz[1][e] = q.zz[0][e];
                q2.zz[2][e] = q.zz[1][e];
                q2.xz[1][e] = q.xz[0][e];
                q2.xz[2][e] = q.xz[1][e];
                q2.yz[1][e] = q.yz[0][e];
                q2.yz[2][e] = q.yz[1][e];
            }
        }
        __syncthreads();
        if (j >= 2 && outw) {  // second step at z2 = z1 - 1: y1 planes z1-2 .. z1
            const int z2 = z1 - 1;
            T Y[3][3][VEC], M2[VEC], D2[VEC], o2[VEC];
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dz = 0; dz < 3; ++dz) lds_ldrow<T, VEC>(Y[dy][dz], yr[(z2 - 1 + dz) & 3][w - 1 + dy], lane);
            var19_row<ZQ, T, TC, VEC>(Y, q2, C, N, g, y, z2, off, ih2, M2, D2);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const T yc = Y[1][1][e];
                o2[e] = yc + a2 * (yc - U[1][0][e]) + c2 * (bo[e] - M2[e]) / D2[e];
            }
            strow<T, VEC>(y2 + g.row(y, z2) + off, o2);
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) bo[e] = bb[e];
        if constexpr (ZQ) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                q2.zz[0][e] = q.zz[0][e];
                q2.xz[0][e] = q.xz[0][e];
                q2.yz[0][e] = q.yz[0][e];
            }
        }
        if (more) ring_shift<T, VEC, NW>(rg, U, hr, xn, hn);
        cq_shift<ZQ, T, VEC>(q);
    }
}

// =====================================================================================
// residual r = b - M x (scratch of the two-pass residual restriction) / apply
// =====================================================================================
template <typename T, typename TC, int VEC, bool WITHB, bool ZQ = (VEC <= 4)>
__global__ __launch_bounds__(kBlock) void k_var_resid_row(int n, T ih2, const TC* __restrict__ C,
                                                          const T* __restrict__ x, const T* __restrict__ b,
                                                          T* __restrict__ out, int nz, int nyb) {
    const RowGrid g{64 * VEC, 64 * VEC - 1};
    constexpr size_t N = (size_t)(64 * VEC) * (64 * VEC) * (64 * VEC);
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int y = yb * kWaves + wave_id();
    const int z0 = zc * nz;
    const size_t off = (size_t)(threadIdx.x & 63) * VEC;
    const PlainRows<T, T, VEC> src{x};
    T U[3][3][VEC];
    CQueue<T, VEC> q;
    load_plane3<T, VEC>(U, 0, src, g, y, z0 - 1, off);
    load_plane3<T, VEC>(U, 1, src, g, y, z0, off);
    cq_load<ZQ, T, TC, VEC>(q, 0, C, N, g, y, z0 - 1, off);
    cq_load<ZQ, T, TC, VEC>(q, 1, C, N, g, y, z0, off);
    for (int k = 0; k < nz; ++k) {
        const int z = z0 + k;
        load_plane3<T, VEC>(U, 2, src, g, y, z + 1, off);
        cq_load<ZQ, T, TC, VEC>(q, 2, C, N, g, y, z + 1, off);
        const size_t r = g.row(y, z) + off;
        T Mu[VEC], D[VEC], o[VEC];
        var19_row<ZQ, T, TC, VEC>(U, q, C, N, g, y, z, off, ih2, Mu, D);
        if constexpr (WITHB) {
            T bb[VEC];
            ldrow<T, VEC>(bb, b + r);
#pragma unroll
            for (int e = 0; e < VEC; ++e) o[e] = bb[e] - Mu[e];
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) o[e] = Mu[e];
        }
        strow<T, VEC>(out + r, o);
        shift_queue<T, VEC>(U);
        cq_shift<ZQ, T, VEC>(q);
    }
}

// The residual (apply) with the iterate's y-neighbour rows through LDS (Ring).
template <typename T, typename TC, int VEC, int W, bool WITHB, bool ZQ>
__global__ __launch_bounds__(64 * W) void k_var_resid_lds(int n, T ih2, const TC* __restrict__ C,
                                                          const T* __restrict__ x, const T* __restrict__ b,
                                                          T* __restrict__ out, int nz, int nyb) {
    constexpr int NR = 64 * VEC;
    constexpr size_t N = (size_t)NR * NR * NR;
    __shared__ T ring[4][W + 2][NR];
    const RowGrid g{NR, NR - 1};
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int w = wave_id();
    const int y0 = yb * W, y = y0 + w;
    const int z0 = zc * nz;
    const int lane = threadIdx.x & 63;
    const size_t off = (size_t)lane * VEC;
    const bool lo = w == 0, hi = w == W - 1;
    const int yh = lo ? y0 - 1 : y0 + W;
    const Ring<T, VEC, W> rg{ring, w, lo ? 0 : W + 1, lane, lo || hi};
    const PlainRows<T, T, VEC> src{x};
    T U[3][3][VEC], hr[VEC], xn[VEC], hn[VEC];
    ring_start<T, VEC, W>(rg, U, hr, src, g, y, yh, z0, off);
    CQueue<T, VEC> q;
    cq_load<ZQ, T, TC, VEC>(q, 0, C, N, g, y, z0 - 1, off);
    cq_load<ZQ, T, TC, VEC>(q, 1, C, N, g, y, z0, off);
    for (int k = 0; k < nz; ++k) {
        const int z = z0 + k;
        const bool more = k + 1 < nz;
        if (more) {
            src.load(xn, g.row(y, z + 2) + off);
            if (rg.edge) src.load(hn, g.row(yh, z + 2) + off);
        }
        ring_publish<T, VEC, W>(rg, U, hr, z);
        cq_load<ZQ, T, TC, VEC>(q, 2, C, N, g, y, z + 1, off);
        const size_t r = g.row(y, z) + off;
        // (the double residual measured slower with its C rows loaded early: 157 -> 161 us at 256^3)
        constexpr bool EARLY = kVarCrowsEarly && sizeof(T) == sizeof(float);
        CRows<T, VEC> cr;
        if constexpr (EARLY) cr_load<T, TC, VEC>(cr, C, N, g, y, z, off);
        T bb[VEC], Mu[VEC], D[VEC], o[VEC];
        if constexpr (WITHB) ldrow<T, VEC>(bb, b + r);
        __syncthreads();
        ring_gather<T, VEC, W>(rg, U, z);
        if constexpr (!EARLY) cr_load<T, TC, VEC>(cr, C, N, g, y, z, off);
        var19_row_c<ZQ, T, TC, VEC>(U, q, cr, C, N, g, y, z, off, ih2, Mu, D);
#pragma unroll
        for (int e = 0; e < VEC; ++e) o[e] = WITHB ? bb[e] - Mu[e] : Mu[e];
        strow<T, VEC>(out + r, o);
        if (more) ring_shift<T, VEC, W>(rg, U, hr, xn, hn);
        cq_shift<ZQ, T, VEC>(q);
    }
}

// =====================================================================================
// outer defect correction in TA: value = phi (+ e), r = (b - bmean) - M value,
// optional x1 = c0 D^-1 r, partial sums of r^2
// =====================================================================================
template <typename TA, typename TR, typename TE, typename TC, int VEC, bool UPDATE, bool ZQ = (VEC <= 4)>
__global__ __launch_bounds__(kBlock) void k_var_outer_row(int n, TA ih2, const TC* __restrict__ C,
                                                          const double* __restrict__ phi_in,
                                                          const TE* __restrict__ e, double* __restrict__ phi_out,
                                                          const double* __restrict__ b, double bmean,
                                                          TR* __restrict__ r, TR* __restrict__ x1, TA c0,
                                                          double* __restrict__ partials, int nz, int nyb) {
    __shared__ double sh[3 * kWaves];
    const RowGrid g{64 * VEC, 64 * VEC - 1};
    constexpr size_t N = (size_t)(64 * VEC) * (64 * VEC) * (64 * VEC);
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int yb = lb % nyb, zc = lb / nyb;
    const int wave = wave_id();
    const int y = yb * kWaves + wave;
    const int z0 = zc * nz;
    const size_t off = (size_t)(threadIdx.x & 63) * VEC;
    double ss = 0.0, sb = 0.0, sp = 0.0;
    auto body = [&](const auto& src) {
        TA U[3][3][VEC];
        CQueue<TA, VEC> q;
        load_plane3<TA, VEC>(U, 0, src, g, y, z0 - 1, off);
        load_plane3<TA, VEC>(U, 1, src, g, y, z0, off);
        cq_load<ZQ, TA, TC, VEC>(q, 0, C, N, g, y, z0 - 1, off);
        cq_load<ZQ, TA, TC, VEC>(q, 1, C, N, g, y, z0, off);
        for (int k = 0; k < nz; ++k) {
            const int z = z0 + k;
            load_plane3<TA, VEC>(U, 2, src, g, y, z + 1, off);
            cq_load<ZQ, TA, TC, VEC>(q, 2, C, N, g, y, z + 1, off);
            const size_t row = g.row(y, z) + off;
            double bb[VEC];
            ldrow<double, VEC>(bb, b + row);
            TA Mu[VEC], D[VEC];
            TR ro[VEC];
            var19_row<ZQ, TA, TC, VEC>(U, q, C, N, g, y, z, off, ih2, Mu, D);
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const double bq = bb[q] - bmean;
                const TA ri = (TA)bq - Mu[q];
                ro[q] = (TR)ri;
                ss += (double)ri * (double)ri;
                sb += bq * bq;
            }
            strow<TR, VEC>(r + row, ro);
            if (x1) {
                TR xo[VEC];
#pragma unroll
                for (int q = 0; q < VEC; ++q) xo[q] = (TR)(c0 * (TA)ro[q] / D[q]);
                strow<TR, VEC>(x1 + row, xo);
            }
            // the row's value (phi or phi + e) in double: the queue's own row when
            // TA is double, else read again
            double po[VEC];
            if constexpr (sizeof(TA) == sizeof(double)) {
#pragma unroll
                for (int q = 0; q < VEC; ++q) po[q] = (double)U[1][1][q];
            } else if constexpr (UPDATE) {
                double p[VEC];
                TE qv[VEC];
                ldrow<double, VEC>(p, phi_in + row);
                ldrow<TE, VEC>(qv, e + row);
#pragma unroll
                for (int q = 0; q < VEC; ++q) po[q] = p[q] + (double)qv[q];
            } else {
                ldrow<double, VEC>(po, phi_in + row);
            }
            if constexpr (UPDATE) strow<double, VEC>(phi_out + row, po);
#pragma unroll
            for (int q = 0; q < VEC; ++q) sp += po[q];
            shift_queue<TA, VEC>(U);
            cq_shift<ZQ, TA, VEC>(q);
        }
    };
    if constexpr (UPDATE) body(SumRows<TA, TE, VEC>{phi_in, e});
    else body(PlainRows<TA, double, VEC>{phi_in});
    // fixed-order block reduction of the three partial sums, arrays of gridDim.x:
    // [0] sum (b - bmean)^2, [1] sum r^2, [2] sum phi
    for (int o = 32; o > 0; o >>= 1) {
        sb += __shfl_xor(sb, o, 64);
        ss += __shfl_xor(ss, o, 64);
        sp += __shfl_xor(sp, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[wave] = sb;
        sh[kWaves + wave] = ss;
        sh[2 * kWaves + wave] = sp;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const double* t = sh + threadIdx.x * kWaves;
        partials[threadIdx.x * gridDim.x + blockIdx.x] = (t[0] + t[1]) + (t[2] + t[3]);
    }
}

void shape(int n, int& nz, int& nyb, int& blocks) {
    nyb = n / kWaves;
    nz = n;
    while (nz > 4 && nyb * (n / nz) < 2048) nz >>= 1;
    blocks = nyb * (n / nz);
}

}  // namespace

bool var_row_kernels_apply(int n) { return n >= 64 && n <= 1024 && (n & (n - 1)) == 0; }

// The kernels with the iterate's y-neighbour rows through LDS (Ring):
// kVarLdsWaves rows per block, chunks giving at least 1024 blocks, where a
// ring of four planes fits 80 KB (float n <= 512, double n <= 256).
constexpr int kVarLdsWaves = 8;
inline bool var_lds_applies(int n, size_t elem) {
    return kVarLds && n >= 128 && 4ull * (kVarLdsWaves + 2) * n * elem <= 80 * 1024;
}
inline void var_lds_shape(int n, int& nz, int& nyb, int& blocks) {
    nyb = n / kVarLdsWaves;
    nz = n;
    while (nz > 4 && nyb * (n / nz) < 1024) nz >>= 1;
    blocks = nyb * (n / nz);
}

int var_row_blocks(int n) {
    int nz, nyb, blocks;
    shape(n, nz, nyb, blocks);
    return blocks;
}

#define DISPATCH_VEC(n, ...)                                       \
    switch (n) {                                                   \
        case 64: { constexpr int VEC = 1; __VA_ARGS__; break; }    \
        case 128: { constexpr int VEC = 2; __VA_ARGS__; break; }   \
        case 256: { constexpr int VEC = 4; __VA_ARGS__; break; }   \
        case 512: { constexpr int VEC = 8; __VA_ARGS__; break; }   \
        case 1024: { constexpr int VEC = 16; __VA_ARGS__; break; } \
        default: return hipErrorInvalidValue;                      \
    }

template <typename T, typename TC>
hipError_t launch_var_smooth_row(int n, double ih2, const TC* C, const T* x, const T* xprev, const T* b, T* out,
                                 double a, double c, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    int nz, nyb, blocks;
    if (x != nullptr && var_lds_applies(n, sizeof(T))) {
        constexpr int Wv = kVarLdsWaves;
        var_lds_shape(n, nz, nyb, blocks);
        DISPATCH_VEC(n, {
            constexpr bool ZQ = VEC * sizeof(T) <= 16;
            if constexpr (4ull * (Wv + 2) * 64 * VEC * sizeof(T) <= 80 * 1024) {
                if (xprev == nullptr)
                    MG_LAUNCH((k_var_smooth_lds<T, TC, VEC, Wv, false, ZQ>), dim3(blocks), dim3(64 * Wv), s, ev0, ev1,
                              n, (T)ih2, C, x, xprev, b, out, (T)a, (T)c, nz, nyb);
                else
                    MG_LAUNCH((k_var_smooth_lds<T, TC, VEC, Wv, true, ZQ>), dim3(blocks), dim3(64 * Wv), s, ev0, ev1,
                              n, (T)ih2, C, x, xprev, b, out, (T)a, (T)c, nz, nyb);
            } else {
                return hipErrorInvalidValue;
            }
        })
        return hipGetLastError();
    }
    shape(n, nz, nyb, blocks);
    DISPATCH_VEC(n, {
        if (x == nullptr)
            MG_LAUNCH((k_var_smooth_row<T, TC, VEC, false, false>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, (T)ih2, C, x, xprev, b, out, (T)a, (T)c, nz, nyb);
        else if (xprev == nullptr)
            MG_LAUNCH((k_var_smooth_row<T, TC, VEC, true, false>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, (T)ih2, C, x, xprev, b, out, (T)a, (T)c, nz, nyb);
        else
            MG_LAUNCH((k_var_smooth_row<T, TC, VEC, true, true>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, (T)ih2, C, x, xprev, b, out, (T)a, (T)c, nz, nyb);
    })
    return hipGetLastError();
}

// The two-step kernel: float rows of up to 1 KB (n = 128, 256), blocks of
// kVarPairWaves waves (kVarPairWaves - 2 output rows; a last block that
// overhangs the grid is ragged), chunks of at most kVarPairNz planes giving
// at least 256 blocks.  At 256^3 (A/B, mixed moving mesh): 8-wave blocks
// with 16-plane chunks 246 us per pair, 10 waves 207 us, 12 waves 236 us,
// 10 waves with 32-plane chunks 200 us; four waves per SIMD forced (two
// blocks per CU) spilled and took 483 us.
constexpr int kVarPairWaves = 10;
constexpr int kVarPairNz = 32;
bool var_pair_applies(int n, size_t elem) {
    return kVarLds && elem == sizeof(float) && n >= 128 && (size_t)n * elem <= 1024;
}

template <typename T, typename TC>
hipError_t launch_var_smooth_pair(int n, double ih2, const TC* C, const T* x, const T* xp, const T* b, T* y2,
                                  double a1, double c1, double a2, double c2, hipStream_t s, hipEvent_t ev0,
                                  hipEvent_t ev1) {
    if (!var_pair_applies(n, sizeof(T)) || x == nullptr || y2 == x || y2 == xp) return hipErrorInvalidValue;
    constexpr int NW = kVarPairWaves, W = NW - 2;
    const int nyb = (n + W - 1) / W;
    int nz = kVarPairNz;
    while (nz > 4 && nyb * (n / nz) < 256) nz >>= 1;
    const int blocks = nyb * (n / nz);
    DISPATCH_VEC(n, {
        if constexpr (sizeof(T) == sizeof(float) && VEC >= 2 && VEC <= 4) {
            if (xp)
                MG_LAUNCH((k_var_smooth2_lds<T, TC, VEC, NW, true, true>), dim3(blocks), dim3(64 * NW), s, ev0, ev1,
                          n, (T)ih2, C, x, xp, b, y2, (T)a1, (T)c1, (T)a2, (T)c2, nz, nyb);
            else
                MG_LAUNCH((k_var_smooth2_lds<T, TC, VEC, NW, false, true>), dim3(blocks), dim3(64 * NW), s, ev0,
                          ev1, n, (T)ih2, C, x, xp, b, y2, (T)a1, (T)c1, (T)a2, (T)c2, nz, nyb);
        } else {
            return hipErrorInvalidValue;
        }
    })
    return hipGetLastError();
}

template <typename T, typename TC>
hipError_t launch_var_resid_row(int n, double ih2, const TC* C, const T* x, const T* b, T* out, hipStream_t s,
                                hipEvent_t ev0, hipEvent_t ev1) {
    int nz, nyb, blocks;
    if (var_lds_applies(n, sizeof(T))) {
        constexpr int Wv = kVarLdsWaves;
        var_lds_shape(n, nz, nyb, blocks);
        DISPATCH_VEC(n, {
            constexpr bool ZQ = VEC <= 4;
            if constexpr (4ull * (Wv + 2) * 64 * VEC * sizeof(T) <= 80 * 1024) {
                if (b)
                    MG_LAUNCH((k_var_resid_lds<T, TC, VEC, Wv, true, ZQ>), dim3(blocks), dim3(64 * Wv), s, ev0, ev1,
                              n, (T)ih2, C, x, b, out, nz, nyb);
                else
                    MG_LAUNCH((k_var_resid_lds<T, TC, VEC, Wv, false, ZQ>), dim3(blocks), dim3(64 * Wv), s, ev0, ev1,
                              n, (T)ih2, C, x, b, out, nz, nyb);
            } else {
                return hipErrorInvalidValue;
            }
        })
        return hipGetLastError();
    }
    shape(n, nz, nyb, blocks);
    DISPATCH_VEC(n, {
        if (b)
            MG_LAUNCH((k_var_resid_row<T, TC, VEC, true>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, (T)ih2, C, x,
                      b, out, nz, nyb);
        else
            MG_LAUNCH((k_var_resid_row<T, TC, VEC, false>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n, (T)ih2, C,
                      x, b, out, nz, nyb);
    })
    return hipGetLastError();
}

template <typename TA, typename TR, typename TE, typename TC>
hipError_t launch_var_outer_row(int n, double ih2, const TC* C, const double* phi_in, const TE* e, double* phi_out,
                                const double* b, double bmean, TR* r, TR* x1, double c0, double* partials,
                                hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    int nz, nyb, blocks;
    shape(n, nz, nyb, blocks);
    DISPATCH_VEC(n, {
        if (e)
            MG_LAUNCH((k_var_outer_row<TA, TR, TE, TC, VEC, true>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n,
                      (TA)ih2, C, phi_in, e, phi_out, b, bmean, r, x1, (TA)c0, partials, nz, nyb);
        else
            MG_LAUNCH((k_var_outer_row<TA, TR, TE, TC, VEC, false>), dim3(blocks), dim3(kBlock), s, ev0, ev1, n,
                      (TA)ih2, C, phi_in, e, phi_out, b, bmean, r, x1, (TA)c0, partials, nz, nyb);
    })
    return hipGetLastError();
}

#define INST_VAR(T, TC)                                                                                            \
    template hipError_t launch_var_smooth_row<T, TC>(int, double, const TC*, const T*, const T*, const T*, T*,     \
                                                     double, double, hipStream_t, hipEvent_t, hipEvent_t);         \
    template hipError_t launch_var_smooth_pair<T, TC>(int, double, const TC*, const T*, const T*, const T*, T*,    \
                                                      double, double, double, double, hipStream_t, hipEvent_t,     \
                                                      hipEvent_t);                                                 \
    template hipError_t launch_var_resid_row<T, TC>(int, double, const TC*, const T*, const T*, T*, hipStream_t,   \
                                                    hipEvent_t, hipEvent_t);
INST_VAR(float, float)
INST_VAR(double, double)
INST_VAR(double, float)
INST_VAR(float, double)

#define INST_VOUT(TA, TR, TE, TC)                                                                                  \
    template hipError_t launch_var_outer_row<TA, TR, TE, TC>(int, double, const TC*, const double*, const TE*,     \
                                                             double*, const double*, double, TR*, TR*, double,     \
                                                             double*, hipStream_t, hipEvent_t, hipEvent_t);
INST_VOUT(double, double, double, double)
INST_VOUT(double, double, double, float)
INST_VOUT(double, float, float, float)
INST_VOUT(double, float, float, double)
INST_VOUT(float, float, float, float)
INST_VOUT(float, float, float, double)

}  // namespace mg
