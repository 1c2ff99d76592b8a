// gfx950 kernels of the matrix-free multigrid V-cycle.
//
// Every stencil kernel streams a periodic n^3 field (x fastest) with one
// thread per (x, y) column marching `nz` planes in z; wave64 rows run along
// the contiguous x axis so loads and stores are coalesced, and neighbour
// values are served from the vector L1 / L2 caches.  Reductions are
// per-block LDS trees in a fixed order followed by a single-block pass over
// the partials, so every result is bitwise reproducible run to run.
#include "kernels.h"
#include "flat_row.h"
#include "var_row.h"

#include "launch.h"
#include "stencil.h"
#include "sums.h"

#include <cmath>
#include <cstdint>
#include <type_traits>

namespace mg {
namespace {

// =====================================================================================
// smoothing step
// =====================================================================================
template <typename T, typename TC, bool HASX, bool HASPREV>
__global__ __launch_bounds__(kThreads) void k_smooth(int n, T ih2, const TC* __restrict__ C,
                                                     const T* __restrict__ x, const T* xprev,
                                                     const T* __restrict__ b, T* out, T a, T c,
                                                     int nz) {
    const Grid g{n, n - 1};
    const size_t N = (size_t)n * n * n;
    const int xi = blockIdx.x * blockDim.x + threadIdx.x;
    const int yi = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    const Plain<T, T> u{x};
    const T dflat = T(-6) * ih2;
    for (int z = z0; z < z0 + nz; ++z) {
        const size_t i = g(xi, yi, z);
        const T bi = b[i];
        T val;
        if constexpr (HASX) {
            const T uc = x[i];
            T Mu, D;
            if (C == nullptr) {
                Mu = flat_Mu<T>(u, g, xi, yi, z, uc, ih2);
                D = dflat;
            } else {
                var_Mu<T, TC>(u, C, N, g, xi, yi, z, uc, ih2, Mu, D);
            }
            T xp = T(0);
            if constexpr (HASPREV) xp = xprev[i];
            // seven-point: c arrives as c / D (as in the row kernels)
            val = C == nullptr ? step_pt<T>(uc, xp, bi, Mu, a, c) : uc + a * (uc - xp) + c * (bi - Mu) / D;
        } else {
            val = C == nullptr ? c * bi : c * bi / var_diag<T, TC>(C, N, g, xi, yi, z, ih2);
        }
        out[i] = val;
    }
}

// =====================================================================================
// residual + full weighting
// =====================================================================================
template <typename T, typename TC, bool HASX>
__global__ __launch_bounds__(kThreads) void k_resid_restrict(int n, T ih2, const TC* __restrict__ C,
                                                             const T* __restrict__ x,
                                                             const T* __restrict__ b,
                                                             T* __restrict__ coarse, int nz) {
    const int nc = n >> 1;
    const Grid g{n, n - 1};
    const Grid gc{nc, nc - 1};
    const size_t N = (size_t)n * n * n;
    const int X = blockIdx.x * blockDim.x + threadIdx.x;
    const int Y = blockIdx.y * blockDim.y + threadIdx.y;
    const int Z0 = blockIdx.z * nz;
    const Plain<T, T> u{x};
    const T w1[3] = {T(0.25), T(0.5), T(0.25)};
    for (int Z = Z0; Z < Z0 + nz; ++Z) {
        T acc = T(0);
        for (int dz = -1; dz <= 1; ++dz) {
            T accy = T(0);
            for (int dy = -1; dy <= 1; ++dy) {
                T accx = T(0);
                for (int dx = -1; dx <= 1; ++dx) {
                    const int fx = 2 * X + dx, fy = 2 * Y + dy, fz = 2 * Z + dz;
                    const size_t i = g(fx, fy, fz);
                    T r = b[i];
                    if constexpr (HASX) {
                        const T uc = x[i];
                        T Mu, D;
                        if (C == nullptr) {
                            Mu = flat_Mu<T>(u, g, fx, fy, fz, uc, ih2);
                        } else {
                            var_Mu<T, TC>(u, C, N, g, fx, fy, fz, uc, ih2, Mu, D);
                        }
                        r -= Mu;
                    }
                    accx += w1[dx + 1] * r;
                }
                accy += w1[dy + 1] * accx;
            }
            acc += w1[dz + 1] * accy;
        }
        coarse[gc(X, Y, Z)] = acc;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict(int n, const T* __restrict__ fine,
                                                       T* __restrict__ coarse, int nz) {
    const int nc = n >> 1;
    const Grid g{n, n - 1};
    const Grid gc{nc, nc - 1};
    const int X = blockIdx.x * blockDim.x + threadIdx.x;
    const int Y = blockIdx.y * blockDim.y + threadIdx.y;
    const int Z0 = blockIdx.z * nz;
    for (int Z = Z0; Z < Z0 + nz; ++Z) {
        T v[3][3][3];
        for (int dz = 0; dz < 3; ++dz)
            for (int dy = 0; dy < 3; ++dy)
                for (int dx = 0; dx < 3; ++dx) v[dz][dy][dx] = fine[g(2 * X + dx - 1, 2 * Y + dy - 1, 2 * Z + dz - 1)];
        coarse[gc(X, Y, Z)] = fw_pt<T>(v);
    }
}

// =====================================================================================
// trilinear prolongation + correction
// =====================================================================================
template <typename T>
__global__ __launch_bounds__(kThreads) void k_prolong_add(int n, const T* __restrict__ e, T* x, int nz) {
    const int nc = n >> 1;
    const Grid g{n, n - 1};
    const Grid gc{nc, nc - 1};
    const int xi = blockIdx.x * blockDim.x + threadIdx.x;
    const int yi = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    auto ec = [&](int X, int Y, int Z) { return e[gc(X, Y, Z)]; };
    for (int z = z0; z < z0 + nz; ++z) {
        // interpolate along x on the (up to) 4 coarse lines, then y, then z
        const T p = prolong_pt<T>(ec, xi, yi, z);
        const size_t i = g(xi, yi, z);
        x[i] = add_pt<T>(x[i], p);
    }
}

// =====================================================================================
// operator application
// =====================================================================================
// out = M x, or out = b - M x when b is given
template <typename T, typename TC>
__global__ __launch_bounds__(kThreads) void k_apply(int n, T ih2, const TC* __restrict__ C,
                                                    const T* __restrict__ x, const T* __restrict__ b,
                                                    T* __restrict__ out, int nz) {
    const Grid g{n, n - 1};
    const size_t N = (size_t)n * n * n;
    const int xi = blockIdx.x * blockDim.x + threadIdx.x;
    const int yi = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    const Plain<T, T> u{x};
    for (int z = z0; z < z0 + nz; ++z) {
        const size_t i = g(xi, yi, z);
        const T uc = x[i];
        T Mu, D;
        if (C == nullptr) {
            Mu = flat_Mu<T>(u, g, xi, yi, z, uc, ih2);
        } else {
            var_Mu<T, TC>(u, C, N, g, xi, yi, z, uc, ih2, Mu, D);
        }
        out[i] = b ? b[i] - Mu : Mu;
    }
}

// =====================================================================================
// outer defect correction: optional phi update, residual in TA, sum of r^2
// =====================================================================================
template <typename TA, typename TR, typename TE, typename TC, bool UPDATE>
__global__ __launch_bounds__(kThreads) void k_outer_residual(int n, TA ih2, const TC* __restrict__ C,
                                                             const double* __restrict__ phi_in,
                                                             const TE* __restrict__ e,
                                                             double* __restrict__ phi_out,
                                                             const double* __restrict__ b, double bmean,
                                                             TR* __restrict__ r, TR* __restrict__ x1, TA c0,
                                                             double* partials, int nz) {
    __shared__ double sh[kThreads];
    const Grid g{n, n - 1};
    const size_t N = (size_t)n * n * n;
    const int xi = blockIdx.x * blockDim.x + threadIdx.x;
    const int yi = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    double ss = 0.0, sb = 0.0, sp = 0.0;
    for (int z = z0; z < z0 + nz; ++z) {
        const size_t i = g(xi, yi, z);
        TA Mu, D, uc;
        if constexpr (UPDATE) {
            const double pn = phi_in[i] + (double)e[i];
            phi_out[i] = pn;
            sp += pn;
            uc = (TA)pn;
            const PlusE<TA, TE> u{phi_in, e};
            if (C == nullptr) Mu = flat_Mu<TA>(u, g, xi, yi, z, uc, ih2);
            else var_Mu<TA, TC>(u, C, N, g, xi, yi, z, uc, ih2, Mu, D);
        } else {
            sp += phi_in[i];
            uc = (TA)phi_in[i];
            const Plain<TA, double> u{phi_in};
            if (C == nullptr) Mu = flat_Mu<TA>(u, g, xi, yi, z, uc, ih2);
            else var_Mu<TA, TC>(u, C, N, g, xi, yi, z, uc, ih2, Mu, D);
        }
        const double bq = b[i] - bmean;
        const TA ri = (TA)bq - Mu;
        r[i] = (TR)ri;
        if (x1) {  // first smoothing step from zero, rounded as the smoothing kernels round it
            if (C == nullptr) x1[i] = (TR)c0 * (TR)ri;  // seven-point: c0 arrives as c0 / D
            else x1[i] = (TR)(c0 * (TA)(TR)ri / D);
        }
        ss += (double)ri * (double)ri;
        sb += bq * bq;
    }
    // three partial sums, arrays of the block count: sum (b - bmean)^2, sum r^2, sum phi
    const int nb = gridDim.x * gridDim.y * gridDim.z;
    const double t0 = block_sum(sb, sh);
    const double t1 = block_sum(ss, sh);
    const double t2 = block_sum(sp, sh);
    if (lin_tid() == 0) {
        partials[lin_bid()] = t0;
        partials[nb + lin_bid()] = t1;
        partials[2 * nb + lin_bid()] = t2;
    }
}

// =====================================================================================
// reductions
// =====================================================================================
__global__ __launch_bounds__(kThreads) void k_block_sums(int n, const double* __restrict__ u, double shift, int p,
                                                         double* partials, int nz) {
    __shared__ double sh[kThreads];
    const Grid g{n, n - 1};
    const int xi = blockIdx.x * blockDim.x + threadIdx.x;
    const int yi = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    double s = 0.0;
    // unrolled so that several planes' loads are in flight (39 -> 35 us at 256^3);
    // the sum keeps its z order
#pragma unroll 8
    for (int z = z0; z < z0 + nz; ++z) {
        const double v = u[g(xi, yi, z)] - shift;
        s += p == 2 ? v * v : v;
    }
    const double tot = block_sum(s, sh);
    if (lin_tid() == 0) partials[lin_bid()] = tot;
}

__global__ __launch_bounds__(1024) void k_finalize(const double* __restrict__ partials, int count, double* out,
                                                   int slot, int is_max) {
    __shared__ double sh[1024];
    const int tid = threadIdx.x;
    double v = is_max ? -INFINITY : 0.0;
    for (int i = tid; i < count; i += 1024) v = is_max ? fmax(v, partials[i]) : v + partials[i];
    const double r = is_max ? block_max(v, sh) : block_sum(v, sh);
    if (tid == 0) out[slot] = r;
}

// out[slot + k] = sum of partials[k * count .. (k + 1) * count), k < arrays
// (host_out: pinned host mirror, no separate copy)
__global__ __launch_bounds__(kSumLanes) void k_finalize_multi(SumsJob job) {
    __shared__ double sh[kSumLanes];
    finish_sums(job, sh);
}

// =====================================================================================
// elementwise
// =====================================================================================
__global__ void k_shift(size_t count, const double* src, double shift, double* dst) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i] - shift;
}
template <typename T>
__global__ void k_add(size_t count, const double* src, const T* e, double* dst) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i] + (double)e[i];
}
template <typename TD, typename TS>
__global__ void k_convert(size_t count, const TS* src, TD* dst) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (TD)src[i];
}
template <typename T>
__global__ void k_fill(size_t count, T v, T* dst) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = v;
}
dim3 ew_grid(size_t count) {
    size_t b = (count + kThreads - 1) / kThreads;
    if (b > 65536) b = 65536;
    if (b == 0) b = 1;
    return dim3((unsigned)b);
}

// =====================================================================================
// coefficient checks and Gershgorin bounds
// =====================================================================================
template <typename TC>
__global__ __launch_bounds__(kThreads) void k_gershgorin(int n, const TC* __restrict__ C, double* partials, int nz) {
    __shared__ double sh[kThreads];
    const Grid g{n, n - 1};
    const size_t N = (size_t)n * n * n;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    double m = -INFINITY;
    for (int z = z0; z < z0 + nz; ++z) {
        const size_t i0 = g(x, y, z);
        double face = 0.0;
        for (int a = 0; a < 3; ++a) {
            const TC* c = C + a * N;
            const int dx = a == 0, dy = a == 1, dz = a == 2;
            const double c0 = (double)c[i0];
            face += 0.5 * (c0 + (double)c[g(x + dx, y + dy, z + dz)]) + 0.5 * (c0 + (double)c[g(x - dx, y - dy, z - dz)]);
        }
        double edge = 0.0;
        const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
        for (int p = 0; p < 3; ++p) {
            const TC* c = C + (3 + p) * N;
            for (int sa = -1; sa <= 1; sa += 2)
                for (int sb = -1; sb <= 1; sb += 2) {
                    int ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
                    (pa[p] == 0 ? ax : pa[p] == 1 ? ay : az) = sa;
                    (pb[p] == 0 ? bx : pb[p] == 1 ? by : bz) = sb;
                    edge += fabs((double)c[g(x + ax, y + ay, z + az)] + (double)c[g(x + bx, y + by, z + bz)]) * 0.25;
                }
        }
        m = fmax(m, 1.0 + (face + edge) / face);
    }
    const double tot = block_max(m, sh);
    if (lin_tid() == 0) partials[lin_bid()] = tot;
}

template <typename TC>
__global__ __launch_bounds__(kThreads) void k_coeff_check(int n, const TC* __restrict__ C, double* partials, int nz) {
    __shared__ double sh[kThreads];
    const Grid g{n, n - 1};
    const size_t N = (size_t)n * n * n;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    double bad = 0.0;
    for (int z = z0; z < z0 + nz; ++z) {
        const size_t i = g(x, y, z);
        bool ok = true;
        for (int c = 0; c < 6; ++c) {
            const double v = (double)C[c * N + i];
            if (!isfinite(v)) ok = false;
            if (c < 3 && !(v > 0.0)) ok = false;
        }
        bad += ok ? 0.0 : 1.0;
    }
    const double tot = block_sum(bad, sh);
    if (lin_tid() == 0) partials[lin_bid()] = tot;
}

// =====================================================================================
// coarsest level
// =====================================================================================
// Separable exact solve of the seven-point system: three 1-D basis changes,
// division by the eigenvalue, three inverse basis changes, all in double.
// Every basis change is a set of independent lines (NC^2 lines of NC points
// along one axis): one thread holds a whole line in registers, forms all NC
// outputs and writes them back over the line, so each value crosses LDS once
// per change and the basis matrix, the same for every line, is read with
// uniform loads.  The z change, the division and the inverse z change run on
// the same line in one pass.  LDS rows are padded to NC + 1 values and planes
// to NC (NC + 1), so the lanes of a wave fall on different banks along every
// axis.  Each output is the same sum, in the same order, as a plain basis
// change (acc = 0, then q_j v_j added for j = 0 .. NC-1).  NC (4, 8 or 16) is
// a compile-time constant, so every loop unrolls.  One workgroup of
// coarse_threads(NC) threads (one per line).
constexpr int coarse_threads(int nc) { return nc * nc < 64 ? 64 : nc * nc; }
template <typename T, int NC>
__global__ __launch_bounds__(coarse_threads(NC)) void k_coarse_flat(const double* __restrict__ Q,
                                                                    const double* __restrict__ lam1,
                                                                    const T* __restrict__ r, T* __restrict__ e) {
    constexpr int N = NC * NC * NC;
    constexpr int RP = NC + 1, PP = NC * RP;  // padded row and plane pitches
    constexpr int LINES = NC * NC, NT = coarse_threads(NC);
    __shared__ double A[NC * PP];
    const int tid = threadIdx.x;
    auto at = [](int x, int y, int z) { return x + RP * y + PP * z; };
    for (int i = tid; i < N; i += NT) A[at(i & (NC - 1), (i / NC) & (NC - 1), i / (NC * NC))] = (double)r[i];
    __syncthreads();
    // q[j + NC*k] = basis vector k at point j.  Forward: c_k = sum_j q[j,k] v_j;
    // inverse: v_k = sum_j q[k,j] c_j.  The line's values are all in registers
    // before output k is stored over point k (the thread owns the line), and
    // f(k, c_k) is what is stored.
    auto change = [&](const double(&v)[NC], int base, int stride, bool forward, auto f) {
#pragma unroll 4
        for (int k = 0; k < NC; ++k) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const double w = forward ? Q[j + NC * k] : Q[k + NC * j];
                acc += w * v[j];
            }
            A[base + k * stride] = f(k, acc);
        }
    };
    auto load = [&](double(&v)[NC], int base, int stride) {
#pragma unroll
        for (int j = 0; j < NC; ++j) v[j] = A[base + j * stride];
    };
    auto same = [](int, double c) { return c; };
    const int u = tid & (NC - 1), w = tid / NC;  // line tid: the two other coordinates
    const int bx = at(0, u, w), by = at(u, 0, w), bz = at(u, w, 0);
    double v[NC];
    // forward x and y changes
    if (tid < LINES) {
        load(v, bx, 1);
        change(v, bx, 1, true, same);
    }
    __syncthreads();
    if (tid < LINES) {
        load(v, by, RP);
        change(v, by, RP, true, same);
    }
    __syncthreads();
    // z line of wavenumbers (kx, ky) = (u, w): forward change divided by the
    // eigenvalue (the constant mode set to zero), then the inverse change
    if (tid < LINES) {
        const double lxy = lam1[u] + lam1[w];
        load(v, bz, PP);
        change(v, bz, PP, true, [&](int k, double c) {
            const double l = lxy + lam1[k];
            return (u == 0 && w == 0 && k == 0) ? 0.0 : c / l;
        });
        load(v, bz, PP);
        change(v, bz, PP, false, same);
    }
    __syncthreads();
    // inverse y and x changes
    if (tid < LINES) {
        load(v, by, RP);
        change(v, by, RP, false, same);
    }
    __syncthreads();
    if (tid < LINES) {
        load(v, bx, 1);
        change(v, bx, 1, false, same);
    }
    __syncthreads();
    for (int i = tid; i < N; i += NT) e[i] = (T)A[at(i & (NC - 1), (i / NC) & (NC - 1), i / (NC * NC))];
}

// e = G r, 8 rows per block, 32 lanes per row, fixed-order sums.
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_dense(int N, const double* __restrict__ G, const T* __restrict__ r,
                                                      T* __restrict__ e) {
    __shared__ double sh[256];
    const int row = blockIdx.x * 8 + (threadIdx.x >> 5);
    const int lane = threadIdx.x & 31;
    double acc = 0.0;
    if (row < N)
        for (int j = lane; j < N; j += 32) acc += G[(size_t)row * N + j] * (double)r[j];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 16; s > 0; s >>= 1) {
        if (lane < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (lane == 0 && row < N) e[row] = (T)sh[threadIdx.x];
}

// =====================================================================================
// coefficient gradient (operator VJP)
// =====================================================================================
template <typename TO>
__global__ __launch_bounds__(kThreads) void k_coeff_grad(int n, double ih2, const double* __restrict__ lam,
                                                         const double* __restrict__ phi, TO* __restrict__ out,
                                                         int nz) {
    const Grid g{n, n - 1};
    const size_t N = (size_t)n * n * n;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    for (int z = z0; z < z0 + nz; ++z) {
        const size_t i = g(x, y, z);
        const double l0 = lam[i], p0 = phi[i];
        double lp[3], lm[3], pp[3], pm[3];
        const int d[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int a = 0; a < 3; ++a) {
            const size_t ip = g(x + d[a][0], y + d[a][1], z + d[a][2]);
            const size_t im = g(x - d[a][0], y - d[a][1], z - d[a][2]);
            lp[a] = lam[ip];
            lm[a] = lam[im];
            pp[a] = phi[ip];
            pm[a] = phi[im];
            const double gp = (lp[a] - l0) * (pp[a] - p0);
            const double gm = (l0 - lm[a]) * (p0 - pm[a]);
            out[a * N + i] = (TO)(0.5 * (gp + gm) * ih2);
        }
        const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
        for (int p = 0; p < 3; ++p) {
            const int a = pa[p], b = pb[p];
            const double dla = lp[a] - lm[a], dlb = lp[b] - lm[b];
            const double dpa = pp[a] - pm[a], dpb = pp[b] - pm[b];
            out[(3 + p) * N + i] = (TO)((dla * dpb + dlb * dpa) * 0.25 * ih2);
        }
    }
}

// =====================================================================================
// moving-mesh geometry
// =====================================================================================
template <typename TO>
__global__ __launch_bounds__(kThreads) void k_geometry(int n, double ih2, const double* __restrict__ psi,
                                                       TO* __restrict__ C, double* __restrict__ sqrtg, int nz) {
    const Grid g{n, n - 1};
    const size_t N = (size_t)n * n * n;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    for (int z = z0; z < z0 + nz; ++z) {
        double H[6];
        hess_at(psi, g, x, y, z, ih2, H);
        H[0] += 1.0; H[1] += 1.0; H[2] += 1.0;
        Sym3 J, K, K2;
        sym_from6(H, J);
        const double det = inv3(J, K);
        mul3(K, K, K2);   // J symmetric: J^-1 J^-T = K K
        const size_t i = g(x, y, z);
        C[i] = (TO)(det * K2.m[0][0]);
        C[N + i] = (TO)(det * K2.m[1][1]);
        C[2 * N + i] = (TO)(det * K2.m[2][2]);
        C[3 * N + i] = (TO)(det * K2.m[0][1]);
        C[4 * N + i] = (TO)(det * K2.m[0][2]);
        C[5 * N + i] = (TO)(det * K2.m[1][2]);
        if (sqrtg) sqrtg[i] = det;
    }
}

// Per cell: Jbar = t K - d (P + P^T), P = K G K^2, t = d <G, K^2> + sqrtgbar d,
// G the full symmetric cotangent of C (stored off-diagonals halved).
// Jbar of the planes zlo .. zlo + planes - 1 (mod n): plane p of component c
// at Jbar[c * planes n^2 + p n^2 + y n + x] (the whole grid when zlo = 0 and
// planes = n).
__global__ __launch_bounds__(kThreads) void k_geometry_bwd_cell(int n, double ih2, const double* __restrict__ psi,
                                                                const double* __restrict__ Cbar,
                                                                const double* __restrict__ sbar,
                                                                double* __restrict__ Jbar, int zlo, int planes,
                                                                int nz) {
    const Grid g{n, n - 1};
    const size_t N = (size_t)n * n * n;
    const size_t NS = (size_t)planes * n * n;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int p0 = blockIdx.z * nz;
    for (int p = p0; p < p0 + nz && p < planes; ++p) {
        const int z = (zlo + p) & (n - 1);
        const size_t i = g(x, y, z);
        const size_t is = ((size_t)p * n + y) * n + x;
        double H[6];
        hess_at(psi, g, x, y, z, ih2, H);
        H[0] += 1.0; H[1] += 1.0; H[2] += 1.0;
        Sym3 J, K, K2, G, KG, P;
        sym_from6(H, J);
        const double d = inv3(J, K);
        mul3(K, K, K2);
        double gs[6];
        for (int c = 0; c < 6; ++c) gs[c] = Cbar[c * N + i] * (c < 3 ? 1.0 : 0.5);
        sym_from6(gs, G);
        double t = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) t += G.m[a][b] * K2.m[a][b];
        t *= d;
        if (sbar) t += sbar[i] * d;
        mul3(K, G, KG);
        mul3(KG, K2, P);
        const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
        for (int c = 0; c < 6; ++c) {
            const int a = pa[c], b = pb[c];
            const double jab = t * K.m[a][b] - d * (P.m[a][b] + P.m[b][a]);
            const double jba = t * K.m[b][a] - d * (P.m[b][a] + P.m[a][b]);
            Jbar[c * NS + is] = c < 3 ? jab : jab + jba;
        }
    }
}

// psibar on planes z0 .. z0 + count - 1 from the Jbar planes zlo .. zlo +
// planes - 1 of k_geometry_bwd_cell; they must include z0 - 1 .. z0 + count
// unless they are the whole grid.
__global__ __launch_bounds__(kThreads) void k_hessian_adjoint(int n, double ih2, const double* __restrict__ Jb,
                                                              double* __restrict__ out, int zlo, int planes, int z0,
                                                              int count, int nz) {
    const Grid g{n, n - 1};
    const size_t NS = (size_t)planes * n * n;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int k0 = blockIdx.z * nz;
    for (int k = k0; k < k0 + nz && k < count; ++k) {
        const int z = z0 + k;
        const int q = (z - zlo) & (n - 1);  // plane of z in the Jbar slab
        double acc = 0.0;
        for (int c = 0; c < 6; ++c) {
            const double* u = Jb + c * NS;
            // x and y wrap on the grid, z indexes the slab's planes (and wraps
            // when the slab is the whole grid)
            auto at = [&](int dx, int dy, int dz) {
                return u[g(x + dx, y + dy, 0) + (size_t)((q + dz) & (n - 1)) * n * n];
            };
            // only component c of the Hessian stencil applied to field c is needed
            if (c < 3) {
                const int dx = c == 0, dy = c == 1, dz = c == 2;
                acc += (at(dx, dy, dz) - 2.0 * at(0, 0, 0) + at(-dx, -dy, -dz)) * ih2;
            } else {
                const int a = c == 5 ? 1 : 0, b = c == 3 ? 1 : 2;
                int ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
                (a == 0 ? ax : ay) = 1;
                (b == 1 ? by : bz) = 1;
                acc += (at(ax + bx, ay + by, az + bz) - at(ax - bx, ay - by, az - bz) -
                        at(-ax + bx, -ay + by, -az + bz) + at(-ax - bx, -ay - by, -az - bz)) *
                       0.25 * ih2;
            }
        }
        out[g(x, y, z & (n - 1))] = acc;
    }
}

}  // namespace

// =====================================================================================
// launchers
// =====================================================================================
int stencil_blocks(int n) {
    Shape s = stencil_shape(n);
    return (int)(s.grid.x * s.grid.y * s.grid.z);
}

int outer_blocks(int n, bool flat, bool double_arith) {
    if (flat) return row_kernels_apply(n) ? row_outer_blocks(n, double_arith) : stencil_blocks(n);
    return var_row_kernels_apply(n) ? var_row_blocks(n) : stencil_blocks(n);
}

template <typename T, typename TC>
hipError_t launch_smooth_step(const OpDesc<TC>& op, const T* x, const T* xprev, const T* b, T* out, double a,
                              double c, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (op.coeff == nullptr && row_kernels_apply(op.n))
        return launch_smooth_row<T>(op.n, op.ih2, x, xprev, b, out, a, c / (-6.0 * op.ih2), s, ev0, ev1);
    if (op.coeff != nullptr && var_row_kernels_apply(op.n))
        return launch_var_smooth_row<T, TC>(op.n, op.ih2, op.coeff, x, xprev, b, out, a, c, s, ev0, ev1);
    Shape sh = stencil_shape(op.n);
    if (op.coeff == nullptr) c = c / (-6.0 * op.ih2);  // the seven-point kernel takes c / D
    if (x == nullptr)
        MG_LAUNCH((k_smooth<T, TC, false, false>), sh.grid, sh.block, s, ev0, ev1, op.n, (T)op.ih2, op.coeff, x,
                           xprev, b, out, (T)a, (T)c, sh.nz);
    else if (xprev == nullptr)
        MG_LAUNCH((k_smooth<T, TC, true, false>), sh.grid, sh.block, s, ev0, ev1, op.n, (T)op.ih2, op.coeff, x,
                           xprev, b, out, (T)a, (T)c, sh.nz);
    else
        MG_LAUNCH((k_smooth<T, TC, true, true>), sh.grid, sh.block, s, ev0, ev1, op.n, (T)op.ih2, op.coeff, x,
                           xprev, b, out, (T)a, (T)c, sh.nz);
    return hipGetLastError();
}

template <typename T, typename TC>
hipError_t launch_residual_restrict(const OpDesc<TC>& op, const T* x, const T* b, T* coarse, T* scratch,
                                    hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (op.coeff == nullptr && x != nullptr && row_kernels_apply(op.n))
        return launch_rr_row<T>(op.n, op.ih2, x, b, coarse, s, ev0, ev1);
    if (scratch != nullptr && x != nullptr) {
        if (op.coeff != nullptr && var_row_kernels_apply(op.n)) {
            hipError_t e = launch_var_resid_row<T, TC>(op.n, op.ih2, op.coeff, x, b, scratch, s, ev0, ev1);
            if (e != hipSuccess) return e;
        } else {
            Shape sf = stencil_shape(op.n);
            hipLaunchKernelGGL((k_apply<T, TC>), sf.grid, sf.block, 0, s, op.n, (T)op.ih2, op.coeff, x, b, scratch,
                               sf.nz);
        }
        Shape sc = stencil_shape(op.n / 2);
        hipLaunchKernelGGL((k_restrict<T>), sc.grid, sc.block, 0, s, op.n, (const T*)scratch, coarse, sc.nz);
        return hipGetLastError();
    }
    Shape sh = stencil_shape(op.n / 2);
    if (x)
        hipLaunchKernelGGL((k_resid_restrict<T, TC, true>), sh.grid, sh.block, 0, s, op.n, (T)op.ih2, op.coeff, x, b,
                           coarse, sh.nz);
    else
        hipLaunchKernelGGL((k_resid_restrict<T, TC, false>), sh.grid, sh.block, 0, s, op.n, (T)op.ih2, op.coeff, x, b,
                           coarse, sh.nz);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(int n, const T* fine, T* coarse, int ncomp, hipStream_t s) {
    Shape sh = stencil_shape(n / 2);
    const size_t Nf = (size_t)n * n * n, Nc = Nf / 8;
    for (int c = 0; c < ncomp; ++c)
        hipLaunchKernelGGL((k_restrict<T>), sh.grid, sh.block, 0, s, n, fine + c * Nf, coarse + c * Nc, sh.nz);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(int n, const T* e, T* x, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (row_kernels_apply(n)) return launch_prolong_row<T>(n, e, x, s, ev0, ev1);
    Shape sh = stencil_shape(n);
    MG_LAUNCH((k_prolong_add<T>), sh.grid, sh.block, s, ev0, ev1, n, e, x, sh.nz);
    return hipGetLastError();
}

template <typename T, typename TC>
hipError_t launch_apply(const OpDesc<TC>& op, const T* u, T* out, hipStream_t s) {
    if (op.coeff != nullptr && var_row_kernels_apply(op.n))
        return launch_var_resid_row<T, TC>(op.n, op.ih2, op.coeff, u, (const T*)nullptr, out, s);
    Shape sh = stencil_shape(op.n);
    hipLaunchKernelGGL((k_apply<T, TC>), sh.grid, sh.block, 0, s, op.n, (T)op.ih2, op.coeff, u, (const T*)nullptr,
                       out, sh.nz);
    return hipGetLastError();
}

template <typename TA, typename TR, typename TE, typename TC>
hipError_t launch_outer_residual(const OpDesc<TC>& op, const double* phi_in, const TE* e, double* phi_out,
                                 const double* b, double bmean, TR* r, TR* x1, double c0, double* partials,
                                 hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (op.coeff == nullptr && row_kernels_apply(op.n))
        return launch_outer_row<TA, TR, TE>(op.n, op.ih2, phi_in, e, phi_out, b, bmean, r, x1,
                                            c0 / (-6.0 * op.ih2), partials, s, ev0, ev1);
    if (op.coeff != nullptr && var_row_kernels_apply(op.n))
        return launch_var_outer_row<TA, TR, TE, TC>(op.n, op.ih2, op.coeff, phi_in, e, phi_out, b, bmean, r, x1, c0,
                                                    partials, s, ev0, ev1);
    Shape sh = stencil_shape(op.n);
    if (op.coeff == nullptr) c0 = c0 / (-6.0 * op.ih2);
    if (e)
        MG_LAUNCH((k_outer_residual<TA, TR, TE, TC, true>), sh.grid, sh.block, s, ev0, ev1, op.n, (TA)op.ih2,
                  op.coeff, phi_in, e, phi_out, b, bmean, r, x1, (TA)c0, partials, sh.nz);
    else
        MG_LAUNCH((k_outer_residual<TA, TR, TE, TC, false>), sh.grid, sh.block, s, ev0, ev1, op.n, (TA)op.ih2,
                  op.coeff, phi_in, e, phi_out, b, bmean, r, x1, (TA)c0, partials, sh.nz);
    return hipGetLastError();
}

hipError_t launch_block_sums(int n, const double* u, double shift, int p, double* partials, hipStream_t s) {
    Shape sh = stencil_shape(n);
    hipLaunchKernelGGL(k_block_sums, sh.grid, sh.block, 0, s, n, u, shift, p, partials, sh.nz);
    return hipGetLastError();
}
hipError_t launch_finalize_sum(const double* partials, int count, double* out, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, partials, count, out, slot, 0);
    return hipGetLastError();
}
hipError_t launch_finalize_sums(const double* partials, int count, int arrays, double* out, int slot,
                                hipStream_t s, double* host_out) {
    const SumsJob job{partials, count, arrays, out, slot, host_out};
    hipLaunchKernelGGL(k_finalize_multi, dim3(1), dim3(kSumLanes), 0, s, job);
    return hipGetLastError();
}
hipError_t launch_finalize_max(const double* partials, int count, double* out, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, partials, count, out, slot, 1);
    return hipGetLastError();
}

hipError_t launch_shift(size_t count, const double* src, double shift, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_shift, ew_grid(count), dim3(kThreads), 0, s, count, src, shift, dst);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_add(size_t count, const double* src, const T* e, double* dst, hipStream_t s) {
    hipLaunchKernelGGL((k_add<T>), ew_grid(count), dim3(kThreads), 0, s, count, src, e, dst);
    return hipGetLastError();
}
template <typename TD, typename TS>
hipError_t launch_convert(size_t count, const TS* src, TD* dst, hipStream_t s) {
    hipLaunchKernelGGL((k_convert<TD, TS>), ew_grid(count), dim3(kThreads), 0, s, count, src, dst);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_fill(size_t count, T value, T* dst, hipStream_t s) {
    hipLaunchKernelGGL((k_fill<T>), ew_grid(count), dim3(kThreads), 0, s, count, value, dst);
    return hipGetLastError();
}

template <typename TC>
hipError_t launch_gershgorin(const OpDesc<TC>& op, double* partials, hipStream_t s) {
    Shape sh = stencil_shape(op.n);
    hipLaunchKernelGGL((k_gershgorin<TC>), sh.grid, sh.block, 0, s, op.n, op.coeff, partials, sh.nz);
    return hipGetLastError();
}
template <typename TC>
hipError_t launch_coeff_check(int n, const TC* coeff, double* partials, hipStream_t s) {
    Shape sh = stencil_shape(n);
    hipLaunchKernelGGL((k_coeff_check<TC>), sh.grid, sh.block, 0, s, n, coeff, partials, sh.nz);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_flat(int nc, const double* Q, const double* lam1, const T* r, T* e, hipStream_t s) {
    switch (nc) {
        case 4: hipLaunchKernelGGL((k_coarse_flat<T, 4>), dim3(1), dim3(coarse_threads(4)), 0, s, Q, lam1, r, e); break;
        case 8: hipLaunchKernelGGL((k_coarse_flat<T, 8>), dim3(1), dim3(coarse_threads(8)), 0, s, Q, lam1, r, e); break;
        case 16:
            hipLaunchKernelGGL((k_coarse_flat<T, 16>), dim3(1), dim3(coarse_threads(16)), 0, s, Q, lam1, r, e);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template <typename T>
hipError_t launch_coarse_dense(int N, const double* G, const T* r, T* e, hipStream_t s) {
    hipLaunchKernelGGL((k_coarse_dense<T>), dim3((N + 7) / 8), dim3(256), 0, s, N, G, r, e);
    return hipGetLastError();
}

template <typename TO>
hipError_t launch_coeff_grad(int n, double ih2, const double* lam, const double* phi, TO* cbar, hipStream_t s) {
    Shape sh = stencil_shape(n);
    hipLaunchKernelGGL((k_coeff_grad<TO>), sh.grid, sh.block, 0, s, n, ih2, lam, phi, cbar, sh.nz);
    return hipGetLastError();
}
template <typename TO>
hipError_t launch_geometry(int n, double ih2, const double* psi, TO* C, double* sqrtg, hipStream_t s) {
    Shape sh = stencil_shape(n);
    hipLaunchKernelGGL((k_geometry<TO>), sh.grid, sh.block, 0, s, n, ih2, psi, C, sqrtg, sh.nz);
    return hipGetLastError();
}
hipError_t launch_geometry_bwd_cell(int n, double ih2, const double* psi, const double* Cbar, const double* sbar,
                                    double* Jbar, hipStream_t s, int zlo, int planes) {
    if (planes <= 0) planes = n;
    Shape sh = stencil_shape(n);
    const int chunks = (planes + sh.nz - 1) / sh.nz;
    hipLaunchKernelGGL(k_geometry_bwd_cell, dim3(sh.grid.x, sh.grid.y, chunks), sh.block, 0, s, n, ih2, psi, Cbar,
                       sbar, Jbar, zlo, planes, sh.nz);
    return hipGetLastError();
}
hipError_t launch_hessian_adjoint(int n, double ih2, const double* Jbar, double* psibar, hipStream_t s, int zlo,
                                  int planes, int z0, int count) {
    if (planes <= 0) planes = n;
    if (count <= 0) count = n;
    Shape sh = stencil_shape(n);
    const int chunks = (count + sh.nz - 1) / sh.nz;
    hipLaunchKernelGGL(k_hessian_adjoint, dim3(sh.grid.x, sh.grid.y, chunks), sh.block, 0, s, n, ih2, Jbar, psibar,
                       zlo, planes, z0, count, sh.nz);
    return hipGetLastError();
}

// ---- explicit instantiations ------------------------------------------------------
#define INST_T_TC(T, TC)                                                                                         \
    template hipError_t launch_smooth_step<T, TC>(const OpDesc<TC>&, const T*, const T*, const T*, T*, double,   \
                                                  double, hipStream_t, hipEvent_t, hipEvent_t);                  \
    template hipError_t launch_residual_restrict<T, TC>(const OpDesc<TC>&, const T*, const T*, T*, T*, hipStream_t, \
                                                        hipEvent_t, hipEvent_t);                                  \
    template hipError_t launch_apply<T, TC>(const OpDesc<TC>&, const T*, T*, hipStream_t);
INST_T_TC(float, float)
INST_T_TC(double, double)
INST_T_TC(double, float)
INST_T_TC(float, double)

#define INST_T(T)                                                                                  \
    template hipError_t launch_restrict<T>(int, const T*, T*, int, hipStream_t);                   \
    template hipError_t launch_prolong_add<T>(int, const T*, T*, hipStream_t, hipEvent_t, hipEvent_t); \
    template hipError_t launch_add<T>(size_t, const double*, const T*, double*, hipStream_t);      \
    template hipError_t launch_fill<T>(size_t, T, T*, hipStream_t);                                \
    template hipError_t launch_gershgorin<T>(const OpDesc<T>&, double*, hipStream_t);              \
    template hipError_t launch_coeff_check<T>(int, const T*, double*, hipStream_t);                \
    template hipError_t launch_coarse_flat<T>(int, const double*, const double*, const T*, T*, hipStream_t); \
    template hipError_t launch_coarse_dense<T>(int, const double*, const T*, T*, hipStream_t);     \
    template hipError_t launch_coeff_grad<T>(int, double, const double*, const double*, T*, hipStream_t); \
    template hipError_t launch_geometry<T>(int, double, const double*, T*, double*, hipStream_t);
INST_T(float)
INST_T(double)

template hipError_t launch_convert<float, double>(size_t, const double*, float*, hipStream_t);
template hipError_t launch_convert<double, float>(size_t, const float*, double*, hipStream_t);
template hipError_t launch_convert<double, double>(size_t, const double*, double*, hipStream_t);
template hipError_t launch_convert<float, float>(size_t, const float*, float*, hipStream_t);

#define INST_OUTER(TA, TR, TE, TC)                                                                                \
    template hipError_t launch_outer_residual<TA, TR, TE, TC>(const OpDesc<TC>&, const double*, const TE*, double*, \
                                                              const double*, double, TR*, TR*, double, double*,     \
                                                              hipStream_t, hipEvent_t, hipEvent_t);
INST_OUTER(double, double, double, double)
INST_OUTER(double, double, double, float)
INST_OUTER(double, float, float, float)
INST_OUTER(double, float, float, double)
INST_OUTER(float, float, float, float)
INST_OUTER(float, float, float, double)

}  // namespace mg
