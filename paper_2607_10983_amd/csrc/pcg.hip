// Passes of the multigrid-preconditioned conjugate-gradient solve (the
// preconditioner is one V-cycle from zero, the first iterate the caller's
// phi).  All recurrences run in double; the preconditioner's input and
// output are in the hierarchy's type TI.  The step lengths live in device
// memory and are produced by a one-block kernel between the passes, so a
// whole iteration is enqueued without a host round trip.
//
// Per iteration, with the V-cycle z = B r already applied:
//   dots       (r, z), (z, q_prev)                  reads r, z, q
//   scalars    beta (flexible Polak-Ribiere form), rz
//   direction  p = z + beta p_prev, q = M p, (p, q)  reads z, p_prev; writes p, q
//   scalars    alpha = rz / (p, q)
//   update     phi += alpha p, r -= alpha q, r_in    reads phi, p, r, q; writes phi, r, r_in
//   scalars    (r, r)
#include "kernels.h"
#include "stencil.h"

namespace mg {
namespace {

template <typename TI>
struct ZPlusBetaP {  // new search direction z + beta p_prev, formed in double
    const TI* z;
    const double* p;
    double beta;
    __device__ __forceinline__ double operator()(size_t i) const { return (double)z[i] + beta * p[i]; }
};

template <typename TI, typename TC>
__global__ __launch_bounds__(kThreads) void k_pcg_residual(int n, double ih2, const TC* __restrict__ C,
                                                           const double* __restrict__ phi,
                                                           const double* __restrict__ b, double bmean,
                                                           double* __restrict__ r, TI* __restrict__ rin,
                                                           double* partials, int nz) {
    __shared__ double sh[kThreads];
    const Grid g{n, n - 1};
    const size_t N = (size_t)n * n * n;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    const Plain<double, double> u{phi};
    double ss = 0.0;
    for (int z = z0; z < z0 + nz; ++z) {
        const size_t i = g(x, y, z);
        const double uc = phi[i];
        double Mu, D;
        if (C == nullptr) Mu = flat_Mu<double>(u, g, x, y, z, uc, ih2);
        else var_Mu<double, TC>(u, C, N, g, x, y, z, uc, ih2, Mu, D);
        const double ri = (b[i] - bmean) - Mu;
        r[i] = ri;
        rin[i] = (TI)ri;
        ss += ri * ri;
    }
    const double tot = block_sum(ss, sh);
    if (lin_tid() == 0) partials[lin_bid()] = tot;
}

template <typename TI, bool HASQ>
__global__ __launch_bounds__(kThreads) void k_pcg_dots(int n, const double* __restrict__ r,
                                                       const TI* __restrict__ zv, const double* __restrict__ q,
                                                       double* partials, int nb, int nz) {
    __shared__ double sh[kThreads];
    const Grid g{n, n - 1};
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    double rz = 0.0, zq = 0.0;
    for (int z = z0; z < z0 + nz; ++z) {
        const size_t i = g(x, y, z);
        const double zi = (double)zv[i];
        rz += r[i] * zi;
        if constexpr (HASQ) zq += zi * q[i];
    }
    const double t0 = block_sum(rz, sh);
    const double t1 = block_sum(zq, sh);
    if (lin_tid() == 0) {
        partials[lin_bid()] = t0;
        partials[nb + lin_bid()] = t1;
    }
}

template <typename TI, typename TC, bool RESTART>
__global__ __launch_bounds__(kThreads) void k_pcg_direction(int n, double ih2, const TC* __restrict__ C,
                                                            const TI* __restrict__ zv,
                                                            const double* __restrict__ p_old,
                                                            double* __restrict__ p_new, double* __restrict__ q,
                                                            const double* __restrict__ scal, double* partials,
                                                            int nz) {
    __shared__ double sh[kThreads];
    const Grid g{n, n - 1};
    const size_t N = (size_t)n * n * n;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    const double beta = RESTART ? 0.0 : scal[kPcgBeta];
    double pq = 0.0;
    for (int z = z0; z < z0 + nz; ++z) {
        const size_t i = g(x, y, z);
        double Mu, D, pc;
        if constexpr (RESTART) {
            const Plain<double, TI> u{zv};
            pc = (double)zv[i];
            if (C == nullptr) Mu = flat_Mu<double>(u, g, x, y, z, pc, ih2);
            else var_Mu<double, TC>(u, C, N, g, x, y, z, pc, ih2, Mu, D);
        } else {
            const ZPlusBetaP<TI> u{zv, p_old, beta};
            pc = u(i);
            if (C == nullptr) Mu = flat_Mu<double>(u, g, x, y, z, pc, ih2);
            else var_Mu<double, TC>(u, C, N, g, x, y, z, pc, ih2, Mu, D);
        }
        p_new[i] = pc;
        q[i] = Mu;
        pq += pc * Mu;
    }
    const double tot = block_sum(pq, sh);
    if (lin_tid() == 0) partials[lin_bid()] = tot;
}

template <typename TI>
__global__ __launch_bounds__(kThreads) void k_pcg_update(int n, double* __restrict__ phi,
                                                         const double* __restrict__ p, double* __restrict__ r,
                                                         const double* __restrict__ q, TI* __restrict__ rin,
                                                         const double* __restrict__ scal, double* partials,
                                                         int nz) {
    __shared__ double sh[kThreads];
    const Grid g{n, n - 1};
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * nz;
    const double alpha = scal[kPcgAlpha];
    double ss = 0.0;
    for (int z = z0; z < z0 + nz; ++z) {
        const size_t i = g(x, y, z);
        phi[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        rin[i] = (TI)ri;
        ss += ri * ri;
    }
    const double tot = block_sum(ss, sh);
    if (lin_tid() == 0) partials[lin_bid()] = tot;
}

__global__ __launch_bounds__(1024) void k_pcg_scalars(const double* __restrict__ partials, int nb,
                                                      double* scal, int which, int restart) {
    __shared__ double sh[1024];
    const int tid = threadIdx.x;
    double v0 = 0.0, v1 = 0.0;
    for (int i = tid; i < nb; i += 1024) {
        v0 += partials[i];
        if (which == kPcgBeta) v1 += partials[nb + i];
    }
    const double s0 = block_sum(v0, sh);
    const double s1 = block_sum(v1, sh);
    if (tid != 0) return;
    if (which == kPcgBeta) {
        // flexible CG: beta = (z_k, r_k - r_{k-1}) / (z_{k-1}, r_{k-1}) with
        // r_k - r_{k-1} = -alpha_{k-1} q_{k-1}
        scal[kPcgBeta] = restart ? 0.0 : -scal[kPcgAlpha] * s1 / scal[kPcgRz];
        scal[kPcgRz] = s0;
    } else if (which == kPcgAlpha) {
        scal[kPcgPq] = s0;
        scal[kPcgAlpha] = scal[kPcgRz] / s0;
    } else {
        scal[kPcgRr] = s0;
    }
}

}  // namespace

int pcg_blocks(int n) { return stencil_blocks(n); }

template <typename TI, typename TC>
hipError_t launch_pcg_residual(const OpDesc<TC>& op, const double* phi, const double* b, double bmean,
                               double* r, TI* rin, double* partials, hipStream_t s) {
    const Shape sh = stencil_shape(op.n);
    hipLaunchKernelGGL((k_pcg_residual<TI, TC>), sh.grid, sh.block, 0, s, op.n, op.ih2, op.coeff, phi, b, bmean,
                       r, rin, partials, sh.nz);
    return hipGetLastError();
}

template <typename TI>
hipError_t launch_pcg_dots(int n, const double* r, const TI* z, const double* q, double* partials,
                           hipStream_t s) {
    const Shape sh = stencil_shape(n);
    const int nb = pcg_blocks(n);
    if (q)
        hipLaunchKernelGGL((k_pcg_dots<TI, true>), sh.grid, sh.block, 0, s, n, r, z, q, partials, nb, sh.nz);
    else
        hipLaunchKernelGGL((k_pcg_dots<TI, false>), sh.grid, sh.block, 0, s, n, r, z, q, partials, nb, sh.nz);
    return hipGetLastError();
}

template <typename TI, typename TC>
hipError_t launch_pcg_direction(const OpDesc<TC>& op, const TI* z, const double* p_old, double* p_new,
                                double* q, const double* scal, bool restart, double* partials,
                                hipStream_t s) {
    const Shape sh = stencil_shape(op.n);
    if (restart)
        hipLaunchKernelGGL((k_pcg_direction<TI, TC, true>), sh.grid, sh.block, 0, s, op.n, op.ih2, op.coeff, z,
                           p_old, p_new, q, scal, partials, sh.nz);
    else
        hipLaunchKernelGGL((k_pcg_direction<TI, TC, false>), sh.grid, sh.block, 0, s, op.n, op.ih2, op.coeff, z,
                           p_old, p_new, q, scal, partials, sh.nz);
    return hipGetLastError();
}

template <typename TI>
hipError_t launch_pcg_update(int n, double* phi, const double* p, double* r, const double* q, TI* rin,
                             const double* scal, double* partials, hipStream_t s) {
    const Shape sh = stencil_shape(n);
    hipLaunchKernelGGL((k_pcg_update<TI>), sh.grid, sh.block, 0, s, n, phi, p, r, q, rin, scal, partials, sh.nz);
    return hipGetLastError();
}

hipError_t launch_pcg_scalars(const double* partials, int nb, double* scal, int which, bool restart,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_scalars, dim3(1), dim3(1024), 0, s, partials, nb, scal, which, (int)restart);
    return hipGetLastError();
}

#define MG_PCG_INST(TI, TC)                                                                                       \
    template hipError_t launch_pcg_residual<TI, TC>(const OpDesc<TC>&, const double*, const double*, double,     \
                                                    double*, TI*, double*, hipStream_t);                         \
    template hipError_t launch_pcg_direction<TI, TC>(const OpDesc<TC>&, const TI*, const double*, double*,       \
                                                     double*, const double*, bool, double*, hipStream_t);
MG_PCG_INST(float, float)
MG_PCG_INST(float, double)
MG_PCG_INST(double, float)
MG_PCG_INST(double, double)
#undef MG_PCG_INST
template hipError_t launch_pcg_dots<float>(int, const double*, const float*, const double*, double*, hipStream_t);
template hipError_t launch_pcg_dots<double>(int, const double*, const double*, const double*, double*, hipStream_t);
template hipError_t launch_pcg_update<float>(int, double*, const double*, double*, const double*, float*,
                                             const double*, double*, hipStream_t);
template hipError_t launch_pcg_update<double>(int, double*, const double*, double*, const double*, double*,
                                              const double*, double*, hipStream_t);

}  // namespace mg
