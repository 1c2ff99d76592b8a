// Internal launch interface between the host orchestration (mg_api.cpp) and
// the gfx950 kernels (kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace mg {

// Operator of one level: constant-coefficient seven-point Laplacian when
// coeff == nullptr, otherwise the 19-point flux-form operator whose six
// coefficient fields start at coeff (stride n^3 elements).
template <typename TC>
struct OpDesc {
    int n;
    double ih2;          // 1 / h^2 of this level
    const TC* coeff;     // nullptr for the seven-point operator
};

// Number of thread blocks a stencil launch over an n^3 grid uses; partial
// sums buffers must hold at least this many doubles.
int stencil_blocks(int n);
// Number of per-block partial sums launch_outer_residual writes (seven-point
// operator when flat is true; residual in double when double_arith is true).
int outer_blocks(int n, bool flat, bool double_arith);

// ---- smoothing (Chebyshev / Jacobi step) ---------------------------------
// out = x + a (x - xprev) + c D^-1 (b - M x)      (xprev == nullptr: xprev = 0;
//                                                  x == nullptr: x = 0)
// out may alias xprev but not x or b.  Non-null events ev0/ev1 are recorded
// by the kernel's own dispatch (start and end of execution).
template <typename T, typename TC>
hipError_t launch_smooth_step(const OpDesc<TC>& op, const T* x, const T* xprev, const T* b,
                              T* out, double a, double c, hipStream_t s, hipEvent_t ev0 = nullptr,
                              hipEvent_t ev1 = nullptr);

// ---- residual + full-weighting restriction ---------------------------------
// coarse = R(b - M x) on the (n/2)^3 grid; x == nullptr means x = 0.  When the
// fused row kernel does not apply and `scratch` (n^3 elements, distinct from
// x, b and coarse) is given, the residual is formed there first and then
// restricted (two passes); without scratch a fused gather kernel is used.
template <typename T, typename TC>
hipError_t launch_residual_restrict(const OpDesc<TC>& op, const T* x, const T* b, T* coarse,
                                    T* scratch, hipStream_t s, hipEvent_t ev0 = nullptr,
                                    hipEvent_t ev1 = nullptr);

// coarse = R(fine), componentwise for `ncomp` consecutive fields.
template <typename T>
hipError_t launch_restrict(int n, const T* fine, T* coarse, int ncomp, hipStream_t s);

// ---- prolongation ------------------------------------------------------------
// x (n^3) += P e ((n/2)^3), trilinear.
template <typename T>
hipError_t launch_prolong_add(int n, const T* e, T* x, hipStream_t s, hipEvent_t ev0 = nullptr,
                              hipEvent_t ev1 = nullptr);

// ---- operator application ----------------------------------------------------
template <typename T, typename TC>
hipError_t launch_apply(const OpDesc<TC>& op, const T* u, T* out, hipStream_t s);

// ---- outer defect correction (double or float arithmetic TA) -----------------
// If e != nullptr: phi_out = phi_in + e, else phi_out unused (may be nullptr)
// and phi is phi_in.  r = (b - bmean) - M phi written as TR; per-block sums of
// r^2 (in double) written to partials[block].  phi_out must not alias phi_in.
// If x1 != nullptr it also receives c0 D^-1 r, the first smoothing step of the
// next V-cycle started from zero.
// partials receives three arrays of outer_blocks() per-block sums: sum of
// (b - bmean)^2, sum of r^2, and sum of the potential whose residual is formed
// (phi_out when e != nullptr, else phi_in), all in double.
template <typename TA, typename TR, typename TE, typename TC>
hipError_t launch_outer_residual(const OpDesc<TC>& op, const double* phi_in, const TE* e,
                                 double* phi_out, const double* b, double bmean, TR* r,
                                 TR* x1, double c0, double* partials, hipStream_t s,
                                 hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// ---- reductions ----------------------------------------------------------------
// partials[block] = sum over the block of (u - shift)^p, p in {1, 2}.
hipError_t launch_block_sums(int n, const double* u, double shift, int p, double* partials,
                             hipStream_t s);
// out[slot + k] = sum_{i < count} partials[k * count + i], k < arrays (one block);
// also into host_out[slot + k] (pinned host memory, visible to the host once an
// event recorded after the launch has completed) when host_out is not null.
hipError_t launch_finalize_sums(const double* partials, int count, int arrays, double* out, int slot,
                                hipStream_t s, double* host_out = nullptr);
// out[slot] = sum_{i < count} partials[i] in a fixed order (one block).
hipError_t launch_finalize_sum(const double* partials, int count, double* out, int slot,
                               hipStream_t s);
// out[slot] = max_{i < count} partials[i].
hipError_t launch_finalize_max(const double* partials, int count, double* out, int slot,
                               hipStream_t s);

// ---- elementwise -----------------------------------------------------------------
// dst = src - shift (double, may alias)
hipError_t launch_shift(size_t count, const double* src, double shift, double* dst, hipStream_t s);
// dst = src + e (double += T)
template <typename T>
hipError_t launch_add(size_t count, const double* src, const T* e, double* dst, hipStream_t s);
template <typename TD, typename TS>
hipError_t launch_convert(size_t count, const TS* src, TD* dst, hipStream_t s);
template <typename T>
hipError_t launch_fill(size_t count, T value, T* dst, hipStream_t s);

// ---- coefficient hierarchy -------------------------------------------------------
// partials[block] = max over the block of the Gershgorin bound of D^-1 M.
template <typename TC>
hipError_t launch_gershgorin(const OpDesc<TC>& op, double* partials, hipStream_t s);
// partials[block] = number of cells with a non-finite component or C^{aa} <= 0.
template <typename TC>
hipError_t launch_coeff_check(int n, const TC* coeff, double* partials, hipStream_t s);

// ---- coarsest level ----------------------------------------------------------------
// Seven-point operator: e = Q diag(1/lambda) Q^T r with the separable real
// Fourier basis Q (nc x nc, column-major basis vectors) and eigenvalues
// lam1[nc] per axis (lambda = lam1[kx] + lam1[ky] + lam1[kz], the zero mode
// dropped).  nc <= 16.  One block.
template <typename T>
hipError_t launch_coarse_flat(int nc, const double* Q, const double* lam1, const T* r, T* e,
                              hipStream_t s);
// Variable coefficients: e = G r with the dense symmetric pseudo-inverse G
// (N x N, N = nc^3 <= 512).
template <typename T>
hipError_t launch_coarse_dense(int N, const double* G, const T* r, T* e, hipStream_t s);

// ---- gradients and geometry ---------------------------------------------------------
template <typename TO>
hipError_t launch_coeff_grad(int n, double ih2, const double* lam, const double* phi, TO* cbar,
                             hipStream_t s);
template <typename TO>
hipError_t launch_geometry(int n, double ih2, const double* psi, TO* C, double* sqrtg,
                           hipStream_t s);
// Jbar (symmetric storage: off-diagonal = Jbar_ab + Jbar_ba) of the planes
// zlo .. zlo + planes - 1 (mod n), 6 planes n^2 doubles laid out [c][plane][y][x];
// planes = 0: the whole grid (6 n^3 doubles, zlo = 0).
hipError_t launch_geometry_bwd_cell(int n, double ih2, const double* psi, const double* Cbar,
                                    const double* sqrtgbar, double* Jbar, hipStream_t s,
                                    int zlo = 0, int planes = 0);
// psibar = sum_ab Hess_ab(Jbar_ab) on the planes z0 .. z0 + count - 1, from a
// Jbar slab (zlo, planes) that holds z0 - 1 .. z0 + count (or the whole grid:
// planes = 0, count = 0).
hipError_t launch_hessian_adjoint(int n, double ih2, const double* Jbar, double* psibar,
                                  hipStream_t s, int zlo = 0, int planes = 0, int z0 = 0,
                                  int count = 0);

// ---- multigrid-preconditioned conjugate gradients (double recurrences) ----------
// Scalars live in device memory so no pass waits for the host:
enum PcgSlot { kPcgRz = 0, kPcgAlpha = 1, kPcgBeta = 2, kPcgRr = 3, kPcgPq = 4, kPcgSlots = 8 };
// Per-block partial sums written by the passes below: `pcg_blocks(n)` per sum.
int pcg_blocks(int n);
// r = (b - bmean) - M phi (double), rin = r in the preconditioner's type TI;
// partials[blk] = sum of r^2.
template <typename TI, typename TC>
hipError_t launch_pcg_residual(const OpDesc<TC>& op, const double* phi, const double* b, double bmean,
                               double* r, TI* rin, double* partials, hipStream_t s);
// partials[blk] = sum r z, partials[nb + blk] = sum z q (0 when q == nullptr).
template <typename TI>
hipError_t launch_pcg_dots(int n, const double* r, const TI* z, const double* q, double* partials,
                           hipStream_t s);
// p_new = z + beta p_old (p_old unread when restart), q = M p_new,
// partials[blk] = sum p_new q.  beta = scal[kPcgBeta].
template <typename TI, typename TC>
hipError_t launch_pcg_direction(const OpDesc<TC>& op, const TI* z, const double* p_old, double* p_new,
                                double* q, const double* scal, bool restart, double* partials,
                                hipStream_t s);
// phi += alpha p, r -= alpha q, rin = r; partials[blk] = sum r^2.  alpha = scal[kPcgAlpha].
template <typename TI>
hipError_t launch_pcg_update(int n, double* phi, const double* p, double* r, const double* q, TI* rin,
                             const double* scal, double* partials, hipStream_t s);
// Sums of the partials and the scalar recurrences, one block:
//   kPcgBeta:  rz_new = sum r z; beta = restart ? 0 : -alpha (sum z q) / rz_old (flexible,
//              Polak-Ribiere form); scal[kPcgRz] = rz_new
//   kPcgAlpha: alpha = scal[kPcgRz] / sum p q
//   kPcgRr:    scal[kPcgRr] = sum r^2
hipError_t launch_pcg_scalars(const double* partials, int nb, double* scal, int which, bool restart,
                              hipStream_t s);

// ---- initial guesses and force readout ----------------------------------------------
// out = c1 phi1 + c2 phi2 + c3 phi3 (terms with a zero coefficient are not read).
hipError_t launch_combine3(size_t count, double c1, const double* phi1, double c2, const double* phi2,
                           double c3, const double* phi3, double* out, hipStream_t s);
// a = -scale J^-1 grad4 phi, J = I + Hess psi (psi == nullptr: J = I); a: 3 n^3 of TO.
template <typename TO>
hipError_t launch_accel(int n, double h, const double* phi, const double* psi, double scale, TO* a,
                        hipStream_t s);

}  // namespace mg
