/*
 * mg.h - C ABI of a matrix-free geometric-multigrid solver for periodic 3-D
 * Poisson problems on one AMD Instinct MI355X (gfx950).
 *
 * Problems solved (paper: "Fast(er)PM and Moving Mesh: JAX-native Geometric
 * Multigrid Methods"):
 *   - the periodic particle-mesh Poisson equation discretised with the
 *     second-order seven-point Laplacian, M phi = b (Sec. 2.1, eqs. poisson
 *     and linsys; Sec. 2.3);
 *   - the moving mesh's variable-coefficient operator in flux form,
 *     M phi = div(C grad phi) = b with a symmetric positive-definite 3x3
 *     coefficient C per cell (Sec. 4.3, eq. LB; Sec. 4.3.1).  C is the
 *     paper's sqrt(g) g^{ab}; its 19-point discretisation averages the
 *     diagonal coefficients onto faces and the tangential fluxes
 *     C^{ab} D0_b phi onto faces, which keeps M symmetric and negative
 *     semidefinite with the constants as null space.
 *
 * Method (Sec. 2.3, Fig. 1; Sec. 3.1; Sec. 3.4): V-cycles with
 * degree-v Chebyshev-accelerated Jacobi smoothing on the interval
 * [lmax/alpha, lmax] of D^-1 M (eq. flat_chebyshev; lmax = 2 for the
 * seven-point operator, a Gershgorin bound per level otherwise, App. C eq.
 * gersh), full-weighting restriction, trilinear prolongation and an exact
 * coarsest-level solve; outer defect correction r = b - M phi, phi += V(r)
 * warm-started from the caller's phi (Sec. 3.1, eq. kwarm).  In
 * MG_MIXED precision the V-cycle runs in float while the outer residual, the
 * update of phi and the coarsest solve run in double.
 *
 * Conventions shared by every entry point
 *   - A field is n*n*n contiguous values indexed [z][y][x] (x fastest),
 *     box length n*h, periodic in all three directions.
 *   - Every field pointer is DEVICE memory owned by the caller (for example
 *     a torch tensor), aligned to at least 16 bytes.  phi, b, lam and phibar
 *     are double.  The library never frees caller memory.
 *   - A coefficient field is 6 consecutive fields in the order
 *     (xx, yy, zz, xy, xz, yz), float or double as its dtype argument says.
 *   - All device work is ordered on the context's stream (hipStream_t passed
 *     as void*, NULL = the legacy default stream).  Entry points that return
 *     residual norms or status information synchronise that stream.
 *   - No exception crosses the ABI.  Every call returns an mg_status; on an
 *     error the context (if any) keeps a message for mg_last_error().
 *   - A context is not thread safe; distinct contexts are independent.
 */
#ifndef MG_H
#define MG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mg_status {
    MG_OK = 0,
    MG_ERR_INVALID = 1,        /* bad argument (sizes, levels, degree, null pointer, mode) */
    MG_ERR_INVALID_COEFF = 2,  /* coefficient field not finite or with C^{aa} <= 0 */
    MG_ERR_NOMEM = 3,          /* device allocation failed */
    MG_ERR_HIP = 4,            /* a HIP runtime call failed */
    MG_ERR_NONFINITE = 5,      /* NaN/Inf met in b, phi or a residual norm */
    MG_ERR_NOT_CONVERGED = 6   /* tolerance not reached in max_cycles; outputs valid */
} mg_status;

enum mg_precision {
    MG_FP64 = 0,   /* every step in double */
    MG_MIXED = 1,  /* V-cycle in float; outer residual, phi update, coarsest solve in double */
    MG_FP32 = 2    /* V-cycle and outer residual in float (phi is stored back as double) */
};

enum mg_smoother {
    MG_CHEBYSHEV = 0,  /* degree-v Chebyshev acceleration of Jacobi (eq. flat_chebyshev) */
    MG_JACOBI = 1      /* weighted Jacobi, omega and sweeps from mg_params (eq. flat_jacobi) */
};

enum mg_dtype {
    MG_DTYPE_F32 = 0,
    MG_DTYPE_F64 = 1
};

/* Reference switches (mg_params.options).  0, the default, runs every fused
 * kernel; each bit replaces one fusion by the plain sequence of single-step
 * kernels it stands for, so that fused and plain paths can be compared bit
 * for bit and timed against each other.  They change no arithmetic. */
enum mg_option {
    MG_OPT_NO_PAIR = 1,        /* every smoothing step its own kernel (no two- or three-step passes,
                                  no prolongation fused into post-smoothing) */
    MG_OPT_NO_VISIT = 2,       /* no fused visits of the 32^3 and 64^3 float levels */
    MG_OPT_NO_TAIL = 4,        /* levels of at most 16^3 points as separate kernels, not one workgroup */
    MG_OPT_NO_FUSED_SUMS = 8,  /* outer residual norms finished by their own kernel */
    MG_OPT_GRAPH = 16,         /* coarse sub-cycle replayed from a captured HIP graph */
    MG_OPT_ALL = 31
};

typedef struct mg_params {
    int n;               /* points per side, power of two, 8 <= n <= 2048 */
    int levels;          /* >= 1; the coarsest level has n >> (levels-1) >= 4 points per side */
    int cheb_degree;     /* 1..8: operator applications per smoothing pass */
    double cheb_alpha;   /* > 1: spectral interval [lmax/alpha, lmax] (paper: alpha ~ 8) */
    double h;            /* fine-grid spacing > 0 (box length 1 <=> h = 1/n) */
    int precision;       /* enum mg_precision */
    int smoother;        /* enum mg_smoother */
    double jacobi_omega; /* weighted-Jacobi factor (paper: 2/3) */
    int jacobi_sweeps;   /* weighted-Jacobi sweeps per smoothing pass (paper: 2) */
    int options;         /* bit mask of enum mg_option; 0 = every fused kernel */
} mg_params;

typedef struct mg_solve_info {
    int cycles;          /* V-cycles (outer iterations) executed */
    double rel_res0;     /* ||b - M phi0|| / ||b|| after projecting the mean out of b */
    double rel_res;      /* final relative residual */
    double* history;     /* optional HOST buffer: rel. residual before cycle 1, after each cycle */
    int history_cap;     /* capacity of history; entries written = min(cycles + 1, cap) */
} mg_solve_info;

typedef struct mg_ctx mg_ctx;

/* Fill *p with defaults for an n^3 grid: levels = log2(n) - 1 (coarsest 4^3,
 * Sec. 4.3.3), degree 3, alpha 8, h = 1/n, MG_MIXED, Chebyshev, omega 2/3,
 * 2 sweeps, options 0.  Host only. */
mg_status mg_params_default(mg_params* p, int n);

/* Check *p against the rules above without touching any device.  Returns
 * MG_OK or MG_ERR_INVALID.  Host only. */
mg_status mg_validate_params(const mg_params* p);

/* Create a solver context (Sec. 2.3: hierarchy of spacings h, 2h, 4h, ...).
 * coeff: NULL selects the constant-coefficient seven-point Laplacian;
 * otherwise a device pointer to 6 n^3 fields (xx, yy, zz, xy, xz, yz) of dtype
 * coeff_dtype, COPIED into the context (the caller may free it on return).
 * Coarse-level coefficients are the componentwise full-weighting restriction
 * of the fine ones (App. B restricts the geometry to every level).  The
 * coarsest level of a variable-coefficient context may have at most 8^3
 * points (it is solved with a dense pseudo-inverse).  stream: hipStream_t or
 * NULL.  On success *out owns its device memory until mg_destroy.
 * Errors: MG_ERR_INVALID (parameters), MG_ERR_INVALID_COEFF (coefficients not
 * finite or a diagonal component <= 0), MG_ERR_NOMEM, MG_ERR_HIP. */
mg_status mg_create(const mg_params* p, const void* coeff, int coeff_dtype,
                    void* stream, mg_ctx** out);

/* Variable-coefficient context rediscretised on every level from the
 * deformation potential (Sec. 4.3; App. B restricts the deformation field to
 * each coarse level): psi (device double n^3, read during the call only) is
 * restricted by full weighting level by level, psi_{l+1} = R psi_l, and the
 * coefficients of level l are C(psi_l) of mg_geometry at spacing 2^l h.
 * The fine level's coefficients are exactly mg_geometry(psi); in MG_MIXED the
 * outer residual uses them in double and the hierarchy in float.  Same
 * parameter rules as mg_create (coarsest level at most 8^3 points).
 * Errors as mg_create; MG_ERR_INVALID_COEFF also when the restricted
 * potential folds a coarse level's mesh (a diagonal coefficient <= 0 or not
 * finite there). */
mg_status mg_create_psi(const mg_params* p, const double* psi, void* stream, mg_ctx** out);

/* Free everything the context owns.  NULL is accepted. */
mg_status mg_destroy(mg_ctx* ctx);

/* Order all later work of the context on stream (hipStream_t, may be NULL). */
mg_status mg_set_stream(mg_ctx* ctx, void* stream);

/* One outer iteration in place: phi <- phi + V(b - M phi), the V-cycle of
 * Sec. 2.3 applied to the defect (Sec. 3.1 defect correction).  b's mean is
 * projected out first.  If rel_res_out is not NULL it receives
 * ||b - M phi_new|| / ||b|| (host pointer; the call then synchronises).
 * phi keeps whatever mean it had. */
mg_status mg_vcycle(mg_ctx* ctx, double* phi, const double* b, double* rel_res_out);

/* Solve M phi = b (Sec. 2.1, 2.3; warm start Sec. 3.1): project the mean out
 * of b, start from phi (initial guess, e.g. the previous step's solution),
 * test ||b - M phi|| / ||b|| <= tol before each cycle, run at most max_cycles
 * cycles, then remove the mean of phi (gauge).  phi is overwritten with the
 * solution.  If b is zero after projection, phi = 0 and rel_res = 0.
 * The loop also stops when the residual has failed to decrease by 0.1% over
 * two consecutive cycles (stagnation at the rounding floor of the precision).
 * info may be NULL.  Returns MG_ERR_NOT_CONVERGED (phi still valid) when the
 * tolerance is not reached, MG_ERR_NONFINITE on NaN/Inf.  Synchronises the
 * stream once per cycle (one 8-byte norm read back). */
mg_status mg_solve(mg_ctx* ctx, double* phi, const double* b, double tol,
                   int max_cycles, mg_solve_info* info);

/* A fixed number of warm-started cycles (Sec. 3.1: after an accurate first
 * solve, each time step runs a small, fixed number of defect-correction
 * cycles from the previous potential; the results section times warm solves
 * of one to four cycles).  Projects the mean out of b, runs exactly `cycles`
 * iterations phi <- phi + V(b - M phi) from the caller's phi with no
 * convergence test and no host wait between them, then removes the mean of
 * phi (gauge) as mg_solve does.  cycles >= 0 (0 only evaluates the residual
 * and gauge-fixes).  rel_res_out (host pointer, may be NULL) receives
 * ||b - M phi|| / ||b|| of the returned phi (0 if b is zero after
 * projection, in which case phi = 0).  Synchronises the stream twice: for
 * the mean of b at the start and for the final norms at the end.  Errors:
 * MG_ERR_INVALID, MG_ERR_NONFINITE (NaN/Inf in b or in the final residual),
 * MG_ERR_HIP. */
mg_status mg_cycles(mg_ctx* ctx, double* phi, const double* b, int cycles, double* rel_res_out);

/* Multigrid-preconditioned conjugate gradients (Sec. 3.2: the recycled
 * potential seeds a CG iteration preconditioned by multigrid): one V-cycle
 * from zero is the preconditioner B, phi the first iterate.  Flexible
 * (Polak-Ribiere) step beta = (z_k, r_k - r_{k-1}) / (z_{k-1}, r_{k-1}),
 * identical to textbook PCG for a fixed symmetric B and robust to the float
 * rounding of an MG_MIXED or MG_FP32 preconditioner.  The recurrences (r, p,
 * q = M p, phi) run in double in every precision mode.  Stops when the
 * recursively updated residual meets tol and the true residual confirms it;
 * if the true residual misses tol the iteration restarts from it, and stops
 * at the rounding floor when a restart brings no 0.1% improvement.
 * info->cycles counts CG iterations (one V-cycle each), history holds the
 * recursive residuals (the true one where a restart happened) and rel_res
 * the true final residual.  b's mean is projected out first and phi's mean
 * removed at the end, as in mg_solve.  Allocates four n^3 double work fields
 * in the context on first use.  Same errors as mg_solve. */
mg_status mg_solve_pcg(mg_ctx* ctx, double* phi, const double* b, double tol,
                       int max_iter, mg_solve_info* info);

/* Adjoint solve lam = M^+ phibar (Sec. 4.8, eq. adj_rhs): M is symmetric, so
 * this is the forward machinery on the cotangent; lam holds the initial
 * guess on entry and the zero-mean result on return.  With the paper's
 * weighted operator A = W^-1 M (eq. curv_operator) and b = sqrt(g) f, the
 * source cotangent is fbar = sqrt(g) * lam.  Same errors as mg_solve. */
mg_status mg_solve_adjoint(mg_ctx* ctx, double* lam, const double* phibar,
                           double tol, int max_cycles, mg_solve_info* info);

/* Operator VJP at a converged solution (Sec. 4.8, eq. adj_op): overwrite cbar
 * (device, 6 n^3 fields of dtype cbar_dtype) with dL/dC = -d(lam^T M(C) phi)/dC
 * for L with dL/db = lam.  Diagonal components: mean over the two a-faces of
 * (D+_a lam)(D+_a phi); off-diagonal (a,b): D0_a lam D0_b phi + D0_b lam D0_a phi
 * (the stored component carries both (a,b) and (b,a)).  lam and phi are double
 * device fields.  MG_ERR_INVALID for a seven-point (coeff == NULL) context. */
mg_status mg_coeff_grad(mg_ctx* ctx, const double* lam, const double* phi,
                        void* cbar, int cbar_dtype);

/* Moving-mesh geometry (Sec. 4.2, eqs. map, triad, metric): from the
 * deformation potential psi (device double n^3) compute the triad
 * J = I + Hess psi with second-order central stencils, sqrt(g) = det J and
 * C = det(J) J^-1 J^-T.  C_out: device, 6 n^3 fields of dtype (float or
 * double); sqrtg_out: device double n^3 (may be NULL).  n power of two >= 4. */
mg_status mg_geometry(int n, double h, const double* psi, void* C_out, int dtype,
                      double* sqrtg_out, void* stream);

/* Reverse mode of mg_geometry: psibar = (dC/dpsi)^T Cbar + (dsqrtg/dpsi)^T sqrtgbar.
 * Cbar: device double 6 n^3 with the symmetric storage convention of
 * mg_coeff_grad; sqrtgbar: device double n^3 or NULL (treated as zero);
 * psibar: device double n^3, overwritten.  Allocates a temporary of 6 n^3
 * doubles. */
mg_status mg_geometry_bwd(int n, double h, const double* psi, const double* Cbar,
                          const double* sqrtgbar, double* psibar, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops with a fixed memory budget, harnesses that forbid
 * hipMalloc): mg_geometry_bwd with the same arguments and the same result
 * bits, but its 6 n^3 double temporary replaced by a library-owned device
 * array of MG_NOALLOC_SCRATCH_BYTES per GPU (allocated when the library's
 * code is loaded on that GPU, held until the process ends), through which
 * the grid is processed in z slabs.  n <= MG_NOALLOC_MAX_N, else
 * MG_ERR_INVALID.  Calls no hipMalloc, hipFree or allocating routine and does
 * not synchronise (stream-ordered).  Every call on one GPU uses that GPU's
 * array, so calls that overlap on one GPU (different streams or threads)
 * race and must be ordered by the caller. */
#define MG_NOALLOC_MAX_N 512
#define MG_NOALLOC_SCRATCH_BYTES (48u * 1024u * 1024u)
mg_status mg_geometry_bwd_noalloc(int n, double h, const double* psi, const double* Cbar,
                                  const double* sqrtgbar, double* psibar, void* stream);

/* ---- initial guesses and force readout ----------------------------------- */

enum mg_predictor {
    MG_PREDICT_RECYCLE = 0,   /* out = phi1 */
    MG_PREDICT_GROWTH = 1,    /* out = growth * phi1, growth = D(a_n) / D(a_{n-1}) (eq. growth) */
    MG_PREDICT_LINEAR = 2,    /* out = 2 phi1 - phi2 */
    MG_PREDICT_QUADRATIC = 3  /* out = 3 phi1 - 3 phi2 + phi3 */
};

/* Initial guess for the next solve from earlier solutions (Sec. 3.2:
 * recycling, growth-scaled and polynomial-extrapolation predictors); phi1 is
 * the newest (phi_{n-1}), phi2 = phi_{n-2}, phi3 = phi_{n-3}.  Device double
 * n^3 fields; pointers the kind does not use may be NULL.  out may alias any
 * input (elementwise).  Stream-ordered, no synchronisation.
 * MG_ERR_INVALID for a bad n, kind, missing field or non-finite growth. */
mg_status mg_predict(int n, int kind, const double* phi1, const double* phi2,
                     const double* phi3, double growth, double* out, void* stream);

/* Force readout after a solve (Sec. 3.4: fourth-order finite-difference
 * gradient; Sec. 4.5.1, eq. accel): a = -scale J^-1 grad phi with
 * grad_a phi = (phi_{i-2} - 8 phi_{i-1} + 8 phi_{i+1} - phi_{i+2}) / (12 h)
 * along each axis and J = I + Hess psi (second-order stencils of
 * mg_geometry).  psi == NULL: uniform mesh, a = -scale grad phi.  scale is
 * the caller's normalisation (the paper's 3/2 Omega_m; 1 gives -grad phi).
 * phi, psi: device double n^3; a_out: device, 3 n^3 values (x, y, z
 * components, each an n^3 field) of dtype.  Stream-ordered. */
mg_status mg_accel(int n, double h, const double* phi, const double* psi,
                   double scale, void* a_out, int dtype, void* stream);

/* ---- single steps of the V-cycle, for testing and composition ------------
 * These act on caller double fields at level `level` of the context's
 * hierarchy (level 0 = fine, n >> level points per side) with the context's
 * operator, in double arithmetic.  They do not touch the context's solve
 * state. */

/* out = M_level u. */
mg_status mg_apply(mg_ctx* ctx, int level, const double* u, double* out);

/* One smoothing pass in place on level `level` (pre- and post-smoothing use
 * the same pass): x <- S(x, b), Chebyshev of the context's degree or weighted
 * Jacobi. */
mg_status mg_smooth(mg_ctx* ctx, int level, double* x, const double* b);

/* coarse = R(b - M_level x): residual and full-weighting restriction to
 * level + 1.  x may be NULL (treated as zero: coarse = R b). */
mg_status mg_residual_restrict(mg_ctx* ctx, int level, const double* x,
                               const double* b, double* coarse);

/* x += P e: trilinear prolongation from level + 1 to level, added to x. */
mg_status mg_prolong_add(mg_ctx* ctx, int level, const double* e, double* x);

/* e = zero-mean exact solution of M_c e = r - mean(r) on the coarsest level. */
mg_status mg_coarse_solve(mg_ctx* ctx, const double* r, double* e);

/* Gershgorin bound lmax of D^-1 M on each level (host array of `levels`
 * doubles; 2 for the seven-point operator). */
mg_status mg_level_lmax(const mg_ctx* ctx, double* lmax_out);

/* ---- steps of the inner V-cycle in the context's own precision -------------
 * One step of the V-cycle on level `level`, run through exactly the kernels
 * mg_solve launches there (row-wave, two- and three-step passes, the pass
 * from zero, the prolongation fused into post-smoothing, the fused 32^3 and
 * 64^3 visits and the single-workgroup tail kernel), in the context's inner
 * precision: float for MG_MIXED and MG_FP32, double for MG_FP64.  The double
 * inputs are rounded to that precision on entry and the result is widened to
 * double on exit, so a float step can be compared point by point with a
 * double reference.  Operations (Sec. 2.3, Fig. 1; eq. flat_chebyshev):
 *   MG_STEP_SMOOTH          out = S(x, b), one smoothing pass from x
 *   MG_STEP_SMOOTH_ZERO     out = S(0, b), the pass from zero (x unused)
 *   MG_STEP_PROLONG_SMOOTH  out = S(x + P e, b), prolongation of the coarse
 *                           correction e then the post-smoothing pass
 *   MG_STEP_RESIDUAL_RESTRICT  out = R(b - M x) on level + 1 (x, b unused: e)
 *   MG_STEP_PROLONG         out = x + P e
 *   MG_STEP_VCYCLE          out = V(0, b), the inner cycle from zero on
 *                           levels level .. coarsest (level 0: the cycle
 *                           that each defect-correction iteration applies to
 *                           its residual)
 * x, b, out: level-`level` fields (out on level + 1 for the restriction);
 * e: level-(level + 1) field; pointers an operation does not use may be
 * NULL.  All are caller-owned double device fields; out may alias an input.
 * The step works in the context's hierarchy buffers, so it must not overlap
 * a solve on the same context.  Stream-ordered, no synchronisation.
 * Errors: MG_ERR_INVALID (operation, level, missing pointer). */
enum mg_step {
    MG_STEP_SMOOTH = 0,
    MG_STEP_SMOOTH_ZERO = 1,
    MG_STEP_PROLONG_SMOOTH = 2,
    MG_STEP_RESIDUAL_RESTRICT = 3,
    MG_STEP_PROLONG = 4,
    MG_STEP_VCYCLE = 5
};
mg_status mg_inner_step(mg_ctx* ctx, int step, int level, const double* x, const double* e,
                        const double* b, double* out);

/* ---- timing of the dominant kernels ---------------------------------------
 * When enabled, every launch of a fine-level kernel inside mg_solve /
 * mg_cycles / mg_vcycle / mg_solve_pcg whose kind is in the mask is bracketed
 * by HIP events recorded by the kernel's own dispatch on the context's
 * stream.  Kinds: MG_TIME_STEP, the one-step smoothing kernels; MG_TIME_PAIR,
 * the kernels that apply two consecutive smoothing steps in one pass (and
 * the pass from zero that forms its first step on the fly); MG_TIME_TRIPLE,
 * the kernels that apply three steps in one pass from a nonzero iterate (with
 * the prolongation fused in front where it is); MG_TIME_OUTER, the outer
 * defect-correction kernel (phi update, FP64 residual, norms); MG_TIME_TRANSFER,
 * the fine level's residual + restriction and its separate prolongation.
 * mg_kernel_timing
 * returns, since the previous call: the number of such launches, their summed
 * duration in milliseconds and their summed algorithmic HBM bytes (every
 * field element the launch reads or writes counted once: iterate, previous
 * iterate, right-hand side, outputs and the six coefficient fields of a
 * variable-coefficient operator).  It synchronises the stream.  enable is the
 * mask (0 disables, the default); other values give MG_ERR_INVALID. */
enum mg_timing_kind {
    MG_TIME_STEP = 1,
    MG_TIME_PAIR = 2,
    MG_TIME_TRIPLE = 4,
    MG_TIME_OUTER = 8,
    MG_TIME_TRANSFER = 16
};
mg_status mg_enable_kernel_timing(mg_ctx* ctx, int enable);
mg_status mg_kernel_timing(mg_ctx* ctx, int* launches, double* total_ms, double* alg_bytes);

const char* mg_status_string(mg_status s);
const char* mg_last_error(const mg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* MG_H */
