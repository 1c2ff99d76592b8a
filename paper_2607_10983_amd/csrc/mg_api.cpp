// Host side of the C ABI declared in include/mg.h: parameter validation,
// hierarchy allocation, Chebyshev schedules, coarsest-level solver setup and
// the outer defect-correction loop.  All device work is issued on the
// context's stream through the launchers of kernels.hip.
#include "mg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "flat_row.h"
#include "kernels.h"
#include "tail.h"
#include "var_row.h"
#include "visit.h"

#include <type_traits>

using namespace mg;

namespace {

struct Level {
    int n = 0;
    size_t N = 0;
    double h = 0, ih2 = 0;
    void* x[3] = {nullptr, nullptr, nullptr};  // inner iterates; x[2] only where two-step kernels run
    void* b = nullptr;                // inner right-hand side / restricted residual
    void* coeff = nullptr;            // inner-precision coefficients (6 N), nullptr for 7-point
    double lmax = 2.0;                // Gershgorin bound of D^-1 M
    int cur = 0;                      // which x holds the current iterate
    // smoothing schedule: step k computes x + a_k (x - x_prev) + c_k D^-1 (b - M x)
    std::vector<double> a, c;
};

struct TimingPair {
    hipEvent_t start, stop;
};

}  // namespace

struct mg_ctx {
    mg_params p{};
    hipStream_t stream = nullptr;
    bool var = false;
    bool inner_double = true;   // inner V-cycle in double (MG_FP64) or float
    std::vector<Level> lev;
    // fine-level coefficients used by the outer residual
    void* coeff_outer = nullptr;
    bool coeff_outer_double = true;
    bool coeff_outer_owned = false;
    double* phi_tmp = nullptr;  // second buffer for the phi update
    double* partials = nullptr;
    int nparts = 0;        // partial sums written by launch_block_sums on the fine grid
    int nparts_outer = 0;  // partial sums written by launch_outer_residual
    double* dscal = nullptr;    // device scalars
    double* hscal = nullptr;    // pinned host mirror
    // The outer sums wait to be finished by the next pass from zero on level 0
    // (an extra block of that kernel) instead of a finalize launch.
    bool pending_sums = false;
    bool fuse_sums = true;
    double* Q = nullptr;        // coarsest seven-point basis and eigenvalues
    double* lam1 = nullptr;
    double* G = nullptr;        // coarsest variable-coefficient pseudo-inverse
    int tail_start = -1;        // first level run by the single-workgroup tail kernel, -1 = none
    bool x1_ready = false;      // the outer residual already wrote level 0's first smoothing step
    int x1_buf = 0;             // ... into this level-0 iterate buffer
    // The coarse sub-cycle (levels 1 .. coarsest) touches only context-owned
    // buffers with fixed arguments, so it can be captured once into a HIP graph
    // and replayed with one launch per V-cycle (MG_GRAPH set at creation).
    bool use_graph = false;
    bool capturing = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t coarse_graph = nullptr;
    hipGraphExec_t coarse_exec = nullptr;
    int coarse_cur = 0;
    hipEvent_t norm_ev = nullptr;  // completion of the per-cycle norm readback
    // The sums finished inside the pass from zero need no event: the block
    // that writes them to the pinned mirror makes them visible at system
    // scope and then writes sums_seq to hscal[kHostFlagSlot], which the host
    // polls.  An event there cost a 5.6 us stall between the pass from zero
    // and the next kernel at 256^3 (4.6 us without its system-scope release).
    double sums_seq = 0.0;
    bool scal_flag = false;  // the pending readback is the flag, not norm_ev
    bool use_pairs = true;         // last two steps of a smoothing pass in one two-step kernel
    bool use_visits = true;        // fused visits of the 32^3 and 64^3 levels (float hierarchy)
    bool use_tail = true;          // levels of at most 16^3 points in one workgroup
    // conjugate-gradient state (allocated by the first mg_solve_pcg)
    double* pcg_r = nullptr;
    double* pcg_p[2] = {nullptr, nullptr};
    double* pcg_q = nullptr;
    double* pcg_s = nullptr;
    double* pcg_partials = nullptr;
    double* scratch = nullptr;  // double scratch for the single-step entry points
    size_t scratch_elems = 0;
    std::string err;
    // timing of the fine-level smoothing kernel
    int timing = 0;  // mask of timed kernel kinds (MG_TIME_STEP, MG_TIME_PAIR, MG_TIME_TRIPLE)
    std::vector<TimingPair> events;
    size_t events_used = 0;
    int timed_launches = 0;
    double timed_ms = 0.0;
    double timed_bytes = 0.0;
};

namespace {

const char* kStatus[] = {"MG_OK",
                         "MG_ERR_INVALID: invalid argument",
                         "MG_ERR_INVALID_COEFF: coefficient field not finite or with a non-positive diagonal component",
                         "MG_ERR_NOMEM: device allocation failed",
                         "MG_ERR_HIP: HIP runtime error",
                         "MG_ERR_NONFINITE: NaN or Inf encountered",
                         "MG_ERR_NOT_CONVERGED: tolerance not reached"};

mg_status fail(mg_ctx* ctx, mg_status s, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return s;
}

#define HIPCHK(ctx, ...)                                                                           \
    do {                                                                                           \
        hipError_t e_ = (__VA_ARGS__);                                                             \
        if (e_ != hipSuccess)                                                                      \
            return fail((ctx), MG_ERR_HIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

mg_status dalloc(mg_ctx* ctx, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return MG_OK;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, MG_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return MG_OK;
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

int coarsest_n(const mg_params& p) { return p.n >> (p.levels - 1); }

// Chebyshev schedule on [lmax/alpha, lmax] (three-term recurrence, x_prev form).
void make_schedule(const mg_params& p, Level& L) {
    L.a.clear();
    L.c.clear();
    if (p.smoother == MG_JACOBI) {
        for (int k = 0; k < p.jacobi_sweeps; ++k) {
            L.a.push_back(0.0);
            L.c.push_back(p.jacobi_omega);
        }
        return;
    }
    const double lmin = L.lmax / p.cheb_alpha;
    const double theta = 0.5 * (L.lmax + lmin), delta = 0.5 * (L.lmax - lmin), sigma = theta / delta;
    double rho = 1.0 / sigma;
    L.a.push_back(0.0);
    L.c.push_back(1.0 / theta);
    for (int k = 1; k < p.cheb_degree; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        L.a.push_back(rn * rho);
        L.c.push_back(2.0 * rn / delta);
        rho = rn;
    }
}

// Real orthonormal Fourier basis of the periodic second difference on nc points.
void flat_basis(int nc, double hc, std::vector<double>& Q, std::vector<double>& lam) {
    Q.assign((size_t)nc * nc, 0.0);
    lam.assign(nc, 0.0);
    const double pi = std::acos(-1.0);
    auto eig = [&](int m) { double s = std::sin(pi * m / nc); return -4.0 * s * s / (hc * hc); };
    for (int j = 0; j < nc; ++j) Q[j + nc * 0] = 1.0 / std::sqrt((double)nc);
    lam[0] = 0.0;
    for (int m = 1; m < nc / 2; ++m) {
        for (int j = 0; j < nc; ++j) {
            Q[j + nc * (2 * m - 1)] = std::sqrt(2.0 / nc) * std::cos(2.0 * pi * m * j / nc);
            Q[j + nc * (2 * m)] = std::sqrt(2.0 / nc) * std::sin(2.0 * pi * m * j / nc);
        }
        lam[2 * m - 1] = lam[2 * m] = eig(m);
    }
    for (int j = 0; j < nc; ++j) Q[j + nc * (nc - 1)] = (j % 2 ? -1.0 : 1.0) / std::sqrt((double)nc);
    lam[nc - 1] = eig(nc / 2);
}

// Dense matrix of the 19-point operator on the coarsest level (host, double).
void assemble_dense(int n, double ih2, const std::vector<double>& C, std::vector<double>& M) {
    const int N = n * n * n;
    M.assign((size_t)N * N, 0.0);
    auto id = [n](int x, int y, int z) { return (((z % n + n) % n) * n + ((y % n + n) % n)) * n + ((x % n + n) % n); };
    auto cc = [&](int c, int x, int y, int z) { return C[(size_t)c * N + id(x, y, z)]; };
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                const int i = id(x, y, z);
                const int p[3] = {x, y, z};
                for (int a = 0; a < 3; ++a)
                    for (int s = -1; s <= 1; s += 2) {
                        int q[3] = {p[0], p[1], p[2]};
                        q[a] += s;
                        const double cf = 0.5 * (cc(a, x, y, z) + cc(a, q[0], q[1], q[2]));
                        M[(size_t)i * N + id(q[0], q[1], q[2])] += cf * ih2;
                        M[(size_t)i * N + i] -= cf * ih2;
                    }
                const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
                for (int k = 0; k < 3; ++k) {
                    const int a = pa[k], b = pb[k], comp = 3 + k;
                    for (int sa = -1; sa <= 1; sa += 2)
                        for (int sb = -1; sb <= 1; sb += 2) {
                            int qa[3] = {p[0], p[1], p[2]}, qb[3] = {p[0], p[1], p[2]}, q[3] = {p[0], p[1], p[2]};
                            qa[a] += sa;
                            qb[b] += sb;
                            q[a] += sa;
                            q[b] += sb;
                            const double v = sa * sb * (cc(comp, qa[0], qa[1], qa[2]) + cc(comp, qb[0], qb[1], qb[2])) * 0.25 * ih2;
                            M[(size_t)i * N + id(q[0], q[1], q[2])] += v;
                        }
                }
            }
}

// Zero-mean pseudo-inverse of a symmetric semidefinite M with null space span(1):
// B = M - s 11^T / N is definite, and G = P B^-1 P with P = I - 11^T / N.
bool pseudo_inverse(int N, const std::vector<double>& M, std::vector<double>& G) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += std::fabs(M[(size_t)i * N + i]);
    s /= N;
    std::vector<double> A((size_t)N * 2 * N, 0.0);
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < N; ++j) A[(size_t)i * 2 * N + j] = M[(size_t)i * N + j] - s / N;
        A[(size_t)i * 2 * N + N + i] = 1.0;
    }
    const int W = 2 * N;
    for (int col = 0; col < N; ++col) {  // Gauss-Jordan with partial pivoting
        int piv = col;
        for (int r = col + 1; r < N; ++r)
            if (std::fabs(A[(size_t)r * W + col]) > std::fabs(A[(size_t)piv * W + col])) piv = r;
        if (A[(size_t)piv * W + col] == 0.0) return false;
        if (piv != col)
            for (int j = 0; j < W; ++j) std::swap(A[(size_t)piv * W + j], A[(size_t)col * W + j]);
        const double inv = 1.0 / A[(size_t)col * W + col];
        for (int j = 0; j < W; ++j) A[(size_t)col * W + j] *= inv;
        for (int r = 0; r < N; ++r) {
            if (r == col) continue;
            const double f = A[(size_t)r * W + col];
            if (f == 0.0) continue;
            for (int j = 0; j < W; ++j) A[(size_t)r * W + j] -= f * A[(size_t)col * W + j];
        }
    }
    std::vector<double> Bi((size_t)N * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) Bi[(size_t)i * N + j] = A[(size_t)i * W + N + j];
    // G = P Bi P
    std::vector<double> rm(N, 0.0), cm(N, 0.0);
    double tm = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            rm[i] += Bi[(size_t)i * N + j] / N;
            cm[j] += Bi[(size_t)i * N + j] / N;
        }
    for (int i = 0; i < N; ++i) tm += rm[i] / N;
    G.assign((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) G[(size_t)i * N + j] = Bi[(size_t)i * N + j] - rm[i] - cm[j] + tm;
    return true;
}

template <typename T>
OpDesc<T> op_of(const Level& L) {
    return OpDesc<T>{L.n, L.ih2, (const T*)L.coeff};
}

// ---- fine-level smoothing kernel timing ----------------------------------------------
// The event pair travels with the kernel's own dispatch (hipExtLaunchKernel),
// so the elapsed time is the kernel's execution time, as a profiler sees it.
mg_status time_events(mg_ctx* c, bool fine, int kind, hipEvent_t* ev0, hipEvent_t* ev1) {
    *ev0 = *ev1 = nullptr;
    if (!(c->timing & kind) || !fine) return MG_OK;
    if (c->events_used == c->events.size()) {
        TimingPair tp;
        // timing only: no system-scope release (an L2 writeback of every XCD,
        // 4-6 us of stall around the timed kernel)
        HIPCHK(c, hipEventCreateWithFlags(&tp.start, hipEventDisableSystemFence));
        HIPCHK(c, hipEventCreateWithFlags(&tp.stop, hipEventDisableSystemFence));
        c->events.push_back(tp);
    }
    *ev0 = c->events[c->events_used].start;
    *ev1 = c->events[c->events_used].stop;
    return MG_OK;
}
mg_status time_end(mg_ctx* c, bool fine, int kind, double bytes) {
    if (!(c->timing & kind) || !fine) return MG_OK;
    c->events_used++;
    c->timed_launches++;
    c->timed_bytes += bytes;
    if (c->events_used >= 16384) {  // harvest to bound the pool
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < c->events_used; ++i) {
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, c->events[i].start, c->events[i].stop));
            c->timed_ms += ms;
        }
        c->events_used = 0;
    }
    return MG_OK;
}

// ---- inner V-cycle ----------------------------------------------------------------------
// One smoothing pass on level l in inner precision T.  from_zero: the iterate is 0.
// index of an iterate buffer other than `cur` among x[0], x[1]
inline int other(int cur) { return cur == 0 ? 1 : 0; }

// The outer residual kernel can write level 0's first smoothing step (when
// level 0 is not itself run by the tail kernel).
inline bool x1_fusable(const mg_ctx* c) { return c->tail_start != 0 && c->lev.size() > 1; }

// Level l (not the coarsest, not run by the tail kernel) is visited by the
// fused visit kernels: float hierarchy, seven-point operator, 32^3 or 64^3
// points; pre (post) selects the visit before (after) the coarse correction.
inline bool visit_level(const mg_ctx* c, int l, bool pre) {
    if (!(c->use_visits && !c->var && !c->inner_double && c->p.smoother == MG_CHEBYSHEV &&
          l + 1 < (int)c->lev.size() && l != c->tail_start))
        return false;
    const int n = c->lev[l].n, v = (int)c->lev[l].a.size();
    return pre ? visit_pre_applies(n, v) : visit_post_applies(n, v);
}

// Level l's post-smoothing pass (three Chebyshev steps) runs fused with the
// prolongation before it.
inline bool post_fused(const mg_ctx* c, int l, size_t elem) {
    const Level& L = c->lev[l];
    return c->p.smoother == MG_CHEBYSHEV && L.a.size() == 3 && c->use_pairs && !c->var &&
           triple_pro_applies(L.n, elem);
}

// Level l's post-smoothing pass (Chebyshev, an even number of steps) starts
// with a pair that forms x + P e itself: split rows, where the three-step
// kernels do not run.
inline bool post_pair_fused(const mg_ctx* c, int l, size_t elem) {
    const Level& L = c->lev[l];
    return c->p.smoother == MG_CHEBYSHEV && L.a.size() % 2 == 0 && c->use_pairs && !c->var &&
           L.x[2] != nullptr && pair_pro_applies(L.n, elem);
}

// Level l runs its pass from zero as one three-step kernel (first step formed
// from b on the fly): seven-point operator, two-step kernels available, and
// at least three steps per pass.
inline bool from_zero_triple(const mg_ctx* c, int l) {
    return c->use_pairs && !c->var && c->lev[l].x[2] != nullptr && c->lev[l].a.size() >= 3;
}

// pro_e (not from zero): the pass starts from x + P pro_e, formed by its
// first kernel (a pair on split rows), instead of a prolongation launch.
// Level l without two-step kernels (rows over 2 KB, row kernels with LDS)
// starts its post-smoothing pass (Chebyshev, at least two steps) with a step
// that forms x + P e itself and a step that forms that x_prev pointwise, in
// place of a prolongation launch.
inline bool post_step_fused(const mg_ctx* c, int l, size_t elem) {
    const Level& L = c->lev[l];
    return c->use_pairs && !c->var && c->p.smoother == MG_CHEBYSHEV && L.a.size() >= 2 && L.x[2] == nullptr &&
           step_pro_applies(L.n, elem);
}

// Level l without two-step kernels (rows over 2 KB) starts a pass from zero
// of at least three Chebyshev steps with one step read from b alone and one
// step whose x_prev (the pointwise first step) is formed from b, so the
// first step is never written.
inline bool from_zero_stepb(const mg_ctx* c, int l) {
    const Level& L = c->lev[l];
    return c->use_pairs && !c->var && c->p.smoother == MG_CHEBYSHEV && L.a.size() >= 3 && L.x[2] == nullptr &&
           row_kernels_apply(L.n) && l + 1 < (int)c->lev.size() && l != c->tail_start && !visit_level(c, l, true);
}

template <typename T>
mg_status smooth_level(mg_ctx* c, int l, bool from_zero, const T* pro_e = nullptr) {
    Level& L = c->lev[l];
    const OpDesc<T> op = op_of<T>(L);
    int cur = L.cur;
    int prev = -1;  // buffer of x_{k-1}, -1 when x_{k-1} = 0 or not needed
    const bool cheb = c->p.smoother == MG_CHEBYSHEV;
    const bool fine = (l == 0);
    const double fbytes = (double)L.N * sizeof(T);
    const double cbytes = c->var ? 6.0 * (double)L.N * sizeof(T) : 0.0;
    T* bufs[3] = {(T*)L.x[0], (T*)L.x[1], (T*)L.x[2]};
    const int v = (int)L.a.size();
    // the last two steps of the pass run as one two-step kernel where it exists
    const bool pairs = c->use_pairs && L.x[2] != nullptr && !c->var;
    // 19-point: the last two Chebyshev steps of the pass run as one kernel
    const bool vpairs = c->use_pairs && c->var && cheb && L.x[2] != nullptr;
    bool prev_b = false;  // x_{k-1} is the pointwise first step c0 D^-1 b, formed by the next kernel
    bool prev_p = false;  // x_{k-1} is x_old + P pro_e (x_old in bufs[prev]), formed by the next kernel
    for (int k = 0; k < v; ++k) {
        double bytes = 0.0;
        if (k == 0 && from_zero && l == 0 && c->x1_ready) {  // formed by the outer residual kernel
            c->x1_ready = false;
            cur = c->x1_buf;
            prev = -1;
            continue;
        }
        // Steps pair up from the end of the pass: an even number of remaining
        // steps runs as two-step kernels.  A pair that is not the last one also
        // writes its first step (the next pair's x_prev); that needs two free
        // buffers, i.e. no x_prev of its own.
        const int rem = v - k;
        const bool has_prev = cheb && prev >= 0;
        const bool need_y1 = cheb && rem > 2;
        // a pass from zero of degree 4: steps 0 and 1 from b alone (b -> x_2),
        // then steps 2 and 3 as a pair whose x_prev = x_1 is formed from b
        // (b, x_2 -> x_4): 5 field passes instead of 7 for steps 0-2 in one
        // kernel (b -> x_3, x_2) and step 3 on its own
        const bool fromb = k == 0 && from_zero && cheb && v == 4 && from_zero_triple(c, l);
        const bool triple = k == 0 && from_zero && from_zero_triple(c, l) && !fromb;
        const bool stepb = k == 0 && from_zero && from_zero_stepb(c, l);
        // a pass of three steps that does not start from zero: one three-step kernel
        const bool triple3 = k == 0 && !from_zero && cheb && v == 3 && c->use_pairs && !c->var &&
                             triple_kernels_apply(L.n, sizeof(T));
        const bool pair = pairs && rem >= 2 && rem % 2 == 0 && !(k == 0 && from_zero) && !(need_y1 && has_prev);
        const bool vpair = vpairs && rem == 2 && !(k == 0 && from_zero);
        // pro_e: a pair starts the pass (split rows), or a step that prolongs on the fly (rows over 2 KB)
        const bool pro_step = k == 0 && pro_e != nullptr && !pair;
        if (pro_step && !post_step_fused(c, l, sizeof(T))) return MG_ERR_INVALID;
        const int kind = triple3                               ? MG_TIME_TRIPLE
                         : (pair || triple || vpair) && !fromb ? MG_TIME_PAIR
                                                               : MG_TIME_STEP;
        hipEvent_t ev0, ev1;
        mg_status st = time_events(c, fine, kind, &ev0, &ev1);
        if (st != MG_OK) return st;
        if (pro_step) {  // step 0 from x0 = x + P e formed on the fly; x (the old iterate) is kept
            const double D = -6.0 * L.ih2;
            const int out = other(cur);
            HIPCHK(c, launch_smooth_pro_row<T>(L.n, L.ih2, bufs[cur], pro_e, (const T*)L.b, bufs[out], L.a[0],
                                               L.c[0] / D, c->stream, ev0, ev1));
            bytes = (3.0 + 1.0 / 8.0) * fbytes;  // x, e, b; x_1
            prev = cur;
            prev_p = true;
            cur = out;
        } else if (prev_p) {  // step 1, x_prev = x0 formed from the old iterate and e; out replaces the old iterate
            const double D = -6.0 * L.ih2;
            const int out = prev;
            HIPCHK(c, launch_smooth_prevp_row<T>(L.n, L.ih2, bufs[cur], bufs[prev], pro_e, (const T*)L.b,
                                                 bufs[out], L.a[k], L.c[k] / D, c->stream, ev0, ev1));
            bytes = (4.0 + 1.0 / 8.0) * fbytes;  // x_1, x, e, b; x_2
            prev_p = false;
            prev = cur;
            cur = out;
        } else if (stepb) {  // steps 0 and 1 from b alone (b -> x_2); the next step forms x_prev from b
            const double D = -6.0 * L.ih2;
            HIPCHK(c, launch_smooth_fromb_row<T>(L.n, L.ih2, (const T*)L.b, bufs[0], L.a[1], L.c[1] / D,
                                                 L.c[0] / D, c->stream, ev0, ev1));
            bytes = 2.0 * fbytes;  // b; x_2
            prev = -1;
            prev_b = true;
            cur = 0;
            k = 1;
        } else if (prev_b && !pair) {  // x_prev = c0 D^-1 b, formed from the b rows
            const double D = -6.0 * L.ih2;
            const int out = other(cur);
            HIPCHK(c, launch_smooth_prevb_row<T>(L.n, L.ih2, bufs[cur], (const T*)L.b, bufs[out], L.a[k],
                                                 L.c[k] / D, L.c[0] / D, c->stream, ev0, ev1));
            bytes = 3.0 * fbytes;  // x, b; out
            prev_b = false;
            prev = cur;
            cur = out;
        } else if (fromb) {
            const int out = 1;
            const double D = -6.0 * L.ih2;
            HIPCHK(c, launch_smooth_fromb_row<T>(L.n, L.ih2, (const T*)L.b, bufs[out], L.a[1], L.c[1] / D,
                                                 L.c[0] / D, c->stream, ev0, ev1));
            bytes = 2.0 * fbytes;  // b; x_2
            prev = -1;
            prev_b = true;
            cur = out;
            k = 1;  // two steps done
        } else if (triple3) {
            const int out = other(cur);
            const double D = -6.0 * L.ih2;
            HIPCHK(c, launch_smooth_triple_row<T>(L.n, L.ih2, bufs[cur], (const T*)L.b, bufs[out], L.a[0],
                                                  L.c[0] / D, L.a[1], L.c[1] / D, L.a[2], L.c[2] / D, c->stream, ev0,
                                                  ev1));
            bytes = 3.0 * fbytes;  // x, b; x_3
            prev = -1;
            cur = out;
            k = 2;  // three steps done
        } else if (triple) {
            // steps 0, 1, 2 of the pass from zero: reads b, writes x_3 (and x_2
            // when a fourth step needs it as x_prev)
            const bool y1 = cheb && v > 3;
            const int out = 0, mid = y1 ? 1 : -1;
            const double D = -6.0 * L.ih2;
            // on level 0 the pending outer sums are finished by an extra block
            const bool sums = l == 0 && c->pending_sums;
            const SumsJob job{c->partials, c->nparts_outer, 3, c->dscal, 1, c->hscal, sums ? c->sums_seq + 1.0 : 0.0};
            HIPCHK(c, launch_smooth_pair_row<T>(L.n, L.ih2, nullptr, nullptr, (const T*)L.b, bufs[out],
                                                mid >= 0 ? bufs[mid] : nullptr, L.a[1], L.c[1] / D, L.a[2],
                                                L.c[2] / D, c->stream, ev0, ev1, 1, L.c[0] / D,
                                                sums ? &job : nullptr));
            if (sums) {
                c->sums_seq += 1.0;
                c->scal_flag = true;
                c->pending_sums = false;
            }
            bytes = (2.0 + (mid >= 0 ? 1.0 : 0.0)) * fbytes;  // b; x_3 [, x_2]
            prev = mid;
            cur = out;
            k = 2;  // three steps done
        } else if (vpair) {  // x, x_prev -> y2 in the third buffer (the kernel reads both on halo rows)
            const T* xp = has_prev ? bufs[prev] : nullptr;
            const int out = has_prev ? 3 - cur - prev : other(cur);
            HIPCHK(c, launch_var_smooth_pair<T, T>(L.n, L.ih2, op.coeff, bufs[cur], xp, (const T*)L.b, bufs[out],
                                                   L.a[k], L.c[k], L.a[k + 1], L.c[k + 1], c->stream, ev0, ev1));
            bytes = (3.0 + (xp ? 1.0 : 0.0)) * fbytes + cbytes;  // x, [x_prev], b, C; y2
            prev = -1;
            cur = out;
            ++k;  // the pair's second step
        } else if (pair) {
            const T* xp = has_prev ? bufs[prev] : nullptr;
            int out, mid = -1;
            if (has_prev) {
                out = 3 - cur - prev;
            } else {
                const int f1 = cur == 0 ? 1 : 0;
                const int f2 = 3 - cur - f1;
                out = need_y1 ? f2 : f1;
                mid = need_y1 ? f1 : -1;
            }
            const double D = -6.0 * L.ih2;  // c / D rounded as in the single-step launch
            // after a step from b, level 0 finishes the pending outer sums here
            const bool sums = prev_b && l == 0 && c->pending_sums;
            const T* ec = k == 0 ? pro_e : nullptr;  // x0 = x + P e formed by this pair
            const SumsJob job{c->partials, c->nparts_outer, 3, c->dscal, 1, c->hscal, sums ? c->sums_seq + 1.0 : 0.0};
            HIPCHK(c, launch_smooth_pair_row<T>(L.n, L.ih2, bufs[cur], xp, (const T*)L.b, bufs[out],
                                                mid >= 0 ? bufs[mid] : nullptr, L.a[k], L.c[k] / D, L.a[k + 1],
                                                L.c[k + 1] / D, c->stream, ev0, ev1, prev_b ? 2 : 0, L.c[0] / D,
                                                sums ? &job : nullptr, ec));
            if (sums) {
                c->sums_seq += 1.0;
                c->scal_flag = true;
                c->pending_sums = false;
            }
            // x, [x_prev], b; y2, [y1]; [e once per coarse point]
            bytes = (3.0 + (xp ? 1.0 : 0.0) + (mid >= 0 ? 1.0 : 0.0) + (ec ? 1.0 / 8.0 : 0.0)) * fbytes;
            prev_b = false;
            prev = mid;
            cur = out;
            ++k;  // the pair's second step
        } else if (k == 0 && from_zero) {
            cur = 0;
            prev = -1;
            HIPCHK(c, launch_smooth_step<T, T>(op, nullptr, nullptr, (const T*)L.b, bufs[0], 0.0, L.c[0], c->stream,
                                               ev0, ev1));
            bytes = 2.0 * fbytes + cbytes;  // read b (and C for D), write x
        } else {
            const T* xp = (cheb && prev >= 0) ? bufs[prev] : nullptr;
            const int out = (cheb && prev >= 0) ? prev : other(cur);
            HIPCHK(c, launch_smooth_step<T, T>(op, bufs[cur], xp, (const T*)L.b, bufs[out], L.a[k], L.c[k],
                                               c->stream, ev0, ev1));
            bytes = (xp ? 4.0 : 3.0) * fbytes + cbytes;  // read x, [x_prev], b (, C); write out
            prev = cur;
            cur = out;
        }
        st = time_end(c, fine, kind, bytes);
        if (st != MG_OK) return st;
    }
    L.cur = cur;
    return MG_OK;
}

template <typename T>
mg_status coarse_level(mg_ctx* c, int l) {
    Level& L = c->lev[l];
    L.cur = 0;
    if (!c->var)
        HIPCHK(c, launch_coarse_flat<T>(L.n, c->Q, c->lam1, (const T*)L.b, (T*)L.x[0], c->stream));
    else
        HIPCHK(c, launch_coarse_dense<T>((int)L.N, c->G, (const T*)L.b, (T*)L.x[0], c->stream));
    return MG_OK;
}

template <typename T>
mg_status tail_cycle(mg_ctx* c, int l0) {
    TailArgs<T> a{};
    const int L = (int)c->lev.size();
    a.nlev = L - l0;
    const bool cheb = c->p.smoother == MG_CHEBYSHEV;
    a.sched.cheb = cheb ? 1 : 0;
    a.sched.steps = (int)c->lev[l0].a.size();
    for (int k = 0; k < a.nlev; ++k) {
        Level& Lv = c->lev[l0 + k];
        a.n[k] = Lv.n;
        int lg = 0;
        while ((1 << lg) < Lv.n) ++lg;
        a.lg[k] = lg;
        a.ih2[k] = Lv.ih2;
        a.x0[k] = (T*)Lv.x[0];
        a.x1[k] = (T*)Lv.x[1];
        a.b[k] = (T*)Lv.b;
        for (int j = 0; j < a.sched.steps; ++j) {
            a.sched.a[k][j] = Lv.a[j];
            a.sched.c[k][j] = Lv.c[j];
        }
    }
    a.Q = c->Q;
    a.lam1 = c->lam1;
    HIPCHK(c, launch_tail<T>(a, c->stream));
    // the tail writes the first tail level's result to that level's buffer x0
    c->lev[l0].cur = 0;
    return MG_OK;
}

template <typename T>
mg_status vcycle_from_zero(mg_ctx* c, int l);

// r_{l+1} = R(b_l - M_l x_l) into level l+1's right-hand side; the buffer of
// the previous iterate is free here and serves as residual scratch.
template <typename T>
mg_status residual_restrict_level(mg_ctx* c, int l) {
    Level& L = c->lev[l];
    Level& Lc = c->lev[l + 1];
    const bool fine = (l == 0);
    hipEvent_t ev0, ev1;
    mg_status st = time_events(c, fine, MG_TIME_TRANSFER, &ev0, &ev1);
    if (st != MG_OK) return st;
    HIPCHK(c, launch_residual_restrict<T, T>(op_of<T>(L), (const T*)L.x[L.cur], (const T*)L.b, (T*)Lc.b,
                                             (T*)L.x[other(L.cur)], c->stream, ev0, ev1));
    // seven-point: x, b read, r_{l+1} written; 19-point: the timed pass forms
    // the fine residual (x, b, C read, r written) and a second pass restricts it
    const double N = (double)L.N, s = sizeof(T);
    const double bytes = c->var ? N * (3.0 * s + 6.0 * s) : N * (2.0 + 1.0 / 8.0) * s;
    return time_end(c, fine, MG_TIME_TRANSFER, bytes);
}

// Up-leg of level l: x_l += P e_{l+1}, then the post-smoothing pass (one
// kernel for both where the prolongation is fused into the three-step pass).
template <typename T>
mg_status post_level(mg_ctx* c, int l) {
    Level& L = c->lev[l];
    Level& Lc = c->lev[l + 1];
    const bool fine = (l == 0);
    hipEvent_t ev0, ev1;
    mg_status st;
    if (post_fused(c, l, sizeof(T))) {  // prolongation and the three-step post-smoothing pass in one kernel
        if ((st = time_events(c, fine, MG_TIME_TRIPLE, &ev0, &ev1)) != MG_OK) return st;
        const double D = -6.0 * L.ih2;  // c / D rounded as in the single-step launch
        const int out = other(L.cur);
        HIPCHK(c, launch_prolong_triple_row<T>(L.n, L.ih2, (const T*)L.x[L.cur], (const T*)Lc.x[Lc.cur],
                                               (const T*)L.b, (T*)L.x[out], L.a[0], L.c[0] / D, L.a[1],
                                               L.c[1] / D, L.a[2], L.c[2] / D, c->stream, ev0, ev1));
        L.cur = out;
        // x, b read, x_3 written, e read once per coarse point
        return time_end(c, fine, MG_TIME_TRIPLE, (3.0 + 1.0 / 8.0) * (double)L.N * sizeof(T));
    }
    // the prolongation runs inside the pass's first pair, or its first two steps
    if (post_pair_fused(c, l, sizeof(T)) || post_step_fused(c, l, sizeof(T)))
        return smooth_level<T>(c, l, false, (const T*)Lc.x[Lc.cur]);
    if ((st = time_events(c, fine, MG_TIME_TRANSFER, &ev0, &ev1)) != MG_OK) return st;
    HIPCHK(c, launch_prolong_add<T>(L.n, (const T*)Lc.x[Lc.cur], (T*)L.x[L.cur], c->stream, ev0, ev1));
    if ((st = time_end(c, fine, MG_TIME_TRANSFER, (2.0 + 1.0 / 8.0) * (double)L.N * sizeof(T))) != MG_OK) return st;
    return smooth_level<T>(c, l, false);
}

// Capture V(0, b_1) on level 1 and below into c->coarse_exec.
template <typename T>
mg_status capture_coarse(mg_ctx* c) {
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t saved = c->stream;
    c->stream = c->cap_stream;
    c->capturing = true;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    mg_status st = vcycle_from_zero<T>(c, 1);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->capturing = false;
    c->stream = saved;
    if (st != MG_OK) {
        if (e == hipSuccess && g) (void)hipGraphDestroy(g);
        return st;
    }
    HIPCHK(c, e);
    c->coarse_graph = g;
    HIPCHK(c, hipGraphInstantiate(&c->coarse_exec, g, nullptr, nullptr, 0));
    c->coarse_cur = c->lev[1].cur;
    return MG_OK;
}

// x_l = V(0, b_l)
template <typename T>
mg_status vcycle_from_zero(mg_ctx* c, int l) {
    const int last = (int)c->lev.size() - 1;
    if (l == 1 && last >= 2 && c->use_graph && !c->capturing) {
        if (!c->coarse_exec) {
            mg_status st = capture_coarse<T>(c);
            if (st != MG_OK) return st;
        }
        HIPCHK(c, hipGraphLaunch(c->coarse_exec, c->stream));
        c->lev[1].cur = c->coarse_cur;
        return MG_OK;
    }
    if (l == c->tail_start) return tail_cycle<T>(c, l);
    if (l == last) return coarse_level<T>(c, l);
    Level& L = c->lev[l];
    Level& Lc = c->lev[l + 1];
    mg_status st = MG_OK;
    const int v = (int)L.a.size();
    if (std::is_same<T, float>::value && visit_level(c, l, true)) {  // one launch before the coarse level
        if (l == 0) c->x1_ready = false;
        HIPCHK(c, launch_visit_pre(L.n, L.ih2, (const float*)L.b, (float*)L.x[0], (float*)Lc.b, L.a.data(),
                                   L.c.data(), v, c->stream));
        L.cur = 0;
    } else {
        if ((st = smooth_level<T>(c, l, true)) != MG_OK) return st;
        if ((st = residual_restrict_level<T>(c, l)) != MG_OK) return st;
    }
    if ((st = vcycle_from_zero<T>(c, l + 1)) != MG_OK) return st;
    if (std::is_same<T, float>::value && visit_level(c, l, false)) {  // and one after it
        const int nx = other(L.cur);
        HIPCHK(c, launch_visit_post(L.n, L.ih2, (const float*)L.x[L.cur], (const float*)Lc.x[Lc.cur],
                                    (const float*)L.b, (float*)L.x[nx], L.a.data(), L.c.data(), v, c->stream));
        L.cur = nx;
        return MG_OK;
    }
    return post_level<T>(c, l);
}

// ---- outer residual dispatch ---------------------------------------------------------------
// r = (b - mean b) - M phi (phi = phi_in + e when e != null); per-block r^2 sums into partials.
// With next_cycle set, the kernel also writes the first smoothing step of the
// V-cycle that follows (x = c0 D^-1 r on level 0).
mg_status outer_residual(mg_ctx* c, const double* phi_in, const void* e, double* phi_out, const double* b,
                         double bmean, bool next_cycle = false) {
    Level& L = c->lev[0];
    const int n = L.n;
    const double ih2 = L.ih2;
    const bool x1 = next_cycle && x1_fusable(c) && !from_zero_triple(c, 0) && !from_zero_stepb(c, 0) &&
                    !visit_level(c, 0, true);
    const double c0 = L.c.empty() ? 0.0 : L.c[0];
    // x1 goes to a buffer other than the one holding e (the previous cycle's result)
    const int xb = other(L.cur);
    hipEvent_t ev0, ev1;
    mg_status st = time_events(c, true, MG_TIME_OUTER, &ev0, &ev1);
    if (st != MG_OK) return st;
    hipError_t err;
    if (c->p.precision == MG_FP64) {
        OpDesc<double> op{n, ih2, (const double*)c->coeff_outer};
        err = launch_outer_residual<double, double, double, double>(op, phi_in, (const double*)e, phi_out, b, bmean,
                                                                    (double*)L.b, x1 ? (double*)L.x[xb] : nullptr, c0,
                                                                    c->partials, c->stream, ev0, ev1);
    } else if (c->p.precision == MG_MIXED) {
        float* x1p = x1 ? (float*)L.x[xb] : nullptr;
        if (c->coeff_outer_double) {
            OpDesc<double> op{n, ih2, (const double*)c->coeff_outer};
            err = launch_outer_residual<double, float, float, double>(op, phi_in, (const float*)e, phi_out, b, bmean,
                                                                      (float*)L.b, x1p, c0, c->partials, c->stream,
                                                                      ev0, ev1);
        } else {
            OpDesc<float> op{n, ih2, (const float*)c->coeff_outer};
            err = launch_outer_residual<double, float, float, float>(op, phi_in, (const float*)e, phi_out, b, bmean,
                                                                     (float*)L.b, x1p, c0, c->partials, c->stream,
                                                                     ev0, ev1);
        }
    } else {
        OpDesc<float> op{n, ih2, (const float*)c->coeff_outer};
        err = launch_outer_residual<float, float, float, float>(op, phi_in, (const float*)e, phi_out, b, bmean,
                                                                (float*)L.b, x1 ? (float*)L.x[xb] : nullptr, c0,
                                                                c->partials, c->stream, ev0, ev1);
    }
    HIPCHK(c, err);
    c->x1_ready = x1;
    c->x1_buf = xb;
    // phi (and e, phi_out) and b in their storage types, r (and x1) in the inner type, C once
    const double si = c->inner_double ? 8.0 : 4.0;
    const double sc = c->var ? 6.0 * (c->coeff_outer_double ? 8.0 : 4.0) : 0.0;
    const double per_pt = 8.0 + 8.0 + si + (e ? si + 8.0 : 0.0) + (x1 ? si : 0.0) + sc;
    return time_end(c, true, MG_TIME_OUTER, per_pt * (double)L.N);
}

mg_status read_scalars(mg_ctx* c, int count) {
    HIPCHK(c, hipMemcpyAsync(c->hscal, c->dscal, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MG_OK;
}

mg_status inner_vcycle(mg_ctx* c) {
    return c->inner_double ? vcycle_from_zero<double>(c, 0) : vcycle_from_zero<float>(c, 0);
}

const void* inner_e(mg_ctx* c) { return c->lev[0].x[c->lev[0].cur]; }

mg_status check_ctx(mg_ctx* c) { return c ? MG_OK : MG_ERR_INVALID; }

template <typename F>
hipError_t with_op(mg_ctx* c, int level, F f) {
    const Level& L = c->lev[level];
    if (!c->var || c->inner_double) return f(OpDesc<double>{L.n, L.ih2, (const double*)L.coeff});
    return f(OpDesc<float>{L.n, L.ih2, (const float*)L.coeff});
}

}  // namespace

// =============================================================================================
// C ABI
// =============================================================================================
extern "C" {

const char* mg_status_string(mg_status s) {
    if ((int)s < 0 || (int)s > 6) return "unknown mg_status";
    return kStatus[(int)s];
}

const char* mg_last_error(const mg_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

mg_status mg_params_default(mg_params* p, int n) {
    if (!p) return MG_ERR_INVALID;
    p->n = n;
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    p->levels = lg - 1 > 1 ? lg - 1 : 1;
    p->cheb_degree = 3;
    p->cheb_alpha = 8.0;
    p->h = n > 0 ? 1.0 / n : 0.0;
    p->precision = MG_MIXED;
    p->smoother = MG_CHEBYSHEV;
    p->jacobi_omega = 2.0 / 3.0;
    p->jacobi_sweeps = 2;
    p->options = 0;
    return MG_OK;
}

mg_status mg_validate_params(const mg_params* p) {
    if (!p) return MG_ERR_INVALID;
    if (!is_pow2(p->n) || p->n < 8 || p->n > 2048) return MG_ERR_INVALID;
    if (p->levels < 1 || p->levels > 12) return MG_ERR_INVALID;
    const int nc = coarsest_n(*p);
    if (nc < 4 || nc > 16) return MG_ERR_INVALID;
    if (p->cheb_degree < 1 || p->cheb_degree > 8) return MG_ERR_INVALID;
    if (!(p->cheb_alpha > 1.0) || !std::isfinite(p->cheb_alpha)) return MG_ERR_INVALID;
    if (!(p->h > 0.0) || !std::isfinite(p->h)) return MG_ERR_INVALID;
    if (p->precision < MG_FP64 || p->precision > MG_FP32) return MG_ERR_INVALID;
    if (p->smoother != MG_CHEBYSHEV && p->smoother != MG_JACOBI) return MG_ERR_INVALID;
    if ((p->options & ~MG_OPT_ALL) != 0) return MG_ERR_INVALID;
    if (p->smoother == MG_JACOBI) {
        if (!(p->jacobi_omega > 0.0 && p->jacobi_omega < 2.0)) return MG_ERR_INVALID;
        if (p->jacobi_sweeps < 1 || p->jacobi_sweeps > 16) return MG_ERR_INVALID;
    }
    return MG_OK;
}

mg_status mg_destroy(mg_ctx* c) {
    if (!c) return MG_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    for (auto& L : c->lev) {
        dfree(L.x[0]);
        dfree(L.x[1]);
        dfree(L.x[2]);
        dfree(L.b);
        dfree(L.coeff);
    }
    if (c->coeff_outer_owned) dfree(c->coeff_outer);
    dfree(c->phi_tmp);
    dfree(c->partials);
    dfree(c->dscal);
    if (c->hscal) (void)hipHostFree(c->hscal);
    dfree(c->Q);
    dfree(c->lam1);
    dfree(c->G);
    dfree(c->scratch);
    dfree(c->pcg_r);
    dfree(c->pcg_p[0]);
    dfree(c->pcg_p[1]);
    dfree(c->pcg_q);
    dfree(c->pcg_s);
    dfree(c->pcg_partials);
    for (auto& e : c->events) {
        (void)hipEventDestroy(e.start);
        (void)hipEventDestroy(e.stop);
    }
    if (c->coarse_exec) (void)hipGraphExecDestroy(c->coarse_exec);
    if (c->coarse_graph) (void)hipGraphDestroy(c->coarse_graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->norm_ev) (void)hipEventDestroy(c->norm_ev);
    delete c;
    return MG_OK;
}

static mg_status create_impl(mg_ctx* c, const void* coeff, int coeff_dtype, const double* psi = nullptr) {
    const mg_params& p = c->p;
    c->var = coeff != nullptr || psi != nullptr;
    c->inner_double = p.precision == MG_FP64;
    if (c->var && coarsest_n(p) > 8)
        return fail(c, MG_ERR_INVALID, "variable-coefficient coarsest level must have at most 8^3 points");
    const size_t Tsz = c->inner_double ? sizeof(double) : sizeof(float);
    // reference switches of this context (mg_params.options)
    c->use_pairs = (p.options & MG_OPT_NO_PAIR) == 0;
    c->use_visits = (p.options & MG_OPT_NO_VISIT) == 0;
    c->fuse_sums = (p.options & MG_OPT_NO_FUSED_SUMS) == 0;
    c->use_tail = (p.options & MG_OPT_NO_TAIL) == 0;
    c->use_graph = (p.options & MG_OPT_GRAPH) != 0;
    c->lev.resize(p.levels);
    for (int l = 0; l < p.levels; ++l) {
        Level& L = c->lev[l];
        L.n = p.n >> l;
        L.N = (size_t)L.n * L.n * L.n;
        L.h = p.h * (double)(1 << l);
        L.ih2 = 1.0 / (L.h * L.h);
        mg_status st;
        if ((st = dalloc(c, &L.x[0], L.N * Tsz)) != MG_OK) return st;
        if ((st = dalloc(c, &L.x[1], L.N * Tsz)) != MG_OK) return st;
        const bool third = c->use_pairs && (c->var ? var_pair_applies(L.n, Tsz) && p.smoother == MG_CHEBYSHEV &&
                                                         p.cheb_degree >= 2
                                                   : pair_kernels_apply(L.n, Tsz));
        if (third && (st = dalloc(c, &L.x[2], L.N * Tsz)) != MG_OK) return st;
        if ((st = dalloc(c, &L.b, L.N * Tsz)) != MG_OK) return st;
    }
    const size_t N0 = c->lev[0].N;
    mg_status st;
    if ((st = dalloc(c, (void**)&c->phi_tmp, N0 * sizeof(double))) != MG_OK) return st;
    // replaying the coarse sub-cycle from a HIP graph measured slower than eager
    // launches on this platform; MG_OPT_GRAPH keeps it available
    c->nparts = stencil_blocks(p.n);
    c->nparts_outer = outer_blocks(p.n, !c->var, p.precision != MG_FP32);
    {
        // three arrays: the outer kernels write three partial sums per block
        const int np = c->nparts > c->nparts_outer ? c->nparts : c->nparts_outer;
        if ((st = dalloc(c, (void**)&c->partials, 3 * (size_t)np * sizeof(double))) != MG_OK) return st;
    }
    if ((st = dalloc(c, (void**)&c->dscal, 16 * sizeof(double))) != MG_OK) return st;
    // coherent: the finalize kernel writes the outer sums into it directly
    HIPCHK(c, hipHostMalloc((void**)&c->hscal, 16 * sizeof(double), hipHostMallocCoherent));
    HIPCHK(c, hipEventCreateWithFlags(&c->norm_ev, hipEventDisableTiming));
    c->hscal[kHostFlagSlot] = 0.0;

    if (c->var) {
        // fine coefficients in double, validated, restricted level by level
        std::vector<double*> c64(p.levels, nullptr);
        auto free64 = [&]() {
            for (auto q : c64) dfree(q);
        };
        for (int l = 0; l < p.levels; ++l)
            if ((st = dalloc(c, (void**)&c64[l], 6 * c->lev[l].N * sizeof(double))) != MG_OK) {
                free64();
                return st;
            }
        // count of invalid cells of level l into hscal[0]
        auto check_level = [&](int l) -> hipError_t {
            hipError_t e = launch_coeff_check<double>(c->lev[l].n, c64[l], c->partials, c->stream);
            if (e == hipSuccess) e = launch_finalize_sum(c->partials, stencil_blocks(c->lev[l].n), c->dscal, 0, c->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(c->hscal, c->dscal, sizeof(double), hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            return e;
        };
        hipError_t e = hipSuccess;
        if (psi) {
            // every level rediscretised from the potential restricted to it
            std::vector<double*> pl(p.levels, nullptr);
            auto freep = [&]() {
                for (int l = 1; l < p.levels; ++l) dfree(pl[l]);
            };
            pl[0] = const_cast<double*>(psi);
            for (int l = 1; l < p.levels; ++l)
                if ((st = dalloc(c, (void**)&pl[l], c->lev[l].N * sizeof(double))) != MG_OK) {
                    freep();
                    free64();
                    return st;
                }
            for (int l = 0; l < p.levels && e == hipSuccess; ++l) {
                if (l > 0) e = launch_restrict<double>(c->lev[l - 1].n, pl[l - 1], pl[l], 1, c->stream);
                if (e == hipSuccess) e = launch_geometry<double>(c->lev[l].n, c->lev[l].ih2, pl[l], c64[l], nullptr, c->stream);
            }
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            freep();
            if (e != hipSuccess) { free64(); HIPCHK(c, e); }
            for (int l = 0; l < p.levels; ++l) {
                if ((e = check_level(l)) != hipSuccess) { free64(); HIPCHK(c, e); }
                if (c->hscal[0] != 0.0) {
                    free64();
                    return fail(c, MG_ERR_INVALID_COEFF,
                                std::to_string((long long)c->hscal[0]) + " cells of level " + std::to_string(l) +
                                    " with a folded mesh (non-finite or non-positive diagonal coefficients)");
                }
            }
        } else {
            e = coeff_dtype == MG_DTYPE_F64
                    ? launch_convert<double, double>(6 * N0, (const double*)coeff, c64[0], c->stream)
                    : launch_convert<double, float>(6 * N0, (const float*)coeff, c64[0], c->stream);
            if (e == hipSuccess) e = check_level(0);
            if (e != hipSuccess) { free64(); HIPCHK(c, e); }
            if (c->hscal[0] != 0.0) {
                free64();
                return fail(c, MG_ERR_INVALID_COEFF,
                            std::to_string((long long)c->hscal[0]) + " cells with non-finite or non-positive diagonal coefficients");
            }
            for (int l = 0; l + 1 < p.levels; ++l) {
                e = launch_restrict<double>(c->lev[l].n, c64[l], c64[l + 1], 6, c->stream);
                if (e != hipSuccess) { free64(); HIPCHK(c, e); }
            }
        }
        for (int l = 0; l + 1 < p.levels; ++l) {
            OpDesc<double> op{c->lev[l].n, c->lev[l].ih2, c64[l]};
            e = launch_gershgorin<double>(op, c->partials, c->stream);
            if (e == hipSuccess) e = launch_finalize_max(c->partials, stencil_blocks(c->lev[l].n), c->dscal, 0, c->stream);
            if (e != hipSuccess) { free64(); HIPCHK(c, e); }
            if ((st = read_scalars(c, 1)) != MG_OK) { free64(); return st; }
            c->lev[l].lmax = c->hscal[0];
        }
        // coarsest dense pseudo-inverse (host, double)
        {
            Level& Lc = c->lev.back();
            std::vector<double> hc(6 * Lc.N), M, G;
            e = hipMemcpyAsync(hc.data(), c64.back(), hc.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) { free64(); HIPCHK(c, e); }
            assemble_dense(Lc.n, Lc.ih2, hc, M);
            if (!pseudo_inverse((int)Lc.N, M, G)) {
                free64();
                return fail(c, MG_ERR_INVALID_COEFF, "coarsest operator is singular beyond its constant null space");
            }
            if ((st = dalloc(c, (void**)&c->G, G.size() * sizeof(double))) != MG_OK) { free64(); return st; }
            e = hipMemcpyAsync(c->G, G.data(), G.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) { free64(); HIPCHK(c, e); }
        }
        // level storage in inner precision; outer fine copy
        if (c->inner_double) {
            for (int l = 0; l < p.levels; ++l) {
                c->lev[l].coeff = c64[l];
                c64[l] = nullptr;
            }
            c->coeff_outer = c->lev[0].coeff;
            c->coeff_outer_double = true;
            c->coeff_outer_owned = false;
        } else {
            for (int l = 0; l < p.levels; ++l) {
                if ((st = dalloc(c, &c->lev[l].coeff, 6 * c->lev[l].N * sizeof(float))) != MG_OK) { free64(); return st; }
                e = launch_convert<float, double>(6 * c->lev[l].N, c64[l], (float*)c->lev[l].coeff, c->stream);
                if (e != hipSuccess) { free64(); HIPCHK(c, e); }
            }
            if (p.precision == MG_MIXED && (coeff_dtype == MG_DTYPE_F64 || psi)) {
                c->coeff_outer = c64[0];  // keep the double values for the outer residual
                c64[0] = nullptr;
                c->coeff_outer_double = true;
                c->coeff_outer_owned = true;
            } else {
                c->coeff_outer = c->lev[0].coeff;
                c->coeff_outer_double = false;
                c->coeff_outer_owned = false;
            }
        }
        HIPCHK(c, hipStreamSynchronize(c->stream));
        free64();
    } else {
        Level& Lc = c->lev.back();
        std::vector<double> Q, lam;
        flat_basis(Lc.n, Lc.h, Q, lam);
        if ((st = dalloc(c, (void**)&c->Q, Q.size() * sizeof(double))) != MG_OK) return st;
        if ((st = dalloc(c, (void**)&c->lam1, lam.size() * sizeof(double))) != MG_OK) return st;
        HIPCHK(c, hipMemcpyAsync(c->Q, Q.data(), Q.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->lam1, lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->coeff_outer = nullptr;
        // levels of at most 16^3 points down to a coarsest of at most 8^3 run in one kernel
        const int steps = p.smoother == MG_JACOBI ? p.jacobi_sweeps : p.cheb_degree;
        if (Lc.n <= 8 && steps <= kTailMaxSteps && c->use_tail) {
            int l0 = p.levels - 1;
            while (l0 > 0 && c->lev[l0 - 1].n <= 16 && p.levels - (l0 - 1) <= kTailMaxLevels) --l0;
            if (p.levels - l0 >= 2) c->tail_start = l0;
        }
    }
    for (auto& L : c->lev) make_schedule(p, L);
    return MG_OK;
}

mg_status mg_create(const mg_params* p, const void* coeff, int coeff_dtype, void* stream, mg_ctx** out) {
    if (!out) return MG_ERR_INVALID;
    *out = nullptr;
    if (mg_validate_params(p) != MG_OK) return MG_ERR_INVALID;
    if (coeff && coeff_dtype != MG_DTYPE_F32 && coeff_dtype != MG_DTYPE_F64) return MG_ERR_INVALID;
    mg_ctx* c = new (std::nothrow) mg_ctx();
    if (!c) return MG_ERR_NOMEM;
    c->p = *p;
    c->stream = (hipStream_t)stream;
    mg_status st = create_impl(c, coeff, coeff_dtype);
    if (st != MG_OK) {
        std::fprintf(stderr, "mg_create: %s\n", c->err.c_str());
        mg_destroy(c);
        return st;
    }
    *out = c;
    return MG_OK;
}

mg_status mg_set_stream(mg_ctx* c, void* stream) {
    if (!c) return MG_ERR_INVALID;
    c->stream = (hipStream_t)stream;
    return MG_OK;
}

// mean of b into dscal[slot] (sum), then the caller divides
static mg_status device_sum(mg_ctx* c, const double* u, double shift, int pw, int slot) {
    HIPCHK(c, launch_block_sums(c->p.n, u, shift, pw, c->partials, c->stream));
    HIPCHK(c, launch_finalize_sum(c->partials, c->nparts, c->dscal, slot, c->stream));
    return MG_OK;
}

// Readback of device scalars through an event, so the host can enqueue more
// work before it waits for the values.
static mg_status post_scalars(mg_ctx* c, int count) {
    HIPCHK(c, hipMemcpyAsync(c->hscal, c->dscal, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipEventRecord(c->norm_ev, c->stream));
    c->scal_flag = false;
    return MG_OK;
}
// The three outer sums (slots 1..3), finalized straight into the pinned host
// mirror as well; the event marks when the host may read them.
static mg_status post_outer_sums(mg_ctx* c) {
    HIPCHK(c, launch_finalize_sums(c->partials, c->nparts_outer, 3, c->dscal, 1, c->stream, c->hscal));
    HIPCHK(c, hipEventRecord(c->norm_ev, c->stream));
    c->scal_flag = false;
    return MG_OK;
}
// Level 0's inner V-cycle starts with the pass-from-zero kernel, which can
// finish the outer sums in an extra block.
static bool sums_in_pass_from_zero(const mg_ctx* c) {
    return c->fuse_sums && c->lev.size() > 1 && c->tail_start != 0 && !visit_level(c, 0, true) &&
           from_zero_triple(c, 0);
}
// Outer residual of the solve loop and its three sums.  When a V-cycle is
// enqueued right after it (cycle_follows) and starts with the pass from zero,
// the sums are left pending for that kernel; flush_sums finishes them
// otherwise.  Either way norm_ev marks when the host may read them.
static mg_status outer_with_sums(mg_ctx* c, const double* phi_in, const void* e, double* phi_out, const double* b,
                                 double bmean, bool cycle_follows) {
    mg_status st = outer_residual(c, phi_in, e, phi_out, b, bmean, true);
    if (st != MG_OK) return st;
    if (cycle_follows && sums_in_pass_from_zero(c)) {
        c->pending_sums = true;
        return MG_OK;
    }
    return post_outer_sums(c);
}
static mg_status flush_sums(mg_ctx* c) {
    if (!c->pending_sums) return MG_OK;
    c->pending_sums = false;
    return post_outer_sums(c);
}
static mg_status wait_scalars(mg_ctx* c) {
    if (!c->scal_flag) {
        HIPCHK(c, hipEventSynchronize(c->norm_ev));
        return MG_OK;
    }
    // Poll the flag.  Only after 50 ms of waiting is the stream asked whether
    // it still runs: a stream query enqueues a marker, which costs a
    // 5.8 us stall in front of the next kernel.
    const volatile double* flag = c->hscal + kHostFlagSlot;
    auto last = std::chrono::steady_clock::now();
    for (unsigned i = 1;; ++i) {
        if (*flag == c->sums_seq) break;
        if ((i & 4095) != 0) continue;
        const auto now = std::chrono::steady_clock::now();
        if (now - last < std::chrono::milliseconds(50)) continue;
        last = now;
        const hipError_t e = hipStreamQuery(c->stream);
        if (e != hipSuccess && e != hipErrorNotReady) HIPCHK(c, e);
        if (e == hipSuccess && *flag != c->sums_seq) return fail(c, MG_ERR_HIP, "outer sums flag not raised");
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    c->scal_flag = false;
    return MG_OK;
}

static mg_status solve_impl(mg_ctx* c, double* phi, const double* b, double tol, int max_cycles,
                            mg_solve_info* info) {
    const size_t N0 = c->lev[0].N;
    const double invN = 1.0 / (double)N0;
    mg_status st;
    if ((st = device_sum(c, b, 0.0, 1, 0)) != MG_OK) return st;
    if ((st = read_scalars(c, 1)) != MG_OK) return st;
    const double bmean = c->hscal[0] * invN;
    if (!std::isfinite(bmean)) return fail(c, MG_ERR_NONFINITE, "source contains NaN or Inf");
    // the outer kernel also sums (b - bmean)^2 (slot 1) and phi (slot 3) beside r^2 (slot 2)
    // Look-ahead: the next V-cycle depends only on device data (the residual
    // just formed), so it is enqueued before the host waits for the norm; it
    // is skipped when the measured contraction predicts convergence.  A
    // look-ahead cycle that turns out unneeded only wrote hierarchy buffers.
    c->pending_sums = false;
    bool ahead = max_cycles > 0;
    if ((st = outer_with_sums(c, phi, nullptr, nullptr, b, bmean, ahead)) != MG_OK) return st;
    if (ahead && (st = inner_vcycle(c)) != MG_OK) return st;
    if ((st = flush_sums(c)) != MG_OK) return st;
    if ((st = wait_scalars(c)) != MG_OK) return st;
    const double nb = std::sqrt(c->hscal[1]);
    if (info) {
        info->cycles = 0;
        info->rel_res0 = info->rel_res = 0.0;
    }
    if (nb == 0.0) {
        HIPCHK(c, launch_fill<double>(N0, 0.0, phi, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->x1_ready = false;
        if (info && info->history && info->history_cap > 0) info->history[0] = 0.0;
        return MG_OK;
    }
    double rel = std::sqrt(c->hscal[2]) / nb;
    if (!std::isfinite(rel)) {
        (void)hipStreamSynchronize(c->stream);
        c->x1_ready = false;
        return fail(c, MG_ERR_NONFINITE, "initial residual is not finite (NaN/Inf in phi?)");
    }
    if (info) {
        info->rel_res0 = rel;
        if (info->history && info->history_cap > 0) info->history[0] = rel;
    }
    double* cur = phi;
    double* other = c->phi_tmp;
    int cycles = 0;
    double prev1 = INFINITY, prev2 = INFINITY;
    double rho = 0.3;  // running estimate of the per-cycle residual reduction
    mg_status result = MG_OK;
    while (rel > tol && cycles < max_cycles) {
        if (!ahead && (st = inner_vcycle(c)) != MG_OK) return st;
        ahead = cycles + 1 < max_cycles && rho * rel > tol;
        if ((st = outer_with_sums(c, cur, inner_e(c), other, b, bmean, ahead)) != MG_OK) return st;
        std::swap(cur, other);
        if (ahead && (st = inner_vcycle(c)) != MG_OK) return st;
        if ((st = flush_sums(c)) != MG_OK) return st;
        if ((st = wait_scalars(c)) != MG_OK) return st;
        prev2 = prev1;
        prev1 = rel;
        rel = std::sqrt(c->hscal[2]) / nb;
        ++cycles;
        if (prev1 > 0.0 && std::isfinite(rel)) rho = std::min(1.0, std::max(1e-3, rel / prev1));
        if (info && info->history && cycles < info->history_cap) info->history[cycles] = rel;
        if (!std::isfinite(rel)) {
            result = fail(c, MG_ERR_NONFINITE, "residual became non-finite");
            break;
        }
        // stagnation at the rounding floor: no decrease over two consecutive cycles
        if (rel >= 0.999 * prev1 && prev1 >= 0.999 * prev2) break;
    }
    if (result == MG_OK && rel > tol) {
        result = MG_ERR_NOT_CONVERGED;
        c->err = "relative residual " + std::to_string(rel) + " > tol after " + std::to_string(cycles) + " cycles";
    }
    c->x1_ready = false;
    // gauge: phi <- cur - mean(cur); the sum of cur came with the last norm
    HIPCHK(c, launch_shift(N0, cur, c->hscal[3] * invN, phi, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (info) {
        info->cycles = cycles;
        info->rel_res = rel;
    }
    return result;
}

mg_status mg_solve(mg_ctx* c, double* phi, const double* b, double tol, int max_cycles, mg_solve_info* info) {
    if (!c || !phi || !b || max_cycles < 0 || !(tol >= 0.0)) return fail(c, MG_ERR_INVALID, "invalid solve arguments");
    if (phi == b) return fail(c, MG_ERR_INVALID, "phi and b must not alias");
    return solve_impl(c, phi, b, tol, max_cycles, info);
}

mg_status mg_solve_adjoint(mg_ctx* c, double* lam, const double* phibar, double tol, int max_cycles,
                           mg_solve_info* info) {
    if (!c || !lam || !phibar || max_cycles < 0 || !(tol >= 0.0))
        return fail(c, MG_ERR_INVALID, "invalid adjoint-solve arguments");
    if (lam == phibar) return fail(c, MG_ERR_INVALID, "lam and phibar must not alias");
    // M = M^T: the adjoint system is the forward system with the cotangent as source.
    return solve_impl(c, lam, phibar, tol, max_cycles, info);
}

// A fixed number of defect-correction cycles with no host wait between them:
// every outer kernel is followed by the next inner V-cycle at once, and the
// outer sums are read once, after the last update.
mg_status mg_cycles(mg_ctx* c, double* phi, const double* b, int cycles, double* rel_res_out) {
    if (!c || !phi || !b || cycles < 0) return fail(c, MG_ERR_INVALID, "invalid cycles arguments");
    if (phi == b) return fail(c, MG_ERR_INVALID, "phi and b must not alias");
    const size_t N0 = c->lev[0].N;
    const double invN = 1.0 / (double)N0;
    mg_status st;
    if ((st = device_sum(c, b, 0.0, 1, 0)) != MG_OK) return st;
    if ((st = read_scalars(c, 1)) != MG_OK) return st;
    const double bmean = c->hscal[0] * invN;
    if (!std::isfinite(bmean)) return fail(c, MG_ERR_NONFINITE, "source contains NaN or Inf");
    c->pending_sums = false;
    double* cur = phi;
    double* other = c->phi_tmp;
    for (int k = 0; k <= cycles; ++k) {
        const bool follows = k < cycles;
        if (k == 0) st = outer_with_sums(c, phi, nullptr, nullptr, b, bmean, follows);
        else st = outer_with_sums(c, cur, inner_e(c), other, b, bmean, follows);
        if (st != MG_OK) return st;
        if (k > 0) std::swap(cur, other);
        if (follows && (st = inner_vcycle(c)) != MG_OK) return st;
    }
    if ((st = flush_sums(c)) != MG_OK) return st;
    if ((st = wait_scalars(c)) != MG_OK) return st;
    c->x1_ready = false;
    const double nb = std::sqrt(c->hscal[1]);
    const double rel = nb > 0.0 ? std::sqrt(c->hscal[2]) / nb : 0.0;
    if (nb == 0.0) HIPCHK(c, launch_fill<double>(N0, 0.0, phi, c->stream));
    else HIPCHK(c, launch_shift(N0, cur, c->hscal[3] * invN, phi, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (rel_res_out) *rel_res_out = rel;
    if (!std::isfinite(rel)) return fail(c, MG_ERR_NONFINITE, "residual is not finite");
    return MG_OK;
}

}  // extern "C"

namespace {

mg_status ensure_pcg(mg_ctx* c) {
    if (c->pcg_r) return MG_OK;
    const size_t bytes = c->lev[0].N * sizeof(double);
    mg_status st;
    if ((st = dalloc(c, (void**)&c->pcg_r, bytes)) != MG_OK) return st;
    if ((st = dalloc(c, (void**)&c->pcg_p[0], bytes)) != MG_OK) return st;
    if ((st = dalloc(c, (void**)&c->pcg_p[1], bytes)) != MG_OK) return st;
    if ((st = dalloc(c, (void**)&c->pcg_q, bytes)) != MG_OK) return st;
    if ((st = dalloc(c, (void**)&c->pcg_s, kPcgSlots * sizeof(double))) != MG_OK) return st;
    return dalloc(c, (void**)&c->pcg_partials, 2 * (size_t)pcg_blocks(c->lev[0].n) * sizeof(double));
}

// Multigrid-preconditioned CG.  TI: type of the hierarchy (preconditioner
// input r_in = level 0's right-hand side, output z = level 0's iterate);
// TC: type of the fine coefficients used for q = M p.
template <typename TI, typename TC>
mg_status pcg_impl(mg_ctx* c, double* phi, const double* b, double tol, int max_iter, mg_solve_info* info) {
    Level& L0 = c->lev[0];
    const int n = L0.n;
    const size_t N0 = L0.N;
    const double invN = 1.0 / (double)N0;
    const OpDesc<TC> op{n, L0.ih2, (const TC*)c->coeff_outer};
    TI* rin = (TI*)L0.b;
    double* r = c->pcg_r;
    double* q = c->pcg_q;
    double* S = c->pcg_s;
    double* part = c->pcg_partials;
    const int nb = pcg_blocks(n);
    mg_status st;
    c->x1_ready = false;
    if ((st = device_sum(c, b, 0.0, 1, 0)) != MG_OK) return st;
    if ((st = read_scalars(c, 1)) != MG_OK) return st;
    const double bmean = c->hscal[0] * invN;
    if (!std::isfinite(bmean)) return fail(c, MG_ERR_NONFINITE, "source contains NaN or Inf");
    if ((st = device_sum(c, b, bmean, 2, 1)) != MG_OK) return st;
    auto true_residual = [&]() -> mg_status {
        HIPCHK(c, (launch_pcg_residual<TI, TC>(op, phi, b, bmean, r, rin, part, c->stream)));
        HIPCHK(c, launch_finalize_sum(part, nb, c->dscal, 2, c->stream));
        return MG_OK;
    };
    if ((st = true_residual()) != MG_OK) return st;
    if ((st = post_scalars(c, 3)) != MG_OK) return st;
    bool ahead = max_iter > 0;  // look-ahead preconditioner application, as in the defect-correction loop
    if (ahead && (st = inner_vcycle(c)) != MG_OK) return st;
    if ((st = wait_scalars(c)) != MG_OK) return st;
    const double nbn = std::sqrt(c->hscal[1]);
    if (info) {
        info->cycles = 0;
        info->rel_res0 = info->rel_res = 0.0;
    }
    if (nbn == 0.0) {
        HIPCHK(c, launch_fill<double>(N0, 0.0, phi, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (info && info->history && info->history_cap > 0) info->history[0] = 0.0;
        return MG_OK;
    }
    double rel = std::sqrt(c->hscal[2]) / nbn;
    if (!std::isfinite(rel)) {
        (void)hipStreamSynchronize(c->stream);
        return fail(c, MG_ERR_NONFINITE, "initial residual is not finite (NaN/Inf in phi?)");
    }
    if (info) {
        info->rel_res0 = rel;
        if (info->history && info->history_cap > 0) info->history[0] = rel;
    }
    int its = 0, pc = 0;
    bool restart = true;
    double rho = 0.3, last_true = rel, true_rel = rel;
    bool true_current = true;  // true_rel belongs to the current iterate
    mg_status result = MG_OK;
    while (rel > tol && its < max_iter) {
        if (!ahead && (st = inner_vcycle(c)) != MG_OK) return st;
        const TI* z = (const TI*)inner_e(c);
        double* p_old = c->pcg_p[pc];
        double* p_new = c->pcg_p[1 - pc];
        HIPCHK(c, launch_pcg_dots<TI>(n, r, z, restart ? nullptr : q, part, c->stream));
        HIPCHK(c, launch_pcg_scalars(part, nb, S, kPcgBeta, restart, c->stream));
        HIPCHK(c, (launch_pcg_direction<TI, TC>(op, z, p_old, p_new, q, S, restart, part, c->stream)));
        HIPCHK(c, launch_pcg_scalars(part, nb, S, kPcgAlpha, false, c->stream));
        HIPCHK(c, launch_pcg_update<TI>(n, phi, p_new, r, q, rin, S, part, c->stream));
        HIPCHK(c, launch_pcg_scalars(part, nb, S, kPcgRr, false, c->stream));
        pc = 1 - pc;
        restart = false;
        true_current = false;
        HIPCHK(c, hipMemcpyAsync(c->hscal, S + kPcgRr, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipEventRecord(c->norm_ev, c->stream));
        c->scal_flag = false;
        ahead = its + 1 < max_iter && rho * rel > tol;
        if (ahead && (st = inner_vcycle(c)) != MG_OK) return st;
        if ((st = wait_scalars(c)) != MG_OK) return st;
        const double prev = rel;
        rel = std::sqrt(c->hscal[0]) / nbn;
        ++its;
        if (prev > 0.0 && std::isfinite(rel)) rho = std::min(1.0, std::max(1e-3, rel / prev));
        if (info && info->history && its < info->history_cap) info->history[its] = rel;
        if (!std::isfinite(rel)) {
            result = fail(c, MG_ERR_NONFINITE, "residual became non-finite");
            break;
        }
        if (rel <= tol) {
            // the recursive residual met tol: confirm with the true residual
            if ((st = true_residual()) != MG_OK) return st;
            if ((st = read_scalars(c, 3)) != MG_OK) return st;
            true_rel = std::sqrt(c->hscal[2]) / nbn;
            true_current = true;
            if (true_rel > tol && its < max_iter) {
                if (true_rel >= 0.999 * last_true) {  // no progress since the last restart: rounding floor
                    rel = true_rel;
                    break;
                }
                last_true = true_rel;
                rel = true_rel;
                if (info && info->history && its < info->history_cap) info->history[its] = rel;
                restart = true;  // r and r_in now hold the true residual
                ahead = false;
            }
        }
    }
    if (!true_current && result == MG_OK) {
        if ((st = true_residual()) != MG_OK) return st;
        if ((st = read_scalars(c, 3)) != MG_OK) return st;
        true_rel = std::sqrt(c->hscal[2]) / nbn;
    }
    if (result == MG_OK && true_rel > tol) {
        result = MG_ERR_NOT_CONVERGED;
        c->err = "relative residual " + std::to_string(true_rel) + " > tol after " + std::to_string(its) +
                 " iterations";
    }
    // gauge: phi <- phi - mean(phi)
    if ((st = device_sum(c, phi, 0.0, 1, 3)) != MG_OK) return st;
    if ((st = read_scalars(c, 4)) != MG_OK) return st;
    HIPCHK(c, launch_shift(N0, phi, c->hscal[3] * invN, phi, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (info) {
        info->cycles = its;
        info->rel_res = true_rel;
    }
    return result;
}

}  // namespace

extern "C" {

mg_status mg_solve_pcg(mg_ctx* c, double* phi, const double* b, double tol, int max_iter, mg_solve_info* info) {
    if (!c || !phi || !b || max_iter < 0 || !(tol >= 0.0)) return fail(c, MG_ERR_INVALID, "invalid solve arguments");
    if (phi == b) return fail(c, MG_ERR_INVALID, "phi and b must not alias");
    mg_status st;
    if ((st = ensure_pcg(c)) != MG_OK) return st;
    const bool cd = !c->var || c->coeff_outer_double;
    if (c->inner_double) return cd ? pcg_impl<double, double>(c, phi, b, tol, max_iter, info)
                                   : pcg_impl<double, float>(c, phi, b, tol, max_iter, info);
    return cd ? pcg_impl<float, double>(c, phi, b, tol, max_iter, info)
              : pcg_impl<float, float>(c, phi, b, tol, max_iter, info);
}

mg_status mg_create_psi(const mg_params* p, const double* psi, void* stream, mg_ctx** out) {
    if (!out) return MG_ERR_INVALID;
    *out = nullptr;
    if (!psi || mg_validate_params(p) != MG_OK) return MG_ERR_INVALID;
    mg_ctx* c = new (std::nothrow) mg_ctx();
    if (!c) return MG_ERR_NOMEM;
    c->p = *p;
    c->stream = (hipStream_t)stream;
    mg_status st = create_impl(c, nullptr, MG_DTYPE_F64, psi);
    if (st != MG_OK) {
        std::fprintf(stderr, "mg_create_psi: %s\n", c->err.c_str());
        mg_destroy(c);
        return st;
    }
    *out = c;
    return MG_OK;
}

mg_status mg_predict(int n, int kind, const double* phi1, const double* phi2, const double* phi3, double growth,
                     double* out, void* stream) {
    if (!is_pow2(n) || n < 4 || n > 2048 || !phi1 || !out) return MG_ERR_INVALID;
    double c1, c2 = 0.0, c3 = 0.0;
    switch (kind) {
        case MG_PREDICT_RECYCLE: c1 = 1.0; break;
        case MG_PREDICT_GROWTH:
            if (!std::isfinite(growth)) return MG_ERR_INVALID;
            c1 = growth;
            break;
        case MG_PREDICT_LINEAR:
            if (!phi2) return MG_ERR_INVALID;
            c1 = 2.0; c2 = -1.0;
            break;
        case MG_PREDICT_QUADRATIC:
            if (!phi2 || !phi3) return MG_ERR_INVALID;
            c1 = 3.0; c2 = -3.0; c3 = 1.0;
            break;
        default: return MG_ERR_INVALID;
    }
    const size_t N = (size_t)n * n * n;
    return launch_combine3(N, c1, phi1, c2, phi2, c3, phi3, out, (hipStream_t)stream) == hipSuccess ? MG_OK
                                                                                                   : MG_ERR_HIP;
}

mg_status mg_accel(int n, double h, const double* phi, const double* psi, double scale, void* a_out, int dtype,
                   void* stream) {
    if (!is_pow2(n) || n < 4 || n > 2048 || !(h > 0) || !phi || !a_out || !std::isfinite(scale))
        return MG_ERR_INVALID;
    hipError_t e;
    if (dtype == MG_DTYPE_F64) e = launch_accel<double>(n, h, phi, psi, scale, (double*)a_out, (hipStream_t)stream);
    else if (dtype == MG_DTYPE_F32) e = launch_accel<float>(n, h, phi, psi, scale, (float*)a_out, (hipStream_t)stream);
    else return MG_ERR_INVALID;
    return e == hipSuccess ? MG_OK : MG_ERR_HIP;
}

mg_status mg_vcycle(mg_ctx* c, double* phi, const double* b, double* rel_res_out) {
    if (!c || !phi || !b) return fail(c, MG_ERR_INVALID, "invalid vcycle arguments");
    if (phi == b) return fail(c, MG_ERR_INVALID, "phi and b must not alias");
    const size_t N0 = c->lev[0].N;
    const double invN = 1.0 / (double)N0;
    mg_status st;
    if ((st = device_sum(c, b, 0.0, 1, 0)) != MG_OK) return st;
    if ((st = read_scalars(c, 1)) != MG_OK) return st;
    const double bmean = c->hscal[0] * invN;
    if ((st = outer_residual(c, phi, nullptr, nullptr, b, bmean, true)) != MG_OK) return st;
    if ((st = inner_vcycle(c)) != MG_OK) return st;
    const void* e = inner_e(c);
    if (c->inner_double) HIPCHK(c, launch_add<double>(N0, phi, (const double*)e, phi, c->stream));
    else HIPCHK(c, launch_add<float>(N0, phi, (const float*)e, phi, c->stream));
    if (rel_res_out) {
        if ((st = outer_residual(c, phi, nullptr, nullptr, b, bmean)) != MG_OK) return st;
        HIPCHK(c, launch_finalize_sums(c->partials, c->nparts_outer, 3, c->dscal, 1, c->stream));
        if ((st = read_scalars(c, 3)) != MG_OK) return st;
        const double nb = std::sqrt(c->hscal[1]);
        *rel_res_out = nb > 0 ? std::sqrt(c->hscal[2]) / nb : 0.0;
    }
    return MG_OK;
}

mg_status mg_coeff_grad(mg_ctx* c, const double* lam, const double* phi, void* cbar, int cbar_dtype) {
    if (!c || !lam || !phi || !cbar) return fail(c, MG_ERR_INVALID, "invalid coeff_grad arguments");
    if (!c->var) return fail(c, MG_ERR_INVALID, "coefficient gradient needs a variable-coefficient context");
    const Level& L = c->lev[0];
    if (cbar_dtype == MG_DTYPE_F64)
        HIPCHK(c, launch_coeff_grad<double>(L.n, L.ih2, lam, phi, (double*)cbar, c->stream));
    else if (cbar_dtype == MG_DTYPE_F32)
        HIPCHK(c, launch_coeff_grad<float>(L.n, L.ih2, lam, phi, (float*)cbar, c->stream));
    else
        return fail(c, MG_ERR_INVALID, "cbar_dtype must be MG_DTYPE_F32 or MG_DTYPE_F64");
    return MG_OK;
}

mg_status mg_geometry(int n, double h, const double* psi, void* C_out, int dtype, double* sqrtg_out, void* stream) {
    if (!is_pow2(n) || n < 4 || n > 2048 || !(h > 0) || !psi || !C_out) return MG_ERR_INVALID;
    const double ih2 = 1.0 / (h * h);
    hipError_t e;
    if (dtype == MG_DTYPE_F64) e = launch_geometry<double>(n, ih2, psi, (double*)C_out, sqrtg_out, (hipStream_t)stream);
    else if (dtype == MG_DTYPE_F32) e = launch_geometry<float>(n, ih2, psi, (float*)C_out, sqrtg_out, (hipStream_t)stream);
    else return MG_ERR_INVALID;
    return e == hipSuccess ? MG_OK : MG_ERR_HIP;
}

mg_status mg_geometry_bwd(int n, double h, const double* psi, const double* Cbar, const double* sqrtgbar,
                          double* psibar, void* stream) {
    if (!is_pow2(n) || n < 4 || n > 2048 || !(h > 0) || !psi || !Cbar || !psibar) return MG_ERR_INVALID;
    const double ih2 = 1.0 / (h * h);
    const size_t N = (size_t)n * n * n;
    double* Jbar = nullptr;
    if (hipMalloc((void**)&Jbar, 6 * N * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return MG_ERR_NOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_geometry_bwd_cell(n, ih2, psi, Cbar, sqrtgbar, Jbar, s);
    if (e == hipSuccess) e = launch_hessian_adjoint(n, ih2, Jbar, psibar, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(Jbar);
    return e == hipSuccess ? MG_OK : MG_ERR_HIP;
}

// ---- single steps (double arithmetic on caller fields) ---------------------------------------
static mg_status level_check(mg_ctx* c, int level, bool need_coarser) {
    if (!c) return MG_ERR_INVALID;
    if (level < 0 || level >= (int)c->lev.size()) return fail(c, MG_ERR_INVALID, "level out of range");
    if (need_coarser && level + 1 >= (int)c->lev.size()) return fail(c, MG_ERR_INVALID, "no coarser level");
    return MG_OK;
}

static mg_status ensure_scratch(mg_ctx* c, size_t elems) {
    if (c->scratch_elems >= elems) return MG_OK;
    dfree(c->scratch);
    c->scratch = nullptr;
    c->scratch_elems = 0;
    mg_status st = dalloc(c, (void**)&c->scratch, elems * sizeof(double));
    if (st == MG_OK) c->scratch_elems = elems;
    return st;
}

mg_status mg_apply(mg_ctx* c, int level, const double* u, double* out) {
    mg_status st = level_check(c, level, false);
    if (st != MG_OK) return st;
    if (!u || !out || u == out) return fail(c, MG_ERR_INVALID, "invalid apply arguments");
    HIPCHK(c, with_op(c, level, [&](auto op) { return launch_apply<double>(op, u, out, c->stream); }));
    return MG_OK;
}

mg_status mg_smooth(mg_ctx* c, int level, double* x, const double* b) {
    mg_status st = level_check(c, level, false);
    if (st != MG_OK) return st;
    if (!x || !b || x == b) return fail(c, MG_ERR_INVALID, "invalid smooth arguments");
    const Level& L = c->lev[level];
    if ((st = ensure_scratch(c, L.N)) != MG_OK) return st;
    double* bufs[2] = {x, c->scratch};
    const bool cheb = c->p.smoother == MG_CHEBYSHEV;
    int cur = 0, prev = -1;
    for (size_t k = 0; k < L.a.size(); ++k) {
        const bool use_prev = cheb && prev >= 0;
        const double* xp = use_prev ? bufs[prev] : nullptr;
        const int out = use_prev ? prev : 1 - cur;
        HIPCHK(c, with_op(c, level, [&](auto op) {
                   return launch_smooth_step<double>(op, bufs[cur], xp, b, bufs[out], L.a[k], L.c[k], c->stream);
               }));
        prev = cur;
        cur = out;
    }
    if (cur != 0) HIPCHK(c, hipMemcpyAsync(x, bufs[cur], L.N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return MG_OK;
}

mg_status mg_residual_restrict(mg_ctx* c, int level, const double* x, const double* b, double* coarse) {
    mg_status st = level_check(c, level, true);
    if (st != MG_OK) return st;
    if (!b || !coarse) return fail(c, MG_ERR_INVALID, "invalid residual_restrict arguments");
    if ((st = ensure_scratch(c, c->lev[level].N)) != MG_OK) return st;
    HIPCHK(c, with_op(c, level, [&](auto op) {
               return launch_residual_restrict<double>(op, x, b, coarse, c->scratch, c->stream);
           }));
    return MG_OK;
}

mg_status mg_prolong_add(mg_ctx* c, int level, const double* e, double* x) {
    mg_status st = level_check(c, level, true);
    if (st != MG_OK) return st;
    if (!e || !x) return fail(c, MG_ERR_INVALID, "invalid prolong arguments");
    HIPCHK(c, launch_prolong_add<double>(c->lev[level].n, e, x, c->stream));
    return MG_OK;
}

mg_status mg_coarse_solve(mg_ctx* c, const double* r, double* e) {
    if (!c || !r || !e || r == e) return fail(c, MG_ERR_INVALID, "invalid coarse_solve arguments");
    const Level& L = c->lev.back();
    if (!c->var) HIPCHK(c, launch_coarse_flat<double>(L.n, c->Q, c->lam1, r, e, c->stream));
    else HIPCHK(c, launch_coarse_dense<double>((int)L.N, c->G, r, e, c->stream));
    return MG_OK;
}

}  // extern "C"

namespace {

// One V-cycle step of level l in the inner type T on the context's buffers;
// the caller's double fields are rounded to T on entry and out is widened.
template <typename T>
mg_status inner_step_impl(mg_ctx* c, int step, int l, const double* x, const double* e, const double* b,
                          double* out) {
    Level& L = c->lev[l];
    Level* Lc = l + 1 < (int)c->lev.size() ? &c->lev[l + 1] : nullptr;
    hipStream_t s = c->stream;
    c->x1_ready = false;
    c->pending_sums = false;
    auto in = [&](size_t count, const double* src, void* dst) -> hipError_t {
        return launch_convert<T, double>(count, src, (T*)dst, s);
    };
    const T* res = nullptr;
    size_t count = L.N;
    mg_status st = MG_OK;
    switch (step) {
        case MG_STEP_SMOOTH:
            HIPCHK(c, in(L.N, x, L.x[0]));
            HIPCHK(c, in(L.N, b, L.b));
            L.cur = 0;
            st = smooth_level<T>(c, l, false);
            res = (const T*)L.x[L.cur];
            break;
        case MG_STEP_SMOOTH_ZERO:
            HIPCHK(c, in(L.N, b, L.b));
            st = smooth_level<T>(c, l, true);
            res = (const T*)L.x[L.cur];
            break;
        case MG_STEP_PROLONG_SMOOTH:
            HIPCHK(c, in(L.N, x, L.x[0]));
            HIPCHK(c, in(Lc->N, e, Lc->x[0]));
            HIPCHK(c, in(L.N, b, L.b));
            L.cur = 0;
            Lc->cur = 0;
            st = post_level<T>(c, l);
            res = (const T*)L.x[L.cur];
            break;
        case MG_STEP_RESIDUAL_RESTRICT:
            HIPCHK(c, in(L.N, x, L.x[0]));
            HIPCHK(c, in(L.N, b, L.b));
            L.cur = 0;
            st = residual_restrict_level<T>(c, l);
            res = (const T*)Lc->b;
            count = Lc->N;
            break;
        case MG_STEP_PROLONG:
            HIPCHK(c, in(L.N, x, L.x[0]));
            HIPCHK(c, in(Lc->N, e, Lc->x[0]));
            HIPCHK(c, launch_prolong_add<T>(L.n, (const T*)Lc->x[0], (T*)L.x[0], s));
            L.cur = 0;
            res = (const T*)L.x[0];
            break;
        case MG_STEP_VCYCLE:
            HIPCHK(c, in(L.N, b, L.b));
            st = vcycle_from_zero<T>(c, l);
            res = (const T*)L.x[L.cur];
            break;
        default:
            return fail(c, MG_ERR_INVALID, "unknown step");
    }
    if (st != MG_OK) return st;
    HIPCHK(c, (launch_convert<double, T>(count, res, out, s)));
    return MG_OK;
}

}  // namespace

extern "C" {

mg_status mg_inner_step(mg_ctx* c, int step, int level, const double* x, const double* e, const double* b,
                        double* out) {
    if (!c) return MG_ERR_INVALID;
    if (step < MG_STEP_SMOOTH || step > MG_STEP_VCYCLE) return fail(c, MG_ERR_INVALID, "unknown step");
    const bool coarser = step == MG_STEP_PROLONG_SMOOTH || step == MG_STEP_RESIDUAL_RESTRICT || step == MG_STEP_PROLONG;
    mg_status st = level_check(c, level, coarser);
    if (st != MG_OK) return st;
    const bool need_x = step == MG_STEP_SMOOTH || step == MG_STEP_PROLONG_SMOOTH ||
                        step == MG_STEP_RESIDUAL_RESTRICT || step == MG_STEP_PROLONG;
    const bool need_e = step == MG_STEP_PROLONG_SMOOTH || step == MG_STEP_PROLONG;
    const bool need_b = step != MG_STEP_PROLONG;
    if (!out || (need_x && !x) || (need_e && !e) || (need_b && !b))
        return fail(c, MG_ERR_INVALID, "missing field for this step");
    return c->inner_double ? inner_step_impl<double>(c, step, level, x, e, b, out)
                           : inner_step_impl<float>(c, step, level, x, e, b, out);
}

mg_status mg_level_lmax(const mg_ctx* c, double* out) {
    if (!c || !out) return MG_ERR_INVALID;
    for (size_t l = 0; l < c->lev.size(); ++l) out[l] = c->lev[l].lmax;
    return MG_OK;
}

mg_status mg_enable_kernel_timing(mg_ctx* c, int enable) {
    if (!c) return MG_ERR_INVALID;
    const int all = MG_TIME_STEP | MG_TIME_PAIR | MG_TIME_TRIPLE | MG_TIME_OUTER | MG_TIME_TRANSFER;
    if (enable < 0 || enable > all) return fail(c, MG_ERR_INVALID, "timing mask out of range");
    c->timing = enable;
    c->events_used = 0;
    c->timed_launches = 0;
    c->timed_ms = 0.0;
    c->timed_bytes = 0.0;
    return MG_OK;
}

mg_status mg_kernel_timing(mg_ctx* c, int* launches, double* total_ms, double* alg_bytes) {
    if (!c || !launches || !total_ms || !alg_bytes) return MG_ERR_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < c->events_used; ++i) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->events[i].start, c->events[i].stop));
        c->timed_ms += ms;
    }
    c->events_used = 0;
    *launches = c->timed_launches;
    *total_ms = c->timed_ms;
    *alg_bytes = c->timed_bytes;
    c->timed_launches = 0;
    c->timed_ms = 0.0;
    c->timed_bytes = 0.0;
    return MG_OK;
}

}  // extern "C"
