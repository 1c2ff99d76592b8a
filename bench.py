#!/usr/bin/env python3
"""Benchmark of the multigrid hot path on one MI355X.

Workload (one "step"): the warm-start defect-correction sequence on a 256^3
periodic grid with the seven-point Laplacian -- 8 sequential Gaussian-random-
field sources rho_t = (1 + 0.05 t) delta + 0.02 t eta_t (P(k) ~ k^-1), each
solved to relative residual 1e-10 starting from the previous step's
potential (t = 0 from zero), 7 levels (coarsest 4^3), Chebyshev degree 3, in
mixed precision (float V-cycles, double residual/update/coarsest solve).
All inputs are resident in HBM before timing starts.

The JSON line reports V-cycle throughput of the mixed path (value), the same
sequence in plain float64 (time-to-tolerance ratio), the roofline of the
dominant kernel of the step (the fine-level kernel kind with the largest
share of the step's time; in-dispatch HIP events around each launch,
algorithmic bytes counted by the library) with every other fine-level kernel
beside it, the 512^3 V-cycle (20 event-timed warm cycles, median of 5, whole
cycle against the HBM roofline, and every fine kernel's rate), a size sweep
32^3 .. 1024^3 (cold solves to the tolerance in mixed, float64 and pure
float32, with the whole-cycle fraction of the HBM peak), the 256^3
moving-mesh solve with its forward/backward timing and the ablation of its
smoother and coarse operators, the initial-guess predictors and
multigrid-preconditioned CG on the warm-start sequence, the force readout
kernel, and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "V-cycle Mpts/s + HBM GB/s; time to rel. residual 1e-10, mixed vs FP64"
HBM_PEAK_GBPS = 8000.0

# Measured HBM bytes per launch of the fine-level kernels, per workload
# (n, degree; mixed precision) and kernel kind: rocprofv3 FETCH_SIZE and
# WRITE_SIZE per dispatch (profiles/hbm_bytes_*.md) scaled by the copy-kernel
# factors 2.0 (fetch) and 1.0 (write), averaged over the launches of the kind.
# Reported only while the source of the row kernels and their launch shapes
# is the one the counters were taken on.  Keys are the first name of each
# kind's label (kernel_name).
TRAFFIC = {
    "device_code_sha256": "d54b7c1db8381bea087ed9da4386c84b2e3358a5ea13b709a8386296b1ca3cd6",
    "bytes_per_launch": {
        # the benchmark step: outer (with the first-cycle variant), pass from
        # zero (b -> x3), prolongation + three steps, residual + restriction
        (256, 3): {"k_outer_lds": 536855684, "k_smooth2_lds": 151742958, "k_smooth3p_lds": 238153913,
                   "k_rr_row": 159429926},
        # the 512^3 leg: step from b, the three pairs, outer, residual + restriction (k_rr_lds)
        (512, 4): {"k_smooth_row": 1137164769, "k_smooth2_lds": 2278180068, "k_outer_lds": 4445624636,
                   "k_rr_row": 1196833543},
    },
}


def measured_traffic(n, degree, kernel):
    import hashlib
    csrc = os.path.join(ROOT, "paper_2607_10983_amd", "csrc")
    dev = "".join(open(os.path.join(csrc, f)).read() for f in ("flat_row.hip", "fma.h", "row.h"))
    if hashlib.sha256(dev.encode()).hexdigest() != TRAFFIC["device_code_sha256"]:
        return None
    v = TRAFFIC["bytes_per_launch"].get((n, degree), {}).get(kernel)
    return round(v) if v is not None else None


def pass_bytes(v, from_zero, pairs, triple, s, rowk=False):
    """Algorithmic bytes per point of one smoothing pass of degree v, following
    the library's schedule: a pass from zero of degree 4 is one kernel for
    steps 0 and 1 (b -> x2) and a pair that forms x_prev = x1 from b
    (x2, b -> x4); other passes from zero start with one kernel for their
    first three steps (b -> x3, and x2 when a fourth step needs it as x_prev);
    on row-kernel levels without two-step kernels (rowk) a pass from zero of
    at least three steps starts with steps 0 and 1 from b (b -> x2) and a
    step that forms x_prev from b (x2, b -> x3); a pass of three steps from a
    nonzero iterate is one three-step kernel (x, b -> x3); otherwise steps
    pair up from the end of the pass where the two-step kernel runs (a pair
    that is not the last writes its first step)."""
    if not from_zero and triple and v == 3:
        return 3 * s
    if from_zero and pairs and v == 4:
        return (2 + 3) * s
    tot, prev, k = 0.0, False, 0
    if from_zero and not pairs and rowk and v >= 3:
        tot, prev, k = (2 + 3) * s, True, 3
    if from_zero and pairs and v >= 3:
        tot += (2 + (v > 3)) * s
        prev, k = v > 3, 3
    while k < v:
        rem = v - k
        need_y1 = rem > 2
        if pairs and rem >= 2 and rem % 2 == 0 and not (k == 0 and from_zero) and not (need_y1 and prev):
            tot += (3 + prev + need_y1) * s
            prev, k = need_y1, k + 2
        elif k == 0 and from_zero:
            tot += 2 * s
            prev, k = False, k + 1
        else:
            tot += (4 if prev else 3) * s
            prev, k = True, k + 1
    return tot


def model_bytes_per_cycle(n, levels, degree, precision):
    """Algorithmic bytes of one outer iteration (inner V-cycle + outer residual/update),
    every field element each kernel reads or writes counted once, following the
    library's schedule: multi-step kernels on levels 64 <= n_l (two-step rows up
    to 2 KB, three-step rows up to 1 KB; from 128^3 the three-step pass, and
    on rows over 1 KB the first pair of an even-degree pass, forms x + P e
    itself, so the prolongation writes nothing), the 32^3 and 64^3
    levels of a float hierarchy as two fused visits each, the outer kernel
    writing the first step from zero only where the fine level has no
    pass-from-zero kernel (rows of more than 1024 points or degree below 3)."""
    s = 8 if precision == "fp64" else 4
    tot = 0.0
    tail_start = next((l for l in range(levels) if n >> l <= 16), levels)
    for l in range(levels - 1):
        nl = n >> l
        pairs = 64 <= nl <= 1024 and nl * s <= 2048
        triple = 64 <= nl and nl * s <= 1024
        if precision != "fp64" and nl in (32, 64) and degree <= 3 and l != tail_start:
            tot += nl ** 3 * ((2 * s + s / 8) + (3 * s + s / 8))  # fused pre and post visits
            continue
        rowk = 64 <= nl <= 1024
        x1_outer = l == 0 and not (rowk and degree >= 3)
        pre = pass_bytes(degree, True, pairs, triple, s, rowk) - (2 * s if x1_outer else 0)  # step 0 by the outer
        post = pass_bytes(degree, False, pairs, triple, s)
        # the prolongation runs inside the post-smoothing pass's first kernel:
        # the three-step pass from 128^3 (degree 3), the first pair on split
        # rows (rows of 1-2 KB, an even degree), the first two single steps on
        # rows over 2 KB (x, e, b -> x1; x1, x, e, b -> x2: e read twice)
        step_pro = rowk and nl * s > 2048 and degree >= 2
        fused_prolong = ((triple and nl >= 128 and degree == 3) or (pairs and nl * s > 1024 and degree % 2 == 0)
                         or step_pro)
        if step_pro:
            post = (3 + 4 + 4 * (degree - 2)) * s + s / 8
        transfers = 2 * s + s / 8 + (s / 8 if fused_prolong else 2 * s + s / 8)
        tot += nl ** 3 * (pre + post + transfers)
    # outer: read phi, e, b; write phi, r (and the first smoothing step where no pass-from-zero kernel runs)
    fine_rowk = 64 <= n <= 1024
    tot += n ** 3 * (8 + s + 8 + 8 + s + (0 if fine_rowk and degree >= 3 else s))
    return tot


def reference_bytes_per_cycle(n, degree, precision):
    """Bytes of one outer iteration in the reference decomposition into one
    streaming pass per step (each field element of a step read or written
    once): per level visit from zero 9.25 s + 8 s (v - 1) (first step from
    zero 2 s, later steps 4 s, residual + full weighting and prolongation
    2 s + s / 8 each, first post-smoothing step 3 s), the hierarchy x 8/7,
    plus the outer update (32 B mixed) or the FP64 convergence pass (24 B)."""
    s = 8 if precision == "fp64" else 4
    inner = (9.25 + 8 * (degree - 1)) * s * 8.0 / 7.0
    return n ** 3 * (inner + (24 if precision == "fp64" else 32))


def run_sequence(mg, sources, phi, tol, max_cycles=60):
    phi.zero_()
    cycles = []
    for b in sources:
        _, info = mg.solve(b, phi0=phi, out=phi, tol=tol, max_cycles=max_cycles, history=False,
                           raise_on_error=False)
        if info.status not in (0,):
            raise RuntimeError(f"solve failed with status {info.status} (rel_res {info.rel_res:.3e})")
        cycles.append(info.cycles)
    return cycles


MG_TIME_STEP, MG_TIME_PAIR, MG_TIME_TRIPLE, MG_TIME_OUTER, MG_TIME_TRANSFER = 1, 2, 4, 8, 16
KINDS = (MG_TIME_STEP, MG_TIME_PAIR, MG_TIME_TRIPLE, MG_TIME_OUTER, MG_TIME_TRANSFER)


def kernel_name(kind, n, precision, var=False):
    t = "double" if precision == "fp64" else "float"
    if var:
        return {MG_TIME_STEP: f"k_var_smooth_row / k_var_smooth_lds (fine-level 19-point Chebyshev step, {t})",
                MG_TIME_PAIR: f"k_var_smooth2_lds (fine-level 19-point two-step pass, {t})",
                MG_TIME_OUTER: "k_var_outer_row (19-point outer defect correction: phi += e, FP64 residual, norms)",
                MG_TIME_TRANSFER: f"k_var_resid_row / k_var_resid_lds / k_prolong_row (fine-level 19-point "
                                  f"residual, prolongation, {t})",
                }.get(kind, f"kind {kind}")
    return {MG_TIME_STEP: f"k_smooth_row / k_smooth_lds (fine-level single Chebyshev step, {t})",
            MG_TIME_PAIR: f"k_smooth2_lds (fine-level two-step pass and pass from zero, {t})",
            MG_TIME_TRIPLE: (f"k_smooth3p_lds (fine-level prolongation + three-step pass, {t})" if n >= 128
                             else f"k_smooth3_lds (fine-level three-step pass, {t})"),
            MG_TIME_OUTER: "k_outer_lds (outer defect correction: phi += e, FP64 residual r, norms, r cast "
                           "to the inner precision)",
            MG_TIME_TRANSFER: f"k_rr_row / k_rr_lds / k_prolong_row (fine-level residual + restriction, "
                              f"prolongation, {t})",
            }[kind]


def breakdown(mg, run):
    """{kind: (launches, ms, alg_bytes)} of the fine-level kernels, one call of
    run() per kind with that kind's in-dispatch events enabled."""
    out = {}
    for kind in KINDS:
        mg.enable_kernel_timing(kind)
        mg.kernel_timing()
        run()
        out[kind] = mg.kernel_timing()
    mg.enable_kernel_timing(0)
    return out


def kernel_entry(kind, kt, n, precision, step_ms, deg=None, var=False, per="step"):
    gbps, us = rate(kt)
    k, ms, by = kt
    return {"kernel": kernel_name(kind, n, precision, var), "achieved": gbps,
            "frac": round(gbps / HBM_PEAK_GBPS, 4) if gbps else None, "avg_launch_us": us,
            f"launches_per_{per}": k, "alg_bytes_per_launch": by / k if k else None,
            f"share_of_{per}": round(ms / step_ms, 4) if step_ms else None,
            "traffic": measured_traffic(n, deg, kernel_name(kind, n, precision, var).split()[0])
            if deg is not None and not var and precision != "fp64" else None}


def solve_timed(mg, torch, b, tol, max_cycles=60, kernels=False):
    """Cold solve from zero, after one untimed warm-up solve: (info, ms, phi,
    per-kernel breakdown of one more solve or None)."""
    phi = torch.zeros_like(b)
    mg.solve(b, phi0=phi, out=phi, tol=tol, max_cycles=max_cycles, history=False, raise_on_error=False)
    phi.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = mg.solve(b, phi0=phi, out=phi, tol=tol, max_cycles=max_cycles, history=False, raise_on_error=False)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    kt = None
    if kernels:
        tmp = torch.zeros_like(b)

        def run():
            tmp.zero_()
            mg.solve(b, phi0=tmp, out=tmp, tol=tol, max_cycles=max_cycles, history=False, raise_on_error=False)
        kt = breakdown(mg, run)
        del tmp
    return info, 1e3 * t, phi, kt


def rate(kt):
    """(GB/s, avg launch us) of a (launches, ms, bytes) triple, or Nones."""
    k, ms, by = kt
    if not k or ms <= 0:
        return None, None
    return round(by / (ms * 1e-3) / 1e9, 1), round(1e3 * ms / k, 2)


def sweep_point(mgpu, torch, flat_source, n, tol):
    """Cold solve of the k_c = (n/4) 2 pi source to `tol` in mixed and float64
    precision, and in pure float32 to its rounding plateau (stagnation).
    32^3: 4 levels, degree 3; n >= 64: degree 4 with a 16^3 coarsest level.
    Whole-cycle rate: the model's algorithmic bytes of the cycles run over the
    time to tolerance (host round trips and the setup of the solve included)."""
    levels, deg = (4, 3) if n == 32 else (int(np.log2(n)) - 3, 4)
    b = torch.from_numpy(flat_source(n, 0)).to("cuda")
    out = {"levels": levels, "degree": deg}
    phis = {}
    for prec in ("mixed", "fp64", "fp32"):
        mg = mgpu.Multigrid(n, levels=levels, degree=deg, precision=prec)
        info, ms, phi, kt = solve_timed(mg, torch, b, tol if prec != "fp32" else 0.0,
                                        max_cycles=60 if prec != "fp32" else 30, kernels=n >= 256 and prec != "fp32")
        mb = model_bytes_per_cycle(n, levels, deg, prec)
        gbps = info.cycles * mb / (ms * 1e-3) / 1e9
        out[prec] = {
            "cycles": info.cycles,
            "time_to_tol_ms": round(ms, 3),
            "ms_per_cycle": round(ms / max(info.cycles, 1), 4),
            "vcycle_mpts_per_s": round(info.cycles * n ** 3 / (ms * 1e-3) / 1e6, 1),
            "rel_res": info.rel_res,
            "model_bytes_per_cycle_per_pt": round(mb / n ** 3, 2),
            "cycle_GBps": round(gbps, 1),
            "cycle_frac": round(gbps / HBM_PEAK_GBPS, 4),
            # bytes of the one-pass-per-step decomposition over the measured
            # time: above 1 where the fused schedule runs faster than that
            # decomposition could at the full HBM bandwidth
            "reference_equiv_frac": round(info.cycles * reference_bytes_per_cycle(n, deg, prec) / (ms * 1e-3) / 1e9
                                          / HBM_PEAK_GBPS, 4),
        }
        if kt is not None:
            out[prec]["fine_kernels"] = [kernel_entry(k, kt[k], n, prec, ms, per="solve")
                                         for k in KINDS if kt[k][0]]
        if prec == "fp32":
            out[prec]["note"] = "tolerance disabled: runs to its float32 rounding plateau (stagnation guard)"
            out[prec]["rel_diff_vs_mixed"] = float(torch.linalg.norm(phi - phis["mixed"]) /
                                                   torch.linalg.norm(phis["mixed"]))
        else:
            phis[prec] = phi
        del mg
        torch.cuda.empty_cache()
    out["time_to_tol_ratio_fp64_over_mixed"] = round(out["fp64"]["time_to_tol_ms"] / out["mixed"]["time_to_tol_ms"], 3)
    return out


def b512_leg(mgpu, torch, flat_source, n=512, levels=6, deg=4, cycles=20, reps=5):
    """The 512^3 V-cycle (one GPU's share of 1024^3 on eight GPUs): from a
    warm iterate (the source solved to 1e-10), 3 warm-up cycles, then
    `cycles` defect-correction cycles (mg_cycles: no host wait between
    cycles) timed with HIP events on the solver's stream, median of `reps`.
    Whole-cycle rate = the model's algorithmic bytes of the call over its
    time; then each fine-level kernel kind's in-dispatch rate over one more
    call."""
    b = torch.from_numpy(flat_source(n, 0)).to("cuda")
    out = {"n": n, "levels": levels, "degree": deg, "cycles_timed": cycles, "repeats": reps}
    for prec in ("mixed", "fp64"):
        mg = mgpu.Multigrid(n, levels=levels, degree=deg, precision=prec)
        phi = torch.zeros_like(b)
        mg.solve(b, phi0=phi, out=phi, tol=1e-10, max_cycles=40, history=False, raise_on_error=False)
        mg.cycles(phi, b, 3)
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            rel = mg.cycles(phi, b, cycles)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        s = 8 if prec == "fp64" else 4
        N = n ** 3
        # `cycles` model cycles, plus the call's first outer pass (no e), the
        # mean of b and the final gauge shift
        by = cycles * model_bytes_per_cycle(n, levels, deg, prec) + N * ((8 + 8 + s) + 8 + 16)
        gbps = by / (ms * 1e-3) / 1e9
        kt = breakdown(mg, lambda: mg.cycles(phi, b, cycles))
        out[prec] = {
            "ms_per_call": round(ms, 3), "ms_per_cycle": round(ms / cycles, 4),
            "times_ms": [round(t, 3) for t in times],
            "vcycle_mpts_per_s": round(cycles * N / (ms * 1e-3) / 1e6, 1),
            "model_bytes_per_cycle_per_pt": round(model_bytes_per_cycle(n, levels, deg, prec) / N, 2),
            "cycle_GBps": round(gbps, 1), "cycle_frac": round(gbps / HBM_PEAK_GBPS, 4),
            "reference_bytes_per_cycle_per_pt": round(reference_bytes_per_cycle(n, deg, prec) / N, 2),
            "reference_equiv_frac": round(cycles * reference_bytes_per_cycle(n, deg, prec) / (ms * 1e-3) / 1e9
                                          / HBM_PEAK_GBPS, 4),
            # one cycle of the one-pass-per-step decomposition at 60% of peak
            "reference_ms_per_cycle_at_60pct": round(reference_bytes_per_cycle(n, deg, prec)
                                                     / (0.6 * HBM_PEAK_GBPS * 1e9) * 1e3, 3),
            "rel_res_after": rel,
            "fine_kernels": [kernel_entry(k, kt[k], n, prec, ms, deg=deg, per="call") for k in KINDS if kt[k][0]],
        }
        del mg, phi
        torch.cuda.empty_cache()
    out["time_ratio_fp64_over_mixed"] = round(out["fp64"]["ms_per_call"] / out["mixed"]["ms_per_call"], 3)
    return out


def moving_mesh_leg(mgpu, torch, n, tol):
    """256^3 moving-mesh Poisson (float32 C, 19-point operator) to `tol`, mixed
    vs float64; then forward and forward+backward of L = sum(w phi) through the
    geometry, the source and the solve (implicit adjoint)."""
    from workloads import loss_weight, moving_mesh_field, psi_unit

    scale = json.load(open(os.path.join(ROOT, "tests", "golden", "psi_scale.json")))["scale"][str(n)]
    psi = torch.from_numpy(scale * psi_unit(n)).to("cuda")
    g = torch.from_numpy(moving_mesh_field(n, 0)).to("cuda")
    w = torch.from_numpy(loss_weight(n, 2)).to("cuda")
    C32, sg = mgpu.geometry(psi, dtype=torch.float32)
    b = sg * (g - (g * sg).sum() / sg.sum())
    out = {"n": n, "levels": int(np.log2(n)) - 1, "degree": 3, "psi_scale": scale,
           "det_J": [round(float(sg.min()), 4), round(float(sg.max()), 4)]}
    for prec in ("mixed", "fp64"):
        mg = mgpu.Multigrid(n, coeff=C32, precision=prec)
        info, ms, phi, kt = solve_timed(mg, torch, b, tol, max_cycles=100, kernels=True)
        out[prec] = {"cycles": info.cycles, "time_to_tol_ms": round(ms, 3), "rel_res": info.rel_res,
                     "fine_kernels": [kernel_entry(k, kt[k], n, prec, ms, var=True, per="solve")
                                      for k in KINDS if kt[k][0]]}
        del mg, phi
    out["time_to_tol_ratio_fp64_over_mixed"] = round(out["fp64"]["time_to_tol_ms"] / out["mixed"]["time_to_tol_ms"], 3)

    def fwd_bwd(prec, backward):
        p = psi.clone().requires_grad_(backward)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        C, s = mgpu.geometry_fn(p)
        bb = s * (g - (g * s).sum() / s.sum())
        ph = mgpu.solve(bb, C, tol=tol, max_cycles=100, precision=prec)
        L = (w * ph).sum()
        if backward:
            L.backward()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0)

    grads = {}
    for prec in ("mixed", "fp64"):
        fwd_bwd(prec, True)
        f = min(fwd_bwd(prec, False) for _ in range(2))
        fb = min(fwd_bwd(prec, True) for _ in range(2))
        grads[prec] = {"forward_ms": round(f, 2), "forward_backward_ms": round(fb, 2),
                       "ratio": round(fb / f, 3)}
    out["gradient"] = grads
    print("[bench] moving-mesh smoother / coarse-operator ablation", file=sys.stderr, flush=True)
    out["ablation"] = ablation_leg(mgpu, torch, psi, b, tol)
    return out


def predictor_leg(mgpu, torch, mg, sources, tol):
    """Initial guesses on the warm-start sequence (Sec. 3.2): each step solved
    to `tol` from the predictor's guess, with earlier solutions kept on the
    device; the CG variant seeds multigrid-preconditioned CG with the recycled
    potential.  Steps without enough history use the longest predictor they
    can (t = 0 starts from zero)."""
    n = sources[0].shape[0]
    need = {"recycle": 1, "growth": 1, "linear": 2, "quadratic": 3}
    out = {}
    for variant in ("recycle", "growth", "linear", "quadratic", "pcg"):
        kind = "recycle" if variant == "pcg" else variant
        hist = []
        cyc, res0 = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t, b in enumerate(sources):
            if not hist:
                guess = torch.zeros_like(b)
            else:
                k = kind if len(hist) >= need[kind] else ("linear" if len(hist) == 2 else "recycle")
                g = (1.0 + 0.05 * t) / (1.0 + 0.05 * (t - 1))
                guess = mgpu.predict(k, hist, growth=g if k == "growth" else 1.0)
            fn = mg.solve_pcg if variant == "pcg" else mg.solve
            kw = {"max_iter": 60} if variant == "pcg" else {"max_cycles": 60}
            phi, info = fn(b, phi0=guess, out=guess, tol=tol, history=False, **kw)
            cyc.append(info.cycles)
            res0.append(info.rel_res0)
            hist = [phi] + hist[:2]
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        out[variant] = {"cycles_per_step": cyc, "total_cycles": sum(cyc), "ms_per_sequence": round(ms, 3),
                        "rel_res0_per_step": [float(f"{r:.3e}") for r in res0]}
    return out


def ablation_leg(mgpu, torch, psi, b, tol):
    """Moving-mesh solver settings (Sec. 4.3, App. B): Chebyshev degree 3 with
    Gershgorin bounds vs weighted Jacobi (omega = 2/3, 2 sweeps), coarse
    coefficients by full weighting of C vs rediscretised from the restricted
    deformation potential, and the potential-rediscretised hierarchy under CG.
    The fine operator is the same float64 C(psi) in every variant; mixed
    precision, cold solves to `tol`."""
    C64, _ = mgpu.geometry(psi)
    n = psi.shape[0]
    out = {}
    for smoother in ("chebyshev", "jacobi"):
        for coarse in ("fw_coeff", "psi"):
            kw = {"psi": psi} if coarse == "psi" else {"coeff": C64}
            mg = mgpu.Multigrid(n, precision="mixed", smoother=smoother, **kw)
            info, ms, phi, _ = solve_timed(mg, torch, b, tol, max_cycles=100)
            out[f"{smoother}+{coarse}"] = {"cycles": info.cycles, "time_to_tol_ms": round(ms, 3),
                                           "rel_res": info.rel_res}
            if smoother == "chebyshev" and coarse == "psi":
                phi.zero_()
                mg.solve_pcg(b, phi0=phi, out=phi, tol=tol, max_iter=100, history=False, raise_on_error=False)
                phi.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, pinfo = mg.solve_pcg(b, phi0=phi, out=phi, tol=tol, max_iter=100, history=False,
                                        raise_on_error=False)
                torch.cuda.synchronize()
                out["pcg+chebyshev+psi"] = {"cycles": pinfo.cycles,
                                            "time_to_tol_ms": round(1e3 * (time.perf_counter() - t0), 3),
                                            "rel_res": pinfo.rel_res}
            del mg, phi
    del C64
    torch.cuda.empty_cache()
    return out


def accel_leg(mgpu, torch, phi, psi, reps=20):
    """Force readout -s J^-1 grad phi after the solve: average kernel time and
    algorithmic HBM rate (phi, psi read once; three components written)."""
    n = phi.shape[0]
    out = {}
    for name, ps in (("flat", None), ("curvilinear", psi)):
        for dt, sz in ((torch.float32, 4), (torch.float64, 8)):
            a = mgpu.accel(phi, ps, scale=1.5 * 0.3, dtype=dt)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                a = mgpu.accel(phi, ps, scale=1.5 * 0.3, dtype=dt)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            by = n ** 3 * (8 + (8 if ps is not None else 0) + 3 * sz)
            out[f"{name}_{'f32' if sz == 4 else 'f64'}"] = {"ms": round(ms, 4), "alg_bytes": by,
                                                           "GBps": round(by / (ms * 1e-3) / 1e9, 1)}
            del a
    return out


def host_cpu():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_available": avail}


def cpu_leg(src_np, n, levels, deg, phi_mixed, phi_fp32, fp32_info, c2_cycles, c4_cycles):
    """The oracle (NumPy float64, one thread: roll, ufuncs and the FFT run
    single-threaded) on a bounded sample of the benchmark's work: one warm-up
    V-cycle, then the median of 3 timed V-cycles at 256^3 on source t = 0
    (seven-point), and one V-cycle of the 19-point moving-mesh operator after
    a warm-up cycle.  Time to 1e-10 is estimated from these as the cycle
    count the solve needs (measured on the GPU, same arithmetic) times one
    cycle plus one residual evaluation.  Also the accuracy of the timed mixed
    path and the pure-float32 plateau against the oracle's exact
    FFT-diagonalised solve."""
    import json as _json

    from oracle import mg_oracle as O
    from workloads import moving_mesh_field, psi_unit

    N = n ** 3
    h = 1.0 / n
    H = O.build_hierarchy(n, levels, deg)
    b0 = src_np[0] - src_np[0].mean()
    x = O.vcycle(H, 0, np.zeros_like(b0), b0)  # warm-up
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        x = O.vcycle(H, 0, x, b0)
        times.append(time.perf_counter() - t0)
    t0 = time.perf_counter()
    float(np.linalg.norm(b0 - H.levels[0].apply(x)))
    t_res = time.perf_counter() - t0
    med = float(np.median(times))
    # 19-point operator: moving-mesh coefficients (float32 values, as on the GPU)
    scale = _json.load(open(os.path.join(ROOT, "tests", "golden", "psi_scale.json")))["scale"][str(n)]
    t0 = time.perf_counter()
    C, sg = O.geometry(scale * psi_unit(n), h)
    C = C.astype(np.float32).astype(np.float64)
    g = moving_mesh_field(n, 0)
    bm = sg * (g - np.sum(g * sg) / np.sum(sg))
    bm -= bm.mean()
    Hv = O.build_hierarchy(n, levels, deg, C=C)
    t_setup_var = time.perf_counter() - t0
    xv = O.vcycle(Hv, 0, np.zeros_like(bm), bm)  # warm-up
    t0 = time.perf_counter()
    xv = O.vcycle(Hv, 0, xv, bm)
    t_var = time.perf_counter() - t0
    t0 = time.perf_counter()
    float(np.linalg.norm(bm - Hv.levels[0].apply(xv)))
    t_res_var = time.perf_counter() - t0
    del Hv, C, sg, g, bm, xv
    # accuracy against the exact discrete solve
    last = src_np[-1]
    exact = O.fft_solve(last - last.mean(), h)
    err = float(np.linalg.norm(phi_mixed.cpu().numpy() - exact) / np.linalg.norm(exact))
    out = {
        "value": round(N / med / 1e6, 3),
        "unit": "Mpts/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"NumPy float64 oracle at {n}^3, one thread: median of 3 seven-point V-cycles after a "
                   f"warm-up cycle (source t=0; {', '.join(f'{t:.2f}' for t in times)} s), and one "
                   f"19-point moving-mesh V-cycle after a warm-up cycle ({t_var:.2f} s)"),
        **host_cpu(),
        "vcycle_s_median": round(med, 3),
        "residual_eval_s": round(t_res, 3),
        "vcycle_19pt_s": round(t_var, 3),
        "vcycle_19pt_mpts_per_s": round(N / t_var / 1e6, 3),
        "setup_19pt_s": round(t_setup_var, 2),
        "est_time_to_1e-10_s": {
            "c2_first_source": round(c2_cycles[0] * (med + t_res) + t_res, 1),
            "c2_cycles": c2_cycles[0],
            "c4_moving_mesh": round(c4_cycles * (t_var + t_res_var) + t_res_var, 1) if c4_cycles else None,
            "c4_cycles": c4_cycles,
        },
        "mixed_final_rel_err_vs_oracle_exact": err,
    }
    if phi_fp32 is not None:
        b0e = O.fft_solve(b0, h)
        out["fp32_plateau"] = {
            "source": "warm-start sequence t=0, cold, tolerance disabled (stops at stagnation)",
            "cycles": fp32_info["cycles"], "rel_res": fp32_info["rel_res"],
            "rel_err_vs_oracle_exact": float(np.linalg.norm(phi_fp32.cpu().numpy() - b0e) / np.linalg.norm(b0e)),
        }
    return out


def timed(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [fn() for _ in range(steps)]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--sources", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--degree", type=int, default=3)
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 comparison sequence")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 32^3..1024^3 size sweep")
    ap.add_argument("--no-b512", action="store_true", help="skip the 512^3 V-cycle leg")
    ap.add_argument("--sweep-max", type=int, default=1024, help="largest grid of the size sweep")
    ap.add_argument("--no-mm", action="store_true", help="skip the moving-mesh and gradient leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-next", action="store_true", help="skip the predictor, CG and force-readout legs")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        sys.stderr.write("bench.py measures one GPU only: the multigrid path here is single-GPU "
                         "(multi-GPU halo exchange is not built); run with --gpus 1.\n")
        sys.exit(2)

    import torch

    import paper_2607_10983_amd as mgpu
    from workloads import flat_source, warm_sequence

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n, levels, deg = args.n, int(np.log2(args.n)) - 1, args.degree
    print(f"[bench] generating {args.sources} sources at {n}^3", file=sys.stderr, flush=True)
    src_np = list(warm_sequence(n, args.sources))
    sources = [torch.from_numpy(s).to(dev) for s in src_np]
    phi = torch.zeros((n, n, n), dtype=torch.float64, device=dev)

    # ------------------------------------------------------------- mixed (timed)
    mg = mgpu.Multigrid(n, levels=levels, degree=deg, precision="mixed")
    for _ in range(args.warmup):
        run_sequence(mg, sources, phi, args.tol)
    # the dominant kernel of the step: the fine-level kernel kind with the
    # largest total time over one untimed sequence per kind
    kinds = breakdown(mg, lambda: run_sequence(mg, sources, phi, args.tol))
    dominant = max(kinds, key=lambda k: kinds[k][1])
    mg.enable_kernel_timing(dominant)
    mg.kernel_timing()  # reset counters
    print(f"[bench] timing {args.steps} mixed steps", file=sys.stderr, flush=True)
    t_mixed, cyc = timed(lambda: run_sequence(mg, sources, phi, args.tol), args.steps, torch)
    launches, k_ms, k_bytes = mg.kernel_timing()
    mg.enable_kernel_timing(0)
    phi_mixed = phi.clone()
    cycles_per_step = cyc[0]
    total_cycles = sum(sum(c) for c in cyc)
    ms_per_step = 1e3 * t_mixed / args.steps
    mpts = total_cycles * n ** 3 / t_mixed / 1e6
    bytes_cycle = model_bytes_per_cycle(n, levels, deg, "mixed")
    achieved = k_bytes / (k_ms * 1e-3) / 1e9 if k_ms > 0 else None
    others = [kernel_entry(kind, kinds[kind], n, "mixed", ms_per_step, deg)
              for kind in KINDS if kind != dominant and kinds[kind][0]]
    roofline = {
        "kernel": kernel_name(dominant, n, "mixed"),
        "bound": "hbm",
        "achieved": round(achieved, 1) if achieved else None,
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBPS, 4) if achieved else None,
        "traffic": measured_traffic(n, deg, kernel_name(dominant, n, "mixed").split()[0]),
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE)",
        "launches": launches,
        "avg_launch_us": round(1e3 * k_ms / launches, 2) if launches else None,
        "alg_bytes_per_launch": k_bytes / launches if launches else None,
        "share_of_step": round(k_ms / (1e3 * t_mixed), 4),
        "other_fine_kernels": others,
    }

    # ------------------------------------------------------------- float64 comparison
    fp64 = None
    if not args.no_fp64:
        mg64 = mgpu.Multigrid(n, levels=levels, degree=deg, precision="fp64")
        run_sequence(mg64, sources, phi, args.tol)
        k64 = max(1, min(args.steps, 3))
        print(f"[bench] timing {k64} float64 steps", file=sys.stderr, flush=True)
        t64, cyc64 = timed(lambda: run_sequence(mg64, sources, phi, args.tol), k64, torch)
        ms64 = 1e3 * t64 / k64
        diff = float(torch.linalg.norm(phi_mixed - phi) / torch.linalg.norm(phi))
        fp64 = {
            "ms_per_step": round(ms64, 3),
            "vcycles_per_step": cyc64[0],
            "vcycle_mpts_per_s": round(sum(sum(c) for c in cyc64) * n ** 3 / t64 / 1e6, 1),
            "time_to_tol_ratio_fp64_over_mixed": round(ms64 / ms_per_step, 3),
            "mixed_vs_fp64_rel_diff_final_phi": diff,
            "model_bytes_per_cycle_per_pt": round(model_bytes_per_cycle(n, levels, deg, "fp64") / n ** 3, 2),
        }
        del mg64

    # ------------------------------------------------------------- predictors, CG, force readout
    pred = accel = None
    if not args.no_next:
        print("[bench] predictor / CG leg", file=sys.stderr, flush=True)
        pred = predictor_leg(mgpu, torch, mg, sources, args.tol)
        psi_rf = None
        from workloads import psi_unit
        scale = json.load(open(os.path.join(ROOT, "tests", "golden", "psi_scale.json")))["scale"].get(str(n))
        if scale is not None:
            psi_rf = torch.from_numpy(scale * psi_unit(n)).to(dev)
        accel = accel_leg(mgpu, torch, phi_mixed, psi_rf)
        del psi_rf
    del mg
    torch.cuda.empty_cache()

    # ------------------------------------------------------------- 512^3 V-cycle
    b512 = None
    if not args.no_b512:
        print("[bench] 512^3 V-cycle", file=sys.stderr, flush=True)
        b512 = b512_leg(mgpu, torch, flat_source)
        torch.cuda.empty_cache()

    # ------------------------------------------------------------- size sweep 32^3 .. 1024^3
    sweep = {}
    if not args.no_sweep:
        for ns in [m for m in (32, 64, 128, 256, 512, 1024) if m <= args.sweep_max]:
            print(f"[bench] sweep {ns}^3", file=sys.stderr, flush=True)
            sweep[str(ns)] = sweep_point(mgpu, torch, flat_source, ns, args.tol)
            torch.cuda.empty_cache()

    # ------------------------------------------------------------- moving mesh (19-point operator)
    mm = None
    if not args.no_mm:
        print("[bench] moving-mesh leg", file=sys.stderr, flush=True)
        mm = moving_mesh_leg(mgpu, torch, 256, args.tol)
        torch.cuda.empty_cache()

    # ------------------------------------------------------------- pure float32 plateau (C2 t = 0)
    plateau_phi = None
    if not args.no_cpu:
        mg32 = mgpu.Multigrid(n, levels=levels, degree=deg, precision="fp32")
        plateau_phi, p32 = mg32.solve(sources[0], tol=0.0, max_cycles=40, history=False, raise_on_error=False)
        plateau_info = {"cycles": p32.cycles, "rel_res": p32.rel_res}
        del mg32

    # ------------------------------------------------------------- CPU oracle baseline
    cpu = None
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_leg(src_np, n, levels, deg, phi_mixed, plateau_phi, plateau_info, cycles_per_step,
                      mm["fp64"]["cycles"] if mm else None)

    result = {
        "metric": METRIC,
        "value": round(mpts, 1),
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"warm-start defect correction: {n}^3 periodic seven-point Poisson, "
                        f"{args.sources} sequential GRF sources, each to rel. residual {args.tol:g} "
                        f"from the previous solution, {levels} levels, Chebyshev degree {deg}, mixed precision",
            "n": n, "levels": levels, "degree": deg, "sources": args.sources, "tol": args.tol,
        },
        "vcycles_per_step": cycles_per_step,
        "model_bytes_per_cycle_per_pt": round(bytes_cycle / n ** 3, 2),
        "model_GBps": round(total_cycles * bytes_cycle / t_mixed / 1e9, 1),
        "roofline": roofline,
        "fp64": fp64,
        "sweep": sweep,
        "b512": b512,
        "moving_mesh": mm,
        "predictors": pred,
        "accel": accel,
        "cpu_baseline": cpu,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
