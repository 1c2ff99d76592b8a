"""The kernels of the inner V-cycle, in the precision the solver runs them,
against the CPU float64 oracle, point by point.

``mg_inner_step`` runs one step of the V-cycle through exactly the kernels
``mg_solve`` launches on that level (row-wave single steps, two- and
three-step passes, the pass from zero, the prolongation fused into the
post-smoothing pass, the fused 32^3 / 64^3 visits, the single-workgroup tail)
in the context's inner precision.  Inputs are rounded to that precision
first, and the oracle receives the rounded values, so the comparison measures
the kernels' arithmetic only.

Bars (max-norm error relative to the max-norm of the oracle's result):
float kernels 5e-6 for one pass (a few float roundings per step, at most
four steps) and 2e-5 for a whole inner V-cycle; double kernels 1e-12.

Sizes up to 256^3 are compared on the full grid.  At 512^3 the kernels run on
the full grid in the launch shapes of the 512^3 benchmark leg and the oracle
evaluates periodic windows that straddle the boundary: a smoothing step reads
one neighbour per axis, so a window with a halo of v + 1 points gives exact
oracle values in its interior.
"""
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import mg_oracle as O  # noqa: E402
import workloads as W  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PSI_SCALE = json.load(open(os.path.join(ROOT, "tests", "golden", "psi_scale.json")))["scale"]

FLOAT_PASS_BAR = 5e-6
FLOAT_CYCLE_BAR = 2e-5
DOUBLE_BAR = 1e-12


@pytest.fixture(scope="module")
def mgpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_10983_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rounded(a, precision):
    """The values the inner kernels see: float32-rounded unless the context is fp64."""
    return a if precision == "fp64" else a.astype(np.float32).astype(np.float64)


def maxrel(out, ref):
    return float(np.max(np.abs(out - ref)) / np.max(np.abs(ref)))


def bar(precision, cycle=False):
    if precision == "fp64":
        return DOUBLE_BAR
    return FLOAT_CYCLE_BAR if cycle else FLOAT_PASS_BAR


def field(rng, n, precision):
    return rounded(rng.standard_normal((n, n, n)), precision)


def win(a, start, size):
    """Periodic window a[start:start+size] along every axis (indices wrap)."""
    n = a.shape[0]
    idx = [(np.arange(s, s + size) % n) for s in start]
    return a[np.ix_(*idx)]


# ------------------------------------------------------------------ passes on the full grid

@pytest.mark.parametrize("n", [64, 128, 256])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("degree", [3, 4])
def test_smoothing_passes(mgpu, n, precision, degree):
    """S(x, b), S(0, b) and S(x + P e, b) on the fine level of a benchmark-shaped hierarchy."""
    rng = np.random.default_rng(100 * n + degree)
    levels = int(math.log2(n)) - 1
    mg = mgpu.Multigrid(n, levels=levels, degree=degree, precision=precision)
    H = O.build_hierarchy(n, levels, degree)
    lev = H.levels[0]
    x = field(rng, n, precision)
    b = field(rng, n, precision)
    e = rounded(rng.standard_normal((n // 2,) * 3), precision)
    cases = {
        "smooth": (dict(x=dev(x), b=dev(b)), lambda: O.smooth(H, lev, x, b)),
        "smooth_zero": (dict(b=dev(b)), lambda: O.smooth(H, lev, np.zeros_like(b), b)),
        "prolong_smooth": (dict(x=dev(x), e=dev(e), b=dev(b)), lambda: O.smooth(H, lev, x + O.prolong(e), b)),
    }
    for step, (kw, ref_fn) in cases.items():
        out = host(mg.inner_step(step, 0, **kw))
        err = maxrel(out, ref_fn())
        print(f"{n}^3 {precision} degree {degree} {step}: max rel err {err:.2e}", flush=True)
        assert err <= bar(precision), (step, err)


@pytest.mark.parametrize("n", [64, 128, 256])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_transfers(mgpu, n, precision):
    """R(b - M x) and x + P e through the row kernels of the fine level."""
    rng = np.random.default_rng(7 * n)
    levels = int(math.log2(n)) - 1
    mg = mgpu.Multigrid(n, levels=levels, degree=3, precision=precision)
    x = field(rng, n, precision)
    b = field(rng, n, precision)
    e = rounded(rng.standard_normal((n // 2,) * 3), precision)
    out = host(mg.inner_step("residual_restrict", 0, x=dev(x), b=dev(b)))
    err = maxrel(out, O.restrict_fw(b - O.apply_flat(x, 1.0 / n)))
    print(f"{n}^3 {precision} residual_restrict: {err:.2e}", flush=True)
    assert err <= bar(precision)
    out = host(mg.inner_step("prolong", 0, x=dev(x), e=dev(e)))
    err = maxrel(out, x + O.prolong(e))
    print(f"{n}^3 {precision} prolong: {err:.2e}", flush=True)
    assert err <= bar(precision)


# ------------------------------------------------------------------ inner V-cycle from zero

@pytest.mark.parametrize("n,levels,degree", [(32, 4, 3), (64, 5, 3), (64, 3, 4), (128, 6, 3), (128, 4, 4),
                                             (256, 7, 3), (256, 5, 4)])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_inner_vcycle_from_zero(mgpu, n, levels, degree, precision):
    """e = V(0, r): the inner cycle each defect-correction iteration applies to
    its residual, every level's kernels included (visits at 32^3 and 64^3, the
    tail kernel below 16^3, the exact 16^3 solve where it is the coarsest)."""
    r = W.flat_source(n, 3)
    r = rounded(r - r.mean(), precision)
    mg = mgpu.Multigrid(n, levels=levels, degree=degree, precision=precision)
    out = host(mg.inner_step("vcycle", 0, b=dev(r)))
    H = O.build_hierarchy(n, levels, degree)
    ref = O.vcycle(H, 0, np.zeros_like(r), r)
    err = maxrel(out, ref)
    print(f"{n}^3 levels {levels} degree {degree} {precision}: V(0, r) max rel err {err:.2e}", flush=True)
    assert err <= bar(precision, cycle=True)


@pytest.mark.parametrize("n", [64, 128])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_inner_steps_19_point(mgpu, n, precision):
    """The 19-point row kernels in the inner precision (coefficients stored
    in it too) against the oracle's flux-form operator."""
    rng = np.random.default_rng(11 * n)
    levels = int(math.log2(n)) - 2
    psi = PSI_SCALE[str(n)] * W.psi_unit(n)
    C = rounded(O.geometry(psi, 1.0 / n)[0], precision)
    mg = mgpu.Multigrid(n, levels=levels, degree=3, coeff=dev(C), precision=precision)
    H = O.build_hierarchy(n, levels, 3, C=C)
    lev = H.levels[0]
    x = field(rng, n, precision)
    b = field(rng, n, precision)
    e = rounded(rng.standard_normal((n // 2,) * 3), precision)
    checks = [
        ("smooth", dict(x=dev(x), b=dev(b)), O.smooth(H, lev, x, b), False),
        ("smooth_zero", dict(b=dev(b)), O.smooth(H, lev, np.zeros_like(b), b), False),
        ("prolong_smooth", dict(x=dev(x), e=dev(e), b=dev(b)), O.smooth(H, lev, x + O.prolong(e), b), False),
        ("residual_restrict", dict(x=dev(x), b=dev(b)), O.restrict_fw(b - O.apply_var(x, C, 1.0 / n)), False),
    ]
    r = W.flat_source(n, 4)
    r = rounded(r - r.mean(), precision)
    checks.append(("vcycle", dict(b=dev(r)), O.vcycle(H, 0, np.zeros_like(r), r), True))
    for step, kw, ref, cyc in checks:
        out = host(mg.inner_step(step, 0, **kw))
        err = maxrel(out, ref)
        print(f"19-point {n}^3 {precision} {step}: {err:.2e}", flush=True)
        # (the coarse levels' float coefficients are the double restriction
        # rounded to float, one more float rounding inside the cycle's bar)
        assert err <= bar(precision, cycle=cyc), (step, err)


# ------------------------------------------------------------------ 512^3 on periodic windows

@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("degree", [3, 4])
def test_passes_512_windows(mgpu, precision, degree):
    n, levels = 512, 6
    g = torch.Generator(device="cuda").manual_seed(512 + degree)
    xd = torch.randn((n, n, n), generator=g, device="cuda", dtype=torch.float64)
    bd = torch.randn((n, n, n), generator=g, device="cuda", dtype=torch.float64)
    ed = torch.randn((n // 2,) * 3, generator=g, device="cuda", dtype=torch.float64)
    if precision != "fp64":
        xd, bd, ed = (t.float().double() for t in (xd, bd, ed))
    mg = mgpu.Multigrid(n, levels=levels, degree=degree, precision=precision)
    H = O.build_hierarchy(n, 1, degree)
    lev = H.levels[0]
    outs = {
        "smooth": host(mg.inner_step("smooth", 0, x=xd, b=bd)),
        "smooth_zero": host(mg.inner_step("smooth_zero", 0, b=bd)),
        "prolong_smooth": host(mg.inner_step("prolong_smooth", 0, x=xd, e=ed, b=bd)),
        "residual_restrict": host(mg.inner_step("residual_restrict", 0, x=xd, b=bd)),
        "prolong": host(mg.inner_step("prolong", 0, x=xd, e=ed)),
    }
    x, b, e = host(xd), host(bd), host(ed)
    del xd, bd, ed
    halo, size = degree + 1, 40
    for start in [(0, 0, 0), (n - 13, 100, 257), (300, n - 7, 64), (2 * 77, 2 * 200, n - 20)]:
        start = tuple(s - s % 2 for s in start)  # even, so coarse points line up
        lo = tuple(s - 2 * halo for s in start)
        W_ = size + 4 * halo
        xw, bw = win(x, lo, W_), win(b, lo, W_)
        ew = win(e, tuple(s // 2 for s in lo), W_ // 2)
        inner = (slice(2 * halo, 2 * halo + size),) * 3
        refs = {
            "smooth": O.smooth(H, lev, xw, bw),
            "smooth_zero": O.smooth(H, lev, np.zeros_like(bw), bw),
            "prolong_smooth": O.smooth(H, lev, xw + O.prolong(ew), bw),
            "prolong": xw + O.prolong(ew),
        }
        for step, ref in refs.items():
            got = win(outs[step], start, size)
            err = maxrel(got, ref[inner])
            print(f"512^3 {precision} degree {degree} {step} window {start}: {err:.2e}", flush=True)
            assert err <= bar(precision), (step, start, err)
        # restriction: coarse window [start/2, start/2 + size/2) from the fine window
        rc = O.restrict_fw(bw - O.apply_flat(xw, 1.0 / n))
        cs = tuple(s // 2 for s in start)
        got = win(outs["residual_restrict"], cs, size // 2)
        ref = rc[(slice(halo, halo + size // 2),) * 3]
        err = maxrel(got, ref)
        print(f"512^3 {precision} residual_restrict window {start}: {err:.2e}", flush=True)
        assert err <= bar(precision)


def test_inner_step_rejects_bad_arguments(mgpu):
    mg = mgpu.Multigrid(32, levels=3, degree=3, precision="mixed")
    b = torch.zeros((32, 32, 32), dtype=torch.float64, device="cuda")
    lib = mgpu._lib.load()
    assert lib.mg_inner_step(mg._ctx, 9, 0, None, None, mgpu._ptr(b), mgpu._ptr(b)) == mgpu._lib.MG_ERR_INVALID
    assert lib.mg_inner_step(mg._ctx, mgpu._lib.MG_STEP_SMOOTH, 0, None, None, mgpu._ptr(b),
                             mgpu._ptr(b)) == mgpu._lib.MG_ERR_INVALID
    assert lib.mg_inner_step(mg._ctx, mgpu._lib.MG_STEP_PROLONG, 2, mgpu._ptr(b), mgpu._ptr(b), None,
                             mgpu._ptr(b)) == mgpu._lib.MG_ERR_INVALID
    assert lib.mg_inner_step(mg._ctx, mgpu._lib.MG_STEP_VCYCLE, 3, None, None, mgpu._ptr(b),
                             mgpu._ptr(b)) == mgpu._lib.MG_ERR_INVALID


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_smoothing_1024_windows(mgpu, precision):
    """1024^3 (rows of 8 KB in double, 4 KB in float, split over four and
    two waves per row): one smoothing pass from x, from zero and from
    x + P e, the prolongation and residual + restriction, on periodic
    windows."""
    n, levels, degree = 1024, 7, 4
    free, _ = torch.cuda.mem_get_info()
    if free < 64 * 2**30:
        pytest.skip("needs ~64 GiB of free device memory")
    g = torch.Generator(device="cuda").manual_seed(1024)
    xd = torch.randn((n, n, n), generator=g, device="cuda", dtype=torch.float64)
    bd = torch.randn((n, n, n), generator=g, device="cuda", dtype=torch.float64)
    ed = torch.randn((n // 2,) * 3, generator=g, device="cuda", dtype=torch.float64)
    if precision != "fp64":
        xd, bd, ed = xd.float().double(), bd.float().double(), ed.float().double()
    mg = mgpu.Multigrid(n, levels=levels, degree=degree, precision=precision)
    H = O.build_hierarchy(n, 1, degree)
    lev = H.levels[0]
    halo, size = degree + 1, 32
    starts = [(0, 0, 0), (n - 11, 500, 1000), (600, n - 5, 30)]
    lo = [tuple(s - s % 2 - 2 * halo for s in st) for st in starts]
    W_ = size + 4 * halo
    xw = [win_t(xd, l, W_) for l in lo]
    bw = [win_t(bd, l, W_) for l in lo]
    ew = [win_t(ed, tuple(s // 2 for s in l), W_ // 2) for l in lo]
    inner = (slice(2 * halo, 2 * halo + size),) * 3
    for step in ("prolong", "prolong_smooth"):
        out = mg.inner_step(step, 0, x=xd, e=ed, b=bd if step == "prolong_smooth" else None)
        for k, l in enumerate(lo):
            got = win_t(out, tuple(s + 2 * halo for s in l), size)
            x0 = xw[k] + O.prolong(ew[k])
            ref = (x0 if step == "prolong" else O.smooth(H, lev, x0, bw[k]))[inner]
            err = maxrel(got, ref)
            print(f"1024^3 {precision} {step} window {starts[k]}: {err:.2e}", flush=True)
            assert err <= bar(precision), (step, starts[k], err)
        del out
    for step in ("smooth", "smooth_zero"):
        out = mg.inner_step(step, 0, x=xd if step == "smooth" else None, b=bd)
        for k, l in enumerate(lo):
            got = win_t(out, tuple(s + 2 * halo for s in l), size)
            x0 = xw[k] if step == "smooth" else np.zeros_like(bw[k])
            ref = O.smooth(H, lev, x0, bw[k])[inner]
            err = maxrel(got, ref)
            print(f"1024^3 {precision} {step} window {starts[k]}: {err:.2e}", flush=True)
            assert err <= bar(precision), (step, starts[k], err)
        del out
    # residual + restriction (rows split over waves in both precisions at this size)
    out = mg.inner_step("residual_restrict", 0, x=xd, b=bd)
    for k, l in enumerate(lo):
        rc = O.restrict_fw(bw[k] - O.apply_flat(xw[k], 1.0 / n))
        got = win_t(out, tuple((s + 2 * halo) // 2 for s in l), size // 2)
        err = maxrel(got, rc[(slice(halo, halo + size // 2),) * 3])
        print(f"1024^3 {precision} residual_restrict window {starts[k]}: {err:.2e}", flush=True)
        assert err <= bar(precision), ("residual_restrict", starts[k], err)


def win_t(t, start, size):
    """Periodic window of a device field, copied to the host."""
    n = t.shape[0]
    idx = [torch.arange(s, s + size, device=t.device) % n for s in start]
    return t[idx[0]][:, idx[1]][:, :, idx[2]].cpu().numpy()
