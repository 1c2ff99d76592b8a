"""Parity of the HIP path (through the C ABI) with the CPU float64 oracle.

Floating-point bars: plain float64 path <= 1e-12 relative L2 against the
oracle (residual histories <= 1e-12 absolute; histories are already divided
by ||b||); mixed precision <= 1e-10 relative error against the exact
discrete solution; pure float32 plateau <= 1e-5.  Single steps are compared
element by element at sizes that span several thread blocks and wrap the
periodic boundary.
"""
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import mg_oracle as O  # noqa: E402
from workloads import flat_source, moving_mesh_field, psi_unit  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PSI_SCALE = json.load(open(os.path.join(ROOT, "tests", "golden", "psi_scale.json")))["scale"]
RNG = np.random.default_rng(2024)


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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def moving_mesh_coeff(n, dtype=np.float64):
    """C and sqrt(g) of the admissible moving-mesh deformation (oracle geometry)."""
    psi = PSI_SCALE[str(n)] * psi_unit(n)
    C, sg = O.geometry(psi, 1.0 / n)
    return psi, C.astype(dtype), sg


def random_spd(n, amp=0.3):
    A = amp * RNG.standard_normal((n, n, n, 3, 3))
    S = np.eye(3) + A @ np.swapaxes(A, -1, -2)
    idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    return np.stack([S[..., a, b] for a, b in idx])


# ------------------------------------------------------------------ single steps

@pytest.mark.parametrize("n", [8, 16, 64])
@pytest.mark.parametrize("var", [False, True])
def test_apply(mgpu, n, var):
    C = random_spd(n) if var else None
    levels = max(1, int(math.log2(n)) - 2)
    mg = mgpu.Multigrid(n, levels=levels, coeff=dev(C) if var else None, precision="fp64")
    u = RNG.standard_normal((n, n, n))
    ref = O.apply_var(u, C, 1.0 / n) if var else O.apply_flat(u, 1.0 / n)
    out = host(mg.apply(dev(u)))
    assert np.max(np.abs(out - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("var,n", [(False, 16), (True, 16), (False, 64), (False, 128), (False, 256),
                                   (True, 64), (True, 128)])
@pytest.mark.parametrize("degree", [1, 3, 4])
def test_smooth(mgpu, var, n, degree):
    C = random_spd(n) if var else None
    levels = 2 if n == 16 else int(math.log2(n)) - 2
    mg = mgpu.Multigrid(n, levels=levels, degree=degree, coeff=dev(C) if var else None, precision="fp64")
    H = O.build_hierarchy(n, levels if var else 1, degree, C=C)
    x = RNG.standard_normal((n, n, n))
    b = RNG.standard_normal((n, n, n))
    ref = O.smooth(H, H.levels[0], x, b)
    out = host(mg.smooth(dev(x), dev(b)))
    assert rel(out, ref) <= 1e-13
    if var:
        assert mg.level_lmax()[0] == pytest.approx(H.levels[0].cheb.lmax, rel=1e-14)
    else:
        assert mg.level_lmax()[0] == 2.0


def test_smooth_jacobi(mgpu):
    n = 16
    mg = mgpu.Multigrid(n, levels=2, smoother="jacobi", precision="fp64")
    H = O.build_hierarchy(n, 2, 3, smoother="jacobi")
    x = RNG.standard_normal((n, n, n))
    b = RNG.standard_normal((n, n, n))
    assert rel(host(mg.smooth(dev(x), dev(b))), O.smooth(H, H.levels[0], x, b)) <= 1e-13


@pytest.mark.parametrize("n", [8, 32, 64, 128, 256])
@pytest.mark.parametrize("var", [False, True])
def test_residual_restrict_and_prolong(mgpu, n, var):
    C = random_spd(n) if var else None
    levels = max(2, int(math.log2(n)) - 2)
    mg = mgpu.Multigrid(n, levels=levels, coeff=dev(C) if var else None, precision="fp64")
    h = 1.0 / n
    x = RNG.standard_normal((n, n, n))
    b = RNG.standard_normal((n, n, n))
    Mx = O.apply_var(x, C, h) if var else O.apply_flat(x, h)
    ref = O.restrict_fw(b - Mx)
    out = host(mg.residual_restrict(dev(x), dev(b)))
    assert np.max(np.abs(out - ref)) <= 1e-13 * np.max(np.abs(ref))
    out0 = host(mg.residual_restrict(None, dev(b)))
    assert np.max(np.abs(out0 - O.restrict_fw(b))) <= 1e-15 * 10
    e = RNG.standard_normal((n // 2,) * 3)
    outp = host(mg.prolong_add(dev(e), dev(x)))
    assert np.max(np.abs(outp - (x + O.prolong(e)))) <= 1e-15 * 10


@pytest.mark.parametrize("nc", [4, 8, 16])
def test_coarse_solve_flat(mgpu, nc):
    n = nc * 4
    mg = mgpu.Multigrid(n, levels=3, precision="fp64")
    r = RNG.standard_normal((nc, nc, nc))
    hc = 4.0 / n
    ref = O.fft_solve(r - r.mean(), hc)
    out = host(mg.coarse_solve(dev(r)))
    assert rel(out, ref) <= 1e-13


def test_coarse_solve_var(mgpu):
    n = 16
    C = random_spd(n)
    mg = mgpu.Multigrid(n, levels=3, coeff=dev(C), precision="fp64")
    H = O.build_hierarchy(n, 3, 3, C=C)
    r = RNG.standard_normal((4, 4, 4))
    ref = O.coarse_solve(H.levels[-1], r - r.mean())
    out = host(mg.coarse_solve(dev(r)))
    assert rel(out, ref) <= 1e-12


# ------------------------------------------------------------------ V-cycle and solve

@pytest.mark.parametrize("var", [False, True])
def test_single_vcycle(mgpu, var):
    n = 32
    levels = 4 if not var else 3
    C = moving_mesh_coeff(n)[1] if var else None
    mg = mgpu.Multigrid(n, levels=levels, coeff=dev(C) if var else None, precision="fp64")
    H = O.build_hierarchy(n, levels, 3, C=C)
    b = flat_source(n, 3)
    b -= b.mean()
    phi = RNG.standard_normal((n, n, n))
    ref = O.vcycle(H, 0, phi, b)
    p = dev(phi)
    r = mg.vcycle(p, dev(b), rel_res=True)
    assert rel(host(p), ref) <= 1e-12
    Mref = O.apply_var(ref, C, 1.0 / n) if var else O.apply_flat(ref, 1.0 / n)
    assert r == pytest.approx(np.linalg.norm(b - Mref) / np.linalg.norm(b), rel=1e-10)


def test_config1_fp64_solution_and_history(mgpu):
    """32^3, 4 levels, Chebyshev degree 3, zero guess, 10 V-cycles, float64."""
    n = 32
    b = flat_source(n, 0)
    mg = mgpu.Multigrid(n, levels=4, degree=3, precision="fp64")
    phi, info = mg.solve(dev(b), tol=0.0, max_cycles=10, raise_on_error=False)
    ref = O.solve(O.build_hierarchy(n, 4, 3), b, tol=0.0, max_cycles=10)
    assert info.cycles == 10
    assert rel(host(phi), ref.phi) <= 1e-12
    assert np.max(np.abs(np.array(info.history) - np.array(ref.history))) <= 1e-12
    assert abs(host(phi).mean()) < 1e-15


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_flat_solve_reaches_exact_solution(mgpu, precision, bar):
    n = 64
    b = flat_source(n, 1)
    mg = mgpu.Multigrid(n, levels=5, degree=4, precision=precision)
    phi, info = mg.solve(dev(b), tol=1e-13 if precision == "fp64" else 1e-11, max_cycles=40,
                         raise_on_error=False)
    exact = O.fft_solve(b - b.mean(), 1.0 / n)
    err = float(rel(host(phi), exact))
    assert err <= bar, err
    assert info.rel_res <= (2e-13 if precision == "fp64" else 1e-11)


def test_mixed_history_tracks_fp64(mgpu):
    n = 64
    b = flat_source(n, 2)
    h64 = mgpu.Multigrid(n, levels=5, precision="fp64").solve(dev(b), tol=0, max_cycles=8, raise_on_error=False)[1]
    hmx = mgpu.Multigrid(n, levels=5, precision="mixed").solve(dev(b), tol=0, max_cycles=8, raise_on_error=False)[1]
    a, m = np.array(h64.history), np.array(hmx.history)
    assert np.all(np.abs(m - a) <= 1e-4 * a + 1e-12)


def test_fp32_plateau(mgpu):
    n = 64
    b = flat_source(n, 0)
    mg = mgpu.Multigrid(n, levels=5, precision="fp32")
    phi, info = mg.solve(dev(b), tol=1e-12, max_cycles=30, raise_on_error=False)
    exact = O.fft_solve(b - b.mean(), 1.0 / n)
    assert rel(host(phi), exact) <= 1e-5


def test_warm_start_saves_cycles(mgpu):
    n = 64
    from workloads import Spectrum, grf
    delta = grf(n, Spectrum(-1.0), 0)
    mg = mgpu.Multigrid(n, levels=5, precision="mixed")
    phi, i0 = mg.solve(dev(delta), tol=1e-10)
    b1 = 1.05 * delta + 0.02 * grf(n, Spectrum(-1.0), 101)
    _, cold = mg.solve(dev(b1), tol=1e-10)
    _, warm = mg.solve(dev(b1), phi0=phi, tol=1e-10)
    assert warm.cycles < cold.cycles
    ref = O.fft_solve(b1 - b1.mean(), 1.0 / n)
    phi1, _ = mg.solve(dev(b1), phi0=phi, tol=1e-11)
    assert rel(host(phi1), ref) <= 1e-10


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("mixed", 1e-10)])
@pytest.mark.parametrize("cdtype", [np.float64, np.float32])
def test_moving_mesh_solve(mgpu, precision, bar, cdtype):
    n = 32
    psi, C, sg = moving_mesh_coeff(n, cdtype)
    g = moving_mesh_field(n, 0)
    b = sg * (g - np.sum(g * sg) / np.sum(sg))
    Cd = C.astype(np.float64)
    H = O.build_hierarchy(n, 4, 3, C=Cd)
    ref = O.solve(H, b, tol=1e-13, max_cycles=200)
    mg = mgpu.Multigrid(n, levels=4, coeff=dev(C), precision=precision)
    phi, info = mg.solve(dev(b), tol=1e-13 if precision == "fp64" else 1e-11, max_cycles=200,
                         raise_on_error=False)
    assert info.rel_res <= (2e-13 if precision == "fp64" else 1e-11)
    assert rel(host(phi), ref.phi) <= bar
    if precision == "fp64":
        lm = O.gershgorin_lmax_var(Cd, 1.0 / n)
        assert mg.level_lmax()[0] == pytest.approx(lm, rel=1e-13)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_moving_mesh_solve_64(mgpu, precision, bar):
    """64^3: the fine level runs the 19-point row kernels."""
    n = 64
    psi, C, sg = moving_mesh_coeff(n)
    g = moving_mesh_field(n, 0)
    b = sg * (g - np.sum(g * sg) / np.sum(sg))
    ref = O.solve(O.build_hierarchy(n, 5, 3, C=C), b, tol=1e-13, max_cycles=60)
    mg = mgpu.Multigrid(n, levels=5, coeff=dev(C), precision=precision)
    phi, info = mg.solve(dev(b), tol=1e-13 if precision == "fp64" else 1e-11, max_cycles=60,
                         raise_on_error=False)
    assert rel(host(phi), ref.phi) <= bar
    if precision == "fp64":
        h6 = O.solve(O.build_hierarchy(n, 5, 3, C=C), b, tol=0.0, max_cycles=5).history
        _, i5 = mg.solve(dev(b), tol=0.0, max_cycles=5, raise_on_error=False)
        assert np.max(np.abs(np.array(i5.history) - np.array(h6))) <= 1e-12


def test_moving_mesh_fp64_history(mgpu):
    n = 32
    psi, C, sg = moving_mesh_coeff(n)
    b = moving_mesh_field(n, 0) * sg
    mg = mgpu.Multigrid(n, levels=4, coeff=dev(C), precision="fp64")
    phi, info = mg.solve(dev(b), tol=0.0, max_cycles=6, raise_on_error=False)
    ref = O.solve(O.build_hierarchy(n, 4, 3, C=C), b, tol=0.0, max_cycles=6)
    assert rel(host(phi), ref.phi) <= 1e-12
    assert np.max(np.abs(np.array(info.history) - np.array(ref.history))) <= 1e-12


# ------------------------------------------------------------------ adjoint, gradients, geometry

@pytest.mark.parametrize("n", [16, 32])
def test_geometry_forward(mgpu, n):
    psi = PSI_SCALE[str(n)] * psi_unit(n)
    Cref, sref = O.geometry(psi, 1.0 / n)
    C, sg = mgpu.geometry(dev(psi))
    assert rel(host(sg), sref) <= 1e-14
    assert np.max(np.abs(host(C) - Cref)) <= 1e-13 * np.max(np.abs(Cref))
    C32, _ = mgpu.geometry(dev(psi), dtype=torch.float32)
    assert np.max(np.abs(host(C32) - Cref)) <= 1e-6 * np.max(np.abs(Cref))


def test_geometry_backward(mgpu):
    n = 16
    psi = PSI_SCALE[str(n)] * psi_unit(n)
    Cbar = RNG.standard_normal((6, n, n, n))
    sbar = RNG.standard_normal((n, n, n))
    ref = O.geometry_bwd(psi, Cbar, sbar, 1.0 / n)
    out = host(mgpu.geometry_bwd(dev(psi), dev(Cbar), dev(sbar)))
    assert rel(out, ref) <= 1e-12
    out0 = host(mgpu.geometry_bwd(dev(psi), dev(Cbar), None))
    assert rel(out0, O.geometry_bwd(psi, Cbar, np.zeros((n, n, n)), 1.0 / n)) <= 1e-12


def test_coeff_grad(mgpu):
    n = 16
    C = random_spd(n)
    mg = mgpu.Multigrid(n, levels=2, coeff=dev(C), precision="fp64")
    lam = RNG.standard_normal((n, n, n))
    phi = RNG.standard_normal((n, n, n))
    ref = O.coeff_grad(lam, phi, 1.0 / n)
    out = host(mg.coeff_grad(dev(lam), dev(phi)))
    assert np.max(np.abs(out - ref)) <= 1e-13 * np.max(np.abs(ref))
    with pytest.raises(mgpu.MGError):
        mgpu.Multigrid(n, levels=2, precision="fp64").coeff_grad(dev(lam), dev(phi))


def test_adjoint_solve(mgpu):
    n = 32
    psi, C, sg = moving_mesh_coeff(n)
    w = RNG.standard_normal((n, n, n))
    mg = mgpu.Multigrid(n, levels=4, coeff=dev(C), precision="fp64")
    lam, info = mg.solve_adjoint(dev(w), tol=1e-12, max_cycles=100)
    ref = O.solve_adjoint(O.build_hierarchy(n, 4, 3, C=C), w, tol=1e-13, max_cycles=200)
    assert rel(host(lam), ref.phi) <= 1e-11


def test_autograd_matches_oracle_gradient(mgpu):
    """L = sum(w * phi), phi = solve(b(psi), C(psi)); dL/dpsi and dL/db vs the oracle."""
    n = 16
    h = 1.0 / n
    psi = PSI_SCALE[str(n)] * psi_unit(n)
    g = moving_mesh_field(n, 0)
    w = RNG.standard_normal((n, n, n))
    # GPU: differentiable geometry + torch-built source + differentiable solve
    psi_t = dev(psi).requires_grad_(True)
    g_t = dev(g)
    C_t, sg_t = mgpu.geometry_fn(psi_t)
    b_t = sg_t * (g_t - (g_t * sg_t).sum() / sg_t.sum())
    phi_t = mgpu.solve(b_t, C_t, tol=1e-13, max_cycles=200, levels=3, precision="fp64")
    L = (dev(w) * phi_t).sum()
    L.backward()
    gpu_grad = host(psi_t.grad)
    # oracle: same chain written with oracle pieces
    C, sg = O.geometry(psi, h)
    m = np.sum(g * sg) / np.sum(sg)
    b = sg * (g - m)
    H = O.build_hierarchy(n, 3, 3, C=C)
    phi = O.solve(H, b, tol=1e-14, max_cycles=300).phi
    lam = O.solve(H, w, tol=1e-14, max_cycles=300).phi
    Cbar = O.coeff_grad(lam, phi, h)
    # b = sg (g - m), m = sum(g sg)/sum(sg):  d/dsg
    S = np.sum(sg)
    sbar = lam * (g - m) - (g - m) / S * np.sum(lam * sg)
    ref = O.geometry_bwd(psi, Cbar, sbar, h)
    assert rel(gpu_grad, ref) <= 1e-8
    assert float(L) == pytest.approx(np.sum(w * phi), rel=1e-11)


def test_solve_fn_raises_when_not_converged(mgpu):
    """The implicit adjoint is valid only at a converged solve: the
    differentiable solve raises instead of returning silent gradients."""
    n = 16
    psi, C, sg = moving_mesh_coeff(n)
    b = dev(moving_mesh_field(n, 0) * sg).requires_grad_(True)
    with pytest.raises(mgpu.MGError) as e:
        mgpu.solve(b, dev(C), tol=1e-30, max_cycles=2, levels=2, precision="fp64")
    assert e.value.status == 6
    # converged: the context built for C is reused by the next call with the same tensor
    Ct = dev(C)
    p1 = mgpu.solve(b, Ct, tol=1e-12, max_cycles=100, levels=2, precision="fp64")
    p2 = mgpu.solve(b, Ct, tol=1e-12, max_cycles=100, levels=2, precision="fp64")
    assert torch.equal(p1, p2)
    (p2 * p2).sum().backward()
    assert b.grad is not None and torch.isfinite(b.grad).all()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_fixed_cycles_match_solve(mgpu, precision):
    """mg_cycles (a fixed number of warm cycles, no host wait between them)
    launches the same kernels in the same order as mg_solve with the
    tolerance disabled: bitwise the same potential and final residual."""
    n = 64
    b = dev(flat_source(n, 6))
    mg = mgpu.Multigrid(n, levels=5, degree=3, precision=precision)
    phi_s, info = mg.solve(b, tol=0.0, max_cycles=4, raise_on_error=False)
    phi_c = torch.zeros_like(phi_s)
    r = mg.cycles(phi_c, b, 4)
    assert info.cycles == 4
    assert torch.equal(phi_s, phi_c)
    assert r == info.rel_res
    # warm continuation: two more cycles from the gauge-fixed result equal a
    # 6-cycle solve up to rounding (the float inner cycle of mixed precision
    # sees the shifted iterate's residual rounded differently)
    mg.cycles(phi_c, b, 2)
    phi_6, info6 = mg.solve(b, tol=0.0, max_cycles=6, raise_on_error=False)
    assert rel(host(phi_c), host(phi_6)) <= (1e-13 if precision == "fp64" else 1e-11)
    z = torch.zeros_like(phi_c)
    assert mg.cycles(z, dev(np.full((n, n, n), 1.5)), 3) == 0.0 and float(z.abs().max()) == 0.0


# ------------------------------------------------------------------ errors, determinism

def test_invalid_coefficients_rejected(mgpu):
    n = 16
    C = random_spd(n)
    C[1, 3, 4, 5] = -1.0
    with pytest.raises(mgpu.MGError) as e:
        mgpu.Multigrid(n, levels=2, coeff=dev(C), precision="fp64")
    assert e.value.status == 2
    C = random_spd(n)
    C[4, 0, 0, 0] = np.nan
    with pytest.raises(mgpu.MGError):
        mgpu.Multigrid(n, levels=2, coeff=dev(C), precision="mixed")


def test_nonfinite_source_and_not_converged(mgpu):
    n = 16
    mg = mgpu.Multigrid(n, levels=2, precision="fp64")
    b = RNG.standard_normal((n, n, n))
    bad = b.copy()
    bad[1, 2, 3] = np.inf
    with pytest.raises(mgpu.MGError) as e:
        mg.solve(dev(bad))
    assert e.value.status == 5
    phi, info = mg.solve(dev(b), tol=1e-30, max_cycles=3, raise_on_error=False)
    assert info.status == 6 and info.cycles == 3
    z, info = mg.solve(dev(np.full((n, n, n), 2.5)))
    assert info.cycles == 0 and float(z.abs().max()) == 0.0


def test_bitwise_reproducible(mgpu):
    n = 64
    b = dev(flat_source(n, 5))
    mg = mgpu.Multigrid(n, levels=5, precision="mixed")
    p1, i1 = mg.solve(b, tol=1e-10)
    p2, i2 = mg.solve(b, tol=1e-10)
    assert torch.equal(p1, p2) and i1.history == i2.history


@pytest.mark.parametrize("var", [False, True])
def test_graph_replay_matches_eager(mgpu, var):
    """The coarse sub-cycle replayed from a captured HIP graph gives bitwise the
    same iterates as eager launches, replay after replay, with unrelated eager
    GPU work and synchronisations between the replays."""
    n = 64
    C = dev(moving_mesh_coeff(n)[1]) if var else None
    eager = mgpu.Multigrid(n, levels=5, coeff=C, precision="mixed")
    graph = mgpu.Multigrid(n, levels=5, coeff=C, precision="mixed", options=mgpu._lib.MG_OPT_GRAPH)
    pe = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    pg = torch.zeros_like(pe)
    for seed in (11, 12, 13, 14):
        b = dev(flat_source(n, seed))
        _, ie = eager.solve(b, phi0=pe, out=pe, tol=1e-10, max_cycles=40)
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        _, ig = graph.solve(b, phi0=pg, out=pg, tol=1e-10, max_cycles=40)
        assert float(junk) == float(junk)
        assert ig.cycles == ie.cycles and ig.history == ie.history
        assert torch.equal(pe, pg)


@pytest.mark.parametrize("n,prec", [(64, "mixed"), (128, "fp64"), (256, "mixed"), (256, "fp64"), (512, "mixed"),
                                    (512, "fp64")])
@pytest.mark.parametrize("degree,smoother", [(2, "chebyshev"), (3, "chebyshev"), (4, "chebyshev"), (6, "chebyshev"),
                                             (3, "jacobi")])
def test_two_step_kernel_matches_single_steps(mgpu, n, prec, degree, smoother):
    """The fused smoothing kernels (two or three steps in one pass over
    memory, steps formed from b, the prolongation inside the first pair)
    compute each step in the same order as the single-step kernel: solves
    agree bitwise with MG_OPT_NO_PAIR, cycle by cycle.  Rows of more than
    1 KB (512^3 float, 256^3 double) run the two-step kernels split over two
    waves per row; 512^3 double rows take no two-step kernel but start each
    pass from zero from b."""
    b = dev(flat_source(n, 3))
    levels = int(math.log2(n)) - 1
    kw = dict(levels=levels, degree=degree, precision=prec, smoother=smoother, sweeps=degree)
    single = mgpu.Multigrid(n, options=mgpu._lib.MG_OPT_NO_PAIR, **kw)
    fused = mgpu.Multigrid(n, **kw)
    out = []
    for mg in (single, fused):
        phi, info = mg.solve(b, tol=1e-10, max_cycles=12, raise_on_error=False)
        out.append((phi, info))
    (ps, is_), (pf, if_) = out
    assert is_.cycles == if_.cycles and is_.history == if_.history
    assert torch.equal(ps, pf)


@pytest.mark.parametrize("n", [128, 256])
@pytest.mark.parametrize("degree", [2, 3, 4])
def test_19_point_pair_matches_single_steps(mgpu, n, degree):
    """The 19-point two-step kernel (float rows of up to 1 KB: the last two
    Chebyshev steps of every pass on those levels) forms each step as the
    single-step kernel: moving-mesh mixed solves (float32 coefficients from the
    GPU geometry) agree bitwise with MG_OPT_NO_PAIR, cycle by cycle."""
    psi = PSI_SCALE[str(n)] * psi_unit(n)
    C32, sg = mgpu.geometry(dev(psi), dtype=torch.float32)
    g = dev(moving_mesh_field(n, 0))
    b = sg * (g - (g * sg).sum() / sg.sum())
    kw = dict(levels=int(math.log2(n)) - 1, degree=degree, coeff=C32, precision="mixed")
    single = mgpu.Multigrid(n, options=mgpu._lib.MG_OPT_NO_PAIR, **kw)
    fused = mgpu.Multigrid(n, **kw)
    out = []
    for mg in (single, fused):
        phi, info = mg.solve(b, tol=1e-10, max_cycles=8, raise_on_error=False)
        out.append((phi, info))
    (ps, is_), (pf, if_) = out
    print(f"19-point n={n} degree {degree}: {if_.cycles} cycles, rel_res {if_.rel_res:.2e}", flush=True)
    assert is_.cycles == if_.cycles and is_.history == if_.history
    assert torch.equal(ps, pf)


@pytest.mark.parametrize("n,levels", [(32, 4), (32, 2), (64, 5), (64, 3), (128, 6), (256, 7)])
@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_level_visit_matches_unfused(mgpu, n, levels, degree):
    """The fused visits of the 32^3 and 64^3 levels (smoothing from zero,
    residual and full weighting in one launch; prolongation and smoothing in
    another) use the point formulas of the separate kernels: mixed-precision
    solves agree bitwise with MG_OPT_NO_VISIT, cycle by cycle.  Degree 4 runs
    the 64^3 level's pre-smoothing unfused and its post visit fused."""
    b = dev(flat_source(n, 5))
    kw = dict(levels=levels, degree=degree, precision="mixed")
    plain = mgpu.Multigrid(n, options=mgpu._lib.MG_OPT_NO_VISIT, **kw)
    fused = mgpu.Multigrid(n, **kw)
    out = []
    for mg in (plain, fused):
        phi, info = mg.solve(b, tol=1e-10, max_cycles=10, raise_on_error=False)
        out.append((phi, info))
    (pp, ip), (pf, if_) = out
    assert ip.cycles == if_.cycles and ip.history == if_.history
    assert torch.equal(pp, pf)
