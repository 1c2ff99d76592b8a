"""Parity of the HIP path (through the C ABI) with the CPU float64 oracle for
the extensions beyond the core solve: coarse levels rediscretised from the
restricted deformation potential, multigrid-preconditioned CG, the
initial-guess predictors and the force readout.

Bars as in the core parity tests: float64 paths <= 1e-12 relative (residual
histories <= 1e-12 absolute); mixed precision <= 1e-10 relative error against
the float64 solution; elementwise kernels to a few ulps.
"""
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import mg_oracle as O  # noqa: E402
from workloads import flat_source, moving_mesh_field, psi_unit, warm_sequence  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PSI_SCALE = json.load(open(os.path.join(ROOT, "tests", "golden", "psi_scale.json")))["scale"]
RNG = np.random.default_rng(77)


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


def psi_of(n):
    return PSI_SCALE[str(n)] * psi_unit(n)


def mm_source(n, psi):
    """Moving-mesh source b = sqrt(g) (g - <g sqrt g>/<sqrt g>)."""
    _, sg = O.geometry(psi, 1.0 / n)
    g = moving_mesh_field(n)
    return sg * (g - np.sum(g * sg) / np.sum(sg))


# ------------------------------------------------ coarse levels from psi

@pytest.mark.parametrize("n,levels", [(16, 2), (32, 3)])
def test_psi_levels_apply(mgpu, n, levels):
    """Every level's operator equals the oracle's rediscretised one."""
    psi = psi_of(n)
    mg = mgpu.Multigrid(n, levels=levels, psi=dev(psi), precision="fp64")
    H = O.build_hierarchy(n, levels, psi=psi)
    fw = O.build_hierarchy(n, levels, C=O.geometry(psi, 1.0 / n)[0])
    for l, lev in enumerate(H.levels):
        nl = n >> l
        u = RNG.standard_normal((nl, nl, nl))
        ref = lev.apply(u)
        out = host(mg.apply(dev(u), level=l))
        assert np.max(np.abs(out - ref)) <= 1e-13 * np.max(np.abs(ref)), l
        if l > 0:   # and it is not the full-weighting coefficient hierarchy
            assert rel(fw.levels[l].apply(u), ref) > 1e-6
    # Gershgorin bounds of every smoothed level (the coarsest is solved exactly)
    np.testing.assert_allclose(mg.level_lmax()[:-1], [lev.cheb.lmax for lev in H.levels[:-1]], rtol=1e-13)


@pytest.mark.parametrize("smoother", ["chebyshev", "jacobi"])
def test_psi_solve_fp64_history(mgpu, smoother):
    n, levels = 32, 3
    psi = psi_of(n)
    b = mm_source(n, psi)
    mg = mgpu.Multigrid(n, levels=levels, psi=dev(psi), precision="fp64", smoother=smoother)
    H = O.build_hierarchy(n, levels, psi=psi, smoother=smoother)
    ref = O.solve(H, b, tol=0.0, max_cycles=8)
    phi, info = mg.solve(dev(b), tol=0.0, max_cycles=8, raise_on_error=False)
    assert info.cycles == 8
    assert np.max(np.abs(np.array(info.history) - np.array(ref.history))) <= 1e-12
    assert rel(host(phi), ref.phi) <= 1e-12


def test_psi_solve_mixed_matches_fp64(mgpu):
    n, levels = 32, 3
    psi = psi_of(n)
    b = dev(mm_source(n, psi))
    out = {}
    for prec in ("fp64", "mixed"):
        mg = mgpu.Multigrid(n, levels=levels, psi=dev(psi), precision=prec)
        phi, info = mg.solve(b, tol=1e-12, max_cycles=60)
        assert info.rel_res <= 1e-12
        out[prec] = host(phi)
    assert rel(out["mixed"], out["fp64"]) <= 1e-10
    # the converged solution does not depend on how the coarse levels were built
    C = O.geometry(psi, 1.0 / n)[0]
    mg = mgpu.Multigrid(n, levels=levels, coeff=dev(C), precision="fp64")
    phi, info = mg.solve(b, tol=1e-12, max_cycles=60)
    assert rel(host(phi), out["fp64"]) <= 1e-10


def test_psi_folded_mesh_rejected(mgpu):
    """A potential that folds the mesh is an error, not a silently invalid
    hierarchy."""
    n = 16
    psi = 50.0 * PSI_SCALE[str(n)] * psi_unit(n)
    with pytest.raises(mgpu.MGError) as exc:
        mgpu.Multigrid(n, levels=2, psi=dev(psi), precision="fp64")
    assert exc.value.status == 2


# ------------------------------------------------ multigrid-preconditioned CG

@pytest.mark.parametrize("var", [False, True])
def test_pcg_fp64_matches_oracle(mgpu, var):
    n, levels = (32, 3) if var else (32, 4)
    C = None
    if var:
        psi = psi_of(n)
        C = O.geometry(psi, 1.0 / n)[0]
        b = mm_source(n, psi)
    else:
        b = flat_source(n)
    phi0 = RNG.standard_normal((n, n, n)) * 1e-3
    H = O.build_hierarchy(n, levels, C=C)
    ref = O.solve_pcg(H, b, phi0=phi0, tol=0.0, max_iter=6)
    mg = mgpu.Multigrid(n, levels=levels, coeff=dev(C) if var else None, precision="fp64")
    phi, info = mg.solve_pcg(dev(b), phi0=dev(phi0), tol=0.0, max_iter=6, raise_on_error=False)
    assert info.cycles == 6
    assert np.max(np.abs(np.array(info.history) - np.array(ref.history))) <= 1e-12
    assert rel(host(phi), ref.phi) <= 1e-12
    assert info.rel_res == pytest.approx(O.true_rel_residual(H, b, ref.phi), rel=1e-6)


@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp32"])
def test_pcg_reaches_exact(mgpu, prec):
    n = 64
    b = flat_source(n)
    exact = O.fft_solve(b - b.mean(), 1.0 / n)
    mg = mgpu.Multigrid(n, levels=5, degree=3, precision=prec)
    phi, info = mg.solve_pcg(dev(b), tol=1e-11, max_iter=40)
    assert info.rel_res <= 1e-11
    assert rel(host(phi), exact) <= 1e-10
    if prec != "fp32":   # the float32 defect correction stops at its plateau
        ir_phi, ir = mg.solve(dev(b), tol=1e-11, max_cycles=40)
        assert info.cycles <= ir.cycles


def test_pcg_mixed_moving_mesh(mgpu):
    n, levels = 32, 3
    psi = psi_of(n)
    b = dev(mm_source(n, psi))
    ref_mg = mgpu.Multigrid(n, levels=levels, psi=dev(psi), precision="fp64")
    ref, _ = ref_mg.solve(b, tol=1e-12, max_cycles=60)
    mg = mgpu.Multigrid(n, levels=levels, psi=dev(psi), precision="mixed")
    phi, info = mg.solve_pcg(b, tol=1e-12, max_iter=60)
    assert info.rel_res <= 1e-12
    assert rel(host(phi), host(ref)) <= 1e-10


def test_pcg_zero_source_and_warm_exact(mgpu):
    n = 16
    mg = mgpu.Multigrid(n, levels=3, precision="fp64")
    z = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    phi, info = mg.solve_pcg(z, phi0=torch.ones_like(z))
    assert info.cycles == 0 and info.rel_res == 0.0
    assert float(phi.abs().max()) == 0.0
    b = flat_source(n)
    exact = O.fft_solve(b - b.mean(), 1.0 / n)
    phi, info = mg.solve_pcg(dev(b), phi0=dev(exact), tol=1e-10)
    assert info.cycles == 0


# ------------------------------------------------ predictors

@pytest.mark.parametrize("kind", ["recycle", "growth", "linear", "quadratic"])
def test_predict(mgpu, kind):
    n = 32
    hist = [RNG.standard_normal((n, n, n)) for _ in range(3)]
    g = 1.0 + 0.05 / 1.3
    ref = O.predict(hist, kind, g)
    dh = [dev(h) for h in hist]
    out = host(mgpu.predict(kind, dh, growth=g))
    assert np.max(np.abs(out - ref)) <= 1e-14 * np.max(np.abs(ref))
    # in place over the newest solution
    mgpu.predict(kind, dh, growth=g, out=dh[0])
    assert np.max(np.abs(host(dh[0]) - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_predict_growth_beats_recycling(mgpu):
    """On the warm-start sequence rho_t = (1 + 0.05 t) delta + 0.02 t eta_t the
    growth-scaled guess removes the growing delta part exactly, so it starts
    closer than plain recycling (Sec. 3.2).  Polynomial extrapolation has no
    such advantage here (the eta_t are independent) and is only run."""
    n = 64
    seq = list(warm_sequence(n, 4))
    mg = mgpu.Multigrid(n, levels=5, precision="mixed")
    sols = []
    for t, rho in enumerate(seq):
        phi, _ = mg.solve(dev(rho), phi0=sols[-1] if sols else None, tol=1e-12, max_cycles=40)
        sols.append(phi)
    b = dev(seq[3])
    res0 = {}
    for kind, hist, g in (("recycle", [sols[2]], 1.0), ("growth", [sols[2]], 1.15 / 1.10),
                          ("linear", [sols[2], sols[1]], 1.0), ("quadratic", [sols[2], sols[1], sols[0]], 1.0)):
        guess = mgpu.predict(kind, hist, growth=g)
        _, info = mg.solve(b, phi0=guess, tol=1e-10, max_cycles=0, raise_on_error=False)
        res0[kind] = info.rel_res0
    assert res0["growth"] < 0.9 * res0["recycle"]
    assert all(math.isfinite(v) for v in res0.values())


# ------------------------------------------------ force readout

@pytest.mark.parametrize("n", [4, 8, 32, 64, 128, 256])
@pytest.mark.parametrize("curv", [False, True])
def test_accel(mgpu, n, curv):
    """Element-wise against the oracle: the column kernel below 64^3, the
    row-wave kernel (x-neighbours by lane rotation, z queue) from 64^3."""
    h = 1.0 / n
    phi = RNG.standard_normal((n, n, n))
    psi = None
    if curv:
        psi = psi_unit(n)
        psi *= 0.5 * (PSI_SCALE[str(n)] if str(n) in PSI_SCALE else O.admissible_scale(psi, h))
    ref = O.accel(phi, h, psi, 0.45)
    out = host(mgpu.accel(dev(phi), dev(psi) if curv else None, scale=0.45))
    assert np.max(np.abs(out - ref)) <= 1e-13 * np.max(np.abs(ref))
    out32 = host(mgpu.accel(dev(phi), dev(psi) if curv else None, scale=0.45, dtype=torch.float32))
    assert out32.dtype == np.float32
    assert np.max(np.abs(out32 - ref)) <= 1e-6 * np.max(np.abs(ref))


def test_accel_after_solve_flat(mgpu):
    """Force of the solved potential: fourth-order gradient of the GPU
    solution equals the oracle's gradient of the exact discrete solution."""
    n = 64
    b = flat_source(n)
    exact = O.fft_solve(b - b.mean(), 1.0 / n)
    mg = mgpu.Multigrid(n, levels=5, precision="mixed")
    phi, _ = mg.solve(dev(b), tol=1e-12, max_cycles=40)
    a = host(mgpu.accel(phi, scale=1.5 * 0.3))
    ref = O.accel(exact, 1.0 / n, None, 1.5 * 0.3)
    assert rel(a, ref) <= 1e-9
