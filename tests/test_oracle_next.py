"""Pins of the oracle's extensions beyond the core V-cycle: coarse operators
rebuilt from the restricted deformation potential, initial-guess predictors,
multigrid-preconditioned CG, and the force readout.

Each test checks the oracle against something other than itself: closed-form
Fourier symbols, exact reproduction of polynomial trajectories, the Krylov
optimality of CG computed from an explicit basis, and O(h^4) convergence to
the continuum derivative.
"""
import math

import numpy as np
import pytest

from oracle import mg_oracle as O
import workloads as W


def grid(n):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return x, y, z


def moving_psi(n, seed=1):
    """Deformation potential of the moving-mesh workload, scaled to 90% of the
    admissible amplitude (det J in [0.3, 3], J positive definite)."""
    psi = W.psi_unit(n, seed)
    return O.admissible_scale(psi, 1.0 / n) * 0.9 * psi


# ---------------------------------------------- coarse operators from psi (App. B)

def test_psi_hierarchy_flat_limit():
    """psi = 0: every level carries C = I, the hierarchy is the flat one."""
    n, L = 16, 3
    H = O.build_hierarchy(n, L, psi=np.zeros((n, n, n)))
    F = O.build_hierarchy(n, L)
    for lev in H.levels:
        np.testing.assert_array_equal(lev.C[:3], 1.0)
        np.testing.assert_array_equal(lev.C[3:], 0.0)
    b = W.grf(n, W.Spectrum(-1.0), 3)
    x = O.vcycle(H, 0, np.zeros_like(b), b)
    y = O.vcycle(F, 0, np.zeros_like(b), b)
    np.testing.assert_allclose(x, y, atol=1e-13 * np.abs(y).max())


def test_psi_hierarchy_level1_closed_form():
    """psi = eps cos(kx x + ky y): full weighting multiplies the mode by
    cos^2(kx h/2) cos^2(ky h/2); the level-1 Hessian at spacing H = 2h is
    -4 sin^2(k H/2)/H^2 on the diagonal and -sin(kx H) sin(ky H)/H^2 across,
    times the mode.  C = det(J) J^-2 is then written out for the 2x2 block."""
    n, mx, my, eps = 16, 1, 2, 2e-4
    h = 1.0 / n
    x, y, z = grid(n)
    kx, ky = 2 * np.pi * mx, 2 * np.pi * my
    psi = eps * np.cos(kx * x * h + ky * y * h)
    Hier = O.build_hierarchy(n, 2, psi=psi)
    C1 = Hier.levels[1].C
    Hc = 2 * h
    nc = n // 2
    X, Y, Z = grid(nc)
    amp = eps * math.cos(kx * h / 2) ** 2 * math.cos(ky * h / 2) ** 2
    mode = np.cos(kx * X * Hc + ky * Y * Hc)
    A = -amp * 4 * math.sin(kx * Hc / 2) ** 2 / Hc**2 * mode
    D = -amp * 4 * math.sin(ky * Hc / 2) ** 2 / Hc**2 * mode
    B = -amp * math.sin(kx * Hc) * math.sin(ky * Hc) / Hc**2 * mode
    det = (1 + A) * (1 + D) - B * B
    # J^-1 = [[1+D, -B], [-B, 1+A]] / det on the xy block; C = det J^-2
    cxx = ((1 + D) ** 2 + B * B) / det
    cyy = (B * B + (1 + A) ** 2) / det
    cxy = -B * ((1 + D) + (1 + A)) / det
    np.testing.assert_allclose(C1[0], cxx, rtol=1e-13)
    np.testing.assert_allclose(C1[1], cyy, rtol=1e-13)
    np.testing.assert_allclose(C1[2], det, rtol=1e-13)
    np.testing.assert_allclose(C1[3], cxy, atol=1e-14)
    np.testing.assert_array_equal(C1[4], 0.0)
    np.testing.assert_array_equal(C1[5], 0.0)


def test_psi_hierarchy_same_solution_as_fw_coefficients():
    """The coarse operators change only the convergence rate: solved to the
    rounding floor, both hierarchies give the same fine solution."""
    n, L = 16, 3
    psi = moving_psi(n)
    C, sg = O.geometry(psi, 1.0 / n)
    b = W.grf(n, W.Spectrum(-1.0), 5)
    Hp = O.build_hierarchy(n, L, psi=psi)
    Hc = O.build_hierarchy(n, L, C=C)
    np.testing.assert_array_equal(Hp.levels[0].C, C)
    sp = O.solve(Hp, b, tol=1e-13, max_cycles=60)
    sc = O.solve(Hc, b, tol=1e-13, max_cycles=60)
    assert sp.history[-1] <= 1e-13 and sc.history[-1] <= 1e-13
    np.testing.assert_allclose(sp.phi, sc.phi, atol=1e-11 * np.abs(sc.phi).max())
    # the rediscretised hierarchy converges (contraction well below one)
    rho = (sp.history[-1] / sp.history[0]) ** (1.0 / sp.cycles)
    assert rho < 0.35


@pytest.mark.parametrize("smoother", ["chebyshev", "jacobi"])
def test_psi_hierarchy_coarse_levels_are_spd(smoother):
    n, L = 16, 3
    H = O.build_hierarchy(n, L, psi=moving_psi(n), smoother=smoother)
    for lev in H.levels:
        S = O._to_mat(lev.C)
        assert np.linalg.eigvalsh(S.reshape(-1, 3, 3)).min() > 0


# ---------------------------------------------- predictors (Sec. 3.2)

def test_predictors_reproduce_their_trajectories():
    rng = np.random.default_rng(7)
    A, B, Cq = (rng.standard_normal((4, 4, 4)) for _ in range(3))
    lin = lambda t: A + B * t
    quad = lambda t: A + B * t + Cq * t * t
    t = 5
    np.testing.assert_allclose(O.predict([lin(t - 1), lin(t - 2)], "linear"), lin(t), atol=1e-13)
    np.testing.assert_allclose(O.predict([quad(t - 1), quad(t - 2), quad(t - 3)], "quadratic"),
                               quad(t), atol=1e-12)
    # linear extrapolation misses the quadratic drift by exactly C (second difference)
    np.testing.assert_allclose(quad(t) - O.predict([quad(t - 1), quad(t - 2)], "linear"),
                               2 * Cq, atol=1e-12)
    D = lambda t: 1.0 + 0.05 * t
    np.testing.assert_allclose(O.predict([D(t - 1) * A], "growth", D(t) / D(t - 1)), D(t) * A, rtol=1e-15)
    np.testing.assert_array_equal(O.predict([A], "recycle"), A)


# ---------------------------------------------- MG-preconditioned CG (Sec. 3.2)

def test_pcg_exact_preconditioner_one_iteration():
    """With a single level the V-cycle is the exact solve: one CG step."""
    n = 8
    H = O.build_hierarchy(n, 1)
    b = W.grf(n, W.Spectrum(-1.0), 1)
    res = O.solve_pcg(H, b, tol=1e-12)
    assert res.cycles == 1
    np.testing.assert_allclose(res.phi, O.fft_solve(b - b.mean(), 1.0 / n), atol=1e-12)


@pytest.mark.parametrize("var", [False, True])
def test_pcg_iterates_are_krylov_optimal(var):
    """Iterate k minimises the energy norm of the error over
    phi0 + span{B r0, (B M) B r0, ..., (B M)^{k-1} B r0}; computed here from an
    explicit orthonormal basis of that space and the exact dense solution."""
    n, L = 8, 2
    rng = np.random.default_rng(3)
    C = None
    if var:
        C = O.geometry(moving_psi(n), 1.0 / n)[0]
    H = O.build_hierarchy(n, L, C=C)
    lev = H.levels[0]
    A = -O.dense_from_apply(lev.apply, n)            # SPD on zero-mean fields
    b = W.grf(n, W.Spectrum(-1.0), 2)
    b = b - b.mean()
    phi_star = (np.linalg.pinv(A) @ -b.ravel()).reshape(b.shape)
    phi0 = rng.standard_normal(b.shape)
    phi0 -= phi0.mean()
    B = lambda r: O.vcycle(H, 0, np.zeros_like(r), r)
    r0 = b - lev.apply(phi0)
    vecs = [B(r0)]
    for k in range(1, 4):
        vecs.append(B(lev.apply(vecs[-1])))
    for k in range(1, 5):
        V, _ = np.linalg.qr(np.stack([v.ravel() for v in vecs[:k]], axis=1))
        e0 = (phi_star - phi0).ravel()
        y = np.linalg.solve(V.T @ A @ V, V.T @ A @ e0)
        best = phi0.ravel() + V @ y
        best -= best.mean()   # the variable-coefficient smoother does not keep the mean
        res = O.solve_pcg(H, b, phi0=phi0, tol=0.0, max_iter=k)
        assert res.cycles == k
        got = res.phi.ravel()
        err = lambda v: math.sqrt((v - phi_star.ravel()) @ A @ (v - phi_star.ravel()))
        assert abs(err(got) - err(best)) <= 1e-9 * err(phi0.ravel())
        np.testing.assert_allclose(got, best, atol=1e-9 * np.abs(phi_star).max())


def test_pcg_energy_error_decreases_and_reaches_fft():
    n, L = 16, 3
    H = O.build_hierarchy(n, L)
    b = W.grf(n, W.Spectrum(-1.0), 4)
    exact = O.fft_solve(b - b.mean(), 1.0 / n)
    res = O.solve_pcg(H, b, tol=1e-12)
    assert res.history[-1] <= 1e-12
    assert O.true_rel_residual(H, b, res.phi) <= 1.5e-12
    np.testing.assert_allclose(res.phi, exact, atol=1e-11 * np.abs(exact).max())
    lev = H.levels[0]
    errs = []
    for k in range(1, 6):
        e = O.solve_pcg(H, b, tol=0.0, max_iter=k).phi - exact
        errs.append(math.sqrt(-np.vdot(e, lev.apply(e))))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    # fewer iterations than plain V-cycles to the same tolerance
    assert res.cycles <= O.solve(H, b, tol=1e-12).cycles


# ---------------------------------------------- force readout (Sec. 3.4; eq. accel)

@pytest.mark.parametrize("m", [(1, 2, 3), (5, 0, 7), (8, 8, 1)])
def test_gradient4_fourier_symbol(m):
    """d/dx of cos(k.x) by the fourth-order difference is
    -(8 sin(k_a h) - sin(2 k_a h)) / (6 h) * sin(k.x) along direction a."""
    n = 16
    h = 1.0 / n
    x, y, z = grid(n)
    k = [2 * np.pi * mi for mi in m]
    arg = (k[0] * x + k[1] * y + k[2] * z) * h
    g = O.gradient4(np.cos(arg), h)
    for a in range(3):
        sym = (8 * math.sin(k[a] * h) - math.sin(2 * k[a] * h)) / (6 * h)
        np.testing.assert_allclose(g[a], -sym * np.sin(arg), atol=1e-12 * (abs(sym) + 1))


def test_gradient4_fourth_order_convergence():
    """Smooth periodic field: the error against the analytic gradient falls by
    16 per halving of h."""
    errs = []
    for n in (32, 64, 128):
        h = 1.0 / n
        x, y, z = (c * h for c in grid(n))
        tx, ty, tz = 2 * np.pi * x, 2 * np.pi * y, 2 * np.pi * z
        f = np.exp(np.sin(tx) + 0.5 * np.cos(ty)) * np.sin(tz)
        exact = [2 * np.pi * np.cos(tx) * f,
                 -np.pi * np.sin(ty) * f,
                 2 * np.pi * np.exp(np.sin(tx) + 0.5 * np.cos(ty)) * np.cos(tz)]
        g = O.gradient4(f, h)
        errs.append(max(np.abs(g[a] - exact[a]).max() for a in range(3)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 14.5 < r1 < 17.0 and 15.5 < r2 < 16.5, (r1, r2)


def test_accel_flat_and_curvilinear():
    n = 16
    h = 1.0 / n
    phi = W.grf(n, W.Spectrum(-2.0), 9)
    g = O.gradient4(phi, h)
    np.testing.assert_array_equal(O.accel(phi, h, None, 1.5), -1.5 * g)
    np.testing.assert_allclose(O.accel(phi, h, np.zeros_like(phi), 1.5), -1.5 * g, atol=1e-15)
    # curvilinear: J a = -s grad phi, checked by multiplying back
    psi = moving_psi(n)
    a = O.accel(phi, h, psi, 0.45)
    J = O.triad(psi, h)
    back = np.einsum("...ab,b...->a...", J, a)
    np.testing.assert_allclose(back, -0.45 * g, atol=1e-12 * np.abs(g).max())
    # psi varying along x only: J is diagonal with J_xx = 1 + d2psi/dx2
    x, _, _ = grid(n)
    kx = 2 * np.pi * 3
    psi1 = 1e-4 * np.cos(kx * x * h)
    a1 = O.accel(phi, h, psi1, 1.0)
    jxx = 1 - 1e-4 * 4 * math.sin(kx * h / 2) ** 2 / h**2 * np.cos(kx * x * h)
    np.testing.assert_allclose(a1[0], -g[0] / jxx, rtol=1e-12)
    np.testing.assert_allclose(a1[1], -g[1], rtol=1e-12)
    np.testing.assert_allclose(a1[2], -g[2], rtol=1e-12)
