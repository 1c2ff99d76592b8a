"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed-form
eigenvalues and Fourier symbols, an independently written table of matrix
entries, library routines (``numpy.polynomial.chebyshev``, ``eigh``), the
continuum operator (manufactured solutions, O(h^2) convergence), invariants
(symmetry, null space, homogeneity) and central finite differences.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import mg_oracle as O

RNG = np.random.default_rng(12345)


def fourier_mode(n, m):
    """cos(2 pi m . i / n) on the [z, y, x] grid, m = (mx, my, mz)."""
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return np.cos(2 * np.pi * (m[0] * x + m[1] * y + m[2] * z) / n)


def random_spd_field(n, amp=0.4, rng=RNG):
    """Random symmetric positive-definite 3x3 field in (xx,yy,zz,xy,xz,yz) storage."""
    A = amp * rng.standard_normal((n, n, n, 3, 3))
    S = np.eye(3) + A @ np.swapaxes(A, -1, -2)
    C = np.empty((6, n, n, n))
    idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for c, (a, b) in enumerate(idx):
        C[c] = S[..., a, b]
    return C


# ---------------------------------------------------------------- operators

@pytest.mark.parametrize("m", [(1, 0, 0), (1, 2, 3), (4, 4, 4), (7, 0, 5)])
def test_flat_eigen_on_fourier_mode(m):
    n, h = 16, 1.0 / 16
    u = fourier_mode(n, m)
    lam = -(4 / h**2) * sum(math.sin(math.pi * mi / n) ** 2 for mi in m)
    np.testing.assert_allclose(O.apply_flat(u, h), lam * u, atol=1e-14 * abs(lam) * 1.0 + 1e-9)


def test_flat_dense_spectrum_8():
    n, h = 8, 0.125
    A = O.dense_from_apply(lambda u: O.apply_flat(u, h), n)
    w = np.sort(np.linalg.eigvalsh(A))
    ms = np.arange(n)
    s = np.sin(np.pi * ms / n) ** 2
    closed = -(4 / h**2) * (s[:, None, None] + s[None, :, None] + s[None, None, :])
    np.testing.assert_allclose(w, np.sort(closed.ravel()), atol=1e-10 * 4 * 3 / h**2)


def test_var_reduces_to_flat_at_identity():
    n, h = 8, 0.3
    C = np.zeros((6, n, n, n))
    C[0] = C[1] = C[2] = 1.0
    u = RNG.standard_normal((n, n, n))
    np.testing.assert_allclose(O.apply_var(u, C, h), O.apply_flat(u, h), atol=1e-15 / h**2 * 10)


@pytest.mark.parametrize("m", [(1, 2, 3), (3, 1, 0), (2, 5, 7)])
def test_var_constant_anisotropic_symbol(m):
    n, h = 16, 1.0 / 16
    c = np.array([1.3, 0.7, 1.1, 0.2, -0.15, 0.1])
    C = c[:, None, None, None] * np.ones((6, n, n, n))
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    k = [2 * np.pi * mi / n for mi in m]            # k_a h
    u = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    sym = -sum(c[a] * 4 * math.sin(k[a] / 2) ** 2 for a in range(3))
    for (a, b, comp) in [(0, 1, 3), (0, 2, 4), (1, 2, 5)]:
        sym -= 2 * c[comp] * math.sin(k[a]) * math.sin(k[b])
    sym /= h * h
    out = O.apply_var(u.real, C, h) + 1j * O.apply_var(u.imag, C, h)
    np.testing.assert_allclose(out, sym * u, atol=1e-12 / h**2)


def dense_var_table(C, h):
    """Independent assembly of the 19-point matrix from its entry table.

    Row i: faces i +- e_a carry the face-averaged diagonal coefficient;
    edges i + sa e_a + sb e_b carry sa*sb*(C^{ab}_{i+sa e_a} + C^{ab}_{i+sb e_b})/(4h^2);
    the diagonal is minus the sum of the six face coefficients."""
    n = C.shape[1]
    N = n**3
    A = np.zeros((N, N))

    def idx(x, y, z):
        return ((z % n) * n + (y % n)) * n + (x % n)

    comp = {(0, 1): 3, (0, 2): 4, (1, 2): 5}
    for z in range(n):
        for y in range(n):
            for x in range(n):
                i = idx(x, y, z)
                p = [x, y, z]
                for a in range(3):
                    for s in (1, -1):
                        q = list(p)
                        q[a] += s
                        cf = 0.5 * (C[a][z, y, x] + C[a][q[2] % n, q[1] % n, q[0] % n])
                        A[i, idx(*q)] += cf / h**2
                        A[i, i] -= cf / h**2
                for (a, b), c in comp.items():
                    for sa in (1, -1):
                        for sb in (1, -1):
                            qa = list(p); qa[a] += sa
                            qb = list(p); qb[b] += sb
                            q = list(p); q[a] += sa; q[b] += sb
                            val = sa * sb * (C[c][qa[2] % n, qa[1] % n, qa[0] % n]
                                             + C[c][qb[2] % n, qb[1] % n, qb[0] % n]) / (4 * h * h)
                            A[i, idx(*q)] += val
    return A


def test_var_matches_independent_entry_table():
    n, h = 5, 0.7
    C = random_spd_field(n)
    A_tab = dense_var_table(C, h)
    A_mv = O.dense_from_apply(lambda u: O.apply_var(u, C, h), n)
    np.testing.assert_allclose(A_mv, A_tab, atol=1e-12 * np.abs(A_tab).max())
    # 19 nonzeros per row (n >= 3 keeps neighbours distinct)
    assert np.all((np.abs(A_tab) > 0).sum(axis=1) == 19)
    # diagonal and Gershgorin bound from the dense matrix
    np.testing.assert_allclose(O.diag_var(C, h).ravel(), np.diag(A_tab), rtol=1e-13)
    d = np.abs(np.diag(A_tab))
    g = np.max(1 + (np.abs(A_tab).sum(axis=1) - d) / d)
    assert abs(O.gershgorin_lmax_var(C, h) - g) < 1e-12 * g


def test_var_invariants_dense_8():
    n, h = 8, 1.0 / 8
    C = random_spd_field(n)
    A = O.dense_from_apply(lambda u: O.apply_var(u, C, h), n)
    scale = np.abs(A).max()
    assert np.abs(A - A.T).max() <= 1e-14 * scale
    w = np.linalg.eigvalsh(A)
    assert w.max() <= 1e-12 * scale                      # negative semidefinite
    assert np.sum(np.abs(w) <= 1e-10 * scale) == 1       # one-dimensional null space
    ones = np.ones(n**3)
    assert np.abs(A @ ones).max() <= 1e-13 * scale       # M 1 = 0
    u = RNG.standard_normal(n**3)
    assert abs((A @ u).sum()) <= 1e-12 * scale * np.abs(u).sum()   # sum(M u) = 0
    # Gershgorin really bounds the spectrum of D^-1 M
    Dinv = 1.0 / np.diag(A)
    mu = np.linalg.eigvals(Dinv[:, None] * A).real
    assert mu.max() <= O.gershgorin_lmax_var(C, h) + 1e-12


def _manufactured(n):
    """Trigonometric C (SPD) and phi; f = div(C grad phi) evaluated exactly on
    the grid by spectral differentiation (all fields are band-limited)."""
    h = 1.0 / n
    z, y, x = np.meshgrid(np.arange(n) * h, np.arange(n) * h, np.arange(n) * h, indexing="ij")
    tp = 2 * np.pi
    phi = np.sin(tp * x) * np.cos(tp * y) + 0.5 * np.sin(tp * (x + 2 * z)) + 0.3 * np.cos(tp * (y - z))
    C = np.empty((6, n, n, n))
    C[0] = 1.5 + 0.3 * np.sin(tp * y)
    C[1] = 1.2 + 0.2 * np.cos(tp * (x + z))
    C[2] = 1.0 + 0.25 * np.sin(tp * x) * np.cos(tp * y)
    C[3] = 0.2 * np.cos(tp * z)
    C[4] = 0.15 * np.sin(tp * (x - y))
    C[5] = -0.1 * np.cos(tp * x)
    k = tp * np.fft.fftfreq(n, d=h)

    def deriv(u, a):
        ax = O.AXIS[a]
        shape = [1, 1, 1]
        shape[ax] = n
        return np.fft.ifftn(1j * k.reshape(shape) * np.fft.fftn(u)).real

    grads = [deriv(phi, b) for b in range(3)]
    f = np.zeros_like(phi)
    for a in range(3):
        flux = sum(C[O.COMP[(a, b)]] * grads[b] for b in range(3))
        f += deriv(flux, a)
    return phi, C, f, h


def test_var_manufactured_second_order():
    errs = []
    for n in (16, 32, 64):
        phi, C, f, h = _manufactured(n)
        errs.append(np.abs(O.apply_var(phi, C, h) - f).max() / np.abs(f).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.7 < r2 < 4.3, errs


def test_var_manufactured_solution_converges():
    errs = []
    for n in (16, 32):
        phi, C, f, h = _manufactured(n)
        H = O.build_hierarchy(n, int(math.log2(n)) - 1, 3, h, C)
        res = O.solve(H, f, tol=1e-13, max_cycles=60)
        ref = phi - phi.mean()
        errs.append(np.abs(res.phi - ref).max() / np.abs(ref).max())
    assert 3.3 < errs[0] / errs[1] < 4.7, errs


# ---------------------------------------------------------------- smoothers

@pytest.mark.parametrize("v", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("m", [(1, 0, 0), (3, 2, 1), (8, 8, 8), (5, 7, 2)])
def test_chebyshev_error_polynomial(v, m):
    n, h = 16, 1.0 / 16
    u = fourier_mode(n, m)
    lam = -(4 / h**2) * sum(math.sin(math.pi * mi / n) ** 2 for mi in m)
    mu = lam / O.diag_flat(n, h)                      # eigenvalue of D^-1 M
    cc = O.cheb_coeffs(2.0, 8.0)
    out = O.chebyshev(u, np.zeros_like(u), lambda w: O.apply_flat(w, h),
                      1.0 / O.diag_flat(n, h), cc, v)
    Tv = np.zeros(v + 1)
    Tv[v] = 1.0
    factor = npcheb.chebval((cc.theta - mu) / cc.delta, Tv) / npcheb.chebval(cc.sigma, Tv)
    np.testing.assert_allclose(out, factor * u, atol=1e-13)


def test_chebyshev_interval_is_paper_interval():
    cc = O.cheb_coeffs(2.0, 8.0)
    assert cc.theta - cc.delta == pytest.approx(2.0 / 8.0)
    assert cc.theta + cc.delta == pytest.approx(2.0)


@pytest.mark.parametrize("m", [(1, 0, 0), (8, 8, 8), (3, 5, 1)])
def test_jacobi_damping(m):
    n, h = 16, 1.0 / 16
    u = fourier_mode(n, m)
    lam = -(4 / h**2) * sum(math.sin(math.pi * mi / n) ** 2 for mi in m)
    mu = lam / O.diag_flat(n, h)
    out = O.jacobi(u, np.zeros_like(u), lambda w: O.apply_flat(w, h), 1.0 / O.diag_flat(n, h), 2 / 3, 2)
    np.testing.assert_allclose(out, (1 - 2 / 3 * mu) ** 2 * u, atol=1e-13)


# ---------------------------------------------------------------- transfers

def test_transfer_adjoint_and_constants():
    nc = 4
    n = 2 * nc
    R = np.empty((nc**3, n**3))
    e = np.zeros(n**3)
    for j in range(n**3):
        e[j] = 1
        R[:, j] = O.restrict_fw(e.reshape(n, n, n)).ravel()
        e[j] = 0
    P = np.empty((n**3, nc**3))
    e = np.zeros(nc**3)
    for j in range(nc**3):
        e[j] = 1
        P[:, j] = O.prolong(e.reshape(nc, nc, nc)).ravel()
        e[j] = 0
    np.testing.assert_allclose(P, 8 * R.T, atol=1e-15)
    np.testing.assert_allclose(R @ np.ones(n**3), 1.0, atol=1e-15)
    np.testing.assert_allclose(P @ np.ones(nc**3), 1.0, atol=1e-15)
    assert np.all((R > 0).sum(axis=1) == 27)


@pytest.mark.parametrize("m", [(1, 0, 0), (2, 3, 1), (5, 0, 7)])
def test_full_weighting_symbol(m):
    n = 16
    u = fourier_mode(n, m)
    sym = np.prod([math.cos(math.pi * mi / n) ** 2 for mi in m])
    np.testing.assert_allclose(O.restrict_fw(u), sym * u[::2, ::2, ::2], atol=1e-14)


def test_prolong_trilinear_exact_on_linear_profile():
    # trilinear interpolation reproduces a linear function away from the wrap
    nc = 8
    Z, Y, X = np.meshgrid(np.arange(nc), np.arange(nc), np.arange(nc), indexing="ij")
    e = 1.0 * X + 2.0 * Y - 0.5 * Z
    f = O.prolong(e)
    z, y, x = np.meshgrid(np.arange(2 * nc), np.arange(2 * nc), np.arange(2 * nc), indexing="ij")
    ref = (1.0 * x + 2.0 * y - 0.5 * z) / 2
    inner = (x < 2 * nc - 1) & (y < 2 * nc - 1) & (z < 2 * nc - 1)
    np.testing.assert_allclose(f[inner], ref[inner], atol=1e-14)


# ---------------------------------------------------------------- exact solves

def test_fft_solve_is_exact():
    n, h = 16, 1.0 / 16
    b = RNG.standard_normal((n, n, n))
    b -= b.mean()
    x = O.fft_solve(b, h)
    assert abs(x.mean()) < 1e-14
    np.testing.assert_allclose(O.apply_flat(x, h), b, atol=1e-11 * np.abs(b).max())


def test_coarse_solve_flat_equals_dense_pinv():
    n, h = 4, 0.25
    H = O.build_hierarchy(n, 1, 3, h)
    r = RNG.standard_normal((n, n, n))
    A = O.dense_from_apply(lambda u: O.apply_flat(u, h), n)
    ref = np.linalg.lstsq(A, r.ravel() - r.mean(), rcond=None)[0]
    np.testing.assert_allclose(O.coarse_solve(H.levels[0], r).ravel(), ref, atol=1e-13)


def test_coarse_solve_var_equals_lstsq():
    n, h = 4, 0.5
    C = random_spd_field(n)
    H = O.build_hierarchy(n, 1, 3, h, C)
    r = RNG.standard_normal((n, n, n))
    A = dense_var_table(C, h)
    ref = np.linalg.lstsq(A, r.ravel() - r.mean(), rcond=None)[0]
    out = O.coarse_solve(H.levels[0], r).ravel()
    np.testing.assert_allclose(out, ref, atol=1e-12 * np.abs(ref).max())
    assert abs(out.mean()) < 1e-13


# ---------------------------------------------------------------- V-cycle / solve

def _vcycle_error_matrix(H, n):
    N = n**3
    E = np.empty((N, N))
    e = np.zeros(N)
    for j in range(N):
        e[j] = 1
        E[:, j] = O.vcycle(H, 0, e.reshape(n, n, n), np.zeros((n, n, n))).ravel()
        e[j] = 0
    return E


@pytest.mark.parametrize("var", [False, True])
def test_vcycle_is_symmetric_and_contracting(var):
    n, h = 8, 1.0 / 8
    C = random_spd_field(n, 0.3) if var else None
    H = O.build_hierarchy(n, 2, 3, h, C)
    E = _vcycle_error_matrix(H, n)
    A = O.dense_from_apply(H.levels[0].apply, n)
    ME = A @ E
    assert np.abs(ME - ME.T).max() <= 1e-9 * np.abs(ME).max()   # M-self-adjoint cycle
    Pi = np.eye(n**3) - 1.0 / n**3
    rho = np.max(np.abs(np.linalg.eigvals(Pi @ E @ Pi)))
    assert rho < 0.5


def test_contraction_factor_order_0p1():
    # The paper quotes rho ~ 0.1 for a well-tuned cycle on the model problem.
    n = 32
    from workloads import flat_source
    b = flat_source(n, 0)
    H = O.build_hierarchy(n, 4, 3)
    res = O.solve(H, b, tol=1e-30, max_cycles=8)
    hist = np.array(res.history)
    rates = hist[3:] / hist[2:-1]
    assert 0.03 < np.median(rates) < 0.2, rates


def test_solve_flat_reaches_fft_solution():
    n = 32
    from workloads import flat_source
    b = flat_source(n, 0)
    H = O.build_hierarchy(n, 4, 3)
    res = O.solve(H, b, tol=1e-13, max_cycles=40)
    ref = O.fft_solve(b - b.mean(), 1.0 / n)
    assert np.linalg.norm(res.phi - ref) / np.linalg.norm(ref) < 1e-12
    assert res.history[-1] <= 1e-13


def test_solve_var_reaches_dense_solution_and_ignores_guess():
    n, h = 8, 1.0 / 8
    C = random_spd_field(n, 0.3)
    H = O.build_hierarchy(n, 2, 3, h, C)
    b = RNG.standard_normal((n, n, n))
    A = dense_var_table(C, h)
    ref = np.linalg.lstsq(A, b.ravel() - b.mean(), rcond=None)[0].reshape(n, n, n)
    r1 = O.solve(H, b, tol=1e-14, max_cycles=200)
    r2 = O.solve(H, b, phi0=RNG.standard_normal((n, n, n)), tol=1e-14, max_cycles=200)
    for r in (r1, r2):
        assert np.linalg.norm(r.phi - ref) / np.linalg.norm(ref) < 1e-12


def test_warm_start_saves_cycles():
    n = 32
    from workloads import flat_source
    b0 = flat_source(n, 0)
    b1 = b0 + 0.02 * flat_source(n, 7)
    H = O.build_hierarchy(n, 4, 3)
    p0 = O.solve(H, b0, tol=1e-10).phi
    cold = O.solve(H, b1, tol=1e-10)
    warm = O.solve(H, b1, phi0=p0, tol=1e-10)
    assert warm.cycles < cold.cycles
    assert warm.history[0] < 0.1


def test_zero_source():
    H = O.build_hierarchy(8, 2, 3)
    r = O.solve(H, np.full((8, 8, 8), 3.0))
    assert r.cycles == 0 and np.all(r.phi == 0)


# ---------------------------------------------------------------- adjoint / gradients

def _exact_solver(C, h, n):
    A = dense_var_table(C, h)
    Ap = np.linalg.pinv(A, rcond=1e-10)
    return lambda b: (Ap @ (b.ravel() - b.mean())).reshape(n, n, n)


def test_adjoint_solve_map_symmetry_and_homogeneity():
    n, h = 8, 1.0 / 8
    C = random_spd_field(n, 0.3)
    H = O.build_hierarchy(n, 2, 3, h, C)
    b = RNG.standard_normal((n, n, n))
    w = RNG.standard_normal((n, n, n))
    Sb = O.solve(H, b, tol=1e-14, max_cycles=200).phi
    Sw = O.solve_adjoint(H, w, tol=1e-14, max_cycles=200).phi
    assert abs(np.vdot(w, Sb) - np.vdot(Sw, b)) < 1e-12 * np.linalg.norm(w) * np.linalg.norm(Sb)
    L = np.vdot(w, Sb)
    assert abs(np.vdot(b, Sw) - L) < 1e-12 * abs(L) * 10


def test_coeff_grad_fd_and_homogeneity():
    n, h = 5, 0.6
    C = random_spd_field(n, 0.3)
    b = RNG.standard_normal((n, n, n))
    w = RNG.standard_normal((n, n, n))
    S = _exact_solver(C, h, n)
    phi = S(b)
    lam = S(w)
    L = np.vdot(w, phi)
    G = O.coeff_grad(lam, phi, h)
    # homogeneity: phi(s C) = phi(C)/s  =>  <C, dL/dC> = -L
    assert abs(np.vdot(C, G) + L) < 1e-11 * abs(L)
    eps = 1e-6
    for k in range(4):
        d = RNG.standard_normal(C.shape)
        Lp = np.vdot(w, _exact_solver(C + eps * d, h, n)(b))
        Lm = np.vdot(w, _exact_solver(C - eps * d, h, n)(b))
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - np.vdot(G, d)) < 1e-6 * abs(fd), (fd, np.vdot(G, d))


# ---------------------------------------------------------------- geometry

def test_geometry_identity():
    n = 8
    C, sg = O.geometry(np.zeros((n, n, n)), 1.0 / n)
    np.testing.assert_allclose(sg, 1.0, atol=0)
    np.testing.assert_allclose(C[:3], 1.0, atol=1e-15)
    np.testing.assert_allclose(C[3:], 0.0, atol=1e-15)


@pytest.mark.parametrize("m", [(1, 2, 0), (3, 1, 2)])
def test_hessian_symbols(m):
    n, h = 16, 1.0 / 16
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    k = [2 * np.pi * mi / n for mi in m]
    u = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    Hr, Hi = O.hessian(u.real, h), O.hessian(u.imag, h)
    Hc = Hr + 1j * Hi
    for a in range(3):
        np.testing.assert_allclose(Hc[a], -4 * math.sin(k[a] / 2) ** 2 / h**2 * u, atol=1e-10)
    for (a, b, c) in [(0, 1, 3), (0, 2, 4), (1, 2, 5)]:
        np.testing.assert_allclose(Hc[c], -math.sin(k[a]) * math.sin(k[b]) / h**2 * u, atol=1e-10)


def test_hessian_self_adjoint():
    n, h = 6, 0.4
    u = RNG.standard_normal((6, n, n, n))
    v = RNG.standard_normal((6, n, n, n))
    a = np.sum(O.hessian_components(u, h) * v, axis=(1, 2, 3))
    b = np.sum(u * O.hessian_components(v, h), axis=(1, 2, 3))
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_geometry_linearisation_at_identity():
    # C(J) = det(J) J^-2 for symmetric J; at J = I + t dJ:  dC/dt = tr(dJ) I - 2 dJ
    n, h = 6, 1.0 / 6
    psi = RNG.standard_normal((n, n, n)) * 1e-3
    t = 1e-4
    Hs = O.hessian(psi, h)
    Cp, sp = O.geometry(t * psi, h)
    Cm, sm = O.geometry(-t * psi, h)
    dC = (Cp - Cm) / (2 * t)
    tr = Hs[0] + Hs[1] + Hs[2]
    for a in range(3):
        np.testing.assert_allclose(dC[a], tr - 2 * Hs[a], rtol=1e-6, atol=1e-8 * np.abs(Hs).max())
    for c in range(3, 6):
        np.testing.assert_allclose(dC[c], -2 * Hs[c], rtol=1e-6, atol=1e-8 * np.abs(Hs).max())
    np.testing.assert_allclose((sp - sm) / (2 * t), tr, rtol=1e-6, atol=1e-8 * np.abs(Hs).max())


def test_geometry_values_against_matrix_inverse():
    # C = det(J) (J^T J)^-1 assembled directly from the Hessian components
    n, h = 4, 0.5
    psi = 0.02 * RNG.standard_normal((n, n, n))
    C, sg = O.geometry(psi, h)
    Hs = O.hessian(psi, h)
    for (z, y, x) in [(0, 0, 0), (1, 2, 3), (3, 3, 1)]:
        J = np.eye(3)
        J[0, 0] += Hs[0][z, y, x]; J[1, 1] += Hs[1][z, y, x]; J[2, 2] += Hs[2][z, y, x]
        J[0, 1] = J[1, 0] = Hs[3][z, y, x]
        J[0, 2] = J[2, 0] = Hs[4][z, y, x]
        J[1, 2] = J[2, 1] = Hs[5][z, y, x]
        d = np.linalg.det(J)
        Cm = d * np.linalg.inv(J.T @ J)
        assert sg[z, y, x] == pytest.approx(d, rel=1e-14)
        got = [C[c][z, y, x] for c in range(6)]
        want = [Cm[0, 0], Cm[1, 1], Cm[2, 2], Cm[0, 1], Cm[0, 2], Cm[1, 2]]
        np.testing.assert_allclose(got, want, rtol=1e-13)


def test_geometry_bwd_matches_fd():
    n, h = 6, 1.0 / 6
    psi = 0.001 * RNG.standard_normal((n, n, n))       # admissible: lambda_min(J) ~ 0.6
    assert np.linalg.eigvalsh(O.triad(psi, h).reshape(-1, 3, 3)).min() > 0.3
    Cbar = RNG.standard_normal((6, n, n, n))
    sbar = RNG.standard_normal((n, n, n))
    pbar = O.geometry_bwd(psi, Cbar, sbar, h)
    eps = 1e-7
    for _ in range(3):
        d = RNG.standard_normal((n, n, n))
        Cp, sp = O.geometry(psi + eps * d, h)
        Cm, sm = O.geometry(psi - eps * d, h)
        fd = (np.vdot(Cbar, Cp - Cm) + np.vdot(sbar, sp - sm)) / (2 * eps)
        assert abs(fd - np.vdot(pbar, d)) < 1e-7 * abs(fd)


def test_admissible_scale():
    n = 16
    from workloads import psi_unit
    psi = psi_unit(n)
    h = 1.0 / n
    s = O.admissible_scale(psi, h)
    for ss, expect in ((s, True), (s * 1.001, False)):
        J = O.triad(ss * psi, h)
        lam = np.linalg.eigvalsh(J.reshape(-1, 3, 3))
        det = lam.prod(axis=1)
        good = lam.min() > 0 and det.min() >= 0.3 - 1e-12 and det.max() <= 3.0 + 1e-12
        assert good == expect
