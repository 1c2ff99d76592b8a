"""Plain, slow CPU float64 oracle of the geometric-multigrid method.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this module.  It shares no code with the HIP library and
imports nothing from it.  Everything here is plain NumPy in float64, with
periodic shifts written as ``numpy.roll`` so each formula can be read against
the paper by eye.

Conventions
-----------
* A field is a float64 array of shape ``(n, n, n)`` indexed ``[z, y, x]``
  (C order, x fastest).  Component ``a`` of a direction (0 = x, 1 = y,
  2 = z) is array axis ``AXIS[a]``.
* Box length ``n * h``; coarse level ``l`` has ``n >> l`` points and spacing
  ``h * 2**l``; coarse point ``I`` sits on fine point ``2 I`` (vertex centred).
* The symmetric coefficient tensor ``C`` is stored as ``(6, n, n, n)`` with
  components ordered ``(xx, yy, zz, xy, xz, yz)``.  ``C`` plays the role of the
  paper's ``sqrt(g) g^{ab}`` (Sec. 4.3.1).
* The operator ``M`` is negative semidefinite with the constants as its null
  space, and the library solves ``M phi = b`` directly (Sec. 2.1, eq. linsys).

Readings of the paper taken here (listed with the reasons in the design notes):
* cross terms average the tangential *flux* ``C^{ab} D0_b u`` onto the faces,
  giving ``D0_a (C^{ab} D0_b u)``: symmetric, negative semidefinite, 19 points,
  and exactly the 7-point Laplacian at ``C = I`` (Sec. 4.3.1 states these
  properties; averaging only the derivative would break the symmetry);
* face values of diagonal coefficients are the mean of the two cells (App. B);
* the symmetric form ``M phi = b`` is solved (no ``1/sqrt(g)`` prefactor);
  the paper's form maps onto it by ``b = sqrt(g) f`` (eq. curv_operator);
* Chebyshev degree ``v`` = ``v`` operator applications, interval
  ``[lmax/alpha, lmax]`` with ``lmax`` the Gershgorin bound of ``D^-1 M``
  (exactly 2 for the 7-point operator, the paper's interval [2/alpha, 2]);
* pre- and post-smoothing use the same polynomial;
* coarse coefficients are the full-weighting restriction of ``C``;
* the coarsest level is solved exactly (zero-mean pseudo-inverse).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

AXIS = (2, 1, 0)                       # direction a -> array axis
PAIRS = ((0, 1, 3), (0, 2, 4), (1, 2, 5))   # (a, b, component) for a < b
COMP = {}
for _a in range(3):
    COMP[(_a, _a)] = _a
for _a, _b, _c in PAIRS:
    COMP[(_a, _b)] = _c
    COMP[(_b, _a)] = _c


def _sh(u: np.ndarray, a: int, s: int) -> np.ndarray:
    """``out[i] = u[i + s e_a]`` (periodic)."""
    return np.roll(u, -s, axis=AXIS[a])


# ---------------------------------------------------------------------------
# Operators (Sec. 2.3: seven-point Laplacian; Sec. 4.3.1: flux-form operator)
# ---------------------------------------------------------------------------

def apply_flat(u: np.ndarray, h: float) -> np.ndarray:
    """Seven-point periodic Laplacian ``(sum_a u_{i+e_a} + u_{i-e_a} - 6 u_i) / h^2``."""
    out = -6.0 * u
    for a in range(3):
        out = out + _sh(u, a, 1) + _sh(u, a, -1)
    return out / (h * h)


def face_coeff(C: np.ndarray, a: int) -> np.ndarray:
    """``C^{aa}`` on the face ``i + 1/2 e_a``: mean of the two adjacent cells."""
    c = C[a]
    return 0.5 * (c + _sh(c, a, 1))


def apply_var(u: np.ndarray, C: np.ndarray, h: float) -> np.ndarray:
    """Flux-form operator ``div(C grad u)``.

    Normal flux on the ``a``-face: face coefficient times the compact
    two-point difference; divergence of the face fluxes.  Cross terms:
    ``D0_a (C^{ab} D0_b u)`` for every ordered pair ``a != b``.
    """
    out = np.zeros_like(u)
    for a in range(3):
        flux = face_coeff(C, a) * (_sh(u, a, 1) - u) / h          # at i + 1/2
        out = out + (flux - _sh(flux, a, -1)) / h
    for a in range(3):
        for b in range(3):
            if a == b:
                continue
            g = C[COMP[(a, b)]] * (_sh(u, b, 1) - _sh(u, b, -1)) / (2.0 * h)
            out = out + (_sh(g, a, 1) - _sh(g, a, -1)) / (2.0 * h)
    return out


def diag_flat(n: int, h: float) -> float:
    return -6.0 / (h * h)


def diag_var(C: np.ndarray, h: float) -> np.ndarray:
    """Diagonal of the flux-form operator: minus the sum of the six face
    coefficients over ``h^2`` (App. B, without the ``1/sqrt(g)`` factor);
    cross terms do not touch the diagonal."""
    d = np.zeros(C.shape[1:])
    for a in range(3):
        cf = face_coeff(C, a)
        d = d - (cf + _sh(cf, a, -1))
    return d / (h * h)


def gershgorin_lmax_var(C: np.ndarray, h: float) -> float:
    """Gershgorin upper bound of the spectrum of ``D^-1 M``:
    ``max_i (1 + sum_{j != i} |M_ij| / |M_ii|)`` (App. C, eq. gersh, applied
    to the row of ``D^-1 M``)."""
    face = np.zeros(C.shape[1:])
    for a in range(3):
        cf = face_coeff(C, a)
        face = face + cf + _sh(cf, a, -1)
    edge = np.zeros(C.shape[1:])
    for a, b, c in PAIRS:
        cab = C[c]
        for sa in (1, -1):
            for sb in (1, -1):
                # entry at i + sa e_a + sb e_b collects the ordered pairs (a,b)
                # and (b,a): sa*sb*(C_{i+sa e_a} + C_{i+sb e_b}) / (4 h^2)
                edge = edge + np.abs(_sh(cab, a, sa) + _sh(cab, b, sb)) / 4.0
    return float(np.max(1.0 + (face + edge) / face))


# ---------------------------------------------------------------------------
# Chebyshev smoother (Sec. 2.3, eq. flat_chebyshev)
# ---------------------------------------------------------------------------

@dataclass
class ChebCoeffs:
    lmax: float
    alpha: float
    theta: float
    delta: float
    sigma: float


def cheb_coeffs(lmax: float, alpha: float) -> ChebCoeffs:
    lmin = lmax / alpha
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    return ChebCoeffs(lmax, alpha, theta, delta, theta / delta)


def chebyshev(x, b, apply, dinv, cc: ChebCoeffs, v: int):
    """Degree-``v`` Chebyshev acceleration of Jacobi: ``v`` applications of the
    operator, the error polynomial is ``T_v((theta - mu)/delta) / T_v(sigma)``
    on each eigenvalue ``mu`` of ``D^-1 M`` (three-term recurrence of Saad,
    Iterative Methods for Sparse Linear Systems, Alg. 12.1)."""
    rho = 1.0 / cc.sigma
    z = dinv * (b - apply(x))
    d = z / cc.theta
    x = x + d
    for _ in range(1, v):
        rho_new = 1.0 / (2.0 * cc.sigma - rho)
        z = dinv * (b - apply(x))
        d = rho_new * rho * d + (2.0 * rho_new / cc.delta) * z
        x = x + d
        rho = rho_new
    return x


def jacobi(x, b, apply, dinv, omega: float, sweeps: int):
    """Weighted Jacobi ``x += omega D^-1 (b - M x)`` (eq. flat_jacobi / eq. jacobi)."""
    for _ in range(sweeps):
        x = x + omega * dinv * (b - apply(x))
    return x


# ---------------------------------------------------------------------------
# Grid transfers (Sec. 2.3; App. B)
# ---------------------------------------------------------------------------

def restrict_fw(r: np.ndarray) -> np.ndarray:
    """Full weighting: ``[1/4, 1/2, 1/4]`` along each axis, then keep every
    second point (coarse ``I`` <- fine ``2 I``)."""
    t = r
    for ax in range(3):
        t = 0.25 * np.roll(t, 1, axis=ax) + 0.5 * t + 0.25 * np.roll(t, -1, axis=ax)
    return np.ascontiguousarray(t[::2, ::2, ::2])


def _prolong_axis(a: np.ndarray, ax: int) -> np.ndarray:
    n = a.shape[ax]
    shape = list(a.shape)
    shape[ax] = 2 * n
    out = np.empty(shape)
    even = [slice(None)] * 3
    odd = [slice(None)] * 3
    even[ax] = slice(0, 2 * n, 2)
    odd[ax] = slice(1, 2 * n, 2)
    out[tuple(even)] = a
    out[tuple(odd)] = 0.5 * (a + np.roll(a, -1, axis=ax))
    return out


def prolong(e: np.ndarray) -> np.ndarray:
    """Trilinear interpolation: fine ``2 I`` copies coarse ``I``; a fine point
    between two coarse points along an axis takes their mean, axis by axis."""
    t = e
    for ax in range(3):
        t = _prolong_axis(t, ax)
    return t


# ---------------------------------------------------------------------------
# Exact solves (eq. fftsolve; coarsest level)
# ---------------------------------------------------------------------------

def flat_eigenvalues(n: int, h: float) -> np.ndarray:
    """``lambda(k) = -(4/h^2) sum_i sin^2(k_i h / 2)`` on the rfftn grid (eq. fftsolve)."""
    m = np.fft.fftfreq(n, d=1.0 / n)
    mr = np.fft.rfftfreq(n, d=1.0 / n)
    s = lambda mm: np.sin(math.pi * mm / n) ** 2          # sin^2(k h / 2), k h = 2 pi m / n
    return -(4.0 / (h * h)) * (s(m)[:, None, None] + s(m)[None, :, None] + s(mr)[None, None, :])


def fft_solve(b: np.ndarray, h: float, workers: int = 1) -> np.ndarray:
    """Exact zero-mean solution of the seven-point system by FFT diagonalisation
    (``workers`` threads for the library FFT on large grids)."""
    import scipy.fft as sfft

    n = b.shape[0]
    lam = flat_eigenvalues(n, h)
    B = sfft.rfftn(b, workers=workers)
    lam[0, 0, 0] = 1.0
    B /= lam
    B[0, 0, 0] = 0.0
    del lam
    return sfft.irfftn(B, s=b.shape, axes=(0, 1, 2), workers=workers)


def dense_from_apply(apply, n: int) -> np.ndarray:
    """Matrix of a linear map on ``n^3`` fields, column by column."""
    N = n ** 3
    A = np.empty((N, N))
    e = np.zeros(N)
    for j in range(N):
        e[j] = 1.0
        A[:, j] = apply(e.reshape(n, n, n)).ravel()
        e[j] = 0.0
    return A


def pinv_symmetric(A: np.ndarray) -> np.ndarray:
    """Pseudo-inverse of a symmetric matrix through its eigendecomposition."""
    w, V = np.linalg.eigh(0.5 * (A + A.T))
    tol = 1e-10 * np.max(np.abs(w))
    winv = np.where(np.abs(w) > tol, 1.0 / np.where(np.abs(w) > tol, w, 1.0), 0.0)
    return (V * winv) @ V.T


# ---------------------------------------------------------------------------
# Hierarchy, V-cycle and solve (Sec. 2.3; Sec. 3.1; Sec. 4.3)
# ---------------------------------------------------------------------------

@dataclass
class Level:
    n: int
    h: float
    C: Optional[np.ndarray]
    dinv: object
    cheb: Optional[ChebCoeffs]
    coarse_pinv: Optional[np.ndarray] = None

    def apply(self, u):
        if self.C is None:
            return apply_flat(u, self.h)
        return apply_var(u, self.C, self.h)


@dataclass
class Hierarchy:
    levels: List[Level]
    degree: int
    alpha: float
    smoother: str = "chebyshev"
    omega: float = 2.0 / 3.0
    sweeps: int = 2


def build_hierarchy(n: int, levels: int, degree: int = 3, h: Optional[float] = None,
                    C: Optional[np.ndarray] = None, alpha: float = 8.0,
                    smoother: str = "chebyshev", omega: float = 2.0 / 3.0,
                    sweeps: int = 2, psi: Optional[np.ndarray] = None) -> Hierarchy:
    """Levels ``0..levels-1``; the coefficients of level ``l+1`` are the
    full-weighting restriction of those of level ``l`` (componentwise).

    With ``psi`` (and no ``C``) every level is instead rediscretised from the
    deformation potential restricted to it (Sec. 4.3; App. B):
    ``psi_0 = psi``, ``psi_{l+1} = R psi_l`` and ``C_l = geometry(psi_l, h_l)``."""
    if h is None:
        h = 1.0 / n
    if n >> (levels - 1) < 2:
        raise ValueError("too many levels")
    if psi is not None and C is not None:
        raise ValueError("give C or psi, not both")
    out = []
    psil = None if psi is None else np.asarray(psi, dtype=np.float64)
    Cl = None if C is None else np.asarray(C, dtype=np.float64)
    if psil is not None:
        Cl = geometry(psil, h)[0]
    for l in range(levels):
        nl = n >> l
        hl = h * (1 << l)
        if Cl is None:
            dinv = 1.0 / diag_flat(nl, hl)
            lmax = 2.0
        else:
            dinv = 1.0 / diag_var(Cl, hl)
            lmax = gershgorin_lmax_var(Cl, hl)
        lev = Level(nl, hl, Cl, dinv, cheb_coeffs(lmax, alpha))
        if l == levels - 1 and Cl is not None:
            lev.coarse_pinv = pinv_symmetric(dense_from_apply(lev.apply, nl))
        out.append(lev)
        if l + 1 < levels and psil is not None:
            psil = restrict_fw(psil)
            Cl = geometry(psil, hl * 2.0)[0]
        elif Cl is not None and l + 1 < levels:
            Cl = np.stack([restrict_fw(Cl[c]) for c in range(6)])
    return Hierarchy(out, degree, alpha, smoother, omega, sweeps)


def coarse_solve(lev: Level, r: np.ndarray) -> np.ndarray:
    """Exact zero-mean solution on the coarsest level (the paper solves the
    coarsest level directly)."""
    if lev.C is None:
        return fft_solve(r - r.mean(), lev.h)
    return (lev.coarse_pinv @ r.ravel()).reshape(r.shape)


def smooth(H: Hierarchy, lev: Level, x, b):
    if H.smoother == "jacobi":
        return jacobi(x, b, lev.apply, lev.dinv, H.omega, H.sweeps)
    return chebyshev(x, b, lev.apply, lev.dinv, lev.cheb, H.degree)


def vcycle(H: Hierarchy, l: int, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """One V-cycle on level ``l``: smooth, restrict the residual, solve the
    coarse error equation recursively (exactly on the coarsest level),
    prolong and add the correction, smooth again (Sec. 2.3, Fig. 1)."""
    lev = H.levels[l]
    if l == len(H.levels) - 1:
        return coarse_solve(lev, b)
    x = smooth(H, lev, x, b)
    rc = restrict_fw(b - lev.apply(x))
    e = vcycle(H, l + 1, np.zeros_like(rc), rc)
    x = x + prolong(e)
    x = smooth(H, lev, x, b)
    return x


@dataclass
class SolveResult:
    phi: np.ndarray
    cycles: int
    history: List[float] = field(default_factory=list)


def solve(H: Hierarchy, b: np.ndarray, phi0: Optional[np.ndarray] = None,
          tol: float = 1e-10, max_cycles: int = 50) -> SolveResult:
    """Warm-startable solve: project the mean out of ``b`` (Sec. 2.1), start
    from ``phi0`` (the previous step's solution for a warm start, Sec. 3.1),
    apply V-cycles until ``||b - M phi|| / ||b|| <= tol`` (tested before each
    cycle) or ``max_cycles``, and return ``phi`` with its mean removed."""
    lev = H.levels[0]
    b = b - b.mean()
    nb = np.linalg.norm(b)
    phi = np.zeros_like(b) if phi0 is None else np.array(phi0, dtype=np.float64)
    if nb == 0.0:
        return SolveResult(np.zeros_like(b), 0, [0.0])
    hist = [np.linalg.norm(b - lev.apply(phi)) / nb]
    cycles = 0
    while hist[-1] > tol and cycles < max_cycles:
        phi = vcycle(H, 0, phi, b)
        cycles += 1
        hist.append(np.linalg.norm(b - lev.apply(phi)) / nb)
    phi = phi - phi.mean()
    return SolveResult(phi, cycles, hist)


def solve_pcg(H: Hierarchy, b: np.ndarray, phi0: Optional[np.ndarray] = None,
              tol: float = 1e-10, max_iter: int = 50) -> SolveResult:
    """Multigrid-preconditioned conjugate gradients (Sec. 3.2): one V-cycle from
    zero is the preconditioner ``B`` and ``phi0`` the first iterate.

    Textbook preconditioned CG (Saad, Iterative Methods for Sparse Linear
    Systems, Alg. 9.1) written directly in ``M`` and ``B``.  Both are negative
    semidefinite on the same space, so every step size is that of CG on
    ``-M`` preconditioned by ``-B``.  ``history`` holds the relative norm of the
    recursively updated residual.  When the recursive residual meets ``tol`` the true
    residual ``b - M phi`` is formed; if it misses ``tol`` the iteration
    restarts from it.  ``cycles`` counts CG iterations; each applies the
    preconditioner once."""
    lev = H.levels[0]
    b = b - b.mean()
    nb = np.linalg.norm(b)
    phi = np.zeros_like(b) if phi0 is None else np.array(phi0, dtype=np.float64)
    if nb == 0.0:
        return SolveResult(np.zeros_like(b), 0, [0.0])
    precond = lambda r: vcycle(H, 0, np.zeros_like(r), r)
    r = b - lev.apply(phi)
    hist = [np.linalg.norm(r) / nb]
    its = 0
    while hist[-1] > tol and its < max_iter:
        z = precond(r)
        p = z
        rz = np.vdot(r, z)
        while its < max_iter:
            q = lev.apply(p)
            alpha = rz / np.vdot(p, q)
            phi = phi + alpha * p
            r = r - alpha * q
            its += 1
            hist.append(np.linalg.norm(r) / nb)
            if hist[-1] <= tol:
                break
            z = precond(r)
            rz_new = np.vdot(r, z)
            p = z + (rz_new / rz) * p
            rz = rz_new
        r = b - lev.apply(phi)          # restart from the true residual
        if np.linalg.norm(r) / nb > tol and its < max_iter:
            hist[-1] = np.linalg.norm(r) / nb
    phi = phi - phi.mean()
    return SolveResult(phi, its, hist)


def true_rel_residual(H: Hierarchy, b: np.ndarray, phi: np.ndarray) -> float:
    b = b - b.mean()
    return float(np.linalg.norm(b - H.levels[0].apply(phi)) / np.linalg.norm(b))


# ---------------------------------------------------------------------------
# Initial guesses (Sec. 3.2: recycling, eq. growth, polynomial extrapolation)
# ---------------------------------------------------------------------------

def predict(history: List[np.ndarray], kind: str, growth: float = 1.0) -> np.ndarray:
    """Initial guess for step ``n`` from earlier solutions, newest first
    (``history[0] = phi_{n-1}``, ``history[1] = phi_{n-2}``, ...):

    * ``recycle``: ``phi_{n-1}``;
    * ``growth``: ``(D_n / D_{n-1}) phi_{n-1}`` with ``growth = D_n / D_{n-1}``;
    * ``linear``: ``2 phi_{n-1} - phi_{n-2}``;
    * ``quadratic``: ``3 phi_{n-1} - 3 phi_{n-2} + phi_{n-3}``."""
    if kind == "recycle":
        return np.array(history[0], dtype=np.float64)
    if kind == "growth":
        return growth * history[0]
    if kind == "linear":
        return 2.0 * history[0] - history[1]
    if kind == "quadratic":
        return 3.0 * history[0] - 3.0 * history[1] + history[2]
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# Force readout (Sec. 3.4: fourth-order gradient; Sec. 4.5.1, eq. accel)
# ---------------------------------------------------------------------------

def gradient4(phi: np.ndarray, h: float) -> np.ndarray:
    """Fourth-order central first differences along each direction,
    ``(u_{i-2} - 8 u_{i-1} + 8 u_{i+1} - u_{i+2}) / (12 h)``; ``(3, n, n, n)``
    in direction order (x, y, z)."""
    out = np.empty((3,) + phi.shape)
    for a in range(3):
        out[a] = (_sh(phi, a, -2) - 8.0 * _sh(phi, a, -1)
                  + 8.0 * _sh(phi, a, 1) - _sh(phi, a, 2)) / (12.0 * h)
    return out


def accel(phi: np.ndarray, h: float, psi: Optional[np.ndarray] = None,
          scale: float = 1.0) -> np.ndarray:
    """``a = -scale J^-1 grad phi`` (eq. accel; ``scale`` is the paper's
    ``3/2 Omega_m``), ``grad`` the fourth-order difference and ``J = I + Hess psi``
    (eq. triad).  Without ``psi`` the mesh is uniform (``J = I``) and ``a`` is
    the plain force ``-scale grad phi``."""
    g = gradient4(phi, h)
    if psi is None:
        return -scale * g
    J = triad(psi, h)
    gv = np.moveaxis(g, 0, -1)[..., None]            # (n, n, n, 3, 1)
    a = np.linalg.solve(J, gv)[..., 0]
    return -scale * np.moveaxis(a, -1, 0)


# ---------------------------------------------------------------------------
# Adjoint and gradients (Sec. 4.8, eqs. adj_rhs and adj_op)
# ---------------------------------------------------------------------------

def solve_adjoint(H: Hierarchy, phibar: np.ndarray, tol: float = 1e-10,
                  max_cycles: int = 50, lam0=None) -> SolveResult:
    """``lambda = M^+ phibar`` for the symmetric operator: the same solver on
    the cotangent (with ``b = sqrt(g) f`` the paper's ``Fbar = sqrt(g) lambda``
    follows)."""
    return solve(H, phibar, lam0, tol, max_cycles)


def coeff_grad(lam: np.ndarray, phi: np.ndarray, h: float) -> np.ndarray:
    """``dL/dC = -d(lam^T M(C) phi)/dC`` at fixed ``lam, phi`` (operator VJP).

    Diagonal components: mean over the two faces of ``D+_a lam * D+_a phi``.
    Off-diagonal ``(a, b)``: ``D0_a lam D0_b phi + D0_b lam D0_a phi`` (both
    ordered pairs share the stored component)."""
    out = np.empty((6,) + phi.shape)
    for a in range(3):
        g = (_sh(lam, a, 1) - lam) * (_sh(phi, a, 1) - phi) / (h * h)   # face i+1/2
        out[a] = 0.5 * (g + _sh(g, a, -1))
    d0 = lambda u, a: (_sh(u, a, 1) - _sh(u, a, -1)) / (2.0 * h)
    for a, b, c in PAIRS:
        out[c] = d0(lam, a) * d0(phi, b) + d0(lam, b) * d0(phi, a)
    return out


# ---------------------------------------------------------------------------
# Moving-mesh geometry (Sec. 4.2: eqs. map, triad, metric)
# ---------------------------------------------------------------------------

def hessian(psi: np.ndarray, h: float) -> np.ndarray:
    """Second-order central Hessian stencils, ``(6, n, n, n)`` in component order."""
    H = np.empty((6,) + psi.shape)
    for a in range(3):
        H[a] = (_sh(psi, a, 1) - 2.0 * psi + _sh(psi, a, -1)) / (h * h)
    for a, b, c in PAIRS:
        pp = _sh(_sh(psi, a, 1), b, 1)
        pm = _sh(_sh(psi, a, 1), b, -1)
        mp = _sh(_sh(psi, a, -1), b, 1)
        mm = _sh(_sh(psi, a, -1), b, -1)
        H[c] = (pp - pm - mp + mm) / (4.0 * h * h)
    return H


def _to_mat(S: np.ndarray) -> np.ndarray:
    """``(6, ...)`` symmetric storage -> ``(..., 3, 3)`` matrices."""
    n = S.shape[1:]
    A = np.empty(n + (3, 3))
    for a in range(3):
        for b in range(3):
            A[..., a, b] = S[COMP[(a, b)]]
    return A


def _from_mat(A: np.ndarray) -> np.ndarray:
    S = np.empty((6,) + A.shape[:-2])
    for a in range(3):
        S[a] = A[..., a, a]
    for a, b, c in PAIRS:
        S[c] = A[..., a, b]
    return S


def triad(psi: np.ndarray, h: float) -> np.ndarray:
    """``J = I + Hess psi`` as ``(n, n, n, 3, 3)`` symmetric matrices (eq. triad)."""
    J = _to_mat(hessian(psi, h))
    for a in range(3):
        J[..., a, a] += 1.0
    return J


def geometry(psi: np.ndarray, h: float):
    """``C = sqrt(g) g^{-1} = det(J) J^-1 J^-T`` and ``sqrt(g) = det J`` (eq. metric)."""
    J = triad(psi, h)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    g_inv = Jinv @ np.swapaxes(Jinv, -1, -2)
    C = _from_mat(det[..., None, None] * g_inv)
    return C, det


def geometry_bwd(psi: np.ndarray, Cbar: np.ndarray, sqrtgbar: np.ndarray, h: float) -> np.ndarray:
    """Reverse mode of :func:`geometry`.

    ``Cbar`` uses the symmetric storage convention: the stored off-diagonal
    entry's cotangent is the sum of the cotangents of ``C_ab`` and ``C_ba``.
    Per cell, with ``K = J^-1`` and ``d = det J`` (``J`` symmetric) and ``G``
    the full-matrix cotangent of ``C = d K K``:
    ``Jbar = d <G, K K> K - d (K K G K)^T - d (K G K K)^T + sqrtgbar d K``.
    Then ``psibar = sum_{a,b} Hess_ab^T Jbar_ab``; the stencils are
    self-adjoint on the periodic grid.
    """
    J = triad(psi, h)
    d = np.linalg.det(J)
    K = np.linalg.inv(J)
    G = np.empty(J.shape)
    for a in range(3):
        for b in range(3):
            G[..., a, b] = Cbar[COMP[(a, b)]] if a == b else 0.5 * Cbar[COMP[(a, b)]]
    K2 = K @ K
    t = d * np.einsum("...ab,...ab->...", G, K2)
    Jbar = (t + sqrtgbar * d)[..., None, None] * K
    Jbar = Jbar - d[..., None, None] * np.swapaxes(K2 @ G @ K, -1, -2)
    Jbar = Jbar - d[..., None, None] * np.swapaxes(K @ G @ K2, -1, -2)
    # dJ_ab = Hess_ab dpsi for all (a, b); sum the adjoint stencils
    Hb = np.empty((6,) + psi.shape)
    for a in range(3):
        Hb[a] = Jbar[..., a, a]
    for a, b, c in PAIRS:
        Hb[c] = Jbar[..., a, b] + Jbar[..., b, a]
    return np.sum(hessian_adjoint(Hb, h), axis=0)


def hessian_adjoint(Hb: np.ndarray, h: float) -> np.ndarray:
    """Transpose of each Hessian stencil applied to its component; equal to
    the stencil itself because each stencil is symmetric under ``i -> -i``."""
    return hessian_components(Hb, h)


def hessian_components(S: np.ndarray, h: float) -> np.ndarray:
    out = np.empty_like(S)
    for a in range(3):
        u = S[a]
        out[a] = (_sh(u, a, 1) - 2.0 * u + _sh(u, a, -1)) / (h * h)
    for a, b, c in PAIRS:
        u = S[c]
        out[c] = (_sh(_sh(u, a, 1), b, 1) - _sh(_sh(u, a, 1), b, -1)
                  - _sh(_sh(u, a, -1), b, 1) + _sh(_sh(u, a, -1), b, -1)) / (4.0 * h * h)
    return out


def admissible_scale(psi: np.ndarray, h: float, det_min: float = 0.3,
                     det_max: float = 3.0, steps: int = 60) -> float:
    """Largest ``s`` with ``det_min <= det(I + s Hess psi) <= det_max`` and
    ``lambda_min(I + s Hess psi) > 0`` in every cell, by bisection on
    ``[0, s_hi]`` (cf. App. C, eq. bisection).  The eigenvalues of
    ``I + s H`` are ``1 + s mu`` for the eigenvalues ``mu`` of ``H``."""
    H = _to_mat(hessian(psi, h))
    mu = np.linalg.eigvalsh(H.reshape(-1, 3, 3))
    del H

    def ok(s):
        lam = 1.0 + s * mu
        if np.min(lam) <= 0.0:
            return False
        det = np.prod(lam, axis=1)
        return det.min() >= det_min and det.max() <= det_max

    lo, hi = 0.0, 1.0
    while ok(hi):
        lo, hi = hi, 2.0 * hi
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if ok(mid):
            lo = mid
        else:
            hi = mid
    return lo
