"""Seeded synthetic inputs shared by the tests, the benchmark and the CPU oracle.

This module only *generates inputs*: Gaussian random fields with a prescribed
isotropic power spectrum, and the named workloads built from them.  It holds
none of the multigrid method's arithmetic (no operator, smoother, transfer,
solve, geometry or gradient), so that the oracle and the HIP path can share
inputs without sharing any of the computation they are compared on.

Recipe of a Gaussian random field (GRF) on an ``n**3`` periodic grid of box
length 1:

1. ``w = numpy.random.default_rng(seed).standard_normal((n, n, n))``
2. ``W = rfftn(w)`` (scipy.fft, multithreaded); wavevector ``k = 2*pi*m`` for integer frequencies ``m``
   (cycles per box), ``|k|`` taken over the full grid;
3. multiply ``W`` by ``sqrt(P(|k|))`` with ``P(0) = 0``;
4. ``irfftn``, subtract the mean, divide by the population standard deviation.

The spectra are ``P(k) = k**p * exp(-(k/k_c)**2)`` (no cutoff when ``k_c`` is
None).  The particle-mesh density contrasts and the moving-mesh run the paper
measures on are not available; these fields take their shapes, sizes and
spectral slopes (paper, Sec. 3 and Sec. 4) as stand-ins.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.fft as sfft

# FFT worker threads (pocketfft through scipy); results do not depend on it
FFT_WORKERS = min(16, os.cpu_count() or 1)

TWO_PI = 2.0 * math.pi


@dataclass(frozen=True)
class Spectrum:
    """Isotropic power spectrum ``P(k) = k**power * exp(-(k/kc)**2)``."""

    power: float
    kc: Optional[float] = None  # cutoff wavenumber in radians per box length

    def __call__(self, k: np.ndarray) -> np.ndarray:
        out = np.zeros_like(k)
        nz = k > 0
        kk = k[nz]
        val = kk ** self.power
        if self.kc is not None:
            val = val * np.exp(-((kk / self.kc) ** 2))
        out[nz] = val
        return out


def _kmag(n: int) -> np.ndarray:
    m = np.fft.fftfreq(n, d=1.0 / n)          # integer frequencies, full axis
    mr = np.fft.rfftfreq(n, d=1.0 / n)        # last (half) axis
    kz = TWO_PI * m[:, None, None]
    ky = TWO_PI * m[None, :, None]
    kx = TWO_PI * mr[None, None, :]
    return np.sqrt(kz * kz + ky * ky + kx * kx)


def white_noise(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((n, n, n))


def grf(n: int, spectrum: Spectrum, seed: int) -> np.ndarray:
    """Zero-mean, unit-variance float64 GRF of shape ``(n, n, n)``."""
    w = white_noise(n, seed)
    W = sfft.rfftn(w, workers=FFT_WORKERS)
    del w
    W *= np.sqrt(spectrum(_kmag(n)))
    f = sfft.irfftn(W, s=(n, n, n), axes=(0, 1, 2), workers=FFT_WORKERS)
    del W
    f -= f.mean()
    sd = f.std()
    if sd > 0:
        f /= sd
    return np.ascontiguousarray(f)


# ---------------------------------------------------------------------------
# Named workloads.  Seeds and spectra follow the benchmark configurations:
#   C1  32^3 source, P ~ k^-1 exp(-(k/(8*2pi))^2), seed 0
#   C2  256^3 warm-start sequence rho_t = (1 + 0.05 t) delta + 0.02 t eta_t,
#       t = 0..7, delta seed 0, eta_t seed 100 + t, P ~ k^-1 (no cutoff)
#   C3  1024^3 source, P ~ k^-1 exp(-(k/(256*2pi))^2), seed 0
#   C4  moving mesh: psi seed 1, P ~ k^-4 exp(-(k/(16*2pi))^2); source field
#       g seed 0, P ~ k^-1 exp(-(k/((n/4)*2pi))^2); loss weight w seed 2
#   B512 / sweep  source with k_c = (n/4)*2pi, seed 0
# ---------------------------------------------------------------------------

def source_spectrum(n: int) -> Spectrum:
    """Source spectrum with the ``k_c = (n/4) * 2*pi`` cutoff rule (C1, C3, sweep)."""
    return Spectrum(-1.0, (n / 4.0) * TWO_PI)


def flat_source(n: int, seed: int = 0) -> np.ndarray:
    return grf(n, source_spectrum(n), seed)


def warm_sequence(n: int, steps: int = 8):
    """Yield ``rho_t`` for the warm-start defect-correction sequence (C2)."""
    spec = Spectrum(-1.0, None)
    delta = grf(n, spec, 0)
    for t in range(steps):
        if t == 0:
            yield delta.copy()
        else:
            eta = grf(n, spec, 100 + t)
            yield (1.0 + 0.05 * t) * delta + 0.02 * t * eta


def psi_unit(n: int, seed: int = 1) -> np.ndarray:
    """Unit-variance deformation potential before scaling (C4)."""
    return grf(n, Spectrum(-4.0, 16.0 * TWO_PI), seed)


def moving_mesh_field(n: int, seed: int = 0) -> np.ndarray:
    """Source field ``g`` of the moving-mesh problem (C4), before the
    volume weighting and the solvability projection."""
    return grf(n, source_spectrum(n), seed)


def loss_weight(n: int, seed: int = 2) -> np.ndarray:
    """Fixed unit-variance weight ``w`` of the loss ``L = sum(w * phi)`` (C5)."""
    return grf(n, source_spectrum(n), seed)


def fd_direction_psi(n: int, k: int) -> np.ndarray:
    """Finite-difference direction ``k`` (0..15) for psi: GRF with psi's spectrum."""
    return grf(n, Spectrum(-4.0, 16.0 * TWO_PI), 1000 + k)


def fd_direction_white(n: int, k: int) -> np.ndarray:
    """Finite-difference direction ``k`` (0..15) for a source: white noise."""
    return white_noise(n, 1000 + k)
