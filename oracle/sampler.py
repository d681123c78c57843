"""Composed PSE displacement and error bounds (oracle).

TEST INFRASTRUCTURE ONLY.

The Brownian displacement over a step dt (eqs. langevin, split):

    dx = dt M F + sqrt(2 kT dt) ( M_r^{1/2} z1 + M_w^{1/2} z2 )

with M_r^{1/2} the symmetric root (the exact object the Krylov sample
approximates) and M_w^{1/2} z2 the direct Fourier sum over the grid k-set.
"""
from dataclasses import dataclass
from math import erfc, exp, pi, sqrt

import numpy as np

from . import ewald, lanczos, philox, rpy


@dataclass
class Params:
    L: float          # cubic box side
    a: float = 1.0    # sphere radius
    eta: float = 1.0  # viscosity
    kT: float = 1.0
    xi: float = 0.5   # splitting parameter
    rc: float = 8.0   # real-space cutoff
    M: int = 64       # grid points per side (sets the k-set)


def real_sample(x, z1, p):
    """y_r = M_r^{1/2} z1 by eigendecomposition (Sec. II B.1)."""
    Mr = rpy.real_block_dense(x, p.L, p.a, p.eta, p.xi, p.rc)
    return lanczos.sqrt_apply(Mr, z1).reshape(-1, 3)


def displacement(x, z1, zeta, p, dt=1.0, forces=None):
    """dx = sqrt(2 kT dt)(M_r^{1/2} z1 + y_w(zeta)) + dt (M_r + M_w) F.
    zeta: conjugate-symmetric k-space noise on the full grid [3, M, M, M]."""
    x = np.asarray(x, dtype=np.float64)
    yr = real_sample(x, np.asarray(z1, dtype=np.float64).ravel(), p)
    yw = ewald.wave_sample_direct(x, zeta, p.L, p.a, p.eta, p.xi)
    out = sqrt(2.0 * p.kT * dt) * (yr + yw)
    if forces is not None:
        out = out + dt * mobility_apply(x, forces, p)
    return out


def mobility_apply(x, F, p):
    """(M_r + M_w) F, M_w over the grid k-set (eqs. Mreal, Mwave)."""
    Mr = rpy.real_block_dense(x, p.L, p.a, p.eta, p.xi, p.rc)
    ur = (Mr @ np.asarray(F, dtype=np.float64).ravel()).reshape(-1, 3)
    uw = ewald.wave_apply_direct(x, F, p.M, p.L, p.a, p.eta, p.xi)
    return ur + uw


def displacement_from_grid_noise(x, z1, W, p, dt=1.0, forces=None):
    """Same, with the wave noise given as real white noise W[3, M, M, M] on the
    grid: zeta = DFT(W)/M^{3/2}."""
    return displacement(x, z1, ewald.zeta_from_grid_noise(W), p, dt, forces)


def displacement_philox(x, p, seed, sample, dt=1.0, forces=None, bits=53):
    """Same, with z1 and zeta drawn from Philox-4x64-10 as specified in
    oracle.philox."""
    z1 = philox.real_noise(len(x), seed, sample, bits)
    zeta = philox.wave_noise_full(p.M, seed, sample, bits)
    return displacement(x, z1, zeta, p, dt, forces)


# ---------------------------------------------------------------------------
# truncation / quadrature error bounds (Sec. II C, Sec. II D)
# ---------------------------------------------------------------------------
def eps_real(xi, rc):
    """Real-space truncation error ~ exp(-xi^2 rc^2) (Sec. II A, Sec. II C)."""
    return exp(-(xi * rc) ** 2)


def eps_wave_bound(kc, xi, a):
    """Bound on the relative wave-space truncation error of the self mobility
    for the PSE kernel (last display of Sec. II D):
    [4 kc^-1 e^{-kc^2/4xi^2} - sqrt(pi) xi^-1 erfc(kc/2xi)] / (2 pi a)."""
    return (4.0 / kc * exp(-kc * kc / (4 * xi * xi)) - sqrt(pi) / xi * erfc(kc / (2 * xi))) / (2 * pi * a)


def eps_wave_exact_self(kc, xi, a, kmax_factor=14.0, n=200000):
    """The quantity that bound controls, eq. (errbound) with the PSE kernel:
    (2a/pi) int_{kc}^inf sinc^2(ka) H(k, xi) dk (midpoint rule, fine grid)."""
    kmax = max(kc, kmax_factor * xi)
    if kmax <= kc:
        return 0.0
    k = np.linspace(kc, kmax, n + 1)
    km = 0.5 * (k[1:] + k[:-1])
    f = rpy._sinc2(km * a) * rpy.H_split(km, xi)
    return float(2 * a / pi * np.sum(f) * (k[1] - k[0]))


def eps_quadrature(P, m):
    """Spectral-Ewald quadrature error ~ exp(-pi^2 P^2 / 2 m^2) + erfc(m/sqrt 2)
    (Sec. II C)."""
    return exp(-(pi * P) ** 2 / (2 * m * m)) + erfc(m / sqrt(2.0))
