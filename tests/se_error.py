"""Error estimates of the spectral-Ewald wave-space part, used as test bars.
Host-side arithmetic on the oracle's B(k); nothing here runs on the GPU."""
import numpy as np
from scipy.special import erfc

from oracle import ewald


def se_quadrature_bound(P):
    """Quadrature error bound of Sec. II C, e^{-pi^2 P^2 / 2 m^2} +
    erfc(m / sqrt 2), at the Gaussian width m = sqrt(pi P) used here
    (the first term is then e^{-pi P / 2})."""
    m = np.sqrt(np.pi * P)
    return float(np.exp(-np.pi**2 * P**2 / (2 * m * m)) + erfc(m / np.sqrt(2.0)))


def se_aliasing_estimate(L, M, xi, P, a=1.0, m=None):
    """Relative error of a spectral-Ewald wave sample from aliasing: the
    interpolation with the Gaussian window g (std sigma = P h / 2m,
    m = sqrt(pi P) unless given) sees each grid mode k also at k + 2 pi n / h, with
    amplitude ratio ghat(k + 2 pi n / h) / ghat(k).  Weighted by B(k) over the
    k-set, with the first alias shell (n in {-1, 0, 1}^3, n != 0):
        err^2 ~ sum_k B(k) sum_n (ghat(k + 2 pi n/h) / ghat(k))^2 / sum_k B(k).
    At h = 0.94a (256^3 in a 240.8a box) the modes near the Nyquist frequency
    still carry weight and this is ~5e-4; at h = 0.54a it is ~3e-5."""
    h = L / M
    s = P * h / (2.0 * (np.sqrt(np.pi * P) if not m else m))
    j = np.fft.fftfreq(M, 1.0 / M)
    k1 = 2 * np.pi * j / L
    ok1 = np.abs(j) < M // 2
    # the shell sum factorises over the axes:
    #   sum_{n != 0} prod_d r(k_d, n_d) = prod_d (1 + r(k_d, -1) + r(k_d, 1)) - 1
    r1 = lambda k, n: np.exp(-((k + 2 * np.pi * n / h) ** 2 - k**2) * s * s)
    f1 = 1.0 + r1(k1, -1) + r1(k1, 1)
    K2 = (k1 * k1)[:, None, None] + (k1 * k1)[None, :, None] + (k1 * k1)[None, None, :]
    ok = ok1[:, None, None] & ok1[None, :, None] & ok1[None, None, :] & (K2 > 0)
    B = np.zeros_like(K2)
    B[ok] = ewald.B_kernel(K2[ok], a, xi)
    del K2
    tot = f1[:, None, None] * f1[None, :, None] * f1[None, None, :] - 1.0
    return float(np.sqrt((B * tot)[ok].sum() / B[ok].sum()))
