"""Real-space part of the positively split RPY mobility, FP64 (oracle).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.

Everything here is dimensionless in the sense of Appendix A: the scalar
functions are 6*pi*eta*a times the mobility, so that

    6 pi eta a M^(r)_ij = F(r) (I - rr) + G(r) rr            (App. A, first eq.)

The normalisation in eqs. (int1)/(int2) carries 1/eta instead; multiplying
those integrals by 6 pi eta a gives the prefactors 3a/pi and 6a/pi used below.
"""
import numpy as np
from scipy.special import erfc

SQRT_PI = np.sqrt(np.pi)


# ---------------------------------------------------------------------------
# free-space RPY tensor, eq. (RPY_free_space)
# ---------------------------------------------------------------------------
def rpy_free_FG(r, a):
    """Free-space RPY tensor written as F (I - rr) + G rr, times 6 pi eta a.

    eq. (RPY_free_space): for r > 2a the coefficient of I is 3a/4r + a^3/2r^3
    and of rr is 3a/4r - 3a^3/2r^3; for r <= 2a they are 1 - 9r/32a and 3r/32a.
    In the (I - rr, rr) basis F = coeff(I) and G = coeff(I) + coeff(rr).
    """
    r = np.asarray(r, dtype=np.float64)
    far = r > 2.0 * a
    with np.errstate(divide="ignore", invalid="ignore"):
        cI_far = 3.0 * a / (4.0 * r) + a**3 / (2.0 * r**3)
        crr_far = 3.0 * a / (4.0 * r) - 3.0 * a**3 / (2.0 * r**3)
    cI_near = 1.0 - 9.0 * r / (32.0 * a)
    crr_near = 3.0 * r / (32.0 * a)
    cI = np.where(far, cI_far, cI_near)
    crr = np.where(far, crr_far, crr_near)
    return cI, cI + crr


def rpy_free_tensor(d, a, eta):
    """3x3 free-space RPY block for separation vector d (eq. RPY_free_space).
    d = 0 gives the Stokes drag 1/(6 pi eta a) I."""
    d = np.asarray(d, dtype=np.float64)
    r = np.linalg.norm(d)
    if r == 0.0:
        return np.eye(3) / (6.0 * np.pi * eta * a)
    F, G = rpy_free_FG(r, a)
    rr = np.outer(d, d) / r**2
    return (F * (np.eye(3) - rr) + G * rr) / (6.0 * np.pi * eta * a)


# ---------------------------------------------------------------------------
# closed forms of Appendix A (Case 1: r > 2a, Case 2: r <= 2a)
# ---------------------------------------------------------------------------
def real_FG_closed(r, xi, a):
    """Appendix A closed forms for F(r, xi), G(r, xi) (dimensionless).

    Case 1 (r > 2a) has f0 = g0 = 0; Case 2 (r <= 2a) adds the polynomial
    terms f0, g0.  All other coefficients are common to both cases.
    Evaluated in FP64; valid away from r -> 0, where the terms grow like
    1/(r^3 xi^4) and cancel (see real_FG for the small-r route).
    """
    r = np.asarray(r, dtype=np.float64)
    x = xi
    sp = SQRT_PI
    f1 = (18 * r**2 * x**2 + 3) / (64 * sp * a * r**2 * x**3)
    f2 = (2 * x**2 * (2 * a - r) * (4 * a**2 + 4 * a * r + 9 * r**2) - 2 * a - 3 * r) / (128 * sp * a * r**3 * x**3)
    f3 = (-2 * x**2 * (2 * a + r) * (4 * a**2 - 4 * a * r + 9 * r**2) + 2 * a - 3 * r) / (128 * sp * a * r**3 * x**3)
    f4 = (3 - 36 * r**4 * x**4) / (128 * a * r**3 * x**4)
    f5 = (4 * x**4 * (r - 2 * a) ** 2 * (4 * a**2 + 4 * a * r + 9 * r**2) - 3) / (256 * a * r**3 * x**4)
    f6 = (4 * x**4 * (2 * a + r) ** 2 * (4 * a**2 - 4 * a * r + 9 * r**2) - 3) / (256 * a * r**3 * x**4)
    g1 = (6 * r**2 * x**2 - 3) / (32 * sp * a * r**2 * x**3)
    g2 = (-2 * x**2 * (r - 2 * a) ** 2 * (2 * a + 3 * r) + 2 * a + 3 * r) / (64 * sp * a * r**3 * x**3)
    g3 = (2 * x**2 * (2 * a + r) ** 2 * (2 * a - 3 * r) - 2 * a + 3 * r) / (64 * sp * a * r**3 * x**3)
    g4 = -(3 * (4 * r**4 * x**4 + 1)) / (64 * a * r**3 * x**4)
    g5 = (3 - 4 * x**4 * (2 * a - r) ** 3 * (2 * a + 3 * r)) / (128 * a * r**3 * x**4)
    g6 = (3 - 4 * x**4 * (2 * a - 3 * r) * (2 * a + r) ** 3) / (128 * a * r**3 * x**4)
    near = r <= 2 * a
    f0 = np.where(near, -((r - 2 * a) ** 2) * (4 * a**2 + 4 * a * r + 9 * r**2) / (32 * a * r**3), 0.0)
    g0 = np.where(near, (2 * a - r) ** 3 * (2 * a + 3 * r) / (16 * a * r**3), 0.0)
    e1 = np.exp(-(r**2) * x**2)
    e2 = np.exp(-((r - 2 * a) ** 2) * x**2)
    e3 = np.exp(-((r + 2 * a) ** 2) * x**2)
    c1 = erfc(r * x)
    c2 = erfc((r - 2 * a) * x)
    c3 = erfc((r + 2 * a) * x)
    F = f0 + f1 * e1 + f2 * e2 + f3 * e3 + f4 * c1 + f5 * c2 + f6 * c3
    G = g0 + g1 * e1 + g2 * e2 + g3 * e3 + g4 * c1 + g5 * c2 + g6 * c3
    return F, G


def real_self(xi, a):
    """Real-space self mobility times 6 pi eta a, eq. (self)."""
    return (1.0 - np.exp(-4.0 * a**2 * xi**2) + 4.0 * SQRT_PI * a * xi * erfc(2.0 * a * xi)) / (4.0 * SQRT_PI * xi * a)


# ---------------------------------------------------------------------------
# H-weighted wave integrals (eqs. int1/int2 with H in place of 1 - H)
# ---------------------------------------------------------------------------
def H_split(k, xi):
    """Hasimoto splitting function H(k, xi) = (1 + k^2/4xi^2) exp(-k^2/4xi^2)
    (Sec. II A, definition under eq. Mreal)."""
    q = np.asarray(k, dtype=np.float64) ** 2 / (4.0 * xi**2)
    return (1.0 + q) * np.exp(-q)


def H_beenakker(k, xi):
    """Beenakker's splitting function (1 + k^2/4xi^2 + k^4/8xi^4) e^{-k^2/4xi^2},
    the counter-example of Sec. II A.1: it exceeds 1 for some k."""
    q = np.asarray(k, dtype=np.float64) ** 2 / (4.0 * xi**2)
    return (1.0 + q + 2.0 * q**2) * np.exp(-q)


def _sinc2(ka):
    ka = np.asarray(ka, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(ka == 0.0, 1.0, np.sin(ka) / np.where(ka == 0.0, 1.0, ka))
    return s * s


def _series(u, coef_fn, nterms=12):
    out = np.zeros_like(u)
    for n in range(nterms, 0, -1):
        out = out * u * u + coef_fn(n)
    return out


def _fact(n):
    return float(np.prod(np.arange(1, n + 1, dtype=np.float64))) if n > 0 else 1.0


def kernel_KF(u):
    """(u cos u + (u^2 - 1) sin u)/u^3, the radial kernel of eq. (int1).
    Power series 2/3 - 2u^2/15 + u^4/140 - ... below u = 0.5 (cancellation)."""
    u = np.asarray(u, dtype=np.float64)
    small = u < 0.5

    def c(n):  # coefficient of u^(2n-2)
        return (-1) ** n * (1.0 / _fact(2 * n) - 1.0 / _fact(2 * n + 1) - 1.0 / _fact(2 * n - 1))

    us = np.where(small, u, 1.0)
    ul = np.where(small, 1.0, u)
    return np.where(small, _series(us, c), (ul * np.cos(ul) + (ul**2 - 1) * np.sin(ul)) / ul**3)


def kernel_KG(u):
    """(sin u - u cos u)/u^3, the radial kernel of eq. (int2).
    Power series 1/3 - u^2/30 + u^4/840 - ... below u = 0.5."""
    u = np.asarray(u, dtype=np.float64)
    small = u < 0.5

    def c(n):
        return (-1) ** n * (1.0 / _fact(2 * n + 1) - 1.0 / _fact(2 * n))

    us = np.where(small, u, 1.0)
    ul = np.where(small, 1.0, u)
    return np.where(small, _series(us, c), (np.sin(ul) - ul * np.cos(ul)) / ul**3)


def _gl_panels(kmax, width, npts=24):
    """Composite Gauss-Legendre nodes/weights on [0, kmax] with panels of
    about `width` (resolves the oscillation of the integrands)."""
    npan = max(1, int(np.ceil(kmax / width)))
    t, w = np.polynomial.legendre.leggauss(npts)
    edges = np.linspace(0.0, kmax, npan + 1)
    lo, hi = edges[:-1, None], edges[1:, None]
    nodes = (0.5 * (hi - lo) * t[None, :] + 0.5 * (hi + lo)).ravel()
    weights = (0.5 * (hi - lo) * w[None, :]).ravel()
    return nodes, weights


def wave_FG_quad(r, xi, a, H=H_split):
    """H-weighted counterpart of eqs. (int1)/(int2), times 6 pi eta a:

        F_w(r) = (3a/pi) int_0^inf H(k) sinc^2(ka) K_F(kr) dk
        G_w(r) = (6a/pi) int_0^inf H(k) sinc^2(ka) K_G(kr) dk

    The integrand decays like a Gaussian, so composite Gauss-Legendre on
    [0, 14 xi] is exact to rounding.  F = F_free - F_w and G = G_free - G_w
    because the sinc^2-weighted integrals without H give the free RPY tensor
    (Sec. II A, last paragraph before II A.1)."""
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    kmax = 14.0 * xi
    F = np.empty_like(r)
    G = np.empty_like(r)
    for idx, rv in enumerate(r):
        width = 0.5 / max(rv, 2.0 * a, 1.0 / xi)
        k, w = _gl_panels(kmax, width)
        base = H(k, xi) * _sinc2(k * a) * w
        F[idx] = 3.0 * a / np.pi * np.sum(base * kernel_KF(k * rv))
        G[idx] = 6.0 * a / np.pi * np.sum(base * kernel_KG(k * rv))
    return F, G


def real_FG(r, xi, a):
    """F, G of eq. (Mreal) for any r >= 0 (dimensionless, Appendix A).

    Closed forms of Appendix A wherever they are well conditioned
    (r^3 xi^4 >= 1e-3 a^-1 ... i.e. the 1/(r^3 xi^4) terms stay below ~1e3);
    below that, F = F_free - F_w with F_w by quadrature (same identity, no
    cancellation).  r = 0 gives eq. (self) for both."""
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    F = np.empty_like(r)
    G = np.empty_like(r)
    closed = r**3 * xi**4 >= 1e-3 * a**3
    if closed.any():
        F[closed], G[closed] = real_FG_closed(r[closed], xi, a)
    small = ~closed
    if small.any():
        Ff, Gf = rpy_free_FG(r[small], a)
        Fw, Gw = wave_FG_quad(r[small], xi, a)
        F[small] = Ff - Fw
        G[small] = Gf - Gw
    zero = r == 0.0
    if zero.any():
        F[zero] = G[zero] = real_self(xi, a)
    return F, G


# ---------------------------------------------------------------------------
# dense real-space grand mobility block M_r (eqs. Mreal, self; sum over images)
# ---------------------------------------------------------------------------
def _image_shifts(L, rc):
    n = int(np.ceil(rc / L))
    rng = np.arange(-n, n + 1)
    return L * np.array(np.meshgrid(rng, rng, rng, indexing="ij")).reshape(3, -1).T


def real_pairs(x, L, xi, a, rc):
    """All (i, j, d) with d = x_i - x_j + R, 0 < |d| <= rc, over every lattice
    image R (so rc may exceed L/2).  Returns i, j, d (arrays).
    Positions are defined modulo L (the Green's function of eq. green is
    periodic); they are wrapped into [0, L) first so that the image range
    |R| <= ceil(rc/L) L covers every pair."""
    x = np.mod(np.asarray(x, dtype=np.float64), L)
    N = len(x)
    shifts = _image_shifts(L, rc)
    I, J, D = [], [], []
    for i in range(N):
        d = (x[i][None, None, :] - x[None, :, :]) + shifts[:, None, :]  # (S, N, 3)
        r = np.sqrt(np.einsum("snk,snk->sn", d, d))
        s_idx, j_idx = np.nonzero((r <= rc) & ((r > 0) | (np.arange(N)[None, :] != i)))
        I.append(np.full(len(j_idx), i))
        J.append(j_idx)
        D.append(d[s_idx, j_idx])
    return np.concatenate(I), np.concatenate(J), np.concatenate(D)


def real_block_dense(x, L, a, eta, xi, rc):
    """Dense 3N x 3N real-space mobility M_r (FP64).

    M_r^{ij} = (6 pi eta a)^-1 [ sum_{R: 0<|d|<=rc} F(|d|)(I - dd) + G(|d|) dd
                                 + delta_ij F_self I ],   d = x_i - x_j + R
    (eq. Mreal with Appendix A; self term eq. self).  Distinct particles at
    the same point get F(0) = G(0) = F_self, the r -> 0 limit."""
    x = np.asarray(x, dtype=np.float64)
    N = len(x)
    Mr = np.zeros((3 * N, 3 * N))
    I, J, D = real_pairs(x, L, xi, a, rc)
    if len(I):
        r = np.linalg.norm(D, axis=1)
        F, G = real_FG(r, xi, a)
        with np.errstate(invalid="ignore", divide="ignore"):
            dh = np.where(r[:, None] > 0, D / np.where(r > 0, r, 1.0)[:, None], 0.0)
        rr = dh[:, :, None] * dh[:, None, :]
        blocks = F[:, None, None] * (np.eye(3)[None] - rr) + G[:, None, None] * rr
        Mr4 = Mr.reshape(N, 3, N, 3)
        np.add.at(Mr4, (I, slice(None), J, slice(None)), blocks)
    Mr += real_self(xi, a) * np.eye(3 * N)
    return Mr / (6.0 * np.pi * eta * a)


def real_matvec_rows(x, v, rows, L, a, eta, xi, rc):
    """Rows of w = M_r v for the particles in `rows` (minimum image, rc < L/2),
    by brute force over all N particles: the exact per-row definition used
    to check large systems one output at a time."""
    if not rc < 0.5 * L:
        raise ValueError("real_matvec_rows needs rc < L/2 (minimum image)")
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((len(rows), 3))
    Fs = real_self(xi, a)
    for n, i in enumerate(rows):
        d = x[i] - x
        d -= L * np.round(d / L)
        r = np.sqrt(np.einsum("nk,nk->n", d, d))
        sel = np.nonzero(r <= rc)[0]
        sel = sel[sel != i]
        acc = Fs * v[i]
        if len(sel):
            rs = r[sel]
            F, G = real_FG(rs, xi, a)
            dh = np.where(rs[:, None] > 0, d[sel] / np.where(rs > 0, rs, 1.0)[:, None], 0.0)
            vj = v[sel]
            proj = np.einsum("nk,nk->n", dh, vj)
            acc = acc + np.sum(F[:, None] * vj + ((G - F) * proj)[:, None] * dh, axis=0)
        out[n] = acc
    return out / (6.0 * np.pi * eta * a)
