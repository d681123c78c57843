"""Wave-space part of the positively split RPY mobility, FP64 (oracle).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.

Conventions.  The box is cubic with side L and volume V = L^3.  A k-set is
given as integer triples j (k = 2 pi j / L).  Grid arrays over an M^3 grid are
indexed in the usual DFT order (index n stands for the signed frequency n for
n < M/2 and n - M otherwise).
"""
import numpy as np

from .rpy import H_split, _sinc2


def B_kernel(k2, a, xi):
    """sinc^2(ka) H(k, xi) / k^2, the non-negative wave-space factor of
    eq. (Mwave) (Sec. II B.2 writes B with the extra 1/(eta V))."""
    k2 = np.asarray(k2, dtype=np.float64)
    k = np.sqrt(k2)
    return _sinc2(k * a) * H_split(k, xi) / k2


def kset_grid(M):
    """Integer wave vectors of an M^3 grid with k = 0 and every Nyquist
    index (|j_d| = M/2) removed: j_d in [-(M/2-1), M/2-1].  The k = 0 mode is
    excluded by eq. (green); the Nyquist modes have no conjugate partner on
    the grid, so they are left out to keep the sample real."""
    h = M // 2 - 1
    r = np.arange(-h, h + 1)
    J = np.array(np.meshgrid(r, r, r, indexing="ij")).reshape(3, -1).T
    return J[np.any(J != 0, axis=1)]


def kset_converged(L, xi, eps=1e-17):
    """All nonzero lattice wave vectors with exp(-k^2/4xi^2) > eps (the wave
    sum of eq. Mwave converged to rounding)."""
    kc = 2.0 * xi * np.sqrt(-np.log(eps))
    n = int(np.ceil(kc * L / (2 * np.pi)))
    r = np.arange(-n, n + 1)
    J = np.array(np.meshgrid(r, r, r, indexing="ij")).reshape(3, -1).T
    k2 = (2 * np.pi / L) ** 2 * np.sum(J * J, axis=1)
    return J[(k2 > 0) & (k2 <= kc * kc)]


def wave_block_dense(x, L, a, eta, xi, J, chunk=20000):
    """Dense 3N x 3N wave-space mobility over the k-set J, eq. (Mwave):

        M_w^{ij} = (1/eta V) sum_k cos(k.(x_i - x_j)) B(k) (I - k k / k^2)

    (the sum over +-k of e^{ik.(x_i-x_j)} is real, so the cosine form is
    the same sum)."""
    x = np.asarray(x, dtype=np.float64)
    N = len(x)
    V = L**3
    out = np.zeros((3, 3, N, N))
    for s in range(0, len(J), chunk):
        k = (2 * np.pi / L) * J[s : s + chunk].astype(np.float64)
        k2 = np.sum(k * k, axis=1)
        B = B_kernel(k2, a, xi)
        ph = x @ k.T
        C, S = np.cos(ph), np.sin(ph)
        for p in range(3):
            for q in range(3):
                w = B * ((p == q) - k[:, p] * k[:, q] / k2)
                out[p, q] += (C * w) @ C.T + (S * w) @ S.T
    return out.transpose(2, 0, 3, 1).reshape(3 * N, 3 * N) / (eta * V)


# ---------------------------------------------------------------------------
# direct non-uniform Fourier sums over the grid k-set
# ---------------------------------------------------------------------------
def _signed(M):
    return np.fft.fftfreq(M, 1.0 / M)  # 0, 1, ..., M/2-1, -M/2, ..., -1


def grid_kvectors(M, L):
    """k components along one axis (DFT order) and the mask of the grid
    k-set (no k = 0, no Nyquist index)."""
    j = _signed(M)
    kx = 2 * np.pi * j / L
    ok1 = np.abs(j) != M // 2
    KX, KY, KZ = np.meshgrid(kx, kx, kx, indexing="ij")
    OK = ok1[:, None, None] & ok1[None, :, None] & ok1[None, None, :]
    K2 = KX**2 + KY**2 + KZ**2
    OK &= K2 > 0
    return KX, KY, KZ, K2, OK


def project(KX, KY, KZ, K2, Z):
    """(I - k k / k^2) applied to the 3-vector field Z[c] (c = x, y, z)."""
    K2s = np.where(K2 > 0, K2, 1.0)
    kdz = KX * Z[0] + KY * Z[1] + KZ * Z[2]
    return np.stack([Z[0] - KX * kdz / K2s, Z[1] - KY * kdz / K2s, Z[2] - KZ * kdz / K2s])


def _phases(xcol, M, L):
    """e^{i k_d x_d} for every particle (rows) and grid frequency (cols)."""
    j = _signed(M)
    return np.exp(1j * (2 * np.pi / L) * np.outer(xcol, j))


def nudft_type2(x, Uhat, L, chunk=64):
    """u_i = sum_k e^{i k.x_i} Uhat[:, k] over the whole grid array Uhat[3,M,M,M]
    (already zero off the k-set), evaluated directly with separable phases.
    Returns the real part (the sums used here are real by conjugate symmetry;
    Re only removes rounding)."""
    x = np.asarray(x, dtype=np.float64)
    M = Uhat.shape[1]
    out = np.zeros((len(x), 3))
    for s in range(0, len(x), chunk):
        xs = x[s : s + chunk]
        ex, ey, ez = _phases(xs[:, 0], M, L), _phases(xs[:, 1], M, L), _phases(xs[:, 2], M, L)
        t = np.einsum("cabd,nd->cabn", Uhat, ez, optimize=True)
        t = np.einsum("cabn,nb->can", t, ey, optimize=True)
        t = np.einsum("can,na->cn", t, ex, optimize=True)
        out[s : s + chunk] = np.real(t).T
    return out


def nudft_type1(x, F, M, L, chunk=64):
    """Fhat[c, k] = sum_j e^{-i k.x_j} F_j[c] on the full M^3 grid of k (DFT order)."""
    x = np.asarray(x, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64).reshape(-1, 3)
    Fhat = np.zeros((3, M, M, M), dtype=np.complex128)
    for s in range(0, len(x), chunk):
        xs = x[s : s + chunk]
        ex = np.conj(_phases(xs[:, 0], M, L))
        ey = np.conj(_phases(xs[:, 1], M, L))
        ez = np.conj(_phases(xs[:, 2], M, L))
        Fhat += np.einsum("nc,na,nb,nd->cabd", F[s : s + chunk], ex, ey, ez, optimize=True)
    return Fhat


def wave_sample_direct(x, zeta, L, a, eta, xi):
    """Wave-space sample (Sec. II B.2):

        y_i = sum_{k in K_grid} e^{i k.x_i} sqrt(B(k)/(eta V)) (I - kk) zeta(k)

    with zeta[3, M, M, M] a conjugate-symmetric complex field on the grid
    (zeta(-k) = conj zeta(k)), evaluated as a direct non-uniform Fourier sum.
    Covariance: E[y y^T] = M_w over K_grid when E[zeta zeta^H] = I."""
    M = zeta.shape[1]
    KX, KY, KZ, K2, OK = grid_kvectors(M, L)
    c = np.zeros_like(K2)
    c[OK] = np.sqrt(B_kernel(K2[OK], a, xi) / (eta * L**3))
    U = project(KX, KY, KZ, K2, zeta) * c[None]
    U[:, ~OK] = 0.0
    return nudft_type2(x, U, L)


def wave_apply_direct(x, F, M, L, a, eta, xi):
    """u = M_w F over the grid k-set, by direct sums (eq. Mwave):

        u_i = (1/eta V) sum_k e^{i k.x_i} B(k) (I - kk) sum_j e^{-i k.x_j} F_j
    """
    KX, KY, KZ, K2, OK = grid_kvectors(M, L)
    Fhat = nudft_type1(x, F, M, L)
    w = np.zeros_like(K2)
    w[OK] = B_kernel(K2[OK], a, xi) / (eta * L**3)
    U = project(KX, KY, KZ, K2, Fhat) * w[None]
    U[:, ~OK] = 0.0
    return nudft_type2(x, U, L)


def zeta_from_grid_noise(W):
    """Conjugate-symmetric unit-variance k-space noise from real white noise
    W[3, M, M, M] on the grid nodes: zeta = DFT(W) / M^{3/2}
    (E[zeta zeta^H] = I by unitarity of the scaled DFT)."""
    M = W.shape[1]
    return np.fft.fftn(W, axes=(1, 2, 3)) / M**1.5
