"""Learned block preconditioner of the real-space Krylov sample, FP64 (oracle).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.

The unpreconditioned real-space sample of Sec. II B.1 is M_r^{1/2} z by
Lanczos.  With an invertible block-diagonal P (one 3x3 block per particle)
the Krylov iteration can run on A = P M_r P^T instead, and

    y = P^{-1} A^{1/2} z

has covariance P^{-1} A P^{-T} = M_r, the same law as the plain sample (a
different square root of M_r).  P is predicted per particle by a small MLP
from 24 geometry features of the particle's near field.  The paper uses no
preconditioner; the features, the network and the training target below are
this library's definitions (stated in the design notes), restated here in
plain FP64 so that the device kernels can be checked against them.

Features of particle i, over its near neighbours j (minimum image,
0 <= r < 4.5a, d = x_i - x_j, r = |d|, dh = d / r, and dh = 0 when r = 0),
with F, G the dimensionless Appendix A functions; only f3 counts every
neighbour within rc:

    f0..f3    #{r < 2.2a} / 4, #{r < 3a} / 8, #{r < 4.5a} / 16, #{r <= rc} / 128
    f4        sum F(r) / 8
    f5..f10   sum (G - F)(r) dh dh^T   (xx, yy, zz, xy, xz, yz)
    f11..f16  sum_{r < 3a} dh dh^T      (xx, yy, zz, xy, xz, yz) / 4
    f17..f19  sum_{r < 3a} dh           / 4
    f20       sum (G - F)(r)
    f21       min(r) / 4.5a  (1 if there is no near neighbour)
    f22       sum_{r < 3a} (3a - r) / a / 4
    f23       F_self (eq. self)

Network (bf16 weights, inputs and hidden activations; fp32 sums):
    h1 = relu(W1 x + b1)  (64),  h2 = relu(W2 h1 + b2)  (64),  y = W3 h2 + b3 (9)
    P_i = I + y reshaped row-major to 3 x 3.
A block falls back to I when it is not finite, when |det P_i| < 1e-6, or
when ||P_i||_F ||P_i^{-1}||_F > 1e3 (this product lies between cond_2 and
3 cond_2).

Training target: T_i = ([M_patch^{-1}]_ii)^{1/2} (symmetric root of the ii
block of the inverse of M_r restricted to i and its neighbours within the
patch radius), normalised by its isolated-particle value (mu0 F_self)^{-1/2},
so that an isolated particle has target I; the regression target of y is
T_i / s - I, squared error summed over the 9 entries.
"""
import numpy as np

from . import rpy

NFEAT = 24
NH = 64
NOUT = 9


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------
def features(x, L, a, xi, rc):
    """(N, 24) FP64 features, definitions in the module docstring."""
    if not rc < 0.5 * L:
        raise ValueError("features need rc < L/2 (minimum image)")
    x = np.mod(np.asarray(x, dtype=np.float64), L)
    N = len(x)
    f = np.zeros((N, NFEAT))
    Fs = rpy.real_self(xi, a)
    for i in range(N):
        d = x[i][None, :] - x
        d -= L * np.round(d / L)
        r = np.sqrt(np.einsum("nk,nk->n", d, d))
        sel = (r <= rc) & (np.arange(N) != i)
        nall = int(np.sum(sel))
        sel &= r < 4.5 * a
        d, r = d[sel], r[sel]
        F, G = rpy.real_FG(r, xi, a) if len(r) else (np.zeros(0), np.zeros(0))
        with np.errstate(invalid="ignore", divide="ignore"):
            dh = np.where(r[:, None] > 0, d / np.where(r > 0, r, 1.0)[:, None], 0.0)
        near = r < 3.0 * a
        comps = lambda w, u: np.array([
            np.sum(w * u[:, 0] * u[:, 0]), np.sum(w * u[:, 1] * u[:, 1]), np.sum(w * u[:, 2] * u[:, 2]),
            np.sum(w * u[:, 0] * u[:, 1]), np.sum(w * u[:, 0] * u[:, 2]), np.sum(w * u[:, 1] * u[:, 2])])
        f[i, 0] = np.sum(r < 2.2 * a) / 4.0
        f[i, 1] = np.sum(near) / 8.0
        f[i, 2] = np.sum(r < 4.5 * a) / 16.0
        f[i, 3] = nall / 128.0
        f[i, 4] = np.sum(F) / 8.0
        f[i, 5:11] = comps(G - F, dh)
        f[i, 11:17] = comps(near.astype(np.float64), dh) / 4.0
        f[i, 17:20] = np.sum(dh[near], axis=0) / 4.0
        f[i, 20] = np.sum(G - F)
        f[i, 21] = (np.min(r) / (4.5 * a)) if len(r) else 1.0
        f[i, 22] = np.sum((3.0 * a - r[near]) / a) / 4.0
        f[i, 23] = Fs
    return f


# ---------------------------------------------------------------------------
# bf16 rounding (round to nearest even on the float32 value)
# ---------------------------------------------------------------------------
def bf16_round(v):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    NaN stays NaN; the float32 value is rounded on its bit pattern."""
    f = np.asarray(v, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def init_weights(seed, scale=0.1):
    """A seeded weight set {W1 (64,24), b1, W2 (64,64), b2, W3 (9,64), b3}."""
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.standard_normal((NH, NFEAT)) * scale,
        "b1": rng.standard_normal(NH) * scale,
        "W2": rng.standard_normal((NH, NH)) * scale,
        "b2": rng.standard_normal(NH) * scale,
        "W3": rng.standard_normal((NOUT, NH)) * scale,
        "b3": rng.standard_normal(NOUT) * scale,
    }


def mlp_forward(w, x, bf16=True):
    """y (N, 9) and the cache (x, h1, h2).  With bf16, weights, inputs and the
    hidden activations are rounded to bfloat16 where the device stores them;
    sums are exact (FP64)."""
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = (rnd(w[k]) for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    x = rnd(x)
    h1 = rnd(np.maximum(x @ W1.T + b1, 0.0))
    h2 = rnd(np.maximum(h1 @ W2.T + b2, 0.0))
    y = h2 @ W3.T + b3
    return y, (x, h1, h2)


def mlp_backward(w, cache, dy):
    """Gradients of sum_n <dy_n, y_n> with respect to every weight (FP64),
    by the chain rule through relu (derivative 1 where the activation is > 0)."""
    x, h1, h2 = cache
    W2, W3 = np.asarray(w["W2"], np.float64), np.asarray(w["W3"], np.float64)
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    d2 = (dy @ W3) * (h2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ W2) * (h1 > 0)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(0)
    return g


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) of the arrays p in place, with
    bias-corrected first and second moments; returns nothing."""
    m *= b1
    m += (1.0 - b1) * g
    v *= b2
    v += (1.0 - b2) * g * g
    mh = m / (1.0 - b1**t)
    vh = v / (1.0 - b2**t)
    p -= lr * mh / (np.sqrt(vh) + eps)


# ---------------------------------------------------------------------------
# blocks, fallback, preconditioned sample
# ---------------------------------------------------------------------------
def blocks_from_output(y):
    """P_i = I + y_i (row-major 3 x 3) with the per-particle fallback to I.
    Returns (P (N,3,3), fallback mask)."""
    y = np.asarray(y, dtype=np.float64)
    P = np.eye(3)[None] + y.reshape(-1, 3, 3)
    bad = ~np.all(np.isfinite(P), axis=(1, 2))
    Pz = np.where(bad[:, None, None], np.eye(3)[None], P)
    det = np.linalg.det(Pz)
    bad |= np.abs(det) < 1e-6
    Pz = np.where(bad[:, None, None], np.eye(3)[None], Pz)
    cond = np.linalg.norm(Pz, axis=(1, 2)) * np.linalg.norm(np.linalg.inv(Pz), axis=(1, 2))
    bad |= cond > 1e3
    return np.where(bad[:, None, None], np.eye(3)[None], P), bad


def block_diag(P):
    N = len(P)
    B = np.zeros((3 * N, 3 * N))
    for i in range(N):
        B[3 * i:3 * i + 3, 3 * i:3 * i + 3] = P[i]
    return B


def precond_real_sample(Mr, P, z):
    """y = P^{-1} (P M_r P^T)^{1/2} z with the symmetric root of A = P M_r P^T
    by eigendecomposition (LAPACK)."""
    B = block_diag(P)
    A = B @ Mr @ B.T
    A = 0.5 * (A + A.T)
    lam, Q = np.linalg.eigh(A)
    s = Q @ (np.sqrt(np.maximum(lam, 0.0)) * (Q.T @ np.ravel(z)))
    return np.linalg.solve(B, s)


# ---------------------------------------------------------------------------
# training target
# ---------------------------------------------------------------------------
def _sqrtm_spd(S):
    lam, Q = np.linalg.eigh(0.5 * (S + S.T))
    return (Q * np.sqrt(np.maximum(lam, 0.0))) @ Q.T


def targets(x, idx, L, a, eta, xi, rc, radius=None):
    """Normalised targets T_i / s for the particles in idx (module docstring);
    radius defaults to rc.  Returns (len(idx), 3, 3)."""
    radius = rc if radius is None else radius
    x = np.mod(np.asarray(x, dtype=np.float64), L)
    s = (rpy.real_self(xi, a) / (6.0 * np.pi * eta * a)) ** -0.5
    out = []
    for i in idx:
        d = x[i][None, :] - x
        d -= L * np.round(d / L)
        r = np.sqrt(np.einsum("nk,nk->n", d, d))
        patch = np.concatenate([[i], np.nonzero((r <= radius) & (np.arange(len(x)) != i))[0]])
        Mp = rpy.real_block_dense(x[patch], L, a, eta, xi, rc)
        E = np.zeros((3 * len(patch), 3))
        E[:3] = np.eye(3)
        X = np.linalg.solve(Mp, E)
        out.append(_sqrtm_spd(X[:3]) / s)
    return np.array(out)
