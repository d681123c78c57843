"""Square roots of SPD matrices (oracle).

TEST INFRASTRUCTURE ONLY.

sqrt_apply     the symmetric square root A^{1/2} z = Q diag(sqrt(lam)) Q^T z by
               LAPACK eigendecomposition: the exact object the real-space
               Krylov sample approximates (Sec. II B.1).
lanczos_sqrt   Krylov (Lanczos) approximation of A^{1/2} z after Chow and Saad
               (ref. chow-saad, used in Sec. II B.1), with full
               re-orthogonalisation so that its iterates are the ones exact
               arithmetic would produce.
"""
import numpy as np


def sqrt_apply(A, z):
    """A^{1/2} z with the symmetric root of a symmetric positive (semi)definite
    A.  Eigenvalues below zero that come only from rounding are clipped."""
    lam, Q = np.linalg.eigh(A)
    lam = np.clip(lam, 0.0, None)
    return Q @ (np.sqrt(lam) * (Q.T @ z))


def tridiag_sqrt_e1(alpha, beta):
    """s = T^{1/2} e_1 for the symmetric tridiagonal T with diagonal alpha and
    off-diagonal beta (len(beta) = len(alpha) - 1)."""
    m = len(alpha)
    T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1) if m > 1 else np.array([[alpha[0]]])
    lam, Q = np.linalg.eigh(T)
    lam = np.clip(lam, 0.0, None)
    return Q @ (np.sqrt(lam) * Q[0])


def lanczos_sqrt(matvec, z, tol, max_iter=64, breakdown=1e-12):
    """Krylov approximation y_m = ||z|| V_m T_m^{1/2} e_1 of A^{1/2} z.

    Lanczos three-term recurrence on v_1 = z/||z||; after step m the iterate
    is y_m; stop when ||y_m - y_{m-1}|| <= tol ||y_m|| (the successive-iterate
    criterion of Chow-Saad), or when the next Lanczos vector vanishes
    (beta_m <= breakdown * ||A v|| : the Krylov space is invariant, y_m is exact).
    Full re-orthogonalisation keeps V_m orthonormal.

    Returns (y, iterations, history) with history the list of iterates."""
    z = np.asarray(z, dtype=np.float64)
    b0 = np.linalg.norm(z)
    if b0 == 0.0:
        return np.zeros_like(z), 0, []
    V = [z / b0]
    alpha, beta = [], []
    hist = []
    y_prev = None
    for m in range(1, max_iter + 1):
        w = matvec(V[-1])
        wn = np.linalg.norm(w)
        if m > 1:
            w = w - beta[-1] * V[-2]
        alpha.append(float(V[-1] @ w))
        w = w - alpha[-1] * V[-1]
        Vm = np.array(V)
        w = w - Vm.T @ (Vm @ w)
        w = w - Vm.T @ (Vm @ w)
        bm = float(np.linalg.norm(w))
        s = tridiag_sqrt_e1(np.array(alpha), np.array(beta))
        y = b0 * (Vm.T @ s)
        hist.append(y)
        if bm <= breakdown * max(wn, 1e-300):
            return y, m, hist
        if y_prev is not None and np.linalg.norm(y - y_prev) <= tol * np.linalg.norm(y):
            return y, m, hist
        y_prev = y
        beta.append(bm)
        V.append(w / bm)
    return hist[-1], max_iter, hist
