"""Error measures of the GPU parity tests (host arithmetic only).

A relative 2-norm over a whole 3N vector can hide one wrong particle: at
N = 1000 a single row off by 0.3 % moves it by only ~1e-4.  Every parity
check therefore also bounds the worst row.  A row's error is normalised by
the RMS row norm of the reference, not by the row's own norm, which is
arbitrarily small for some rows of a random vector; with uniformly spread
rounding or truncation error the worst row then sits at about 2.5 times the
2-norm error (the largest of N chi-distributed row norms over their RMS), so
a row bar of 10 times the vector bar passes every correct result and fails
any single row that is wrong by 10 bars.
"""
import numpy as np

ROW_FACTOR = 10.0


def rows3(a):
    return np.asarray(a, dtype=np.float64).reshape(-1, 3)


def rel(a, b):
    """||a - b||_2 / ||b||_2 over the whole vector."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def row_err(a, b):
    """max_i ||a_i - b_i|| / rms_j ||b_j|| over the 3-vectors of the rows."""
    A, B = rows3(a), rows3(b)
    d = np.linalg.norm(A - B, axis=1)
    rms = np.sqrt(np.mean(np.sum(B * B, axis=1)))
    return float(np.max(d) / rms)


def row_rel_own(a, b):
    """max_i ||a_i - b_i|| / ||b_i|| (rows whose norm is below a tenth of
    the RMS are measured against that tenth); reported, not asserted."""
    A, B = rows3(a), rows3(b)
    d = np.linalg.norm(A - B, axis=1)
    nb = np.linalg.norm(B, axis=1)
    rms = np.sqrt(np.mean(nb * nb))
    return float(np.max(d / np.maximum(nb, 0.1 * rms)))


def check(a, b, bar, label="", row_bar=None, skip_rows=None):
    """Assert the 2-norm error <= bar and the worst-row error <= row_bar
    (default ROW_FACTOR * bar); rows flagged in skip_rows (a boolean mask)
    are left out of the worst-row bound only.  Returns (2-norm error,
    worst-row error)."""
    e, o = rel(a, b), row_rel_own(a, b)
    A, B = rows3(a), rows3(b)
    keep = np.ones(len(B), bool) if skip_rows is None else ~np.asarray(skip_rows, bool)
    r = row_err(A[keep], B[keep]) if keep.any() else 0.0
    rb = ROW_FACTOR * bar if row_bar is None else row_bar
    sk = "" if skip_rows is None else f", {int((~keep).sum())} row(s) with a pair at the cutoff left out"
    print(f"{label}: rel err {e:.2e} (bar {bar:.1e}), worst row {r:.2e} (bar {rb:.1e}), "
          f"worst row / own norm {o:.2e}{sk}", flush=True)
    assert e <= bar, f"{label}: rel err {e:.3e} > {bar:.1e}"
    assert r <= rb, f"{label}: worst row {r:.3e} > {rb:.1e}"
    return e, r


def cutoff_rows(x, L, rc, rows=None, delta=None):
    """Rows (of `rows`, or all) with a partner at |r - rc| < delta.  The
    near-field sum includes a pair when r <= rc: a pair that close to the
    cutoff is in or out depending on rounding (FP32 positions of a box of
    side L carry ~L 2^-24 of it), and M_r jumps there by the pair's F(rc),
    G(rc) (up to exp(-xi^2 rc^2) of the self term: 1e-3 at a 1e-3
    tolerance).  Such rows are compared in the 2-norm but not row by row.
    delta defaults to 8 L 2^-24."""
    from scipy.spatial import cKDTree

    x = np.mod(np.asarray(x, dtype=np.float64), L)
    x[x >= L] = 0.0
    if delta is None:
        delta = 8.0 * L * 2.0**-24
    t = cKDTree(x, boxsize=L)
    q = x if rows is None else x[np.asarray(rows)]
    hi = t.query_ball_point(q, rc + delta, return_length=True)
    lo = t.query_ball_point(q, rc - delta, return_length=True)
    return np.asarray(hi) != np.asarray(lo)

# FP32 near-field product against the FP64 definition: linear interpolation
# between table nodes rc/2048 apart errs by at most max|F''| dr^2 / 8, which
# is 0.8e-6 of |M_r v| at volume fraction 0.1 (rc = 8a) plus FP32 rounding;
# denser suspensions put more pairs near contact, where F'' is largest
# (about 2e-6 at volume fraction 0.4).
FP32_NEAR_BAR = 2e-6
# With most pairs near contact (volume fraction 0.3 - 0.4) the interpolation
# error of a host emulation of the same table is 1.6e-6 - 2.1e-6, and the
# FP32 positions of large boxes (L up to 350a: rounding up to 2e-5 a) add
# about as much again.
FP32_NEAR_BAR_DENSE = 6e-6
