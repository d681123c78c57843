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


def check(a, b, bar, label="", row_bar=None):
    """Assert the 2-norm error <= bar and the worst-row error <= row_bar
    (default ROW_FACTOR * bar); returns (2-norm error, worst-row error)."""
    e, r, o = rel(a, b), row_err(a, b), row_rel_own(a, b)
    rb = ROW_FACTOR * bar if row_bar is None else row_bar
    print(f"{label}: rel err {e:.2e} (bar {bar:.1e}), worst row {r:.2e} (bar {rb:.1e}), "
          f"worst row / own norm {o:.2e}", flush=True)
    assert e <= bar, f"{label}: rel err {e:.3e} > {bar:.1e}"
    assert r <= rb, f"{label}: worst row {r:.3e} > {rb:.1e}"
    return e, r

# FP32 near-field product against the FP64 definition: linear interpolation
# of the F and G - F table between nodes rc/1024 apart errs by at most
# max|F''| dr^2 / 8 ~ 3e-6 relative (measured 3.1e-6), plus FP32 rounding.
FP32_NEAR_BAR = 1e-5
