"""The tolerance experiment of Sec. II C (Fig. parity): the relative error of
the mobility product U = M F for a random suspension of 5000 hard spheres
(volume fraction 0.2) under a uniform sedimentation force, against the
result computed at a 1e-10 tolerance, as the requested tolerance varies, for
several xi.  The parameters (rc, grid, support) come from the library's error
model for each tolerance (pse_choose_params with xi fixed); the claim checked
is the paper's: the error stays at or below the requested tolerance.

The exact mobility does not depend on xi (M_r + M_w = M for every split,
pinned on the oracle), so one reference at xi a = 0.5 serves every xi; that
reference is itself checked against the oracle's direct sums on 300 rows."""
import numpy as np
import pytest

import synth
from oracle import ewald, rpy
from parity import check, rel

pytestmark = pytest.mark.gpu

N, PHI = 5000, 0.2


@pytest.fixture(scope="module")
def susp():
    x, L = synth.hard_spheres(N, PHI, seed=1500, sweeps=50)
    F = np.zeros((N, 3))
    F[:, 2] = -1.0
    return x, L, F


def mobility(gpu_lib, x, L, F, tol, xi, precision="fp64"):
    import torch

    base = gpu_lib.make_params(N, L, precision=precision)
    p, info = gpu_lib.pse_choose_params(base, gpu_lib.Tuning(tol=tol, xi=xi, max_grid=512, with_forces=1, deterministic=1))
    p.lanczos_max_iter = 64
    s = gpu_lib.Sampler(N, L, params=p)
    dt = s.dtype
    s.set_positions(torch.as_tensor(x, dtype=dt, device="cuda"))
    u = s.mobility_apply(torch.as_tensor(F, dtype=dt, device="cuda"))
    torch.cuda.synchronize()
    out = u.double().cpu().numpy()
    s.close()
    return out, p


@pytest.fixture(scope="module")
def exact(gpu_lib, susp):
    x, L, F = susp
    u, p = mobility(gpu_lib, x, L, F, 1e-10, 0.5)
    print(f"reference: xi={p.xi} rc={p.rcut:.2f} grid={p.grid} P={p.support}", flush=True)
    return u, p


def test_reference_matches_the_oracle(gpu_lib, susp, exact):
    """The tol-1e-10 reference on 300 rows: near field by brute force
    (eq. Mreal) and wave part by the direct Fourier sums over its grid's
    k-set (eq. Mwave)."""
    x, L, F = susp
    u, p = exact
    rows = np.sort(np.random.default_rng(3).choice(N, 300, replace=False))
    ur = rpy.real_matvec_rows(x, F, rows, L, 1.0, 1.0, p.xi, p.rcut)
    uw = ewald.wave_apply_direct(x, F, p.grid, L, 1.0, 1.0, p.xi)[rows]
    check(u[rows], ur + uw, 1e-9, "tol-1e-10 reference vs oracle rows")


@pytest.mark.parametrize("xi", [0.3, 0.5, 0.7])
def test_error_stays_below_the_tolerance(gpu_lib, susp, exact, xi):
    x, L, F = susp
    u_ex, _ = exact
    errs = {}
    for tol in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7):
        u, p = mobility(gpu_lib, x, L, F, tol, xi)
        errs[tol] = e = rel(u, u_ex)
        print(f"xi a={xi} tol {tol:.0e}: error {e:.2e} (rc={p.rcut:.2f}, grid {p.grid}, P={p.support}, "
              f"m={p.gauss_m:.2f})", flush=True)
    assert all(e <= tol for tol, e in errs.items()), errs


def test_fp32_error_floor(gpu_lib, susp, exact):
    """FP32 storage: the same control down to the single-precision floor."""
    x, L, F = susp
    u_ex, _ = exact
    errs = {}
    for tol in (1e-2, 1e-3, 1e-4):
        u, p = mobility(gpu_lib, x, L, F, tol, 0.5, precision="fp32")
        errs[tol] = e = rel(u, u_ex)
        print(f"fp32 tol {tol:.0e}: error {e:.2e} (grid {p.grid}, P={p.support}, m={p.gauss_m:.2f})", flush=True)
    assert all(e <= tol for tol, e in errs.items()), errs
