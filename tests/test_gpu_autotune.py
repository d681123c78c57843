"""Launch-shape autotuning (pse_autotune, pse_batch_autotune): the choices
are valid launch shapes for the grid, the tuned wave-space sample agrees
with the built-in one to rounding (only the order in which a node sums its
particles may change), and stays within the oracle bar of the direct
Fourier sum."""
import numpy as np
import pytest

import synth
from oracle import ewald

pytestmark = pytest.mark.gpu

XI, RC, P = 0.5, 8.0, 8


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("n,phi,grid,precision", [(1000, 0.1, 64, "fp32"), (1000, 0.1, 64, "fp64"),
                                                   (6000, 0.3, 64, "mixed"), (20000, 0.3, 128, "mixed")])
def test_autotune_choice_valid_and_sample_unchanged(gpu_lib, n, phi, grid, precision):
    import torch

    x, L = synth.hard_spheres(n, phi, seed=2100 + n, sweeps=5)
    s = gpu_lib.Sampler(n, L, xi=XI, rcut=RC, grid=grid, support=P, tol=1e-6, precision=precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    s.set_positions(torch.as_tensor(x, dtype=dt, device="cuda"))
    W = synth.normals(2200 + n, (3, grid, grid, grid))
    Wd = torch.as_tensor(W, dtype=dt, device="cuda")
    y0 = host(s.wave_sample(Wd))
    depth, lanes = s.autotune()
    print(f"n={n} M={grid} {precision}: spreading tile depth {depth}, interpolation lanes {lanes}", flush=True)
    assert lanes in (256, 512, 1024)
    assert depth in (8, 16, 32, 64)
    assert grid % depth == 0 and grid >= 2 * max(8, depth) + P
    y1 = host(s.wave_sample(Wd))
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert rel(y1, y0) < tol
    if n <= 1000:
        y_ref = ewald.wave_sample_direct(x, ewald.zeta_from_grid_noise(W), L, 1.0, 1.0, XI)
        assert rel(y1, y_ref) < 1e-4
    s.close()


def test_autotune_needs_positions(gpu_lib):
    x, L = synth.hard_spheres(500, 0.1, seed=2300)
    s = gpu_lib.Sampler(500, L, xi=XI, rcut=RC, grid=64, support=P, precision="fp32")
    with pytest.raises(gpu_lib.PSEError):
        s.autotune()
    s.close()


def test_batch_autotune(gpu_lib):
    import torch

    specs, pos = [], []
    for k, (n, phi, M) in enumerate([(2000, 0.2, 64), (3000, 0.3, 64), (9000, 0.3, 128)]):
        x, L = synth.hard_spheres(n, phi, seed=2400 + k, sweeps=5)
        specs.append(dict(n=n, box=L, xi=XI, rcut=RC, grid=M, support=P, tol=1e-6, precision="mixed"))
        pos.append(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
    b = gpu_lib.Batch(specs)
    b.set_positions(pos)
    out0, _ = b.sample(5, 0, dt=0.01)
    y0 = [host(o) for o in out0]
    b.autotune()
    out1, st = b.sample(5, 0, dt=0.01)
    for r, o in enumerate(out1):
        y1 = host(o)
        assert np.all(np.isfinite(y1))
        assert rel(y1, y0[r]) < 1e-5, r
    b.close()
