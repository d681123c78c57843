"""Every compiled support size P of the Gaussian window (Sec. II C), against
the oracle's direct Fourier sums on the same inputs and noise:

- the wave-space sample M_w^{1/2} zeta (interpolation) and M_w F (spreading,
  then interpolation) at N = 1000, phi = 0.1, 64^3 (owner-computes spreading
  tiles), P = 2 ... 16;
- a 16^3 grid, where the tiles do not fit and spreading uses atomics, at
  P = 2 and 4 (FP64 against the oracle, FP32 against FP64);
- radix-3 grids, and a clustered configuration (a dense blob in a sparse
  box: tiles with several listing rounds beside empty tiles) on the
  matrix-core (FP32) and VALU (FP64) spreading tiles.

Bar: the window's error is the paper's quadrature bound at m = sqrt(pi P)
plus the aliasing estimate of the grid spacing (both computed on the host
from B(k) alone), times 3, plus a rounding floor of the precision.  At P = 8
the estimate gives 3.0e-5 for the sample and the kernels measure 3.0e-5."""
import numpy as np
import pytest

import synth
from oracle import ewald
from se_error import se_aliasing_estimate, se_quadrature_bound

pytestmark = pytest.mark.gpu

XI, RC = 0.5, 8.0
FLOOR = {"fp64": 1e-11, "fp32": 1e-5}


from parity import check


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def dev(a, dtype):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def bar(L, M, P, precision):
    return 3.0 * (se_quadrature_bound(P) + se_aliasing_estimate(L, M, XI, P)) + FLOOR[precision]


@pytest.fixture(scope="module")
def box64():
    x, L = synth.hard_spheres(1000, 0.1, seed=1000)
    M = 64
    W = synth.normals(3, (3, M, M, M))
    F = synth.normals(4, (len(x), 3))
    y_ref = ewald.wave_sample_direct(x, ewald.zeta_from_grid_noise(W), L, 1.0, 1.0, XI)
    u_ref = ewald.wave_apply_direct(x, F, M, L, 1.0, 1.0, XI)
    return x, L, M, W, F, y_ref, u_ref


@pytest.mark.parametrize("P", [2, 4, 6, 10, 12, 14, 16])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_support_size_matches_direct_sums(gpu_lib, box64, P, precision):
    x, L, M, W, F, y_ref, u_ref = box64
    s = gpu_lib.Sampler(len(x), L, xi=XI, rcut=RC, grid=M, support=P, tol=1e-6, precision=precision)
    s.set_positions(dev(x, s.dtype))
    y = host(s.wave_sample(dev(W, s.dtype)))
    u = host(s.wave_apply(dev(F, s.dtype)))
    s.close()
    b = bar(L, M, P, precision)
    check(y, y_ref, b, f"P={P} {precision} sample")
    check(u, u_ref, b, f"P={P} {precision} apply")


@pytest.mark.parametrize("P", [2, 4])
def test_atomic_spreading_on_small_grids(gpu_lib, P):
    x, L = synth.hard_spheres(300, 0.1, seed=1200)
    M = 16
    W = synth.normals(5, (3, M, M, M))
    F = synth.normals(6, (len(x), 3))
    out = {}
    for precision in ("fp64", "fp32"):
        s = gpu_lib.Sampler(len(x), L, xi=XI, rcut=RC, grid=M, support=P, tol=1e-6, precision=precision)
        s.set_positions(dev(x, s.dtype))
        out[precision] = (host(s.wave_sample(dev(W, s.dtype))), host(s.wave_apply(dev(F, s.dtype))))
        s.close()
    y_ref = ewald.wave_sample_direct(x, ewald.zeta_from_grid_noise(W), L, 1.0, 1.0, XI)
    u_ref = ewald.wave_apply_direct(x, F, M, L, 1.0, 1.0, XI)
    (y64, u64), (y32, u32) = out["fp64"], out["fp32"]
    b = bar(L, M, P, "fp64")
    check(y64, y_ref, b, f"M=16 P={P} sample")
    check(u64, u_ref, b, f"M=16 P={P} apply")
    check(y32, y64, FLOOR["fp32"], f"M=16 P={P} sample fp32 vs fp64")
    check(u32, u64, FLOOR["fp32"], f"M=16 P={P} apply fp32 vs fp64")


@pytest.mark.parametrize("M", [24, 48, 96, 192])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_radix3_grids_match_direct_sums(gpu_lib, M, precision):
    """Grids of 3 x 2^k points (mixed radix-2/3 FFT plans): the wave sample
    and M_w F against the direct Fourier sums over the same k-set; boxes sized
    so that h is about 0.6a (VALU spreading tiles on 24^3 and in FP64,
    matrix-core tiles from 48^3 up in FP32)."""
    n = {24: 60, 48: 400, 96: 1000, 192: 800}[M]
    L = 0.6 * M
    x = synth.uniform_positions(n, L, seed=1300 + M)
    W = synth.normals(1301 + M, (3, M, M, M))
    F = synth.normals(1302 + M, (n, 3))
    rc = min(RC, 0.49 * L)
    s = gpu_lib.Sampler(n, L, xi=XI, rcut=rc, grid=M, support=8, tol=1e-6, precision=precision)
    s.set_positions(dev(x, s.dtype))
    y = host(s.wave_sample(dev(W, s.dtype)))
    u = host(s.wave_apply(dev(F, s.dtype)))
    s.close()
    y_ref = ewald.wave_sample_direct(x, ewald.zeta_from_grid_noise(W), L, 1.0, 1.0, XI)
    u_ref = ewald.wave_apply_direct(x, F, M, L, 1.0, 1.0, XI)
    b = bar(L, M, 8, precision)
    check(y, y_ref, b, f"M={M} {precision} sample")
    check(u, u_ref, b, f"M={M} {precision} apply")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_clustered_particles_and_empty_tiles(gpu_lib, precision):
    """A dense blob (1200 spheres at phi = 0.45 in a 22a cube) in a 48a box
    with 300 spheres scattered around it, 64^3: the tiles over the blob list
    several hundred candidates (several listing rounds of the tiled
    spreading), most other tiles none.  M_w F and the wave sample against
    the direct Fourier sums."""
    blob, L0 = synth.hard_spheres(1200, 0.45, seed=1400)
    L, M = 48.0, 64
    x = np.concatenate([blob + 3.0, synth.uniform_positions(300, L, seed=1401)])
    n = len(x)
    W = synth.normals(1402, (3, M, M, M))
    F = synth.normals(1403, (n, 3))
    s = gpu_lib.Sampler(n, L, xi=XI, rcut=RC, grid=M, support=8, tol=1e-6, precision=precision)
    s.set_positions(dev(x, s.dtype))
    y = host(s.wave_sample(dev(W, s.dtype)))
    u = host(s.wave_apply(dev(F, s.dtype)))
    s.close()
    y_ref = ewald.wave_sample_direct(x, ewald.zeta_from_grid_noise(W), L, 1.0, 1.0, XI)
    u_ref = ewald.wave_apply_direct(x, F, M, L, 1.0, 1.0, XI)
    b = bar(L, M, 8, precision)
    print(f"blob side {L0:.1f}a", flush=True)
    check(y, y_ref, b, f"clustered {precision} sample")
    check(u, u_ref, b, f"clustered {precision} apply")
