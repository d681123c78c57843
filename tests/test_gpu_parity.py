"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same
seeded inputs and noise.

Tolerances: real-space product 1e-12 (FP64) / 2e-6 (FP32 table); Krylov
sample within its Lanczos tolerance; wave-space sample and M_w F within 1e-4
relative (the Spectral-Ewald quadrature error at P = 8 is ~4e-6, Sec. II C);
Philox noise is bit-identical on both sides, so full samples match to the
same bars.
"""
import numpy as np
import pytest

import synth
from oracle import ewald, lanczos, philox, rpy, sampler

pytestmark = pytest.mark.gpu


from parity import FP32_NEAR_BAR, FP32_NEAR_BAR_DENSE, check


def to_dev(x, dtype):
    import torch

    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.double().cpu().numpy()


# ----------------------------------------------------- config 0 (FP64, N=1000)
XI, RC, M0, P = 0.5, 8.0, 64, 8


@pytest.fixture(scope="module")
def cfg0():
    x, L = synth.hard_spheres(1000, 0.1, seed=1000)
    Mr = rpy.real_block_dense(x, L, 1.0, 1.0, XI, RC)
    return x, L, Mr


def make(gpu_lib, n, L, precision, grid=M0, tol=1e-6, xi=XI, rc=RC, support=P, max_iter=64, kT=1.0, eta=1.0):
    return gpu_lib.Sampler(n, L, a=1.0, eta=eta, kT=kT, xi=xi, rcut=rc, grid=grid, support=support, tol=tol,
                           max_iter=max_iter, precision=precision)


# FP32 bar: linear interpolation between the 2050 nodes of the F, G table on
# [0, rc] (see parity.FP32_NEAR_BAR).
@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("fp32", FP32_NEAR_BAR), ("mixed", FP32_NEAR_BAR)])
def test_real_matvec_matches_dense_oracle(gpu_lib, cfg0, precision, bar):
    x, L, Mr = cfg0
    s = make(gpu_lib, len(x), L, precision)
    s.set_positions(to_dev(x, s.dtype))
    v = synth.normals(1, (len(x), 3))
    w = host(s.real_matvec(to_dev(v, s.dtype)))
    check(w, Mr @ v.ravel(), bar, f"real_matvec {precision}")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("mixed", 1e-4), ("fp32", 1e-4)])
def test_real_sample_matches_symmetric_root(gpu_lib, cfg0, precision, tol):
    x, L, Mr = cfg0
    s = make(gpu_lib, len(x), L, precision, tol=tol)
    s.set_positions(to_dev(x, s.dtype))
    z = synth.normals(2, (len(x), 3))
    y, st = s.real_sample(to_dev(z, s.dtype))
    y = host(y)
    y_ex = lanczos.sqrt_apply(Mr, z.ravel())
    _, it_ref, _ = lanczos.lanczos_sqrt(lambda v: Mr @ v, z.ravel(), tol)
    print(f"real_sample {precision}: iters gpu {st.lanczos_iters} oracle {it_ref}", flush=True)
    assert st.converged == 1
    check(y, y_ex, tol, f"real_sample {precision}")
    assert abs(st.lanczos_iters - it_ref) <= 1


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_wave_sample_matches_direct_fourier_sum(gpu_lib, cfg0, precision):
    x, L, _ = cfg0
    s = make(gpu_lib, len(x), L, precision)
    s.set_positions(to_dev(x, s.dtype))
    W = synth.normals(3, (3, M0, M0, M0))
    y = host(s.wave_sample(to_dev(W, s.dtype)))
    y_ref = ewald.wave_sample_direct(x, ewald.zeta_from_grid_noise(W), L, 1.0, 1.0, XI)
    check(y, y_ref, 1e-4, f"wave_sample {precision}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_wave_apply_and_mobility_match_oracle(gpu_lib, cfg0, precision):
    x, L, Mr = cfg0
    s = make(gpu_lib, len(x), L, precision)
    s.set_positions(to_dev(x, s.dtype))
    F = synth.normals(4, (len(x), 3))
    uw = host(s.wave_apply(to_dev(F, s.dtype)))
    uw_ref = ewald.wave_apply_direct(x, F, M0, L, 1.0, 1.0, XI)
    check(uw, uw_ref, 1e-4, f"wave_apply {precision}")
    u = host(s.mobility_apply(to_dev(F, s.dtype)))
    check(u, uw_ref + (Mr @ F.ravel()).reshape(-1, 3), 1e-4, f"mobility_apply {precision}")


@pytest.mark.parametrize("precision,bits,tol", [("fp64", 53, 1e-7), ("mixed", 24, 1e-5)])
def test_full_sample_with_philox_noise(gpu_lib, cfg0, precision, bits, tol):
    """pse_sample draws z1 and zeta from Philox-4x64-10 exactly as the oracle
    does; the whole displacement (real + wave + dt M F) then matches."""
    x, L, Mr = cfg0
    s = make(gpu_lib, len(x), L, precision, tol=tol, kT=1.3)
    s.set_positions(to_dev(x, s.dtype))
    F = synth.normals(5, (len(x), 3))
    dt, seed, counter = 0.7, 1234, 42
    d, st = s.sample(seed, counter, dt=dt, forces=to_dev(F, s.dtype))
    d = host(d)
    p = sampler.Params(L=L, xi=XI, rc=RC, M=M0, kT=1.3)
    z1 = philox.real_noise(len(x), seed, counter, bits)
    zeta = philox.wave_noise_full(M0, seed, counter, bits)
    yr = lanczos.sqrt_apply(Mr, z1).reshape(-1, 3)
    yw = ewald.wave_sample_direct(x, zeta, L, 1.0, 1.0, XI)
    u = (Mr @ F.ravel()).reshape(-1, 3) + ewald.wave_apply_direct(x, F, M0, L, 1.0, 1.0, XI)
    ref = np.sqrt(2 * p.kT * dt) * (yr + yw) + dt * u
    print(f"sample/philox {precision}: iters {st.lanczos_iters}", flush=True)
    check(d, ref, 1e-4, f"sample/philox {precision}")


def test_grid_noise_sample_equals_parts(gpu_lib, cfg0):
    """pse_sample_with_noise = sqrt(2kT dt)(real sample + wave sample) + dt M F."""
    x, L, Mr = cfg0
    s = make(gpu_lib, len(x), L, "fp64", tol=1e-8)
    s.set_positions(to_dev(x, s.dtype))
    z1 = synth.normals(6, (len(x), 3))
    W = synth.normals(7, (3, M0, M0, M0))
    F = synth.normals(8, (len(x), 3))
    d, _ = s.sample_with_noise(to_dev(z1, s.dtype), to_dev(W, s.dtype), dt=0.3, forces=to_dev(F, s.dtype))
    ref = sampler.displacement_from_grid_noise(x, z1, W, sampler.Params(L=L, xi=XI, rc=RC, M=M0), dt=0.3, forces=F)
    check(host(d), ref, 1e-4, "sample/grid-noise fp64")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_kspace_noise_sample_matches_direct_fourier_sum(gpu_lib, cfg0, precision):
    """Caller-supplied zeta on the stored half spectrum (PSE_FLAG_NOISE_KSPACE):
    the wave sample against the direct Fourier sum with the full field the
    half spectrum stands for (canonical pairs on jz = 0, Nyquist and k = 0
    dropped); then zeta = DFT(W)/M^{3/2} gives the grid-noise sample."""
    import torch

    x, L, _ = cfg0
    H = M0 // 2
    rng = np.random.default_rng(14)
    zh = (rng.standard_normal((3, M0, M0, H)) + 1j * rng.standard_normal((3, M0, M0, H))) / np.sqrt(2.0)
    ctype = torch.complex128 if precision == "fp64" else torch.complex64
    s = gpu_lib.Sampler(len(x), L, xi=XI, rcut=RC, grid=M0, support=P, tol=1e-6, precision=precision,
                        flags=gpu_lib.FLAG_NOISE_KSPACE)
    s.set_positions(to_dev(x, s.dtype))
    y = host(s.wave_sample(torch.as_tensor(zh, dtype=ctype, device="cuda")))
    ref = ewald.wave_sample_direct(x, philox.half_spectrum_to_full(zh), L, 1.0, 1.0, XI)
    check(y, ref, 1e-4, f"k-space noise wave sample {precision}")
    # the same sample through the grid-noise path
    W = synth.normals(15, (3, M0, M0, M0))
    zW = (np.fft.fftn(W, axes=(1, 2, 3)) / M0**1.5)[..., :H]
    yk = host(s.wave_sample(torch.as_tensor(zW, dtype=ctype, device="cuda")))
    g = make(gpu_lib, len(x), L, precision)
    g.set_positions(to_dev(x, g.dtype))
    yw = host(g.wave_sample(to_dev(W, g.dtype)))
    check(yk, yw, 1e-12 if precision == "fp64" else 1e-5, f"k-space vs grid noise {precision}")


# ------------------------------------------------------------- edge cases
@pytest.mark.parametrize("precision,bar_r", [("fp64", 1e-12), ("fp32", FP32_NEAR_BAR_DENSE),
                                             ("mixed", FP32_NEAR_BAR_DENSE)])
def test_ragged_overlapping_unwrapped_positions(gpu_lib, precision, bar_r):
    """N = 1001 (ragged against every block size), uniform positions with
    overlaps and one coincident pair, coordinates outside [0, L) and exactly
    at L (maps to 0).  The 20a box holds 2^3 cells of the cell list, too few
    for LDS blocks: FP32 storage takes the global neighbour list and table
    product here."""
    L, M = 20.0, 32
    x = synth.uniform_positions(1001, L, seed=9)
    x[1] = x[0]                      # coincident spheres
    x[2] = x[3] + [0.3, -0.2, 0.1]   # strong overlap
    x[10:20] += L * np.array([1, -1, 2])
    x[30] = [L, 0.0, L]
    s = make(gpu_lib, len(x), L, precision, grid=M)
    s.set_positions(to_dev(x, s.dtype))
    Mr = rpy.real_block_dense(x, L, 1.0, 1.0, XI, RC)
    v = synth.normals(10, (len(x), 3))
    check(host(s.real_matvec(to_dev(v, s.dtype))), Mr @ v.ravel(), bar_r, f"ragged/overlap {precision} M_r v")
    W = synth.normals(11, (3, M, M, M))
    y = host(s.wave_sample(to_dev(W, s.dtype)))
    check(y, ewald.wave_sample_direct(x, ewald.zeta_from_grid_noise(W), L, 1.0, 1.0, XI), 1e-4,
          f"ragged/overlap {precision} wave")


def test_single_particle(gpu_lib):
    L = 20.0
    x = np.array([[3.0, 19.99, 0.01]])
    s = make(gpu_lib, 1, L, "fp64", grid=32)
    s.set_positions(to_dev(x, s.dtype))
    d, st = s.sample(7, 1, dt=1.0)
    ref = sampler.displacement_philox(x, sampler.Params(L=L, xi=XI, rc=RC, M=32), 7, 1, bits=53)
    check(host(d), ref, 1e-4, "N=1")


def test_nonfinite_positions_rejected(gpu_lib):
    x = synth.uniform_positions(50, 20.0, seed=1)
    x[5, 1] = np.nan
    s = make(gpu_lib, 50, 20.0, "fp32", grid=32)
    with pytest.raises(gpu_lib.PSEError) as e:
        s.set_positions(to_dev(x, s.dtype))
    assert e.value.status == -5
    with pytest.raises(gpu_lib.PSEError) as e2:
        s.sample(1, 1)
    assert e2.value.status == -7


def test_not_converged_still_writes_best_iterate(gpu_lib, cfg0):
    x, L, Mr = cfg0
    s = make(gpu_lib, len(x), L, "fp64", max_iter=2, tol=1e-12)
    s.set_positions(to_dev(x, s.dtype))
    z = synth.normals(2, (len(x), 3))
    y, st = s.real_sample(to_dev(z, s.dtype))
    assert st.converged == 0 and st.lanczos_iters == 2
    # the 2-step Krylov iterate of the oracle
    _, _, hist = lanczos.lanczos_sqrt(lambda v: Mr @ v, z.ravel(), 1e-30, max_iter=2)
    check(host(y), hist[-1], 1e-10, "2-step iterate")


# ------------------------------------------------------------ statistics
def test_sample_covariance_is_mobility(gpu_lib):
    """Sample covariance of pse_sample over many counters tends to
    2 kT dt (M_r + M_w) (fluctuation-dissipation, eq. langevin); per-entry
    5 sigma."""
    import torch

    L, M, xi, rc = 8.0, 16, 1.0, 3.9
    x = np.array([[1.0, 1.0, 1.0], [2.2, 1.5, 0.7], [5.0, 6.0, 4.0]])
    s = make(gpu_lib, 3, L, "fp64", grid=M, xi=xi, rc=rc, support=6, tol=1e-10)
    s.set_positions(to_dev(x, s.dtype))
    n = 20000
    out = torch.empty((n, 3, 3), dtype=torch.float64, device="cuda")
    for t in range(n):
        s.sample(99, t, dt=1.0, out=out[t])
    Y = host(out).reshape(n, 9)
    Mt = 2.0 * (rpy.real_block_dense(x, L, 1.0, 1.0, xi, rc) +
                ewald.wave_block_dense(x, L, 1.0, 1.0, xi, ewald.kset_grid(M)))
    C = Y.T @ Y / n
    d = np.sqrt(np.diag(Mt))
    sig = np.sqrt((np.outer(d, d) ** 2 + Mt**2) / n)
    assert np.all(np.abs(C - Mt) < 5 * sig)
    assert np.all(np.abs(Y.mean(0)) < 5 * d / np.sqrt(n))


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_zero_temperature_gives_the_deterministic_drift(gpu_lib, cfg0, precision, bar):
    """kT = 0 removes both noise terms of eq. split: the displacement is
    dt (M_r + M_w) F, the mobility product; without forces it is zero."""
    x, L, Mr = cfg0
    s = make(gpu_lib, len(x), L, precision, kT=0.0)
    s.set_positions(to_dev(x, s.dtype))
    F = synth.normals(12, (len(x), 3))
    d, _ = s.sample(5, 9, dt=0.25, forces=to_dev(F, s.dtype))
    u = host(s.mobility_apply(to_dev(F, s.dtype)))
    check(host(d), 0.25 * u, bar, f"kT = 0 {precision} drift")
    d0, _ = s.sample(5, 10, dt=0.25)
    assert not np.any(host(d0))
