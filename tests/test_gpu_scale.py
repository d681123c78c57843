"""Parity at the benchmark's full size (N = 10^6 hard spheres at volume
fraction 0.3, 256^3 grid, P = 8, xi a = 0.5, rc = 8a, the launch
configuration bench.py times) on outputs the oracle computes one at a time,
plus an independent 2000-sphere box at the same volume fraction checked
against the full oracle, and rows of the scale configuration (4 10^6 spheres
at volume fraction 0.4, 512^3).

- near-field rows: brute-force rows of M_r v (exact definition, eq. Mreal),
  2000 random particles;
- wave-space rows: direct non-uniform Fourier sums with the same k-space noise
  (zeta = DFT(W)/M^{3/2} of the same grid noise W), the same 2000 particles;
- the Krylov sample at tol 1e-3 against the same sampler converged in FP64
  (self-convergence; no dense root exists at this size).
The structure comes from RSA plus a few Monte Carlo sweeps (the kernels see
the same sizes, densities and neighbour counts as after 2000 sweeps)."""
import numpy as np
import pytest

import synth
from oracle import ewald, rpy, sampler
from se_error import se_aliasing_estimate

pytestmark = pytest.mark.gpu

N, PHI, M, XI, RC = 1_000_000, 0.3, 256, 0.5, 8.0


from parity import FP32_NEAR_BAR_DENSE, check, rel

NROWS = 2000


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.fixture(scope="module")
def big():
    x, L = synth.hard_spheres(N, PHI, a=1.0, seed=1003, sweeps=5)
    rows = np.sort(np.random.default_rng(77).choice(N, NROWS, replace=False))
    print(f"[scale] N={N} L={L:.3f}", flush=True)
    return x, L, rows


def make(gpu_lib, L, precision, tol=1e-3, n=N, grid=M):
    return gpu_lib.Sampler(n, L, a=1.0, eta=1.0, kT=1.0, xi=XI, rcut=RC, grid=grid, support=8, tol=tol,
                           max_iter=64, precision=precision)


def test_near_field_rows_at_full_size(gpu_lib, big):
    import torch

    x, L, rows = big
    v = synth.normals(31, (N, 3))
    ref = rpy.real_matvec_rows(x, v, rows, L, 1.0, 1.0, XI, RC)
    for precision in ("mixed", "fp32"):
        s = make(gpu_lib, L, precision)
        s.set_positions(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
        w = host(s.real_matvec(torch.as_tensor(v, dtype=torch.float32, device="cuda")))
        check(w[rows], ref, FP32_NEAR_BAR_DENSE, f"[scale] M_r v, {NROWS} rows ({precision})")
        s.close()


def test_wave_rows_at_full_size(gpu_lib, big):
    """Bar: the aliasing error the grid spacing implies (estimated above
    from the window and B(k) alone, no GPU data), within the 1e-3
    tolerance of the sampled displacement."""
    import torch

    x, L, rows = big
    s = make(gpu_lib, L, "mixed")
    s.set_positions(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
    W = np.random.default_rng(32).standard_normal((3, M, M, M)).astype(np.float32)
    y = host(s.wave_sample(torch.as_tensor(W, device="cuda")))
    s.close()
    zeta = ewald.zeta_from_grid_noise(W.astype(np.float64))
    del W
    ref = ewald.wave_sample_direct(x[rows], zeta, L, 1.0, 1.0, XI)
    est = se_aliasing_estimate(L, M, XI, 8)
    print(f"[scale] aliasing estimate {est:.2e}")
    check(y[rows], ref, max(1e-4, 1.5 * est), f"[scale] wave sample, {NROWS} rows")
    assert rel(y[rows], ref) < 1e-3


def test_krylov_sample_at_full_size_converges(gpu_lib, big):
    """The tol-1e-3 samples of both timed precisions (FP32 and mixed) against
    the FP64 sampler at tol 1e-8 on the same z: the error of the stopped
    iterate stays below the tolerance."""
    import torch

    x, L, _ = big
    z = synth.normals(33, (N, 3))
    r = make(gpu_lib, L, "fp64", tol=1e-8)
    r.set_positions(torch.as_tensor(x, dtype=torch.float64, device="cuda"))
    yr, str_ = r.real_sample(torch.as_tensor(z, dtype=torch.float64, device="cuda"))
    yr = host(yr)
    r.close()
    assert str_.converged
    for precision in ("mixed", "fp32"):
        s = make(gpu_lib, L, precision, tol=1e-3)
        s.set_positions(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
        y, st = s.real_sample(torch.as_tensor(z, dtype=torch.float32, device="cuda"))
        y = host(y)
        s.close()
        print(f"[scale] Krylov sample ({precision}): {st.lanczos_iters} iterations at tol 1e-3 vs"
              f" {str_.lanczos_iters} at 1e-8")
        assert st.converged
        check(y, yr, 1e-3, f"[scale] Krylov sample ({precision}, tol 1e-3) vs FP64 tol 1e-8")


@pytest.mark.timeout(900)
def test_scale_configuration_rows(gpu_lib):
    """The scale configuration: 4 10^6 spheres at volume fraction 0.4 (FCC
    start + MC sweeps), 512^3 grid, mixed precision: 256 brute-force rows of
    M_r v and 256 rows of the wave sample against the direct Fourier sums
    (bar: the aliasing estimate of this grid spacing, h = 0.68a, with the
    quadrature bound, as at 256^3)."""
    import torch

    n4, phi4, m4 = 4_000_000, 0.4, 512
    x, L = synth.hard_spheres(n4, phi4, a=1.0, seed=1004, sweeps=3)
    rows = np.sort(np.random.default_rng(78).choice(n4, 256, replace=False))
    print(f"[scale] N={n4} phi={phi4} L={L:.3f} M={m4}", flush=True)
    s = make(gpu_lib, L, "mixed", n=n4, grid=m4)
    s.set_positions(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
    v = synth.normals(41, (n4, 3))
    w = host(s.real_matvec(torch.as_tensor(v, dtype=torch.float32, device="cuda")))[rows]
    check(w, rpy.real_matvec_rows(x, v, rows, L, 1.0, 1.0, XI, RC), FP32_NEAR_BAR_DENSE, "[scale 4M] M_r v, 256 rows")
    del v
    W = np.random.default_rng(42).standard_normal((3, m4, m4, m4), dtype=np.float32)
    y = host(s.wave_sample(torch.as_tensor(W, device="cuda")))[rows]
    s.close()
    torch.cuda.empty_cache()
    zeta = ewald.zeta_from_grid_noise(W)
    del W
    ref = ewald.wave_sample_direct(x[rows], zeta, L, 1.0, 1.0, XI)
    del zeta
    est = se_aliasing_estimate(L, m4, XI, 8)
    check(y, ref, max(1e-4, 1.5 * est), f"[scale 4M] wave sample, 256 rows (aliasing estimate {est:.1e})")


@pytest.mark.parametrize("phi", [PHI, 0.4])
def test_independent_2000_sphere_box_full_oracle(gpu_lib, phi):
    """N = 2000 at volume fraction 0.3 (L = 30.34a, RSA start) and 0.4
    (L = 27.57a, FCC start), 64^3 grid (h = 0.47a, 0.43a): the whole
    displacement with forces, Philox noise on both sides."""
    import torch

    x, L = synth.hard_spheres(2000, phi, a=1.0, seed=1099, sweeps=200)
    F = synth.normals(34, (2000, 3))
    s = make(gpu_lib, L, "mixed", tol=1e-6, n=2000, grid=64)
    s.set_positions(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
    out, st = s.sample(2024, 5, dt=1e-3, forces=torch.as_tensor(F, dtype=torch.float32, device="cuda"))
    got = host(out)
    s.close()
    ref = sampler.displacement_philox(x, sampler.Params(L=L, xi=XI, rc=RC, M=64), 2024, 5, dt=1e-3, forces=F, bits=24)
    print(f"[scale] N=2000 box at phi={phi}: {st.lanczos_iters} iterations")
    check(got, ref, 1e-4, f"[scale] N=2000 box at phi={phi}")


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_largest_grid_512(gpu_lib, precision):
    """The largest supported grid, 512^3 (h = 0.23a in a 120a box): M_w F for
    64 spheres against the direct Fourier sums (exercises the 512-point
    transforms and the 512^3 spreading and interpolation tiles)."""
    import torch

    L, M = 120.0, 512
    x = synth.uniform_positions(64, L, seed=91)
    F = synth.normals(92, (64, 3))
    dt = torch.float64 if precision == "fp64" else torch.float32
    s = make(gpu_lib, L, precision, n=64, grid=M)
    s.set_positions(torch.as_tensor(x, dtype=dt, device="cuda"))
    u = host(s.wave_apply(torch.as_tensor(F, dtype=dt, device="cuda")))
    s.close()
    ref = ewald.wave_apply_direct(x, F, M, L, 1.0, 1.0, XI)
    check(u, ref, 1e-4, f"[scale] 512^3 M_w F ({precision})")


def test_products_symmetric_positive_at_full_size(gpu_lib, big):
    """Both halves of the split are symmetric positive-definite operators
    (Sec. II A; the wave part as S^T F^-1 B F S with interpolation the
    adjoint of spreading): at full size, <u, M v> = <M u, v> to FP32 rounding
    and <v, M v> > 0, for M_r and M_w."""
    import torch

    x, L, _ = big
    s = make(gpu_lib, L, "mixed")
    s.set_positions(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
    u = torch.as_tensor(synth.normals(35, (N, 3)), dtype=torch.float32, device="cuda")
    v = torch.as_tensor(synth.normals(36, (N, 3)), dtype=torch.float32, device="cuda")
    for name, op in (("M_r", s.real_matvec), ("M_w", s.wave_apply)):
        Mu, Mv = host(op(u)), host(op(v))
        uh, vh = host(u), host(v)
        a, b = float(np.sum(uh * Mv)), float(np.sum(Mu * vh))
        asym = abs(a - b) / (np.linalg.norm(uh) * np.linalg.norm(Mv))
        print(f"[scale] {name}: <u,Mv> {a:.6e} <Mu,v> {b:.6e} asym {asym:.1e} <v,Mv> {np.sum(vh * Mv):.4e}")
        assert asym < 1e-6
        assert np.sum(vh * Mv) > 0 and np.sum(uh * Mu) > 0
    s.close()
