"""Launch-shape autotuning (pse_autotune, pse_batch_autotune): the choices
are valid launch shapes for the grid, the tuned wave-space sample and
near-field product agree with the built-in ones to rounding (only the order
in which a node sums its particles, or a row its neighbour chunks, may
change), and stay within the oracle bars of the direct Fourier sum and the
dense real-space block."""
import numpy as np
import pytest

import synth
from oracle import ewald, rpy

pytestmark = pytest.mark.gpu

XI, RC, P = 0.5, 8.0, 8


from parity import FP32_NEAR_BAR, FP32_NEAR_BAR_DENSE, check, cutoff_rows


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
    v = synth.normals(2250 + n, (n, 3))
    vd = torch.as_tensor(v, dtype=dt, device="cuda")
    y0, w0 = host(s.wave_sample(Wd)), host(s.real_matvec(vd))
    depth, lanes, plane = s.autotune()
    print(f"n={n} M={grid} {precision}: spreading tile depth {depth}, interpolation lanes {lanes},"
          f" product lanes per target {plane}", flush=True)
    assert lanes in (256, 512, 1024)
    assert depth in (8, 16, 32, 64)
    assert grid % depth == 0 and grid >= 2 * max(8, depth) + P
    assert plane in ((0,) if precision == "fp64" else (0, 2, 3, 4))
    y1, w1 = host(s.wave_sample(Wd)), host(s.real_matvec(vd))
    tol = 1e-12 if precision == "fp64" else 1e-6
    check(y1, y0, tol, "wave sample, tuned vs built-in")
    check(w1, w0, tol, "M_r v, tuned vs built-in")
    if n <= 1000:
        y_ref = ewald.wave_sample_direct(x, ewald.zeta_from_grid_noise(W), L, 1.0, 1.0, XI)
        check(y1, y_ref, 1e-4, "tuned wave sample vs oracle")
        w_ref = rpy.real_block_dense(x, L, 1.0, 1.0, XI, RC) @ v.ravel()
        check(w1, w_ref, 1e-12 if precision == "fp64" else FP32_NEAR_BAR, "tuned M_r v vs oracle")
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
        check(y1, y0[r], 1e-5, f"replica {r}, tuned vs built-in")
    b.close()


@pytest.mark.parametrize("plane", [2, 3, 4])
@pytest.mark.parametrize("n,phi,precision", [(1000, 0.1, "fp32"), (1000, 0.1, "mixed"), (6000, 0.3, "mixed")])
def test_product_lanes_per_target_match_oracle(gpu_lib, n, phi, precision, plane):
    """Each lanes-per-target variant of the LDS product (forces product and
    the fused Lanczos product inside a Krylov sample) against the oracle:
    brute-force rows of M_r v (wrapped halo at N = 1000, 4^3 cells;
    unwrapped at N = 6000, 5^3 cells) within the FP32 table bar, and the
    Krylov sample against the dense symmetric root at N = 1000."""
    import torch

    x, L = synth.hard_spheres(n, phi, seed=2500 + n, sweeps=5)
    s = gpu_lib.Sampler(n, L, xi=XI, rcut=RC, grid=64, support=P, tol=1e-6, precision=precision)
    s.set_launch_shape(0, 0, plane)
    s.set_positions(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
    v = synth.normals(2600 + n, (n, 3))
    w = host(s.real_matvec(torch.as_tensor(v, dtype=torch.float32, device="cuda")))
    rows = np.random.default_rng(n).choice(n, 64, replace=False)
    e, _ = check(w[rows], rpy.real_matvec_rows(x, v, rows, L, 1.0, 1.0, XI, RC),
                 FP32_NEAR_BAR if phi < 0.2 else FP32_NEAR_BAR_DENSE,
                 f"n={n} {precision} lanes {plane} M_r v rows")
    msg = f"n={n} {precision} lanes {plane}: rows {e:.2e}"
    if n <= 1000:
        z = synth.normals(2700 + n, (n, 3))
        y, st = s.real_sample(torch.as_tensor(z, dtype=torch.float32, device="cuda"))
        Mr = rpy.real_block_dense(x, L, 1.0, 1.0, XI, RC)
        lam, Q = np.linalg.eigh(Mr)
        ref = Q @ (np.sqrt(lam) * (Q.T @ z.ravel()))
        e2, _ = check(host(y), ref, 1e-4, f"n={n} {precision} lanes {plane} Krylov sample")
        msg += f", Krylov sample {e2:.2e} ({st.lanczos_iters} iterations)"
        assert st.converged
    print(msg, flush=True)
    s.close()


def test_set_launch_shape_rejects_invalid_shapes(gpu_lib):
    x, L = synth.hard_spheres(500, 0.1, seed=2800)
    s = gpu_lib.Sampler(500, L, xi=XI, rcut=RC, grid=64, support=P, precision="fp32")
    for bad in [(12, 0, 0), (128, 0, 0), (0, 384, 0), (0, 0, 5), (0, 0, 1)]:
        with pytest.raises(gpu_lib.PSEError) as e:
            s.set_launch_shape(*bad)
        assert e.value.status == -1, bad
    s.set_launch_shape(16, 512, 2)
    s.set_launch_shape(0, 0, 0)
    s.close()


@pytest.mark.parametrize("n,rc,edge", [(20000, 4.69, 4), (30000, 6.0, 3), (4000, 8.0, 2)])
def test_block_edge_follows_cell_occupancy(gpu_lib, n, rc, edge):
    """Fewer particles per cell (smaller rc) take blocks of more cells: the
    LDS product and neighbour build at block edges 4, 3 and 2 against
    brute-force rows of M_r v, and the Krylov sample against the FP64
    sampler converged at tol 1e-10 on the same z."""
    import torch

    x, L = synth.hard_spheres(n, 0.3, seed=2800 + n, sweeps=5)
    xi = 0.56
    grid = 64 if L / 64 < 0.9 else 128  # keeps eta_SE below 1
    s = gpu_lib.Sampler(n, L, xi=xi, rcut=rc, grid=grid, support=P, tol=1e-6, precision="mixed")
    s.set_positions(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
    v = synth.normals(2900 + n, (n, 3))
    w = host(s.real_matvec(torch.as_tensor(v, dtype=torch.float32, device="cuda")))
    z = torch.as_tensor(synth.normals(2950 + n, (n, 3)), dtype=torch.float32, device="cuda")
    y, st = s.real_sample(z)
    print(f"n={n} rc={rc}: block edge {st.lds_block_edge}, {st.neighbor_pairs / n:.1f} neighbours", flush=True)
    assert st.lds_block_edge == edge
    rows = np.random.default_rng(n).choice(n, 200, replace=False)
    check(w[rows], rpy.real_matvec_rows(x, v, rows, L, 1.0, 1.0, xi, rc), FP32_NEAR_BAR_DENSE,
          f"block edge {edge}: M_r v rows", skip_rows=cutoff_rows(x, L, rc, rows))
    r = gpu_lib.Sampler(n, L, xi=xi, rcut=rc, grid=grid, support=P, tol=1e-10, precision="fp64")
    r.set_positions(torch.as_tensor(x, dtype=torch.float64, device="cuda"))
    yr, _ = r.real_sample(z.double())
    check(host(y), host(yr), 1e-5, f"block edge {edge}: Krylov sample vs FP64", skip_rows=cutoff_rows(x, L, rc))
    s.close()
    r.close()


def test_spreading_tile_depths_agree(gpu_lib):
    """M_w F (FP32) at every valid spreading tile depth: the matrix-core
    tiles (16 x 8 x depth, depths 8 to 32) against the direct Fourier sums
    and against each other (each sub-tile lists its particles in candidate
    order at every depth; they agree to rounding, or exactly); on a 192^3
    grid the VALU tiles (8 x 8 x 64) against the matrix-core ones."""
    import torch

    x, L = synth.hard_spheres(2000, 0.2, seed=2300, sweeps=5)
    F = synth.normals(2301, (len(x), 3))
    Fd = torch.as_tensor(F, dtype=torch.float32, device="cuda")
    u_ref = ewald.wave_apply_direct(x, F, 128, L, 1.0, 1.0, XI)
    out = {}
    s = gpu_lib.Sampler(len(x), L, xi=XI, rcut=RC, grid=128, support=P, tol=1e-6, precision="fp32")
    s.set_positions(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
    for depth in (8, 16, 32):
        s.set_launch_shape(depth, 0, 0)
        out[depth] = host(s.wave_apply(Fd))
        check(out[depth], u_ref, 1e-4, f"M_w F, 128^3, tile depth {depth}, vs direct sums")
    s.close()
    for depth in (16, 32):
        check(out[depth], out[8], 1e-6, f"M_w F, tile depth {depth} vs 8")
    # 192^3: depth 64 takes the VALU tiles, depth 8 the matrix cores
    s = gpu_lib.Sampler(len(x), L, xi=XI, rcut=RC, grid=192, support=P, tol=1e-6, precision="fp32")
    s.set_positions(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
    u = {}
    for depth in (8, 64):
        s.set_launch_shape(depth, 0, 0)
        u[depth] = host(s.wave_apply(Fd))
    s.close()
    # two FP32 summation schemes for every node (per-lane FMAs against 4-term
    # matrix-core steps): the FP32 rounding floor of the other wave tests
    check(u[64], u[8], 1e-5, "M_w F, 192^3, VALU tiles (depth 64) vs matrix-core tiles (depth 8)")
