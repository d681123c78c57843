"""The full-mobility Krylov sample (pse_full_sample), the comparator of
Sec. III: Lanczos on M = M_r + M_w, each product a near-field product plus a
wave-space product.  Against the oracle's eigendecomposition root of the
dense M_r + M_w over the grid k-set, with the iteration count of the
oracle's own Lanczos process; then the growth of the iteration count with
N that the near-field sample does not show (Sec. II B.1, Fig. eigenspectrum)."""
import numpy as np
import pytest

import synth
from oracle import ewald, lanczos, rpy
from parity import check

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-4)])
def test_full_sample_matches_dense_root(gpu_lib, precision, tol):
    import torch

    x, L = synth.hard_spheres(500, 0.1, seed=1900, sweeps=20)
    xi, rc, M = 0.5, 8.0, 64
    s = gpu_lib.Sampler(len(x), L, xi=xi, rcut=rc, grid=M, support=12, tol=tol, max_iter=256, precision=precision,
                        flags=gpu_lib.FLAG_FULL_LANCZOS)
    dt = s.dtype
    s.set_positions(torch.as_tensor(x, dtype=dt, device="cuda"))
    z = synth.normals(1901, (len(x), 3))
    y, st = s.full_sample(torch.as_tensor(z, dtype=dt, device="cuda"))
    torch.cuda.synchronize()
    Mt = rpy.real_block_dense(x, L, 1.0, 1.0, xi, rc) + ewald.wave_block_dense(x, L, 1.0, 1.0, xi, ewald.kset_grid(M))
    ref = lanczos.sqrt_apply(Mt, z.ravel())
    _, it_ref, _ = lanczos.lanczos_sqrt(lambda v: Mt @ v, z.ravel(), tol, max_iter=256)
    print(f"full sample {precision}: {st.lanczos_iters} iterations (oracle Lanczos {it_ref})", flush=True)
    assert st.converged
    # the spectral-Ewald error of the wave products (P = 12, h = 0.5a) sits
    # far below both tolerances
    check(y.double().cpu().numpy(), ref, max(tol, 1e-6) * 3, f"full-mobility Krylov sample {precision}")
    assert abs(st.lanczos_iters - it_ref) <= 1
    s.close()


def test_iterations_grow_with_n_on_the_full_mobility(gpu_lib):
    """At volume fraction 0.1 and tolerance 1e-3: the near-field sample's
    iteration count does not grow from 1000 to 27000 spheres, the full
    mobility's does (its condition number grows with the box)."""
    import torch

    res = {}
    for n in (1000, 27000):
        x, L = synth.hard_spheres(n, 0.1, seed=1950 + n, sweeps=5)
        M = 32 if n == 1000 else 96
        s = gpu_lib.Sampler(n, L, xi=0.5, rcut=5.3, grid=M, support=8, tol=1e-3, max_iter=256, precision="mixed",
                            flags=gpu_lib.FLAG_FULL_LANCZOS)
        s.set_positions(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
        z = torch.as_tensor(synth.normals(1960 + n, (n, 3)), dtype=torch.float32, device="cuda")
        _, st_r = s.real_sample(z)
        _, st_f = s.full_sample(z)
        res[n] = (st_r.lanczos_iters, st_f.lanczos_iters)
        print(f"N={n}: near-field {st_r.lanczos_iters} iterations, full mobility {st_f.lanczos_iters}", flush=True)
        assert st_f.converged
        s.close()
    assert res[27000][0] <= res[1000][0] + 1
    assert res[27000][1] > res[1000][1]
