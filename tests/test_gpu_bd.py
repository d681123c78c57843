"""The Euler-Maruyama Brownian-dynamics step (pse_bd_step, eq. langevin):
positions move by dt M (F_ext + F_rep) + sqrt(2 kT dt) M^{1/2} dW with the
overlap repulsion F_rep accumulated by the neighbour-list scan.

- kT = 0: the move is dt M F, checked against the oracle's dense mobility
  (FP64) with an analytic overlap force, and against the library's own
  mobility product with the repulsion computed on the host (FP32, LDS path);
- with noise and no overlaps the step equals pse_sample plus the position
  update, bit for bit (same Philox noise);
- a short run keeps near-hard spheres from interpenetrating."""
import numpy as np
import pytest

import synth
from oracle import ewald, rpy
from parity import check

pytestmark = pytest.mark.gpu


def rep_force(x, L, a, krep):
    """Host overlap repulsion: sum_{r < 2a} krep (2a - r) d / r, d = x_i - x_j
    (minimum image)."""
    n = len(x)
    f = np.zeros((n, 3))
    for i in range(n):
        d = x[i] - x
        d -= L * np.round(d / L)
        r = np.linalg.norm(d, axis=1)
        m = (r < 2 * a) & (r > 0)
        f[i] = np.sum((krep * (2 * a - r[m]) / r[m])[:, None] * d[m], axis=0)
    return f


def test_deterministic_step_with_overlaps_matches_oracle(gpu_lib):
    import torch

    L, M, xi, rc = 20.0, 64, 0.5, 8.0
    x = synth.uniform_positions(300, L, seed=5)
    x[1] = x[0] + [1.2, 0.3, -0.4]  # overlapping pairs
    x[3] = x[2] + [0.0, 1.9, 0.0]
    x[7] = x[6] + [0.05, 0.0, 0.0]
    Fext = synth.normals(6, (len(x), 3))
    krep, dt = 3.0, 0.01
    s = gpu_lib.Sampler(len(x), L, xi=xi, rcut=rc, grid=M, support=12, tol=1e-8, kT=0.0, precision="fp64")
    pos = torch.as_tensor(x, device="cuda")
    disp = torch.empty_like(pos)
    s.bd_step(pos, 1, 0, dt, krep=krep, forces=torch.as_tensor(Fext, device="cuda"), disp=disp)
    torch.cuda.synchronize()
    F = Fext + rep_force(x, L, 1.0, krep)
    Mt = rpy.real_block_dense(x, L, 1.0, 1.0, xi, rc) + ewald.wave_block_dense(x, L, 1.0, 1.0, xi, ewald.kset_grid(M))
    ref = dt * (Mt @ F.ravel()).reshape(-1, 3)
    check(disp.cpu().numpy(), ref, 1e-6, "BD step, kT = 0, with overlaps (FP64)")
    check(pos.cpu().numpy(), x + ref, 1e-9, "positions after the step")
    s.close()


def test_lds_path_repulsion(gpu_lib):
    """FP32 storage at 20000 spheres (LDS neighbour build with the fused
    repulsion): the step's displacement equals dt M F_rep with F_rep from
    the host.  Bar: the overlap 2a - r is a difference of FP32 coordinates of
    size L ~ 60a (rounding ~4e-6 a) against overlaps of ~0.02a, so each
    force carries ~2e-4 relative error."""
    import torch

    x, L = synth.hard_spheres(20000, 0.3, seed=1600, sweeps=5)
    x = x + 0.06 * synth.normals(1601, x.shape)  # some pairs now overlap
    krep, dt = 2.0, 0.05
    F = rep_force(x, L, 1.0, krep)
    print(f"overlapping spheres: {np.count_nonzero(np.linalg.norm(F, axis=1))}", flush=True)
    s = gpu_lib.Sampler(len(x), L, xi=0.56, rcut=4.69, grid=128, support=8, tol=1e-6, kT=0.0, precision="mixed")
    pos = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    disp = torch.empty_like(pos)
    st = s.bd_step(pos, 2, 0, dt, krep=krep, disp=disp)
    assert st.lds_block_edge > 0
    ref = s.mobility_apply(torch.as_tensor(F, dtype=torch.float32, device="cuda")) * dt
    torch.cuda.synchronize()
    check(disp.double().cpu().numpy(), ref.double().cpu().numpy(), 1e-3, "BD step repulsion, LDS path")
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_step_equals_sample_plus_update(gpu_lib, precision):
    import torch

    x, L = synth.hard_spheres(3000, 0.2, seed=1700, sweeps=10)
    dtp = torch.float64 if precision == "fp64" else torch.float32
    F = torch.as_tensor(synth.normals(1701, x.shape), dtype=dtp, device="cuda")
    s = gpu_lib.Sampler(len(x), L, xi=0.5, rcut=8.0, grid=64, support=8, tol=1e-4, precision=precision)
    pos = torch.as_tensor(x, dtype=dtp, device="cuda")
    s.set_positions(pos)
    ref, _ = s.sample(77, 5, dt=1e-3, forces=F)
    ref = ref.clone()
    p2 = pos.clone()
    disp = torch.empty_like(pos)
    s.bd_step(p2, 77, 5, 1e-3, krep=0.0, forces=F, disp=disp)
    torch.cuda.synchronize()
    assert torch.equal(disp, ref)
    assert torch.equal(p2, pos + ref)
    s.close()


def test_short_run_keeps_spheres_apart(gpu_lib):
    """200 steps at volume fraction 0.3 (dt = 1e-3 in units of a^2 / D0 with
    D0 = kT / 6 pi eta a): with a stiff repulsion (dt mu0 krep = 0.27 of an
    overlap removed per step) the closest pair stays above 1.8a, while
    without it the Brownian motion (rms 0.25a) lets spheres interpenetrate."""
    import torch

    x, L = synth.hard_spheres(4000, 0.3, seed=1800, sweeps=20)
    dmin = {}
    for krep in (5000.0, 0.0):
        s = gpu_lib.Sampler(len(x), L, xi=0.56, rcut=4.69, grid=64, support=8, tol=1e-3, precision="mixed")
        pos = torch.as_tensor(x, dtype=torch.float32, device="cuda")
        for step in range(200):
            s.bd_step(pos, 9, step, 1e-3, krep=krep)
        xs = pos.double().cpu().numpy()
        s.close()
        dmin[krep] = synth.min_pair_distance(np.mod(xs, L), L)
        moved = np.sqrt(np.mean(np.sum((xs - x) ** 2, axis=1)))
        print(f"krep {krep}: rms displacement {moved:.3f}a, closest pair {dmin[krep]:.3f}a", flush=True)
        assert moved > 0.05
    assert dmin[5000.0] > 1.8
    assert dmin[0.0] < dmin[5000.0] - 0.2
