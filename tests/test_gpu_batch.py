"""Batched replicas (pse_batch_*): every replica's displacement equals the
one its own context gives alone with key seed + r (same kernels, same
order: bit-identical), one replica against the FP64 oracle, the
per-replica completion times, and the captured step (per-replica and
batched launches) against the eager step."""
import numpy as np
import pytest

import synth
from parity import check
from oracle import sampler

pytestmark = pytest.mark.gpu

SPECS = [(700, 0.1, 64, "fp64"), (1500, 0.3, 64, "mixed"), (300, 0.2, 32, "fp32"), (2500, 0.05, 64, "mixed"),
         (1000, 0.35, 32, "mixed")]


@pytest.fixture(scope="module")
def systems():
    out = []
    for k, (n, phi, M, prec) in enumerate(SPECS):
        x, L = synth.hard_spheres(n, phi, seed=1500 + k, sweeps=10)
        out.append(dict(x=x, L=L, spec=dict(n=n, box=L, xi=0.5, rcut=8.0 if L > 16.5 else 0.49 * L, grid=M,
                                           support=8, tol=1e-6, precision=prec)))
    return out


def test_batch_equals_single_contexts(gpu_lib, systems):
    import torch

    b = gpu_lib.Batch([s["spec"] for s in systems])
    dts = [torch.float64 if s["spec"]["precision"] == "fp64" else torch.float32 for s in systems]
    pos = [torch.as_tensor(s["x"], dtype=dt, device="cuda") for s, dt in zip(systems, dts)]
    F = [torch.as_tensor(synth.normals(60 + r, (s["spec"]["n"], 3)), dtype=dt, device="cuda")
         for r, (s, dt) in enumerate(zip(systems, dts))]
    b.set_positions(pos)
    out, st = b.sample(77, 3, dt=0.01, forces=F)
    torch.cuda.synchronize()
    lat = b.latency()
    print("batch latencies (ms):", [round(v, 3) for v in lat])
    assert all(v > 0 for v in lat)
    for r, s in enumerate(systems):
        sp = s["spec"]
        one = gpu_lib.Sampler(sp["n"], sp["box"], xi=sp["xi"], rcut=sp["rcut"], grid=sp["grid"], support=8,
                              tol=sp["tol"], precision=sp["precision"])
        one.set_positions(pos[r])
        ref, st1 = one.sample(77 + r, 3, dt=0.01, forces=F[r])
        torch.cuda.synchronize()
        assert torch.equal(out[r], ref), r
        assert st[r].lanczos_iters == st1.lanczos_iters
        one.close()
    # a second call with the same batch reuses every buffer
    out2, _ = b.sample(77, 4, dt=0.01, forces=F)
    torch.cuda.synchronize()
    assert not torch.equal(out2[1], out[1])
    b.close()


def test_batch_replica_matches_oracle(gpu_lib, systems):
    import torch

    s = systems[0]
    sp = s["spec"]
    b = gpu_lib.Batch([t["spec"] for t in systems[:2]])
    pos = [torch.as_tensor(systems[0]["x"], dtype=torch.float64, device="cuda"),
           torch.as_tensor(systems[1]["x"], dtype=torch.float32, device="cuda")]
    b.set_positions(pos)
    out, st = b.sample(2024, 9, dt=1.0)
    torch.cuda.synchronize()
    ref = sampler.displacement_philox(s["x"], sampler.Params(L=s["L"], xi=sp["xi"], rc=sp["rcut"], M=sp["grid"]),
                                      2024, 9, bits=53)
    check(out[0].cpu().numpy(), ref, 1e-4, "batch replica 0 vs oracle")
    b.close()


def test_batch_with_a_preconditioned_replica(gpu_lib):
    """A replica created with the learned preconditioner (weights set through
    its replica context) gives, inside the batch, the displacement of its own
    context with the same weights, bit for bit; so does a plain replica next
    to it."""
    import torch

    from oracle import precond as opc
    from paper_1611_09322_amd import precond as ppc

    bits = ppc.bf16_bits(ppc.pack(opc.init_weights(41, scale=0.1)))
    specs, pos, F = [], [], []
    for k, (n, phi, M, prec, pc) in enumerate([(1500, 0.3, 64, "mixed", 1), (900, 0.2, 64, "fp32", 0)]):
        x, L = synth.hard_spheres(n, phi, seed=1700 + k, sweeps=10)
        specs.append(dict(n=n, box=L, xi=0.5, rcut=8.0, grid=M, support=8, tol=1e-6, precision=prec, precond=pc))
        pos.append(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
        F.append(torch.as_tensor(synth.normals(1800 + k, (n, 3)), dtype=torch.float32, device="cuda"))
    b = gpu_lib.Batch(specs)
    b.set_precond_weights(0, bits)
    b.set_positions(pos)
    out, st = b.sample(91, 2, dt=0.01, forces=F)
    torch.cuda.synchronize()
    for r, sp in enumerate(specs):
        one = gpu_lib.Sampler(sp["n"], sp["box"], xi=0.5, rcut=8.0, grid=sp["grid"], support=8, tol=1e-6,
                              precision=sp["precision"], precond=sp["precond"])
        if sp["precond"]:
            one.set_precond_weights(bits)
        one.set_positions(pos[r])
        ref, st1 = one.sample(91 + r, 2, dt=0.01, forces=F[r])
        torch.cuda.synchronize()
        print(f"replica {r}: {st[r].lanczos_iters} iterations, {st[r].precond_fallbacks} fallbacks", flush=True)
        assert torch.equal(out[r], ref), r
        assert st[r].lanczos_iters == st1.lanczos_iters and st[r].precond_fallbacks == st1.precond_fallbacks
        one.close()
    b.close()


def _eager_reference(gpu_lib, systems, pos, F, seed, counter):
    """The same replicas stepped eagerly by a batch of their own."""
    import torch

    b = gpu_lib.Batch([s["spec"] for s in systems])
    b.set_positions(pos)
    out, st = b.sample(seed, counter, dt=0.01, forces=F)
    torch.cuda.synchronize()
    return b, [o.clone() for o in out], st


def test_graph_replay_equals_eager_steps(gpu_lib, systems):
    """A captured batch step (pse_batch_graph_*) replayed with new counters
    and with the positions moved in place between replays: every replay
    equals the eager step with the same key and counter (bit for bit while
    the block edge stays that of the capture), and no replica is redone."""
    import torch

    b = gpu_lib.Batch([s["spec"] for s in systems])
    dts = [torch.float64 if s["spec"]["precision"] == "fp64" else torch.float32 for s in systems]
    pos = [torch.as_tensor(s["x"], dtype=dt, device="cuda") for s, dt in zip(systems, dts)]
    F = [torch.as_tensor(synth.normals(80 + r, (s["spec"]["n"], 3)), dtype=dt, device="cuda")
         for r, (s, dt) in enumerate(zip(systems, dts))]
    out = [torch.empty_like(p) for p in pos]
    b.graph_create(pos, out, 0.01, forces=F, extra_iters=4, headroom=0.25)
    ref_b = None
    for step, counter in enumerate((11, 12, 13)):
        if step == 2:
            # move every particle a little, in place (the graph reads the same buffers)
            for r, p in enumerate(pos):
                p.add_(torch.as_tensor(0.05 * synth.normals(90 + r, tuple(p.shape)), dtype=p.dtype, device="cuda"))
        status, st, redone = b.graph_step(5, counter)
        torch.cuda.synchronize()
        got = [o.clone() for o in out]
        ref_b, ref, st_e = _eager_reference(gpu_lib, systems, pos, F, 5, counter)
        print(f"step {step}: redone {redone}, iterations {[s.lanczos_iters for s in st]}, "
              f"block edges {[s.lds_block_edge for s in st]} / eager {[s.lds_block_edge for s in st_e]}", flush=True)
        assert redone == 0
        for r in range(len(systems)):
            if st[r].lds_block_edge == st_e[r].lds_block_edge:
                assert torch.equal(got[r], ref[r]), (step, r)
            else:
                check(got[r].double().cpu().numpy(), ref[r].double().cpu().numpy(), 1e-6, f"replica {r}")
            assert st[r].lanczos_iters == st_e[r].lanczos_iters
        ref_b.close()
    b.graph_destroy()
    b.close()


def test_graph_replay_redoes_overflowing_replicas(gpu_lib, systems):
    """Captured with no headroom; then 300 spheres of one replica are
    gathered into a dense lattice: its neighbour list and the halo of the
    blocks around the lattice outgrow the captured capacities, the kernels
    skip that work and flag it, and the step redoes the replica eagerly;
    every result equals the eager step.  The next replay captures anew and
    needs no redo."""
    import torch

    b = gpu_lib.Batch([s["spec"] for s in systems])
    dts = [torch.float64 if s["spec"]["precision"] == "fp64" else torch.float32 for s in systems]
    pos = [torch.as_tensor(s["x"], dtype=dt, device="cuda") for s, dt in zip(systems, dts)]
    out = [torch.empty_like(p) for p in pos]
    b.graph_create(pos, out, 0.01, extra_iters=2, headroom=0.0)
    # 300 spheres of the dilute replica (volume fraction 0.05, 7 cells per
    # side) on a simple cubic lattice of spacing 2.05a: a local volume
    # fraction near 0.5, about ten times the neighbours per sphere
    g = np.arange(7, dtype=np.float64)
    lat = 2.05 * np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)[:300]
    x3 = systems[3]["x"].copy()
    x3[:300] = x3[0] + lat
    pos[3].copy_(torch.as_tensor(x3, dtype=pos[3].dtype, device="cuda"))
    for counter, want_redo in ((21, True), (22, False)):
        status, st, redone = b.graph_step(9, counter)
        torch.cuda.synchronize()
        got = [o.clone() for o in out]
        ref_b, ref, st_e = _eager_reference(gpu_lib, systems, pos, None, 9, counter)
        print(f"counter {counter}: redone {redone}, iterations {[s.lanczos_iters for s in st]}", flush=True)
        assert (redone == 1) if want_redo else (redone == 0)
        for r in range(len(systems)):
            assert torch.equal(got[r], ref[r]), (counter, r)
        ref_b.close()
    b.graph_destroy()
    b.close()


@pytest.mark.parametrize("with_forces", [False, True])
def test_batched_graph_of_many_mixed_replicas_equals_eager(gpu_lib, with_forces):
    """40 replicas of uneven size (N log-uniform in [300, 3000], volume
    fraction in [0.05, 0.35]) with parameters chosen per replica for a 1e-3
    error (radix-2 and radix-3 grids up to 96^3, xi per replica), FP32 and
    mixed precision, one with the learned preconditioner, with and without
    forces: in the captured step most replicas run entirely in launches
    shared by all of them (binning, neighbour build, noise, forces' gather
    and M_r F, Krylov loop, spreading and wave-space part, final sum).
    Every replay equals the eager step with the same key and counter, bit
    for bit, also after the positions moved in place (within 1e-5 where
    forces are spread with atomics, on grids where the 8 x 8 x 8 tiles do
    not fit: M < 16 + P)."""
    import torch

    from oracle import precond as opc
    from paper_1611_09322_amd import precond as ppc

    rng = np.random.default_rng(2600)
    specs, pos = [], []
    for r in range(40):
        n = int(round(np.exp(rng.uniform(np.log(300), np.log(3000)))))
        phi = float(rng.uniform(0.05, 0.35))
        x, L = synth.hard_spheres(n, phi, seed=2600 + r, sweeps=10)
        prec = "mixed" if r % 2 else "fp32"
        p, _ = gpu_lib.pse_choose_params(gpu_lib.make_params(n, L, precision=prec),
                                         gpu_lib.Tuning(tol=1e-3, max_grid=96, with_forces=0))
        specs.append(dict(n=n, box=L, xi=p.xi, rcut=p.rcut, grid=p.grid, support=p.support, gauss_m=p.gauss_m,
                          tol=1e-3, precision=prec, precond=1 if r == 5 else 0))
        pos.append(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
    print("grids:", sorted({s["grid"] for s in specs}), "supports:", sorted({s["support"] for s in specs}), flush=True)
    bits = ppc.bf16_bits(ppc.pack(opc.init_weights(43, scale=0.1)))
    F = [torch.as_tensor(synth.normals(2650 + r, tuple(p.shape)), dtype=p.dtype, device="cuda")
         for r, p in enumerate(pos)] if with_forces else None
    b = gpu_lib.Batch(specs)
    b.set_precond_weights(5, bits)
    out = [torch.empty_like(p) for p in pos]
    b.graph_create(pos, out, 1e-3, forces=F, extra_iters=2, headroom=0.25)
    ref_b = gpu_lib.Batch(specs)
    ref_b.set_precond_weights(5, bits)
    for step, counter in enumerate((31, 32, 33)):
        if step == 2:
            for r, p in enumerate(pos):
                p.add_(torch.as_tensor(0.03 * synth.normals(2700 + r, tuple(p.shape)), dtype=p.dtype, device="cuda"))
        status, st, redone = b.graph_step(8, counter)
        torch.cuda.synchronize()
        got = [o.clone() for o in out]
        ref_b.set_positions(pos)
        ref, st_e = ref_b.sample(8, counter, dt=1e-3, forces=F)
        torch.cuda.synchronize()
        print(f"step {step}: redone {redone}, mean iterations {np.mean([s.lanczos_iters for s in st]):.2f}",
              flush=True)
        assert redone == 0
        for r in range(len(specs)):
            # grids too small for the 8 x 8 x 8 spreading tiles spread forces
            # with atomics (summation order not fixed)
            atomic = with_forces and specs[r]["grid"] < 16 + specs[r]["support"]
            if st[r].lds_block_edge == st_e[r].lds_block_edge and not atomic:
                assert torch.equal(got[r], ref[r]), (step, r)
                assert st[r].lanczos_iters == st_e[r].lanczos_iters, (step, r)
            else:  # another block edge for the moved positions, or the atomic spreading
                check(got[r].double().cpu().numpy(), ref[r].double().cpu().numpy(), 1e-5, f"replica {r}")
    ref_b.close()
    b.graph_destroy()
    b.close()


def test_batched_graph_with_a_large_replica(gpu_lib):
    """A replica of 70000 spheres next to two small ones: too large for the
    fully batched form (its Krylov start's partial sums would not fit the
    single-system layout), it keeps its own binning, noise, start and final
    sum inside the captured step while sharing the batched neighbour build,
    Krylov loop and wave-space part.  Every replay equals the eager step."""
    import torch

    specs, pos = [], []
    for k, (n, phi) in enumerate([(70000, 0.2), (800, 0.1), (2500, 0.3)]):
        x, L = synth.hard_spheres(n, phi, seed=2800 + k, sweeps=5)
        p, _ = gpu_lib.pse_choose_params(gpu_lib.make_params(n, L, precision="mixed"),
                                         gpu_lib.Tuning(tol=1e-3, max_grid=128, with_forces=0))
        specs.append(dict(n=n, box=L, xi=p.xi, rcut=p.rcut, grid=p.grid, support=p.support, gauss_m=p.gauss_m,
                          tol=1e-3, precision="mixed"))
        pos.append(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
    b = gpu_lib.Batch(specs)
    out = [torch.empty_like(p) for p in pos]
    b.graph_create(pos, out, 1e-3, extra_iters=2, headroom=0.25)
    ref_b = gpu_lib.Batch(specs)
    for counter in (41, 42):
        status, st, redone = b.graph_step(6, counter)
        torch.cuda.synchronize()
        got = [o.clone() for o in out]
        ref_b.set_positions(pos)
        ref, st_e = ref_b.sample(6, counter, dt=1e-3)
        torch.cuda.synchronize()
        print(f"counter {counter}: redone {redone}, iterations {[s.lanczos_iters for s in st]}", flush=True)
        assert redone == 0
        for r in range(len(specs)):
            assert torch.equal(got[r], ref[r]), (counter, r)
    ref_b.close()
    b.graph_destroy()
    b.close()
