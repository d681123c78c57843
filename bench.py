#!/usr/bin/env python3
"""Throughput of the PSE Brownian sampler on one MI355X.

One step = one Brownian displacement of every particle with the whole hot
path: wrap + linked-cell sort + neighbour list (positions change every step),
real-space Philox noise, Lanczos M_r^{1/2} z1, the near-field product M_r F,
Gaussian spreading of the (random) forces, forward FFT, B(k) scaling with the
k-space noise, inverse FFT, interpolation and the final combine
(dx = dt M F + sqrt(2 kT dt) M^{1/2} dW, the combined FFT pair of Sec. III).

Workload (default): N = 1,000,000 hard spheres a = 1 at volume fraction 0.3
(random sequential addition + Monte Carlo sweeps), cubic periodic box,
256^3 grid, P = 8, xi a = 0.5, rc = 8a, relative tolerance 1e-3.

Prints one JSON line.  Metric: samples x particles per second.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "samples·particles/s, N=1M φ=0.3 @1e-3 err: plain FP32 vs mixed+learned precond"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFS = 157.3
SPMV_FLOPS_PER_PAIR = 35
# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes scaled by the same counters on a copy of known size; the
# summary records the hash of the kernel source it was taken on.
TRAFFIC_SUMMARY = {"spmv": ("profiles/spmv_lds_n1M_phi03_traffic.txt", "paper_1611_09322_amd/csrc/k_particles.hip")}
# the workload those counters were taken on; other workloads report null
TRAFFIC_WORKLOAD = {"n": 1_000_000, "phi": 0.3, "grid": 256, "support": 8, "xi": 0.5, "rc": 8.0}


def stage_bytes(stage, n, grid, pairs, lanczos, index_bytes=4):
    """Algorithmic HBM bytes of one launch of a stage (FP32 storage):
    every operand read once and every result written once."""
    g = 3 * grid**3 * 4  # one 3-component real grid (= the half spectrum)
    if stage == "spmv":
        # positions (float4) + source vector + neighbour count + result
        # (+ the stored Lanczos basis vector) + one stored index per pair
        return n * (16 + 12 + 4 + 12 + (12 if lanczos else 0)) + index_bytes * pairs
    if stage == "fft":
        return 2 * g
    if stage == "xfused":
        return 2 * g
    if stage == "spread":
        return n * (16 + 12) + g
    if stage == "interp":
        return g + n * (16 + 12)
    if stage == "nbr":
        return n * (16 + 4) + 4 * pairs
    return None


def start_of(phi):
    """How the generator starts a configuration at this volume fraction."""
    import synth

    return "RSA" if phi <= synth.RSA_MAX_PHI else "randomly vacated FCC lattice"


def measured_traffic(stage, args):
    """Counter-measured HBM bytes per launch, or None when no summary exists,
    the workload is not the one the counters were taken on, or the kernel
    source changed since."""
    import hashlib

    if stage not in TRAFFIC_SUMMARY or any(getattr(args, k) != v for k, v in TRAFFIC_WORKLOAD.items()):
        return None
    summ, src = (os.path.join(ROOT, p) for p in TRAFFIC_SUMMARY[stage])
    if not os.path.exists(summ):
        return None
    fields = {}
    with open(summ) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    with open(src, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if fields.get("kernel_source_sha256") != digest or "hbm_bytes_per_launch" not in fields:
        return None
    return float(fields["hbm_bytes_per_launch"])


def copy_calibration(torch):
    """One elementwise pass over 512 MiB (read 512 MiB, write 512 MiB), for
    scaling the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    a = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    print("[bench] copy calibration: 536870912 bytes read, 536870912 bytes written", file=sys.stderr, flush=True)


def make_workload(args):
    import numpy as np

    import synth

    t0 = time.time()
    print(f"[bench] generating N={args.n} hard spheres at phi={args.phi} ({start_of(args.phi)}, then {args.sweeps} MC sweeps)",
          file=sys.stderr, flush=True)
    x, L = synth.hard_spheres(args.n, args.phi, a=1.0, seed=1003, sweeps=args.sweeps,
                              progress=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
    # caller order is arbitrary: shuffle so that the library's own sort is exercised
    perm = np.random.default_rng(7).permutation(len(x))
    x = np.ascontiguousarray(x[perm])
    F = synth.normals(8, (len(x), 3))
    print(f"[bench] workload: N={len(x)} phi={args.phi} L={L:.3f} sweeps={args.sweeps} "
          f"generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    return x, L, F


def train_precond(pse, torch, args):
    """Learned block preconditioner for this workload's parameters, trained
    (untimed) on small independent boxes at the same volume fraction."""
    import numpy as np

    import synth
    from paper_1611_09322_amd import precond as ppc

    t0 = time.time()
    tr = ppc.Trainer(torch, seed=3, lr=3e-3)
    for k in range(args.train_boxes):
        x, L = synth.hard_spheres(args.train_n, args.phi, a=1.0, seed=2100 + k, sweeps=100)
        s = pse.Sampler(len(x), L, a=1.0, eta=1.0, kT=1.0, xi=args.xi, rcut=args.rc, grid=64, support=args.support,
                        tol=args.tol, max_iter=64, precision="mixed", precond=1)
        s.set_positions(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
        idx = np.random.default_rng(k).choice(len(x), args.train_rows, replace=False).astype(np.int32)
        tr.add(s, x, idx)
        s.close()
    hist = tr.fit(args.train_epochs)
    print(f"[bench] preconditioner trained on {args.train_boxes} x {args.train_rows} rows in {time.time() - t0:.1f}s:"
          f" loss {hist[0]:.3e} -> {hist[-1]:.3e}", file=sys.stderr, flush=True)
    return tr.weights_bits(), hist


def run_variant(pse, torch, x, L, F, args, variant, weights=None):
    precision, precond = (variant.split("+")[0], 1) if variant.endswith("+precond") else (variant, 0)
    s = pse.Sampler(len(x), L, a=1.0, eta=1.0, kT=1.0, xi=args.xi, rcut=args.rc, grid=args.grid,
                    support=args.support, tol=args.tol, max_iter=64, precision=precision, precond=precond)
    if precond:
        s.set_precond_weights(weights)
    pos = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    frc = torch.as_tensor(F, dtype=torch.float32, device="cuda")
    out = torch.empty_like(pos)
    counter = [0]

    def step():
        s.set_positions(pos)
        _, st = s.sample(2024, counter[0], dt=1e-3, forces=frc, out=out)
        counter[0] += 1
        return st

    # one untimed step absorbs first-launch costs; the library then picks its
    # spreading / interpolation launch shapes on these positions (untimed);
    # the warm-up runs with every stage timed: where the GPU time goes
    st = step()
    tuned = s.autotune()
    s.profile(list(pse.STAGES))
    for _ in range(max(args.warmup - 1, 1)):
        st = step()
    torch.cuda.synchronize()
    breakdown = s.profile_read()
    total = sum(v[0] for v in breakdown.values())
    dom = max((k for k in breakdown if stage_bytes(k, 1, 1, 1, False) is not None), key=lambda k: breakdown[k][0])
    # timed region: events only around the dominant kernel's launches
    s.profile([dom])
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step()
        iters.append(st.lanczos_iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dom_t = s.profile_read()[dom]
    s.profile([])
    ms_step = 1e3 * dt / args.steps
    res = {
        "autotune": {"spread_tile_depth": tuned[0], "interp_lanes": tuned[1], "product_lanes_per_target": tuned[2]},
        "precond_fallbacks": st.precond_fallbacks,
        "value": len(x) * args.steps / dt,
        "ms_per_step": ms_step,
        "lanczos_iters_mean": sum(iters) / len(iters),
        "neighbor_pairs": st.neighbor_pairs,
        "nbr_index_bytes": st.nbr_index_bytes,
        "max_neighbors": st.max_neighbors,
        "warmup_breakdown_ms_per_step": {k: round(v[0] / max(args.warmup - 1, 1), 4) for k, v in breakdown.items()},
        "warmup_gpu_ms_per_step": total / max(args.warmup - 1, 1),
        "dominant": dom,
        "dominant_ms_avg": dom_t[0] / max(dom_t[1], 1),
        "dominant_launches_per_step": dom_t[1] / args.steps,
        "dominant_share": breakdown[dom][0] / total if total else None,
    }
    s.close()
    return res


def run_batch(pse, torch, args):
    """Many small independent systems per call (replicas): N log-uniform in
    [1e3, 2e4], volume fraction uniform in [0.05, 0.4], grid the smallest
    power of two with h <= 0.65a.  Each step sets new positions and samples
    every replica; compared with the same replicas sampled one after another
    through their own contexts.  Grids are capped at 128^3 (h up to 0.93a for
    the largest dilute boxes)."""
    import numpy as np

    import synth

    t0 = time.time()
    rng = np.random.default_rng(20000)
    specs, pos = [], []
    for r in range(args.batch_replicas):
        n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(2e4)))))
        phi = float(rng.uniform(0.05, 0.4))
        x, L = synth.hard_spheres(n, phi, a=1.0, seed=20000 + r, sweeps=20)
        M = next((m for m in (32, 64, 128) if L / m <= 0.65), 128)
        specs.append(dict(n=n, box=L, xi=args.xi, rcut=args.rc, grid=M, support=args.support, tol=args.tol,
                          precision="mixed"))
        pos.append(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
    total = sum(sp["n"] for sp in specs)
    print(f"[bench] batch: {len(specs)} replicas, {total} particles, generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    b = pse.Batch(specs)
    for k in range(args.warmup):
        b.set_positions(pos)
        if k == 0:
            b.autotune()  # untimed: launch shapes per grid size and per replica
        b.sample(11, k, dt=1e-3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.batch_steps):
        b.set_positions(pos)
        _, st = b.sample(11, 1000 + k, dt=1e-3)
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t1) / args.batch_steps
    lat = np.array(b.latency())
    # the same replicas one after another, each through its own context
    ctxs = [pse.pse_batch_replica(b.b, r) for r in range(len(specs))]
    outs = [torch.empty((sp["n"], 3), dtype=torch.float32, device="cuda") for sp in specs]
    seq = []
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for r, c in enumerate(ctxs):
        ta = time.perf_counter()
        pse.pse_set_positions(c, pse._ptr(pos[r], torch.float32, 3 * specs[r]["n"], "pos"))
        pse.pse_sample(c, 11 + r, 2000, 1e-3, None, pse._ptr(outs[r], torch.float32, 3 * specs[r]["n"], "out"))
        torch.cuda.synchronize()
        seq.append(1e3 * (time.perf_counter() - ta))
    dt_s = time.perf_counter() - t2
    seq = np.array(seq)
    cum = np.cumsum(seq)
    b.close()
    pct = lambda a, q: float(np.percentile(a, q))
    return {
        "replicas": len(specs), "particles": total, "steps": args.batch_steps,
        "grids": {str(m): sum(1 for sp in specs if sp["grid"] == m) for m in (32, 64, 128)},
        "value": total / dt_b, "unit": "samples·particles/s", "ms_per_step": 1e3 * dt_b,
        "completion_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "lanczos_iters_mean": float(np.mean([s.lanczos_iters for s in st])),
        "sequential": {"value": total / dt_s, "ms_per_step": 1e3 * dt_s,
                       "service_ms": {"p50": pct(seq, 50), "p99": pct(seq, 99)},
                       "completion_ms": {"p50": pct(cum, 50), "p99": pct(cum, 99)}},
    }


def cpu_baseline(args):
    """The FP64 oracle (dense M_r + eigendecomposition root + direct Fourier
    sums), timed on a bounded sample of the same workload: an independent
    1000-particle periodic box at the same volume fraction, xi, rc, P and
    about the same grid spacing."""
    import numpy as np

    import synth
    from oracle import sampler

    try:
        from threadpoolctl import threadpool_info

        blas_threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:  # pragma: no cover
        blas_threads = None
    n = 1000
    x, L = synth.hard_spheres(n, args.phi, seed=1099, sweeps=50)
    p = sampler.Params(L=L, xi=args.xi, rc=args.rc, M=32)
    F = synth.normals(9, (n, 3))
    reps = 0
    t0 = time.perf_counter()
    while True:
        sampler.displacement_philox(x, p, 2024, reps, dt=1e-3, forces=F, bits=24)
        reps += 1
        if time.perf_counter() - t0 > args.cpu_seconds:
            break
    dt = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    return {
        "value": n * reps / dt,
        "unit": "samples·particles/s",
        "cores": blas_threads or cores,
        "kind": "oracle",
        "sample": f"FP64 oracle, {reps} displacement(s) of an independent N={n} box at phi={args.phi} "
                  f"(L={L:.2f}a, 32^3 k-set, xi a={args.xi}, rc={args.rc}a) with forces; "
                  f"{cores} host cores visible, BLAS threads {blas_threads}",
        "seconds": dt,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--phi", type=float, default=0.3)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--support", type=int, default=8)
    ap.add_argument("--xi", type=float, default=0.5)
    ap.add_argument("--rc", type=float, default=8.0)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--sweeps", type=int, default=2000, help="Monte Carlo relaxation sweeps after the start (RSA, or an FCC lattice above phi 0.35)")
    ap.add_argument("--variants", default="fp32,mixed,mixed+precond",
                    help="comma list of fp32, mixed, fp64 and <precision>+precond")
    ap.add_argument("--batch-replicas", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--train-boxes", type=int, default=2)
    ap.add_argument("--train-n", type=int, default=3000)
    ap.add_argument("--train-rows", type=int, default=500)
    ap.add_argument("--train-epochs", type=int, default=300)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 512 MiB elementwise copy (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the sampler runs on one GPU; --gpus {args.gpus} is not supported "
              "(no multi-GPU sharding is implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1611_09322_amd as pse

    pse.load()
    torch.cuda.set_device(0)
    x, L, F = make_workload(args)
    variants = {}
    weights, train_hist = None, None
    for v in args.variants.split(","):
        if v.endswith("+precond") and weights is None:
            weights, train_hist = train_precond(pse, torch, args)
        print(f"[bench] variant {v}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
        variants[v] = run_variant(pse, torch, x, L, F, args, v, weights)
        print(f"[bench] variant {v}: {json.dumps(variants[v])}", file=sys.stderr, flush=True)
    # the metric's subject: mixed precision with the learned preconditioner
    head = next((k for k in ("mixed+precond", "mixed", "fp32") if k in variants), next(iter(variants)))
    hv = variants[head]
    dom = hv["dominant"]
    nbytes = stage_bytes(dom, args.n, args.grid, hv["neighbor_pairs"], lanczos=(dom == "spmv"),
                         index_bytes=hv["nbr_index_bytes"])
    achieved = nbytes / (hv["dominant_ms_avg"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": dom,
                "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": hv["dominant_ms_avg"]}
    if dom == "spmv":
        # the same launches against the FP32 vector peak (matrix-free F/G
        # evaluation per pair; count per pair derived in the design notes)
        roofline["alu_flops_per_pair"] = SPMV_FLOPS_PER_PAIR
        roofline["alu_frac"] = (SPMV_FLOPS_PER_PAIR * hv["neighbor_pairs"] / (hv["dominant_ms_avg"] * 1e-3)
                                / 1e12 / FP32_PEAK_TFS)
    roofline["traffic"] = measured_traffic(dom, args)
    if args.copy_calibration:
        copy_calibration(torch)
    batched = None if args.no_batch else run_batch(pse, torch, args)
    if batched:
        print(f"[bench] batch: {json.dumps(batched)}", file=sys.stderr, flush=True)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args)
    line = {
        "metric": METRIC,
        "value": hv["value"],
        "unit": "samples·particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hv["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"PSE Brownian displacement with random forces, N={args.n} hard spheres a=1, "
                        f"phi={args.phi} ({start_of(args.phi)} + {args.sweeps} MC sweeps), grid {args.grid}^3, P={args.support}, "
                        f"xi a={args.xi}, rc={args.rc}a, tol {args.tol}",
            "variant": head,
            "precond": "learned (trained before timing)" if head.endswith("+precond") else "none",
        },
        "variants": {k: {"value": v["value"], "ms_per_step": v["ms_per_step"],
                         "lanczos_iters_mean": v["lanczos_iters_mean"],
                         "precond_fallbacks": v["precond_fallbacks"],
                         "autotune": v["autotune"], "breakdown_ms": v["warmup_breakdown_ms_per_step"]}
                     for k, v in variants.items()},
        "precond_training": None if train_hist is None else {
            "boxes": args.train_boxes, "n": args.train_n, "rows_per_box": args.train_rows,
            "epochs": args.train_epochs, "loss_first": train_hist[0], "loss_last": train_hist[-1]},
        "roofline": roofline,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
