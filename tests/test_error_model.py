"""The library's error model and parameter choice (host logic, no GPU):
the bounds of Sec. II C-D against the oracle's own formulas, the aliasing
estimate against a full-grid sum written independently in the tests, the
tolerance check of pse_create, and the choice of (xi, rc, M, P)."""
import math

import numpy as np
import pytest

from oracle import sampler
from se_error import se_aliasing_estimate


def lib():
    import paper_1611_09322_amd as pse

    pse.load()
    return pse


@pytest.mark.parametrize("L,M,P,xi", [(34.73, 64, 8, 0.5), (240.8, 256, 8, 0.5), (111.77, 256, 6, 0.6),
                                      (60.0, 128, 10, 0.4), (40.0, 32, 4, 0.5)])
def test_derived_bounds_match_the_oracle_formulas(L, M, P, xi):
    pse = lib()
    p = pse.make_params(100, L, xi=xi, rcut=min(8.0, 0.49 * L), grid=M, support=P)
    d = pse.pse_derive(p)
    m = math.sqrt(math.pi * P)
    h = L / M
    assert d.h == pytest.approx(h, rel=1e-15)
    assert d.sigma == pytest.approx(P * h / (2 * m), rel=1e-15)
    assert d.eta_se == pytest.approx(4 * xi * xi * d.sigma**2, rel=1e-14)
    assert d.eps_real == pytest.approx(sampler.eps_real(xi, p.rcut), rel=1e-12)
    assert d.eps_wave == pytest.approx(sampler.eps_wave_bound(math.pi / h, xi, 1.0), rel=1e-9, abs=1e-300)
    assert d.eps_quad == pytest.approx(sampler.eps_quadrature(P, m), rel=1e-12)
    # the library sums the octant exactly up to 96 frequencies per axis and
    # on index blocks above; the tests' full-grid sum is the reference
    ref = se_aliasing_estimate(L, M, xi, P)
    assert d.eps_alias == pytest.approx(ref, rel=1e-10 if M <= 96 else 0.1)


def test_aliasing_estimate_falls_with_finer_grids_and_wider_windows():
    pse = lib()
    e = [pse.pse_derive(pse.make_params(100, 100.0, xi=0.5, rcut=8.0, grid=M, support=8)).eps_alias
         for M in (128, 256, 512)]
    assert e[0] > e[1] > e[2]
    e = [pse.pse_derive(pse.make_params(100, 100.0, xi=0.3, rcut=8.0, grid=128, support=P)).eps_alias
         for P in (4, 8, 12)]
    assert e[0] > e[1] > e[2]


def test_tolerance_rejects_parameters_above_it():
    pse = lib()
    # the 256^3 grid in a 240.8a box aliases at ~5e-4 (h = 0.94a)
    p = pse.make_params(10, 240.8, xi=0.5, rcut=8.0, grid=256, support=8)
    d = pse.pse_derive(p)
    assert 3e-4 < d.eps_alias < 8e-4
    p.tol = 1e-3
    pse.pse_derive(p)
    p.tol = 1e-4
    with pytest.raises(pse.PSEError) as e:
        pse.pse_derive(p)
    assert e.value.status == -4
    # real-space truncation at volume fraction 0.3 and xi rc = 2: the tail
    # estimate is ~2e-2
    q = pse.make_params(3000, 34.74, xi=0.5, rcut=4.0, grid=64, support=8)
    assert pse.pse_derive(q).eps_real_tail > 1e-2
    q.tol = 1e-3
    with pytest.raises(pse.PSEError):
        pse.pse_derive(q)
    # the same cutoff in a dilute box (10 spheres) has almost no pairs past
    # it: exp(-xi^2 rc^2) = exp(-4) alone would reject it
    q = pse.make_params(10, 60.0, xi=0.5, rcut=4.0, grid=128, support=8, err_tol=1e-3)
    assert pse.pse_derive(q).eps_real_tail < 1e-3 < pse.pse_derive(q).eps_real


def test_real_tail_is_the_shell_integral():
    """eps_real_tail and eps_real_coherent against an adaptive quadrature of
    the oracle's F, G (Appendix A) written here."""
    from scipy.integrate import quad

    from oracle import rpy

    pse = lib()
    for n, L, xi, rc, M in [(3000, 34.74, 0.5, 4.0, 64), (100000, 111.77, 0.56, 5.455, 256), (2000, 34.74, 0.3, 8.0, 64)]:
        rho = n / L**3

        def fg(r):
            F, G = rpy.real_FG(np.array([r]), xi, 1.0)
            return float(F[0]), float(G[0])

        inc = quad(lambda r: 4 * np.pi * r * r * (2 * fg(r)[0] ** 2 + fg(r)[1] ** 2) / 3, rc, rc + 20 / xi,
                   limit=200)[0]
        coh = quad(lambda r: 4 * np.pi * r * r * abs(2 * fg(r)[0] + fg(r)[1]) / 3, rc, rc + 20 / xi, limit=200)[0]
        d = pse.pse_derive(pse.make_params(n, L, xi=xi, rcut=rc, grid=M, support=8))
        assert d.eps_real_tail == pytest.approx(np.sqrt(rho * inc), rel=1e-4)
        assert d.eps_real_coherent == pytest.approx(rho * coh, rel=1e-4)


@pytest.mark.parametrize("n,phi", [(2000, 0.2), (3000, 0.3)])
def test_real_tail_predicts_the_truncation_error(n, phi):
    """The estimates against brute force on the oracle: the real-space
    product of hard-sphere configurations truncated at rc minus the product
    at a cutoff where the tail is below 1e-14 (rows sampled), relative to
    mu0 |F|; random forces for eps_real_tail, a uniform force for
    eps_real_coherent.  exp(-xi^2 rc^2) misses both by up to 7x."""
    import synth
    from oracle import rpy

    pse = lib()
    x, L = synth.hard_spheres(n, phi, seed=1500, sweeps=20)
    rows = np.random.default_rng(3).choice(n, 150, replace=False)
    mu0 = 1 / (6 * np.pi)
    Fr = synth.normals(5, (n, 3))
    Fu = np.zeros((n, 3))
    Fu[:, 2] = -1.0
    for xi, rc in ((0.5, 4.0), (0.5, 5.26), (0.7, 4.0)):
        rbig = min(np.sqrt(-np.log(1e-14)) / xi, 0.49 * L)
        d = pse.pse_derive(pse.make_params(n, L, xi=xi, rcut=rc, grid=64, support=8))
        du = rpy.real_matvec_rows(x, Fr, rows, L, 1, 1, xi, rc) - rpy.real_matvec_rows(x, Fr, rows, L, 1, 1, xi, rbig)
        e_inc = np.sqrt(np.mean(np.sum(du**2, 1)) / np.mean(np.sum(Fr[rows] ** 2, 1))) / mu0
        du = rpy.real_matvec_rows(x, Fu, rows, L, 1, 1, xi, rc) - rpy.real_matvec_rows(x, Fu, rows, L, 1, 1, xi, rbig)
        e_coh = np.sqrt(np.mean(np.sum(du**2, 1))) / mu0
        print(f"xi {xi} rc {rc}: random {e_inc:.3e} (estimate {d.eps_real_tail:.3e}), uniform {e_coh:.3e} "
              f"(estimate {d.eps_real_coherent:.3e}), exp(-xi^2 rc^2) {d.eps_real:.1e}")
        assert 0.8 < e_inc / d.eps_real_tail < 1.25
        assert 0.8 < e_coh / d.eps_real_coherent < 1.25


@pytest.mark.parametrize("tol", [1e-2, 1e-3, 1e-4, 1e-6])
def test_chosen_parameters_meet_every_bound(tol):
    pse = lib()
    base = pse.make_params(1_000_000, 240.8, precision="fp32")
    p, info = pse.pse_choose_params(base, pse.Tuning(tol=tol, with_forces=1))
    assert p.n == base.n and p.box == base.box and p.precision == base.precision
    # a sample has three error sources (real space, wave space, Krylov
    # iteration) adding in variance: each is held at tol / sqrt 3
    ts = tol / math.sqrt(3)
    assert p.lanczos_tol == pytest.approx(ts, rel=1e-15) and p.tol == tol
    d = pse.pse_derive(p)  # passes its own tolerance check
    assert d.eps_real_tail == pytest.approx(ts, rel=1e-6)  # the smallest rc that meets it
    assert info.eps_real_tail == d.eps_real_tail
    # the window (truncated on three axes, and aliased) errs in both the
    # spreading of the forces and the interpolation
    assert d.eps_wave + 2 * (3 * d.eps_quad + d.eps_alias) <= ts * (1 + 1e-9)
    assert d.eta_se < 1
    # independent full-grid aliasing sum at the chosen parameters
    if p.grid <= 256:
        assert se_aliasing_estimate(p.box, p.grid, p.xi, p.support, m=p.gauss_m) < 1.15 * ts
    # the next smaller support misses the tolerance at every width m (or
    # eta_SE reaches 1)
    if p.support > 2:
        P2 = p.support - 2
        for m in np.arange(2.0, 1.4 * math.sqrt(math.pi * P2) + 1e-9, 0.05):
            q = pse.make_params(p.n, p.box, xi=p.xi, rcut=p.rcut, grid=p.grid, support=P2, gauss_m=m)
            try:
                dq = pse.pse_derive(q)
            except pse.PSEError:
                continue  # eta_SE >= 1
            assert dq.eps_wave + 2 * (3 * dq.eps_quad + 0.9 * dq.eps_alias) > ts
    assert info.xi_star > 0 and info.model_seconds > 0


def test_deterministic_choice_bounds_the_coherent_tail():
    pse = lib()
    base = pse.make_params(1_000_000, 240.8 * (2 / 3) ** (1 / 3))  # volume fraction 0.3
    p, info = pse.pse_choose_params(base, pse.Tuning(tol=1e-3, deterministic=1))
    d = pse.pse_derive(p)
    # systematic errors add linearly: half the tolerance for each side
    ts = 1e-3 / 2
    assert d.eps_real_coherent == pytest.approx(ts, rel=1e-6) and info.eps_real_tail == d.eps_real_coherent
    assert d.eps_wave + 2 * (3 * d.eps_quad + d.eps_alias) <= ts * (1 + 1e-9)
    q, _ = pse.pse_choose_params(base, pse.Tuning(tol=1e-3, xi=p.xi))
    assert q.rcut < p.rcut  # the incoherent tail allows a shorter cutoff


def test_tighter_tolerance_costs_more():
    pse = lib()
    base = pse.make_params(100_000, 111.77, precision="mixed")
    prev = None
    for tol in (1e-2, 1e-3, 1e-4, 1e-5):
        p, info = pse.pse_choose_params(base, pse.Tuning(tol=tol))
        if prev is not None:
            assert info.model_seconds > prev.model_seconds
        prev = info


def test_fixed_xi_and_the_work_model_optimum():
    pse = lib()
    base = pse.make_params(1_000_000, 240.8, precision="fp32")
    t = pse.Tuning(tol=1e-3, with_forces=1)
    p, info = pse.pse_choose_params(base, t)
    # keeping the chosen xi gives the same parameters
    t.xi = p.xi
    q, qi = pse.pse_choose_params(base, t)
    assert (q.xi, q.rcut, q.grid, q.support) == (p.xi, p.rcut, p.grid, p.support)
    assert qi.model_seconds == pytest.approx(info.model_seconds, rel=1e-12)
    # any other xi of the scan costs at least as much in the model
    for xa in (0.3, 0.4, 0.7, 0.9):
        t.xi = xa
        try:
            _, oi = pse.pse_choose_params(base, t)
        except pse.PSEError:
            continue
        assert oi.model_seconds >= info.model_seconds * (1 - 1e-12)
    # more expensive pairs push the optimum to larger xi (less real-space work)
    t2 = pse.Tuning(tol=1e-3, with_forces=1, c_pair=4 * 1.96e-12)
    p2, _ = pse.pse_choose_params(base, t2)
    assert p2.xi >= p.xi


def test_optimum_moves_to_larger_xi_with_volume_fraction():
    """Sec. III (Fig. phiall) through eq. (work): real-space work grows
    as phi xi^-3 and the grid as xi^3 / phi at fixed N, so the work model's
    xi* grows with phi (as phi^(1/3) without the grid sizes' steps) while
    the optimal time, 2 sqrt of the product of the two coefficients, does
    not depend on phi.  512,000 hard spheres, tolerance 1e-3."""
    pse = lib()
    n = 512_000
    xs, ts = [], []
    for phi in (0.1, 0.2, 0.3, 0.4):
        L = (n * 4.0 * math.pi / (3.0 * phi)) ** (1.0 / 3.0)
        p, info = pse.pse_choose_params(pse.make_params(n, L, precision="mixed"), pse.Tuning(tol=1e-3, max_grid=512))
        xs.append(p.xi)
        ts.append(info.model_seconds)
    assert all(b >= a for a, b in zip(xs, xs[1:])), xs
    assert xs[-1] / xs[0] > 1.3, xs
    assert max(ts) / min(ts) < 1.25, ts


def test_infeasible_box_is_rejected():
    pse = lib()
    # in a 3a box the cutoff must stay below 1.5a, where the real-space tail
    # at xi a <= 1.5 is ~1e-2, far above 1e-10
    base = pse.make_params(2, 3.0)
    with pytest.raises(pse.PSEError) as e:
        pse.pse_choose_params(base, pse.Tuning(tol=1e-10, max_grid=16))
    assert e.value.status == -4
    with pytest.raises(pse.PSEError) as e:
        pse.pse_choose_params(base, pse.Tuning(tol=0.0))
    assert e.value.status == -1
