"""Pins of the oracle's counter-based noise, composed sample and error bounds
(no GPU)."""
import numpy as np
import pytest

from oracle import ewald, lanczos, philox, rpy, sampler


def test_philox_matches_numpy_bit_generator():
    """oracle.philox.philox4x64_10 is the published Philox-4x64-10 block
    function: numpy's Philox bit generator (an independent implementation
    of the same definition) returns block(ctr + 1, key) as its next four
    words."""
    rng = np.random.default_rng(0)
    for _ in range(5):
        ctr = [int(v) for v in rng.integers(0, 2**63, 4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2**63, 2, dtype=np.uint64)]
        bg = np.random.Philox(counter=ctr, key=key)
        got = bg.random_raw(8)
        for blk in range(2):
            c = ctr.copy()
            c[0] += 1 + blk  # no carry for these counters
            w = philox.philox4x64_10([np.uint64(v) for v in c], [np.uint64(v) for v in key])
            assert [int(v) for v in w] == [int(v) for v in got[4 * blk : 4 * blk + 4]]


def test_mulhilo_exact():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2**64 - 1, 64, dtype=np.uint64, endpoint=True)
    b = rng.integers(0, 2**64 - 1, 64, dtype=np.uint64, endpoint=True)
    hi, lo = philox.mulhilo64(a, b)
    for x, y, h, l in zip(a, b, hi, lo):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & (2**64 - 1)


@pytest.mark.parametrize("bits", [53, 24])
def test_normals_moments(bits):
    z = philox.real_noise(40000, seed=9, sample=3, bits=bits)
    assert abs(z.mean()) < 5 * 1 / np.sqrt(len(z))
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / len(z))
    # different sample counters give independent vectors
    z2 = philox.real_noise(40000, seed=9, sample=4, bits=bits)
    assert abs(np.corrcoef(z, z2)[0, 1]) < 5 / np.sqrt(len(z))


def test_wave_noise_conjugate_symmetric_and_unit():
    M = 8
    Z = philox.wave_noise_full(M, seed=5, sample=0)
    s = np.fft.fftfreq(M, 1.0 / M).astype(int)
    neg = (-np.arange(M)) % M
    # zeta(-k) = conj zeta(k) everywhere
    np.testing.assert_array_equal(Z[:, neg][:, :, neg][:, :, :, neg], np.conj(Z))
    assert np.all(Z[:, 0, 0, 0] == 0)
    ny = np.abs(s) == M // 2
    assert np.all(Z[:, ny] == 0) and np.all(Z[:, :, ny] == 0) and np.all(Z[:, :, :, ny] == 0)
    # over many draws: E|zeta|^2 = 1 and E zeta^2 = 0 on the k-set
    acc2 = 0.0
    accsq = 0.0
    n = 300
    for t in range(n):
        Zt = philox.wave_noise_full(M, seed=5, sample=t)
        acc2 = acc2 + np.abs(Zt) ** 2
        accsq = accsq + Zt**2
    _, _, _, _, OK = ewald.grid_kvectors(M, 1.0)
    m2 = (acc2 / n)[:, OK]
    assert abs(m2.mean() - 1) < 0.01
    assert np.abs((accsq / n)[:, OK]).mean() < 0.1


def test_wave_sample_from_philox_covariance_is_wave_mobility():
    """Sampled covariance of y_w built from the Philox k-space noise tends to
    M_w over the grid k-set (per-entry 5 sigma)."""
    rng = np.random.default_rng(3)
    L, M, xi = 5.0, 8, 0.9
    x = rng.uniform(0, L, (2, 3))
    Mw = ewald.wave_block_dense(x, L, 1.0, 1.0, xi, ewald.kset_grid(M))
    n = 4000
    Y = np.array([ewald.wave_sample_direct(x, philox.wave_noise_full(M, 17, t), L, 1.0, 1.0, xi).ravel()
                  for t in range(n)])
    C = Y.T @ Y / n
    d = np.sqrt(np.diag(Mw))
    sig = np.sqrt((np.outer(d, d) ** 2 + Mw**2) / n)
    assert np.all(np.abs(C - Mw) < 5 * sig + 1e-15)


def test_displacement_composition_scales():
    """dx = sqrt(2 kT dt)(y_r + y_w) + dt M F: linear in each noise and in F
    with the stated scalings (eq. langevin, eq. split)."""
    rng = np.random.default_rng(2)
    p = sampler.Params(L=9.0, xi=0.7, rc=4.0, M=8, kT=1.7, eta=0.9)
    x = rng.uniform(0, p.L, (4, 3))
    z1 = rng.standard_normal(12)
    W = rng.standard_normal((3, 8, 8, 8))
    F = rng.standard_normal((4, 3))
    d1 = sampler.displacement_from_grid_noise(x, z1, W, p, dt=0.25)
    d0 = sampler.displacement_from_grid_noise(x, z1, 0 * W, p, dt=0.25)
    dw = sampler.displacement_from_grid_noise(x, 0 * z1, W, p, dt=0.25)
    np.testing.assert_allclose(d1, d0 + dw, atol=1e-14)
    Mr = rpy.real_block_dense(x, p.L, p.a, p.eta, p.xi, p.rc)
    np.testing.assert_allclose(d0.ravel(), np.sqrt(2 * p.kT * 0.25) * lanczos.sqrt_apply(Mr, z1), atol=1e-14)
    dF = sampler.displacement_from_grid_noise(x, 0 * z1, 0 * W, p, dt=0.25, forces=F)
    Mw = ewald.wave_block_dense(x, p.L, p.a, p.eta, p.xi, ewald.kset_grid(p.M))
    np.testing.assert_allclose(dF.ravel(), 0.25 * (Mr + Mw) @ F.ravel(), atol=1e-14)


@pytest.mark.parametrize("xi", [0.3, 0.5, 1.0])
def test_wave_truncation_bound_holds(xi):
    """The analytic bound of Sec. II D is an upper bound on the truncated
    wave-space self-mobility error (eq. errbound with the PSE kernel)."""
    for kc in [2.0, 4.0, 6.0]:
        exact = sampler.eps_wave_exact_self(kc, xi, 1.0)
        bound = sampler.eps_wave_bound(kc, xi, 1.0)
        assert exact <= bound * (1 + 1e-9) + 1e-300


def test_real_truncation_error_scale():
    """Cutting M_r at rc changes it by O(exp(-xi^2 rc^2)) (Sec. II C)."""
    rng = np.random.default_rng(4)
    L, xi = 20.0, 0.5
    x = rng.uniform(0, L, (30, 3))
    ref = rpy.real_block_dense(x, L, 1.0, 1.0, xi, 9.5)
    for rc in [4.0, 5.0, 6.0]:
        diff = np.abs(rpy.real_block_dense(x, L, 1.0, 1.0, xi, rc) - ref).max() * 6 * np.pi
        assert diff < 10 * sampler.eps_real(xi, rc)


def test_quadrature_error_formula():
    """m = sqrt(pi P) balances the two terms of eps_q (Sec. II C); P = 8
    gives about 4e-6."""
    P = 8
    m = np.sqrt(np.pi * P)
    e = sampler.eps_quadrature(P, m)
    assert 1e-6 < e < 1e-5
