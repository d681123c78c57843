"""Pins of the oracle's periodic (Ewald) mobility and wave-space sums (no GPU)."""
import json
import os

import numpy as np
import pytest

from oracle import ewald, lanczos, rpy

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _total(x, L, xi, a=1.0, eta=1.0):
    rc = 7.0 / xi
    Mr = rpy.real_block_dense(x, L, a, eta, xi, rc)
    Mw = ewald.wave_block_dense(x, L, a, eta, xi, ewald.kset_converged(L, xi))
    return Mr, Mw


def test_total_mobility_independent_of_xi():
    """M = M_r + M_w does not depend on the splitting parameter (the split of
    eq. pairmobility into eqs. Mwave + Mreal is exact), including an
    overlapping pair."""
    L = 9.0
    x = np.array([[1.0, 1.0, 1.0], [2.3, 1.4, 0.6], [5.0, 6.0, 7.5], [8.6, 0.2, 4.4]])
    tots = []
    for xi in [0.3, 0.6, 1.2]:
        Mr, Mw = _total(x, L, xi)
        tots.append(Mr + Mw)
    scale = np.abs(tots[0]).max()
    assert np.abs(tots[1] - tots[0]).max() < 1e-12 * scale
    assert np.abs(tots[2] - tots[0]).max() < 1e-12 * scale


def test_hasimoto_self_mobility():
    """One sphere in a periodic box: mu_self/mu_0 = 1 - 2.837297 a/L +
    (4 pi/3)(a/L)^3 (Hasimoto's constant for the periodic Green's function
    of eq. green)."""
    g = json.load(open(os.path.join(GOLD, "hasimoto_self_mobility.json")))
    for L in g["L_over_a"]:
        Mr, Mw = _total(np.array([[0.3, 0.2, 0.1]]), L, 0.6)
        mu = (Mr + Mw) * 6 * np.pi
        expect = 1 - g["c1"] / L + 4 * np.pi / 3 / L**3
        np.testing.assert_allclose(np.diag(mu), expect, atol=g["tolerance_abs"])
        assert np.abs(mu - np.diag(np.diag(mu))).max() < 1e-13


@pytest.mark.parametrize("r", [1.5, 3.0])
def test_large_box_pair_tends_to_free_rpy(r):
    """A pair in a large box: the periodic pair mobility is the free RPY
    tensor (eq. RPY_free_space; both the overlapping and the separated
    branch) shifted by the uniform periodic correction -2.837297 a/L I, up to
    O(a r^2 / L^3)."""
    L, xi = 200.0, 0.1
    d = np.array([r, 0.0, 0.0]) / np.sqrt(1.0)
    rot = np.linalg.qr(np.random.default_rng(1).standard_normal((3, 3)))[0]
    d = rot @ d
    x = np.array([[50.0, 60.0, 70.0], [50.0, 60.0, 70.0] + d])
    Mr, Mw = _total(x, L, xi)
    M = (Mr + Mw) * 6 * np.pi
    pair = M[0:3, 3:6]
    expect = rpy.rpy_free_tensor(-d, 1.0, 1.0) * 6 * np.pi - 2.837297 / L * np.eye(3)
    np.testing.assert_allclose(pair, expect, atol=2e-5)


@pytest.mark.parametrize("xi", [0.1, 0.3, 0.5, 1.0, 2.0])
def test_both_parts_positive_definite_with_overlaps(xi):
    """App. B: with 0 <= H <= 1 both split parts are SPD for every
    configuration, overlapping ones included."""
    rng = np.random.default_rng(int(xi * 100))
    L = 8.0
    x = rng.uniform(0, L, (24, 3))  # dense: many overlapping pairs
    x[1] = x[0] + 0.05  # a nearly coincident pair
    Mr, Mw = _total(x, L, xi)
    lr = np.linalg.eigvalsh(Mr)
    lw = np.linalg.eigvalsh(Mw)
    assert lr.min() > 0
    assert lw.min() > -1e-13 * lw.max()


def test_beenakker_splitting_is_not_bounded_by_one():
    """Negative control from Sec. II A.1: Beenakker's H_B exceeds 1 for some
    k, so 1 - H_B < 0 and the real-space weight is not non-negative, while
    Hasimoto's H stays in [0, 1]."""
    k = np.linspace(0, 20, 20001)
    assert rpy.H_beenakker(k, 1.0).max() > 1.0
    h = rpy.H_split(k, 1.0)
    assert h.max() <= 1.0 + 1e-15 and h.min() >= 0.0


def test_grid_nudft_matches_dense_wave_block():
    """M_w F by separable type-1/type-2 sums equals the dense cos/sin form of
    eq. (Mwave) over the same grid k-set."""
    rng = np.random.default_rng(5)
    L, M, xi = 7.0, 8, 0.9
    x = rng.uniform(-3, 10, (5, 3))  # unwrapped coordinates are fine
    F = rng.standard_normal((5, 3))
    Mw = ewald.wave_block_dense(x, L, 1.0, 1.3, xi, ewald.kset_grid(M))
    u = ewald.wave_apply_direct(x, F, M, L, 1.0, 1.3, xi)
    np.testing.assert_allclose(u.ravel(), Mw @ F.ravel(), atol=1e-14 * np.abs(Mw).max() * 10)


def test_wave_sample_map_reproduces_wave_mobility():
    """The wave sample is linear in the grid noise W: y = A W.  Its covariance
    A A^T must equal M_w over the grid k-set exactly (Sec. II B.2: M_w =
    (D^H B^{1/2})(D^H B^{1/2})^H), which fixes the scaling, the projector
    and the conjugate-symmetric construction of zeta."""
    rng = np.random.default_rng(7)
    L, M, xi, a, eta = 6.0, 8, 0.8, 1.0, 0.7
    x = rng.uniform(0, L, (3, 3))
    x[1] = x[0] + np.array([0.5, 0.3, -0.2])  # overlapping pair
    cols = []
    for c in range(3):
        for idx in range(M**3):
            W = np.zeros((3, M, M, M))
            W[c].flat[idx] = 1.0
            cols.append(ewald.wave_sample_direct(x, ewald.zeta_from_grid_noise(W), L, a, eta, xi).ravel())
    A = np.array(cols).T
    Mw = ewald.wave_block_dense(x, L, a, eta, xi, ewald.kset_grid(M))
    np.testing.assert_allclose(A @ A.T, Mw, atol=1e-14 * np.abs(Mw).max() * 10)


def test_lanczos_reference_converges_to_symmetric_root():
    """The Krylov iterate tends to the eigendecomposition root, and any root
    satisfies y^T M_r^{-1} y = |z|^2."""
    rng = np.random.default_rng(11)
    L, xi = 10.0, 0.5
    x = rng.uniform(0, L, (40, 3))
    Mr = rpy.real_block_dense(x, L, 1.0, 1.0, xi, 4.9)
    z = rng.standard_normal(120)
    y_ex = lanczos.sqrt_apply(Mr, z)
    assert abs(y_ex @ np.linalg.solve(Mr, y_ex) - z @ z) < 1e-10 * (z @ z)
    y, it, _ = lanczos.lanczos_sqrt(lambda v: Mr @ v, z, tol=1e-12, max_iter=120)
    assert np.linalg.norm(y - y_ex) < 1e-10 * np.linalg.norm(y_ex)
    y3, it3, _ = lanczos.lanczos_sqrt(lambda v: Mr @ v, z, tol=1e-3)
    assert np.linalg.norm(y3 - y_ex) <= 1e-3 * np.linalg.norm(y_ex)
    assert it3 < it
