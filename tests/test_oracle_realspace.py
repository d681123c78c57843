"""Pins of the oracle's real-space functions against what the paper and the
mathematics fix (no GPU)."""
import numpy as np
import pytest

from oracle import lanczos, rpy


XIS = [0.2, 0.5, 1.0, 3.0]
RS = [0.35, 1.0, 1.7, 1.999, 2.0, 2.001, 2.5, 3.0, 5.0, 8.0]


@pytest.mark.parametrize("xi", XIS)
def test_closed_forms_plus_wave_integral_give_free_rpy(xi):
    """Appendix A (real part, 1 - H) + the H-weighted integral (wave part)
    = the sinc^2-weighted integral = free RPY, eq. (RPY_free_space), for
    r on both sides of 2a.  A dropped term, wrong sign or swapped F/G in the
    transcribed closed forms breaks this identity."""
    a = 1.0
    r = np.array(RS)
    keep = r**3 * xi**4 > 2e-4
    r = r[keep]
    F, G = rpy.real_FG_closed(r, xi, a)
    Fw, Gw = rpy.wave_FG_quad(r, xi, a)
    Ff, Gf = rpy.rpy_free_FG(r, a)
    np.testing.assert_allclose(F + Fw, Ff, rtol=0, atol=2e-11)
    np.testing.assert_allclose(G + Gw, Gf, rtol=0, atol=2e-11)


@pytest.mark.parametrize("xi", [0.3, 0.5, 1.0, 2.0])
def test_self_term_is_limit_and_complements_wave_self(xi):
    """eq. (self) is the r -> 0 limit of F and G, and the real plus wave self
    mobility is exactly the Stokes drag (6 pi eta a M_ii = 1)."""
    a = 1.0
    Fs = rpy.real_self(xi, a)
    Fw0, Gw0 = rpy.wave_FG_quad(np.array([0.0]), xi, a)
    assert abs(Fs + Fw0[0] - 1.0) < 1e-13
    assert abs(Fs + Gw0[0] - 1.0) < 1e-13
    F, G = rpy.real_FG(np.array([1e-6, 1e-4]), xi, a)
    # leading departure from the self value is the free RPY -9r/32a (F), -3r/16a (G)
    np.testing.assert_allclose(F, Fs - 9 / 32 * np.array([1e-6, 1e-4]), atol=1e-8)
    np.testing.assert_allclose(G, Fs - 3 / 16 * np.array([1e-6, 1e-4]), atol=1e-8)


@pytest.mark.parametrize("xi", [0.3, 0.7, 2.0])
def test_case_boundary_continuity(xi):
    """Case 1 and Case 2 of Appendix A meet continuously at r = 2a
    (f0 = g0 = 0 there)."""
    eps = 1e-9
    Fl, Gl = rpy.real_FG_closed(np.array([2.0 - eps]), xi, 1.0)
    Fr, Gr = rpy.real_FG_closed(np.array([2.0 + eps]), xi, 1.0)
    assert abs(Fl[0] - Fr[0]) < 1e-8 and abs(Gl[0] - Gr[0]) < 1e-8


def test_small_r_route_matches_closed_forms_where_both_hold():
    """The quadrature route (F_free - F_w) and the closed forms agree in the
    range where the closed forms are still well conditioned."""
    for xi in [0.5, 1.0]:
        r = np.array([0.4, 0.8, 1.5])
        Fc, Gc = rpy.real_FG_closed(r, xi, 1.0)
        Ff, Gf = rpy.rpy_free_FG(r, 1.0)
        Fw, Gw = rpy.wave_FG_quad(r, xi, 1.0)
        np.testing.assert_allclose(Fc, Ff - Fw, atol=1e-12)
        np.testing.assert_allclose(Gc, Gf - Gw, atol=1e-12)


def test_kernel_series_continuity():
    u = np.array([0.4999999, 0.5000001])
    # series below 0.5, closed form above: values agree across the switch
    assert abs(np.diff(rpy.kernel_KF(u))[0]) < 1e-7
    assert abs(np.diff(rpy.kernel_KG(u))[0]) < 1e-7
    # the u -> 0 limits are the isotropic 2/3 and 1/3
    assert abs(rpy.kernel_KF(np.array([0.0]))[0] - 2 / 3) < 1e-15
    assert abs(rpy.kernel_KG(np.array([0.0]))[0] - 1 / 3) < 1e-15


def test_real_block_symmetric_and_rows_match():
    """M_r is symmetric; the brute-force row product equals the dense rows."""
    rng = np.random.default_rng(3)
    L, xi, rc = 12.0, 0.6, 5.0
    x = rng.uniform(0, L, (25, 3))
    Mr = rpy.real_block_dense(x, L, 1.0, 1.0, xi, rc)
    assert np.abs(Mr - Mr.T).max() < 1e-15
    v = rng.standard_normal(75)
    rows = [0, 7, 24]
    got = rpy.real_matvec_rows(x, v, rows, L, 1.0, 1.0, xi, rc)
    ref = (Mr @ v).reshape(-1, 3)[rows]
    np.testing.assert_allclose(got, ref, atol=1e-14)


def test_single_particle_real_sample_closed_form():
    """N = 1 with rc < L/2: M_r = F_self/(6 pi eta a) I, so the symmetric root
    sample is sqrt(F_self/(6 pi eta a)) z."""
    L, xi, rc, a, eta = 20.0, 0.5, 8.0, 1.0, 1.3
    x = np.array([[3.0, 4.0, 5.0]])
    Mr = rpy.real_block_dense(x, L, a, eta, xi, rc)
    z = np.array([0.3, -1.2, 2.0])
    y = lanczos.sqrt_apply(Mr, z)
    np.testing.assert_allclose(y, np.sqrt(rpy.real_self(xi, a) / (6 * np.pi * eta * a)) * z, rtol=1e-14)


def test_free_rpy_tensor_values():
    """eq. (RPY_free_space) at contact r = 2a from both branches, and the
    Stokes drag at r = 0."""
    a = 1.0
    d = np.array([2.0, 0.0, 0.0])
    T = rpy.rpy_free_tensor(d, a, 1.0) * 6 * np.pi
    # r <= 2a branch at r = 2a: I coeff 1 - 9/16, rr coeff 3/16
    np.testing.assert_allclose(np.diag(T), [1 - 9 / 16 + 3 / 16, 1 - 9 / 16, 1 - 9 / 16], atol=1e-15)
    # r > 2a branch just outside: 3/8 + 1/16 and 3/8 - 3/16
    T2 = rpy.rpy_free_tensor(np.array([2.0 + 1e-12, 0, 0]), a, 1.0) * 6 * np.pi
    np.testing.assert_allclose(T2, T, atol=1e-11)
    np.testing.assert_allclose(rpy.rpy_free_tensor(np.zeros(3), a, 1.0) * 6 * np.pi, np.eye(3))


def test_real_block_is_periodic_in_positions():
    """Shifting any particle by a lattice vector (several box lengths)
    leaves M_r unchanged: positions are defined modulo L."""
    rng = np.random.default_rng(8)
    L, xi, rc = 10.0, 0.6, 4.5
    x = rng.uniform(0, L, (12, 3))
    y = x.copy()
    y[3] += L * np.array([2, -3, 1])
    y[7] -= L * np.array([0, 0, 4])
    np.testing.assert_allclose(rpy.real_block_dense(y, L, 1.0, 1.0, xi, rc),
                               rpy.real_block_dense(x, L, 1.0, 1.0, xi, rc), atol=1e-15)
