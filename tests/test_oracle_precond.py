"""Pins of the oracle's learned-preconditioner functions (no GPU): closed
forms for small configurations, invariances, finite differences, an
independent bf16 conversion and algebraic identities of the root."""
import numpy as np
import pytest
import torch

from oracle import lanczos, precond, rpy

A, ETA, XI, RC, L = 1.0, 1.0, 0.5, 6.0, 20.0


def test_pair_features_closed_form():
    """Two spheres 1.5a apart along x: every feature follows from the
    definitions with d = +-1.5 e_x."""
    r = 1.5
    x = np.array([[5.0, 5.0, 5.0], [5.0 - r, 5.0, 5.0]])
    f = precond.features(x, L, A, XI, RC)
    F, G = rpy.real_FG(np.array([r]), XI, A)
    F, G = F[0], G[0]
    exp0 = np.zeros(24)
    exp0[0:4] = [1 / 4, 1 / 8, 1 / 16, 1 / 128]
    exp0[4] = F / 8
    exp0[5] = G - F              # (G - F) dh_x dh_x
    exp0[11] = 1 / 4             # dh_x dh_x for r < 3a
    exp0[17] = +1 / 4            # dh = (x0 - x1)/r = +e_x
    exp0[20] = G - F
    exp0[21] = r / 4.5
    exp0[22] = (3 - r) / 4
    exp0[23] = rpy.real_self(XI, A)
    np.testing.assert_allclose(f[0], exp0, atol=1e-15)
    exp1 = exp0.copy()
    exp1[17] = -1 / 4
    np.testing.assert_allclose(f[1], exp1, atol=1e-15)


def test_features_count_far_neighbours_only_in_f3():
    """A neighbour at 5a (inside rc = 6a, outside the 4.5a near shell) enters
    f3 alone."""
    x = np.array([[5.0, 5.0, 5.0], [10.0, 5.0, 5.0]])
    f = precond.features(x, L, A, XI, RC)
    exp = np.zeros(24)
    exp[3] = 1 / 128
    exp[21] = 1.0
    exp[23] = rpy.real_self(XI, A)
    np.testing.assert_allclose(f, np.stack([exp, exp]), atol=1e-15)


def test_features_isolated_particle():
    f = precond.features(np.array([[1.0, 2.0, 3.0], [11.0, 12.0, 13.0]]), L, A, XI, RC)
    exp = np.zeros(24)
    exp[21] = 1.0
    exp[23] = rpy.real_self(XI, A)
    np.testing.assert_allclose(f, np.stack([exp, exp]), atol=1e-15)


def test_features_invariances():
    """Translation (with wrapping) leaves the features unchanged; a
    permutation permutes them; a 90 degree turn about z maps
    (xx, yy, zz, xy, xz, yz) -> (yy, xx, zz, -xy, -yz, xz) and (x, y, z) -> (-y, x, z)."""
    rng = np.random.default_rng(4)
    x = rng.uniform(0, L, (40, 3))
    f = precond.features(x, L, A, XI, RC)
    np.testing.assert_allclose(precond.features(x + np.array([7.3, -2.1, 31.0]), L, A, XI, RC), f, atol=1e-12)
    perm = rng.permutation(40)
    np.testing.assert_allclose(precond.features(x[perm], L, A, XI, RC), f[perm], atol=1e-12)
    c = L / 2
    xr = np.stack([c - (x[:, 1] - c), x[:, 0], x[:, 2]], axis=1)  # (x, y) -> (-y, x) about the centre
    fr = precond.features(xr, L, A, XI, RC)

    def rot_t(t):
        xx, yy, zz, xy, xz, yz = t.T
        return np.stack([yy, xx, zz, -xy, -yz, xz], axis=1)

    np.testing.assert_allclose(fr[:, 5:11], rot_t(f[:, 5:11]), atol=1e-12)
    np.testing.assert_allclose(fr[:, 11:17], rot_t(f[:, 11:17]), atol=1e-12)
    np.testing.assert_allclose(fr[:, 17:20], np.stack([-f[:, 18], f[:, 17], f[:, 19]], 1), atol=1e-12)
    scal = [0, 1, 2, 3, 4, 20, 21, 22, 23]
    np.testing.assert_allclose(fr[:, scal], f[:, scal], atol=1e-12)


def test_bf16_round_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000), [0.0, -0.0, 1e-40]])
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(precond.bf16_round(v), ref)
    assert precond.bf16_round(1 + 2.0**-8) == 1.0                       # tie -> even
    assert precond.bf16_round(1 + 3 * 2.0**-8) == 1 + 2.0**-6           # tie -> even (upwards)


def test_mlp_backward_matches_finite_differences():
    w = precond.init_weights(1, scale=0.3)
    x = np.random.default_rng(2).standard_normal((7, 24))
    dy = np.random.default_rng(3).standard_normal((7, 9))
    y, cache = precond.mlp_forward(w, x, bf16=False)
    g = precond.mlp_backward(w, cache, dy)
    h = 1e-6
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = w[k].reshape(-1)
        for idx in np.random.default_rng(6).choice(flat.size, 6, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            yp, _ = precond.mlp_forward(w, x, bf16=False)
            flat[idx] = old - h
            ym, _ = precond.mlp_forward(w, x, bf16=False)
            flat[idx] = old
            fd = np.sum(dy * (yp - ym)) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx)


def test_adam_constant_gradient_moves_by_lr_per_step():
    """With a constant gradient the bias-corrected moments are g and g^2, so
    every Adam step moves each weight by lr g / (|g| + eps)."""
    p = np.zeros(5)
    g = np.array([3.0, -0.5, 1e-3, 2.0, -7.0])
    m, v = np.zeros(5), np.zeros(5)
    for t in range(1, 6):
        before = p.copy()
        precond.adam_step(p, g, m, v, t, lr=0.01)
        np.testing.assert_allclose(p - before, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_block_fallback_rules():
    y = np.zeros((5, 9))
    y[1, 0] = np.nan                                  # not finite
    y[2] = (np.array([[0, 1, 0], [0, 0, 0], [0, 0, -1.0]]) - 0).reshape(9)  # P = [[1,1,0],[0,1,0],[0,0,0]]: singular
    y[3, 8] = 1e-4 - 1.0                              # P = diag(1, 1, 1e-4): cond 1e4
    y[4] = 0.1 * np.arange(9) / 9                     # a fine block
    P, bad = precond.blocks_from_output(y)
    assert list(bad) == [False, True, True, True, False]
    np.testing.assert_array_equal(P[0], np.eye(3))
    for i in (1, 2, 3):
        np.testing.assert_array_equal(P[i], np.eye(3))
    np.testing.assert_allclose(P[4], np.eye(3) + y[4].reshape(3, 3))


@pytest.fixture(scope="module")
def small_system():
    rng = np.random.default_rng(9)
    x = rng.uniform(0, 12.0, (20, 3))
    Mr = rpy.real_block_dense(x, 12.0, A, ETA, XI, 5.0)
    return x, Mr


def test_precond_root_identities(small_system):
    """P = I gives the plain symmetric root; for any invertible P the map
    S = P^-1 A^1/2 satisfies S S^T = M_r, and y^T M_r^-1 y = |z|^2."""
    x, Mr = small_system
    rng = np.random.default_rng(10)
    z = rng.standard_normal(60)
    P0 = np.tile(np.eye(3), (20, 1, 1))
    np.testing.assert_allclose(precond.precond_real_sample(Mr, P0, z), lanczos.sqrt_apply(Mr, z), atol=1e-13)
    P = np.eye(3)[None] + 0.3 * rng.standard_normal((20, 3, 3))
    S = np.stack([precond.precond_real_sample(Mr, P, e) for e in np.eye(60)], axis=1)
    np.testing.assert_allclose(S @ S.T, Mr, atol=1e-13)
    y = precond.precond_real_sample(Mr, P, z)
    assert abs(y @ np.linalg.solve(Mr, y) - z @ z) < 1e-9 * (z @ z)


def test_target_isolated_particle_is_identity():
    x = np.array([[2.0, 2.0, 2.0], [12.0, 12.0, 12.0]])
    T = precond.targets(x, [0, 1], L, A, ETA, XI, RC)
    np.testing.assert_allclose(T, np.stack([np.eye(3)] * 2), atol=1e-12)


def test_target_pair_closed_form():
    """Two particles r apart along x, nothing else within reach: the patch
    matrix is [[s I, B], [B, s I]] with B = mu0 diag(G, F, F) and s = mu0
    F_self, so [M^-1]_11 = diag(s / (s^2 - b^2)) and the normalised target is
    diag(1 / sqrt(1 - (b / s)^2)) with b = (G, F, F) mu0."""
    r = 2.7
    x = np.array([[6.0, 6.0, 6.0], [6.0 + r, 6.0, 6.0]])
    T = precond.targets(x, [0], L, A, ETA, XI, RC)[0]
    F, G = rpy.real_FG(np.array([r]), XI, A)
    Fs = rpy.real_self(XI, A)
    exp = np.diag(1.0 / np.sqrt(1.0 - (np.array([G[0], F[0], F[0]]) / Fs) ** 2))
    np.testing.assert_allclose(T, exp, atol=1e-12)


@pytest.mark.parametrize("kind,phi,xi", [("hard spheres", 0.3, 0.5), ("gel", 0.05, 0.5), ("gel", 0.05, 0.2)])
def test_ideal_block_preconditioner_leaves_the_krylov_work_unchanged(kind, phi, xi):
    """Hard spheres at phi = 0.3 and a DLCA gel at phi = 0.05 (contact
    chains, d_f ~ 2), at xi a = 0.5 and, for the gel, 0.2 (a smaller xi moves
    work into real space and raises kappa(M_r)), rc from exp(-xi^2 rc^2) =
    1e-3.  Every diagonal block of M_r is the self term plus a little, and
    the spread of its spectrum comes from pair coupling.  Even the ideal
    block preconditioner, the symmetric root of the ii block of M_r^{-1},
    lowers kappa(P M_r P^T) by at most ~12 % and the tol-1e-3 Krylov sample
    needs as many iterations.  This is why the learned blocks cannot pay for
    themselves on these structures."""
    import synth

    if kind == "gel":
        x, Lb, _, _ = synth.dlca_gel(500, phi, seed=3)
    else:
        x, Lb = synth.hard_spheres(300, phi, a=1.0, seed=3, sweeps=20)
    rc = min(np.sqrt(-np.log(1e-3)) / xi * 1.1, 0.49 * Lb)
    Mr = rpy.real_block_dense(x, Lb, A, ETA, xi, rc)
    Minv = np.linalg.inv(Mr)
    P = np.array([precond._sqrtm_spd(Minv[3 * i:3 * i + 3, 3 * i:3 * i + 3]) for i in range(len(x))])
    B = precond.block_diag(P)
    Ap = B @ Mr @ B.T
    lam0 = np.linalg.eigvalsh(Mr)
    lam1 = np.linalg.eigvalsh(0.5 * (Ap + Ap.T))
    k0, k1 = lam0[-1] / lam0[0], lam1[-1] / lam1[0]
    z = np.random.default_rng(1).standard_normal(3 * len(x))
    _, m0, _ = lanczos.lanczos_sqrt(lambda v: Mr @ v, z, 1e-3)
    _, m1, _ = lanczos.lanczos_sqrt(lambda v: Ap @ v, z, 1e-3)
    print(f"{kind} phi {phi} xi {xi}: kappa {k0:.3f} -> {k1:.3f}, iterations {m0} -> {m1}")
    assert k1 >= 0.85 * k0
    assert m1 >= m0
