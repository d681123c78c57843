"""The seeded input generators (no method arithmetic): hard-sphere
configurations are non-overlapping at every volume fraction the workloads
use, including above the random-sequential-addition range."""
import numpy as np

import synth


def test_lattice_start_is_fcc_and_non_overlapping():
    n, phi = 3000, 0.4
    L = synth.box_side(n, phi)
    x = synth.lattice_positions(n, L, 1.0, seed=4)
    assert x.shape == (n, 3)
    assert np.all(x >= 0.0) and np.all(x < L)
    assert len(np.unique(np.round(x, 9), axis=0)) == n
    m = int(np.ceil((n / 4.0) ** (1.0 / 3.0)))
    # nearest neighbours of an FCC lattice of cube edge L / m: L / (m sqrt 2)
    assert abs(synth.min_pair_distance(x, L) - L / (m * np.sqrt(2.0))) < 1e-9


def test_hard_spheres_above_rsa_range():
    for n, phi in [(2000, 0.4), (3000, 0.45)]:
        x, L = synth.hard_spheres(n, phi, seed=11, sweeps=60)
        assert x.shape == (n, 3)
        assert abs(n * 4.0 / 3.0 * np.pi / L**3 - phi) < 1e-12
        assert synth.min_pair_distance(x, L) >= 2.0
        assert np.all(x >= 0.0) and np.all(x < L)


def test_hard_spheres_below_the_switch_use_rsa():
    x, L = synth.hard_spheres(500, synth.RSA_MAX_PHI - 0.05, seed=3)
    assert synth.min_pair_distance(x, L) >= 2.0
    # RSA places spheres at random: no lattice nearest-neighbour distance
    m = int(np.ceil((500 / 4.0) ** (1.0 / 3.0)))
    assert abs(synth.min_pair_distance(x, L) - L / (m * np.sqrt(2.0))) > 1e-6


def test_dlca_gel_is_one_touching_fractal_network():
    """The gel generator: no overlaps (contacts at 2a up to rounding), one
    cluster holding at least 90 % of the spheres, every sphere of a cluster
    of two or more touching another of its own cluster, and a mass-radius
    slope well below the 3 of a uniform suspension at the same volume
    fraction (about 2.2 on [2.5a, 6a] at phi = 0.05)."""
    from scipy.spatial import cKDTree

    n, phi = 6000, 0.05
    x, L, lab, st = synth.dlca_gel(n, phi, seed=11)
    assert synth.min_pair_distance(x, L) > 2.0 - 1e-9
    assert st["largest"] >= 0.9 * n and st["clusters"] >= 1
    big = np.bincount(lab).argmax()
    assert np.count_nonzero(lab == big) == st["largest"]
    t = cKDTree(np.mod(x, L), boxsize=L)
    sizes = np.bincount(lab)
    for i, j in ((i, j) for i, j in t.query_pairs(2.0 + 1e-7)):
        assert lab[i] == lab[j]  # contacts join clusters
    touching = np.zeros(n, bool)
    for i, j in t.query_pairs(2.0 + 1e-7):
        touching[i] = touching[j] = True
    assert np.all(touching[sizes[lab] > 1])
    s_gel = synth.mass_radius_slope(x, L, 2.5, 6.0)
    s_hs = synth.mass_radius_slope(synth.rsa_positions(n, L, seed=12), L, 2.5, 6.0)
    print(f"gel slope {s_gel:.2f}, uniform {s_hs:.2f}, {st}")
    assert 1.7 < s_gel < 2.6 and s_hs > 2.8


def test_dlca_gel_is_seeded():
    a = synth.dlca_gel(800, 0.05, seed=3)
    b = synth.dlca_gel(800, 0.05, seed=3)
    c = synth.dlca_gel(800, 0.05, seed=4)
    assert np.array_equal(a[0], b[0]) and not np.array_equal(a[0], c[0])
