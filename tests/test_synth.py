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
