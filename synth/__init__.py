"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module generates inputs only (particle configurations and plain i.i.d.
normal arrays); it holds none of the sampler's arithmetic.

Configurations follow the paper's workloads (random hard-sphere suspensions
and colloidal gels, Sec. III): random sequential addition (RSA) at volume
fraction phi in a cubic periodic box, optionally relaxed by hard-sphere Monte
Carlo sweeps; gels by diffusion-limited cluster aggregation from an RSA
start; uniform random points (overlaps allowed, for the overlap cases of the
RPY tensor).
The C part (csrc/hs_gen.c) is compiled on first use with gcc -fopenmp.
"""
import ctypes
import os
import subprocess
from math import pi

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "hs_gen.c")
_LIB = os.path.join(_HERE, "_hs_gen.so")
_lib = None


def build(force=False):
    """Compile the generator library in-tree (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.rsa_fill.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, dp, ctypes.c_longlong]
        lib.rsa_fill.restype = ctypes.c_int
        lib.mc_relax.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int, ctypes.c_uint64,
                                 ctypes.c_double, dp, ctypes.c_int]
        lib.mc_relax.restype = ctypes.c_double
        lib.min_pair_distance.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        lib.min_pair_distance.restype = ctypes.c_double
        lib.dlca_gel.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_longlong, dp,
                                 ctypes.POINTER(ctypes.c_int32), dp]
        lib.dlca_gel.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(arr):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def box_side(n, phi, a=1.0):
    """Side of the cubic box holding n spheres of radius a at volume fraction phi."""
    return (n * 4.0 * pi * a**3 / (3.0 * phi)) ** (1.0 / 3.0)


def uniform_positions(n, L, seed):
    """n points uniform in [0, L)^3 (overlaps allowed)."""
    return np.random.default_rng(seed).uniform(0.0, L, size=(n, 3))


def rsa_positions(n, L, a=1.0, seed=0, max_attempts=None):
    """Random sequential addition of n non-overlapping spheres."""
    x = np.zeros((n, 3), dtype=np.float64)
    if max_attempts is None:
        max_attempts = 2000 * n + 10**6
    placed = _load().rsa_fill(n, L, a, seed, _dp(x), max_attempts)
    if placed != n:
        raise RuntimeError(f"RSA placed only {placed} of {n} spheres (phi too high for RSA)")
    return x


def mc_relax(x, L, a=1.0, sweeps=100, seed=0, target_acc=0.4, adapt_sweeps=None):
    """Hard-sphere MC displacement sweeps in place; returns (x, step, last acceptance)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    step = ctypes.c_double(0.1 * a)
    if adapt_sweeps is None:
        adapt_sweeps = min(sweeps, 50)
    acc = _load().mc_relax(len(x), L, a, _dp(x), sweeps, seed, target_acc, ctypes.byref(step), adapt_sweeps)
    return x, step.value, acc


def min_pair_distance(x, L, a=1.0):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return _load().min_pair_distance(len(x), L, a, _dp(x))


# Random sequential addition slows sharply on its way to its jamming limit
# (phi ~ 0.38); above this volume fraction the start is a lattice instead.
RSA_MAX_PHI = 0.35


def lattice_positions(n, L, a=1.0, seed=0):
    """n spheres on a randomly vacated FCC lattice filling the box: m^3 unit
    cells (4 sites each, m the smallest with 4 m^3 >= n), n sites drawn
    without replacement.  Non-overlapping when the nearest-neighbour
    distance L / (m sqrt 2) is at least 2a (checked)."""
    m = int(np.ceil((n / 4.0) ** (1.0 / 3.0) - 1e-9))
    while 4 * m**3 < n:
        m += 1
    s = L / m
    if s / np.sqrt(2.0) < 2.0 * a:
        raise RuntimeError(f"an FCC lattice of {4 * m**3} sites in a box of {L:.3f} overlaps spheres of radius {a}")
    g = np.arange(m, dtype=np.float64)
    cx, cy, cz = np.meshgrid(g, g, g, indexing="ij")
    corner = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    sites = ((corner[:, None, :] + basis[None, :, :]).reshape(-1, 3) + 0.25) * s
    pick = np.sort(np.random.default_rng(seed).choice(len(sites), n, replace=False))
    return np.ascontiguousarray(sites[pick])


def hard_spheres(n, phi, a=1.0, seed=0, sweeps=0, progress=None):
    """Non-overlapping spheres at volume fraction phi, then `sweeps` MC
    sweeps.  Returns (x, L).  The start is RSA up to phi = RSA_MAX_PHI and a
    randomly vacated FCC lattice above it (the sweeps then melt it: hard
    spheres are fluid below phi ~ 0.49).

    With `progress` (a callable taking a message) the sweeps run in chunks of
    250 (each chunk its own random streams, step carried over) and each chunk
    is reported."""
    L = box_side(n, phi, a)
    x = rsa_positions(n, L, a, seed) if phi <= RSA_MAX_PHI else lattice_positions(n, L, a, seed)
    # relabel particles in spatial (cell) order: the same configuration, but
    # memory-local for the Monte Carlo neighbour checks
    c = np.floor(x / (3.0 * a)).astype(np.int64)
    x = np.ascontiguousarray(x[np.lexsort((c[:, 2], c[:, 1], c[:, 0]))])
    if sweeps and progress is None:
        x, _, _ = mc_relax(x, L, a, sweeps, seed + 7919)
    elif sweeps:
        done, step = 0, 0.1 * a
        while done < sweeps:
            k = min(250, sweeps - done)
            x = np.ascontiguousarray(x, dtype=np.float64)
            st = ctypes.c_double(step)
            acc = _load().mc_relax(len(x), L, a, _dp(x), k, seed + 7919 + 104729 * done, 0.4, ctypes.byref(st),
                                   min(k, 50) if done == 0 else 0)
            step = st.value
            done += k
            progress(f"MC sweeps {done}/{sweeps} (step {step:.3f}a, acceptance {acc:.2f})")
    return x, L


def dlca_gel(n, phi, a=1.0, seed=0, step=0.5, gamma=0.5, stop_frac=0.9, max_moves=None):
    """Colloidal gel by off-lattice diffusion-limited cluster aggregation
    (csrc/hs_gen.c): n spheres placed by RSA at volume fraction phi; clusters
    picked uniformly move by `step` (accepted with probability s^-gamma for
    size s) and stick at first contact, until one cluster holds stop_frac of
    the spheres.  Returns (x, L, cluster label per sphere, stats dict)."""
    L = box_side(n, phi, a)
    x = rsa_positions(n, L, a, seed)
    lab = np.zeros(n, dtype=np.int32)
    st = np.zeros(3)
    if max_moves is None:
        max_moves = 2000 * n
    rc = _load().dlca_gel(n, L, a, seed + 104723, step * a, gamma, stop_frac, max_moves, _dp(x),
                          lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(st))
    if rc != 0:
        raise RuntimeError(f"dlca_gel failed ({rc})")
    return x, L, lab, {"moves": int(st[0]), "clusters": int(st[1]), "largest": int(st[2])}


def mass_radius_slope(x, L, r_lo, r_hi, centers=2000, seed=0):
    """Slope of log N(r) against log r on [r_lo, r_hi], N(r) the mean number
    of spheres within r of a sphere (minimum image): the mass fractal
    dimension of the structure on that range (3 for a uniform suspension)."""
    from scipy.spatial import cKDTree

    x = np.mod(np.asarray(x, dtype=np.float64), L)
    x[x >= L] = 0.0
    t = cKDTree(x, boxsize=L)
    idx = np.random.default_rng(seed).choice(len(x), min(centers, len(x)), replace=False)
    rs = np.geomspace(r_lo, r_hi, 8)
    cnt = [np.mean(t.query_ball_point(x[idx], r, return_length=True)) - 1.0 for r in rs]
    return float(np.polyfit(np.log(rs), np.log(cnt), 1)[0])


def normals(seed, shape):
    """i.i.d. standard normals (numpy PCG64), float64."""
    return np.random.default_rng(seed).standard_normal(shape)
