"""Philox-4x64-10 and the noise built from it (oracle side, numpy).

TEST INFRASTRUCTURE ONLY.

The random numbers the sampler draws are defined by a counter-based generator
so that the CPU oracle and the GPU library can each produce the same noise
from (seed, counter) without sharing code.  Generator: Philox-4x64 with 10
rounds (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11): round multipliers 0xD2E7470EE14C6C93, 0xCA5A826395121157,
Weyl key increments 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B.

Noise layout (both sides implement this independently):
  * uniform from a 64-bit word w: bits = 53 -> ((w >> 11) + 0.5) * 2^-53,
    bits = 24 -> ((w >> 40) + 0.5) * 2^-24 (the single-precision modes);
  * Box-Muller on a word pair (wa, wb): rho = sqrt(-2 ln ua), th = 2 pi ub,
    na = rho cos th, nb = rho sin th;
  * real-space noise z1 (length 3N, element q = 3*i + d in the caller's
    particle order): key (seed, 0), counter (q >> 2, sample, 0, 0); element
    q takes normal number (q & 3) of the block (words 0,1 -> normals 0,1;
    words 2,3 -> normals 2,3);
  * wave-space noise zeta on the stored half spectrum (element
    e = ((c*M + jx)*M + jy)*(M/2) + jz, jz < M/2): key (seed, 1), counter
    (e >> 1, sample, 0, 0); zeta = (n_{2p} + i n_{2p+1})/sqrt 2 with p = e & 1.
    On the plane jz = 0 only the canonical member of each pair (k, -k) draws
    (signed sy > 0, or sy = 0 and sx > 0); its partner is the complex
    conjugate.  k = 0 and any Nyquist index (jx or jy = M/2) are zero.
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a, b):
    """(high, low) 64-bit halves of the 128-bit product a*b, elementwise."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    al, ah = a & _LO32, a >> _S32
    bl, bh = b & _LO32, b >> _S32
    ll = al * bl
    hl = ah * bl
    lh = al * bh
    hh = ah * bh
    cross = (ll >> _S32) + (hl & _LO32) + lh
    hi = hh + (hl >> _S32) + (cross >> _S32)
    lo = (cross << _S32) | (ll & _LO32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Philox-4x64-10 block function.  ctr: 4 uint64 arrays, key: 2 uint64
    arrays (broadcastable).  Returns the 4 output words."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) for k in key)
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = mulhilo64(M0, c0)
            hi1, lo1 = mulhilo64(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform(w, bits):
    w = np.asarray(w, dtype=np.uint64)
    if bits == 53:
        return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0**-53
    if bits == 24:
        return ((w >> np.uint64(40)).astype(np.float64) + 0.5) * 2.0**-24
    raise ValueError("bits must be 53 or 24")


def box_muller(wa, wb, bits):
    ua, ub = uniform(wa, bits), uniform(wb, bits)
    rho = np.sqrt(-2.0 * np.log(ua))
    th = 2.0 * np.pi * ub
    return rho * np.cos(th), rho * np.sin(th)


def block_normals(blocks, sample, seed, stream, bits):
    """Four normals per counter block: array (len(blocks), 4)."""
    blocks = np.asarray(blocks, dtype=np.uint64)
    z = np.zeros_like(blocks)
    w = philox4x64_10((blocks, np.full_like(blocks, np.uint64(sample)), z, z),
                      (np.uint64(seed), np.uint64(stream)))
    n0, n1 = box_muller(w[0], w[1], bits)
    n2, n3 = box_muller(w[2], w[3], bits)
    return np.stack([n0, n1, n2, n3], axis=1)


def real_noise(n, seed, sample, bits=53):
    """z1 (length 3n, caller order) as specified in the module docstring."""
    q = np.arange(3 * n, dtype=np.uint64)
    nb = block_normals(q >> np.uint64(2), sample, seed, 0, bits)
    return nb[np.arange(3 * n), (q & np.uint64(3)).astype(np.int64)]


def wave_noise_full(M, seed, sample, bits=53):
    """zeta on the full M^3 grid (DFT order, shape [3, M, M, M]) following the
    half-spectrum layout and canonical-pair rule of the module docstring.
    Entries at jz = M/2 (Nyquist) are zero; entries at jz > M/2 are the
    conjugates of their mirror images (-k)."""
    H = M // 2
    e = np.arange(3 * M * M * H, dtype=np.uint64)
    nb = block_normals(e >> np.uint64(1), sample, seed, 1, bits)
    p = (e & np.uint64(1)).astype(np.int64)
    idx = np.arange(len(e))
    zh = (nb[idx, 2 * p] + 1j * nb[idx, 2 * p + 1]) / np.sqrt(2.0)
    return half_spectrum_to_full(zh.reshape(3, M, M, H))


def half_spectrum_to_full(zh):
    """The full conjugate-symmetric field [3, M, M, M] (DFT order) from values
    on the stored half spectrum zh[3, M, M, M/2] (jz < M/2): on the plane
    jz = 0 the canonical member of each (k, -k) pair (signed jy > 0, or
    jy = 0 and jx > 0) keeps its value and its partner takes the conjugate;
    k = 0 and the Nyquist entries are zero; entries at jz > M/2 are the
    conjugates of their mirror images (-k)."""
    zh = np.array(zh, dtype=np.complex128)
    M = zh.shape[1]
    H = M // 2
    s = np.fft.fftfreq(M, 1.0 / M).astype(np.int64)  # signed index per position
    nyq = np.abs(s) == H
    # plane jz = 0: keep canonical draws, partners get conjugates
    SX, SY = np.meshgrid(s, s, indexing="ij")
    canon = (SY > 0) | ((SY == 0) & (SX > 0))
    plane = zh[:, :, :, 0].copy()
    mirror = plane[:, (-SX) % M, (-SY) % M]
    plane = np.where(canon[None], plane, np.conj(mirror))
    zh[:, :, :, 0] = plane
    zh[:, nyq, :, :] = 0.0
    zh[:, :, nyq, :] = 0.0
    zh[:, 0, 0, 0] = 0.0

    Z = np.zeros((3, M, M, M), dtype=np.complex128)
    Z[:, :, :, :H] = zh
    # jz in (H, M): zeta(k) = conj zeta(-k); -k has index ((-jx)%M, (-jy)%M, M-jz)
    jz = np.arange(H + 1, M)
    ix = (-np.arange(M)) % M
    Z[:, :, :, H + 1:] = np.conj(zh[:, ix][:, :, ix][:, :, :, M - jz])
    return Z
