"""Counter-based random number generators used to build seeded synthetic scans.

Both generators are written from their published definitions:

* SplitMix64 -- G. L. Steele, D. Lea, C. H. Flood, "Fast splittable pseudorandom
  number generators", OOPSLA 2014.  Used for per-scan parameters (positions,
  reflectivities, permittivity, batch shapes).
* Philox4x32-10 -- J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel
  random numbers: as easy as 1, 2, 3", SC 2011.  Used for the additive noise,
  keyed by (seed) and indexed by (antenna, sample pair), so any device that
  implements the same definition draws the same stream.
* Box--Muller (G. E. P. Box, M. E. Muller, 1958) turns two uniforms into two
  standard normal deviates.

Nothing in this module knows about imaging; it only produces numbers.
"""
from __future__ import annotations

import numpy as np

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """Sequential SplitMix64 stream (golden-gamma increment, two xor-shift-multiply mixes)."""

    GAMMA = 0x9E3779B97F4A7C15

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + self.GAMMA) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniforms(self, n: int) -> np.ndarray:
        return np.array([self.uniform() for _ in range(n)], dtype=np.float64)

    def choice(self, options):
        return options[self.next_u64() % len(options)]


# Philox4x32 round constants (Salmon et al. 2011, Table 2 / reference implementation).
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85


def philox4x32_10(ctr: np.ndarray, key: tuple[int, int]) -> np.ndarray:
    """Philox4x32 with 10 rounds, vectorised over rows.

    ctr: uint32 array [..., 4]; key: two 32-bit words.  Returns uint32 [..., 4].
    """
    c = [ctr[..., j].astype(np.uint64) for j in range(4)]
    k0 = np.uint64(key[0] & 0xFFFFFFFF)
    k1 = np.uint64(key[1] & 0xFFFFFFFF)
    m32 = np.uint64(0xFFFFFFFF)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & m32
            k1 = (k1 + np.uint64(PHILOX_W1)) & m32
        p0 = np.uint64(PHILOX_M0) * c[0]
        p1 = np.uint64(PHILOX_M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & m32
        hi1, lo1 = p1 >> np.uint64(32), p1 & m32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


# Domain tag in the third counter word keeps the noise stream apart from any
# other Philox use of the same seed.
NOISE_TAG = 0x4E4F4953  # "NOIS"


def u32_to_open_unit(x: np.ndarray) -> np.ndarray:
    """Map uint32 to the open interval (0, 1): (x + 1/2) / 2^32."""
    return (x.astype(np.float64) + 0.5) * (1.0 / 4294967296.0)


def gaussian_noise(seed: int, n_ant: int, n_samp: int) -> np.ndarray:
    """Standard normal deviates N[i, n], fp64, shape [n_ant, n_samp].

    Sample pair p = n // 2 of antenna i comes from one Philox call with counter
    (p, i, NOISE_TAG, 0) and key (seed low word, seed high word); the first two
    output words feed Box--Muller, giving samples 2p (cosine branch) and 2p+1
    (sine branch).
    """
    n_pair = (n_samp + 1) // 2
    pi, ii = np.meshgrid(np.arange(n_pair, dtype=np.uint64), np.arange(n_ant, dtype=np.uint64))
    ctr = np.zeros((n_ant, n_pair, 4), dtype=np.uint32)
    ctr[..., 0] = pi.astype(np.uint32)
    ctr[..., 1] = ii.astype(np.uint32)
    ctr[..., 2] = NOISE_TAG
    out = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    u1 = u32_to_open_unit(out[..., 0])
    u2 = u32_to_open_unit(out[..., 1])
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty((n_ant, 2 * n_pair), dtype=np.float64)
    z[:, 0::2] = r * np.cos(2.0 * np.pi * u2)
    z[:, 1::2] = r * np.sin(2.0 * np.pi * u2)
    return z[:, :n_samp]
