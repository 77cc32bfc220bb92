"""Seeded synthetic monostatic scans that stand in for the paper's missing phantom data.

The paper's two phantom datasets (Section IV) are not available, so every input is
simulated: point scatterers in a homogeneous medium, each antenna records the
round-trip echo of a short pulse, scaled by a 1/r^2 spreading factor and summed
with white Gaussian noise.  The recipes C1..C5 follow the workload descriptions
used for this library (2D ring, 2D ring with clutter, 3D hemisphere, uneven batch,
learned-proposal training set).

This module is the *only* code shared by the oracle and the GPU path.  It holds
the forward physics of the test scene and nothing of the imaging method.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .rng import SplitMix64, gaussian_noise

C0 = 299_792_458.0           # speed of light in vacuum, m/s
DT = 20e-12                  # 50 GS/s sampling
RING_R = 0.07                # antenna radius, m
REGION = 0.05                # imaged half-width, m ([-5, 5] cm)
PULSE_F0 = 6e9               # pulse centre frequency, Hz
PULSE_SIGMA = 60e-12         # pulse Gaussian width, s
PULSE_SUPPORT = 6.0          # pulse truncated at |t| <= 6 sigma
REF_DIST = 0.01              # 1/r^2 amplitude normalised at 1 cm


@dataclasses.dataclass
class Grid:
    origin: tuple            # centre of voxel (0,0,0), metres
    pitch: tuple             # voxel pitch per axis, metres
    dims: tuple              # (nx, ny, nz); nz == 1 means a 2D image

    @property
    def n_voxels(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])

    def positions(self, idx: np.ndarray) -> np.ndarray:
        """Voxel centres (fp64) for integer indices idx [..., 3] = (ix, iy, iz)."""
        o = np.asarray(self.origin, dtype=np.float64)
        p = np.asarray(self.pitch, dtype=np.float64)
        return o + np.asarray(idx, dtype=np.float64) * p


@dataclasses.dataclass
class Scan:
    ant_pos: np.ndarray      # [M, 3] float32, metres
    traces: np.ndarray       # [M, T] float32
    dt: float                # sampling period, s
    t0: float                # time of sample 0 relative to the excitation peak, s
    v: float                 # propagation speed, m/s
    grid: Grid
    seed: int = 0
    tumour: np.ndarray | None = None      # [3] metres
    eps_r: float = 9.0
    sigma_n: float = 0.0
    multistatic: bool = False             # traces [M*M, T]: channel i*M + j = transmitter i, receiver j

    @property
    def n_ant(self) -> int:
        return int(self.ant_pos.shape[0])

    @property
    def n_samp(self) -> int:
        return int(self.traces.shape[1])


# ----------------------------------------------------------------------------------
# pulse
# ----------------------------------------------------------------------------------

def _sin_gauss_raw(t):
    return np.sin(2.0 * np.pi * PULSE_F0 * t) * np.exp(-(t * t) / (2.0 * PULSE_SIGMA ** 2))


def _sin_gauss_peak() -> float:
    t = np.linspace(0.0, 3.0 * PULSE_SIGMA, 2_000_001)
    return float(np.max(_sin_gauss_raw(t)))


_PEAK = {"sin_gauss": _sin_gauss_peak(), "dgauss": math.exp(-0.5)}


def pulse(t: np.ndarray, kind: str = "sin_gauss") -> np.ndarray:
    """Excitation pulse, peak-normalised to 1, truncated to |t| <= 6 sigma.

    sin_gauss: sin(2 pi f0 t) exp(-t^2 / 2 sigma^2), centre 6 GHz, sigma 60 ps.
    dgauss:    -(t / sigma) exp(-t^2 / 2 sigma^2) (first-derivative Gaussian).
    """
    t = np.asarray(t, dtype=np.float64)
    if kind == "sin_gauss":
        y = _sin_gauss_raw(t)
    elif kind == "dgauss":
        y = -(t / PULSE_SIGMA) * np.exp(-(t * t) / (2.0 * PULSE_SIGMA ** 2))
    else:
        raise ValueError(kind)
    y = y / _PEAK[kind]
    return np.where(np.abs(t) <= PULSE_SUPPORT * PULSE_SIGMA, y, 0.0)


# ----------------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------------

def ring_antennas(m: int, radius: float = RING_R) -> np.ndarray:
    th = 2.0 * np.pi * np.arange(m) / m
    a = np.stack([radius * np.cos(th), radius * np.sin(th), np.zeros(m)], axis=1)
    return a.astype(np.float32)


def hemisphere_antennas(m: int, radius: float = RING_R) -> np.ndarray:
    """Fibonacci placement on the z >= 0 hemisphere: z_i = R (i+1/2)/m, phi_i = i pi (3 - sqrt 5)."""
    i = np.arange(m, dtype=np.float64)
    z = radius * (i + 0.5) / m
    phi = i * np.pi * (3.0 - math.sqrt(5.0))
    rho = np.sqrt(radius * radius - z * z)
    a = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)
    return a.astype(np.float32)


def square_grid(n: int, half: float = REGION) -> Grid:
    p = 2.0 * half / n
    o = -half + 0.5 * p
    return Grid((o, o, 0.0), (p, p, p), (n, n, 1))


def cube_grid(n: int, half: float = REGION) -> Grid:
    p = 2.0 * half / n
    o = -half + 0.5 * p
    return Grid((o, o, o), (p, p, p), (n, n, n))


def _disc_point(rng: SplitMix64, radius: float = REGION) -> np.ndarray:
    r = radius * math.sqrt(rng.uniform())
    th = 2.0 * math.pi * rng.uniform()
    return np.array([r * math.cos(th), r * math.sin(th), 0.0])


def _half_ball_point(rng: SplitMix64, radius: float = REGION) -> np.ndarray:
    r = radius * rng.uniform() ** (1.0 / 3.0)
    ct = rng.uniform()                       # cos(polar) uniform on [0,1): z >= 0
    st = math.sqrt(max(0.0, 1.0 - ct * ct))
    ph = 2.0 * math.pi * rng.uniform()
    return np.array([r * st * math.cos(ph), r * st * math.sin(ph), r * ct])


# ----------------------------------------------------------------------------------
# forward model
# ----------------------------------------------------------------------------------

def synthesize(ant_pos, points, refl, n_samp, v, dt=DT, t0=0.0, kind="sin_gauss"):
    """Clean traces Y[i, n] = sum_s A_is p(t0 + n dt - 2|x_s - a_i| / v),  A_is = rho_s (1 cm / |x_s - a_i|)^2."""
    a = np.asarray(ant_pos, dtype=np.float64)
    x = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    rho = np.asarray(refl, dtype=np.float64).reshape(-1)
    m = a.shape[0]
    dist = np.linalg.norm(x[None, :, :] - a[:, None, :], axis=2)          # [M, S]
    tau = 2.0 * dist / v                                                   # [M, S] seconds
    amp = rho[None, :] * (REF_DIST / dist) ** 2
    half = PULSE_SUPPORT * PULSE_SIGMA
    n0 = np.floor((tau - half - t0) / dt).astype(np.int64)
    span = int(math.ceil(2.0 * half / dt)) + 3
    out = np.zeros((m, n_samp), dtype=np.float64)
    for j in range(span):
        n = n0 + j
        t = t0 + n * dt - tau
        val = amp * pulse(t, kind)
        ok = (n >= 0) & (n < n_samp)
        rows = np.broadcast_to(np.arange(m)[:, None], n.shape)
        np.add.at(out, (rows[ok], n[ok]), val[ok])
    return out


def tumour_power(ant_pos, tumour, n_samp, v, dt=DT, t0=0.0, kind="sin_gauss"):
    """Mean over antennas of the tumour echo's mean square over samples within 3 sigma of its arrival."""
    clean = synthesize(ant_pos, tumour[None, :], [1.0], n_samp, v, dt, t0, kind)
    a = np.asarray(ant_pos, dtype=np.float64)
    tau = 2.0 * np.linalg.norm(a - tumour[None, :], axis=1) / v
    n = np.arange(n_samp)
    p = []
    for i in range(a.shape[0]):
        sel = np.abs(t0 + n * dt - tau[i]) <= 3.0 * PULSE_SIGMA
        p.append(np.mean(clean[i, sel] ** 2) if np.any(sel) else 0.0)
    return float(np.mean(p))


def make_scan(ant_pos, grid, tumour, n_samp, eps_r, snr_db, seed, clutter=None,
              clutter_refl=None, noiseless=False, kind="sin_gauss", t0=0.0) -> Scan:
    v = C0 / math.sqrt(eps_r)
    pts = [tumour[None, :]]
    refl = [np.array([1.0])]
    if clutter is not None and not noiseless:
        pts.append(clutter)
        refl.append(clutter_refl)
    pts = np.concatenate(pts, axis=0)
    refl = np.concatenate(refl)
    y = synthesize(ant_pos, pts, refl, n_samp, v, DT, t0, kind)
    sigma_n = 0.0
    if not noiseless and snr_db is not None:
        ps = tumour_power(ant_pos, tumour, n_samp, v, DT, t0, kind)
        sigma_n = math.sqrt(ps / 10.0 ** (snr_db / 10.0))
        y = y + sigma_n * gaussian_noise(seed, ant_pos.shape[0], n_samp)
    return Scan(np.ascontiguousarray(ant_pos, dtype=np.float32), np.ascontiguousarray(y, dtype=np.float32),
                DT, t0, v, grid, seed, tumour, eps_r, sigma_n)


# ----------------------------------------------------------------------------------
# the workload recipes
# ----------------------------------------------------------------------------------

_SALT = {"c1": 0x01, "c2": 0x02, "c3": 0x03, "c4": 0x04, "c5": 0x05}


def _rng(cfg: str, seed: int) -> SplitMix64:
    return SplitMix64(seed ^ (_SALT[cfg] << 56))


def c1_scan(seed: int, noiseless: bool = False, n_grid: int = 128, n_ant: int = 16,
            n_samp: int = 1024, kind: str = "sin_gauss") -> Scan:
    """2D ring, 16 antennas, T=1024, eps_r=9, one tumour in the 5 cm disc, SNR 30 dB, 128x128 grid."""
    rng = _rng("c1", seed)
    tumour = _disc_point(rng)
    return make_scan(ring_antennas(n_ant), square_grid(n_grid), tumour, n_samp, 9.0,
                     30.0, seed, noiseless=noiseless, kind=kind)


def c2_scan(seed: int, noiseless: bool = False, n_grid: int = 512, n_ant: int = 32,
            n_samp: int = 2048, n_clutter: int = 200, kind: str = "sin_gauss") -> Scan:
    """2D ring, 32 antennas, T=2048, tumour + 200 clutter (rho ~ U(0, 0.1)), SNR 20 dB, 512x512 grid."""
    rng = _rng("c2", seed)
    tumour = _disc_point(rng)
    cl = np.array([_disc_point(rng) for _ in range(n_clutter)]).reshape(-1, 3)
    rho = 0.1 * rng.uniforms(n_clutter)
    return make_scan(ring_antennas(n_ant), square_grid(n_grid), tumour, n_samp, 9.0, 20.0,
                     seed, clutter=cl, clutter_refl=rho, noiseless=noiseless, kind=kind)


def c3_scan(seed: int, noiseless: bool = False, n_grid: int = 256, n_ant: int = 64,
            n_samp: int = 4096, n_clutter: int = 1000, kind: str = "sin_gauss") -> Scan:
    """3D hemisphere (Fibonacci), 64 antennas, T=4096, eps_r ~ U(8,10), tumour + 1000 clutter, SNR 20 dB, 256^3 grid."""
    rng = _rng("c3", seed)
    eps_r = 8.0 + 2.0 * rng.uniform()
    tumour = _half_ball_point(rng)
    cl = np.array([_half_ball_point(rng) for _ in range(n_clutter)]).reshape(-1, 3)
    rho = 0.1 * rng.uniforms(n_clutter)
    return make_scan(hemisphere_antennas(n_ant), cube_grid(n_grid), tumour, n_samp, eps_r, 20.0,
                     seed, clutter=cl, clutter_refl=rho, noiseless=noiseless, kind=kind)


C4_ANTS = (16, 32, 48, 64)
C4_SAMPS = (1024, 2048, 4096)
C4_SIDES = (64, 128, 256, 512)


def c4_shape(seed: int):
    rng = _rng("c4", seed)
    return rng.choice(C4_ANTS), rng.choice(C4_SAMPS), rng.choice(C4_SIDES), rng


def c4_scan(seed: int, noiseless: bool = False, kind: str = "sin_gauss") -> Scan:
    """One scan of the uneven batch: M, T, side drawn per seed, otherwise generated as in C1."""
    m, t, side, rng = c4_shape(seed)
    tumour = _disc_point(rng)
    return make_scan(ring_antennas(m), square_grid(side), tumour, t, 9.0, 30.0, seed,
                     noiseless=noiseless, kind=kind)


def point_scan(ant_pos, grid, points, refl, n_samp, v, dt=DT, t0=0.0, kind="sin_gauss") -> Scan:
    """Noiseless scan of arbitrary point scatterers (used by unit checks)."""
    y = synthesize(ant_pos, points, refl, n_samp, v, dt, t0, kind)
    return Scan(np.ascontiguousarray(ant_pos, dtype=np.float32), np.ascontiguousarray(y, dtype=np.float32),
                dt, t0, v, grid, 0, np.asarray(points, dtype=np.float64).reshape(-1, 3)[0])


def random_scan(seed: int, n_ant: int, n_samp: int, grid: Grid, v: float = C0 / 3.0,
                dt: float = DT, t0: float = 0.0, radius: float = RING_R) -> Scan:
    """Antennas on a ring with white-noise traces: unstructured data for parity and invariant checks."""
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((n_ant, n_samp))
    return Scan(ring_antennas(n_ant, radius), np.ascontiguousarray(y, dtype=np.float32), dt, t0, v, grid, seed)


# ----------------------------------------------------------------------------------
# multistatic scans (every antenna transmits, every antenna receives)
# ----------------------------------------------------------------------------------

def synthesize_ms(ant_pos, points, refl, n_samp, v, dt=DT, t0=0.0, kind="sin_gauss"):
    """Clean multistatic traces Y[i*M + j, n] = sum_s A_ijs p(t0 + n dt - (|x_s - a_i| + |x_s - a_j|) / v),
    A_ijs = rho_s (1 cm / |x_s - a_i|) (1 cm / |x_s - a_j|) (the monostatic 1/r^2 law split over both legs)."""
    a = np.asarray(ant_pos, dtype=np.float64)
    x = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    rho = np.asarray(refl, dtype=np.float64).reshape(-1)
    m = a.shape[0]
    dist = np.linalg.norm(x[None, :, :] - a[:, None, :], axis=2)          # [M, S]
    n = np.arange(n_samp)
    out = np.zeros((m * m, n_samp), dtype=np.float64)
    for i in range(m):
        for j in range(m):
            for s in range(x.shape[0]):
                tau = (dist[i, s] + dist[j, s]) / v
                amp = rho[s] * (REF_DIST / dist[i, s]) * (REF_DIST / dist[j, s])
                out[i * m + j] += amp * pulse(t0 + n * dt - tau, kind)
    return out


def ms_scan(seed: int, dataset: int = 1, noiseless: bool = False, n_ant: int = 12, n_samp: int = 1024,
            kind: str = "sin_gauss") -> Scan:
    """Multistatic ring of 12 antennas standing in for the two datasets of Section IV: a point tumour at
    (-2, -3, 0) cm inside a 10 cm phantom (ring radius 12 cm, 20 x 20 cm grid at 1 mm), or at (2, 0, 1) cm inside
    a 5 cm phantom (ring radius 7 cm, 10 x 10 cm slice through z = 1 cm at 1 mm); eps_r = 9, SNR 30 dB."""
    if dataset == 1:
        ant, tumour = ring_antennas(n_ant, 0.12), np.array([-0.02, -0.03, 0.0])
        grid = Grid((-0.1 + 0.0005, -0.1 + 0.0005, 0.0), (0.001, 0.001, 0.001), (200, 200, 1))
    else:
        ant, tumour = ring_antennas(n_ant, RING_R), np.array([0.02, 0.0, 0.01])
        grid = Grid((-0.05 + 0.0005, -0.05 + 0.0005, 0.01), (0.001, 0.001, 0.001), (100, 100, 1))
    v = C0 / 3.0
    y = synthesize_ms(ant, tumour[None, :], [1.0], n_samp, v, DT, 0.0, kind)
    sigma_n = 0.0
    if not noiseless:
        a = np.asarray(ant, dtype=np.float64)
        d = np.linalg.norm(a - tumour[None, :], axis=1)
        n = np.arange(n_samp)
        p = []
        for i in range(n_ant):
            for j in range(n_ant):
                sel = np.abs(n * DT - (d[i] + d[j]) / v) <= 3.0 * PULSE_SIGMA
                p.append(np.mean(y[i * n_ant + j, sel] ** 2) if np.any(sel) else 0.0)
        sigma_n = math.sqrt(float(np.mean(p)) / 10.0 ** (30.0 / 10.0))
        y = y + sigma_n * gaussian_noise(seed, n_ant * n_ant, n_samp)
    return Scan(np.ascontiguousarray(ant, dtype=np.float32), np.ascontiguousarray(y, dtype=np.float32), DT, 0.0, v,
                grid, seed, tumour, 9.0, sigma_n, multistatic=True)


def random_scan_ms(seed: int, n_ant: int, n_samp: int, grid: Grid, v: float = C0 / 3.0, dt: float = DT,
                   t0: float = 0.0, radius: float = RING_R) -> Scan:
    """Multistatic ring with white-noise traces [M*M, T]."""
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((n_ant * n_ant, n_samp))
    return Scan(ring_antennas(n_ant, radius), np.ascontiguousarray(y, dtype=np.float32), dt, t0, v, grid, seed,
                multistatic=True)
