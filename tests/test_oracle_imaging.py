"""Pins of the FP64 oracle's imaging (Eq. (1) delay, Eq. (3) DAS, pairwise DMAS of Section II).

Each check ties the oracle to something other than itself: a closed form, a
library routine (numpy's linear interpolation), an algebraic identity or an
invariance of the mathematics, or the physics of a single point scatterer.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from synth import Grid, Scan

# ----------------------------------------------------------------------------------
# closed form at the centre of a ring of equidistant antennas
# ----------------------------------------------------------------------------------

# 12 antennas at exactly 5/128 m from the origin (Pythagorean 3-4-5 points), exact in fp32.
_U = 1.0 / 128.0
_RING12 = np.array([(3, 4), (4, 3), (5, 0), (4, -3), (3, -4), (0, -5), (-3, -4), (-4, -3), (-5, 0),
                    (-4, 3), (-3, 4), (0, 5)], dtype=np.float64) * _U
DT = 2e-11
V = 0.078125 / (40 * DT)      # round trip 2 * 5/128 m takes exactly 40 samples


def _centre_scan(m, amps, t0_samples=0, n_samp=128, kind="sin_gauss"):
    ant = np.zeros((m, 3), dtype=np.float32)
    ant[:, :2] = _RING12[:m]
    t0 = t0_samples * DT
    n = np.arange(n_samp)
    # echo of a scatterer at the origin: arrives 40 samples after the excitation
    y = np.stack([a * synth.pulse(t0 + n * DT - 40 * DT, kind) for a in amps]).astype(np.float32)
    grid = Grid((-1e-3, -1e-3, 0.0), (1e-3, 1e-3, 1e-3), (3, 3, 1))   # voxel (1,1) is the origin
    return Scan(ant, y, DT, t0, V, grid)


def _pulse_samples(window, kind="sin_gauss"):
    h = (window - 1) // 2
    # the traces hold float32 values; evaluate the closed form on the same values
    return np.array([np.float32(synth.pulse(np.array(k * DT), kind)) for k in range(-h, h + 1)],
                    dtype=np.float64)


@pytest.mark.parametrize("m", [1, 2, 3, 7, 12])
@pytest.mark.parametrize("window", [1, 5, 11])
@pytest.mark.parametrize("t0_samples", [0, 5])
def test_centre_closed_form(m, window, t0_samples):
    rng = np.random.default_rng(m * 100 + window)
    amps = 2.0 ** rng.integers(-3, 4, m).astype(np.float64)     # powers of two: A_i p exact in fp32
    scan = _centre_scan(m, amps, t0_samples)
    p = _pulse_samples(window)
    das = oracle.image_indices(scan, oracle.DAS, [[1, 1, 0]], window)[0]
    dmas = oracle.image_indices(scan, oracle.DMAS, [[1, 1, 0]], window)[0]
    # every aligned sample is A_i p_k, so S_k = (sum A) p_k and P_k = (sum_{i<j} A_i A_j) p_k^2
    pair = (amps.sum() ** 2 - (amps ** 2).sum()) / 2.0
    want_das = amps.sum() ** 2 * np.sum(p ** 2)
    want_dmas = pair ** 2 * np.sum(p ** 4)
    assert das == pytest.approx(want_das, rel=1e-10, abs=1e-300)
    if m == 1:
        assert dmas == 0.0
    else:
        assert dmas == pytest.approx(want_dmas, rel=1e-10)


# ----------------------------------------------------------------------------------
# brute force on tiny inputs with an independent formulation (np.interp)
# ----------------------------------------------------------------------------------

def _brute(scan, bf, window):
    """Independent re-statement: numpy interpolation of zero-padded traces, DMAS via ((sum s)^2 - sum s^2)/2."""
    nx, ny, nz = scan.grid.dims
    h = (window - 1) // 2
    t = scan.traces.astype(np.float64)
    T = t.shape[1]
    xp = np.arange(-1, T + 1, dtype=np.float64)
    out = np.zeros((nz, ny, nx))
    for iz, iy, ix in itertools.product(range(nz), range(ny), range(nx)):
        r = np.asarray(scan.grid.origin) + np.array([ix, iy, iz]) * np.asarray(scan.grid.pitch)
        d = np.linalg.norm(r[None, :] - scan.ant_pos.astype(np.float64), axis=1)
        tau = (2 * d / scan.v - scan.t0) / scan.dt
        k = np.arange(-h, h + 1)
        s = np.stack([np.interp(tau[i] + k, xp, np.concatenate([[0.0], t[i], [0.0]]), left=0.0, right=0.0)
                      for i in range(t.shape[0])])                 # [M, W]
        if bf == 0:
            out[iz, iy, ix] = np.sum(s.sum(axis=0) ** 2)
        else:
            out[iz, iy, ix] = np.sum(((s.sum(axis=0) ** 2 - (s ** 2).sum(axis=0)) / 2) ** 2)
    return out


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("bf", [0, 1])
def test_brute_force_tiny(seed, bf):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 4))
    T = int(rng.integers(8, 33))
    window = int(rng.choice([1, 3, 5, 7]))
    ant = rng.uniform(-0.02, 0.02, (m, 3)).astype(np.float32)
    y = rng.standard_normal((m, T)).astype(np.float32)
    # v, dt chosen so the delays over the grid sweep past both ends of the trace
    grid = Grid((-0.01, -0.012, 0.003), (0.007, 0.006, 0.004), (4, 4, 2))
    scan = Scan(ant, y, 1e-11, float(rng.uniform(-5e-11, 5e-11)), 2 * 0.04 / (T * 1e-11), grid)
    got = oracle.image_grid(scan, bf, window)
    want = _brute(scan, bf, window)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-13 * max(1.0, np.abs(want).max()))


def test_brute_force_covers_trace_edges():
    """The tiny cases above really do reach negative and beyond-T sample positions."""
    rng = np.random.default_rng(0)
    T = 16
    ant = np.array([[0.0, 0.0, 0.0]], dtype=np.float32)
    y = rng.standard_normal((1, T)).astype(np.float32)
    grid = Grid((0.0, 0.0, 0.0), (1e-3, 1e-3, 1e-3), (16, 1, 1))
    scan = Scan(ant, y, 1e-11, 3e-11, 2e-3 / 1e-11 / 1.5, grid)   # tau = 1.5 ix - 3
    got = oracle.image_grid(scan, 0, 3)[0, 0]
    np.testing.assert_allclose(got, _brute(scan, 0, 3)[0, 0], rtol=1e-12)
    assert got[0] == 0.0 and got[1] > 0.0       # window entirely before sample 0, then straddling it
    assert got[12] > 0.0 and got[15] == 0.0     # straddling the last sample, then entirely beyond T


# ----------------------------------------------------------------------------------
# invariances
# ----------------------------------------------------------------------------------

def _small_random_scan(seed, m=8, n=12, T=256):
    g = Grid((-0.02, -0.02, 0.0), (0.04 / (n - 1), 0.04 / (n - 1), 1e-3), (n, n, 1))
    return synth.random_scan(seed, m, T, g, radius=0.07)


def test_das_parallelogram_law():
    """S is linear in the traces, so I(Y1+Y2) + I(Y1-Y2) = 2 I(Y1) + 2 I(Y2)."""
    a = _small_random_scan(1)
    b = _small_random_scan(2)
    y1 = a.traces.astype(np.float64)
    y2 = b.traces.astype(np.float64)
    # keep all four trace sets exact in fp32 (small integers)
    y1 = np.round(y1 * 8)
    y2 = np.round(y2 * 8)

    def img(y):
        s = Scan(a.ant_pos, y.astype(np.float32), a.dt, a.t0, a.v, a.grid)
        return oracle.image_grid(s, 0)

    lhs = img(y1 + y2) + img(y1 - y2)
    rhs = 2 * img(y1) + 2 * img(y2)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-11, atol=1e-9 * rhs.max())


@pytest.mark.parametrize("bf,power", [(0, 2), (1, 4)])
def test_amplitude_scaling(bf, power):
    s = _small_random_scan(3)
    c = 2.0 ** 3          # exact in fp32
    s2 = Scan(s.ant_pos, (s.traces * c).astype(np.float32), s.dt, s.t0, s.v, s.grid)
    np.testing.assert_allclose(oracle.image_grid(s2, bf), c ** power * oracle.image_grid(s, bf), rtol=1e-12)


@pytest.mark.parametrize("bf", [0, 1])
def test_antenna_permutation(bf):
    s = _small_random_scan(4)
    p = np.random.default_rng(0).permutation(s.n_ant)
    s2 = Scan(s.ant_pos[p].copy(), s.traces[p].copy(), s.dt, s.t0, s.v, s.grid)
    np.testing.assert_allclose(oracle.image_grid(s2, bf), oracle.image_grid(s, bf), rtol=1e-11)


@pytest.mark.parametrize("bf", [0, 1])
def test_rot90_equivariance(bf):
    """Rotating antennas by +90 degrees about z (traces follow their antenna) rotates the image."""
    m, n = 8, 10
    th = 2 * np.pi * np.arange(m) / m
    ant = np.stack([0.07 * np.cos(th), 0.07 * np.sin(th), np.zeros(m)], 1).astype(np.float32)
    rot = np.stack([-ant[:, 1], ant[:, 0], ant[:, 2]], 1)          # exact in fp32
    y = np.random.default_rng(5).standard_normal((m, 300)).astype(np.float32)
    p = 0.04 / n
    g = Grid((-(n - 1) * p / 2, -(n - 1) * p / 2, 0.0), (p, p, p), (n, n, 1))
    a = oracle.image_grid(Scan(ant, y, 2e-11, 0.0, 1e8, g), bf)[0]
    b = oracle.image_grid(Scan(rot, y, 2e-11, 0.0, 1e8, g), bf)[0]
    # voxel (ix, iy) of the rotated scene sees what voxel (iy, n-1-ix) saw before,
    # i.e. b[iy][ix] = a[n-1-ix][iy], which is numpy's clockwise rot90 of the [y][x] array
    np.testing.assert_allclose(b, np.rot90(a, k=-1), rtol=1e-9, atol=1e-12 * a.max())
    assert not np.allclose(a, b, rtol=1e-3)


def test_dmas_m2_is_product():
    """With two antennas the pairwise sum is s1 s2, so DMAS = sum_k (s1 s2)^2 <= (DAS-derived bound)."""
    s = _small_random_scan(6, m=2)
    one = [Scan(s.ant_pos[i:i + 1].copy(), s.traces[i:i + 1].copy(), s.dt, s.t0, s.v, s.grid) for i in range(2)]
    # window 1: I_DAS(single antenna) = s_i^2, so DMAS = s1^2 s2^2 = I1 * I2
    d = oracle.image_grid(s, 1, 1)
    np.testing.assert_allclose(d, oracle.image_grid(one[0], 0, 1) * oracle.image_grid(one[1], 0, 1), rtol=1e-11)


def test_dmas_identity_window1():
    """Window 1: DAS = (sum s)^2, per-antenna DAS = s_i^2 (sign lost), DMAS = ((sum s)^2 - sum s^2)^2 / 4."""
    s = _small_random_scan(7, m=5)
    das = oracle.image_grid(s, 0, 1)
    sq = sum(oracle.image_grid(Scan(s.ant_pos[i:i + 1].copy(), s.traces[i:i + 1].copy(), s.dt, s.t0, s.v,
                                    s.grid), 0, 1) for i in range(5))
    np.testing.assert_allclose(oracle.image_grid(s, 1, 1), ((das - sq) / 2) ** 2, rtol=1e-9,
                               atol=1e-12 * das.max() ** 2)


# ----------------------------------------------------------------------------------
# physics: a single noiseless point scatterer is found within one voxel
# ----------------------------------------------------------------------------------

def _nearest_voxel(grid, x):
    return np.round((np.asarray(x) - np.asarray(grid.origin)) / np.asarray(grid.pitch)).astype(int)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("bf", [0, 1])
def test_single_scatterer_2d(seed, bf):
    s = synth.c1_scan(seed, noiseless=True)
    arg, _ = oracle.argmax_grid(oracle.image_grid(s, bf))
    nx = s.grid.dims[0]
    got = np.array([arg % nx, arg // nx, 0])
    want = _nearest_voxel(s.grid, s.tumour)
    assert np.max(np.abs(got - want)) <= 1, (got, want)


@pytest.mark.parametrize("bf", [0, 1])
def test_single_scatterer_c2_geometry(bf):
    s = synth.c2_scan(0, noiseless=True, n_grid=128)
    arg, _ = oracle.argmax_grid(oracle.image_grid(s, bf))
    nx = s.grid.dims[0]
    assert np.max(np.abs(np.array([arg % nx, arg // nx, 0]) - _nearest_voxel(s.grid, s.tumour))) <= 1


@pytest.mark.parametrize("bf,n", [(0, 48), (1, 24)])
def test_single_scatterer_3d(bf, n):
    s = synth.c3_scan(1, noiseless=True, n_grid=n, n_ant=64 if bf == 0 else 24)
    img = oracle.image_grid(s, bf)
    arg, _ = oracle.argmax_grid(img)
    got = np.array([arg % n, (arg // n) % n, arg // (n * n)])
    assert np.max(np.abs(got - _nearest_voxel(s.grid, s.tumour))) <= 1


def test_c2_noisy_detection():
    """Clutter at <= 0.1 reflectivity and 20 dB noise do not move the DMAS peak off the tumour."""
    s = synth.c2_scan(3, n_grid=128)
    arg, _ = oracle.argmax_grid(oracle.image_grid(s, 1))
    nx = s.grid.dims[0]
    assert np.max(np.abs(np.array([arg % nx, arg // nx, 0]) - _nearest_voxel(s.grid, s.tumour))) <= 1


def test_argmax_rule():
    v = np.array([1.0, 3.0, 3.0 * (1 - 1e-13), 2.0, 3.0])
    assert oracle.select_max(v, np.arange(5)) == (1, 3.0)
    v = np.array([1.0, 3.0 * (1 - 1e-10), 3.0])
    assert oracle.select_max(v, np.arange(3))[0] == 2
    v = np.array([-2.0, -1.0 * (1 + 1e-13), -1.0])          # negative maxima use |max|
    assert oracle.select_max(v, np.arange(3))[0] == 1
    assert oracle.select_max(np.zeros(4), np.arange(4))[0] == 0
    assert math.isfinite(oracle.select_max(np.array([0.5]), np.array([7]))[1])
