"""Pins of the multistatic oracle (Eq. (2) delay, Eq. (4) DAS, pairwise DMAS over the M^2 channels).

As for the monostatic oracle, each check ties it to something other than itself: a closed form at the centre of
a ring, brute force with numpy's interpolation, the reduction to the monostatic image when only the diagonal
channels carry signal, reciprocity and antenna relabelling, and the physics of a point scatterer.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from synth import Grid, Scan

_U = 1.0 / 128.0
_RING12 = np.array([(3, 4), (4, 3), (5, 0), (4, -3), (3, -4), (0, -5), (-3, -4), (-4, -3), (-5, 0),
                    (-4, 3), (-3, 4), (0, 5)], dtype=np.float64) * _U
DT = 2e-11
V = 0.078125 / (40 * DT)      # transmitter -> centre -> receiver (2 x 5/128 m) takes exactly 40 samples


def _ms(ant, traces, grid, dt=DT, t0=0.0, v=V):
    return Scan(np.asarray(ant, np.float32), np.asarray(traces, np.float32), dt, t0, v, grid, multistatic=True)


@pytest.mark.parametrize("m", [1, 2, 3, 5])
@pytest.mark.parametrize("window", [1, 5, 11])
def test_centre_closed_form(m, window):
    """At the ring's centre every channel's path is 2 x 5/128 m: with Y_c = A_c p(t - 40 dt) the aligned samples are
    A_c p_k, so S_k = (sum A) p_k and P_k = (sum_{c<c'} A_c A_c') p_k^2."""
    rng = np.random.default_rng(m * 10 + window)
    ant = np.zeros((m, 3))
    ant[:, :2] = _RING12[:m]
    amps = 2.0 ** rng.integers(-3, 4, m * m).astype(np.float64)
    n = np.arange(128)
    y = np.stack([a * synth.pulse(n * DT - 40 * DT) for a in amps])
    grid = Grid((-1e-3, -1e-3, 0.0), (1e-3, 1e-3, 1e-3), (3, 3, 1))
    scan = _ms(ant, y, grid)
    h = (window - 1) // 2
    p = np.array([np.float32(synth.pulse(np.array(k * DT))) for k in range(-h, h + 1)], dtype=np.float64)
    das = oracle.image_indices(scan, oracle.DAS, [[1, 1, 0]], window)[0]
    dmas = oracle.image_indices(scan, oracle.DMAS, [[1, 1, 0]], window)[0]
    pair = (amps.sum() ** 2 - (amps ** 2).sum()) / 2.0
    assert das == pytest.approx(amps.sum() ** 2 * np.sum(p ** 2), rel=1e-10, abs=1e-300)
    assert dmas == pytest.approx(pair ** 2 * np.sum(p ** 4), rel=1e-10, abs=1e-300)


def _brute_ms(scan, bf, window):
    """Independent re-statement with np.interp on zero-padded traces; DMAS via ((sum s)^2 - sum s^2) / 2."""
    nx, ny, nz = scan.grid.dims
    h = (window - 1) // 2
    t = scan.traces.astype(np.float64)
    T = t.shape[1]
    m = scan.ant_pos.shape[0]
    xp = np.arange(-1, T + 1, dtype=np.float64)
    out = np.zeros((nz, ny, nx))
    k = np.arange(-h, h + 1)
    for iz, iy, ix in itertools.product(range(nz), range(ny), range(nx)):
        r = np.asarray(scan.grid.origin) + np.array([ix, iy, iz]) * np.asarray(scan.grid.pitch)
        d = np.linalg.norm(r[None, :] - scan.ant_pos.astype(np.float64), axis=1)
        s = []
        for i in range(m):
            for j in range(m):
                tau = ((d[i] + d[j]) / scan.v - scan.t0) / scan.dt
                s.append(np.interp(tau + k, xp, np.concatenate([[0.0], t[i * m + j], [0.0]]), left=0.0, right=0.0))
        s = np.stack(s)
        if bf == 0:
            out[iz, iy, ix] = np.sum(s.sum(axis=0) ** 2)
        else:
            out[iz, iy, ix] = np.sum(((s.sum(axis=0) ** 2 - (s ** 2).sum(axis=0)) / 2) ** 2)
    return out


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("bf", [0, 1])
def test_brute_force_tiny(seed, bf):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 4))
    T = int(rng.integers(8, 33))
    window = int(rng.choice([1, 3, 5]))
    ant = rng.uniform(-0.02, 0.02, (m, 3))
    y = rng.standard_normal((m * m, T))
    grid = Grid((-0.01, -0.012, 0.003), (0.007, 0.006, 0.004), (4, 3, 2))
    scan = _ms(ant, y, grid, 1e-11, float(rng.uniform(-5e-11, 5e-11)), 2 * 0.04 / (T * 1e-11))
    got = oracle.image_grid(scan, bf, window)
    want = _brute_ms(scan, bf, window)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-13 * max(1.0, np.abs(want).max()))


@pytest.mark.parametrize("bf", [0, 1])
def test_diagonal_channels_reduce_to_monostatic(bf):
    """Eq. (2) with i = j is Eq. (1): with only the diagonal channels non-zero the multistatic image equals the
    monostatic image of those traces (zero channels add nothing to the sums or the pair products)."""
    g = Grid((-0.02, -0.02, 0.0), (0.04 / 9, 0.04 / 9, 1e-3), (10, 10, 1))
    mono = synth.random_scan(3, 6, 256, g, radius=0.07)
    m = mono.n_ant
    y = np.zeros((m * m, mono.n_samp), np.float32)
    for i in range(m):
        y[i * m + i] = mono.traces[i]
    ms = _ms(mono.ant_pos, y, g, mono.dt, mono.t0, mono.v)
    np.testing.assert_allclose(oracle.image_grid(ms, bf), oracle.image_grid(mono, bf), rtol=1e-12, atol=0)


@pytest.mark.parametrize("bf", [0, 1])
def test_reciprocity_and_relabelling(bf):
    g = Grid((-0.02, -0.02, 0.0), (0.04 / 7, 0.04 / 7, 1e-3), (8, 8, 1))
    s = synth.random_scan_ms(1, 5, 256, g, radius=0.07)
    m = s.n_ant
    base = oracle.image_grid(s, bf)
    # swapping the roles of transmitter and receiver (channel (i, j) -> (j, i)): same paths, same image
    y = s.traces.reshape(m, m, -1).transpose(1, 0, 2).reshape(m * m, -1)
    np.testing.assert_allclose(oracle.image_grid(_ms(s.ant_pos, y, g, s.dt, s.t0, s.v), bf), base, rtol=1e-11)
    # relabelling the antennas (and their channels accordingly)
    perm = np.array([3, 0, 4, 1, 2])
    y = s.traces.reshape(m, m, -1)[perm][:, perm].reshape(m * m, -1)
    np.testing.assert_allclose(oracle.image_grid(_ms(s.ant_pos[perm], y, g, s.dt, s.t0, s.v), bf), base,
                               rtol=1e-11)


@pytest.mark.parametrize("dataset", [1, 2])
@pytest.mark.parametrize("bf", [0, 1])
def test_point_tumour_found(dataset, bf):
    s = synth.ms_scan(0, dataset, noiseless=True)
    img = oracle.image_grid(s, bf)
    k, _ = oracle.argmax_grid(img)
    nx = s.grid.dims[0]
    pos = np.asarray(s.grid.origin) + np.array([k % nx, k // nx, 0]) * np.asarray(s.grid.pitch)
    assert np.max(np.abs(pos[:2] - s.tumour[:2])) <= 1.0e-3 + 1e-9     # within one voxel


def test_multistatic_needs_m_squared_traces():
    g = Grid((0.0, 0.0, 0.0), (1e-3, 1e-3, 1e-3), (2, 2, 1))
    bad = _ms(np.zeros((3, 3)), np.zeros((4, 16)), g)
    with pytest.raises(ValueError):
        oracle.image_grid(bad, 0)
