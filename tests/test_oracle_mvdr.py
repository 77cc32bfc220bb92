"""Pins of the Capon (MVDR) oracle on the aligned window samples.

Each check ties it to something other than itself: a closed form for a coherent point echo (the
Sherman-Morrison inverse of a rank-one covariance plus loading, worked out by hand), the constrained
minimisation that defines the weights solved through its own optimality system, brute force of the gather with
numpy's interpolation, the limit of heavy loading (uniform weights: the DAS image over M^2), invariances, and the
physics of a point scatterer.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import mvdr
from synth import Grid, Scan

_U = 1.0 / 128.0
_RING12 = np.array([(3, 4), (4, 3), (5, 0), (4, -3), (3, -4), (0, -5), (-3, -4), (-4, -3), (-5, 0),
                    (-4, 3), (-3, 4), (0, 5)], dtype=np.float64) * _U
DT = 2e-11
V = 0.078125 / (40 * DT)      # round trip 2 x 5/128 m takes exactly 40 samples


def _pulse_samples(window):
    h = (window - 1) // 2
    return np.array([np.float32(synth.pulse(np.array(k * DT))) for k in range(-h, h + 1)], dtype=np.float64)


def _coherent_energy(amps, p, loading):
    """Closed form for aligned samples X = A p^T (one echo, channel amplitudes A): the covariance is
    R = c A A^T with c = |p|^2 / W, the loading delta = loading * c |A|^2 / M, and Sherman-Morrison gives
    (R + delta I)^-1 1 = (1 - c (A.1) A / (delta + c |A|^2)) / delta, hence
    w.A = (A.1) delta / (M (delta + c |A|^2) - c (A.1)^2) and I = (w.A)^2 |p|^2."""
    m, w_len = len(amps), len(p)
    s1, s2, pp = amps.sum(), (amps ** 2).sum(), (p ** 2).sum()
    c = pp / w_len
    delta = loading * c * s2 / m
    wa = s1 * delta / (m * (delta + c * s2) - c * s1 ** 2)
    return wa ** 2 * pp


@pytest.mark.parametrize("m", [1, 2, 3, 7, 12])
@pytest.mark.parametrize("window", [5, 11])
@pytest.mark.parametrize("loading", [0.01, 0.1, 1.0])
def test_centre_closed_form(m, window, loading):
    rng = np.random.default_rng(m * 100 + window)
    amps = 2.0 ** rng.integers(-3, 4, m).astype(np.float64)
    ant = np.zeros((m, 3), dtype=np.float32)
    ant[:, :2] = _RING12[:m]
    n = np.arange(128)
    y = np.stack([a * synth.pulse(n * DT - 40 * DT) for a in amps]).astype(np.float32)
    scan = Scan(ant, y, DT, 0.0, V, Grid((-1e-3, -1e-3, 0.0), (1e-3, 1e-3, 1e-3), (3, 3, 1)))
    p = _pulse_samples(window)
    got = oracle.image_indices(scan, oracle.MVDR, [[1, 1, 0]], window, loading=loading)[0]
    assert got == pytest.approx(_coherent_energy(amps, p, loading), rel=1e-10)
    if np.all(amps == amps[0]):
        # equal amplitudes: the weights are uniform whatever the loading, I = I_DAS / M^2
        assert got == pytest.approx(amps[0] ** 2 * np.sum(p ** 2), rel=1e-10)


def test_centre_closed_form_equal_amplitudes():
    m, window = 8, 11
    ant = np.zeros((m, 3), dtype=np.float32)
    ant[:, :2] = _RING12[:m]
    n = np.arange(128)
    y = np.stack([0.5 * synth.pulse(n * DT - 40 * DT) for _ in range(m)]).astype(np.float32)
    scan = Scan(ant, y, DT, 0.0, V, Grid((-1e-3, -1e-3, 0.0), (1e-3, 1e-3, 1e-3), (3, 3, 1)))
    das = oracle.image_indices(scan, oracle.DAS, [[1, 1, 0]], window)[0]
    for loading in (1e-3, 0.1, 10.0):
        got = oracle.image_indices(scan, oracle.MVDR, [[1, 1, 0]], window, loading=loading)[0]
        assert got == pytest.approx(das / m ** 2, rel=1e-10)


def test_multistatic_centre_closed_form():
    """M^2 channels of a ring all meet at the centre after 40 samples: the same closed form over M^2 amplitudes."""
    m, window, loading = 3, 11, 0.1
    rng = np.random.default_rng(5)
    ant = np.zeros((m, 3))
    ant[:, :2] = _RING12[:m]
    amps = 2.0 ** rng.integers(-3, 4, m * m).astype(np.float64)
    n = np.arange(128)
    y = np.stack([a * synth.pulse(n * DT - 40 * DT) for a in amps]).astype(np.float32)
    scan = Scan(ant.astype(np.float32), y, DT, 0.0, V, Grid((-1e-3, -1e-3, 0.0), (1e-3, 1e-3, 1e-3), (3, 3, 1)),
                multistatic=True)
    got = oracle.image_indices(scan, oracle.MVDR, [[1, 1, 0]], window, loading=loading)[0]
    assert got == pytest.approx(_coherent_energy(amps, _pulse_samples(window), loading), rel=1e-10)


@pytest.mark.parametrize("seed", range(5))
def test_weights_solve_the_constrained_minimum(seed):
    """w minimises w^T R_l w subject to w^T 1 = 1.  Its optimality system [[2 R_l, 1], [1^T, 0]] [w; lam] = [0; 1]
    is solved on its own, and feasible perturbations never lower the output power."""
    rng = np.random.default_rng(seed)
    m, w_len = int(rng.integers(2, 17)), int(rng.choice([1, 3, 5, 11]))
    X = rng.standard_normal((4, m, w_len)) * rng.uniform(0.1, 3.0, (4, m, 1))
    loading = float(rng.choice([0.01, 0.1, 1.0]))
    w = mvdr.capon_weights(X, loading)
    for n in range(4):
        R = X[n] @ X[n].T / w_len
        Rl = R + loading * np.trace(R) / m * np.eye(m)
        kkt = np.zeros((m + 1, m + 1))
        kkt[:m, :m] = 2 * Rl
        kkt[:m, m] = 1.0
        kkt[m, :m] = 1.0
        rhs = np.zeros(m + 1)
        rhs[m] = 1.0
        want = np.linalg.solve(kkt, rhs)[:m]
        np.testing.assert_allclose(w[n], want, rtol=1e-9, atol=1e-12)
        assert w[n].sum() == pytest.approx(1.0, rel=1e-12)
        base = w[n] @ Rl @ w[n]
        for _ in range(20):
            v = rng.standard_normal(m)
            v -= v.mean()                      # keeps the distortionless constraint
            assert (w[n] + v) @ Rl @ (w[n] + v) >= base * (1 - 1e-12)
    # the energy is the squared output summed over the window
    e = mvdr.capon_energy(X, loading)
    np.testing.assert_allclose(e, [np.sum((w[n] @ X[n]) ** 2) for n in range(4)], rtol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_aligned_samples_brute_force(seed):
    """The gather handed to the Capon weights, against numpy interpolation of zero-padded traces."""
    rng = np.random.default_rng(seed)
    m, T, window = int(rng.integers(1, 5)), int(rng.integers(8, 33)), int(rng.choice([1, 3, 5, 11]))
    ant = rng.uniform(-0.02, 0.02, (m, 3)).astype(np.float32)
    y = rng.standard_normal((m, T)).astype(np.float32)
    grid = Grid((-0.01, -0.012, 0.003), (0.007, 0.006, 0.004), (4, 4, 2))
    scan = Scan(ant, y, 1e-11, float(rng.uniform(-5e-11, 5e-11)), 2 * 0.04 / (T * 1e-11), grid)
    idx = np.array(list(itertools.product(range(4), range(4), range(2))), dtype=np.int32)
    got = oracle.aligned_samples(scan, idx, window)
    h = (window - 1) // 2
    xp = np.arange(-1, T + 1, dtype=np.float64)
    k = np.arange(-h, h + 1)
    for p, (ix, iy, iz) in enumerate(idx):
        r = np.asarray(grid.origin) + np.array([ix, iy, iz]) * np.asarray(grid.pitch)
        d = np.linalg.norm(r[None, :] - ant.astype(np.float64), axis=1)
        tau = (2 * d / scan.v - scan.t0) / scan.dt
        for i in range(m):
            want = np.interp(tau[i] + k, xp, np.concatenate([[0.0], y[i].astype(np.float64), [0.0]]))
            np.testing.assert_allclose(got[p, i], want, rtol=1e-12, atol=1e-14)


def test_light_loading_cancels_a_slightly_misaligned_echo():
    """The reason for the default loading: at loading 0.1 the voxel nearest a noiseless point tumour (a third of
    a voxel off it) keeps under a tenth of the local maximum; at the default, over a third."""
    s = synth.c1_scan(0, noiseless=True)
    idx = oracle.box_indices((26, 34, 105, 113, 0, 1))
    near = np.round((np.asarray(s.tumour) - np.asarray(s.grid.origin)) / np.asarray(s.grid.pitch)).astype(int)
    j = int(np.nonzero((idx[:, 0] == near[0]) & (idx[:, 1] == near[1]))[0][0])
    light = oracle.image_indices(s, oracle.MVDR, idx, loading=0.1)
    dflt = oracle.image_indices(s, oracle.MVDR, idx)
    assert light[j] < 0.1 * light.max()
    assert dflt[j] > 0.33 * dflt.max()


def test_heavy_loading_gives_uniform_weights():
    """loading -> infinity: R_l ~ delta I, the weights tend to 1/M and the image to the DAS image / M^2."""
    s = synth.c1_scan(3, n_grid=24)
    idx = oracle.box_indices((0, 24, 0, 24, 0, 1))
    das = oracle.image_indices(s, oracle.DAS, idx)
    got = oracle.image_indices(s, oracle.MVDR, idx, loading=1e9)
    np.testing.assert_allclose(got, das / s.n_ant ** 2, rtol=1e-6, atol=1e-12 * das.max())


def test_scale_permutation_and_no_signal():
    s = synth.c1_scan(4, n_grid=12)
    idx = oracle.box_indices((0, 12, 0, 12, 0, 1))
    base = oracle.image_indices(s, oracle.MVDR, idx)
    s2 = Scan(s.ant_pos, (s.traces.astype(np.float64) * 4.0).astype(np.float32), s.dt, s.t0, s.v, s.grid)
    np.testing.assert_allclose(oracle.image_indices(s2, oracle.MVDR, idx), 16.0 * base, rtol=1e-10)
    perm = np.random.default_rng(0).permutation(s.n_ant)
    s3 = Scan(s.ant_pos[perm], s.traces[perm], s.dt, s.t0, s.v, s.grid)
    np.testing.assert_allclose(oracle.image_indices(s3, oracle.MVDR, idx), base, rtol=1e-9)
    s4 = Scan(s.ant_pos, np.zeros_like(s.traces), s.dt, s.t0, s.v, s.grid)
    assert not oracle.image_indices(s4, oracle.MVDR, idx).any()


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("noiseless", [True, False])
def test_point_scatterer_found(seed, noiseless):
    """A point tumour (the 16-antenna ring, 128 x 128 grid; noiseless, and at 30 dB) is detected within one voxel
    at the default loading."""
    s = synth.c1_scan(seed, noiseless=noiseless)
    img = oracle.image_grid(s, oracle.MVDR)
    a, _ = oracle.argmax_grid(img)
    nx = s.grid.dims[0]
    tum = np.round((np.asarray(s.tumour) - np.asarray(s.grid.origin)) / np.asarray(s.grid.pitch)).astype(int)
    assert abs(a % nx - tum[0]) <= 1 and abs(a // nx - tum[1]) <= 1


@pytest.mark.parametrize("walk", ["per_level", "paper"])
def test_framework_over_mvdr_finds_the_full_image_detection(walk):
    """The Section III walk run over the Capon beamformer: on a noisy point-tumour scan its detection is the
    full-resolution MVDR detection, and the walk images far fewer focal points."""
    s = synth.c1_scan(1)
    full = oracle.image_grid(s, oracle.MVDR)
    a, _ = oracle.argmax_grid(full)
    r = oracle.walk(s, oracle.TreeParams(beamformer=oracle.MVDR, walk=walk, coarse=8, min_tumour=0.01,
                                         metric="max", frame_final=0.25))
    nx = s.grid.dims[0]
    assert abs(r.argmax % nx - a % nx) <= 1 and abs(r.argmax // nx - a // nx) <= 1
    assert r.voxels_evaluated < full.size / 3
