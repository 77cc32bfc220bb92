"""GPU parity of multistatic imaging (Eq. (2) delay, Eq. (4) DAS, pairwise DMAS over the M^2 channels), its
FP64-decided argmax and the segment walks, against the FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
from synth import Grid  # noqa: E402


def uwb():
    import paper_1709_02549_amd as m
    return m


def _check_image(got, want, tol=1e-4, voxel_tol=None):
    """The image bar: |error| <= tol x peak everywhere, and <= voxel_tol relative above 1 % of the peak (tol
    unless given; windows under 5 samples take their delay in FP64 and meet the same bar)."""
    peak = np.abs(want).max()
    assert np.max(np.abs(got - want)) <= tol * peak
    big = np.abs(want) > 1e-2 * peak
    rel = np.abs(got[big] - want[big]) / np.abs(want[big])
    assert rel.max() <= (voxel_tol or tol)


@pytest.mark.parametrize("dataset", [1, 2])
@pytest.mark.parametrize("bf", [0, 1])
def test_paper_geometry_images_and_detection(dataset, bf):
    """The 12-antenna rings standing in for the two datasets of Section IV."""
    u = uwb()
    s = synth.ms_scan(dataset, dataset)
    ds = u.DeviceScan.from_host(s)
    img = u.image_multistatic(ds, s.grid, bf)
    want = oracle.image_grid(s, bf)
    _check_image(img.cpu().numpy(), want)
    pk = u.argmax_multistatic(ds, s.grid, img, bf)
    k, v = oracle.argmax_grid(want)
    assert pk.index == k
    assert pk.value == pytest.approx(v, rel=1e-9)


@pytest.mark.parametrize("window", [1, 5, 11, 31])
@pytest.mark.parametrize("bf", [0, 1])
def test_random_channels(window, bf):
    u = uwb()
    g = Grid((-0.03, -0.02, 0.0), (0.0017, 0.0021, 1e-3), (37, 23, 1))      # ragged tiles
    s = synth.random_scan_ms(window, 5, 512, g, radius=0.07)
    img = u.image_multistatic(u.DeviceScan.from_host(s), g, bf, window).cpu().numpy()
    _check_image(img, oracle.image_grid(s, bf, window))


@pytest.mark.parametrize("bf", [0, 1])
def test_3d_grid(bf):
    u = uwb()
    g = Grid((-0.02, -0.02, 0.0), (0.002, 0.002, 0.002), (20, 20, 11))
    ant = synth.hemisphere_antennas(6)
    pts = np.array([[0.004, -0.006, 0.01]])
    y = synth.synthesize_ms(ant, pts, [1.0], 1024, synth.C0 / 3.0)
    s = synth.Scan(ant.astype(np.float32), y.astype(np.float32), synth.DT, 0.0, synth.C0 / 3.0, g, multistatic=True)
    img = u.image_multistatic(u.DeviceScan.from_host(s), g, bf).cpu().numpy()
    want = oracle.image_grid(s, bf)
    _check_image(img, want)
    pk = u.argmax_multistatic(u.DeviceScan.from_host(s), g, torch.tensor(img, device="cuda"), bf)
    assert pk.index == oracle.argmax_grid(want)[0]


@pytest.mark.parametrize("bf", [0, 1])
def test_batch_equals_single(bf):
    u = uwb()
    scans = [synth.ms_scan(k, 2) for k in range(3)]
    b = u.DeviceBatch.from_host(scans)
    imgs = u.image_multistatic_batch(b, scans[0].grid, bf).cpu().numpy()
    for i, s in enumerate(scans):
        one = u.image_multistatic(u.DeviceScan.from_host(s), s.grid, bf).cpu().numpy()
        np.testing.assert_array_equal(imgs[i], one)
    pks = u._peaks(u.argmax_multistatic_batch_async(b, scans[0].grid, torch.tensor(imgs, device="cuda"), bf), 3)
    for i, s in enumerate(scans):
        assert pks[i].index == oracle.argmax_grid(oracle.image_grid(s, bf))[0]


def test_diagonal_channels_match_monostatic():
    """Only the i = j channels carry signal: the multistatic kernels reproduce the monostatic image."""
    u = uwb()
    mono = synth.c1_scan(4)
    m = mono.n_ant
    y = np.zeros((m * m, mono.n_samp), np.float32)
    for i in range(m):
        y[i * m + i] = mono.traces[i]
    ms = synth.Scan(mono.ant_pos, y, mono.dt, mono.t0, mono.v, mono.grid, multistatic=True)
    for bf in (0, 1):
        a = u.image_multistatic(u.DeviceScan.from_host(ms), mono.grid, bf).cpu().numpy()
        b = u.image(u.DeviceScan.from_host(mono), mono.grid, bf).cpu().numpy()
        _check_image(a, b, 2e-5)


@pytest.mark.parametrize("walk,kw", [("paper", dict(min_tumour=0.01)), ("paper", dict(decimation=5, term="wb")),
                                     ("per_level", dict(coarse=50))])
@pytest.mark.parametrize("bf", [0, 1])
def test_walks_match_oracle(walk, kw, bf):
    u = uwb()
    for dataset in (1, 2):
        s = synth.ms_scan(10 + dataset, dataset)
        op = oracle.TreeParams(beamformer=bf, walk=walk, frame_final=0.25, metric="max", **kw)
        gp = u.SegmentTree(beamformer=bf, walk=walk, frame_final=0.25, metric="max", **kw)
        o = oracle.walk(s, op)
        g = u.segment_refine_multistatic(u.DeviceScan.from_host(s), s.grid, gp, want_roi=True)
        assert g.child == o.child and [tuple(b) for b in g.boxes] == [tuple(b) for b in o.boxes]
        assert tuple(g.roi) == tuple(o.roi) and g.argmax == o.argmax
        assert g.peak == pytest.approx(o.peak, rel=1e-9)
        for a, b in zip(g.scores, o.scores):
            np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-300)
        _check_image(g.roi_image, o.roi_image)   # the ROI is imaged in FP32; its detection is FP64 (above)


def test_paper_decimation_finds_the_tumour():
    """The paper's setting: 1 cm tumour, 1 mm resolution -> D = 7; the walk's detection is the full image's."""
    u = uwb()
    s = synth.ms_scan(0, 1)
    gp = u.SegmentTree(beamformer=1, walk="paper", min_tumour=0.01, metric="max", frame_final=0.25)
    g = u.segment_refine_multistatic(u.DeviceScan.from_host(s), s.grid, gp)
    assert g.decimation == 7
    ds = u.DeviceScan.from_host(s)
    full = u.argmax_multistatic(ds, s.grid, u.image_multistatic(ds, s.grid, 1), 1)
    nx = s.grid.dims[0]
    assert abs(g.argmax % nx - full.index % nx) <= 1 and abs(g.argmax // nx - full.index // nx) <= 1


def test_argument_errors():
    u = uwb()
    s = synth.ms_scan(0, 2)
    ds = u.DeviceScan.from_host(s)
    bad = u.DeviceScan(ds.ant_pos, ds.traces[:100].contiguous(), ds.dt, ds.t0, ds.v)
    with pytest.raises(ValueError):
        u.image_multistatic(bad, s.grid, 0)


def test_das_dmas_multistatic_one_launch():
    """Both multistatic images from one launch: DMAS bit for bit as the DMAS call, DAS at the image bar."""
    u = uwb()
    scans = [synth.ms_scan(k, 2) for k in range(3)]
    b = u.DeviceBatch.from_host(scans)
    das, dmas = u.das_dmas_multistatic_batch(b, scans[0].grid)
    torch.cuda.synchronize()
    assert torch.equal(dmas, u.image_multistatic_batch(b, scans[0].grid, 1))
    for i, s in enumerate(scans):
        _check_image(das[i].cpu().numpy(), oracle.image_grid(s, 0))
