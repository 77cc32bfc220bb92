"""GPU parity of the segment walk (Section III) against the oracle: bit-exact child
sequence, boxes, stop level, ROI and argmax; FP64 scores, W/B values and the detection's energy to 1e-12
relative (FP64 on both sides in different summation orders: the largest difference measured over these tests
is about 4e-14, printed at the end of the session)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402

METRICS = ["mean", "var", "eq5", "max", "max_over_mean", "eq5_clamped"]


def uwb():
    import paper_1709_02549_amd as m
    return m


def _params(**kw):
    return oracle.TreeParams(**kw), uwb().SegmentTree(**kw)


# largest relative GPU - oracle difference of the walk's FP64 scores and W/B figures over the session
# (printed in the terminal summary; the decisions themselves are compared exactly)
SCORE_DIFF = {"score": 0.0, "wb": 0.0}


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    d = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
    return float(np.max(np.where(a == b, 0.0, d))) if d.size else 0.0


def _compare(g, o, exact_scores=1e-12):
    assert g.child == o.child
    assert g.n_levels == o.n_levels and g.term_level == o.term_level
    assert [tuple(b) for b in g.boxes] == [tuple(b) for b in o.boxes]
    assert tuple(g.roi) == tuple(o.roi)
    assert g.argmax == o.argmax
    assert g.peak == pytest.approx(o.peak, rel=1e-12)
    assert g.voxels_evaluated == o.voxels_evaluated
    for a, b in zip(g.scores, o.scores):
        np.testing.assert_allclose(a, b, rtol=exact_scores, atol=1e-300)
        SCORE_DIFF["score"] = max(SCORE_DIFF["score"], _rel(a, b))
    assert len(g.wb) == len(o.wb)
    for a, b in zip(g.wb, o.wb):
        np.testing.assert_allclose(a, b, rtol=1e-12)
        SCORE_DIFF["wb"] = max(SCORE_DIFF["wb"], _rel(a, b))
    # the detection was decided in FP64 over the ROI's near-maximal FP32 candidates, the winner among them
    if g.argmax >= 0:
        x0, x1, y0, y1, z0, z1 = g.roi
        assert 1 <= g.guard_hits <= (x1 - x0) * (y1 - y0) * (z1 - z0)
    if o.roi_image is not None and g.roi_image is not None:
        roi_close(g.roi_image, o.roi_image)


def roi_close(got, want, window=11):
    """The ROI is imaged in FP32 (its detection is decided in FP64, checked above): the full-image bar,
    |error| <= 1e-4 x peak everywhere and <= 1e-4 relative above 1 % of the peak."""
    peak = np.abs(want).max()
    assert np.max(np.abs(got - want)) <= 1e-4 * peak
    big = np.abs(want) > 1e-2 * peak
    assert np.max(np.abs(got[big] - want[big]) / np.abs(want[big])) <= 1e-4


def composite_close(got, want, roi):
    """Composite: FP32 ROI voxels at the image bar, every other voxel the FP64 coarse value rounded to FP32."""
    inside = np.zeros(want.shape, bool)
    x0, x1, y0, y1, z0, z1 = roi
    inside[z0:z1, y0:y1, x0:x1] = True   # [nz][ny][nx]
    np.testing.assert_allclose(got[~inside], want[~inside], rtol=1e-6, atol=1e-30)
    roi_close(got[inside], want[inside])


@pytest.mark.parametrize("metric", METRICS)
@pytest.mark.parametrize("term", ["fixed", "wb"])
@pytest.mark.parametrize("bf", [0, 1])
def test_per_level_c1(metric, term, bf):
    s = synth.c1_scan(7)
    op, gp = _params(beamformer=bf, coarse=8, metric=metric, term=term, frame_level=0.25, frame_final=0.25)
    o = oracle.walk(s, op)
    g = uwb().segment_refine(uwb().DeviceScan.from_host(s), s.grid, gp, want_roi=True)
    _compare(g, o)


@pytest.mark.parametrize("metric", METRICS)
@pytest.mark.parametrize("term", ["fixed", "wb"])
@pytest.mark.parametrize("bf", [0, 1])
def test_paper_walk_c1(metric, term, bf):
    s = synth.c1_scan(8)
    op, gp = _params(beamformer=bf, walk="paper", metric=metric, term=term, frame_level=0.25, frame_final=0.25,
                     min_tumour=0.01)
    o = oracle.walk(s, op)
    g = uwb().segment_refine(uwb().DeviceScan.from_host(s), s.grid, gp, want_roi=True)
    assert g.decimation == o.decimation
    _compare(g, o)


@pytest.mark.parametrize("bf", [0, 1])
@pytest.mark.parametrize("metric", ["max", "mean"])
def test_c2_full_size_batch(bf, metric):
    """C2: 512 x 512, g = 8, 32 antennas, T = 2048; 8 scans in one batched launch."""
    scans = [synth.c2_scan(k) for k in range(8)]
    u = uwb()
    b = u.DeviceBatch.from_host(scans)
    op, gp = _params(beamformer=bf, coarse=8, metric=metric, frame_final=0.25)
    res = u.segment_refine_batch(b, scans[0].grid, gp, want_roi=True)
    for s, g in zip(scans, res):
        _compare(g, oracle.walk(s, op))


@pytest.mark.parametrize("metric", ["max", "eq5", "var"])
def test_c2_paper_walk_manual_and_auto(metric):
    s = synth.c2_scan(11)
    for dec in (0, 20):
        op, gp = _params(beamformer=1, walk="paper", decimation=dec, metric=metric, frame_level=0.25, term="wb")
        o = oracle.walk(s, op)
        g = uwb().segment_refine(uwb().DeviceScan.from_host(s), s.grid, gp)
        _compare(g, o)


@pytest.mark.parametrize("bf", [0, 1])
def test_c3_octree(bf):
    """3D octree walk on the C3 geometry (64 antennas, T = 4096) at 64^3 and at the full 256^3."""
    for n, seed in [(64, 0), (256, 1)]:
        s = synth.c3_scan(seed, n_grid=n)
        op, gp = _params(beamformer=bf, coarse=8, metric="max", frame_final=0.25)
        o = oracle.walk(s, op)
        g = uwb().segment_refine(uwb().DeviceScan.from_host(s), s.grid, gp, want_roi=True)
        _compare(g, o)


@pytest.mark.parametrize("coarse,n", [(6, 48), (10, 40)])
@pytest.mark.parametrize("bf", [0, 1])
def test_c3_octree_ragged_lattices(coarse, n, bf):
    """Lattices that are no whole number of 8 x 8 x 4 tiles (6^3 and 10^3 points per level, a 14^3 ROI) are
    evaluated in bands of 256 consecutive points that cross z-slabs; values and decisions stay the oracle's."""
    s = synth.c3_scan(2, n_grid=n)
    op, gp = _params(beamformer=bf, coarse=coarse, metric="max", frame_final=0.25)
    o = oracle.walk(s, op)
    g = uwb().segment_refine(uwb().DeviceScan.from_host(s), s.grid, gp, want_roi=True)
    _compare(g, o)


def test_frame_level_and_depth_limits():
    s = synth.c1_scan(9)
    for kw in [dict(max_depth=2), dict(max_depth=1, term="wb"), dict(coarse=4, frame_level=0.5),
               dict(coarse=16, frame_final=0.0), dict(coarse=2, metric="mean")]:
        op, gp = _params(beamformer=0, **kw)
        _compare(uwb().segment_refine(uwb().DeviceScan.from_host(s), s.grid, gp), oracle.walk(s, op))


@pytest.mark.parametrize("term", ["fixed", "wb"])
@pytest.mark.parametrize("bf", [0, 1])
def test_walk_without_levels(term, bf):
    """A lattice as fine as the grid (g = 16 on 16 x 16) leaves no level to split: the walk keeps the whole grid
    as its box and ROI.  With the W/B stop the one-workgroup walk runs its single level and stops there; with
    a fixed depth there is no level and the set-up and record kernels run alone."""
    s = synth.c1_scan(3, n_grid=16)
    op, gp = _params(beamformer=bf, coarse=16, term=term, frame_final=0.25)
    g = uwb().segment_refine(uwb().DeviceScan.from_host(s), s.grid, gp)
    _compare(g, oracle.walk(s, op))
    assert g.n_levels == 0 and g.child == [] and tuple(g.roi) == (0, 16, 0, 16, 0, 1)


@pytest.mark.parametrize("walk,kw", [("paper", dict(min_tumour=0.01, frame_final=0.25)),
                                     ("per_level", dict(coarse=8, frame_final=0.25)),
                                     ("paper", dict(min_tumour=0.01, frame_final=1.0))])
@pytest.mark.parametrize("bf", [0, 1])
def test_flat_scan_ties_everywhere(walk, kw, bf):
    """All-zero traces: every energy is 0, every child and every ROI voxel ties, so each choice falls to the
    lowest index.  100 and 400 tied ROI voxels fill the pick's candidate list in LDS; 1024 (the whole-frame
    ROI) overflow its 512 entries and take the serial pick, whose 64-entry lane list overflows too."""
    s = synth.c1_scan(3)
    s0 = synth.Scan(s.ant_pos, np.zeros_like(s.traces), s.dt, s.t0, s.v, s.grid)
    op, gp = _params(beamformer=bf, walk=walk, metric="max", **kw)
    o = oracle.walk(s0, op)
    g = uwb().segment_refine(uwb().DeviceScan.from_host(s0), s0.grid, gp, want_roi=True)
    assert g.child == o.child and tuple(g.roi) == tuple(o.roi)
    assert g.argmax == o.argmax == s0.grid.dims[0] * o.roi[2] + o.roi[0]
    assert g.peak == 0.0 and not g.roi_image.any()
    # every ROI voxel ties with the maximum: each one is re-evaluated in FP64
    x0, x1, y0, y1, z0, z1 = g.roi
    assert g.guard_hits == (x1 - x0) * (y1 - y0) * (z1 - z0)


@pytest.mark.parametrize("bf,metric,term", [(0, "max", "fixed"), (1, "eq5", "wb")])
def test_walk_batch_size_invariance(bf, metric, term):
    """A per-level walk of small lattices runs all its levels in one launch for batches up to 1024 scans and
    level by level beyond: 8 scans and 1100 copies of them must give the same results, bit for bit."""
    u = uwb()
    scans = [synth.c1_scan(k) for k in range(8)]
    _, gp = _params(beamformer=bf, coarse=8, metric=metric, term=term, frame_level=0.25, frame_final=0.25)
    small = u.segment_refine_batch(u.DeviceBatch.from_host(scans), scans[0].grid, gp, want_roi=True)
    big = u.segment_refine_batch(u.DeviceBatch.from_host([scans[k % 8] for k in range(1100)]), scans[0].grid, gp,
                                 want_roi=True)
    for k in (0, 1, 7, 8, 555, 1099):
        a, b = small[k % 8], big[k]
        assert a.child == b.child and a.n_levels == b.n_levels and a.term_level == b.term_level
        assert [tuple(x) for x in a.boxes] == [tuple(x) for x in b.boxes] and tuple(a.roi) == tuple(b.roi)
        assert a.argmax == b.argmax and a.peak == b.peak
        assert all(np.array_equal(x, y) for x, y in zip(a.scores, b.scores))
        assert all(np.array_equal(x, y) for x, y in zip(a.wb, b.wb)) and len(a.wb) == len(b.wb)
        assert np.array_equal(a.roi_image, b.roi_image)


def test_walk_deterministic():
    s = synth.c2_scan(2)
    u = uwb()
    ds = u.DeviceScan.from_host(s)
    _, gp = _params(beamformer=1, coarse=8, metric="eq5", term="wb")
    a = u.segment_refine(ds, s.grid, gp, want_roi=True)
    b = u.segment_refine(ds, s.grid, gp, want_roi=True)
    assert a.child == b.child and a.scores == b.scores and a.argmax == b.argmax
    assert np.array_equal(a.roi_image, b.roi_image)


# ----------------------------------------------------------------------------------
# mixed-resolution composite (final imaging)
# ----------------------------------------------------------------------------------

@pytest.mark.parametrize("walk,kw", [("paper", dict(min_tumour=0.01)), ("paper", dict(decimation=5, frame_level=0.25)),
                                     ("per_level", dict(coarse=8)), ("per_level", dict(coarse=16, term="wb"))])
@pytest.mark.parametrize("bf", [0, 1])
def test_composite_matches_oracle(walk, kw, bf):
    from oracle.walk import composite
    scans = [synth.c1_scan(k) for k in range(3)]
    u = uwb()
    op, gp = _params(beamformer=bf, walk=walk, frame_final=0.25, **kw)
    res, img = u.segment_composite_batch(u.DeviceBatch.from_host(scans), scans[0].grid, gp)
    img = img.cpu().numpy()
    for i, s in enumerate(scans):
        o = oracle.walk(s, op)
        assert res[i].child == o.child and tuple(res[i].roi) == tuple(o.roi)
        want = composite(s, op, o)
        composite_close(img[i], want, o.roi)


def test_composite_c3_octree():
    from oracle.walk import composite
    s = synth.c3_scan(0, n_grid=64)
    u = uwb()
    op, gp = _params(beamformer=0, coarse=8, frame_final=0.25)
    res, img = u.segment_composite_batch(u.DeviceBatch.from_host([s]), s.grid, gp)
    o = oracle.walk(s, op)
    assert res[0].child == o.child
    composite_close(img.cpu().numpy()[0], composite(s, op, o), o.roi)


# ----------------------------------------------------------------------------------
# the two-decimation check (no-tumour test)
# ----------------------------------------------------------------------------------

@pytest.mark.parametrize("bf", [0, 1])
def test_tumour_check_matches_oracle(bf):
    """Scans with a tumour (C1) and without (white noise only): same verdict and walks as the oracle."""
    from oracle.walk import tumour_check
    grid = synth.square_grid(128)
    scans = [synth.c1_scan(k) for k in range(4)] + [synth.random_scan(k, 16, 1024, grid) for k in range(4)]
    u = uwb()
    op, gp = _params(beamformer=bf, walk="paper", metric="max", frame_final=0.25)
    agree, ra, rb = u.tumour_check_batch(u.DeviceBatch.from_host(scans), grid, gp, 9, 5)
    verdicts = []
    for i, s in enumerate(scans):
        ok, o1, o2 = tumour_check(s, op, 9, 5)
        assert ra[i].child == o1.child and rb[i].child == o2.child
        assert tuple(ra[i].roi) == tuple(o1.roi) and tuple(rb[i].roi) == tuple(o2.roi)
        assert ra[i].argmax == o1.argmax and rb[i].argmax == o2.argmax
        assert bool(agree[i]) == ok
        verdicts.append(ok)
    assert all(verdicts[:4])          # a tumour: confirmed


def test_tumour_check_argument_errors():
    u = uwb()
    scans = [synth.c1_scan(0)]
    b = u.DeviceBatch.from_host(scans)
    with pytest.raises(u.UwbError):
        u.tumour_check_batch(b, scans[0].grid, u.SegmentTree(walk="paper"), 5, 5)
    with pytest.raises(u.UwbError):
        u.tumour_check_batch(b, scans[0].grid, u.SegmentTree(walk="per_level"), 5, 7)
