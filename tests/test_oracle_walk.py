"""Pins of the oracle's Section III framework (decimation, ROI selection, W/B stop, final imaging)."""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle.walk import TreeParams, composite, metric_value, within_between
from synth import Grid, Scan

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


def test_auto_decimation_paper_example():
    """Section IV: 1 cm tumour, 1 mm resolution -> spatial decimation factor 7."""
    for dmin, pitch, want in _rows("auto_decimation.txt"):
        assert oracle.auto_decimation(float(dmin), float(pitch)) == int(want)


def test_auto_decimation_floor_and_minimum():
    assert oracle.auto_decimation(0.01, 0.0005) == 14       # 7.07 mm / 0.5 mm
    assert oracle.auto_decimation(0.001, 0.001) == 1        # below one voxel -> 1
    with pytest.raises(ValueError):
        oracle.auto_decimation(0.01, 0.0)


# ----------------------------------------------------------------------------------
# metrics, Eq. (5)-(7)
# ----------------------------------------------------------------------------------

def test_basic_metrics_by_hand():
    x = np.array([1.0, 2.0, 3.0, 6.0])
    assert metric_value("mean", x, x) == 3.0
    assert metric_value("var", x, x) == pytest.approx((4 + 1 + 0 + 9) / 4)
    assert metric_value("max", x, x) == 6.0
    assert metric_value("max_over_mean", x, x) == 2.0
    assert metric_value("max_over_mean", np.zeros(3), x) == 0.0


def test_eq5_limits():
    """Section III prose: equal variances -> the mean dominates; a distinct change -> the variance."""
    flat_parent = np.concatenate([np.full(60, 0.5), [1.0, 1.0, 1.0, 1.0]])
    # constant child: sigma_c^2 = 0 -> alpha = 0 -> M = mu
    assert metric_value("eq5", np.full(8, 0.25), flat_parent) == pytest.approx(0.25)
    # parent variance -> 0 with a non-constant child: alpha -> 1 -> M -> sigma_c^2
    child = np.array([0.0, 1.0, 0.0, 1.0])
    par = np.concatenate([np.full(10000, 0.5), child])
    m = metric_value("eq5", child, par)
    assert m == pytest.approx(np.var(child), rel=1e-3)
    # variance equal to the parent's: M = mu exactly
    x = np.array([0.0, 1.0])
    assert metric_value("eq5", x, x) == pytest.approx(0.5)


def test_eq5_clamped_by_hand():
    """The clamped reading of Eq. (5) (alpha limited to [0, 1], Section III prose), on sets small enough to work
    out by hand.  alpha = (var_c - var_p) / var_c can never exceed 1 (variances are >= 0), so the upper bound
    never binds; these sets pin the lower bound, the unclamped interior and the normalisation by the parent's
    maximum, and fail if the clamp is dropped, swapped or applied to the wrong quantity."""
    # child variance below the parent's: literal alpha = -49.75, clamped to 0 -> M = mean
    parent = np.array([0.0, 2.0, 1.0, 1.2])            # max 2 -> normalised [0, 1, 0.5, 0.6], variance 0.126875
    child = np.array([1.0, 1.2])                       # normalised [0.5, 0.6]: mean 0.55, variance 0.0025
    assert metric_value("eq5_clamped", child, parent) == pytest.approx(0.55, rel=1e-14)
    # the literal Eq. (5) keeps alpha = -49.75: (1 + 49.75) * 0.55 - 49.75 * 0.0025
    assert metric_value("eq5", child, parent) == pytest.approx(50.75 * 0.55 - 49.75 * 0.0025, rel=1e-14)
    # child variance above the parent's: alpha = (0.25 - 0.125) / 0.25 = 0.5 inside [0, 1], both readings agree
    parent = np.array([0.0, 4.0, 2.0, 2.0])            # normalised [0, 1, 0.5, 0.5], variance 0.125
    child = np.array([0.0, 4.0])                       # normalised [0, 1]: mean 0.5, variance 0.25
    for name in ("eq5", "eq5_clamped"):
        assert metric_value(name, child, parent) == pytest.approx(0.5 * 0.5 + 0.5 * 0.25, rel=1e-14)
    # parent variance 1/8 of the child's: alpha = 7/8 -> M = mean / 8 + 7 variance / 8
    parent = np.array([0.0, 1.0] + [0.5] * 14)         # variance 0.5 / 16 = 0.03125 (max 1: no scaling)
    child = np.array([0.0, 1.0])                       # mean 0.5, variance 0.25
    sp = np.var(parent)
    assert sp == pytest.approx(0.03125, rel=1e-14)
    a = (0.25 - sp) / 0.25
    assert a == pytest.approx(0.875, rel=1e-14)
    for name in ("eq5", "eq5_clamped"):
        assert metric_value(name, child, parent) == pytest.approx((1 - a) * 0.5 + a * 0.25, rel=1e-14)
    # constant child: variance 0 -> alpha = 0 -> the mean, clamped or not
    for name in ("eq5", "eq5_clamped"):
        assert metric_value(name, np.full(3, 2.0), np.array([0.0, 2.0, 4.0])) == pytest.approx(0.5, rel=1e-14)


def test_eq5_scale_invariant():
    rng = np.random.default_rng(1)
    p = rng.uniform(0, 1, 64)
    assert metric_value("eq5", p[:16], p) == pytest.approx(metric_value("eq5", 7.5 * p[:16], 7.5 * p), rel=1e-12)


def test_within_between_by_hand():
    a = np.array([1.0, 3.0])          # mean 2
    b = np.array([6.0, 6.0, 9.0])     # mean 7
    w, bt = within_between(a, b)
    assert w == pytest.approx(2.0 + 6.0)                 # (1+1) + (1+1+4)
    pooled = 25.0 / 5
    assert bt == pytest.approx(2 * (2 - pooled) ** 2 + 3 * (7 - pooled) ** 2)


# ----------------------------------------------------------------------------------
# walks over synthetic energy images
# ----------------------------------------------------------------------------------

def _grid(n, dims3=False):
    p = 1e-3
    o = -(n - 1) * p / 2
    return Grid((o, o, o if dims3 else 0.0), (p, p, p), (n, n, n if dims3 else 1))


def _fake_scan(grid):
    return Scan(np.zeros((1, 3), np.float32), np.zeros((1, 2), np.float32), 1e-11, 0.0, 1e8, grid)


def _bump(b, w=3.0, bg=1.0):
    b = np.asarray(b, dtype=np.float64)

    def f(idx):
        d2 = np.sum((np.asarray(idx, np.float64) - b) ** 2, axis=1)
        return bg + 1.0 / (1.0 + d2 / (w * w))
    return f


def _morton_path(b, n, g, d):
    """Children containing b while the box side exceeds g."""
    path = []
    lo = [0, 0, 0]
    s = n
    while s > g:
        half = s // 2
        c = 0
        for bit in range(d):
            if b[bit] >= lo[bit] + half:
                c |= 1 << bit
                lo[bit] += half
        path.append(c)
        s = half
    return path


@pytest.mark.parametrize("metric", ["mean", "max"])
@pytest.mark.parametrize("dims3", [False, True])
def test_bump_follows_morton_path(metric, dims3):
    """A radially decreasing bump at odd coordinates is nearer its own lattice cell
    centre than any other, so MEAN and MAX must walk the Morton path of its voxel."""
    rng = np.random.default_rng(2 + dims3)
    n, g = (128, 8) if not dims3 else (64, 4)
    d = 3 if dims3 else 2
    for _ in range(5):
        b = 2 * rng.integers(0, n // 2, 3) + 1
        if not dims3:
            b[2] = 0
        r = oracle.walk(_fake_scan(_grid(n, dims3)), TreeParams(coarse=g, metric=metric), image_fn=_bump(b))
        assert r.child == _morton_path(b, n, g, d)
        lin = b[0] + n * (b[1] + n * b[2])
        assert r.argmax == lin


def test_voxels_evaluated_count():
    n, g = 512, 8
    r = oracle.walk(_fake_scan(_grid(n)), TreeParams(coarse=g, metric="max", frame_final=0.25),
                    image_fn=_bump((101, 301, 0)))
    levels = int(math.log2(n // g))
    roi = r.roi
    roi_vox = (roi[1] - roi[0]) * (roi[3] - roi[2]) * (roi[5] - roi[4])
    assert r.n_levels == levels == 6
    assert roi_vox == 12 * 12                    # side-8 box widened by floor(0.25 * 8) = 2 each side
    assert r.voxels_evaluated == levels * g * g + roi_vox


def test_exhaustive_depth2():
    """Every node of a depth-2 quadtree is scored independently; the walk must take the best child at each level."""
    n, g = 16, 4
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 1, (n, n))

    def image_fn(idx):
        return img[idx[:, 1], idx[:, 0]]

    def node_score(metric, x0, y0, s):
        step = s // g
        xs = [x for x in range(x0, x0 + s) if (x - x0) % step == step // 2]
        ys = [y for y in range(y0, y0 + s) if (y - y0) % step == step // 2]
        parent = np.array([img[y, x] for y in ys for x in xs])
        out = []
        for c in range(4):
            cx0 = x0 + (c & 1) * s // 2
            cy0 = y0 + (c >> 1) * s // 2
            vals = np.array([img[y, x] for y in ys for x in xs if cx0 <= x < cx0 + s // 2 and cy0 <= y < cy0 + s // 2])
            out.append(metric_value(metric, vals, parent))
        return out

    for metric in ["mean", "var", "eq5", "max", "max_over_mean"]:
        r = oracle.walk(_fake_scan(_grid(n)), TreeParams(coarse=g, metric=metric), image_fn=image_fn)
        s0 = node_score(metric, 0, 0, n)
        c0 = int(np.argmax(s0))
        x1, y1 = (c0 & 1) * n // 2, (c0 >> 1) * n // 2
        s1 = node_score(metric, x1, y1, n // 2)
        c1 = int(np.argmax(s1))
        assert r.child == [c0, c1], metric
        np.testing.assert_allclose(r.scores[0], s0, rtol=1e-14)
        np.testing.assert_allclose(r.scores[1], s1, rtol=1e-14)
        # enumerate all 16 depth-2 nodes: the greedy path is the best child of the best child
        best = [max(range(4), key=lambda c: node_score(metric, (a & 1) * n // 2, (a >> 1) * n // 2, n // 2)[c])
                for a in range(4)]
        assert best[c0] == c1


def _scripted(n, g, base, amp):
    """Level l returns base[l] + amp[l] * pattern; the pattern (+3 on child 0's quarter, -1 elsewhere) has mean 0."""
    calls = []

    def f(idx):
        lev = len(calls)
        calls.append(idx)
        if lev >= len(base):
            return np.zeros(idx.shape[0])
        x, y = idx[:, 0], idx[:, 1]
        kx = (x - x.min()) // max(1, (x.max() - x.min()) // (g - 1))
        ky = (y - y.min()) // max(1, (y.max() - y.min()) // (g - 1))
        pat = np.where((kx < g // 2) & (ky < g // 2), 3.0, -1.0)
        return base[lev] + amp[lev] * pat
    return f


def test_wb_stop_on_between_class():
    """B = 8, 32, 8 and W falling: iterations 1 and 2 proceed, iteration 3 stops and undoes its split."""
    n, g = 64, 4
    r = oracle.walk(_fake_scan(_grid(n)), TreeParams(coarse=g, metric="mean", term="wb"),
                    image_fn=_scripted(n, g, [0.0, 1.0, 3.0, 4.0], [2.0, 1.0, 0.5, 0.25]))
    bs = [b for _, b in r.wb]
    ws = [w for w, _ in r.wb]
    assert bs == pytest.approx([8.0, 32.0, 8.0])
    assert ws[1] < ws[0] and ws[2] < ws[1]
    assert r.term_level == 3 and r.n_levels == 2
    assert r.child == [0, 0, 0]
    assert r.boxes[r.n_levels] == (0, 16, 0, 16, 0, 1)


def test_wb_stop_on_within_class():
    """W grows at iteration 2 (spread rises) -> stop there, keep one split."""
    n, g = 64, 4
    r = oracle.walk(_fake_scan(_grid(n)), TreeParams(coarse=g, metric="mean", term="wb"),
                    image_fn=_scripted(n, g, [0.0, 1.0, 3.0, 6.0], [1.0, 1.0, 4.0, 0.25]))
    ws = [w for w, _ in r.wb]
    assert ws[1] > ws[0]
    assert r.term_level == 2 and r.n_levels == 1


def test_wb_runs_to_depth():
    n, g = 64, 4
    r = oracle.walk(_fake_scan(_grid(n)), TreeParams(coarse=g, metric="mean", term="wb"),
                    image_fn=_scripted(n, g, [0.0, 1.0, 3.0, 6.0, 10.0], [4.0, 2.0, 1.0, 0.5, 0.25]))
    assert r.n_levels == r.term_level == 4
    assert len(r.samples) == 5                # the last box is imaged to evaluate its W/B


def test_coarse_samples_are_full_resolution_values():
    """Hierarchy invariant: each coarse sample is the full-resolution image at that voxel (lattice placement)."""
    s = synth.c1_scan(4, noiseless=True, n_grid=64)
    r = oracle.walk(s, TreeParams(coarse=8, metric="max"))
    full = oracle.image_grid(s, 0)
    for idx, vals in r.samples:
        np.testing.assert_allclose(vals, full[idx[:, 2], idx[:, 1], idx[:, 0]], rtol=1e-12, atol=0)
    np.testing.assert_allclose(r.roi_image, full[:, r.roi[2]:r.roi[3], r.roi[0]:r.roi[1]], rtol=1e-12)


def test_frame_level_widens_scoring_only():
    n, g = 128, 8
    b = (61, 67, 0)     # near the centre: frames overlap neighbours
    f = _bump(b)
    a = oracle.walk(_fake_scan(_grid(n)), TreeParams(coarse=g, metric="mean", frame_level=0.0), image_fn=f)
    c = oracle.walk(_fake_scan(_grid(n)), TreeParams(coarse=g, metric="mean", frame_level=0.25), image_fn=f)
    assert all(bx[1] - bx[0] == n >> i for i, bx in enumerate(c.boxes))   # aligned boxes either way
    assert a.child == _morton_path(b, n, g, 2)
    assert c.child == a.child


# ----------------------------------------------------------------------------------
# the paper walk (one decimated image, splits reuse its samples)
# ----------------------------------------------------------------------------------

def test_paper_walk_decimated_lattice_and_stop():
    n = 100
    r = oracle.walk(_fake_scan(_grid(n)), TreeParams(walk="paper", decimation=7, metric="max", frame_level=0.0,
                                                     frame_final=0.0), image_fn=_bump((33, 71, 0)))
    idx, _ = r.samples[0]
    assert set(np.unique(idx[:, 0])) == set(range(3, 100, 7))
    assert r.decimation == 7
    # without frames each split halves the box; it stops once a child would hold < 4 lattice points
    for bx in r.boxes:
        assert bx[0] <= 33 < bx[1] and bx[2] <= 71 < bx[3]
    fb = r.boxes[r.n_levels]
    kids = [oracle.walk.__globals__["_split"](fb, c, (0, 1)) for c in range(4)]
    cnt = [int(np.count_nonzero(oracle.walk.__globals__["_inside"](idx, k))) for k in kids]
    assert min(cnt) < 4
    assert r.voxels_evaluated == idx.shape[0] + (fb[1] - fb[0]) * (fb[3] - fb[2])


def test_paper_walk_auto_decimation_from_pitch():
    g = Grid((0.0, 0.0, 0.0), (1e-3, 1e-3, 1e-3), (120, 120, 1))
    r = oracle.walk(_fake_scan(g), TreeParams(walk="paper", decimation=0, min_tumour=0.01, metric="max"),
                    image_fn=_bump((50, 50, 0)))
    assert r.decimation == 7


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("metric", ["mean", "max"])
def test_paper_walk_finds_tumour(seed, metric):
    """Physics: on noiseless single-tumour scans the framework's detection matches the full-resolution argmax."""
    s = synth.c1_scan(seed, noiseless=True)
    full_arg, _ = oracle.argmax_grid(oracle.image_grid(s, 0))
    r = oracle.walk(s, TreeParams(walk="paper", metric=metric, frame_level=0.25, min_tumour=0.01))
    nx = s.grid.dims[0]
    assert abs(r.argmax % nx - full_arg % nx) <= 1 and abs(r.argmax // nx - full_arg // nx) <= 1
    assert r.voxels_evaluated < s.grid.n_voxels


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("bf", [0, 1])
def test_per_level_walk_finds_tumour_c2(seed, bf):
    s = synth.c2_scan(seed, n_grid=256)
    full_arg, _ = oracle.argmax_grid(oracle.image_grid(s, bf))
    r = oracle.walk(s, TreeParams(beamformer=bf, coarse=8, metric="max"))
    nx = s.grid.dims[0]
    assert abs(r.argmax % nx - full_arg % nx) <= 1 and abs(r.argmax // nx - full_arg // nx) <= 1


def test_walk_rejects_bad_shapes():
    with pytest.raises(ValueError):
        oracle.walk(_fake_scan(_grid(100)), TreeParams(coarse=8))            # 100 is not 8 * 2^L
    with pytest.raises(ValueError):
        oracle.walk(_fake_scan(_grid(64)), TreeParams(coarse=8, metric="median"))


# ----------------------------------------------------------------------------------
# mixed-resolution composite (final imaging)
# ----------------------------------------------------------------------------------

def test_composite_decimation_one_is_the_full_image():
    s = synth.c1_scan(2, n_grid=32)
    p = oracle.TreeParams(beamformer=1, walk="paper", decimation=1, frame_final=0.25)
    res = oracle.walk(s, p)
    np.testing.assert_array_equal(composite(s, p, res), oracle.image_grid(s, 1))


@pytest.mark.parametrize("walk,kw", [("paper", dict(decimation=7)), ("per_level", dict(coarse=8))])
def test_composite_samples_roi_and_blocks(walk, kw):
    s = synth.c1_scan(5)
    p = oracle.TreeParams(beamformer=0, walk=walk, frame_final=0.25, **kw)
    res = oracle.walk(s, p)
    comp = composite(s, p, res)
    full = oracle.image_grid(s, 0)
    r = res.roi
    # inside the ROI: the full-resolution image
    np.testing.assert_array_equal(comp[:, r[2]:r[3], r[0]:r[1]], full[:, r[2]:r[3], r[0]:r[1]])
    # the finest samples outside the ROI carry their own energy
    idx, vals = res.samples[-1] if walk == "per_level" else res.samples[0]
    outside = ~((idx[:, 0] >= r[0]) & (idx[:, 0] < r[1]) & (idx[:, 1] >= r[2]) & (idx[:, 1] < r[3]))
    assert outside.sum() > 0
    np.testing.assert_array_equal(comp[idx[outside, 2], idx[outside, 1], idx[outside, 0]],
                                  full[idx[outside, 2], idx[outside, 1], idx[outside, 0]])
    # only the ROI varies at full resolution: outside it, at most one value per sample
    mask = np.ones(comp.shape, bool)
    mask[:, r[2]:r[3], r[0]:r[1]] = False
    n_samples = sum(len(v) for _, v in res.samples)
    assert len(np.unique(comp[mask])) <= n_samples


# ----------------------------------------------------------------------------------
# the two-decimation check (no-tumour test)
# ----------------------------------------------------------------------------------

def test_rois_intersect_by_hand():
    from oracle.walk import rois_intersect
    assert rois_intersect((0, 10, 0, 10, 0, 1), (9, 20, 5, 6, 0, 1))
    assert not rois_intersect((0, 10, 0, 10, 0, 1), (10, 20, 0, 10, 0, 1))    # touching is not sharing
    assert not rois_intersect((0, 10, 0, 10, 0, 1), (0, 10, 10, 12, 0, 1))
    assert not rois_intersect((0, 4, 0, 4, 0, 2), (0, 4, 0, 4, 2, 3))


def _landscape(spike, bump, n):
    """Energy: a broad bump at `bump` (peak 1) plus a one-voxel spike of 10 at `spike`."""
    def fn(idx):
        idx = np.asarray(idx, dtype=np.float64)
        d2 = (idx[:, 0] - bump[0]) ** 2 + (idx[:, 1] - bump[1]) ** 2
        v = np.exp(-d2 / (2 * (n / 8.0) ** 2))
        hit = (idx[:, 0] == spike[0]) & (idx[:, 1] == spike[1])
        return v + 10.0 * hit
    return fn


def test_tumour_check_on_constructed_landscapes():
    from oracle.walk import tumour_check
    s = synth.c1_scan(0, n_grid=128)
    p = TreeParams(walk="paper", metric="max", frame_final=0.1)
    # the spike sits on the D = 7 lattice (7 k + 3) but on no D = 5 lattice point (5 k + 2): the D = 7 walk
    # goes to the spike, the D = 5 walk to the bump far away -> the ROIs differ: artifacts
    spike, bump = (7 * 3 + 3, 7 * 3 + 3), (100, 100)
    assert (spike[0] - 2) % 5 != 0
    agree, r1, r2 = tumour_check(s, p, 7, 5, image_fn=_landscape(spike, bump, 128))
    assert r1.roi[0] <= spike[0] < r1.roi[1] and r2.roi[0] <= bump[0] < r2.roi[1]
    assert not agree
    # a broad bump alone: both walks find it -> confirmed
    agree, r1, r2 = tumour_check(s, p, 7, 5, image_fn=_landscape((-50, -50), bump, 128))
    assert agree
    with pytest.raises(ValueError):
        tumour_check(s, p, 5, 5)


def test_tumour_check_confirms_a_real_scatterer():
    from oracle.walk import tumour_check
    s = synth.c1_scan(3, noiseless=True)
    agree, r1, r2 = tumour_check(s, TreeParams(beamformer=1, walk="paper", metric="max", frame_final=0.25), 9, 5)
    assert agree
