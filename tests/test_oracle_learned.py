"""Pins of the learned-walk oracle: reductions to the metric walk, a constant network, path geometry by
brute force, and agreement of its training inputs with the walk's own lattices."""
import numpy as np
import pytest

import oracle
from oracle import cnn, learned
from oracle.walk import TreeParams
from synth import scans


def _scan(seed=3, n=128):
    return scans.c1_scan(seed, n_grid=n)


def _tree(**kw):
    base = dict(beamformer=1, walk="per_level", coarse=32, metric="max", term="fixed", frame_final=0.25)
    base.update(kw)
    return TreeParams(**base)


def _constant_net(bias=0.5):
    """All convolution weights zero: every activation is relu(bias), so the four children look alike."""
    p = cnn.Params.init(0)
    p.w = [np.zeros_like(w) for w in p.w]
    p.b = [np.full(cnn.CH, bias) for _ in range(4)]
    return p


@pytest.mark.parametrize("metric", ["max", "mean", "eq5_clamped"])
def test_untrusted_network_is_the_metric_walk(metric):
    """Levels look at the DAS lattice; with DAS everywhere the walk is oracle.walk exactly."""
    s = _scan()
    t = _tree(metric=metric, beamformer=0)
    ref = oracle.walk(s, t)
    got = learned.learned_walk(s, t, cnn.Params.init(1), threshold=1.5)
    assert got.learned_mask == 0
    assert got.child == ref.child == got.fallback
    assert got.boxes == ref.boxes
    np.testing.assert_array_equal(np.array(got.scores), np.array(ref.scores))
    assert got.roi == ref.roi and got.argmax == ref.argmax and got.peak == ref.peak
    assert got.voxels_evaluated == ref.voxels_evaluated


def test_dmas_roi_after_das_levels():
    s = _scan(4)
    ref = oracle.walk(s, _tree(beamformer=0))
    got = learned.learned_walk(s, _tree(beamformer=1), cnn.Params.init(1), threshold=1.5)
    assert got.boxes == ref.boxes and got.roi == ref.roi
    img = oracle.image_grid(s, oracle.DMAS)
    x0, x1, y0, y1, _, _ = got.roi
    sub = np.full(img.shape, -np.inf)
    sub[:, y0:y1, x0:x1] = img[:, y0:y1, x0:x1]
    assert (got.argmax, got.peak) == oracle.argmax_grid(sub)


def test_constant_network_is_uniform_and_takes_child_zero():
    s = _scan(5)
    t = _tree()
    net = _constant_net()
    got = learned.learned_walk(s, t, net, threshold=0.25)
    for p in got.probs:
        np.testing.assert_allclose(p, 0.25, rtol=0, atol=1e-15)
    assert got.learned_mask == 0b11 and got.child == [0, 0]
    assert got.boxes == [(0, 128, 0, 128, 0, 1), (0, 64, 0, 64, 0, 1), (0, 32, 0, 32, 0, 1)]
    assert got.roi == (0, 40, 0, 40, 0, 1)
    # just above a quarter nothing is trusted: the metric walk again
    ref = oracle.walk(s, _tree(beamformer=0))
    got2 = learned.learned_walk(s, t, net, threshold=0.25 + 1e-9)
    assert got2.learned_mask == 0 and got2.child == ref.child


def test_cnn_input_is_normalised():
    v = np.arange(1024, dtype=np.float64)
    x = learned.cnn_input(v)
    assert x.shape == (32, 32) and x.max() == 1.0 and x[0, 1] == 1.0 / 1023.0
    np.testing.assert_array_equal(learned.cnn_input(np.zeros(1024)), 0.0)


@pytest.mark.parametrize("n,depth", [(128, 2), (256, 3), (512, 4)])
def test_path_boxes_brute_force(n, depth):
    rng = np.random.default_rng(n)
    for target in list(rng.integers(0, n * n, 20)) + [0, n - 1, n * n - 1, n * (n - 1)]:
        tx, ty = int(target) % n, int(target) // n
        path = learned.path_boxes(int(target), (n, n, 1), depth)
        assert len(path) == depth
        for lev, (box, lab) in enumerate(path):
            side = n >> lev
            # the one aligned box of this side that holds the target, found by enumeration
            found = [(x0, x0 + side, y0, y0 + side, 0, 1) for x0 in range(0, n, side) for y0 in range(0, n, side)
                     if x0 <= tx < x0 + side and y0 <= ty < y0 + side]
            assert found == [box]
            # the label's child holds the target; the other three do not
            for c in range(4):
                cx0 = box[0] + (c & 1) * side // 2
                cy0 = box[2] + (c >> 1) * side // 2
                inside = cx0 <= tx < cx0 + side // 2 and cy0 <= ty < cy0 + side // 2
                assert inside == (c == lab)


def test_training_inputs_follow_the_walk_lattices():
    """On a clean point scatterer the DAS max-metric walk descends onto the detection, so its per-level lattices
    are exactly the boxes on the detection's path."""
    g = scans.square_grid(128)
    ant = scans.ring_antennas(16)
    pt = np.array([[0.0123, -0.0217, 0.0]])
    s = scans.point_scan(ant, g, pt, [1.0], 1024, scans.C0 / 3.0)
    t = _tree(beamformer=0)
    ref = oracle.walk(s, t)
    x, lab = learned.training_inputs(s, ref.argmax)
    assert x.shape == (2, 32, 32) and list(lab) == ref.child
    for lev in range(2):
        idx, vals = ref.samples[lev]
        np.testing.assert_array_equal(x[lev].ravel(), vals / vals.max())


def test_walk_rejects_other_shapes():
    s = _scan()
    with pytest.raises(ValueError):
        learned.learned_walk(s, _tree(coarse=16), cnn.Params.init(0), 0.5)
    with pytest.raises(ValueError):
        learned.learned_walk(s, _tree(term="wb"), cnn.Params.init(0), 0.5)
    with pytest.raises(ValueError):
        learned.learned_walk(scans.c1_scan(1, n_grid=96), _tree(), cnn.Params.init(0), 0.5)
