"""The binding refuses caller buffers that are too small for the call before anything is enqueued: the library
takes raw device pointers, so a short output would be written past its end (and a short input read past it)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402


def uwb():
    import paper_1709_02549_amd as m
    return m


def _scan():
    return synth.c1_scan(0, n_grid=32)


def test_short_images_are_refused():
    u = uwb()
    s = _scan()
    ds = u.DeviceScan.from_host(s)
    n = 32 * 32
    short = torch.full((n - 1,), -3.0, device="cuda")
    for call in (lambda: u.image(ds, s.grid, 0, out=short), lambda: u.image(ds, s.grid, 1, out=short),
                 lambda: u.das_dmas(ds, s.grid, out_das=short),
                 lambda: u.das_dmas(ds, s.grid, out_dmas=short)):
        with pytest.raises(ValueError):
            call()
    torch.cuda.synchronize()
    assert bool(torch.all(short == -3.0))          # nothing was written


def test_short_batch_buffers_are_refused():
    u = uwb()
    scans = [_scan() for _ in range(3)]
    b = u.DeviceBatch.from_host(scans)
    g = scans[0].grid
    short = torch.full((3 * 32 * 32 - 1,), -3.0, device="cuda")
    with pytest.raises(ValueError):
        u.image_batch(b, g, 1, out=short)
    with pytest.raises(ValueError):
        u.das_dmas_batch(b, g, out_das=short)
    img = u.image_batch(b, g, 1)
    with pytest.raises(ValueError):                 # image shorter than the batch
        u.argmax_batch_async(b, g, img[:2], 1)
    with pytest.raises(ValueError):                 # records for two of three scans
        u.argmax_batch_async(b, g, img, 1, out=torch.empty(2 * ctypes.sizeof(u.UwbPeak), dtype=torch.uint8,
                                                            device="cuda"))
    tree = u.SegmentTree(beamformer=1, coarse=8)
    with pytest.raises(ValueError):
        u.segment_refine_batch_async(b, g, tree, out=torch.empty(ctypes.sizeof(u.UwbSegmentResult) * 2,
                                                                 dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError):
        u.segment_refine_batch_async(b, g, tree, workspace=torch.empty(64, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    assert bool(torch.all(short == -3.0))


def test_mis_shaped_scans_and_plan_outputs_are_refused():
    u = uwb()
    s = _scan()
    ds = u.DeviceScan.from_host(s)
    bad = u.DeviceScan(ds.ant_pos[:-1], ds.traces, ds.dt, ds.t0, ds.v)    # fewer positions than traces
    with pytest.raises(ValueError):
        u.image(bad, s.grid, 0)
    with pytest.raises(ValueError):
        u.BatchPlan([(ds, s.grid, torch.empty(32 * 32 - 1, device="cuda"))], 0)
    net = u.CNN(4, np.zeros(u.lib().uwb_cnn_param_count(), np.float32))
    x = torch.zeros((2, 32, 32), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(ValueError):
        net.forward(x, probs=torch.empty(7, device="cuda"))
    with pytest.raises(ValueError):
        net.gradients(x, torch.zeros(1, dtype=torch.int32, device="cuda"))
    net.close()
