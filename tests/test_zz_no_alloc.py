"""The allocation-free detection (uwb_argmax_batch_noalloc) against the workspace form (uwb_argmax_batch) and
the oracle: two calls in a row through the C ABI, the second on a smaller input, so the library's shared
scratch holds the first call's records when the second starts.  Records must be bit-identical to the
workspace form's (same kernels, same inputs), and the detections equal to the oracle's FP64 argmax."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402


def _case(scans, bf):
    import paper_1709_02549_amd as u
    grid = scans[0].grid
    b = u.DeviceBatch.from_host(scans)
    bc = b.c()
    img = u.image_batch(b, grid, bf, bc=bc)
    n = len(scans)
    sz = ctypes.sizeof(u.UwbPeak)
    out = torch.full((sz * n,), 0xAB, dtype=torch.uint8, device="cuda")     # allocated before the call
    ref = u.argmax_batch_async(b, grid, img, bf)
    u.argmax_batch_noalloc_async(b, grid, img, bf, out, bc=bc)
    torch.cuda.synchronize()
    assert torch.equal(out, ref[:sz * n]), "records differ from uwb_argmax_batch"
    got = u._peaks(out, n)
    for k, s in enumerate(scans):
        a, v = oracle.argmax_grid(oracle.image_grid(s, bf))
        assert got[k].index == a, (k, got[k].index, a)
        assert got[k].value == pytest.approx(v, rel=1e-12)
        assert got[k].candidates >= 1
    return got


def test_noalloc_two_calls_second_smaller():
    # first call: 6 scans of 128 x 128 (4 chunks each), DMAS
    first = [synth.c1_scan(k) for k in range(6)]
    _case(first, 1)
    # second call: 3 scans of 48 x 48 (one ragged chunk each), DAS; the scratch still holds the first call's records
    second = [synth.c1_scan(10 + k, n_grid=48) for k in range(3)]
    _case(second, 0)


def test_noalloc_refuses_oversize_before_launch():
    import paper_1709_02549_amd as u
    scans = [synth.c1_scan(0, n_grid=16)] * 2
    b = u.DeviceBatch.from_host(scans)
    big = synth.Grid((-0.05, -0.05, 0.0), (1e-5, 1e-5, 1e-3), (8192, 8192, 1))   # 16384 chunks per scan
    out = torch.zeros(ctypes.sizeof(u.UwbPeak) * 2, dtype=torch.uint8, device="cuda")
    img = torch.zeros(1, dtype=torch.float32, device="cuda")
    bc, gc = b.c(), u.grid_c(big)
    rc = u.lib().uwb_argmax_batch_noalloc(ctypes.byref(bc), ctypes.byref(gc), 11, 0, img.data_ptr(),
                                          out.data_ptr(), u._stream())
    assert rc == u._abi.UWB_ERANGE
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
