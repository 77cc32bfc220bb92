"""The imaging, detection and walk entry points launch kernels only (no memsets, no host synchronisation), so a
caller can capture them in a HIP graph.  Every replay must reproduce the eager results bit for bit (the kernels
are deterministic), also with the program's own eager work and synchronisations between the replays."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402


def uwb():
    import paper_1709_02549_amd as m
    return m


def test_step_graph_replays_match_eager():
    u = uwb()
    scans = [synth.c1_scan(k) for k in range(6)]
    grid = scans[0].grid
    nx, ny, nz = grid.dims
    B = len(scans)
    batch = u.DeviceBatch.from_host(scans)
    bc = batch.c()
    trees = {bf: u.SegmentTree(beamformer=bf, coarse=8, metric="max", frame_final=0.25) for bf in (0, 1)}
    paper = u.SegmentTree(beamformer=1, walk="paper", min_tumour=0.01, metric="max", frame_final=0.25)
    imgs = {bf: torch.empty((B, nz, ny, nx), dtype=torch.float32, device="cuda") for bf in (0, 1)}
    peaks = {bf: torch.empty(24 * B, dtype=torch.uint8, device="cuda") for bf in (0, 1)}
    import ctypes
    ws_arg = torch.empty(int(u.lib().uwb_argmax_workspace_bytes(ctypes.byref(u.grid_c(grid)), B)), dtype=torch.uint8,
                         device="cuda")
    outs, wss = {}, {}
    for key, tree in [(0, trees[0]), (1, trees[1]), ("paper", paper)]:
        out, _ = u.segment_refine_batch_async(batch, grid, tree, 11, bc=bc)
        outs[key] = out
        need = u.lib().uwb_segment_workspace_bytes(ctypes.byref(u.grid_c(grid)), ctypes.byref(tree.c()), B)
        wss[key] = torch.empty(need, dtype=torch.uint8, device="cuda")

    def step():
        for bf in (0, 1):
            u.image_batch(batch, grid, bf, 11, imgs[bf], bc=bc)
            u.argmax_batch_async(batch, grid, imgs[bf], bf, 11, peaks[bf], ws_arg, bc=bc)
        for key, tree in [(0, trees[0]), (1, trees[1]), ("paper", paper)]:
            u.segment_refine_batch_async(batch, grid, tree, 11, out=outs[key], workspace=wss[key], bc=bc)

    def snapshot():
        torch.cuda.synchronize()
        return ([imgs[bf].cpu().numpy().copy() for bf in (0, 1)] + [peaks[bf].cpu().numpy().copy() for bf in (0, 1)]
                + [outs[k].cpu().numpy().copy() for k in (0, 1, "paper")])

    def clear():   # result records have fields a walk leaves unwritten (levels below its depth)
        for x in list(imgs.values()) + list(peaks.values()) + list(outs.values()):
            x.zero_()

    clear()
    step()
    eager = snapshot()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(3):
        clear()                             # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        got = snapshot()
        for a, b in zip(got, eager):
            assert np.array_equal(a, b), f"replay {rep} differs from the eager run"
