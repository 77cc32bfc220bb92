"""Benchmark of the DAS / DMAS hot path on one MI355X.

Workload (the 2D hierarchical-segmentation configuration): B distinct synthetic
scans, each 32 antennas on a 7 cm ring, 2048 fp32 samples at 50 GS/s, one tumour
plus 200 clutter scatterers, 20 dB SNR, imaged on a 512 x 512 finest grid.  One
step processes the whole batch, inputs already resident in HBM:
  full-resolution DAS and DMAS images (one gather feeds both)  -> FP64-decided
  argmax of each; coarse-to-fine quadtree walks (g = 16 down to 16 x 16 boxes,
  metric = max) with DAS and with DMAS, each ending in a full-resolution ROI and
  its argmax.  The two argmaxes and the two walks are independent of each other
  and run at once on four streams after the imaging launch.
value = full-resolution voxel*antenna pairs per second over the whole step (walks
and argmax included in the time), each pair counted once although it feeds both
the DAS and the DMAS image.

Outside the timed steps: the same step's parts as separate launches; the 2D
single-scan configuration (16 antennas, 128 x 128) as latency; the 3D
configuration (64 antennas on a hemisphere, 4096 samples, 256^3 voxels) as
full-resolution throughput and octree walks against full-resolution DMAS; the
batched uneven-scan plan; the multistatic ring; the learned proposer trained on
GPU-generated scans and compared with the metric walks and full-resolution DMAS;
the device's LDS read bandwidth; and the FP64 oracle timed on the host.

Prints one JSON line (progress goes to stderr).  Only N = 1 GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 work per voxel*antenna with a W-sample window (counted from the operations the
# method prescribes, not from the kernel's instruction mix):
#   delay 11 flops (3 sub, 3 mul, 2 add, sqrt, scale, offset)
#   per window offset: interpolation 3 flops; DAS +1 add; DMAS +3 (product, sum, prefix)
FLOPS_DELAY = 11


def flops_per_va(bf: int, window: int) -> int:
    return FLOPS_DELAY + window * (4 if bf == 0 else 6)


# MI355X vector FP32: 256 CU x 4 SIMD x 32 FP32 lanes per clock x 2 flop (FMA) x 2.4 GHz
PEAK_FP32 = 157.3e12

# HBM bytes per launch of the step's imaging kernel (DMAS writing the DAS image too) at the default
# batch, from two rocprofv3 --pmc runs
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0, factors from a 256 MiB copy); valid only for the kernel
# sources they were taken on (profiles/k_image32_c2_batch256_pmc.md).
TRAFFIC = {"source_hash": "b83de0123ea7e0ee", "batch": 256, "bytes": 640500000,
           "valu_per_va": 44.84}   # SQ_INSTS_VALU per voxel·antenna (64-lane wave slot) of that launch
# LDS bytes the DMAS kernel reads per lane and voxel·antenna at W = 11: the 11 taps' (sample, difference)
# pairs as five 16-byte reads and one 8-byte read (the channel's table entry, read once per four voxels at
# one address for the whole wavefront, is not counted)
LDS_BYTES_DMAS = 88
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 2   # wave64 FP32 VALU instructions/s (two cycles each)


def _kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("image32.h", "image32.hip"):
        with open(os.path.join(ROOT, "paper_1709_02549_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--distinct", type=int, default=0, help="distinct seeded scans in the batch (0: all)")
    ap.add_argument("--coarse", type=int, default=16, help="walk lattice points per side (g)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--c5-train", type=int, default=200_000, help="training scans of the learned proposer")
    ap.add_argument("--c5-eval", type=int, default=10_000, help="held-out scans for its localisation error")
    ap.add_argument("--c5-epochs", type=float, default=1.0)
    ap.add_argument("--no-c5", action="store_true", help="skip training / evaluating the learned proposer")
    ap.add_argument("--c4-scans", type=int, default=1024, help="uneven scans of the batched-serving plan")
    ap.add_argument("--no-c4", action="store_true", help="skip the batched-serving measurement")
    ap.add_argument("--ms-batch", type=int, default=512, help="multistatic scans (12-antenna ring, 200x200 grid)")
    ap.add_argument("--no-ms", action="store_true", help="skip the multistatic and no-tumour-check measurements")
    ap.add_argument("--c3-scans", type=int, default=32, help="3D scans for the octree walks against full DMAS")
    ap.add_argument("--no-c3", action="store_true", help="skip the 3D (256^3) measurements")
    ap.add_argument("--no-c1", action="store_true", help="skip the single-scan latency measurements")
    ap.add_argument("--mvdr-scans", type=int, default=64, help="2D scans of the Capon (MVDR) block")
    ap.add_argument("--no-mvdr", action="store_true", help="skip the Capon (MVDR) measurements")
    ap.add_argument("--no-separate", action="store_true",
                    help="skip timing the DAS and DMAS kernels as separate launches (profiling runs)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="before timing, run one plain device copy of this many MiB (HBM counter reference)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only (--gpus 1); multi-GPU sharding is not implemented",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1709_02549_amd as uwb
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    B, W = args.batch, 11
    t_gen = time.time()
    distinct = [synth.c2_scan(k) for k in range(min(args.distinct, B) if args.distinct > 0 else B)]
    scans = [distinct[k % len(distinct)] for k in range(B)]
    gen_s = time.time() - t_gen
    grid = scans[0].grid
    nx, ny, nz = grid.dims
    M = scans[0].n_ant
    batch = uwb.DeviceBatch.from_host(scans, dev)
    bc = batch.c()
    img_das = torch.empty((B, nz, ny, nx), dtype=torch.float32, device=dev)
    img_dmas = torch.empty_like(img_das)
    pk_das = torch.empty(24 * B, dtype=torch.uint8, device=dev)
    pk_dmas = torch.empty_like(pk_das)
    # the imaging launch writes every tile's maximum of both images; the detections read those instead of
    # making a pass of their own over the images
    n_tiles = uwb.image_tiles(grid)
    tm_das = torch.empty((B, n_tiles), dtype=torch.float32, device=dev)
    tm_dmas = torch.empty_like(tm_das)
    trees = {bf: uwb.SegmentTree(beamformer=bf, coarse=args.coarse, metric="max", frame_final=0.25) for bf in (0, 1)}
    walk_out = {}
    ws_argmax = {bf: torch.empty(int(uwb.lib().uwb_argmax_tilemax_workspace_bytes(
        __import__("ctypes").byref(uwb.grid_c(grid)), B)), dtype=torch.uint8, device=dev) for bf in (0, 1)}
    # the DAS and DMAS detections and the two walks are independent of each other and latency-bound: after
    # the imaging launch the four run at once on four streams (default priority), forked from and joined to
    # the main stream -- the DAS detection on main, the DMAS one on `side`, the walks on `walk_s`
    side = torch.cuda.Stream(device=dev)
    walk_s = {bf: torch.cuda.Stream(device=dev) for bf in (0, 1)}
    ws_walk = {bf: uwb.Workspace() for bf in (0, 1)}
    walk_bufs = {}
    for bf in (0, 1):
        gc, tc = uwb.grid_c(grid), trees[bf].c()
        import ctypes
        need = uwb.lib().uwb_segment_workspace_bytes(ctypes.byref(gc), ctypes.byref(tc), B)
        walk_bufs[bf] = (torch.empty(ctypes.sizeof(uwb.UwbSegmentResult) * B, dtype=torch.uint8, device=dev),
                         torch.empty(need, dtype=torch.uint8, device=dev))

    # one pair of events per component and timed step, read back after the last step: the steps run back to
    # back, with no host synchronisation between them
    ev = {k: [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
          for k in ("img", "arg", "walk")}
    times = {k: [] for k in ev}
    cur = [0]

    def step(record: bool):
        def mark(k, i):
            if record:
                ev[k][cur[0]][i].record()
        # both full-resolution images from one launch (the DMAS kernel's running sums are the DAS sums),
        # with every tile's maximum of each
        mark("img", 0)
        uwb.das_dmas_batch_tilemax(batch, grid, W, img_das, img_dmas, tm_das, tm_dmas, bc=bc)
        mark("img", 1)
        main = torch.cuda.current_stream(dev)
        mark("arg", 0)
        mark("walk", 0)
        for st in (side, walk_s[0], walk_s[1]):
            st.wait_stream(main)
        for bf in (1, 0):
            out, ws = walk_bufs[bf]
            with torch.cuda.stream(walk_s[bf]):
                uwb.segment_refine_batch_async(batch, grid, trees[bf], W, out=out, workspace=ws, bc=bc)
        with torch.cuda.stream(side):
            uwb.argmax_batch_tilemax_async(batch, grid, img_dmas, tm_dmas, 1, W, pk_dmas, ws_argmax[1], bc=bc)
        uwb.argmax_batch_tilemax_async(batch, grid, img_das, tm_das, 0, W, pk_das, ws_argmax[0], bc=bc)
        main.wait_stream(side)
        mark("arg", 1)
        main.wait_stream(walk_s[0])
        main.wait_stream(walk_s[1])
        mark("walk", 1)   # from the fork: the detections and the walks together

    if args.copy_ref_mib > 0:
        src = torch.ones(args.copy_ref_mib * 262144, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        cur[0] = i
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in ev:
        times[k] = [e0.elapsed_time(e1) for e0, e1 in ev[k]]
    ms_step = (t1 - t0) * 1e3 / args.steps
    va = B * nx * ny * nz * M
    # Gvoxel*antenna/s over the whole step; each pair is counted once, although its gathered samples feed both
    # the DAS and the DMAS image
    value = va / (ms_step * 1e-3) / 1e9

    med = {k: float(np.median(v)) for k, v in times.items()}

    # the two beamformers as separate launches (after the timed steps), for their own rates
    def launch_ms(fn, reps=51):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    sep = {}
    if not args.no_separate:
        sep["das"] = launch_ms(lambda: uwb.image_batch(batch, grid, 0, W, img_das, bc=bc))
        sep["dmas"] = launch_ms(lambda: uwb.image_batch(batch, grid, 1, W, img_dmas, bc=bc))
    dmas_ms = sep.get("dmas", med["img"])

    # each walk on its own (the step runs both walks and both detections at once, each on a stream of its own)
    def walk_once(bf):
        out, ws = walk_bufs[bf]
        uwb.segment_refine_batch_async(batch, grid, trees[bf], W, out=out, workspace=ws, bc=bc)

    walk_alone = {bf: launch_ms(lambda bf=bf: walk_once(bf)) for bf in (0, 1)}
    arg_alone = {bf: launch_ms(lambda bf=bf: uwb.argmax_batch_tilemax_async(
        batch, grid, img_dmas if bf else img_das, tm_dmas if bf else tm_das, bf, W, pk_dmas if bf else pk_das,
        ws_argmax[bf], bc=bc)) for bf in (0, 1)}
    # the same detection making its own pass over the image (uwb_argmax_batch), for comparison
    arg_pass = launch_ms(lambda: uwb.argmax_batch_async(batch, grid, img_dmas, 1, W, bc=bc))
    # the last launches above leave the step's detections and walk results in place for the accuracy checks

    # the two walks of a step are launch-bound at this batch (about a dozen small kernels each): the
    # same calls replayed as one HIP graph (kernels only: no memsets, no host synchronisation)
    wg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(wg):
        cap = torch.cuda.current_stream(dev)       # the two walks forked onto two streams
        side.wait_stream(cap)
        for bf in (1, 0):
            out, ws = walk_bufs[bf]
            with torch.cuda.stream(side if bf == 1 else cap):
                uwb.segment_refine_batch_async(batch, grid, trees[bf], W, out=out, workspace=ws, bc=bc)
        cap.wait_stream(side)
    wg.replay()
    torch.cuda.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record()
    for _ in range(20):
        wg.replay()
    g1.record()
    torch.cuda.synchronize()
    walk_graph_ms = g0.elapsed_time(g1) / 20

    # accuracy of the walks against the full-resolution DMAS detection (outside the timed region)
    full = uwb._peaks(pk_dmas, B)
    res = {bf: uwb._results(walk_bufs[bf][0], B, 4) for bf in (0, 1)}

    def within1(a, b):
        return abs(a % nx - b % nx) <= 1 and abs(a // nx - b // nx) <= 1

    loc = {bf: float(np.mean([within1(r.argmax, f.index) for r, f in zip(res[bf], full)])) for bf in (0, 1)}
    full_das = uwb._peaks(pk_das, B)
    das_vs_dmas = float(np.mean([within1(a.index, b.index) for a, b in zip(full_das, full)]))
    hier_vox = float(np.mean([r.voxels_evaluated for r in res[1]]))

    # the timed launch: DMAS plus the DAS energy of its running sums (2 W flops per voxel)
    fpva = flops_per_va(1, W) + 2.0 * W / M
    achieved = fpva * va / (med["img"] * 1e-3)
    counters_valid = TRAFFIC["source_hash"] == _kernel_source_hash()
    va_rate = va / (med["img"] * 1e-3)             # voxel·antenna/s of the launch
    lds = lds_peak(uwb)
    traffic = TRAFFIC["bytes"] if (TRAFFIC["source_hash"] == _kernel_source_hash() and B == TRAFFIC["batch"]) \
        else None
    out = {
        "metric": "DAS/DMAS Gvoxel·antenna/s; scans/s hierarchical vs full at equal loc. error",
        "value": round(value, 2),
        "unit": "Gvoxel·antenna/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D monostatic ring, 32 antennas x 2048 samples, 512x512 grid, window 11, "
                               f"full-res DAS+DMAS (one launch, tile maxima) + FP64-decided detection of each + "
                               f"quadtree walks (g={args.coarse}, max metric)",
                   "batch_scans": B, "distinct_scans": len(distinct), "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "k_image32 DMAS writing DAS too (W=11, 2D)",
                     "achieved": round(achieved / 1e12, 3), "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32, 4), "traffic": traffic,
                     "flops_per_voxel_antenna": round(fpva, 2),
                     "avg_launch_ms": round(med["img"], 5),
                     "hbm_gbs": round(traffic / (med["img"] * 1e-3) / 1e9, 1) if traffic else None,
                     "hbm_frac": round(traffic / (med["img"] * 1e-3) / 8e12, 4) if traffic else None,
                     # the gather's other on-chip bounds: LDS reads against the LDS read bandwidth measured on
                     # this device -- the kernel reads W + 1 = 12 samples (48 B) of algorithmic data per
                     # voxel·antenna, as eleven 8-byte (sample, difference) pairs (88 B) -- and VALU
                     # issue (counted instructions, while the sources match the counters)
                     "lds_bytes_per_voxel_antenna": LDS_BYTES_DMAS,
                     "lds_frac": round(va_rate * LDS_BYTES_DMAS / lds["bytes_per_s"], 4),
                     "lds_frac_algorithmic_48B": round(va_rate * 48 / lds["bytes_per_s"], 4),
                     "valu_issue_frac": round(va_rate * TRAFFIC["valu_per_va"] / 64 / VALU_ISSUE_PEAK, 4)
                     if counters_valid else None},
        "value_counts": "each full-resolution voxel·antenna once; one gather feeds both the DAS and the DMAS image",
        # per step (medians): the imaging launch; then, from the fork after it, the two detections done, and the
        # two detections and the two walks done (the four run at once on four streams)
        "components_ms": {"img": round(med["img"], 5), "detections": round(med["arg"], 5),
                          "detections_and_walks": round(med["walk"], 5)},
        "detection_ms": {"dmas_from_tile_maxima": round(arg_alone[1], 5), "das_from_tile_maxima": round(arg_alone[0], 5),
                         "dmas_with_its_own_image_pass": round(arg_pass, 5)},
        "das_dmas_one_launch_gvas_per_image": round(va / (med["img"] * 1e-3) / 1e9, 2),
        "das_dmas_one_launch_gvas_two_image_sum": round(2 * va / (med["img"] * 1e-3) / 1e9, 2),
        "separate_launch_ms": {k: round(v, 5) for k, v in sep.items()},
        "das_gvas": round(va / (sep["das"] * 1e-3) / 1e9, 2) if sep else None,
        "dmas_gvas": round(va / (sep["dmas"] * 1e-3) / 1e9, 2) if sep else None,
        "lds_read_peak": lds,
        "hierarchical": {
            # one walk per scan: the DMAS walk timed on its own
            "dmas_walk_scans_per_s": round(B / (walk_alone[1] * 1e-3), 1),
            "das_walk_scans_per_s": round(B / (walk_alone[0] * 1e-3), 1),
            "walk_ms": {"dmas": round(walk_alone[1], 5), "das": round(walk_alone[0], 5),
                        "both_on_two_streams_hip_graph": round(walk_graph_ms, 5)},
            # full-resolution DMAS imaging plus its detection, timed on their own
            "full_dmas_scans_per_s": round(B / ((dmas_ms + arg_alone[1]) * 1e-3), 1),
            "dmas_walk_within_1_voxel_of_full_dmas": loc[1],
            "das_walk_within_1_voxel_of_full_dmas": loc[0],
            "full_das_within_1_voxel_of_full_dmas": das_vs_dmas,
            # reported only when the walk's localisation matches full DMAS on every scan of the batch
            "dmas_walk_speedup_vs_full_dmas_at_equal_error":
                round((dmas_ms + arg_alone[1]) / walk_alone[1], 2) if loc[1] >= 1.0 else None,
            "voxels_per_walk": hier_vox,
            "voxel_ratio_full_over_walk": round(nx * ny / hier_vox, 1),
        },
        "input_generation_s": round(gen_s, 2),
    }
    if not args.no_mvdr:
        out["mvdr"] = mvdr_block(args, uwb, synth, dev)
    if not args.no_c1:
        out["c1_latency"] = c1_block(uwb, synth, dev)
    if not args.no_c3:
        out["c3"] = c3_block(args, uwb, synth, dev)

    if not args.no_c5:
        out["learned"] = learned_block(args, uwb, synth, dev)
    if not args.no_c4:
        out["batched_serving"] = c4_block(args, uwb, synth, dev)
    if not args.no_ms:
        out["multistatic"] = multistatic_block(args, uwb, synth, dev)
        out["tumour_check"] = tumour_check_block(uwb, synth, dev)

    if not args.no_cpu:
        import oracle
        t_start = time.perf_counter()
        n_done, vox_done, used = 0, 0, 0
        idx = oracle.box_indices((0, nx, 0, ny, 0, nz))
        while True:
            s = distinct[n_done % len(distinct)]
            for bf in (0, 1):
                _, used = oracle.image_indices(s, bf, idx, W, 0, return_threads=True)
            n_done += 1
            vox_done += 2 * idx.shape[0] * M
            if time.perf_counter() - t_start >= args.cpu_seconds:
                break
        el = time.perf_counter() - t_start
        # the same oracle on one thread, over every 16th voxel of the scans (a quarter of the time above)
        sub = np.ascontiguousarray(idx[::16])
        t1 = time.perf_counter()
        n1, vox1 = 0, 0
        while True:
            s = distinct[n1 % len(distinct)]
            for bf in (0, 1):
                oracle.image_indices(s, bf, sub, W, 1)
            n1 += 1
            vox1 += 2 * sub.shape[0] * M
            if time.perf_counter() - t1 >= args.cpu_seconds / 4:
                break
        el1 = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(vox_done / el / 1e9, 4), "unit": "Gvoxel·antenna/s",
                               "cores": int(used), "kind": "oracle",
                               "sample": f"{n_done} full 512x512 scans, DAS + direct-pairwise DMAS, FP64, "
                                         f"{el:.1f} s",
                               "build": "gcc " + " ".join(oracle.build_flags()) +
                                        " (plain C, one focal point at a time, OpenMP over focal points)",
                               "one_core": {"value": round(vox1 / el1 / 1e9, 5), "cores": 1,
                                            "sample": f"{n1} scans x {sub.shape[0]} voxels (every 16th of 512x512), "
                                                      f"DAS + direct-pairwise DMAS, FP64, {el1:.1f} s"}}
    print(json.dumps(out), flush=True)


def lds_peak(uwb):
    """LDS read bandwidth of the device (16-byte reads, conflict-free, 20 workgroups per CU), and the same in bytes
    per clock per CU at the shader clock measured during the loop."""
    bps, hz = max(uwb.probe_lds_read(16, 4096, 256 * 20) for _ in range(3))
    return {"bytes_per_s": bps, "tb_per_s": round(bps / 1e12, 2), "clock_ghz": round(hz / 1e9, 3),
            "bytes_per_clk_per_cu": round(bps / (hz * 256), 1) if hz > 0 else None,
            "probe": "ds_read_b128 stream, 256 lanes x 20 workgroups per CU, 4096 reads per lane"}


def _event_ms(fn, reps=50):
    """Median over reps of one call bracketed by HIP events on the current stream."""
    import numpy as np
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def mvdr_flops_per_va(window: int, n_ant: int) -> float:
    """Algorithmic FP32 work of the Capon (MVDR) image per voxel·antenna: the delay (11 flops), per window offset
    the interpolation (3) and the window sum (1), the W (W + 1) / 2 Gram products (2 each), and per voxel the W x W
    Cholesky factorisation and two triangular solves (W^3 / 3 + 2 W^2 flops) spread over the voxel's antennas."""
    w = window
    return FLOPS_DELAY + 4 * w + w * (w + 1) + (w ** 3 / 3 + 2 * w * w) / n_ant


def mvdr_block(args, uwb, synth, dev):
    """The framework over the Capon (MVDR) beamformer on the 2D hierarchical configuration (32 antennas, 2048
    samples, 512 x 512, 200 clutter scatterers, 20 dB): full-resolution MVDR images and their detection, and the
    per-level walk over MVDR (g = 16 and 32) against the full-resolution MVDR detection."""
    import ctypes
    import numpy as np
    import torch
    n = args.mvdr_scans
    scans = [synth.c2_scan(5000 + k) for k in range(n)]
    g = scans[0].grid
    nx, ny, nz = g.dims
    M = scans[0].n_ant
    b = uwb.DeviceBatch.from_host(scans, dev)
    bc = b.c()
    img = torch.empty((n, nz, ny, nx), dtype=torch.float32, device=dev)
    t_img = _event_ms(lambda: uwb.image_batch(b, g, 2, out=img, bc=bc), )
    pk = uwb.argmax_batch_async(b, g, img, 2, bc=bc)
    t_arg = _event_ms(lambda: uwb.argmax_batch_async(b, g, img, 2, out=pk, bc=bc), )
    full = uwb._peaks(pk, n)
    va = n * nx * ny * nz * M
    res = {}
    for gg, m in ((16, "max"), (16, "mean"), (32, "max"), (32, "mean")):
        tree = uwb.SegmentTree(beamformer=2, coarse=gg, metric=m, frame_final=0.25)
        gc, tc = uwb.grid_c(g), tree.c()
        ws = torch.empty(uwb.lib().uwb_segment_workspace_bytes(ctypes.byref(gc), ctypes.byref(tc), n),
                         dtype=torch.uint8, device=dev)
        rb = torch.empty(ctypes.sizeof(uwb.UwbSegmentResult) * n, dtype=torch.uint8, device=dev)
        t_w = _event_ms(lambda tree=tree, ws=ws, rb=rb: uwb.segment_refine_batch_async(
            b, g, tree, out=rb, workspace=ws, bc=bc), )
        rr = uwb._results(rb, n, 4)
        w1 = float(np.mean([abs(r.argmax % nx - f.index % nx) <= 1 and abs(r.argmax // nx - f.index // nx) <= 1
                            for r, f in zip(rr, full)]))
        res[f"walk_g{gg}_{m}"] = {"scans_per_s": round(n / (t_w * 1e-3), 1), "ms_per_batch": round(t_w, 4),
                                "within_1_voxel_of_full_mvdr": w1,
                                "speedup_vs_full_mvdr_at_equal_error":
                                    round((t_img + t_arg) / t_w, 1) if w1 >= 1.0 else None}
    fpva = mvdr_flops_per_va(11, M)
    return {"workload": "2D monostatic ring, 32 antennas x 2048 samples, 512x512 grid, window 11, Capon weights "
                        "(diagonal loading 3 x mean channel power) per voxel",
            "scans": n, "image_ms": round(t_img, 4), "gvas": round(va / (t_img * 1e-3) / 1e9, 2),
            "flops_per_voxel_antenna": round(fpva, 1),
            "tflops": round(fpva * va / (t_img * 1e-3) / 1e12, 2),
            "roofline_frac_fp32": round(fpva * va / (t_img * 1e-3) / PEAK_FP32, 4),
            "detection_ms": round(t_arg, 4), "full_mvdr_scans_per_s": round(n / ((t_img + t_arg) * 1e-3), 1),
            **res}


def c1_block(uwb, synth, dev):
    """2D single scan (16-antenna ring, 1024 samples, 128 x 128, window 11): too small to fill the device, so
    reported as the latency of one call (median of 50, HIP events)."""
    s = synth.c1_scan(0)
    ds = uwb.DeviceScan.from_host(s, dev)
    g = s.grid
    nx, ny, nz = g.dims
    va = nx * ny * nz * s.n_ant
    das, dmas = uwb.das_dmas(ds, g)
    pk = uwb.argmax_async(ds, g, dmas, 1)
    lat = {"das_ms": _event_ms(lambda: uwb.image(ds, g, 0, out=das)),
           "dmas_ms": _event_ms(lambda: uwb.image(ds, g, 1, out=dmas)),
           "das_dmas_one_launch_ms": _event_ms(lambda: uwb.das_dmas(ds, g, out_das=das, out_dmas=dmas)),
           "argmax_ms": _event_ms(lambda: uwb.argmax_async(ds, g, dmas, 1, out=pk)),
           "dmas_image_and_detection_ms": _event_ms(lambda: (uwb.image(ds, g, 1, out=dmas),
                                                             uwb.argmax_async(ds, g, dmas, 1, out=pk)))}
    out = {k: round(v, 5) for k, v in lat.items()}
    out.update({"workload": "2D monostatic ring, 16 antennas x 1024 samples, 128x128 grid, window 11, one scan",
                "voxel_antenna": va, "dmas_gvas_at_this_latency": round(va / (lat["dmas_ms"] * 1e-3) / 1e9, 2)})
    return out


def c3_block(args, uwb, synth, dev):
    """3D: 64 antennas on a hemisphere (Fibonacci), 4096 samples, eps_r uniform in 8-10 per scan, 1000 clutter
    scatterers, 20 dB, 256^3 voxels.  Full-resolution DAS / DMAS throughput on one scan per launch, then octree
    walks (g = 8 and 16) on a batch of distinct scans against the full-resolution DMAS detection."""
    import ctypes
    import numpy as np
    import torch
    n = args.c3_scans
    scans = [synth.c3_scan(k) for k in range(n)]
    g = scans[0].grid
    nx, ny, nz = g.dims
    M = scans[0].n_ant
    va = nx * ny * nz * M
    ds = uwb.DeviceScan.from_host(scans[0], dev)
    das = torch.empty((nz, ny, nx), dtype=torch.float32, device=dev)
    dmas = torch.empty_like(das)
    t = {"das_ms": _event_ms(lambda: uwb.image(ds, g, 0, out=das), ),
         "dmas_ms": _event_ms(lambda: uwb.image(ds, g, 1, out=dmas), ),
         "das_dmas_one_launch_ms": _event_ms(lambda: uwb.das_dmas(ds, g, out_das=das, out_dmas=dmas), ),
         "argmax_dmas_ms": _event_ms(lambda: uwb.argmax_async(ds, g, dmas, 1), )}
    del das
    # full-resolution DMAS detection of every scan (the reference of the walks' localisation error)
    full = []
    for s in scans:
        d = uwb.DeviceScan.from_host(s, dev)
        uwb.image(d, g, 1, out=dmas)
        full.append(uwb.argmax(d, g, dmas, 1).index)
        del d
    del dmas
    torch.cuda.empty_cache()
    b = uwb.DeviceBatch.from_host(scans, dev)
    bc = b.c()

    def within1(a, c):
        ia = np.array([a % nx, (a // nx) % ny, a // (nx * ny)])
        ic = np.array([c % nx, (c // nx) % ny, c // (nx * ny)])
        return bool(np.max(np.abs(ia - ic)) <= 1)

    walks = {}
    full_ms = t["dmas_ms"] + t["argmax_dmas_ms"]
    for gg in (8, 16):
        for m in ("max", "mean"):
            tree = uwb.SegmentTree(beamformer=1, coarse=gg, metric=m, frame_final=0.25)
            gc, tc = uwb.grid_c(g), tree.c()
            need = uwb.lib().uwb_segment_workspace_bytes(ctypes.byref(gc), ctypes.byref(tc), n)
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
            res_buf = torch.empty(ctypes.sizeof(uwb.UwbSegmentResult) * n, dtype=torch.uint8, device=dev)
            ms = _event_ms(lambda tree=tree, ws=ws, res_buf=res_buf: uwb.segment_refine_batch_async(
                b, g, tree, out=res_buf, workspace=ws, bc=bc), )
            res = uwb._results(res_buf, n, 8)
            w1 = float(np.mean([within1(r.argmax, f) for r, f in zip(res, full)]))
            vox = float(np.mean([r.voxels_evaluated for r in res]))
            walks[f"g{gg}_{m}"] = {"scans_per_s": round(n / (ms * 1e-3), 1), "ms_per_batch": round(ms, 4),
                                   "within_1_voxel_of_full_dmas": w1, "voxels_per_walk": vox,
                                   "voxel_ratio_full_over_walk": round(nx * ny * nz / vox, 1),
                                   "speedup_vs_full_dmas_at_equal_error":
                                       round(full_ms * n / ms, 1) if w1 >= 1.0 else None}
    return {"workload": "3D monostatic hemisphere, 64 antennas x 4096 samples, 256^3 grid, window 11",
            "voxel_antenna_per_scan": va,
            **{k: round(v, 4) for k, v in t.items()},
            "das_gvas": round(va / (t["das_ms"] * 1e-3) / 1e9, 2),
            "dmas_gvas": round(va / (t["dmas_ms"] * 1e-3) / 1e9, 2),
            "das_dmas_one_launch_gvas_per_image": round(va / (t["das_dmas_one_launch_ms"] * 1e-3) / 1e9, 2),
            "dmas_roofline_frac_fp32": round(flops_per_va(1, 11) * va / (t["dmas_ms"] * 1e-3) / PEAK_FP32, 4),
            "full_dmas_scans_per_s": round(1e3 / full_ms, 1),
            "walk_scans": n, "octree_walks": walks}


def _timed(fn, reps=50):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def c4_block(args, uwb, synth, dev):
    """Batched serving of uneven scans: one persistent graph-captured launch over C4's mixed batch (M in
    {16..64}, T in {1024..4096}, side in {64..512}, seeds 1000 + i), autotuned on the batch itself; scans/s and the
    per-scan completion-time percentiles within a launch."""
    import numpy as np
    import torch
    n = args.c4_scans
    scans = [synth.c4_scan(1000 + k) for k in range(n)]
    devs = [uwb.DeviceScan.from_host(s, dev) for s in scans]
    outs = [torch.empty((1, s.grid.dims[1], s.grid.dims[0]), dtype=torch.float32, device=dev) for s in scans]
    va = sum(s.n_ant * s.grid.dims[0] * s.grid.dims[1] for s in scans)
    res = {"workload": "C4: uneven monostatic scans, antennas 16-64, samples 1024-4096, grid side 64-512, window 11",
           "scans": n, "voxel_antenna_per_launch": int(va)}
    for bf, name in ((0, "das"), (1, "dmas")):
        plan = uwb.BatchPlan([(d, s.grid, o) for d, s, o in zip(devs, scans, outs)], bf)
        cfg = plan.autotune(3)
        ms = _timed(plan.run)
        plan.run()
        ts = plan.timestamps_ns() / 1e6
        res[name] = {"scans_per_s": round(n / (ms * 1e-3), 1), "ms_per_launch": round(ms, 4),
                     "gvas": round(va / (ms * 1e-3) / 1e9, 2), "latency_ms_p50": round(float(np.percentile(ts, 50)), 4),
                     "latency_ms_p99": round(float(np.percentile(ts, 99)), 4), "config": cfg}
        plan.close()
    return res


def multistatic_block(args, uwb, synth, dev):
    """Eq. (2)/(4) on the 12-antenna ring standing in for the paper's first dataset (144 channels, 200 x 200 grid at
    1 mm): full-resolution DAS/DMAS throughput, the paper walk with automatic D (1 cm tumour -> D = 7), and its
    localisation against full-resolution DMAS."""
    import numpy as np
    B = args.ms_batch
    scans = [synth.ms_scan(k, 1) for k in range(min(B, 16))]
    scans = [scans[k % len(scans)] for k in range(B)]
    grid = scans[0].grid
    b = uwb.DeviceBatch.from_host(scans, dev)
    bc = uwb._ms_batch_c(b)
    nx, ny, nz = grid.dims
    img = {bf: torch_empty(B, grid, dev) for bf in (0, 1)}
    ms = {bf: _timed(lambda bf=bf: uwb.image_multistatic_batch(b, grid, bf, out=img[bf], bc=bc)) for bf in (0, 1)}
    vc = B * nx * ny * nz * 144
    walk, within, vox = {}, {}, {}
    for bf in (0, 1):
        tree = uwb.SegmentTree(beamformer=bf, walk="paper", min_tumour=0.01, metric="max", frame_final=0.25)
        walk[bf] = _timed(lambda tree=tree: uwb.segment_refine_multistatic_batch_async(b, grid, tree, bc=bc))
        res = uwb._results(uwb.segment_refine_multistatic_batch_async(b, grid, tree, bc=bc), B, 4)
        pk = uwb._peaks(uwb.argmax_multistatic_batch_async(b, grid, img[bf], bf, bc=bc), B)
        within[bf] = float(np.mean([abs(r.argmax % nx - p.index % nx) <= 1 and
                                    abs(r.argmax // nx - p.index // nx) <= 1 for r, p in zip(res, pk)]))
        vox[bf] = float(np.mean([r.voxels_evaluated for r in res]))
        decim = res[0].decimation
    arg = {bf: _timed(lambda bf=bf: uwb.argmax_multistatic_batch_async(b, grid, img[bf], bf, bc=bc)) for bf in (0, 1)}
    full = {bf: ms[bf] + arg[bf] for bf in (0, 1)}
    return {"workload": "12-antenna multistatic ring (radius 12 cm), 144 channels x 1024 samples, 200x200 grid at 1 mm, "
                        "window 11", "batch_scans": B,
            "das_gvcs": round(vc / (ms[0] * 1e-3) / 1e9, 2), "dmas_gvcs": round(vc / (ms[1] * 1e-3) / 1e9, 2),
            "unit": "Gvoxel·channel/s", "das_ms": round(ms[0], 4), "dmas_ms": round(ms[1], 4),
            "full_dmas_scans_per_s": round(B / (full[1] * 1e-3), 1),
            "paper_walk_scans_per_s": round(B / (walk[1] * 1e-3), 1), "paper_walk_decimation": decim,
            "paper_walk_within_1_voxel_of_full_das": within[0],
            "paper_walk_within_1_voxel_of_full_dmas": within[1],
            "voxel_ratio_full_over_walk": round(nx * ny / vox[1], 1),
            "complexity_reduction": {
                "measured_time_full_over_walk": {"das": round(full[0] / walk[0], 2), "dmas": round(full[1] / walk[1], 2)},
                "measured_focal_points_full_over_walk": round(nx * ny / vox[1], 1),
                "paper": {"das": 5, "dmas": 13,
                          "setting": "Section IV: 12-antenna multistatic ring, two phantoms, 1 mm resolution, automatic "
                                     "D = 7 for a 1 cm tumour; hardware and implementation not stated"}}}


def torch_empty(B, grid, dev):
    import torch
    nx, ny, nz = grid.dims
    return torch.empty((B, nz, ny, nx), dtype=torch.float32, device=dev)


def tumour_check_block(uwb, synth, dev):
    """The two-decimation check of Section IV on 64 C1 scans with a tumour and 64 noise-only scans."""
    import numpy as np
    grid = synth.square_grid(128)
    yes = [synth.c1_scan(k) for k in range(64)]
    no = [synth.random_scan(k, 16, 1024, grid) for k in range(64)]
    tree = uwb.SegmentTree(beamformer=1, walk="paper", metric="max", frame_final=0.25)
    ay, _, _ = uwb.tumour_check_batch(uwb.DeviceBatch.from_host(yes, dev), grid, tree, 9, 5)
    an, _, _ = uwb.tumour_check_batch(uwb.DeviceBatch.from_host(no, dev), grid, tree, 9, 5)
    return {"decimations": [9, 5], "confirmed_with_tumour": float(np.mean(ay)),
            "confirmed_noise_only": float(np.mean(an)), "scans": 64}


def learned_block(args, uwb, synth, dev):
    """Train the proposer (C2 recipe, 200k scans, seeds 1,000,000 + i) and evaluate on held-out seeds
    2,000,000 + i against full-resolution DMAS."""
    import torch
    from paper_1709_02549_amd import proposer as P
    from synth import scans as S

    def note(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    rec = uwb.DiscRecipe(2048, 200, S.C0 / 3.0, S.DT, 0.0, S.REGION, 20.0, S.PULSE_F0, S.PULSE_SIGMA,
                         S._PEAK["sin_gauss"], 0x02)
    ant = torch.tensor(S.ring_antennas(32), dtype=torch.float32, device=dev)
    grid = S.square_grid(512)
    t0 = time.time()
    ts = P.build_training_set(rec, ant, list(range(1_000_000, 1_000_000 + args.c5_train)), grid)
    note(f"training set: {args.c5_train} scans x {ts.levels} levels in {time.time() - t0:.1f} s")
    net = uwb.CNN(2048, P.he_init(0))
    steps = max(1, int(args.c5_epochs * ts.x.shape[0] / 256))
    hist, ms_step = P.train(net, ts, steps, 256, log_every=max(steps // 5, 1))
    note(f"trained {steps} steps, {ms_step:.3f} ms/step, loss {hist[-1][1]:.4f}")
    methods = {}
    for m in ("max", "mean"):
        tree = uwb.SegmentTree(beamformer=1, coarse=32, metric=m, frame_final=0.25)
        methods[f"learned_{m}_fallback"] = P.learned_method(net, tree, grid, 0.9)
        methods[f"das_levels_{m}_no_cnn"] = P.learned_method(net, tree, grid, 2.0)
    for g in (8, 16, 32):
        for m in ("max", "mean"):
            methods[f"walk_g{g}_{m}"] = P.walk_method(uwb.SegmentTree(beamformer=1, coarse=g, metric=m,
                                                                      frame_final=0.25), grid)
    ev = P.evaluate(rec, ant, list(range(2_000_000, 2_000_000 + args.c5_eval)), grid, methods, chunk=2048)
    note("held-out evaluation done")
    n_train_samples = int(ts.x.shape[0])
    net.close()
    del ts
    torch.cuda.empty_cache()
    full = ev["full_dmas"]["scans_per_s"]
    equal = {k: round(v["scans_per_s"] / full, 2) for k, v in ev.items() if k != "full_dmas" and v["within_1"] >= 0.999}
    return {"speedup_vs_full_dmas_at_equal_error": equal,
            "equal_error_rule": "within one voxel (L-inf) of the full-resolution DMAS detection on >= 99.9 % of "
                                "held-out scans",
            "train_scans": args.c5_train, "train_samples": n_train_samples, "steps": steps, "batch": 256,
            "ms_per_train_step": round(ms_step, 4), "train_samples_per_s": round(256 / ms_step * 1e3, 1),
            "final_loss": round(hist[-1][1], 5), "threshold": 0.9, "held_out_scans": args.c5_eval,
            "methods": {k: {kk: round(vv, 5) for kk, vv in v.items()} for k, v in ev.items()}}


if __name__ == "__main__":
    main()
