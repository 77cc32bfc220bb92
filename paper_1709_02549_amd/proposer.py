"""Training and evaluation driver of the learned segment proposer.

Every step runs in the HIP library: scans come from the GPU generator, labels
from full-resolution DMAS and its FP64-decided argmax, inputs from the per-level
32 x 32 DAS lattices on the detection's path, and training from the library's
BF16 forward/backward kernels with Adam.  This module only orders the calls and
slices device buffers.

"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import (CNN, DiscRecipe, SegmentTree, _peaks, _results, argmax_batch_async, cnn_input_levels,
               cnn_training_inputs, generate_disc_scans, image_batch, learned_refine_batch, segment_refine_batch_async)
from ._abi import UWB_DMAS

CH = 32


def he_init(seed: int) -> np.ndarray:
    """He-normal convolutions, zero biases, readout N(0, 1/32); flat in the library's parameter order."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(CH * 9) * np.sqrt(2.0 / 9.0)]
    parts += [rng.standard_normal(CH * CH * 9) * np.sqrt(2.0 / (CH * 9.0)) for _ in range(3)]
    parts += [np.zeros(4 * CH), rng.standard_normal(CH) * np.sqrt(1.0 / CH), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


@dataclasses.dataclass
class TrainingSet:
    x: torch.Tensor          # [n_scans * L, 32, 32] bf16
    labels: torch.Tensor     # [n_scans * L] int32
    levels: int
    n_scans: int
    ms: dict                 # GPU time per stage


def _event():
    e = torch.cuda.Event(enable_timing=True)
    e.record()
    return e


def _peak_indices(buf: torch.Tensor, n: int) -> np.ndarray:
    return np.array([p.index for p in _peaks(buf, n)], dtype=np.int64)


def build_training_set(recipe: DiscRecipe, ant_pos: torch.Tensor, seeds, grid, window: int = 11,
                       chunk: int = 512) -> TrainingSet:
    """Generate the scans, detect with full-resolution DMAS, and image the true path's lattices."""
    dev = ant_pos.device
    L = cnn_input_levels(grid)
    n = len(seeds)
    x = torch.empty((n * L, 32, 32), dtype=torch.bfloat16, device=dev)
    lab = torch.empty(n * L, dtype=torch.int32, device=dev)
    nx, ny, nz = (int(v) for v in grid.dims)
    img = torch.empty((min(chunk, n), nz, ny, nx), dtype=torch.float32, device=dev)
    ms = {"generate": 0.0, "dmas": 0.0, "argmax": 0.0, "inputs": 0.0}
    for c0 in range(0, n, chunk):
        sd = seeds[c0:c0 + chunk]
        k = len(sd)
        e0 = _event()
        b, _ = generate_disc_scans(recipe, ant_pos, sd, want_tumours=False)
        e1 = _event()
        bc = b.c()
        image_batch(b, grid, UWB_DMAS, window, out=img[:k])
        e2 = _event()
        pk = argmax_batch_async(b, grid, img[:k], UWB_DMAS, window, bc=bc)
        e3 = _event()
        cnn_training_inputs(b, grid, pk, window, bc=bc, x=x[c0 * L:(c0 + k) * L], labels=lab[c0 * L:(c0 + k) * L])
        e4 = _event()
        torch.cuda.synchronize(dev)
        for key, (a, z) in zip(ms, ((e0, e1), (e1, e2), (e2, e3), (e3, e4))):
            ms[key] += a.elapsed_time(z)
    return TrainingSet(x, lab, L, n, ms)


def train(net: CNN, ts: TrainingSet, steps: int, batch: int = 256, lr: float = 2e-3, lr_final: float = 5e-4,
          seed: int = 0, log_every: int = 0):
    """Adam over contiguous minibatches of the training set, minibatch order shuffled per epoch; the learning
    rate drops to lr_final for the last 30 % of the steps.  Returns (loss history, ms per step)."""
    nb = ts.x.shape[0] // batch
    if nb < 1:
        raise ValueError("training set smaller than one minibatch")
    rng = np.random.default_rng(seed)
    loss = torch.empty(1, dtype=torch.float32, device=ts.x.device)
    hist = []
    order = rng.permutation(nb)
    e0 = _event()
    for s in range(steps):
        if s and s % nb == 0:
            order = rng.permutation(nb)
        j = int(order[s % nb])
        net.train_step(ts.x[j * batch:(j + 1) * batch], ts.labels[j * batch:(j + 1) * batch],
                       lr if s < 0.7 * steps else lr_final, loss)
        if log_every and (s % log_every == 0 or s == steps - 1):
            hist.append((s, float(loss.item())))
    e1 = _event()
    torch.cuda.synchronize(ts.x.device)
    return hist, e0.elapsed_time(e1) / max(steps, 1)


def linf_voxels(a, b, nx: int) -> np.ndarray:
    """L-infinity distance in voxels between finest-grid linear indices of a planar grid."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    return np.maximum(np.abs(a % nx - b % nx), np.abs(a // nx - b // nx))


def evaluate(recipe: DiscRecipe, ant_pos: torch.Tensor, seeds, grid, methods: dict, window: int = 11,
             chunk: int = 512):
    """Localisation against full-resolution DMAS on held-out scans.

    methods: {name: fn(batch, batch_c) -> device buffer of uwb_segment_result} (launched on the current
    stream).  Returns {name: {"within_1": fraction at L-inf <= 1 voxel, "scans_per_s": GPU rate,
    "cnn_levels": mean fraction of CNN-decided levels}}, with "full_dmas" timing the full-resolution
    DMAS image + argmax of the same scans."""
    dev = ant_pos.device
    nx, ny, nz = (int(v) for v in grid.dims)
    img = torch.empty((min(chunk, len(seeds)), nz, ny, nx), dtype=torch.float32, device=dev)
    acc = {k: [] for k in methods}
    lvl = {k: [] for k in methods}
    ms = {k: 0.0 for k in list(methods) + ["full_dmas"]}
    for c0 in range(0, len(seeds), chunk):
        sd = seeds[c0:c0 + chunk]
        k = len(sd)
        b, _ = generate_disc_scans(recipe, ant_pos, sd, want_tumours=False)
        bc = b.c()
        torch.cuda.synchronize(dev)
        e0 = _event()
        image_batch(b, grid, UWB_DMAS, window, out=img[:k])
        pk = argmax_batch_async(b, grid, img[:k], UWB_DMAS, window, bc=bc)
        e1 = _event()
        torch.cuda.synchronize(dev)
        ms["full_dmas"] += e0.elapsed_time(e1)
        truth = _peak_indices(pk, k)
        for name, fn in methods.items():
            e0 = _event()
            out = fn(b, bc)
            e1 = _event()
            torch.cuda.synchronize(dev)
            ms[name] += e0.elapsed_time(e1)
            res = _results(out, k, 4)
            acc[name].append(linf_voxels([r.argmax for r in res], truth, nx) <= 1)
            lvl[name].append([bin(r.learned_mask).count("1") / max(r.n_levels, 1) for r in res])
    out = {}
    for name in methods:
        out[name] = {"within_1": float(np.mean(np.concatenate(acc[name]))),
                     "scans_per_s": len(seeds) / (ms[name] / 1e3),
                     "cnn_levels": float(np.mean(np.concatenate(lvl[name])))}
    out["full_dmas"] = {"within_1": 1.0, "scans_per_s": len(seeds) / (ms["full_dmas"] / 1e3)}
    return out


def learned_method(net: CNN, tree: SegmentTree, grid, threshold: float, window: int = 11):
    return lambda b, bc: learned_refine_batch(b, grid, tree, net, threshold, window, bc=bc, sync=False)


def walk_method(tree: SegmentTree, grid, window: int = 11):
    return lambda b, bc: segment_refine_batch_async(b, grid, tree, window, bc=bc)[0]
