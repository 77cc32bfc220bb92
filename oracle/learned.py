"""Oracle of the learned segment proposer's use in the walk (test infrastructure only).

The paper's conclusion leaves the choice of the region to keep to better
heuristics; here a small CNN (``oracle.cnn``) proposes it.  The walk is the
per-level quadtree walk of ``oracle.walk`` on a planar grid with g = 32 and a
fixed depth: at every level the current box is imaged (DAS) on its 32 x 32
lattice, exactly as the per-level walk does, and then

* the metric of Section III scores the four children (the fallback choice);
* the lattice divided by its maximum is the CNN's input; its softmax gives one
  probability per child;
* the CNN's child (the first maximal probability) is kept when its probability
  reaches the threshold, otherwise the metric's child.

The final ROI is imaged at full resolution with the tree's beamformer and the
detection is its maximal-energy voxel, as in the walk.  A threshold above one
never trusts the CNN, which reduces this walk to ``oracle.walk`` (a pin).

Training data: for a target voxel (e.g. the full-resolution DMAS detection) the
boxes on its path are the aligned boxes of side N / 2^l that hold it; each is
imaged like a level of the walk and labelled with the child holding the target.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import DAS, box_indices, image_indices, linear_index, select_max
from . import cnn as cnn_oracle
from .walk import TreeParams, _expand, _inside, _lattice, _select, _split, metric_value

G = 32


@dataclasses.dataclass
class LearnedResult:
    child: list            # child kept at every level
    fallback: list         # the metric's child at every level
    probs: list            # CNN probabilities [4] at every level
    learned_mask: int      # bit l set when the CNN decided level l
    boxes: list            # boxes[0] = grid, boxes[l + 1] after decision l
    scores: list           # metric of every child at every level
    inputs: list           # CNN input (lattice / max, FP64, before any rounding) per level
    roi: tuple
    argmax: int
    peak: float
    voxels_evaluated: int


def _depth(dims, params: TreeParams) -> int:
    n = int(dims[0])
    if int(dims[2]) != 1 or int(dims[1]) != n:
        raise ValueError("the learned walk needs a square planar grid")
    if n % G or (n // G) & (n // G - 1):
        raise ValueError("grid side must be 32 * 2^L")
    top = int(round(math.log2(n // G)))
    depth = top if params.max_depth <= 0 else min(int(params.max_depth), top)
    if depth < 1:
        raise ValueError("the learned walk needs at least one split")
    return depth


def box_lattice(box, side):
    """Index array [1024, 3] of the 32 x 32 lattice of a box of the given side (x fastest)."""
    step = side // G
    axes = [box[0] + step * np.arange(G) + step // 2, box[2] + step * np.arange(G) + step // 2,
            np.zeros(1, dtype=np.int64)]
    return _lattice(axes)


def cnn_input(vals):
    """The lattice energies divided by their maximum (left unscaled when the maximum is not positive)."""
    vals = np.asarray(vals, dtype=np.float64)
    m = float(np.max(vals))
    return (vals / m if m > 0.0 else vals).reshape(G, G)


def learned_walk(scan, params: TreeParams, net: cnn_oracle.Params, threshold: float, window: int = 11,
                 act_round=None) -> LearnedResult:
    """The walk above.  ``act_round`` (e.g. ``cnn.bf16_round``) rounds the CNN's input and activations as the
    GPU stores them; ``net`` holds the weights the network computes with."""
    if params.walk != "per_level" or int(params.coarse) != G or params.term != "fixed":
        raise ValueError("the learned walk is the per-level walk with g = 32 and a fixed depth")
    dims = tuple(int(x) for x in scan.grid.dims)
    active = (0, 1)
    depth = _depth(dims, params)
    n = dims[0]
    box = (0, dims[0], 0, dims[1], 0, dims[2])
    boxes = [box]
    child, fallback, probs, scores, inputs = [], [], [], [], []
    mask = 0
    nvox = 0
    for lev in range(depth):
        side = n >> lev
        idx = box_lattice(box, side)
        vals = image_indices(scan, DAS, idx, window)
        nvox += idx.shape[0]
        e = int(math.floor(float(params.frame_level) * (side // 2)))
        sc = []
        for c in range(4):
            cbox = _split(box, c, active)
            sbox = list(cbox)
            for d in active:
                sbox[2 * d] = max(box[2 * d], cbox[2 * d] - e)
                sbox[2 * d + 1] = min(box[2 * d + 1], cbox[2 * d + 1] + e)
            sc.append(metric_value(params.metric, vals[_inside(idx, sbox)], vals))
        fb = _select(sc)
        x = cnn_input(vals)
        logits, _ = cnn_oracle.forward(net, x[None], act_round)
        p = cnn_oracle.softmax(logits)[0]
        arg = int(np.argmax(p))
        c = fb
        if p[arg] >= threshold:
            c = arg
            mask |= 1 << lev
        child.append(c)
        fallback.append(fb)
        probs.append(p)
        scores.append(sc)
        inputs.append(x)
        box = _split(box, c, active)
        boxes.append(box)
    roi = _expand(box, params.frame_final, dims, active)
    ridx = box_indices(roi)
    rvals = image_indices(scan, params.beamformer, ridx, window)
    nvox += ridx.shape[0]
    arg, peak = select_max(rvals, linear_index(ridx, dims))
    return LearnedResult(child, fallback, probs, mask, boxes, scores, inputs, roi, arg, peak, nvox)


def path_boxes(target: int, dims, depth: int):
    """The aligned boxes of side N / 2^l (l = 0 .. depth-1) that hold voxel ``target`` and the child of each
    that holds it."""
    n = int(dims[0])
    tx, ty = int(target) % n, int(target) // n
    out = []
    for lev in range(depth):
        side = n >> lev
        x0, y0 = (tx // side) * side, (ty // side) * side
        box = (x0, x0 + side, y0, y0 + side, 0, 1)
        lab = int(tx >= x0 + side // 2) + 2 * int(ty >= y0 + side // 2)
        out.append((box, lab))
    return out


def training_inputs(scan, target: int, window: int = 11, max_depth: int = 0):
    """CNN inputs [L, 32, 32] (FP64, before rounding) and labels [L] along the path to ``target``."""
    dims = tuple(int(x) for x in scan.grid.dims)
    depth = _depth(dims, TreeParams(coarse=G, max_depth=max_depth))
    xs, labs = [], []
    for lev, (box, lab) in enumerate(path_boxes(target, dims, depth)):
        vals = image_indices(scan, DAS, box_lattice(box, dims[0] >> lev), window)
        xs.append(cnn_input(vals))
        labs.append(lab)
    return np.stack(xs), np.array(labs, dtype=np.int64)
