"""Oracle of the Section III framework: decimation, ROI selection, final imaging.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper describes a heuristic, so it is followed step by step rather than
replaced by "the full-resolution argmax, found faster":

1. Spatial decimation (Section III, first phase).  Beamform only a lattice of
   focal points taken every D-th point of the final-resolution grid.  D is chosen
   manually or automatically from the smallest tumour to detect: the side of the
   square inscribed in that tumour, divided by the resolution (worked example in
   Section IV: 1 cm tumour, 1 mm resolution, D = 7).
2. ROI selection (second phase).  Split the current region into 4 equal squares
   (8 cubes in 3D), score each with a decision metric -- mean, variance, or the
   Eq. (5) blend M = (1 - a) mu + a sigma^2 with a = (sigma_i^2 - sigma_{i-1}^2) / sigma_i^2
   -- keep the best and repeat.  The loop may stop on the within-class (Eq. 6) and
   between-class (Eq. 7) distances of two consecutive iterations: it continues
   while B grows and W shrinks.  A sliding frame widens the kept square in
   proportion to its side so an edge tumour is not cut off.
3. Final imaging (third phase).  Full resolution inside the kept ROI only; the
   detection is the voxel of maximal synthesized energy (Section II-A).

Two walk modes are provided:

* ``paper``: exactly the three phases above -- one decimated image of the whole
  grid, then splits that re-use its samples.
* ``per_level``: every level re-images its current box on a g x g (x g) lattice
  (step D = side / g), a quadtree (octree) walk from the whole grid down to a box
  of side g.  Frames only widen each child's scoring set so boxes stay aligned.

Readings taken where the text is silent or ambiguous (all shared with the GPU):
* lattice samples sit at offset floor(D/2) inside each D-block of the finest grid;
* the split point is x0 + floor(side/2); children are numbered bx + 2 by + 4 bz;
* variance is the population variance (1/n);
* in Eq. (5) sigma_{i-1}^2 is the variance of the parent box's samples; values are
  divided by the parent's sample maximum first; a = 0 when sigma_i^2 = 0; "eq5" keeps a
  as printed (unclamped), "eq5_clamped" clamps a to [0, 1] (the prose's reading);
* Eq. (6)/(7) on scalar energies: the two classes are the sample sets of the
  previous and the current box; W = sum of squared deviations from each class mean,
  B = sum_class n_class (mean_class - pooled mean)^2; the first iteration always
  proceeds; at a later iteration the walk stops as soon as B does not grow or W
  does not shrink, and the failing split is undone;
* ties: the smallest index among values within a relative 1e-12 of the maximum.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

METRICS = ("mean", "var", "eq5", "max", "max_over_mean", "eq5_clamped")
TERMS = ("fixed", "wb")
WALKS = ("per_level", "paper")
MAX_LEVELS = 16
MIN_CHILD_SAMPLES = 4


@dataclasses.dataclass
class TreeParams:
    beamformer: int = 0          # 0 = DAS, 1 = DMAS, 2 = Capon / MVDR (oracle.mvdr)
    walk: str = "per_level"      # "per_level" | "paper"
    coarse: int = 8              # g: lattice points per side per level (per_level)
    decimation: int = 0          # D (paper); 0 = automatic from min_tumour
    min_tumour: float = 0.01     # metres, for automatic D
    max_depth: int = 0           # 0 = as deep as the mode allows
    metric: str = "max"
    term: str = "fixed"          # "fixed" | "wb"
    frame_level: float = 0.0     # sliding frame, fraction of the child side
    frame_final: float = 0.25    # frame applied to the last box before final imaging
    loading: float = 3.0         # MVDR diagonal loading, relative to the mean channel power


@dataclasses.dataclass
class WalkResult:
    n_levels: int                # decisions kept
    term_level: int              # decisions made (one more than kept if the W/B stop undid a split)
    child: list                  # child index of every decision made
    boxes: list                  # boxes[0] = grid, boxes[i+1] = box after decision i; [x0,x1,y0,y1,z0,z1)
    scores: list                 # per decision made: metric of every child
    wb: list                     # (W, B) for every iteration evaluated (iteration 1, 2, ...)
    roi: tuple
    argmax: int                  # finest-grid linear index, x fastest
    peak: float
    voxels_evaluated: int
    decimation: int              # D used by the paper walk (0 for per_level)
    samples: list                # per imaged set: (idx [n,3], energies [n])
    roi_image: np.ndarray | None = None


def auto_decimation(min_tumour: float, pitch: float) -> int:
    """Automatic spatial decimation factor (Section III; worked example in Section IV).

    One lattice point per square inscribed in the smallest tumour: the square's side
    is d_min / sqrt(2); D = floor(side / pitch), at least 1.
    """
    if not (math.isfinite(min_tumour) and math.isfinite(pitch)) or min_tumour <= 0 or pitch <= 0:
        raise ValueError("min_tumour and pitch must be finite and positive")
    d = min_tumour / (math.sqrt(2.0) * pitch)
    return max(1, int(math.floor(d)))


# ----------------------------------------------------------------------------------
# statistics (Section III, Eq. (5)-(7))
# ----------------------------------------------------------------------------------

def _mean(x):
    return float(np.sum(x) / x.size)


def _var(x):
    mu = _mean(x)
    return float(np.sum((x - mu) ** 2) / x.size)


def metric_value(name: str, x: np.ndarray, parent: np.ndarray) -> float:
    x = np.asarray(x, dtype=np.float64)
    parent = np.asarray(parent, dtype=np.float64)
    if name == "mean":
        return _mean(x)
    if name == "var":
        return _var(x)
    if name == "max":
        return float(np.max(x))
    if name == "max_over_mean":
        mu = _mean(x)
        return float(np.max(x)) / mu if mu != 0.0 else 0.0
    if name in ("eq5", "eq5_clamped"):
        pm = float(np.max(parent))
        if pm > 0.0:
            x = x / pm
            parent = parent / pm
        sc = _var(x)
        sp = _var(parent)
        mu = _mean(x)
        alpha = (sc - sp) / sc if sc > 0.0 else 0.0
        if name == "eq5_clamped":
            # reading of the prose after Eq. (5): the blend moves from the mean
            # (similar variances) to the variance (distinct variances)
            alpha = min(max(alpha, 0.0), 1.0)
        return (1.0 - alpha) * mu + alpha * sc
    raise ValueError(name)


def within_between(a: np.ndarray, b: np.ndarray):
    """Eq. (6) W and Eq. (7) B for two classes of scalar energies."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    ma, mb = _mean(a), _mean(b)
    m = float((np.sum(a) + np.sum(b)) / (a.size + b.size))
    w = float(np.sum((a - ma) ** 2) + np.sum((b - mb) ** 2))
    bt = a.size * (ma - m) ** 2 + b.size * (mb - m) ** 2
    return w, float(bt)


def _select(scores):
    from . import select_max
    return select_max(scores, np.arange(len(scores)))[0]


# ----------------------------------------------------------------------------------
# boxes and lattices
# ----------------------------------------------------------------------------------

def _active_dims(dims):
    return (0, 1) if int(dims[2]) == 1 else (0, 1, 2)


def _expand(box, frac, dims, active):
    """Widen each active side by floor(frac * side) on both ends, clipped to the grid."""
    out = list(box)
    for d in active:
        lo, hi = box[2 * d], box[2 * d + 1]
        e = int(math.floor(float(frac) * (hi - lo)))
        out[2 * d] = max(0, lo - e)
        out[2 * d + 1] = min(int(dims[d]), hi + e)
    return tuple(out)


def _split(box, c, active):
    """Child c (Morton bits bx + 2 by + 4 bz) of a box split at x0 + floor(side/2)."""
    out = list(box)
    for bit, d in enumerate(active):
        lo, hi = box[2 * d], box[2 * d + 1]
        mid = lo + (hi - lo) // 2
        if (c >> bit) & 1:
            out[2 * d] = mid
        else:
            out[2 * d + 1] = mid
    return tuple(out)


def _inside(idx, box):
    return ((idx[:, 0] >= box[0]) & (idx[:, 0] < box[1]) & (idx[:, 1] >= box[2]) & (idx[:, 1] < box[3])
            & (idx[:, 2] >= box[4]) & (idx[:, 2] < box[5]))


def _lattice(axes):
    """Index array [n, 3] (x fastest) of the product of per-axis coordinates."""
    zz, yy, xx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1).astype(np.int32)


def _box_voxels(box):
    return (box[1] - box[0]) * (box[3] - box[2]) * (box[5] - box[4])


# ----------------------------------------------------------------------------------
# the walk
# ----------------------------------------------------------------------------------

def walk(scan, params: TreeParams, window: int = 11, image_fn=None, n_threads: int = 0) -> WalkResult:
    """Run the coarse-to-fine framework on one scan (or on ``image_fn``, a function idx[n,3] -> energies)."""
    from . import box_indices, image_indices, linear_index, select_max

    if params.metric not in METRICS or params.term not in TERMS or params.walk not in WALKS:
        raise ValueError("unknown metric / termination / walk")
    dims = tuple(int(x) for x in scan.grid.dims)
    active = _active_dims(dims)
    n_child = 1 << len(active)
    if image_fn is None:
        def image_fn(idx):
            return image_indices(scan, params.beamformer, idx, window, n_threads, loading=params.loading)

    full = (0, dims[0], 0, dims[1], 0, dims[2])
    boxes = [full]
    child, scores, wbs, samples = [], [], [], []
    nvox = 0
    n_kept = 0
    decim = 0

    if params.walk == "per_level":
        n = dims[0]
        g = int(params.coarse)
        if any(dims[d] != n for d in active) or g < 2 or g % 2:
            raise ValueError("per_level walk needs a square/cubic grid and an even g >= 2")
        if n % g or (n // g) & (n // g - 1):
            raise ValueError("grid side must be g * 2^L")
        top = int(round(math.log2(n // g)))
        depth = top if params.max_depth <= 0 else min(int(params.max_depth), top)
        if depth > MAX_LEVELS:
            raise ValueError("too many levels")
        box = full
        for lev in range(depth + 1):
            if lev == depth and params.term != "wb":
                n_kept = depth
                break
            side = n >> lev
            step = side // g
            axes = [np.zeros(1, dtype=np.int64)] * 3
            for d in active:
                axes[d] = box[2 * d] + step * np.arange(g) + step // 2
            idx = _lattice(axes)
            vals = np.asarray(image_fn(idx), dtype=np.float64)
            samples.append((idx, vals))
            nvox += idx.shape[0]
            if params.term == "wb" and lev >= 1:
                w, b = within_between(samples[lev - 1][1], vals)
                wbs.append((w, b))
                if lev >= 2 and (b <= wbs[-2][1] or w >= wbs[-2][0]):
                    n_kept = lev - 1
                    break
            if lev == depth:
                n_kept = depth
                break
            half = side // 2
            e = int(math.floor(float(params.frame_level) * half))
            sc = []
            for c in range(n_child):
                cbox = _split(box, c, active)
                sbox = list(cbox)
                for d in active:
                    sbox[2 * d] = max(box[2 * d], cbox[2 * d] - e)
                    sbox[2 * d + 1] = min(box[2 * d + 1], cbox[2 * d + 1] + e)
                sc.append(metric_value(params.metric, vals[_inside(idx, sbox)], vals))
            c = _select(sc)
            child.append(c)
            scores.append(sc)
            box = _split(box, c, active)
            boxes.append(box)
    else:
        decim = int(params.decimation) if params.decimation > 0 else auto_decimation(params.min_tumour,
                                                                                     scan.grid.pitch[0])
        if any(decim > dims[d] for d in active):
            raise ValueError("decimation larger than the grid")
        depth = MAX_LEVELS if params.max_depth <= 0 else int(params.max_depth)
        if depth > MAX_LEVELS:
            raise ValueError("too many levels")
        axes = [np.zeros(1, dtype=np.int64)] * 3
        for d in active:
            axes[d] = np.arange(decim // 2, dims[d], decim)
        idx = _lattice(axes)
        vals = np.asarray(image_fn(idx), dtype=np.float64)
        samples.append((idx, vals))
        nvox += idx.shape[0]
        box = full
        sets = []
        for lev in range(depth + 1):
            cur = vals[_inside(idx, box)]
            sets.append(cur)
            if params.term == "wb" and lev >= 1:
                w, b = within_between(sets[lev - 1], cur)
                wbs.append((w, b))
                if lev >= 2 and (b <= wbs[-2][1] or w >= wbs[-2][0]):
                    n_kept = lev - 1
                    break
            if lev == depth:
                n_kept = depth
                break
            masks = [_inside(idx, _split(box, c, active)) & _inside(idx, box) for c in range(n_child)]
            if min(int(np.count_nonzero(m)) for m in masks) < MIN_CHILD_SAMPLES:
                n_kept = lev
                break
            sc = [metric_value(params.metric, vals[m], cur) for m in masks]
            c = _select(sc)
            child.append(c)
            scores.append(sc)
            box = _expand(_split(box, c, active), params.frame_level, dims, active)
            boxes.append(box)

    final = boxes[n_kept]
    roi = _expand(final, params.frame_final, dims, active)
    ridx = box_indices(roi)
    rvals = np.asarray(image_fn(ridx), dtype=np.float64)
    nvox += ridx.shape[0]
    arg, peak = select_max(rvals, linear_index(ridx, dims))
    rimg = rvals.reshape(roi[5] - roi[4], roi[3] - roi[2], roi[1] - roi[0])
    return WalkResult(n_kept, len(child), child, boxes, scores, wbs, roi, arg, peak, nvox, decim, samples, rimg)


# ----------------------------------------------------------------------------------
# the mixed-resolution image of the final-imaging phase
# ----------------------------------------------------------------------------------

def composite(scan, params: TreeParams, res: WalkResult) -> np.ndarray:
    """Image [nz, ny, nx] with one region at full resolution and the rest at low resolution (Section III,
    final imaging).  Every coarse sample paints its block of finest voxels, coarse levels first so that finer
    ones overwrite them; the ROI then receives its full-resolution image.

    Blocks: paper walk, lattice point k of an axis covers [D k, D (k + 1)) and the last one runs to the end of
    the grid; per-level walk, point k of level l covers [x0 + D_l k, x0 + D_l (k + 1)) of that level's box."""
    dims = tuple(int(x) for x in scan.grid.dims)
    active = _active_dims(dims)
    img = np.zeros((dims[2], dims[1], dims[0]))
    if params.walk == "paper":
        D = res.decimation
        idx, vals = res.samples[0]
        last = [(dims[d] - 1 - D // 2) // D if d in active else 0 for d in range(3)]
        for (x, y, z), v in zip(idx, vals):
            lo, hi = [], []
            for d, c in enumerate((x, y, z)):
                if d not in active:
                    lo.append(0)
                    hi.append(1)
                    continue
                k = (int(c) - D // 2) // D
                lo.append(D * k)
                hi.append(dims[d] if k == last[d] else D * (k + 1))
            img[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = v
    else:
        g = int(params.coarse)
        for lev, (idx, vals) in enumerate(res.samples):
            step = (dims[0] >> lev) // g
            for (x, y, z), v in zip(idx, vals):
                lo = [int(c) - step // 2 if d in active else 0 for d, c in enumerate((x, y, z))]
                hi = [lo[d] + step if d in active else 1 for d in range(3)]
                img[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = v
    r = res.roi
    img[r[4]:r[5], r[2]:r[3], r[0]:r[1]] = res.roi_image
    return img


# ----------------------------------------------------------------------------------
# the two-decimation check for scans that may hold no tumour
# ----------------------------------------------------------------------------------

def rois_intersect(a, b) -> bool:
    """Whether two boxes [x0, x1, y0, y1, z0, z1) share a voxel."""
    return all(max(a[2 * d], b[2 * d]) < min(a[2 * d + 1], b[2 * d + 1]) for d in range(3))


def tumour_check(scan, params: TreeParams, d1: int, d2: int, window: int = 11, image_fn=None):
    """Section IV, last paragraph: run the three-phase walk with two decimation factors; matching ROIs confirm the
    detection, ROIs in different places mean the walks followed artifacts (no tumour).  "Same location" is read
    as: the two final ROI boxes intersect.  Returns (agree, result with d1, result with d2)."""
    if params.walk != "paper" or d1 < 1 or d2 < 1 or d1 == d2:
        raise ValueError("the check runs the paper walk with two different decimation factors")
    r1 = walk(scan, dataclasses.replace(params, decimation=int(d1)), window, image_fn)
    r2 = walk(scan, dataclasses.replace(params, decimation=int(d2)), window, image_fn)
    return rois_intersect(r1.roi, r2.roi), r1, r2
