"""FP64 oracle for DAS / DMAS imaging and the coarse-to-fine segment walk.

TEST INFRASTRUCTURE ONLY: this package exists to check the GPU library.  Only
the tests, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product path never does.  It shares no code with the GPU library (the
only module both sides use is the seeded scan generator ``synth``).

* ``image_indices`` / ``image_grid``: Eq. (1) delay, Eq. (3) DAS and the direct
  pairwise DMAS of Section II, evaluated voxel by voxel in plain C (liboracle.so).
* ``mvdr``: the Capon (MVDR) beamformer on the same aligned samples (numpy solve per focal point),
  the data-adaptive beamformer Section I names, for the framework over it.
* ``walk``: the Section III framework (spatial decimation, ROI selection with the
  mean / variance / Eq. (5) metrics, the Eq. (6)-(7) within/between-class stop,
  sliding frame, final imaging), written in numpy.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB_PATH, build, build_flags  # noqa: F401

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = ctypes.CDLL(LIB_PATH)
        for name in ("oracle_image_indices", "oracle_image_indices_ms", "oracle_aligned_samples",
                     "oracle_aligned_samples_ms"):
            getattr(_lib, name).restype = ctypes.c_int
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


DAS, DMAS, MVDR = 0, 1, 2


def image_indices(scan, beamformer: int, idx, window: int = 11, n_threads: int = 0,
                  return_threads: bool = False, loading: float | None = None):
    """Energies at voxel indices idx [n, 3] (ix, iy, iz) of scan.grid, fp64.  A multistatic scan
    (``scan.multistatic``: M antennas, M^2 traces, channel i*M + j) uses Eq. (2) / Eq. (4).
    beamformer 2 is the Capon / MVDR beamformer of ``oracle.mvdr`` (loading: its diagonal loading)."""
    if beamformer == MVDR:
        from . import mvdr
        vals = mvdr.image_indices(scan, idx, window, mvdr.DEFAULT_LOADING if loading is None else loading,
                                  n_threads=n_threads)
        return (vals, n_threads) if return_threads else vals
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).reshape(-1, 3))
    ant = np.ascontiguousarray(scan.ant_pos, dtype=np.float32)
    tr = np.ascontiguousarray(scan.traces, dtype=np.float32)
    origin = np.ascontiguousarray(scan.grid.origin, dtype=np.float64)
    pitch = np.ascontiguousarray(scan.grid.pitch, dtype=np.float64)
    out = np.zeros(idx.shape[0], dtype=np.float64)
    ms = bool(getattr(scan, "multistatic", False))
    if ms and tr.shape[0] != ant.shape[0] ** 2:
        raise ValueError("a multistatic scan holds M^2 traces")
    fn = lib().oracle_image_indices_ms if ms else lib().oracle_image_indices
    used = fn(
        ctypes.c_int(beamformer), ctypes.c_int(ant.shape[0]), ctypes.c_int(tr.shape[1]), _ptr(ant),
        _ptr(tr), ctypes.c_double(scan.dt), ctypes.c_double(scan.t0), ctypes.c_double(scan.v),
        ctypes.c_int(window), _ptr(origin), _ptr(pitch), ctypes.c_long(idx.shape[0]), _ptr(idx),
        _ptr(out), ctypes.c_int(n_threads))
    return (out, used) if return_threads else out


def aligned_samples(scan, idx, window: int = 11, n_threads: int = 0):
    """The aligned window samples s_i(r, k) of every channel at voxel indices idx [n, 3]: [n, channels, window]
    fp64 (Eq. (3) argument; Eq. (2) delays over the M^2 channels of a multistatic scan)."""
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).reshape(-1, 3))
    ant = np.ascontiguousarray(scan.ant_pos, dtype=np.float32)
    tr = np.ascontiguousarray(scan.traces, dtype=np.float32)
    origin = np.ascontiguousarray(scan.grid.origin, dtype=np.float64)
    pitch = np.ascontiguousarray(scan.grid.pitch, dtype=np.float64)
    ms = bool(getattr(scan, "multistatic", False))
    n_ch = ant.shape[0] ** 2 if ms else ant.shape[0]
    if tr.shape[0] != n_ch:
        raise ValueError("traces do not match the antennas")
    out = np.zeros((idx.shape[0], n_ch, window), dtype=np.float64)
    fn = lib().oracle_aligned_samples_ms if ms else lib().oracle_aligned_samples
    fn(ctypes.c_int(ant.shape[0]), ctypes.c_int(tr.shape[1]), _ptr(ant), _ptr(tr), ctypes.c_double(scan.dt),
       ctypes.c_double(scan.t0), ctypes.c_double(scan.v), ctypes.c_int(window), _ptr(origin), _ptr(pitch),
       ctypes.c_long(idx.shape[0]), _ptr(idx), _ptr(out), ctypes.c_int(n_threads))
    return out


def box_indices(box):
    """All voxel indices of a box [x0, x1, y0, y1, z0, z1), x fastest, as [n, 3]."""
    x0, x1, y0, y1, z0, z1 = (int(b) for b in box)
    zz, yy, xx = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1).astype(np.int32)


def image_grid(scan, beamformer: int, window: int = 11, n_threads: int = 0, loading: float | None = None):
    """Full-resolution image [nz, ny, nx] of scan.grid."""
    nx, ny, nz = scan.grid.dims
    vals = image_indices(scan, beamformer, box_indices((0, nx, 0, ny, 0, nz)), window, n_threads, loading=loading)
    return vals.reshape(nz, ny, nx)


def linear_index(idx, dims):
    """Finest-grid linear index (x fastest) of voxel indices idx [n, 3]."""
    idx = np.asarray(idx, dtype=np.int64).reshape(-1, 3)
    return idx[:, 0] + int(dims[0]) * (idx[:, 1] + int(dims[1]) * idx[:, 2])


TIE_REL = 1e-12


def select_max(values, keys):
    """Decision rule shared by voxel argmax and child selection.

    The winner is the smallest key among entries whose value is within a relative
    1e-12 of the maximum: value >= max - 1e-12 * |max|.  Returns (key, value).
    """
    values = np.asarray(values, dtype=np.float64)
    keys = np.asarray(keys, dtype=np.int64)
    m = float(np.max(values))
    ok = values >= m - TIE_REL * abs(m)
    j = int(np.argmin(np.where(ok, keys, np.iinfo(np.int64).max)))
    return int(keys[j]), float(values[j])


def argmax_grid(img):
    """Detection by maximal synthesized energy (Section II-A), rule above, on a full image."""
    flat = np.asarray(img, dtype=np.float64).ravel()
    return select_max(flat, np.arange(flat.size))


from .walk import TreeParams, WalkResult, auto_decimation, walk  # noqa: E402,F401
