"""Capon (minimum-variance distortionless-response, MVDR) beamformer on the aligned window samples.
TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names MVDR in Section I as a data-adaptive beamformer (minimum output power with a distortionless
response toward the focal point) and leaves better beamformers inside its framework to Section V; it gives
no formula.  This module is the plain textbook definition (Capon 1969), applied per focal point r to the
aligned samples of the Eq. (3) argument:

    x_i(k)   aligned sample of channel i at window offset k = -h..h (linear interpolation, zero outside the
             trace: the same gather as DAS/DMAS), X = [x_i(k)], M channels x W offsets
    R        = (1/W) sum_k x(k) x(k)^T, the sample covariance over the W window offsets (the snapshots)
    R_l      = R + delta I,  delta = loading * trace(R) / M  (diagonal loading relative to the mean channel
               power: with W < M the sample covariance is singular)
    a        = (1, ..., 1): after alignment the echo of a scatterer at r has the same phase on every channel
    w        = R_l^-1 a / (a^T R_l^-1 a)   (minimises w^T R_l w subject to w^T a = 1)
    y(k)     = w^T x(k),   I(r) = sum_k y(k)^2
    trace(R) = 0 (no signal at all):  I(r) = 0.

Straight from the definition: an M x M solve per focal point (numpy's LAPACK solve), no reformulation.

The default loading (3 x the mean channel power) is a reading, not the paper's: with W < M snapshots a lightly
loaded Capon beamformer cancels a point echo whose delays miss the focal point by a fraction of a voxel (the
grid never puts a voxel exactly on a scatterer), so its peak moves off the scatterer; from about 3 x the mean
power on, a noiseless or noisy point tumour is found within one voxel on the 16-antenna ring.
"""
from __future__ import annotations

import numpy as np

MVDR = 2
DEFAULT_LOADING = 3.0


def capon_weights(X: np.ndarray, loading: float) -> np.ndarray:
    """Weights w [n, M] for aligned samples X [n, M, W]; rows with no signal get zero weights."""
    X = np.asarray(X, dtype=np.float64)
    n, M, W = X.shape
    R = X @ X.transpose(0, 2, 1) / W
    tr = np.trace(R, axis1=1, axis2=2)
    w = np.zeros((n, M))
    ok = tr > 0
    if ok.any():
        Rl = R[ok] + (loading * tr[ok] / M)[:, None, None] * np.eye(M)[None]
        a = np.ones((int(ok.sum()), M, 1))
        ria = np.linalg.solve(Rl, a)[..., 0]
        w[ok] = ria / ria.sum(axis=1, keepdims=True)
    return w


def capon_energy(X: np.ndarray, loading: float, chunk: int = 4096) -> np.ndarray:
    """I(r) = sum_k (w^T x(k))^2 for aligned samples X [n, M, W]."""
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros(X.shape[0])
    for p0 in range(0, X.shape[0], chunk):
        x = X[p0:p0 + chunk]
        w = capon_weights(x, loading)
        y = np.einsum("nm,nmk->nk", w, x)
        out[p0:p0 + chunk] = np.sum(y * y, axis=1)
    return out


def image_indices(scan, idx, window: int = 11, loading: float = DEFAULT_LOADING, chunk: int = 4096,
                  n_threads: int = 0) -> np.ndarray:
    """MVDR energies at voxel indices idx [n, 3] of scan.grid (monostatic or multistatic channels)."""
    from . import aligned_samples
    idx = np.asarray(idx, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(idx.shape[0])
    for p0 in range(0, idx.shape[0], chunk):
        X = aligned_samples(scan, idx[p0:p0 + chunk], window, n_threads)
        out[p0:p0 + chunk] = capon_energy(X, loading)
    return out
