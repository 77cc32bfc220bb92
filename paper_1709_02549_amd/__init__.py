"""Python binding of libuwb (MI355X / gfx950 DAS-DMAS imaging and segment walk).

Argument marshalling only: every step runs in the HIP library behind the C ABI
of include/uwb.h.  Tensors must be CUDA (HIP) tensors; calls are enqueued on
torch's current stream.  If the library is not built the import of an entry
point raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _abi
from ._abi import (METRICS, TERMS, UWB_DAS, UWB_DMAS, UWB_MVDR, UWB_MAX_LEVELS, WALKS, UwbBatchConfig,  # noqa: F401
                   UwbBatchItem, UwbError, UwbGenRecipe, UwbGrid, UwbPeak, UwbScan, UwbScanBatch, UwbSegmentResult,
                   UwbSegmentTree, check, lib)

__all__ = ["BatchPlan", "CNN", "generate_disc_scans", "learned_refine_batch", "cnn_training_inputs", "DeviceScan", "DeviceBatch", "das", "dmas", "mvdr", "das_dmas", "image", "das_batch", "dmas_batch", "das_dmas_batch", "image_batch",
           "argmax", "argmax_batch", "segment_refine", "segment_refine_batch", "auto_decimation",
           "SegmentTree", "UwbError"]


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _need_cuda(t: torch.Tensor, name: str, dtype=torch.float32, numel: int | None = None):
    """t must be a contiguous CUDA tensor of dtype; with numel, it must hold at least that many elements (the
    library takes raw pointers: a short buffer would be written or read past its end on the device)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, the call needs {numel}")


def _need_bytes(t: torch.Tensor, name: str, nbytes: int):
    """A byte buffer (records, workspace) of at least nbytes on the device."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous CUDA (HIP) tensor")
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise ValueError(f"{name} holds {have} bytes, the call needs {nbytes}")


@dataclasses.dataclass
class DeviceScan:
    """One scan resident in device memory: ant_pos [M,3] f32, traces [M,T] f32."""
    ant_pos: torch.Tensor
    traces: torch.Tensor
    dt: float
    t0: float
    v: float

    @classmethod
    def from_host(cls, s, device="cuda"):
        return cls(torch.as_tensor(np.ascontiguousarray(s.ant_pos, np.float32)).to(device),
                   torch.as_tensor(np.ascontiguousarray(s.traces, np.float32)).to(device),
                   float(s.dt), float(s.t0), float(s.v))

    def c(self) -> UwbScan:
        _need_cuda(self.traces, "traces")
        if self.traces.dim() != 2:
            raise ValueError("traces must be [M, T]")
        _need_cuda(self.ant_pos, "ant_pos", numel=3 * self.traces.shape[0])
        return UwbScan(self.traces.shape[0], self.traces.shape[1], self.ant_pos.data_ptr(), self.traces.data_ptr(),
                       self.dt, self.t0, self.v)


@dataclasses.dataclass
class DeviceBatch:
    """Same-shaped scans: ant_pos [B,M,3] f32, traces [B,M,T] f32, params [B,3] f64 (dt, t0, v)."""
    ant_pos: torch.Tensor
    traces: torch.Tensor
    params: torch.Tensor

    @classmethod
    def from_host(cls, scans, device="cuda"):
        pos = np.stack([np.asarray(s.ant_pos, np.float32) for s in scans])
        tr = np.stack([np.asarray(s.traces, np.float32) for s in scans])
        par = np.array([[s.dt, s.t0, s.v] for s in scans], dtype=np.float64)
        return cls(torch.as_tensor(pos).to(device), torch.as_tensor(tr).to(device), torch.as_tensor(par).to(device))

    @property
    def n_scans(self):
        return int(self.traces.shape[0])

    def c(self) -> UwbScanBatch:
        _need_cuda(self.traces, "traces")
        if self.traces.dim() != 3:
            raise ValueError("traces must be [B, M, T]")
        b, m = int(self.traces.shape[0]), int(self.traces.shape[1])
        if self.ant_pos.dim() != 3 or self.ant_pos.shape[2] != 3 or \
                tuple(self.ant_pos.shape[:2]) not in ((b, m), (b, int(round(m ** 0.5)))):
            raise ValueError("ant_pos must be [B, M, 3] (multistatic: [B, sqrt(M), 3])")
        _need_cuda(self.ant_pos, "ant_pos")
        _need_cuda(self.params, "params", torch.float64, numel=3 * b)
        p = self.params.detach().cpu().numpy()
        return UwbScanBatch(self.traces.shape[0], self.traces.shape[1], self.traces.shape[2],
                            self.ant_pos.data_ptr(), self.traces.data_ptr(), self.params.data_ptr(),
                            float(p[:, 2].min()), float(p[:, 0].min()))


def grid_c(g) -> UwbGrid:
    return UwbGrid((ctypes.c_double * 3)(*[float(x) for x in g.origin]),
                   (ctypes.c_double * 3)(*[float(x) for x in g.pitch]),
                   (ctypes.c_int32 * 3)(*[int(x) for x in g.dims]))


def _img_shape(g):
    nx, ny, nz = (int(x) for x in g.dims)
    return (nz, ny, nx)


def _nvox(g) -> int:
    nx, ny, nz = (int(x) for x in g.dims)
    return nx * ny * nz


_IMAGE_FN = {UWB_DAS: "uwb_das", UWB_DMAS: "uwb_dmas", UWB_MVDR: "uwb_mvdr"}


def _bf(beamformer) -> int:
    b = int(beamformer)
    if b not in _IMAGE_FN:
        raise ValueError(f"beamformer must be 0 (DAS), 1 (DMAS) or 2 (MVDR), not {beamformer}")
    return b


def image(scan: DeviceScan, grid, beamformer: int, window: int = 11, out: torch.Tensor | None = None):
    """Full-resolution DAS (beamformer 0), DMAS (1) or Capon / MVDR (2) image [nz, ny, nx] fp32."""
    if out is None:
        out = torch.empty(_img_shape(grid), dtype=torch.float32, device=scan.traces.device)
    _need_cuda(out, "out", numel=_nvox(grid))
    name = _IMAGE_FN[_bf(beamformer)]
    sc, gc = scan.c(), grid_c(grid)
    check(getattr(lib(), name)(ctypes.byref(sc), ctypes.byref(gc), window, out.data_ptr(), _stream(out.device)),
          name)
    return out


def das_dmas(scan: DeviceScan, grid, window: int = 11, out_das=None, out_dmas=None):
    """DAS and DMAS images [nz, ny, nx] of one scan from one launch. Returns (das, dmas)."""
    if out_das is None:
        out_das = torch.empty(_img_shape(grid), dtype=torch.float32, device=scan.traces.device)
    if out_dmas is None:
        out_dmas = torch.empty(_img_shape(grid), dtype=torch.float32, device=scan.traces.device)
    _need_cuda(out_das, "out_das", numel=_nvox(grid))
    _need_cuda(out_dmas, "out_dmas", numel=_nvox(grid))
    sc, gc = scan.c(), grid_c(grid)
    check(lib().uwb_das_dmas(ctypes.byref(sc), ctypes.byref(gc), window, out_das.data_ptr(), out_dmas.data_ptr(),
                             _stream(out_das.device)), "uwb_das_dmas")
    return out_das, out_dmas


def das(scan, grid, window=11, out=None):
    return image(scan, grid, UWB_DAS, window, out)


def dmas(scan, grid, window=11, out=None):
    return image(scan, grid, UWB_DMAS, window, out)


def mvdr(scan, grid, window=11, out=None):
    return image(scan, grid, UWB_MVDR, window, out)


def image_batch(batch: DeviceBatch, grid, beamformer: int, window: int = 11, out=None, bc=None):
    """bc: the batch's descriptor (batch.c()), built once by callers that launch repeatedly or capture the call
    in a graph (building it reads the per-scan parameters back to the host)."""
    if out is None:
        out = torch.empty((batch.n_scans,) + _img_shape(grid), dtype=torch.float32, device=batch.traces.device)
    _need_cuda(out, "out", numel=batch.n_scans * _nvox(grid))
    fn = getattr(lib(), _IMAGE_FN[_bf(beamformer)] + "_batch")
    bc, gc = (bc if bc is not None else batch.c()), grid_c(grid)
    check(fn(ctypes.byref(bc), ctypes.byref(gc), window, out.data_ptr(), _stream(out.device)), "image_batch")
    return out


def das_dmas_batch(batch: DeviceBatch, grid, window: int = 11, out_das=None, out_dmas=None, bc=None):
    """DAS and DMAS images of a batch from one launch (the DMAS kernel's running sums are the DAS sums).
    Returns (das, dmas), each [n_scans, nz, ny, nx] float32."""
    shape = (batch.n_scans,) + _img_shape(grid)
    if out_das is None:
        out_das = torch.empty(shape, dtype=torch.float32, device=batch.traces.device)
    if out_dmas is None:
        out_dmas = torch.empty(shape, dtype=torch.float32, device=batch.traces.device)
    _need_cuda(out_das, "out_das", numel=batch.n_scans * _nvox(grid))
    _need_cuda(out_dmas, "out_dmas", numel=batch.n_scans * _nvox(grid))
    bc, gc = (bc if bc is not None else batch.c()), grid_c(grid)
    check(lib().uwb_das_dmas_batch(ctypes.byref(bc), ctypes.byref(gc), window, out_das.data_ptr(),
                                   out_dmas.data_ptr(), _stream(out_das.device)), "das_dmas_batch")
    return out_das, out_dmas


def das_batch(batch, grid, window=11, out=None):
    return image_batch(batch, grid, UWB_DAS, window, out)


def dmas_batch(batch, grid, window=11, out=None):
    return image_batch(batch, grid, UWB_DMAS, window, out)


@dataclasses.dataclass
class Peak:
    index: int
    value: float
    value32: float
    candidates: int


def _peaks(buf: torch.Tensor, n: int):
    raw = buf.cpu().numpy().tobytes()
    sz = ctypes.sizeof(UwbPeak)
    out = []
    for i in range(n):
        p = UwbPeak.from_buffer_copy(raw[i * sz:(i + 1) * sz])
        out.append(Peak(int(p.index), float(p.value), float(p.value32), int(p.candidates)))
    return out


class Workspace:
    """Grow-only device scratch buffer reused across calls."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != torch.device(device):
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        return self.buf


_ws = Workspace()


def argmax_async(scan: DeviceScan, grid, img: torch.Tensor, beamformer: int, window: int = 11,
                 out: torch.Tensor | None = None, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Enqueue the FP64-decided argmax; returns the device buffer holding one uwb_peak."""
    gc, sc = grid_c(grid), scan.c()
    need = lib().uwb_argmax_workspace_bytes(ctypes.byref(gc), 1)
    ws = workspace if workspace is not None else _ws.get(need, img.device)
    if out is None:
        out = torch.empty(ctypes.sizeof(UwbPeak), dtype=torch.uint8, device=img.device)
    _need_cuda(img, "img", numel=_nvox(grid))
    _need_bytes(out, "out", ctypes.sizeof(UwbPeak))
    _need_bytes(ws, "workspace", need)
    check(lib().uwb_argmax(ctypes.byref(sc), ctypes.byref(gc), window, beamformer, img.data_ptr(), out.data_ptr(),
                           ws.data_ptr(), ws.numel(), _stream(img.device)), "uwb_argmax")
    return out


def argmax(scan, grid, img, beamformer, window=11) -> Peak:
    return _peaks(argmax_async(scan, grid, img, beamformer, window), 1)[0]


def argmax_batch_async(batch: DeviceBatch, grid, img: torch.Tensor, beamformer: int, window: int = 11,
                       out=None, workspace=None, bc=None) -> torch.Tensor:
    gc = grid_c(grid)
    bc = bc if bc is not None else batch.c()
    need = lib().uwb_argmax_workspace_bytes(ctypes.byref(gc), batch.n_scans)
    ws = workspace if workspace is not None else _ws.get(need, img.device)
    if out is None:
        out = torch.empty(ctypes.sizeof(UwbPeak) * batch.n_scans, dtype=torch.uint8, device=img.device)
    _need_cuda(img, "img", numel=batch.n_scans * _nvox(grid))
    _need_bytes(out, "out", ctypes.sizeof(UwbPeak) * batch.n_scans)
    _need_bytes(ws, "workspace", need)
    check(lib().uwb_argmax_batch(ctypes.byref(bc), ctypes.byref(gc), window, beamformer, img.data_ptr(),
                                 out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(img.device)), "uwb_argmax_batch")
    return out


def image_tiles(grid) -> int:
    """Tiles per scan of the full-resolution DAS / DMAS launch (length of one scan's tile maxima)."""
    gc = grid_c(grid)
    n = int(lib().uwb_image_tiles(ctypes.byref(gc)))
    check(min(n, 0), "uwb_image_tiles")
    return n


def das_dmas_batch_tilemax(batch: DeviceBatch, grid, window: int = 11, out_das=None, out_dmas=None, tmax_das=None,
                           tmax_dmas=None, bc=None):
    """das_dmas_batch that also writes every tile's FP32 maximum of each image.
    Returns (das, dmas, tmax_das, tmax_dmas)."""
    shape = (batch.n_scans,) + _img_shape(grid)
    dev = batch.traces.device
    nt = image_tiles(grid)
    if out_das is None:
        out_das = torch.empty(shape, dtype=torch.float32, device=dev)
    if out_dmas is None:
        out_dmas = torch.empty(shape, dtype=torch.float32, device=dev)
    if tmax_das is None:
        tmax_das = torch.empty((batch.n_scans, nt), dtype=torch.float32, device=dev)
    if tmax_dmas is None:
        tmax_dmas = torch.empty((batch.n_scans, nt), dtype=torch.float32, device=dev)
    for t, name, n in ((out_das, "out_das", _nvox(grid)), (out_dmas, "out_dmas", _nvox(grid)),
                       (tmax_das, "tmax_das", nt), (tmax_dmas, "tmax_dmas", nt)):
        _need_cuda(t, name, numel=batch.n_scans * n)
    bc, gc = (bc if bc is not None else batch.c()), grid_c(grid)
    check(lib().uwb_das_dmas_batch_tilemax(ctypes.byref(bc), ctypes.byref(gc), window, out_das.data_ptr(),
                                           out_dmas.data_ptr(), tmax_das.data_ptr(), tmax_dmas.data_ptr(),
                                           _stream(out_das.device)), "uwb_das_dmas_batch_tilemax")
    return out_das, out_dmas, tmax_das, tmax_dmas


def argmax_batch_tilemax_async(batch: DeviceBatch, grid, img: torch.Tensor, tmax: torch.Tensor, beamformer: int,
                               window: int = 11, out=None, workspace=None, bc=None) -> torch.Tensor:
    """argmax_batch_async taking the image's tile maxima (das_dmas_batch_tilemax) instead of a pass over it."""
    gc = grid_c(grid)
    bc = bc if bc is not None else batch.c()
    need = lib().uwb_argmax_tilemax_workspace_bytes(ctypes.byref(gc), batch.n_scans)
    ws = workspace if workspace is not None else _ws.get(need, img.device)
    if out is None:
        out = torch.empty(ctypes.sizeof(UwbPeak) * batch.n_scans, dtype=torch.uint8, device=img.device)
    _need_cuda(img, "img", numel=batch.n_scans * _nvox(grid))
    _need_cuda(tmax, "tmax", numel=batch.n_scans * image_tiles(grid))
    _need_bytes(out, "out", ctypes.sizeof(UwbPeak) * batch.n_scans)
    _need_bytes(ws, "workspace", need)
    check(lib().uwb_argmax_batch_tilemax(ctypes.byref(bc), ctypes.byref(gc), window, beamformer, img.data_ptr(),
                                         tmax.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                                         _stream(img.device)), "uwb_argmax_batch_tilemax")
    return out


ARGMAX_SCRATCH_BYTES = 4 << 20   # UWB_ARGMAX_SCRATCH_BYTES: the allocation-free detection's scratch limit


def argmax_batch_noalloc_async(batch: DeviceBatch, grid, img: torch.Tensor, beamformer: int, out: torch.Tensor,
                               window: int = 11, bc=None) -> torch.Tensor:
    """The allocation-free detection (uwb_argmax_batch_noalloc): the library's own device scratch instead of a
    workspace; the caller passes the output records (one uwb_peak per scan), and nothing is allocated here."""
    gc = grid_c(grid)
    bc = bc if bc is not None else batch.c()
    _need_cuda(img, "img", numel=batch.n_scans * _nvox(grid))
    _need_bytes(out, "out", ctypes.sizeof(UwbPeak) * batch.n_scans)
    check(lib().uwb_argmax_batch_noalloc(ctypes.byref(bc), ctypes.byref(gc), window, beamformer, img.data_ptr(),
                                         out.data_ptr(), _stream(img.device)), "uwb_argmax_batch_noalloc")
    return out


def argmax_batch(batch, grid, img, beamformer, window=11):
    return _peaks(argmax_batch_async(batch, grid, img, beamformer, window), batch.n_scans)


def probe_lds_read(width: int = 16, iters: int = 4096, n_groups: int = 256 * 20):
    """Device LDS read bandwidth: (bytes/s over the device, shader clock Hz measured during the loop)."""
    bps, hz = ctypes.c_double(), ctypes.c_double()
    check(lib().uwb_probe_lds_read(int(width), int(iters), int(n_groups), ctypes.byref(bps), ctypes.byref(hz),
                                   _stream()), "uwb_probe_lds_read")
    return float(bps.value), float(hz.value)


def auto_decimation(min_tumour: float, pitch: float) -> int:
    r = lib().uwb_auto_decimation(float(min_tumour), float(pitch))
    check(min(r, 0), "uwb_auto_decimation")
    return r


# ----------------------------------------------------------------------------------
# segment walk
# ----------------------------------------------------------------------------------

@dataclasses.dataclass
class SegmentTree:
    beamformer: int = 0
    walk: str = "per_level"
    coarse: int = 8
    decimation: int = 0
    min_tumour: float = 0.01
    max_depth: int = 0
    metric: str = "max"
    term: str = "fixed"
    frame_level: float = 0.0
    frame_final: float = 0.25

    def c(self) -> UwbSegmentTree:
        return UwbSegmentTree(int(self.beamformer), WALKS[self.walk], int(self.coarse), int(self.decimation),
                              float(self.min_tumour), int(self.max_depth), METRICS[self.metric], TERMS[self.term],
                              float(self.frame_level), float(self.frame_final))


@dataclasses.dataclass
class SegmentResult:
    n_levels: int
    term_level: int
    decimation: int
    n_samples_level0: int
    child: list
    boxes: list
    scores: list
    wb: list
    roi: tuple
    argmax: int
    peak: float
    voxels_evaluated: int
    learned_mask: int = 0
    guard_hits: int = 0
    roi_image: np.ndarray | None = None


def _results(buf: torch.Tensor, n: int, n_child: int):
    raw = buf.cpu().numpy().tobytes()
    sz = ctypes.sizeof(UwbSegmentResult)
    out = []
    for i in range(n):
        r = UwbSegmentResult.from_buffer_copy(raw[i * sz:(i + 1) * sz])
        made = int(r.term_level)
        out.append(SegmentResult(
            int(r.n_levels), made, int(r.decimation), int(r.n_samples_level0),
            [int(r.child[j]) for j in range(made)],
            [tuple(int(x) for x in r.box[j]) for j in range(made + 1)],
            [[float(r.score[j][c]) for c in range(n_child)] for j in range(made)],
            [(float(r.wb[j][0]), float(r.wb[j][1])) for j in range(int(r.n_wb))],
            tuple(int(x) for x in r.roi), int(r.argmax), float(r.peak), int(r.voxels_evaluated),
            int(r.learned_mask), int(r.guard_hits)))
    return out


def roi_capacity(grid, tree: SegmentTree) -> int:
    gc, tc = grid_c(grid), tree.c()
    cap = lib().uwb_segment_roi_capacity(ctypes.byref(gc), ctypes.byref(tc))
    check(int(min(cap, 0)), "uwb_segment_roi_capacity")
    return int(cap)


def segment_refine_batch_async(batch: DeviceBatch, grid, tree: SegmentTree, window: int = 11, out=None,
                               roi_img=None, workspace=None, bc=None):
    gc, tc = grid_c(grid), tree.c()
    bc = bc if bc is not None else batch.c()
    dev = batch.traces.device
    cap = roi_capacity(grid, tree)
    need = lib().uwb_segment_workspace_bytes(ctypes.byref(gc), ctypes.byref(tc), batch.n_scans)
    ws = workspace if workspace is not None else _ws.get(need, dev)
    if out is None:
        out = torch.empty(ctypes.sizeof(UwbSegmentResult) * batch.n_scans, dtype=torch.uint8, device=dev)
    _need_bytes(out, "out", ctypes.sizeof(UwbSegmentResult) * batch.n_scans)
    _need_bytes(ws, "workspace", need)
    rp = 0
    if roi_img is not None:
        _need_cuda(roi_img, "roi_img")
        if roi_img.numel() < cap * batch.n_scans:
            raise ValueError("roi_img smaller than n_scans * roi capacity")
        rp = roi_img.data_ptr()
    check(lib().uwb_segment_refine_batch(ctypes.byref(bc), ctypes.byref(gc), window, ctypes.byref(tc),
                                         out.data_ptr(), rp, cap, ws.data_ptr(), ws.numel(), _stream(dev)),
          "uwb_segment_refine_batch")
    return out, cap


def segment_refine_batch(batch, grid, tree: SegmentTree, window=11, want_roi=False):
    dev = batch.traces.device
    roi = None
    if want_roi:
        roi = torch.empty(roi_capacity(grid, tree) * batch.n_scans, dtype=torch.float32, device=dev)
    out, cap = segment_refine_batch_async(batch, grid, tree, window, roi_img=roi)
    n_child = 4 if int(grid.dims[2]) == 1 else 8
    res = _results(out, batch.n_scans, n_child)
    if want_roi:
        r = roi.cpu().numpy()
        for i, x in enumerate(res):
            b = x.roi
            shape = (b[5] - b[4], b[3] - b[2], b[1] - b[0])
            x.roi_image = r[i * cap:i * cap + int(np.prod(shape))].reshape(shape)
    return res


def segment_composite_batch(batch: DeviceBatch, grid, tree: SegmentTree, window: int = 11):
    """The batched walk plus its mixed-resolution image: (results, composite [n, nz, ny, nx] fp32 tensor)."""
    gc, tc = grid_c(grid), tree.c()
    bc = batch.c()
    dev = batch.traces.device
    cap = roi_capacity(grid, tree)
    need = lib().uwb_segment_workspace_bytes(ctypes.byref(gc), ctypes.byref(tc), batch.n_scans)
    ws = _ws.get(need, dev)
    out = torch.empty(ctypes.sizeof(UwbSegmentResult) * batch.n_scans, dtype=torch.uint8, device=dev)
    img = torch.empty((batch.n_scans,) + _img_shape(grid), dtype=torch.float32, device=dev)
    check(lib().uwb_segment_composite_batch(ctypes.byref(bc), ctypes.byref(gc), window, ctypes.byref(tc),
                                            out.data_ptr(), 0, cap, ws.data_ptr(), ws.numel(), img.data_ptr(),
                                            _stream(dev)), "uwb_segment_composite_batch")
    return _results(out, batch.n_scans, 4 if int(grid.dims[2]) == 1 else 8), img


def tumour_check_batch(batch: DeviceBatch, grid, tree: SegmentTree, d1: int, d2: int, window: int = 11):
    """The two-decimation check of the three-phase walk: (agree [n] bool array, results with d1, results with d2)."""
    gc, tc = grid_c(grid), tree.c()
    bc = batch.c()
    dev = batch.traces.device
    n = batch.n_scans
    need = lib().uwb_tumour_check_workspace_bytes(ctypes.byref(gc), ctypes.byref(tc), int(d1), int(d2), n)
    if need == 0:
        raise UwbError(-1, "uwb_tumour_check_workspace_bytes")
    ws = _ws.get(need, dev)
    out = torch.empty(ctypes.sizeof(UwbSegmentResult) * 2 * n, dtype=torch.uint8, device=dev)
    agree = torch.empty(n, dtype=torch.int32, device=dev)
    check(lib().uwb_tumour_check_batch(ctypes.byref(bc), ctypes.byref(gc), window, ctypes.byref(tc), int(d1), int(d2),
                                       out.data_ptr(), agree.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dev)),
          "uwb_tumour_check_batch")
    nc = 4 if int(grid.dims[2]) == 1 else 8
    res = _results(out, 2 * n, nc)
    return agree.cpu().numpy().astype(bool), res[:n], res[n:]


def segment_refine(scan: DeviceScan, grid, tree: SegmentTree, window=11, want_roi=False):
    gc, tc, sc = grid_c(grid), tree.c(), scan.c()
    dev = scan.traces.device
    cap = roi_capacity(grid, tree)
    need = lib().uwb_segment_workspace_bytes(ctypes.byref(gc), ctypes.byref(tc), 1)
    ws = _ws.get(need, dev)
    out = torch.empty(ctypes.sizeof(UwbSegmentResult), dtype=torch.uint8, device=dev)
    roi = torch.empty(cap, dtype=torch.float32, device=dev) if want_roi else None
    check(lib().uwb_segment_refine(ctypes.byref(sc), ctypes.byref(gc), window, ctypes.byref(tc), out.data_ptr(),
                                   roi.data_ptr() if roi is not None else 0, cap, ws.data_ptr(), ws.numel(),
                                   _stream(dev)), "uwb_segment_refine")
    res = _results(out, 1, 4 if int(grid.dims[2]) == 1 else 8)[0]
    if want_roi:
        b = res.roi
        shape = (b[5] - b[4], b[3] - b[2], b[1] - b[0])
        res.roi_image = roi[:int(np.prod(shape))].cpu().numpy().reshape(shape)
    return res


# ----------------------------------------------------------------------------------
# batched serving of uneven scans (persistent, graph-captured launch)
# ----------------------------------------------------------------------------------

class BatchPlan:
    """One plan over many scans of uneven shape: items are (DeviceScan, grid, out image tensor)."""

    def __init__(self, items, beamformer: int, window: int = 11, config: dict | None = None):
        self._keep = list(items)
        n = len(self._keep)
        arr = (UwbBatchItem * n)()
        for k, (sc, g, out) in enumerate(self._keep):
            _need_cuda(out, "out", numel=_nvox(g))
            arr[k] = UwbBatchItem(sc.c(), grid_c(g), out.data_ptr())
        self.device = self._keep[0][2].device
        self._h = ctypes.c_void_p()
        cfg = None
        if config is not None:
            cfg = UwbBatchConfig(config["vpl"], config["wgs_per_cu"], config["lds_kb"], config["order"])
        check(lib().uwb_batch_plan_create(ctypes.byref(self._h), arr, n, beamformer, window,
                                          ctypes.byref(cfg) if cfg is not None else None), "uwb_batch_plan_create")
        self.n = n

    def run(self):
        check(lib().uwb_batch_run(self._h, _stream(self.device)), "uwb_batch_run")

    @property
    def config(self) -> dict:
        c = UwbBatchConfig()
        check(lib().uwb_batch_get_config(self._h, ctypes.byref(c)), "uwb_batch_get_config")
        return {"vpl": c.vpl, "wgs_per_cu": c.wgs_per_cu, "lds_kb": c.lds_kb, "order": c.order}

    def set_config(self, config: dict):
        c = UwbBatchConfig(config["vpl"], config["wgs_per_cu"], config["lds_kb"], config["order"])
        check(lib().uwb_batch_set_config(self._h, ctypes.byref(c)), "uwb_batch_set_config")

    def autotune(self, reps: int = 3) -> dict:
        c = UwbBatchConfig()
        check(lib().uwb_batch_autotune(self._h, reps, _stream(self.device), ctypes.byref(c)), "uwb_batch_autotune")
        return {"vpl": c.vpl, "wgs_per_cu": c.wgs_per_cu, "lds_kb": c.lds_kb, "order": c.order}

    def timestamps_ns(self) -> np.ndarray:
        out = (ctypes.c_int64 * self.n)()
        check(lib().uwb_batch_timestamps(self._h, out, _stream(self.device)), "uwb_batch_timestamps")
        return np.frombuffer(out, dtype=np.int64).copy()

    def close(self):
        if self._h:
            lib().uwb_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------------
# learned segment proposer (BF16 CNN)
# ----------------------------------------------------------------------------------

def to_bf16(t: torch.Tensor) -> torch.Tensor:
    """Round a float tensor to bfloat16 (nearest, ties to even) on its device."""
    return t.to(torch.bfloat16).contiguous()


class CNN:
    """Device-resident CNN (parameters, Adam state, activation buffers for up to max_batch samples)."""

    def __init__(self, max_batch: int, init_params):
        p = np.ascontiguousarray(np.asarray(init_params, dtype=np.float32))
        self.n_params = int(lib().uwb_cnn_param_count())
        if p.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        self._h = ctypes.c_void_p()
        check(lib().uwb_cnn_create(ctypes.byref(self._h), int(max_batch), p.ctypes.data_as(ctypes.c_void_p)),
              "uwb_cnn_create")
        self.max_batch = int(max_batch)

    @staticmethod
    def _x(x: torch.Tensor):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.bfloat16 and x.is_contiguous()):
            raise TypeError("x must be a contiguous CUDA bfloat16 tensor [n, 32, 32]")
        if x.dim() != 3 or tuple(x.shape[1:]) != (32, 32):
            raise ValueError("x must be [n, 32, 32]")
        return x

    def forward(self, x: torch.Tensor, probs: torch.Tensor | None = None) -> torch.Tensor:
        x = self._x(x)
        n = int(x.shape[0])
        if probs is None:
            probs = torch.empty((n, 4), dtype=torch.float32, device=x.device)
        _need_cuda(probs, "probs", numel=4 * n)
        check(lib().uwb_cnn_forward(self._h, x.data_ptr(), n, probs.data_ptr(), _stream(x.device)), "uwb_cnn_forward")
        return probs

    def gradients(self, x: torch.Tensor, labels: torch.Tensor):
        x = self._x(x)
        n = int(x.shape[0])
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _need_cuda(labels, "labels", torch.int32, numel=n)
        check(lib().uwb_cnn_gradients(self._h, x.data_ptr(), labels.data_ptr(), n, g.data_ptr(), loss.data_ptr(),
                                      _stream(x.device)), "uwb_cnn_gradients")
        return g, loss

    def train_step(self, x: torch.Tensor, labels: torch.Tensor, lr: float, loss: torch.Tensor | None = None):
        x = self._x(x)
        _need_cuda(labels, "labels", torch.int32, numel=int(x.shape[0]))
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=x.device)
        check(lib().uwb_cnn_train_step(self._h, x.data_ptr(), labels.data_ptr(), int(x.shape[0]), float(lr),
                                       loss.data_ptr(), _stream(x.device)), "uwb_cnn_train_step")
        return loss

    def get_state(self):
        th = np.zeros(self.n_params, np.float32)
        m = np.zeros(self.n_params, np.float32)
        v = np.zeros(self.n_params, np.float32)
        step = ctypes.c_int64()
        check(lib().uwb_cnn_get_state(self._h, th.ctypes.data_as(ctypes.c_void_p), m.ctypes.data_as(ctypes.c_void_p),
                                      v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(step), _stream()),
              "uwb_cnn_get_state")
        return {"theta": th, "m": m, "v": v, "step": int(step.value)}

    def set_state(self, st: dict):
        th, m, v = (np.ascontiguousarray(st[k], dtype=np.float32) for k in ("theta", "m", "v"))
        check(lib().uwb_cnn_set_state(self._h, th.ctypes.data_as(ctypes.c_void_p), m.ctypes.data_as(ctypes.c_void_p),
                                      v.ctypes.data_as(ctypes.c_void_p), int(st["step"]), _stream()),
              "uwb_cnn_set_state")

    def weights_ptr(self) -> int:
        return int(lib().uwb_cnn_weights_bf16(self._h) or 0)

    def close(self):
        if self._h:
            lib().uwb_cnn_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------------
# learned walk, its training inputs, and the GPU scan generator
# ----------------------------------------------------------------------------------

def learned_refine_batch(batch: DeviceBatch, grid, tree: SegmentTree, cnn: CNN, threshold: float,
                         window: int = 11, want_roi: bool = False, out=None, workspace=None, bc=None,
                         sync: bool = True):
    """The per-level walk (g = 32, planar, fixed depth) whose splits the CNN decides when confident."""
    gc, tc = grid_c(grid), tree.c()
    bc = bc if bc is not None else batch.c()
    dev = batch.traces.device
    cap = roi_capacity(grid, tree)
    need = lib().uwb_learned_workspace_bytes(ctypes.byref(gc), ctypes.byref(tc), batch.n_scans)
    if need == 0:
        raise UwbError(-5, "uwb_learned_workspace_bytes")
    ws = workspace if workspace is not None else _ws.get(need, dev)
    if out is None:
        out = torch.empty(ctypes.sizeof(UwbSegmentResult) * batch.n_scans, dtype=torch.uint8, device=dev)
    _need_bytes(out, "out", ctypes.sizeof(UwbSegmentResult) * batch.n_scans)
    _need_bytes(ws, "workspace", need)
    roi = torch.empty(cap * batch.n_scans, dtype=torch.float32, device=dev) if want_roi else None
    check(lib().uwb_learned_refine_batch(ctypes.byref(bc), ctypes.byref(gc), window, ctypes.byref(tc), cnn._h,
                                         float(threshold), out.data_ptr(), roi.data_ptr() if roi is not None else 0,
                                         cap, ws.data_ptr(), ws.numel(), _stream(dev)), "uwb_learned_refine_batch")
    if not sync:
        return out
    res = _results(out, batch.n_scans, 4)
    if want_roi:
        r = roi.cpu().numpy()
        for i, x in enumerate(res):
            b = x.roi
            shape = (b[5] - b[4], b[3] - b[2], b[1] - b[0])
            x.roi_image = r[i * cap:i * cap + int(np.prod(shape))].reshape(shape)
    return res


def cnn_input_levels(grid) -> int:
    gc = grid_c(grid)
    n = int(lib().uwb_cnn_input_levels(ctypes.byref(gc)))
    check(min(n, 0), "uwb_cnn_input_levels")
    return n


def cnn_training_inputs(batch: DeviceBatch, grid, peaks: torch.Tensor, window: int = 11, bc=None, x=None,
                        labels=None):
    """Per-level 32 x 32 DAS lattices along the path to each scan's target voxel, and the true children.
    peaks: device buffer of uwb_peak records (e.g. from argmax_batch_async).  Returns (x [n*L,32,32] bf16,
    labels [n*L] int32), written into x / labels when given."""
    gc = grid_c(grid)
    bc = bc if bc is not None else batch.c()
    dev = batch.traces.device
    L = cnn_input_levels(grid)
    n = batch.n_scans
    if x is None:
        x = torch.empty((n * L, 32, 32), dtype=torch.bfloat16, device=dev)
    if labels is None:
        labels = torch.empty(n * L, dtype=torch.int32, device=dev)
    lab = labels
    if not (x.is_cuda and x.dtype == torch.bfloat16 and x.is_contiguous() and x.numel() >= n * L * 1024):
        raise TypeError("x must be a contiguous CUDA bfloat16 tensor of n * levels * 1024 elements")
    _need_cuda(lab, "labels", torch.int32)
    if lab.numel() < n * L:
        raise ValueError("labels smaller than n * levels")
    check(lib().uwb_cnn_training_inputs(ctypes.byref(bc), ctypes.byref(gc), window, peaks.data_ptr(), x.data_ptr(),
                                        lab.data_ptr(), _stream(dev)), "uwb_cnn_training_inputs")
    return x, lab


@dataclasses.dataclass
class DiscRecipe:
    """A planar disc recipe: ring antennas, tumour + clutter point scatterers, white noise."""
    n_samp: int
    n_clutter: int
    v: float
    dt: float
    t0: float
    radius: float
    snr_db: float
    pulse_f0: float
    pulse_sigma: float
    pulse_peak: float
    salt: int

    def c(self, n_ant: int) -> UwbGenRecipe:
        return UwbGenRecipe(int(n_ant), int(self.n_samp), int(self.n_clutter), self.v, self.dt, self.t0,
                            self.radius, self.snr_db, self.pulse_f0, self.pulse_sigma, self.pulse_peak,
                            int(self.salt))


def generate_disc_scans(recipe: DiscRecipe, ant_pos: torch.Tensor, seeds, want_tumours: bool = True):
    """Synthesise len(seeds) scans on the GPU.  ant_pos [M,3] f32 on the device.  Returns (DeviceBatch,
    tumours [n,3] f64 or None)."""
    _need_cuda(ant_pos, "ant_pos")
    dev = ant_pos.device
    sd = torch.as_tensor(np.asarray(seeds, dtype=np.uint64).view(np.int64)).to(dev)
    n, m = int(sd.numel()), int(ant_pos.shape[0])
    tr = torch.empty((n, m, int(recipe.n_samp)), dtype=torch.float32, device=dev)
    tum = torch.empty((n, 3), dtype=torch.float64, device=dev) if want_tumours else None
    rc = recipe.c(m)
    check(lib().uwb_generate_disc_scans(ctypes.byref(rc), ant_pos.data_ptr(), sd.data_ptr(), n, tr.data_ptr(),
                                        tum.data_ptr() if tum is not None else 0, _stream(dev)),
          "uwb_generate_disc_scans")
    par = torch.tensor([[recipe.dt, recipe.t0, recipe.v]] * n, dtype=torch.float64, device=dev)
    pos = ant_pos.unsqueeze(0).expand(n, m, 3).contiguous()
    return DeviceBatch(pos, tr, par), tum


# ----------------------------------------------------------------------------------
# multistatic scans: M antennas, M^2 traces (channel i*M + j: transmit on i, receive on j)
# ----------------------------------------------------------------------------------

def _ms_scan_c(scan: DeviceScan) -> UwbScan:
    _need_cuda(scan.ant_pos, "ant_pos")
    _need_cuda(scan.traces, "traces")
    m = int(scan.ant_pos.shape[0])
    if scan.traces.shape[0] != m * m:
        raise ValueError("a multistatic scan holds M^2 traces")
    return UwbScan(m, scan.traces.shape[1], scan.ant_pos.data_ptr(), scan.traces.data_ptr(), scan.dt, scan.t0,
                   scan.v)


def _ms_batch_c(batch: DeviceBatch) -> UwbScanBatch:
    bc = batch.c()
    m = int(batch.ant_pos.shape[1])
    if batch.traces.shape[1] != m * m:
        raise ValueError("multistatic scans hold M^2 traces")
    bc.n_ant = m
    return bc


def image_multistatic(scan: DeviceScan, grid, beamformer: int, window: int = 11, out=None):
    """Multistatic DAS (Eq. (4)) or DMAS image [nz, ny, nx] fp32."""
    if out is None:
        out = torch.empty(_img_shape(grid), dtype=torch.float32, device=scan.traces.device)
    _need_cuda(out, "out", numel=_nvox(grid))
    fn = getattr(lib(), _IMAGE_FN[_bf(beamformer)] + "_multistatic")
    sc, gc = _ms_scan_c(scan), grid_c(grid)
    check(fn(ctypes.byref(sc), ctypes.byref(gc), window, out.data_ptr(), _stream(out.device)), "image_multistatic")
    return out


def das_dmas_multistatic_batch(batch: DeviceBatch, grid, window: int = 11, out_das=None, out_dmas=None, bc=None):
    """Both multistatic images from one launch. Returns (das, dmas)."""
    shape = (batch.n_scans,) + _img_shape(grid)
    if out_das is None:
        out_das = torch.empty(shape, dtype=torch.float32, device=batch.traces.device)
    if out_dmas is None:
        out_dmas = torch.empty(shape, dtype=torch.float32, device=batch.traces.device)
    _need_cuda(out_das, "out_das", numel=batch.n_scans * _nvox(grid))
    _need_cuda(out_dmas, "out_dmas", numel=batch.n_scans * _nvox(grid))
    bc = bc if bc is not None else _ms_batch_c(batch)
    gc = grid_c(grid)
    check(lib().uwb_das_dmas_multistatic_batch(ctypes.byref(bc), ctypes.byref(gc), window, out_das.data_ptr(),
                                               out_dmas.data_ptr(), _stream(out_das.device)),
          "das_dmas_multistatic_batch")
    return out_das, out_dmas


def image_multistatic_batch(batch: DeviceBatch, grid, beamformer: int, window: int = 11, out=None, bc=None):
    if out is None:
        out = torch.empty((batch.n_scans,) + _img_shape(grid), dtype=torch.float32, device=batch.traces.device)
    _need_cuda(out, "out", numel=batch.n_scans * _nvox(grid))
    fn = getattr(lib(), _IMAGE_FN[_bf(beamformer)] + "_multistatic_batch")
    bc = bc if bc is not None else _ms_batch_c(batch)
    gc = grid_c(grid)
    check(fn(ctypes.byref(bc), ctypes.byref(gc), window, out.data_ptr(), _stream(out.device)),
          "image_multistatic_batch")
    return out


def argmax_multistatic(scan: DeviceScan, grid, img, beamformer: int, window: int = 11) -> Peak:
    gc, sc = grid_c(grid), _ms_scan_c(scan)
    need = lib().uwb_argmax_workspace_bytes(ctypes.byref(gc), 1)
    ws = _ws.get(need, img.device)
    out = torch.empty(ctypes.sizeof(UwbPeak), dtype=torch.uint8, device=img.device)
    _need_cuda(img, "img", numel=_nvox(grid))
    check(lib().uwb_argmax_multistatic(ctypes.byref(sc), ctypes.byref(gc), window, beamformer, img.data_ptr(),
                                       out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(img.device)),
          "uwb_argmax_multistatic")
    return _peaks(out, 1)[0]


def argmax_multistatic_batch_async(batch: DeviceBatch, grid, img, beamformer: int, window: int = 11, bc=None):
    gc = grid_c(grid)
    bc = bc if bc is not None else _ms_batch_c(batch)
    need = lib().uwb_argmax_workspace_bytes(ctypes.byref(gc), batch.n_scans)
    ws = _ws.get(need, img.device)
    out = torch.empty(ctypes.sizeof(UwbPeak) * batch.n_scans, dtype=torch.uint8, device=img.device)
    _need_cuda(img, "img", numel=batch.n_scans * _nvox(grid))
    check(lib().uwb_argmax_multistatic_batch(ctypes.byref(bc), ctypes.byref(gc), window, beamformer, img.data_ptr(),
                                             out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(img.device)),
          "uwb_argmax_multistatic_batch")
    return out


def segment_refine_multistatic(scan: DeviceScan, grid, tree: SegmentTree, window: int = 11, want_roi=False):
    gc, tc, sc = grid_c(grid), tree.c(), _ms_scan_c(scan)
    dev = scan.traces.device
    cap = roi_capacity(grid, tree)
    need = lib().uwb_segment_workspace_bytes(ctypes.byref(gc), ctypes.byref(tc), 1)
    ws = _ws.get(need, dev)
    out = torch.empty(ctypes.sizeof(UwbSegmentResult), dtype=torch.uint8, device=dev)
    roi = torch.empty(cap, dtype=torch.float32, device=dev) if want_roi else None
    check(lib().uwb_segment_refine_multistatic(ctypes.byref(sc), ctypes.byref(gc), window, ctypes.byref(tc),
                                               out.data_ptr(), roi.data_ptr() if roi is not None else 0, cap,
                                               ws.data_ptr(), ws.numel(), _stream(dev)),
          "uwb_segment_refine_multistatic")
    res = _results(out, 1, 4 if int(grid.dims[2]) == 1 else 8)[0]
    if want_roi:
        b = res.roi
        shape = (b[5] - b[4], b[3] - b[2], b[1] - b[0])
        res.roi_image = roi[:int(np.prod(shape))].cpu().numpy().reshape(shape)
    return res


def segment_refine_multistatic_batch_async(batch: DeviceBatch, grid, tree: SegmentTree, window: int = 11, bc=None):
    gc, tc = grid_c(grid), tree.c()
    bc = bc if bc is not None else _ms_batch_c(batch)
    dev = batch.traces.device
    cap = roi_capacity(grid, tree)
    need = lib().uwb_segment_workspace_bytes(ctypes.byref(gc), ctypes.byref(tc), batch.n_scans)
    ws = _ws.get(need, dev)
    out = torch.empty(ctypes.sizeof(UwbSegmentResult) * batch.n_scans, dtype=torch.uint8, device=dev)
    check(lib().uwb_segment_refine_multistatic_batch(ctypes.byref(bc), ctypes.byref(gc), window, ctypes.byref(tc),
                                                     out.data_ptr(), 0, cap, ws.data_ptr(), ws.numel(), _stream(dev)),
          "uwb_segment_refine_multistatic_batch")
    return out
