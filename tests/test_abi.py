"""C ABI checks that need no GPU: the library loads, exports every declared entry
point, validates its arguments before touching the device, and its pure host
functions (automatic decimation, sizes) give the documented values."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "uwb.h")
FAKE = 0x1000    # a non-null pointer value: never dereferenced because validation fails first


def _abi():
    from paper_1709_02549_amd import _abi as a
    return a


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(uwb_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _abi().lib()
    names = declared_functions()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    for n in names:
        assert n in _abi().PROTOTYPES, f"binding has no prototype for {n}"


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors agree with the C compiler's sizeof / offsetof for every struct of uwb.h."""
    import subprocess
    a = _abi()
    structs = {"uwb_scan": a.UwbScan, "uwb_scan_batch": a.UwbScanBatch, "uwb_grid": a.UwbGrid,
               "uwb_peak": a.UwbPeak, "uwb_segment_tree": a.UwbSegmentTree, "uwb_segment_result": a.UwbSegmentResult,
               "uwb_batch_item": a.UwbBatchItem, "uwb_batch_config": a.UwbBatchConfig,
               "uwb_gen_recipe": a.UwbGenRecipe}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def _scan(**kw):
    a = _abi()
    d = dict(n_ant=4, n_samp=64, ant_pos=FAKE, traces=FAKE, dt=2e-11, t0=0.0, v=1e8)
    d.update(kw)
    return a.UwbScan(**d)


def _grid(dims=(8, 8, 1), pitch=(1e-3, 1e-3, 1e-3), origin=(0.0, 0.0, 0.0)):
    a = _abi()
    return a.UwbGrid((ctypes.c_double * 3)(*origin), (ctypes.c_double * 3)(*pitch), (ctypes.c_int32 * 3)(*dims))


@pytest.mark.parametrize("fn", ["uwb_das", "uwb_dmas"])
def test_image_argument_errors(fn):
    a = _abi()
    f = getattr(a.lib(), fn)
    g = _grid()
    E = a.UWB_EINVAL
    assert f(None, ctypes.byref(g), 11, FAKE, None) == E
    assert f(ctypes.byref(_scan()), None, 11, FAKE, None) == E
    assert f(ctypes.byref(_scan()), ctypes.byref(g), 11, None, None) == E
    assert f(ctypes.byref(_scan(ant_pos=None)), ctypes.byref(g), 11, FAKE, None) == E
    assert f(ctypes.byref(_scan(traces=None)), ctypes.byref(g), 11, FAKE, None) == E
    assert f(ctypes.byref(_scan(n_ant=0)), ctypes.byref(g), 11, FAKE, None) == E
    assert f(ctypes.byref(_scan(n_samp=1)), ctypes.byref(g), 11, FAKE, None) == E
    assert f(ctypes.byref(_scan(n_samp=70000)), ctypes.byref(g), 11, FAKE, None) == a.UWB_EUNSUPPORTED
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        assert f(ctypes.byref(_scan(dt=bad)), ctypes.byref(g), 11, FAKE, None) == E
        assert f(ctypes.byref(_scan(v=bad)), ctypes.byref(g), 11, FAKE, None) == E
    assert f(ctypes.byref(_scan(t0=float("nan"))), ctypes.byref(g), 11, FAKE, None) == E
    for w in (0, 2, 10, -1):
        assert f(ctypes.byref(_scan()), ctypes.byref(g), w, FAKE, None) == E
    assert f(ctypes.byref(_scan()), ctypes.byref(g), 33, FAKE, None) == a.UWB_EUNSUPPORTED
    for dims in [(0, 8, 1), (8, -1, 1), (8, 8, 0)]:
        assert f(ctypes.byref(_scan()), ctypes.byref(_grid(dims=dims)), 11, FAKE, None) == E
    for pitch in [(0.0, 1e-3, 1e-3), (1e-3, float("nan"), 1e-3), (1e-3, 1e-3, -1.0)]:
        assert f(ctypes.byref(_scan()), ctypes.byref(_grid(pitch=pitch)), 11, FAKE, None) == E
    assert f(ctypes.byref(_scan()), ctypes.byref(_grid(origin=(float("inf"), 0, 0))), 11, FAKE, None) == E


def test_das_dmas_argument_errors():
    """Both-images calls: a missing or overlapping output is refused before anything is launched (an 8 x 8
    image is 256 bytes per scan)."""
    a = _abi()
    g = _grid()
    E = a.UWB_EINVAL
    p = 0x10000000
    v = ctypes.c_void_p
    f = a.lib().uwb_das_dmas
    s = ctypes.byref(_scan())
    assert f(s, ctypes.byref(g), 11, None, v(p), None) == E
    assert f(s, ctypes.byref(g), 11, v(p), None, None) == E
    assert f(s, ctypes.byref(g), 11, v(p), v(p), None) == E
    assert f(s, ctypes.byref(g), 11, v(p), v(p + 252), None) == E
    assert f(s, ctypes.byref(g), 11, v(p + 252), v(p), None) == E
    assert f(s, ctypes.byref(g), 2, v(p), v(p + 256), None) == E
    fb = a.lib().uwb_das_dmas_batch
    bb = a.UwbScanBatch(n_scans=2, n_ant=4, n_samp=64, ant_pos=FAKE, traces=FAKE, params=FAKE, v_min=1e8,
                        dt_min=2e-11)
    assert fb(ctypes.byref(bb), ctypes.byref(g), 11, v(p), v(p + 256), None) == E   # 512 bytes each
    assert fb(ctypes.byref(bb), ctypes.byref(g), 11, v(p), None, None) == E


def test_batch_argument_errors():
    a = _abi()
    f = a.lib().uwb_das_batch
    g = _grid()

    def b(**kw):
        d = dict(n_scans=2, n_ant=4, n_samp=64, ant_pos=FAKE, traces=FAKE, params=FAKE, v_min=1e8, dt_min=2e-11)
        d.update(kw)
        return a.UwbScanBatch(**d)

    assert f(ctypes.byref(b(n_scans=0)), ctypes.byref(g), 11, FAKE, None) == a.UWB_EINVAL
    assert f(ctypes.byref(b(params=None)), ctypes.byref(g), 11, FAKE, None) == a.UWB_EINVAL
    assert f(ctypes.byref(b(v_min=0.0)), ctypes.byref(g), 11, FAKE, None) == a.UWB_EINVAL
    assert f(ctypes.byref(b(n_scans=70000)), ctypes.byref(g), 11, FAKE, None) == a.UWB_EUNSUPPORTED


def test_argmax_argument_errors():
    a = _abi()
    L = a.lib()
    g = _grid()
    need = L.uwb_argmax_workspace_bytes(ctypes.byref(g), 1)
    assert need > 0
    s = _scan()
    assert L.uwb_argmax(ctypes.byref(s), ctypes.byref(g), 11, 3, FAKE, FAKE, FAKE, need, None) == a.UWB_EINVAL
    assert L.uwb_argmax(ctypes.byref(s), ctypes.byref(g), 11, 0, None, FAKE, FAKE, need, None) == a.UWB_EINVAL
    assert L.uwb_argmax(ctypes.byref(s), ctypes.byref(g), 11, 0, FAKE, FAKE, FAKE, need - 1, None) == a.UWB_ERANGE
    assert L.uwb_argmax_workspace_bytes(None, 1) == 0


def test_argmax_noalloc_limit_and_errors():
    """The allocation-free detection refuses requests whose records exceed its fixed scratch (before any HIP
    call), and the usual argument errors."""
    a = _abi()
    L = a.lib()
    f = L.uwb_argmax_batch_noalloc
    limit = 4 << 20
    ok = a.UwbScanBatch(n_scans=256, n_ant=32, n_samp=2048, ant_pos=FAKE, traces=FAKE, params=FAKE, v_min=1e8,
                        dt_min=2e-11)
    g512 = _grid(dims=(512, 512, 1))
    assert 0 < L.uwb_argmax_workspace_bytes(ctypes.byref(g512), 256) <= limit      # the documented example fits
    assert 0 < L.uwb_argmax_workspace_bytes(ctypes.byref(_grid(dims=(256, 256, 256))), 1) <= limit
    big = a.UwbScanBatch(n_scans=512, n_ant=32, n_samp=2048, ant_pos=FAKE, traces=FAKE, params=FAKE, v_min=1e8,
                         dt_min=2e-11)
    assert L.uwb_argmax_workspace_bytes(ctypes.byref(g512), 512) > limit
    assert f(ctypes.byref(big), ctypes.byref(g512), 11, 1, FAKE, FAKE, None) == a.UWB_ERANGE
    assert f(ctypes.byref(ok), ctypes.byref(g512), 11, 3, FAKE, FAKE, None) == a.UWB_EINVAL
    assert f(ctypes.byref(ok), ctypes.byref(g512), 11, 1, None, FAKE, None) == a.UWB_EINVAL
    assert f(ctypes.byref(ok), ctypes.byref(g512), 11, 1, FAKE, None, None) == a.UWB_EINVAL
    assert f(ctypes.byref(ok), ctypes.byref(g512), 4, 1, FAKE, FAKE, None) == a.UWB_EINVAL
    assert f(None, ctypes.byref(g512), 11, 1, FAKE, FAKE, None) == a.UWB_EINVAL
    assert f(ctypes.byref(ok), None, 11, 1, FAKE, FAKE, None) == a.UWB_EINVAL


def _tree(**kw):
    a = _abi()
    d = dict(beamformer=0, walk=0, coarse=8, decimation=0, min_tumour=0.01, max_depth=0, metric=3, term=0,
             frame_level=0.0, frame_final=0.25)
    d.update(kw)
    return a.UwbSegmentTree(**d)


def test_segment_sizes_and_errors():
    a = _abi()
    L = a.lib()
    g512 = _grid(dims=(512, 512, 1), pitch=(0.1 / 512,) * 3)
    t = _tree()
    # per-level, fixed depth: last box side 8, widened by floor(0.25 * 8) = 2 on each end
    assert L.uwb_segment_roi_capacity(ctypes.byref(g512), ctypes.byref(t)) == 12 * 12
    # W/B can stop after the first split: box side 256 -> 256 + 2 * 64 = 384
    assert L.uwb_segment_roi_capacity(ctypes.byref(g512), ctypes.byref(_tree(term=1))) == 384 * 384
    g3 = _grid(dims=(256, 256, 256), pitch=(0.1 / 256,) * 3)
    assert L.uwb_segment_roi_capacity(ctypes.byref(g3), ctypes.byref(t)) == 12 ** 3
    E = a.UWB_EINVAL
    assert L.uwb_segment_roi_capacity(ctypes.byref(_grid(dims=(100, 100, 1))), ctypes.byref(t)) == E   # not 8*2^L
    assert L.uwb_segment_roi_capacity(ctypes.byref(_grid(dims=(512, 256, 1))), ctypes.byref(t)) == E   # not square
    assert L.uwb_segment_roi_capacity(ctypes.byref(g512), ctypes.byref(_tree(coarse=7))) == E
    assert L.uwb_segment_roi_capacity(ctypes.byref(g512), ctypes.byref(_tree(metric=6))) == E
    assert L.uwb_segment_roi_capacity(ctypes.byref(g512), ctypes.byref(_tree(term=2))) == E
    assert L.uwb_segment_roi_capacity(ctypes.byref(g512), ctypes.byref(_tree(frame_final=-0.1))) == E
    assert L.uwb_segment_roi_capacity(ctypes.byref(g512), ctypes.byref(_tree(max_depth=17))) == a.UWB_ERANGE
    assert L.uwb_segment_roi_capacity(ctypes.byref(g512), ctypes.byref(_tree(coarse=128))) == E
    assert L.uwb_segment_roi_capacity(ctypes.byref(g3), ctypes.byref(_tree(coarse=32))) == a.UWB_EUNSUPPORTED
    # paper walk: automatic D from min_tumour; manual D larger than the grid is invalid
    gp = _grid(dims=(100, 100, 1), pitch=(1e-3,) * 3)
    assert L.uwb_segment_roi_capacity(ctypes.byref(gp), ctypes.byref(_tree(walk=1))) > 0
    assert L.uwb_segment_roi_capacity(ctypes.byref(gp), ctypes.byref(_tree(walk=1, decimation=101))) == E
    assert L.uwb_segment_roi_capacity(ctypes.byref(gp), ctypes.byref(_tree(walk=1, min_tumour=0.0))) == E
    ws = L.uwb_segment_workspace_bytes(ctypes.byref(g512), ctypes.byref(t), 4)
    assert ws >= 4 * 8 * 144
    s = _scan()
    cap = 144
    assert L.uwb_segment_refine(ctypes.byref(s), ctypes.byref(g512), 11, ctypes.byref(t), None, FAKE, cap, FAKE, ws,
                                None) == E
    assert L.uwb_segment_refine(ctypes.byref(s), ctypes.byref(g512), 11, ctypes.byref(t), FAKE, FAKE, cap - 1,
                                FAKE, ws, None) == a.UWB_ERANGE
    assert L.uwb_segment_refine(ctypes.byref(s), ctypes.byref(g512), 11, ctypes.byref(t), FAKE, FAKE, cap, FAKE, 8,
                                None) == a.UWB_ERANGE
    assert L.uwb_segment_refine(ctypes.byref(s), ctypes.byref(g512), 11, None, FAKE, FAKE, cap, FAKE, ws,
                                None) == E


def test_tilemax_sizes_and_errors():
    """Tiles per scan of the full-resolution launch (16 x 64 in 2D, 8 x 8 x 16 in 3D) and the argument checks
    of the tile-maximum imaging and detection, before anything is launched."""
    a = _abi()
    L = a.lib()
    g512 = _grid(dims=(512, 512, 1))
    assert L.uwb_image_tiles(ctypes.byref(g512)) == 32 * 8
    assert L.uwb_image_tiles(ctypes.byref(_grid(dims=(256, 256, 256)))) == 32 * 32 * 16
    assert L.uwb_image_tiles(ctypes.byref(_grid(dims=(100, 76, 1)))) == 7 * 2
    assert L.uwb_image_tiles(ctypes.byref(_grid(dims=(0, 8, 1)))) == a.UWB_EINVAL
    E = a.UWB_EINVAL
    bb = a.UwbScanBatch(n_scans=2, n_ant=4, n_samp=64, ant_pos=FAKE, traces=FAKE, params=FAKE, v_min=1e8,
                        dt_min=2e-11)
    g = _grid()   # 8 x 8: one tile; images of 2 x 256 bytes
    v = ctypes.c_void_p
    f = L.uwb_das_dmas_batch_tilemax
    P = 0x10000000
    assert f(ctypes.byref(bb), ctypes.byref(g), 11, v(P), v(P + 512), None, v(P + 4096), None) == E
    assert f(ctypes.byref(bb), ctypes.byref(g), 11, v(P), v(P + 512), v(P + 4096), v(P + 4096), None) == E
    assert f(ctypes.byref(bb), ctypes.byref(g), 11, v(P), v(P + 512), v(P + 256), v(P + 4096), None) == E
    need = L.uwb_argmax_tilemax_workspace_bytes(ctypes.byref(g), 2)
    assert need > 0 and L.uwb_argmax_tilemax_workspace_bytes(None, 2) == 0
    d = L.uwb_argmax_batch_tilemax
    assert d(ctypes.byref(bb), ctypes.byref(g), 11, 2, FAKE, FAKE, FAKE, FAKE, need, None) == E
    assert d(ctypes.byref(bb), ctypes.byref(g), 11, 1, FAKE, None, FAKE, FAKE, need, None) == E
    assert d(ctypes.byref(bb), ctypes.byref(g), 11, 1, FAKE, FAKE, FAKE, FAKE, need - 1, None) == a.UWB_ERANGE


def test_mvdr_argument_errors():
    """MVDR windows beyond UWB_MVDR_MAX_WINDOW are refused by the images, the detection and the walk before
    anything is launched; the batch plan and the learned walk do not take MVDR; beamformer 3 does not exist."""
    a = _abi()
    L = a.lib()
    g = _grid()
    s = ctypes.byref(_scan())
    U, E = a.UWB_EUNSUPPORTED, a.UWB_EINVAL
    assert a.UWB_MVDR == 2
    for fn in ("uwb_mvdr", "uwb_mvdr_multistatic"):
        assert getattr(L, fn)(s, ctypes.byref(g), 13, FAKE, None) == U
        assert getattr(L, fn)(s, ctypes.byref(g), 12, FAKE, None) == E
        assert getattr(L, fn)(s, ctypes.byref(g), 11, None, None) == E
    bb = a.UwbScanBatch(n_scans=2, n_ant=4, n_samp=64, ant_pos=FAKE, traces=FAKE, params=FAKE, v_min=1e8,
                        dt_min=2e-11)
    for fn in ("uwb_mvdr_batch", "uwb_mvdr_multistatic_batch"):
        assert getattr(L, fn)(ctypes.byref(bb), ctypes.byref(g), 13, FAKE, None) == U
    need = L.uwb_argmax_workspace_bytes(ctypes.byref(g), 1)
    assert L.uwb_argmax(s, ctypes.byref(g), 13, 2, FAKE, FAKE, FAKE, need, None) == U
    assert L.uwb_argmax(s, ctypes.byref(g), 11, 3, FAKE, FAKE, FAKE, need, None) == E
    g512 = _grid(dims=(512, 512, 1), pitch=(0.1 / 512,) * 3)
    t = _tree(beamformer=2)
    ws = L.uwb_segment_workspace_bytes(ctypes.byref(g512), ctypes.byref(t), 1)
    cap = L.uwb_segment_roi_capacity(ctypes.byref(g512), ctypes.byref(t))
    assert ws > 0 and cap > 0
    assert L.uwb_segment_refine(s, ctypes.byref(g512), 13, ctypes.byref(t), FAKE, FAKE, cap, FAKE, ws, None) == U
    assert L.uwb_segment_roi_capacity(ctypes.byref(g512), ctypes.byref(_tree(beamformer=3))) == E
    lt = _tree(beamformer=2, coarse=32)
    assert L.uwb_learned_workspace_bytes(ctypes.byref(g512), ctypes.byref(lt), 1) == 0
    plan = ctypes.c_void_p()
    item = a.UwbBatchItem()
    assert L.uwb_batch_plan_create(ctypes.byref(plan), ctypes.byref(item), 1, 2, 11, None) == E


def test_paper_walk_roi_bound_covers_oracle_walks():
    """The ROI bound of the paper walk is never below what the oracle's walks end with."""
    import numpy as np
    import oracle
    import synth
    a = _abi()
    for seed in range(3):
        s = synth.c1_scan(seed, noiseless=True)
        for fl in (0.0, 0.25, 0.6):
            for term in ("fixed", "wb"):
                t = _tree(walk=1, frame_level=fl, term=1 if term == "wb" else 0)
                gc = _grid(dims=s.grid.dims, pitch=s.grid.pitch, origin=s.grid.origin)
                cap = a.lib().uwb_segment_roi_capacity(ctypes.byref(gc), ctypes.byref(t))
                r = oracle.walk(s, oracle.TreeParams(walk="paper", frame_level=fl, term=term, metric="max"))
                roi = r.roi
                assert (roi[1] - roi[0]) * (roi[3] - roi[2]) * (roi[5] - roi[4]) <= cap
                assert np.all(np.array(roi) >= 0)


def test_auto_decimation_matches_paper_example():
    a = _abi()
    with open(os.path.join(ROOT, "tests", "golden", "auto_decimation.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                dmin, pitch, want = line.split()
                assert a.lib().uwb_auto_decimation(float(dmin), float(pitch)) == int(want)
    assert a.lib().uwb_auto_decimation(0.0, 1e-3) == a.UWB_EINVAL
    assert a.lib().uwb_auto_decimation(0.01, float("nan")) == a.UWB_EINVAL


def test_status_strings():
    a = _abi()
    for st in (0, -1, -2, -3, -4, -5, -99):
        assert isinstance(a.lib().uwb_status_string(st), bytes)
    assert a.lib().uwb_version().startswith(b"uwb")


def test_product_path_has_no_oracle_dependency():
    """The package never imports the oracle or the generator."""
    pkg = os.path.join(ROOT, "paper_1709_02549_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, fn
                assert "liboracle" not in txt, fn


def test_batch_plan_argument_errors():
    a = _abi()
    L = a.lib()
    h = ctypes.c_void_p()
    item = a.UwbBatchItem(_scan(), _grid(), FAKE)
    items = (a.UwbBatchItem * 2)(item, item)
    E = a.UWB_EINVAL
    assert L.uwb_batch_plan_create(None, items, 2, 0, 11, None) == E
    assert L.uwb_batch_plan_create(ctypes.byref(h), None, 2, 0, 11, None) == E
    assert L.uwb_batch_plan_create(ctypes.byref(h), items, 0, 0, 11, None) == E
    assert L.uwb_batch_plan_create(ctypes.byref(h), items, 2, 3, 11, None) == E
    assert L.uwb_batch_plan_create(ctypes.byref(h), items, 2, 0, 4, None) == E
    for bad in [(3, 4, 16, 0), (2, 0, 16, 0), (2, 4, 2, 0), (2, 4, 16, 2), (2, 64, 16, 0)]:
        cfg = a.UwbBatchConfig(*bad)
        assert L.uwb_batch_plan_create(ctypes.byref(h), items, 2, 0, 11, ctypes.byref(cfg)) == E
    bad_item = (a.UwbBatchItem * 2)(item, a.UwbBatchItem(_scan(n_ant=0), _grid(), FAKE))
    assert L.uwb_batch_plan_create(ctypes.byref(h), bad_item, 2, 0, 11, None) == E
    no_img = (a.UwbBatchItem * 1)(a.UwbBatchItem(_scan(), _grid(), None))
    assert L.uwb_batch_plan_create(ctypes.byref(h), no_img, 1, 0, 11, None) == E
    mixed = (a.UwbBatchItem * 2)(item, a.UwbBatchItem(_scan(), _grid(dims=(8, 8, 4)), FAKE))
    assert L.uwb_batch_plan_create(ctypes.byref(h), mixed, 2, 0, 11, None) == a.UWB_EUNSUPPORTED
    assert L.uwb_batch_run(None, None) == E
    assert L.uwb_batch_plan_destroy(None) == E


def test_lds_probe_argument_errors():
    a = _abi()
    L = a.lib()
    v, hz = ctypes.c_double(), ctypes.c_double()
    E = a.UWB_EINVAL
    assert L.uwb_probe_lds_read(3, 64, 8, ctypes.byref(v), ctypes.byref(hz), None) == E      # width
    assert L.uwb_probe_lds_read(16, 7, 8, ctypes.byref(v), ctypes.byref(hz), None) == E      # iters % 8
    assert L.uwb_probe_lds_read(16, 64, 0, ctypes.byref(v), ctypes.byref(hz), None) == E     # groups
    assert L.uwb_probe_lds_read(16, 64, 8, None, ctypes.byref(hz), None) == E
