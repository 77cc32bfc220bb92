"""GPU parity of the full-resolution DAS / DMAS kernels and the FP64-decided argmax against the oracle.

Tolerance (FP32 images, derived from the arithmetic): the delay is formed in
FP32 from values of magnitude <= ~200 samples (unit roundoff 6e-8 -> ~2e-5
samples), and the pulse changes by at most ~0.8 of its peak per sample, so each
aligned sample carries ~1e-5 relative error; DAS energy doubles it, DMAS energy
quadruples it.  The gate is 1e-4 of the image peak everywhere, and 1e-4
relative on every voxel brighter than 1% of the peak.  Windows of 1 or 3
samples have no averaging over the pulse (a voxel at 1% of the peak can sit on a
flank where |slope| / |s| ~ 8 per sample, ~3e-4 with an FP32 delay), so the
kernels take their delay in FP64 and the same 1e-4 gate holds for them.
Argmax: bit-exact.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
from synth import Grid  # noqa: E402

REL_PEAK = 1e-4
REL_BRIGHT = 1e-4


def uwb():
    import paper_1709_02549_amd as m
    return m


def _check_image(got, want, window=11):
    got = np.asarray(got, dtype=np.float64)
    peak = float(np.max(want))
    assert np.all(np.isfinite(got))
    err = np.max(np.abs(got - want)) / peak
    assert err <= REL_PEAK, f"max |dI| / peak = {err:.3e}"
    bright = want >= 1e-2 * peak
    rel = np.max(np.abs(got[bright] - want[bright]) / want[bright])
    assert rel <= REL_BRIGHT, f"bright-voxel relative error {rel:.3e} (window {window})"
    return err


def _gpu_image(s, bf, window=11):
    u = uwb()
    ds = u.DeviceScan.from_host(s)
    img = u.image(ds, s.grid, bf, window)
    torch.cuda.synchronize()
    return ds, img


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("bf", [0, 1])
def test_c1_parity(seed, bf):
    """C1: 16-antenna ring, 128 x 128 grid, noisy scans."""
    s = synth.c1_scan(seed)
    ds, img = _gpu_image(s, bf)
    want = oracle.image_grid(s, bf)
    _check_image(img.cpu().numpy(), want)
    p = uwb().argmax(ds, s.grid, img, bf)
    a, v = oracle.argmax_grid(want)
    assert p.index == a
    assert p.value == pytest.approx(v, rel=1e-12)


@pytest.mark.parametrize("bf", [0, 1])
@pytest.mark.parametrize("dims", [(100, 76, 1), (37, 5, 1), (1, 1, 1), (19, 21, 11), (9, 8, 13)])
def test_ragged_grids(bf, dims):
    """Grids that are not multiples of the tile, in 2D and 3D, several tiles plus a ragged tail."""
    rng = np.random.default_rng(sum(dims) + bf)
    n = np.array(dims)
    pitch = 0.1 / max(n.max(), 8)
    g = Grid(tuple(-0.5 * pitch * (n - 1)), (pitch, pitch * 1.25, pitch * 0.8), dims)
    if dims[2] > 1:
        ant = synth.hemisphere_antennas(24)
    else:
        ant = synth.ring_antennas(12)
    tum = rng.uniform(-0.02, 0.02, 3) * (1 if dims[2] > 1 else np.array([1, 1, 0]))
    s = synth.point_scan(ant, g, tum[None, :], [1.0], 1024, synth.C0 / 3)
    s.traces = (s.traces + 0.01 * rng.standard_normal(s.traces.shape)).astype(np.float32)
    ds, img = _gpu_image(s, bf)
    want = oracle.image_grid(s, bf)
    _check_image(img.cpu().numpy(), want)
    assert uwb().argmax(ds, g, img, bf).index == oracle.argmax_grid(want)[0]


@pytest.mark.parametrize("window", [1, 3, 5, 9, 13, 31])
@pytest.mark.parametrize("bf", [0, 1])
def test_windows(window, bf):
    s = synth.c1_scan(5, n_grid=48)
    ds, img = _gpu_image(s, bf, window)
    want = oracle.image_grid(s, bf, window)
    _check_image(img.cpu().numpy(), want, window)
    assert uwb().argmax(ds, s.grid, img, bf, window).index == oracle.argmax_grid(want)[0]


@pytest.mark.parametrize("bf", [0, 1])
def test_edge_antennas_and_short_traces(bf):
    """M = 1 and 2, very short traces (T = 2 and 40): windows run off both ends of the trace."""
    for m, T in [(1, 40), (2, 2), (3, 40)]:
        rng = np.random.default_rng(m * 7 + T)
        g = Grid((-0.004, -0.004, 0.0), (0.0005, 0.0005, 0.001), (17, 17, 1))
        ant = rng.uniform(-0.01, 0.01, (m, 3)).astype(np.float32)
        ant[:, 2] = 0
        s = synth.Scan(ant, rng.standard_normal((m, T)).astype(np.float32), 2e-11, -1e-10, 3e8 / 4, g)
        ds, img = _gpu_image(s, bf)
        want = oracle.image_grid(s, bf)
        got = img.cpu().numpy()
        if want.max() == 0:
            assert np.all(got == 0)
            continue
        _check_image(got, want)


def test_dmas_single_antenna_is_zero():
    s = synth.c1_scan(0, n_grid=32, n_ant=1)
    _, img = _gpu_image(s, 1)
    assert torch.count_nonzero(img).item() == 0


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("bf", [0, 1])
def test_c2_full_size(seed, bf):
    """C2 at full size (512 x 512, 32 antennas, T = 2048, 200 clutter scatterers, 20 dB): every voxel against the
    full oracle image at the image bar, and the detection equal to the oracle's argmax over the whole grid."""
    s = synth.c2_scan(seed)
    ds, img = _gpu_image(s, bf)
    want = oracle.image_grid(s, bf)
    _check_image(img.cpu().numpy(), want)
    p = uwb().argmax(ds, s.grid, img, bf)
    a, v = oracle.argmax_grid(want)
    assert p.index == a
    assert p.value == pytest.approx(v, rel=1e-12)


@pytest.mark.parametrize("bf", [0, 1])
def test_c3_full_size(bf):
    """C3 at full size (256^3, 64 antennas on the hemisphere, T = 4096, 1000 clutter scatterers): all 16.8 M voxels
    against the full oracle image (direct pairwise DMAS: 3.7e11 pair products, tens of seconds on the host), and
    the detection equal to the oracle's argmax over the whole volume."""
    s = synth.c3_scan(0)
    ds, img = _gpu_image(s, bf)
    p = uwb().argmax(ds, s.grid, img, bf)
    got = img.cpu().numpy()
    del img
    want = oracle.image_grid(s, bf)
    _check_image(got, want)
    a, v = oracle.argmax_grid(want)
    assert p.index == a
    assert p.value == pytest.approx(v, rel=1e-12)


@pytest.mark.parametrize("bf", [0, 1])
def test_batch_equals_single_and_deterministic(bf):
    scans = [synth.c1_scan(k, n_grid=64) for k in range(5)]
    scans[3] = synth.c3_scan(3, n_grid=64, n_ant=16, n_samp=1024)     # different v inside the batch
    scans[3].ant_pos = scans[0].ant_pos
    scans[3].grid = scans[0].grid
    u = uwb()
    b = u.DeviceBatch.from_host(scans)
    a1 = u.image_batch(b, scans[0].grid, bf)
    a2 = u.image_batch(b, scans[0].grid, bf)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2)
    for k, s in enumerate(scans):
        one = u.image(u.DeviceScan.from_host(s), s.grid, bf)
        assert torch.equal(one, a1[k])
    peaks = u.argmax_batch(b, scans[0].grid, a1, bf)
    for k, s in enumerate(scans):
        assert peaks[k].index == oracle.argmax_grid(oracle.image_grid(s, bf))[0]


@pytest.mark.parametrize("n", [16, 64])
def test_flat_image_argmax_is_lowest_index(n):
    """All-equal energies (constant traces, every window inside the trace): every voxel is a candidate;
    the FP64 decision keeps the lowest index among ties within the 1e-12 band.  256 candidates fit a chunk's
    candidate list (evaluated by its four wavefronts, then re-evaluated for the tie band past the 8 the
    chunk record keeps); 4096 overflow it (each wavefront evaluates its own)."""
    g = Grid((0.0, 0.0, 0.0), (1e-4, 1e-4, 1e-4), (n, n, 1))
    ant = np.array([[-0.1, 0.0, 0.0]], np.float32)
    s = synth.Scan(ant, np.ones((1, 4096), np.float32), 2e-11, 0.0, 1e8, g)
    ds, img = _gpu_image(s, 0)
    p = uwb().argmax(ds, g, img, 0)
    want = oracle.argmax_grid(oracle.image_grid(s, 0))
    assert p.index == want[0] == 0
    assert p.candidates == n * n


# ----------------------------------------------------------------------------------
# both images from one launch
# ----------------------------------------------------------------------------------

def _ragged_scan(dims, seed):
    rng = np.random.default_rng(seed)
    n = np.array(dims)
    pitch = 0.1 / max(n.max(), 8)
    g = Grid(tuple(-0.5 * pitch * (n - 1)), (pitch, pitch * 1.25, pitch * 0.8), dims)
    ant = synth.hemisphere_antennas(24) if dims[2] > 1 else synth.ring_antennas(12)
    tum = rng.uniform(-0.02, 0.02, 3) * (1 if dims[2] > 1 else np.array([1, 1, 0]))
    s = synth.point_scan(ant, g, tum[None, :], [1.0], 1024, synth.C0 / 3)
    s.traces = (s.traces + 0.01 * rng.standard_normal(s.traces.shape)).astype(np.float32)
    return s


@pytest.mark.parametrize("case", ["c1-0", "c1-1", "ragged-2d", "ragged-3d"])
def test_das_dmas_one_launch(case):
    """The DMAS launch's running sums are the DAS sums: both images from one launch.  DMAS equals uwb_dmas bit
    for bit; DAS meets the oracle's bar (and uwb_das's to FP32 rounding); ragged 2D and 3D grids."""
    s = {"c1-0": lambda: synth.c1_scan(0), "c1-1": lambda: synth.c1_scan(1),
         "ragged-2d": lambda: _ragged_scan((100, 76, 1), 5), "ragged-3d": lambda: _ragged_scan((19, 21, 11), 6)}[case]()
    u = uwb()
    ds = u.DeviceScan.from_host(s)
    das, dmas = u.das_dmas(ds, s.grid)
    torch.cuda.synchronize()
    assert torch.equal(dmas, u.image(ds, s.grid, 1))
    want = oracle.image_grid(s, 0)
    _check_image(das.cpu().numpy(), want)
    _check_image(dmas.cpu().numpy(), oracle.image_grid(s, 1))
    ref = u.image(ds, s.grid, 0).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(das.cpu().numpy() - ref)) <= 1e-4 * float(np.max(want))
    assert u.argmax(ds, s.grid, das, 0).index == oracle.argmax_grid(want)[0]


def test_das_dmas_batch_and_errors():
    scans = [synth.c1_scan(k, n_grid=64) for k in range(4)]
    u = uwb()
    b = u.DeviceBatch.from_host(scans)
    das, dmas = u.das_dmas_batch(b, scans[0].grid)
    torch.cuda.synchronize()
    assert torch.equal(dmas, u.image_batch(b, scans[0].grid, 1))
    for k, s in enumerate(scans):
        _check_image(das[k].cpu().numpy(), oracle.image_grid(s, 0))
    # overlapping outputs are refused, nothing is launched
    buf = torch.empty((2 * 4 + 1,) + das.shape[1:], dtype=torch.float32, device="cuda")
    with pytest.raises(u.UwbError):
        u.das_dmas_batch(b, scans[0].grid, out_das=buf[0:4], out_dmas=buf[3:7])
    u.das_dmas_batch(b, scans[0].grid, out_das=buf[0:4], out_dmas=buf[4:8])   # adjacent is fine
    torch.cuda.synchronize()
    assert torch.equal(buf[4:8], dmas) and torch.equal(buf[0:4], das)


# ----------------------------------------------------------------------------------
# detection from the imaging launch's tile maxima (no second pass over the images)
# ----------------------------------------------------------------------------------

def _tile_max_reference(img, grid):
    """Every 16 x 64 (2D) or 8 x 8 x 16 (3D) tile's maximum of img [n][nz][ny][nx], tiles in launch order."""
    nx, ny, nz = grid.dims
    tx, ty, tz = (8, 8, 16) if nz > 1 else (16, 64, 1)
    n = img.shape[0]
    px, py, pz = -nx % tx, -ny % ty, -nz % tz
    x = torch.nn.functional.pad(img, (0, px, 0, py, 0, pz), value=float("-inf"))
    x = x.reshape(n, (nz + pz) // tz, tz, (ny + py) // ty, ty, (nx + px) // tx, tx)
    return x.amax(dim=(2, 4, 6)).reshape(n, -1)


@pytest.mark.parametrize("case", ["c2", "ragged-3d", "ragged-2d"])
def test_tilemax_detection_equals_argmax(case):
    """uwb_das_dmas_batch_tilemax writes the same images as uwb_das_dmas_batch plus every tile's maximum; the
    detection from those maxima returns the uwb_peak records of uwb_argmax_batch byte for byte, which are the
    oracle's argmax."""
    u = uwb()
    if case == "c2":
        scans = [synth.c2_scan(k) for k in range(6)]
    elif case == "ragged-3d":
        scans = [_ragged_scan((19, 21, 11), 20 + k) for k in range(3)]
    else:
        scans = [_ragged_scan((100, 76, 1), 30 + k) for k in range(3)]
    g = scans[0].grid
    b = u.DeviceBatch.from_host(scans)
    das, dmas, tdas, tdmas = u.das_dmas_batch_tilemax(b, g)
    das2, dmas2 = u.das_dmas_batch(b, g)
    torch.cuda.synchronize()
    assert torch.equal(das, das2) and torch.equal(dmas, dmas2)
    assert tdas.shape[1] == u.image_tiles(g)
    assert torch.equal(tdas, _tile_max_reference(das, g)) and torch.equal(tdmas, _tile_max_reference(dmas, g))
    for bf, img, tm in ((0, das, tdas), (1, dmas, tdmas)):
        p_tile = u.argmax_batch_tilemax_async(b, g, img, tm, bf)
        p_ref = u.argmax_batch_async(b, g, img, bf)
        torch.cuda.synchronize()
        assert torch.equal(p_tile, p_ref)
        for k, s in enumerate(scans[:2]):
            assert u._peaks(p_tile, len(scans))[k].index == oracle.argmax_grid(oracle.image_grid(s, bf))[0]


def test_flat_images_overflow_the_chunk_list():
    """All-equal energies: every chunk (16 of 4096 voxels) and every tile (64) holds candidates, more than the
    detection lists per scan, so its candidate passes take every chunk in turn; the lowest index wins."""
    u = uwb()
    g = Grid((0.0, 0.0, 0.0), (1e-4, 1e-4, 1e-4), (256, 256, 1))
    ant = np.array([[-0.1, 0.0, 0.0]], np.float32)
    s = synth.Scan(ant, np.ones((1, 4096), np.float32), 2e-11, 0.0, 1e8, g)
    b = u.DeviceBatch.from_host([s, s])
    das, dmas, tdas, tdmas = u.das_dmas_batch_tilemax(b, g)
    for p in (u.argmax_batch_async(b, g, das, 0), u.argmax_batch_tilemax_async(b, g, das, tdas, 0)):
        pk = u._peaks(p, 2)
        assert [q.index for q in pk] == [0, 0]
        assert [q.candidates for q in pk] == [256 * 256] * 2


def test_grouped_tiles_match_single_tiles():
    """A large launch images four tiles per workgroup from one staging of the traces (the launch holds enough
    workgroups); on a grid whose tiles do not fill the last group of a row (200 x 200: 13 tiles of 16 along x,
    four rows of 64, ragged in both) every image equals the one-scan launch's (one tile per workgroup) bit for
    bit, the tile maxima are the images' own, the detections those of uwb_argmax_batch, and two scans meet the
    oracle's bar."""
    u = uwb()
    g = Grid((-0.05, -0.05, 0.0), (0.1 / 199, 0.1 / 199, 1e-3), (200, 200, 1))
    ant = synth.ring_antennas(4)
    scans = []
    for k in range(320):
        rng = np.random.default_rng(7000 + k)
        tum = np.array([*rng.uniform(-0.03, 0.03, 2), 0.0])
        s = synth.point_scan(ant, g, tum[None, :], [1.0], 512, synth.C0 / 3)
        s.traces = (s.traces + 0.01 * rng.standard_normal(s.traces.shape)).astype(np.float32)
        scans.append(s)
    b = u.DeviceBatch.from_host(scans)
    das, dmas, tdas, tdmas = u.das_dmas_batch_tilemax(b, g)
    torch.cuda.synchronize()
    assert torch.equal(tdas, _tile_max_reference(das, g)) and torch.equal(tdmas, _tile_max_reference(dmas, g))
    for k in (0, 1, 157, 319):
        d1, m1 = u.das_dmas(u.DeviceScan.from_host(scans[k]), g)
        torch.cuda.synchronize()
        assert torch.equal(d1, das[k]) and torch.equal(m1, dmas[k]), k
    for bf, img, tm in ((0, das, tdas), (1, dmas, tdmas)):
        p_tile = u.argmax_batch_tilemax_async(b, g, img, tm, bf)
        p_ref = u.argmax_batch_async(b, g, img, bf)
        torch.cuda.synchronize()
        assert torch.equal(p_tile, p_ref)
    for k in (0, 319):
        _check_image(das[k].cpu().numpy(), oracle.image_grid(scans[k], 0))
        _check_image(dmas[k].cpu().numpy(), oracle.image_grid(scans[k], 1))


def test_nan_trace_detection_is_reported_not_found():
    """A NaN sample propagates into every voxel that reads it (traces are not scanned for NaN); where the whole
    image is NaN both detection forms report no finite candidate: index 0 and a NaN value, identically."""
    u = uwb()
    scans = [synth.c1_scan(k, n_grid=64) for k in range(2)]
    scans[1].traces = np.full_like(scans[1].traces, np.nan)
    g = scans[0].grid
    b = u.DeviceBatch.from_host(scans)
    das, dmas, tdas, tdmas = u.das_dmas_batch_tilemax(b, g)
    torch.cuda.synchronize()
    assert torch.isnan(dmas[1]).all() and torch.isfinite(dmas[0]).all()
    for bf, img, tm in ((0, das, tdas), (1, dmas, tdmas)):
        p_tile = u.argmax_batch_tilemax_async(b, g, img, tm, bf)
        p_ref = u.argmax_batch_async(b, g, img, bf)
        torch.cuda.synchronize()
        assert torch.equal(p_tile, p_ref)
        pk = u._peaks(p_ref, 2)
        assert pk[1].index == 0 and np.isnan(pk[1].value)
        assert pk[0].index == oracle.argmax_grid(oracle.image_grid(scans[0], bf))[0]
