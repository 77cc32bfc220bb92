// Host side of the C ABI declared in include/uwb.h: argument validation and
// dispatch to the kernels.  Validation runs before any HIP call, so an invalid
// request returns its status without touching the device.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "uwb_internal.h"
#include "walk_internal.h"

namespace uwb {

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_window(int32_t w) {
    if (w < 1 || (w % 2) == 0) return UWB_EINVAL;
    if (w > UWB_MAX_WINDOW) return UWB_EUNSUPPORTED;
    return UWB_OK;
}

int check_grid(const uwb_grid *g, GridView *out) {
    if (!g) return UWB_EINVAL;
    for (int d = 0; d < 3; ++d) {
        if (!std::isfinite(g->origin[d]) || !finite_pos(g->pitch[d]) || g->dims[d] < 1) return UWB_EINVAL;
        out->origin[d] = g->origin[d];
        out->pitch[d] = g->pitch[d];
        out->dims[d] = g->dims[d];
    }
    const double nvox = (double)g->dims[0] * g->dims[1] * g->dims[2];
    if (nvox > 1.0e12) return UWB_EUNSUPPORTED;
    return UWB_OK;
}

static int check_sizes(int32_t n_ant, int32_t n_samp) {
    if (n_ant < 1 || n_samp < 2) return UWB_EINVAL;
    if (n_samp > UWB_MAX_SAMPLES || n_ant > (1 << 20)) return UWB_EUNSUPPORTED;
    return UWB_OK;
}

int scan_set(const uwb_scan *s, ScanSet *out) {
    if (!s || !s->ant_pos || !s->traces) return UWB_EINVAL;
    int st = check_sizes(s->n_ant, s->n_samp);
    if (st) return st;
    if (!finite_pos(s->dt) || !finite_pos(s->v) || !std::isfinite(s->t0)) return UWB_EINVAL;
    out->ant_pos = s->ant_pos;
    out->traces = s->traces;
    out->params = nullptr;
    out->pos_stride = 0;
    out->tr_stride = 0;
    out->n_ant = s->n_ant;
    out->n_samp = s->n_samp;
    out->ms = 0;
    out->dt = s->dt;
    out->t0 = s->t0;
    out->v = s->v;
    return UWB_OK;
}

// A multistatic scan: s->n_ant antennas, s->n_ant^2 traces (channel i*M + j).
static int scan_set_ms(const uwb_scan *s, ScanSet *out) {
    int st = scan_set(s, out);
    if (st) return st;
    if (s->n_ant > kMaxMultistaticAnt) return UWB_EUNSUPPORTED;
    out->ms = s->n_ant;
    out->n_ant = s->n_ant * s->n_ant;
    return UWB_OK;
}


int batch_set(const uwb_scan_batch *b, ScanSet *out) {
    if (!b || !b->ant_pos || !b->traces || !b->params) return UWB_EINVAL;
    if (b->n_scans < 1) return UWB_EINVAL;
    if (b->n_scans > 65535) return UWB_EUNSUPPORTED;
    int st = check_sizes(b->n_ant, b->n_samp);
    if (st) return st;
    if (!finite_pos(b->v_min) || !finite_pos(b->dt_min)) return UWB_EINVAL;
    out->ant_pos = b->ant_pos;
    out->traces = b->traces;
    out->params = b->params;
    out->pos_stride = (int64_t)b->n_ant * 3;
    out->tr_stride = (int64_t)b->n_ant * b->n_samp;
    out->n_ant = b->n_ant;
    out->n_samp = b->n_samp;
    out->ms = 0;
    out->dt = b->dt_min;      // lower bounds: size the on-chip staging
    out->t0 = 0.0;
    out->v = b->v_min;
    return UWB_OK;
}

static int batch_set_ms(const uwb_scan_batch *b, ScanSet *out) {
    int st = batch_set(b, out);
    if (st) return st;
    if (b->n_ant > kMaxMultistaticAnt) return UWB_EUNSUPPORTED;
    out->ms = b->n_ant;
    out->n_ant = b->n_ant * b->n_ant;
    out->tr_stride = (int64_t)out->n_ant * b->n_samp;
    return UWB_OK;
}

static int image_common(int bf, const ScanSet &ss, int n, const uwb_grid *grid, int32_t window, float *img,
                        void *stream) {
    GridView g;
    int st = check_grid(grid, &g);
    if (st) return st;
    if ((st = check_window(window))) return st;
    if (!img) return UWB_EINVAL;
    return launch_image32(bf, ss, n, g, window, img, (hipStream_t)stream);
}

static bool overlap(const void *p, const void *q, uintptr_t bytes) {
    const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
    return a < b + bytes && b < a + bytes;
}

// Both images from one DMAS launch; the two outputs must not overlap (nor, when given, the tile maxima).
static int image_both_common(const ScanSet &ss, int n, const uwb_grid *grid, int32_t window, float *img_das,
                             float *img_dmas, void *stream, float *tmax_das = nullptr, float *tmax_dmas = nullptr) {
    GridView g;
    int st = check_grid(grid, &g);
    if (st) return st;
    if ((st = check_window(window))) return st;
    if (!img_das || !img_dmas) return UWB_EINVAL;
    const uintptr_t bytes = (uintptr_t)n * (uintptr_t)g.dims[0] * g.dims[1] * g.dims[2] * sizeof(float);
    if (overlap(img_das, img_dmas, bytes)) return UWB_EINVAL;
    if (tmax_das || tmax_dmas) {
        if (!tmax_das || !tmax_dmas) return UWB_EINVAL;
        const uintptr_t tb = (uintptr_t)n * (uintptr_t)full_tile_count(g) * sizeof(float);
        if (overlap(tmax_das, tmax_dmas, tb) || overlap(tmax_das, img_das, std::max(tb, bytes)) ||
            overlap(tmax_das, img_dmas, std::max(tb, bytes)) || overlap(tmax_dmas, img_das, std::max(tb, bytes)) ||
            overlap(tmax_dmas, img_dmas, std::max(tb, bytes)))
            return UWB_EINVAL;
    }
    return launch_image32(UWB_DMAS, ss, n, g, window, img_dmas, (hipStream_t)stream, img_das, tmax_dmas, tmax_das);
}

// tmax (tile mode): the tile maxima of img from uwb_das_dmas_batch_tilemax.
static int argmax_common(const ScanSet &ss, int n, const uwb_grid *grid, int32_t window, int32_t bf,
                         const float *img, uwb_peak *out, void *ws, size_t ws_bytes, void *stream,
                         const float *tmax = nullptr) {
    GridView g;
    int st = check_grid(grid, &g);
    if (st) return st;
    if ((st = check_window(window))) return st;
    if (bf != UWB_DAS && bf != UWB_DMAS && bf != UWB_MVDR) return UWB_EINVAL;
    if (bf == UWB_MVDR && window > UWB_MVDR_MAX_WINDOW) return UWB_EUNSUPPORTED;
    if (!img || !out || !ws) return UWB_EINVAL;
    if (ws_bytes < argmax_ws_bytes(g, n, tmax != nullptr)) return UWB_ERANGE;
    return launch_argmax(bf, ss, n, g, window, img, out, ws, (hipStream_t)stream, tmax);
}

static int walk_common(const ScanSet &ss, int n, const uwb_grid *finest, int32_t window,
                       const uwb_segment_tree *tree, uwb_segment_result *out, float *roi_img, int64_t roi_capacity,
                       void *ws, size_t ws_bytes, void *stream, float *composite = nullptr) {
    GridView g;
    int st = check_grid(finest, &g);
    if (st) return st;
    if ((st = check_window(window))) return st;
    WalkArgs a;
    int64_t bound = 0;
    size_t need = 0;
    if ((st = plan_walk(g, tree, n, &a, &bound, &need))) return st;
    if (tree->beamformer == UWB_MVDR && window > UWB_MVDR_MAX_WINDOW) return UWB_EUNSUPPORTED;
    if (!out || !ws) return UWB_EINVAL;
    if (roi_img && roi_capacity < bound) return UWB_ERANGE;
    if (!roi_img && roi_capacity != 0 && roi_capacity < bound) return UWB_ERANGE;
    if (ws_bytes < need) return UWB_ERANGE;
    a.ss = ss;
    a.window = window;
    a.out = out;
    a.roi_img = roi_img;
    a.roi_img_stride = roi_img ? roi_capacity : 0;
    assign_walk_ws(&a, ws, n);
    size_walk_lds(&a, ss.n_ant);
    if ((st = launch_walk(a, n, (hipStream_t)stream))) return st;
    return composite ? launch_composite(a, n, composite, (hipStream_t)stream) : UWB_OK;
}

int cnn_max_batch(const uwb_cnn *h);

// The learned walk: per-level quadtree on a planar grid with g = 32 (the CNN's input), fixed depth.
static int learned_plan(const GridView &g, const uwb_segment_tree *t, int n, WalkArgs *a, int64_t *bound,
                        size_t *need) {
    if (!t) return UWB_EINVAL;
    if (t->walk != UWB_WALK_PER_LEVEL || t->coarse != 32 || g.dims[2] != 1 || t->term != UWB_TERM_FIXED_DEPTH)
        return UWB_EUNSUPPORTED;
    if (t->beamformer == UWB_MVDR) return UWB_EUNSUPPORTED;   // the learned walk ends in DAS or DMAS
    int st = plan_walk(g, t, n, a, bound, need);
    if (st) return st;
    if (a->depth < 1) return UWB_EUNSUPPORTED;
    *need += (size_t)n * (32 * 32 * 2 + 4 * 4 + 4) + 3 * 256;
    return UWB_OK;
}

}  // namespace uwb

using namespace uwb;

extern "C" {

int uwb_das(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img, void *stream) {
    ScanSet ss;
    int st = scan_set(scan, &ss);
    return st ? st : image_common(UWB_DAS, ss, 1, grid, window, img, stream);
}

int uwb_dmas(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img, void *stream) {
    ScanSet ss;
    int st = scan_set(scan, &ss);
    return st ? st : image_common(UWB_DMAS, ss, 1, grid, window, img, stream);
}

int uwb_mvdr(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img, void *stream) {
    ScanSet ss;
    int st = scan_set(scan, &ss);
    return st ? st : image_common(UWB_MVDR, ss, 1, grid, window, img, stream);
}

int uwb_mvdr_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img, void *stream) {
    ScanSet ss;
    int st = batch_set(scans, &ss);
    return st ? st : image_common(UWB_MVDR, ss, scans->n_scans, grid, window, img, stream);
}

int uwb_mvdr_multistatic(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img, void *stream) {
    ScanSet ss;
    int st = scan_set_ms(scan, &ss);
    return st ? st : image_common(UWB_MVDR, ss, 1, grid, window, img, stream);
}

int uwb_mvdr_multistatic_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img,
                               void *stream) {
    ScanSet ss;
    int st = batch_set_ms(scans, &ss);
    return st ? st : image_common(UWB_MVDR, ss, scans->n_scans, grid, window, img, stream);
}

int uwb_das_dmas(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img_das, float *img_dmas,
                 void *stream) {
    ScanSet ss;
    int st = scan_set(scan, &ss);
    return st ? st : image_both_common(ss, 1, grid, window, img_das, img_dmas, stream);
}

int uwb_das_dmas_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img_das,
                       float *img_dmas, void *stream) {
    ScanSet ss;
    int st = batch_set(scans, &ss);
    return st ? st : image_both_common(ss, scans->n_scans, grid, window, img_das, img_dmas, stream);
}

int64_t uwb_image_tiles(const uwb_grid *grid) {
    GridView g;
    int st = check_grid(grid, &g);
    return st ? st : full_tile_count(g);
}

int uwb_das_dmas_batch_tilemax(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img_das,
                               float *img_dmas, float *tmax_das, float *tmax_dmas, void *stream) {
    ScanSet ss;
    int st = batch_set(scans, &ss);
    if (st) return st;
    if (!tmax_das || !tmax_dmas) return UWB_EINVAL;
    return image_both_common(ss, scans->n_scans, grid, window, img_das, img_dmas, stream, tmax_das, tmax_dmas);
}

size_t uwb_argmax_tilemax_workspace_bytes(const uwb_grid *grid, int32_t n_scans) {
    GridView g;
    if (check_grid(grid, &g) || n_scans < 1) return 0;
    return argmax_ws_bytes(g, n_scans, true);
}

int uwb_argmax_batch_tilemax(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, int32_t beamformer,
                             const float *img, const float *tmax, uwb_peak *out, void *workspace,
                             size_t workspace_bytes, void *stream) {
    ScanSet ss;
    int st = batch_set(scans, &ss);
    if (st) return st;
    if (beamformer != UWB_DAS && beamformer != UWB_DMAS) return UWB_EINVAL;
    if (!tmax) return UWB_EINVAL;
    return argmax_common(ss, scans->n_scans, grid, window, beamformer, img, out, workspace, workspace_bytes, stream,
                         tmax);
}

int uwb_das_dmas_multistatic_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window,
                                   float *img_das, float *img_dmas, void *stream) {
    ScanSet ss;
    int st = batch_set_ms(scans, &ss);
    return st ? st : image_both_common(ss, scans->n_scans, grid, window, img_das, img_dmas, stream);
}

int uwb_das_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img, void *stream) {
    ScanSet ss;
    int st = batch_set(scans, &ss);
    return st ? st : image_common(UWB_DAS, ss, scans->n_scans, grid, window, img, stream);
}

int uwb_dmas_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img, void *stream) {
    ScanSet ss;
    int st = batch_set(scans, &ss);
    return st ? st : image_common(UWB_DMAS, ss, scans->n_scans, grid, window, img, stream);
}

int uwb_das_multistatic(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img, void *stream) {
    ScanSet ss;
    int st = scan_set_ms(scan, &ss);
    return st ? st : image_common(UWB_DAS, ss, 1, grid, window, img, stream);
}

int uwb_dmas_multistatic(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img, void *stream) {
    ScanSet ss;
    int st = scan_set_ms(scan, &ss);
    return st ? st : image_common(UWB_DMAS, ss, 1, grid, window, img, stream);
}

int uwb_das_multistatic_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img,
                              void *stream) {
    ScanSet ss;
    int st = batch_set_ms(scans, &ss);
    return st ? st : image_common(UWB_DAS, ss, scans->n_scans, grid, window, img, stream);
}

int uwb_dmas_multistatic_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img,
                               void *stream) {
    ScanSet ss;
    int st = batch_set_ms(scans, &ss);
    return st ? st : image_common(UWB_DMAS, ss, scans->n_scans, grid, window, img, stream);
}

int uwb_argmax_multistatic(const uwb_scan *scan, const uwb_grid *grid, int32_t window, int32_t beamformer,
                           const float *img, uwb_peak *out, void *workspace, size_t workspace_bytes, void *stream) {
    ScanSet ss;
    int st = scan_set_ms(scan, &ss);
    return st ? st : argmax_common(ss, 1, grid, window, beamformer, img, out, workspace, workspace_bytes, stream);
}

int uwb_argmax_multistatic_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window,
                                 int32_t beamformer, const float *img, uwb_peak *out, void *workspace,
                                 size_t workspace_bytes, void *stream) {
    ScanSet ss;
    int st = batch_set_ms(scans, &ss);
    return st ? st
              : argmax_common(ss, scans->n_scans, grid, window, beamformer, img, out, workspace, workspace_bytes,
                              stream);
}

int uwb_segment_refine_multistatic(const uwb_scan *scan, const uwb_grid *finest, int32_t window,
                                   const uwb_segment_tree *tree, uwb_segment_result *out, float *roi_img,
                                   int64_t roi_capacity, void *workspace, size_t workspace_bytes, void *stream) {
    ScanSet ss;
    int st = scan_set_ms(scan, &ss);
    return st ? st
              : walk_common(ss, 1, finest, window, tree, out, roi_img, roi_capacity, workspace, workspace_bytes,
                            stream);
}

int uwb_segment_refine_multistatic_batch(const uwb_scan_batch *scans, const uwb_grid *finest, int32_t window,
                                         const uwb_segment_tree *tree, uwb_segment_result *out, float *roi_img,
                                         int64_t roi_capacity, void *workspace, size_t workspace_bytes,
                                         void *stream) {
    ScanSet ss;
    int st = batch_set_ms(scans, &ss);
    return st ? st
              : walk_common(ss, scans->n_scans, finest, window, tree, out, roi_img, roi_capacity, workspace,
                            workspace_bytes, stream);
}

size_t uwb_argmax_workspace_bytes(const uwb_grid *grid, int32_t n_scans) {
    GridView g;
    if (check_grid(grid, &g) || n_scans < 1) return 0;
    return argmax_ws_bytes(g, n_scans);
}

int uwb_argmax(const uwb_scan *scan, const uwb_grid *grid, int32_t window, int32_t beamformer, const float *img,
               uwb_peak *out, void *workspace, size_t workspace_bytes, void *stream) {
    ScanSet ss;
    int st = scan_set(scan, &ss);
    return st ? st : argmax_common(ss, 1, grid, window, beamformer, img, out, workspace, workspace_bytes, stream);
}

int uwb_argmax_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, int32_t beamformer,
                     const float *img, uwb_peak *out, void *workspace, size_t workspace_bytes, void *stream) {
    ScanSet ss;
    int st = batch_set(scans, &ss);
    return st ? st
              : argmax_common(ss, scans->n_scans, grid, window, beamformer, img, out, workspace, workspace_bytes,
                              stream);
}

int uwb_argmax_batch_noalloc(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, int32_t beamformer,
                             const float *img, uwb_peak *out, void *stream) {
    ScanSet ss;
    int st = batch_set(scans, &ss);
    if (st) return st;
    GridView g;
    if ((st = check_grid(grid, &g))) return st;
    if ((st = check_window(window))) return st;
    if (beamformer != UWB_DAS && beamformer != UWB_DMAS && beamformer != UWB_MVDR) return UWB_EINVAL;
    if (beamformer == UWB_MVDR && window > UWB_MVDR_MAX_WINDOW) return UWB_EUNSUPPORTED;
    if (!img || !out) return UWB_EINVAL;
    if (argmax_ws_bytes(g, scans->n_scans) > (size_t)UWB_ARGMAX_SCRATCH_BYTES) return UWB_ERANGE;
    void *ws = nullptr;
    if ((st = argmax_scratch(&ws))) return st;
    return launch_argmax(beamformer, ss, scans->n_scans, g, window, img, out, ws, (hipStream_t)stream);
}

int64_t uwb_segment_roi_capacity(const uwb_grid *finest, const uwb_segment_tree *tree) {
    GridView g;
    int st = check_grid(finest, &g);
    if (st) return st;
    WalkArgs a;
    int64_t bound = 0;
    size_t need = 0;
    if ((st = plan_walk(g, tree, 1, &a, &bound, &need))) return st;
    return bound;
}

size_t uwb_segment_workspace_bytes(const uwb_grid *finest, const uwb_segment_tree *tree, int32_t n_scans) {
    GridView g;
    if (check_grid(finest, &g)) return 0;
    WalkArgs a;
    int64_t bound = 0;
    size_t need = 0;
    if (plan_walk(g, tree, n_scans, &a, &bound, &need)) return 0;
    return need;
}

int uwb_segment_refine(const uwb_scan *scan, const uwb_grid *finest, int32_t window, const uwb_segment_tree *tree,
                       uwb_segment_result *out, float *roi_img, int64_t roi_capacity, void *workspace,
                       size_t workspace_bytes, void *stream) {
    ScanSet ss;
    int st = scan_set(scan, &ss);
    return st ? st
              : walk_common(ss, 1, finest, window, tree, out, roi_img, roi_capacity, workspace, workspace_bytes,
                            stream);
}

int uwb_segment_refine_batch(const uwb_scan_batch *scans, const uwb_grid *finest, int32_t window,
                             const uwb_segment_tree *tree, uwb_segment_result *out, float *roi_img,
                             int64_t roi_capacity, void *workspace, size_t workspace_bytes, void *stream) {
    ScanSet ss;
    int st = batch_set(scans, &ss);
    return st ? st
              : walk_common(ss, scans->n_scans, finest, window, tree, out, roi_img, roi_capacity, workspace,
                            workspace_bytes, stream);
}

int uwb_segment_composite_batch(const uwb_scan_batch *scans, const uwb_grid *finest, int32_t window,
                                const uwb_segment_tree *tree, uwb_segment_result *out, float *roi_img,
                                int64_t roi_capacity, void *workspace, size_t workspace_bytes, float *composite,
                                void *stream) {
    if (!composite) return UWB_EINVAL;
    ScanSet ss;
    int st = batch_set(scans, &ss);
    return st ? st
              : walk_common(ss, scans->n_scans, finest, window, tree, out, roi_img, roi_capacity, workspace,
                            workspace_bytes, stream, composite);
}

size_t uwb_tumour_check_workspace_bytes(const uwb_grid *finest, const uwb_segment_tree *tree, int32_t d1, int32_t d2,
                                        int32_t n_scans) {
    if (!tree || tree->walk != UWB_WALK_PAPER) return 0;
    size_t need = 0;
    for (int32_t d : {d1, d2}) {
        uwb_segment_tree t = *tree;
        t.decimation = d;
        const size_t b = uwb_segment_workspace_bytes(finest, &t, n_scans);
        if (b == 0) return 0;
        need = b > need ? b : need;
    }
    return need;
}

int uwb_tumour_check_batch(const uwb_scan_batch *scans, const uwb_grid *finest, int32_t window,
                           const uwb_segment_tree *tree, int32_t d1, int32_t d2, uwb_segment_result *out,
                           int32_t *agree, void *workspace, size_t workspace_bytes, void *stream) {
    if (!tree || !out || !agree) return UWB_EINVAL;
    if (tree->walk != UWB_WALK_PAPER) return UWB_EUNSUPPORTED;
    if (d1 < 1 || d2 < 1 || d1 == d2) return UWB_EINVAL;
    ScanSet ss;
    int st = batch_set(scans, &ss);
    if (st) return st;
    const int n = scans->n_scans;
    if (workspace_bytes < uwb_tumour_check_workspace_bytes(finest, tree, d1, d2, n)) return UWB_ERANGE;
    for (int k = 0; k < 2; ++k) {
        uwb_segment_tree t = *tree;
        t.decimation = k == 0 ? d1 : d2;
        if ((st = walk_common(ss, n, finest, window, &t, out + (size_t)k * n, nullptr, 0, workspace, workspace_bytes,
                              stream)))
            return st;
    }
    return launch_roi_overlap(out, out + n, agree, n, (hipStream_t)stream);
}

size_t uwb_learned_workspace_bytes(const uwb_grid *finest, const uwb_segment_tree *tree, int32_t n_scans) {
    GridView g;
    if (check_grid(finest, &g) || n_scans < 1) return 0;
    WalkArgs a;
    int64_t bound = 0;
    size_t need = 0;
    if (learned_plan(g, tree, n_scans, &a, &bound, &need)) return 0;
    return need;
}

int uwb_learned_refine_batch(const uwb_scan_batch *scans, const uwb_grid *finest, int32_t window,
                             const uwb_segment_tree *tree, uwb_cnn *cnn, float threshold, uwb_segment_result *out,
                             float *roi_img, int64_t roi_capacity, void *workspace, size_t workspace_bytes,
                             void *stream) {
    ScanSet ss;
    int st = batch_set(scans, &ss);
    if (st) return st;
    GridView g;
    if ((st = check_grid(finest, &g))) return st;
    if ((st = check_window(window))) return st;
    if (!cnn || !out || !workspace || !std::isfinite(threshold)) return UWB_EINVAL;
    const int n = scans->n_scans;
    if (n > cnn_max_batch(cnn)) return UWB_ERANGE;
    WalkArgs a;
    int64_t bound = 0;
    size_t need = 0;
    if ((st = learned_plan(g, tree, n, &a, &bound, &need))) return st;
    if (roi_img && roi_capacity < bound) return UWB_ERANGE;
    if (workspace_bytes < need) return UWB_ERANGE;
    a.ss = ss;
    a.window = window;
    a.out = out;
    a.roi_img = roi_img;
    a.roi_img_stride = roi_img ? roi_capacity : 0;
    assign_walk_ws(&a, workspace, n);
    uintptr_t p = (uintptr_t)(a.state + n);
    p = (p + 255) & ~(uintptr_t)255;
    uint16_t *xin = reinterpret_cast<uint16_t *>(p);
    p += (size_t)n * 32 * 32 * 2;
    p = (p + 255) & ~(uintptr_t)255;
    float *probs = reinterpret_cast<float *>(p);
    p += (size_t)n * 16;
    p = (p + 255) & ~(uintptr_t)255;
    int *fb = reinterpret_cast<int *>(p);
    size_walk_lds(&a, ss.n_ant);
    return launch_learned(a, n, cnn, threshold, xin, probs, fb, tree->beamformer, (hipStream_t)stream);
}

int uwb_cnn_training_inputs(const uwb_scan_batch *scans, const uwb_grid *finest, int32_t window,
                            const uwb_peak *targets, uint16_t *x, int32_t *labels, void *stream) {
    ScanSet ss;
    int st = batch_set(scans, &ss);
    if (st) return st;
    GridView g;
    if ((st = check_grid(finest, &g))) return st;
    if ((st = check_window(window))) return st;
    if (!targets || !x || !labels) return UWB_EINVAL;
    uwb_segment_tree t = {UWB_DAS, UWB_WALK_PER_LEVEL, 32, 0, 0.01, 0, UWB_MAX, UWB_TERM_FIXED_DEPTH, 0.0, 0.0};
    WalkArgs a;
    int64_t bound = 0;
    size_t need = 0;
    if ((st = learned_plan(g, &t, scans->n_scans, &a, &bound, &need))) return st;
    a.ss = ss;
    a.window = window;
    size_walk_lds(&a, ss.n_ant);
    return launch_cnn_inputs(a, scans->n_scans, targets, x, labels, (hipStream_t)stream);
}

int32_t uwb_cnn_input_levels(const uwb_grid *finest) {
    GridView g;
    int st = check_grid(finest, &g);
    if (st) return st;
    uwb_segment_tree t = {UWB_DAS, UWB_WALK_PER_LEVEL, 32, 0, 0.01, 0, UWB_MAX, UWB_TERM_FIXED_DEPTH, 0.0, 0.0};
    WalkArgs a;
    int64_t bound = 0;
    size_t need = 0;
    if ((st = learned_plan(g, &t, 1, &a, &bound, &need))) return st;
    return a.depth;
}

int uwb_auto_decimation(double min_tumour, double pitch) {
    if (!finite_pos(min_tumour) || !finite_pos(pitch)) return UWB_EINVAL;
    const double d = std::floor(min_tumour / (std::sqrt(2.0) * pitch));
    if (!(d < 2147483647.0)) return UWB_EUNSUPPORTED;
    return d < 1.0 ? 1 : (int)d;
}

const char *uwb_status_string(int status) {
    switch (status) {
        case UWB_OK: return "ok";
        case UWB_EINVAL: return "invalid argument";
        case UWB_ERANGE: return "output, workspace or depth out of range";
        case UWB_ENOMEM: return "out of memory";
        case UWB_EHIP: return "HIP runtime or launch error";
        case UWB_EUNSUPPORTED: return "unsupported request";
        default: return "unknown status";
    }
}

const char *uwb_version(void) { return "uwb 0.1 gfx950"; }

}  // extern "C"
