// Coarse-to-fine segment walk (Section III): spatial decimation, ROI selection
// with the mean / variance / Eq. (5) metrics and the Eq. (6)-(7) stop, sliding
// frame, final full-resolution imaging of the ROI.
//
// Launch sequence per batch (stream-ordered, no host round trip):
//   per-level walk, for every level l:
//     k_grid64      g^d lattice of every active scan's box, FP64      -> ws
//     k_pl_level    one wavefront per scan: parent / child statistics by
//                   wavefront reductions, W/B test, selection          -> result, state
//   or, for lattices of at most 256 points and batches up to 1024 scans, every
//   level in one launch of k_pl_fused (walk_grid.hip), one workgroup per scan
//   paper walk:
//     k_grid64      decimated image of the whole grid                  -> ws
//     k_walk_paper  one wavefront per scan runs every level on those samples
//   k_roi32         ROI at full resolution in FP32, box read from the result -> ws
//   k_roi_pick      its maximal-energy voxel, decided in FP64 over the FP32
//                   near-maximal candidates (walk_roi.hip)         -> result, roi_img
// Every energy a decision rests on is evaluated in FP64, so each decision is taken
// in the same precision as a double-precision reference and does not hinge on FP32
// rounding.
#include <climits>
#include <cmath>

#include "uwb_internal.h"
#include "walk_internal.h"
#include "walk_level.h"

namespace uwb {
namespace {

constexpr int kWaves = kBlock / 64;

// ----------------------------------------------------------------------------
// block reduction of small vectors (all threads get the result)
// ----------------------------------------------------------------------------
template <int N>
__device__ void block_max(double (&v)[N], double *red) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_max(v[i]);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) red[w * N + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double s = red[i];
        for (int k = 1; k < kWaves; ++k) s = fmax(s, red[k * N + i]);
        v[i] = s;
    }
}

// FP64 energies of every point of lattice L into lv (LDS), trace spans staged in LDS.
__device__ void eval_lattice(const WalkArgs &a, const ScanConst &sc, const Lattice &L, double *lv, Stage &st,
                             int *tmp) {
    const int tid = threadIdx.x;
    const int P = L.count();
    int blo[3], bhi[3];
    for (int d = 0; d < 3; ++d) { blo[d] = L.x0[d]; bhi[d] = L.x0[d] + L.step * (L.cnt[d] - 1); }
    const bool staged = stage_box(st, tmp, sc, a.ss.n_ant, a.ss.n_samp, a.window, a.g, blo, bhi);
    int G = kBlock / P;                 // lanes per point
    if (G > 64) G = 64;
    if (G < 1) G = 1;
    G = 1 << (31 - __clz(G));
    const int per = kBlock / G;
    for (int q0 = 0; q0 < P; q0 += per) {
        const int p = q0 + tid / G;
        const bool ok = p < P;
        int x, y, z;
        L.coord(ok ? p : 0, x, y, z);
        const double rx = a.g.origin[0] + x * a.g.pitch[0];
        const double ry = a.g.origin[1] + y * a.g.pitch[1];
        const double rz = a.g.origin[2] + z * a.g.pitch[2];
        const double e = energy64_dispatch(a.bf, sc, a.ss.n_ant, a.ss.n_samp, a.window, rx, ry, rz, tid % G, G,
                                           staged ? &st : nullptr);
        if (ok && tid % G == 0) lv[p] = e;
    }
    __syncthreads();
}

// ----------------------------------------------------------------------------
// k_walk_paper: the ROI-selection loop of the three-phase walk, one wavefront
// per scan, over the samples of the decimated image (computed once).
// ----------------------------------------------------------------------------
template <int NACT>
__global__ __launch_bounds__(kBlock) void k_walk_paper(const WalkArgs a, int n_scans) {
    const int scan = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (scan >= n_scans) return;   // uniform per wavefront
    const int tid = threadIdx.x & 63;
    constexpr int nact = NACT;
    constexpr int nchild = 1 << NACT;
    const int dims[3] = {a.g.dims[0], a.g.dims[1], a.g.dims[2]};
    uwb_segment_result &R = a.out[scan];

    int box[6] = {0, dims[0], 0, dims[1], 0, dims[2]};
    if (tid == 0)
        for (int i = 0; i < 6; ++i) R.box[0][i] = box[i];
    double prev_n = 0, prev_mean = 0, prev_m2 = 0, prevW = 0, prevB = 0;
    int n_kept = 0, made = 0, n_wb = 0;

    Lattice L;
    for (int d = 0; d < 3; ++d) { L.x0[d] = a.dec_x0[d]; L.cnt[d] = a.dec_cnt[d]; }
    L.step = a.decimation;
    const double *src = a.dec64 + (int64_t)scan * a.dec_count;
    const int64_t nvox = L.count();

    for (int lev = 0; lev <= a.depth; ++lev) {
        if (lev == a.depth && a.term != UWB_TERM_WB) { n_kept = a.depth; break; }
        int cbox[8][6];
        double sc8[8];
        const LevelStats ls = wave_level_stats<NACT>(a, L, src, box, 0, true, cbox, sc8);
        const double pn = ls.pn, pmean = ls.pmean, pm2 = ls.pm2;
        double cmin = INFINITY;
        for (int c = 0; c < nchild; ++c) cmin = fmin(cmin, ls.count[c]);

        // Eq. (6)-(7) stop on the previous and the current box's samples
        bool stop = false;
        if (a.term == UWB_TERM_WB && lev >= 1) {
            const double pooled = (prev_n * prev_mean + pn * pmean) / (prev_n + pn);
            const double W = prev_m2 + pm2;
            const double B = prev_n * (prev_mean - pooled) * (prev_mean - pooled) + pn * (pmean - pooled) * (pmean - pooled);
            if (tid == 0) { R.wb[n_wb][0] = W; R.wb[n_wb][1] = B; }
            ++n_wb;
            if (lev >= 2 && (B <= prevB || W >= prevW)) { n_kept = lev - 1; stop = true; }
            prevW = W;
            prevB = B;
        }
        if (stop) break;
        prev_n = pn;
        prev_mean = pmean;
        prev_m2 = pm2;
        if (lev == a.depth) { n_kept = a.depth; break; }
        if (cmin < kMinChildSamples) { n_kept = lev; break; }
        // select the child (lowest index within the tie band)
        double best = -INFINITY;
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (c < nchild) best = fmax(best, sc8[c]);
        const double thr = best - kTieRel * fabs(best);
        int sel = 0;
#pragma unroll
        for (int c = 7; c >= 0; --c)
            if (c < nchild && sc8[c] >= thr) sel = c;
        int sbox[6];   // the chosen child's box formed again (a runtime index into cbox would place it in scratch)
        split_box(box, sel, nact, sbox);
        expand_box(sbox, a.frame_level, nact, dims, box);
        if (tid == 0) {
            R.child[made] = sel;
#pragma unroll
            for (int c = 0; c < 8; ++c) R.score[made][c] = c < nchild ? sc8[c] : 0.0;
            for (int i = 0; i < 6; ++i) R.box[lev + 1][i] = box[i];
        }
        ++made;
    }
    if (tid == 0) {
        int roi[6];
        expand_box(R.box[n_kept], a.frame_final, nact, dims, roi);
        R.n_levels = n_kept;
        R.term_level = made;
        R.decimation = a.decimation;
        R.n_samples_level0 = (int)a.dec_count;
        R.n_wb = n_wb;
        for (int i = 0; i < 6; ++i) R.roi[i] = roi[i];
        const int64_t rv = (int64_t)(roi[1] - roi[0]) * (roi[3] - roi[2]) * (roi[5] - roi[4]);
        R.voxels_evaluated = nvox + rv;
        R.argmax = -1;
        R.peak = 0.0;
        R.learned_mask = 0;
        R.guard_hits = 0;
    }
}

// ----------------------------------------------------------------------------
// Level-synchronous per-level walk: for every level, k_grid64 images the g^d
// lattice of each active scan's box (many workgroups per scan) and k_pl_level
// takes that level's statistics, W/B test and decision (one wavefront per
// scan), carrying the previous level's figures in PLState.
// ----------------------------------------------------------------------------
__global__ void k_pl_init(const WalkArgs a, int n_scans) {
    const int scan = blockIdx.x * blockDim.x + threadIdx.x;
    if (scan >= n_scans) return;
    pl_init_state(a, a.state[scan]);
    uwb_segment_result &R = a.out[scan];
    const int full[6] = {0, a.g.dims[0], 0, a.g.dims[1], 0, a.g.dims[2]};
    for (int i = 0; i < 6; ++i) R.box[0][i] = full[i];
}

template <int NACT>
__global__ __launch_bounds__(kBlock) void k_pl_level(const WalkArgs a, int lev, int n_scans) {
    const int scan = blockIdx.x * kWaves + (threadIdx.x >> 6);   // one wavefront per scan
    if (scan >= n_scans) return;
    pl_level_step<NACT>(a, lev, scan);
}

// The same level step with a workgroup per scan, for octree lattices of more than
// kWaveStatsPoints points: the four wavefronts take the statistics together.
template <int NACT>
__global__ __launch_bounds__(kBlock) void k_pl_level_wg(const WalkArgs a, int lev) {
    __shared__ double red[kWaves * (3 * 8 + 3)];
    const int scan = blockIdx.x;
    PLState st = a.state[scan];
    if (!st.active) return;   // uniform per workgroup
    int box[6];
    for (int i = 0; i < 6; ++i) box[i] = a.out[scan].box[lev][i];
    const int P = NACT == 3 ? a.coarse * a.coarse * a.coarse : a.coarse * a.coarse;
    const double *src = a.lat64 + (int64_t)scan * a.lat_stride + (int64_t)lev * P;
    pl_level_core<NACT, kWaves>(a, lev, scan, st, src, box, red);
    if (threadIdx.x == 0) a.state[scan] = st;
}

__global__ void k_pl_finish(const WalkArgs a, int n_scans) {
    const int scan = blockIdx.x * blockDim.x + threadIdx.x;
    if (scan >= n_scans) return;
    pl_finish_record(a, a.state[scan], a.out[scan]);
}

// ----------------------------------------------------------------------------
// k_composite: the mixed-resolution image of the final-imaging phase (Section III):
// full resolution inside the ROI; elsewhere every voxel takes the coarse sample
// whose block holds it -- for the paper walk the decimated lattice (block
// [D k, D k + D), the last block running to the grid's end), for the per-level
// walk the deepest imaged level whose box holds the voxel.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_composite(const WalkArgs a, float *img) {
    const int scan = blockIdx.y;
    const int nx = a.g.dims[0], ny = a.g.dims[1], nz = a.g.dims[2];
    const int64_t nv = (int64_t)nx * ny * nz;
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv) return;
    const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((int64_t)nx * ny));
    const uwb_segment_result &R = a.out[scan];
    double val;
    if (in_box(R.roi, x, y, z)) {
        const int rnx = R.roi[1] - R.roi[0], rny = R.roi[3] - R.roi[2];
        val = a.roi32[(int64_t)scan * a.roi_cap + ((int64_t)(z - R.roi[4]) * rny + (y - R.roi[2])) * rnx + (x - R.roi[0])];
    } else if (a.walk == UWB_WALK_PAPER) {
        const int D = a.decimation;
        const int kx = min(x / D, a.dec_cnt[0] - 1), ky = min(y / D, a.dec_cnt[1] - 1);
        const int kz = nz > 1 ? min(z / D, a.dec_cnt[2] - 1) : 0;
        val = a.dec64[(int64_t)scan * a.dec_count + ((int64_t)kz * a.dec_cnt[1] + ky) * a.dec_cnt[0] + kx];
    } else {
        const int nact = nz > 1 ? 3 : 2;
        const int P = a.coarse * a.coarse * (nact == 3 ? a.coarse : 1);
        const int imaged = a.term == UWB_TERM_WB ? R.term_level + 1 : R.term_level;
        int l = imaged - 1;
        while (l > 0 && !in_box(R.box[l], x, y, z)) --l;
        const int step = (nx >> l) / a.coarse;
        const int kx = (x - R.box[l][0]) / step, ky = (y - R.box[l][2]) / step;
        const int kz = nact == 3 ? (z - R.box[l][4]) / step : 0;
        val = a.lat64[(int64_t)scan * a.lat_stride + (int64_t)l * P + ((int64_t)kz * a.coarse + ky) * a.coarse + kx];
    }
    img[(int64_t)scan * nv + v] = (float)val;
}

// ----------------------------------------------------------------------------
// Learned walk (per-level quadtree, g = 32, planar): each level images the box's
// 32 x 32 lattice (DAS, FP64), scores the children with the configured metric,
// and writes the lattice normalised by its maximum as the CNN's BF16 input; after
// the batched CNN forward, k_learn_decide keeps the CNN's child when its
// probability reaches the threshold and the metric's child otherwise.
// ----------------------------------------------------------------------------
constexpr int kLearnG = 32;

__device__ void lattice_of_box(const int *box, int side, Lattice &L) {
    const int step = side / kLearnG;
    L.x0[0] = box[0] + step / 2;
    L.x0[1] = box[2] + step / 2;
    L.x0[2] = 0;
    L.cnt[0] = kLearnG;
    L.cnt[1] = kLearnG;
    L.cnt[2] = 1;
    L.step = step;
}

// normalise lv (kLearnG^2 values) by its maximum and store it as BF16 [y][x]
__device__ void write_cnn_input(const double *lv, double *red, uint16_t *x) {
    double m[1] = {-INFINITY};
    for (int p = threadIdx.x; p < kLearnG * kLearnG; p += kBlock) m[0] = fmax(m[0], lv[p]);
    block_max(m, red);
    const double inv = m[0] > 0.0 ? 1.0 / m[0] : 1.0;
    for (int p = threadIdx.x; p < kLearnG * kLearnG; p += kBlock) x[p] = f2bf((float)(lv[p] * inv));
}

__global__ __launch_bounds__(kBlock) void k_learn_level(const WalkArgs a, int lev, int n_scans, uint16_t *xin,
                                                        int *fb_child) {
    const int scan = blockIdx.x * kWaves + (threadIdx.x >> 6);   // one wavefront per scan
    if (scan >= n_scans) return;
    const int lane = threadIdx.x & 63;
    uwb_segment_result &R = a.out[scan];
    int box[6];
    for (int i = 0; i < 6; ++i) box[i] = R.box[lev][i];
    const int side = a.g.dims[0] >> lev;
    Lattice L;
    lattice_of_box(box, side, L);
    const double *lv = a.lat64 + (int64_t)scan * a.lat_stride + (int64_t)lev * kLearnG * kLearnG;
    int cbox[8][6];
    double sc8[8];
    wave_level_stats<2>(a, L, lv, box, side, false, cbox, sc8);
    double best = -INFINITY;
#pragma unroll
    for (int c = 0; c < 4; ++c) best = fmax(best, sc8[c]);
    const double thr = best - kTieRel * fabs(best);
    int sel = 0;
#pragma unroll
    for (int c = 3; c >= 0; --c)
        if (sc8[c] >= thr) sel = c;
    if (lane == 0) {
        fb_child[scan] = sel;
#pragma unroll
        for (int c = 0; c < 8; ++c) R.score[lev][c] = c < 4 ? sc8[c] : 0.0;
    }
    // the CNN input: the lattice divided by its maximum, BF16, [y][x]
    double m = -INFINITY;
    for (int p = lane; p < kLearnG * kLearnG; p += 64) m = fmax(m, lv[p]);
    m = wave_max(m);
    const double inv = m > 0.0 ? 1.0 / m : 1.0;
    uint16_t *x = xin + (size_t)scan * kLearnG * kLearnG;
    for (int p = lane; p < kLearnG * kLearnG; p += 64) x[p] = f2bf((float)(lv[p] * inv));
}

__global__ void k_learn_decide(const WalkArgs a, int lev, int n_scans, const float *probs, const int *fb_child,
                               float threshold) {
    const int scan = blockIdx.x * blockDim.x + threadIdx.x;
    if (scan >= n_scans) return;
    uwb_segment_result &R = a.out[scan];
    const float *p = probs + 4 * scan;
    float pm = p[0];
    int arg = 0;
    for (int c = 1; c < 4; ++c)
        if (p[c] > pm) { pm = p[c]; arg = c; }
    int child = fb_child[scan];
    int mask = lev == 0 ? 0 : R.learned_mask;
    if (pm >= threshold) {
        child = arg;
        mask |= 1 << lev;
    }
    R.learned_mask = mask;
    R.child[lev] = child;
    int nb[6];
    split_box(R.box[lev], child, 2, nb);
    for (int i = 0; i < 6; ++i) R.box[lev + 1][i] = nb[i];
}

__global__ void k_learn_finish(const WalkArgs a, int depth, int n_scans) {
    const int scan = blockIdx.x * blockDim.x + threadIdx.x;
    if (scan >= n_scans) return;
    uwb_segment_result &R = a.out[scan];
    int roi[6];
    const int dims[3] = {a.g.dims[0], a.g.dims[1], a.g.dims[2]};
    expand_box(R.box[depth], a.frame_final, 2, dims, roi);
    R.n_levels = depth;
    R.term_level = depth;
    R.decimation = 0;
    R.n_samples_level0 = kLearnG * kLearnG;
    R.n_wb = 0;
    for (int i = 0; i < 6; ++i) R.roi[i] = roi[i];
    const int64_t rv = (int64_t)(roi[1] - roi[0]) * (roi[3] - roi[2]) * (roi[5] - roi[4]);
    R.voxels_evaluated = (int64_t)depth * kLearnG * kLearnG + rv;
    R.argmax = -1;
    R.peak = 0.0;
    R.guard_hits = 0;
}

// Training inputs: the coarse DAS lattice of every box on the path to `target`
// (the aligned boxes of side N / 2^l that contain it), and the child holding it.
__global__ __launch_bounds__(kBlock) void k_cnn_inputs(const WalkArgs a, const uwb_peak *targets, int depth,
                                                       uint16_t *xin, int *labels) {
    extern __shared__ __align__(16) unsigned char dsm[];
    double *lv = reinterpret_cast<double *>(dsm);
    __shared__ double red[kWaves * 32];
    __shared__ int tmp[kWaves];
    Stage st;
    st.lo = reinterpret_cast<int *>(dsm + sizeof(double) * a.pmax);
    st.off = st.lo + a.stage_ant;
    st.len = st.off + a.stage_ant;
    st.buf = reinterpret_cast<float *>(st.len + a.stage_ant);
    st.cap = a.stage_cap;
    const int lev = blockIdx.x, scan = blockIdx.y;
    const ScanConst sc = scan_const(a.ss, scan);
    const int64_t t = targets[scan].index;
    const int nx = a.g.dims[0];
    const size_t k = (size_t)scan * depth + lev;
    if (t < 0 || t >= (int64_t)nx * a.g.dims[1]) {     // no target: zero input, masked label
        for (int p = threadIdx.x; p < kLearnG * kLearnG; p += kBlock) xin[k * kLearnG * kLearnG + p] = 0;
        if (threadIdx.x == 0) labels[k] = -1;
        return;
    }
    const int tx = (int)(t % nx), ty = (int)(t / nx);
    const int side = a.g.dims[0] >> lev;
    int box[6] = {(tx / side) * side, (tx / side) * side + side, (ty / side) * side, (ty / side) * side + side, 0, 1};
    Lattice L;
    lattice_of_box(box, side, L);
    eval_lattice(a, sc, L, lv, st, tmp);
    write_cnn_input(lv, red, xin + k * kLearnG * kLearnG);
    if (threadIdx.x == 0) labels[k] = (tx >= box[0] + side / 2 ? 1 : 0) + (ty >= box[2] + side / 2 ? 2 : 0);
}
}  // namespace

static int64_t lattice_size(const WalkArgs *a) {   // coarse^d points of a per-level lattice
    return (int64_t)a->coarse * a->coarse * (a->g.dims[2] > 1 ? a->coarse : 1);
}

static int64_t lattice_slot(const WalkArgs *a) {   // every level's lattice of one scan
    return a->walk == UWB_WALK_PER_LEVEL ? (int64_t)(a->depth + 1) * lattice_size(a) : 0;
}

static int64_t lattice_points(int n, int step) {   // points D*k + floor(D/2) < n
    const int first = step / 2;
    return first < n ? (int64_t)(n - 1 - first) / step + 1 : 0;
}

static int64_t lattice_in(int lo, int hi, int step) {  // lattice coordinates inside [lo, hi)
    int64_t c = 0;
    for (int x = lo; x < hi; ++x) c += (x % step) == step / 2;
    return c;
}

int plan_walk(const GridView &g, const uwb_segment_tree *t, int n_scans, WalkArgs *a, int64_t *roi_bound,
              size_t *ws_bytes) {
    if (!t) return UWB_EINVAL;
    if (t->beamformer != UWB_DAS && t->beamformer != UWB_DMAS && t->beamformer != UWB_MVDR) return UWB_EINVAL;
    if (t->walk != UWB_WALK_PER_LEVEL && t->walk != UWB_WALK_PAPER) return UWB_EINVAL;
    if (t->metric < UWB_MEAN || t->metric > UWB_EQ5_CLAMPED) return UWB_EINVAL;
    if (t->term != UWB_TERM_FIXED_DEPTH && t->term != UWB_TERM_WB) return UWB_EINVAL;
    if (!std::isfinite(t->frame_level) || t->frame_level < 0 || !std::isfinite(t->frame_final) || t->frame_final < 0)
        return UWB_EINVAL;
    if (t->max_depth < 0) return UWB_EINVAL;
    if (t->max_depth > UWB_MAX_LEVELS) return UWB_ERANGE;
    if (n_scans < 1) return UWB_EINVAL;
    const int nact = g.dims[2] > 1 ? 3 : 2;
    a->g = g;
    a->bf = t->beamformer;
    a->walk = t->walk;
    a->metric = t->metric;
    a->term = t->term;
    a->frame_level = t->frame_level;
    a->frame_final = t->frame_final;
    a->coarse = t->coarse;
    a->decimation = 0;
    a->dec_count = 0;
    for (int d = 0; d < 3; ++d) { a->dec_x0[d] = 0; a->dec_cnt[d] = 1; }
    int64_t bound = 0;
    if (t->walk == UWB_WALK_PER_LEVEL) {
        const int n = g.dims[0], gc = t->coarse;
        if (g.dims[1] != n || (nact == 3 && g.dims[2] != n)) return UWB_EINVAL;
        if (gc < 2 || gc % 2 || gc > 64) return UWB_EINVAL;
        int64_t pts = 1;
        for (int d = 0; d < nact; ++d) pts *= gc;
        if (pts > kMaxCoarsePoints) return UWB_EUNSUPPORTED;
        if (n % gc) return UWB_EINVAL;
        const int q = n / gc;
        if (q & (q - 1)) return UWB_EINVAL;
        int top = 0;
        while ((1 << top) < q) ++top;
        int depth = t->max_depth == 0 ? top : (t->max_depth < top ? t->max_depth : top);
        if (depth > UWB_MAX_LEVELS) return UWB_ERANGE;
        a->depth = depth;
        const int kept_min = t->term == UWB_TERM_WB ? (depth < 1 ? depth : 1) : depth;
        const int s = n >> kept_min;
        int64_t side = s + 2 * (int64_t)std::floor(t->frame_final * (double)s);
        if (side > n) side = n;
        bound = 1;
        for (int d = 0; d < nact; ++d) bound *= side;
        for (int d = 0; d < 3; ++d) a->roi_side[d] = d < nact ? (int)side : 1;
    } else {
        int dec = t->decimation;
        if (dec < 0) return UWB_EINVAL;
        if (dec == 0) {
            if (!std::isfinite(t->min_tumour) || t->min_tumour <= 0) return UWB_EINVAL;
            const double dd = std::floor(t->min_tumour / (std::sqrt(2.0) * g.pitch[0]));
            if (!(dd < 2147483647.0)) return UWB_EUNSUPPORTED;
            dec = dd < 1.0 ? 1 : (int)dd;
        }
        for (int d = 0; d < nact; ++d)
            if (dec > g.dims[d]) return UWB_EINVAL;
        a->decimation = dec;
        int64_t cnt = 1;
        for (int d = 0; d < nact; ++d) {
            a->dec_x0[d] = dec / 2;
            a->dec_cnt[d] = (int)lattice_points(g.dims[d], dec);
            cnt *= a->dec_cnt[d];
        }
        a->dec_count = cnt;
        const int depth = t->max_depth == 0 ? UWB_MAX_LEVELS : t->max_depth;
        a->depth = depth;
        // can the walk stop before its first split?  (data-independent: child sample counts)
        int64_t cmin = INT64_MAX;
        for (int c = 0; c < (1 << nact); ++c) {
            int64_t k = 1;
            for (int d = 0; d < nact; ++d) {
                const int mid = g.dims[d] / 2;
                k *= ((c >> d) & 1) ? lattice_in(mid, g.dims[d], dec) : lattice_in(0, mid, dec);
            }
            cmin = k < cmin ? k : cmin;
        }
        const int lmin = (depth >= 1 && cmin >= (int64_t)kMinChildSamples) ? 1 : 0;
        // largest box side per axis at each level, then the largest ROI over reachable levels
        int64_t side[3] = {g.dims[0], g.dims[1], g.dims[2]};
        for (int d = 0; d < 3; ++d) a->roi_side[d] = 1;
        for (int l = 0; l <= depth; ++l) {
            if (l >= lmin) {
                int64_t v = 1;
                for (int d = 0; d < nact; ++d) {
                    int64_t r = side[d] + 2 * (int64_t)std::floor(t->frame_final * (double)side[d]);
                    r = r < g.dims[d] ? r : g.dims[d];
                    v *= r;
                    if (r > a->roi_side[d]) a->roi_side[d] = (int)r;
                }
                bound = v > bound ? v : bound;
            }
            for (int d = 0; d < nact; ++d) {
                const int64_t c = (side[d] + 1) / 2;
                int64_t s2 = c + 2 * (int64_t)std::floor(t->frame_level * (double)c);
                side[d] = s2 < g.dims[d] ? s2 : g.dims[d];
            }
        }
    }
    *roi_bound = bound;
    a->roi_cap = bound;
    const size_t lat = (size_t)lattice_slot(a);
    *ws_bytes = 4 * 256 + (size_t)n_scans * (4 * (size_t)bound + 8 * ((size_t)a->dec_count + lat) + sizeof(PLState));
    return UWB_OK;
}

static uintptr_t align256(uintptr_t p) { return (p + 255) & ~(uintptr_t)255; }

void assign_walk_ws(WalkArgs *a, void *ws, int n_scans) {
    uintptr_t p = align256((uintptr_t)ws);
    a->roi32 = reinterpret_cast<float *>(p);
    p = align256(p + (size_t)n_scans * a->roi_cap * 4);
    a->dec64 = reinterpret_cast<double *>(p);
    p = align256(p + (size_t)n_scans * a->dec_count * 8);
    a->lat64 = reinterpret_cast<double *>(p);
    a->lat_stride = lattice_slot(a);
    p = align256(p + (size_t)n_scans * a->lat_stride * 8);
    a->state = reinterpret_cast<PLState *>(p);
}

// LDS sizes of the walk kernels for M antennas (stage tables for up to kStageMaxAnt).
void size_walk_lds(WalkArgs *a, int n_ant) {
    constexpr int kWalkLds = 60 * 1024, kLatticeLds = 40 * 1024;
    a->pmax = a->walk == UWB_WALK_PER_LEVEL ? a->coarse * a->coarse * (a->g.dims[2] > 1 ? a->coarse : 1) : 0;
    a->stage_ant = n_ant < kStageMaxAnt ? n_ant : kStageMaxAnt;
    const int fixed = 8 * a->pmax + 12 * a->stage_ant;
    a->stage_cap = (kWalkLds - fixed) / 4;
    if (a->stage_cap < 0) a->stage_cap = 0;
    a->lds_walk = (size_t)fixed + 4 * (size_t)a->stage_cap;
    a->lattice_stage_cap = (kLatticeLds - 12 * a->stage_ant) / 4;
    if (a->lattice_stage_cap < 0) a->lattice_stage_cap = 0;
    a->lds_lattice = (size_t)12 * a->stage_ant + 4 * (size_t)a->lattice_stage_cap;
}

// The per-level walk runs as one fused launch (one workgroup per scan, every level) when
// a level's lattice is one workgroup's worth of points and the batch is small enough
// that launch gaps, not occupancy, decide the time: measured on 512 x 512 scans, g = 16,
// 28 % faster at 256 scans, 3 % at 1024, 8 % slower at 4096; a lattice of several groups
// (g = 32) is slower fused at every batch size, its groups serialised in one workgroup.
constexpr int kFuseMaxScans = 1024;
static bool fuse_levels(const WalkArgs &a, int n_scans) {
    const int64_t pts = (int64_t)a.coarse * a.coarse * (a.g.dims[2] > 1 ? a.coarse : 1);
    return pts <= kBlock && n_scans <= kFuseMaxScans;
}

static Grid64Args grid_args(const WalkArgs &a, int mode) {
    Grid64Args g;
    g.ss = a.ss;
    g.g = a.g;
    g.window = a.window;
    g.bf = a.bf;
    g.mode = mode;
    g.lev = 0;
    g.coarse = a.coarse;
    g.step = 1;
    for (int d = 0; d < 3; ++d) { g.x0[d] = 0; g.cnt[d] = 1; }
    g.res = a.out;
    g.state = nullptr;
    g.out64 = nullptr;
    g.out_stride = 0;
    g.out_offset = 0;
    g.out32 = nullptr;
    g.out32_stride = 0;
    return g;
}

// Two walks of the same scans agree when their final ROIs intersect.
__global__ void k_roi_overlap(const uwb_segment_result *ra, const uwb_segment_result *rb, int32_t *agree, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool ov = true;
    for (int d = 0; d < 3; ++d)
        ov = ov && max(ra[i].roi[2 * d], rb[i].roi[2 * d]) < min(ra[i].roi[2 * d + 1], rb[i].roi[2 * d + 1]);
    agree[i] = ov ? 1 : 0;
}

int launch_roi_overlap(const uwb_segment_result *ra, const uwb_segment_result *rb, int32_t *agree, int n,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_roi_overlap, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ra, rb, agree, n);
    return hipGetLastError() == hipSuccess ? UWB_OK : UWB_EHIP;
}

int launch_composite(const WalkArgs &a, int n_scans, float *img, hipStream_t st) {
    const int64_t nv = (int64_t)a.g.dims[0] * a.g.dims[1] * a.g.dims[2];
    const int64_t nb = (nv + kBlock - 1) / kBlock;
    if (nb > 0x7fffffff || n_scans > 65535) return UWB_EUNSUPPORTED;
    hipLaunchKernelGGL(k_composite, dim3((unsigned)nb, n_scans), dim3(kBlock), 0, st, a, img);
    return hipGetLastError() == hipSuccess ? UWB_OK : UWB_EHIP;
}

int launch_walk(const WalkArgs &a, int n_scans, hipStream_t st) {
    int rc;
    if (a.walk == UWB_WALK_PAPER) {
        Grid64Args g = grid_args(a, kGridFixed);
        g.step = a.decimation;
        for (int d = 0; d < 3; ++d) { g.x0[d] = a.dec_x0[d]; g.cnt[d] = a.dec_cnt[d]; }
        g.out64 = a.dec64;
        g.out_stride = a.dec_count;
        if ((rc = launch_grid64(g, a.dec_cnt, a.decimation, n_scans, st))) return rc;
        const dim3 gw((unsigned)((n_scans + kWaves - 1) / kWaves));
        if (a.g.dims[2] > 1) hipLaunchKernelGGL(k_walk_paper<3>, gw, dim3(kBlock), 0, st, a, n_scans);
        else hipLaunchKernelGGL(k_walk_paper<2>, gw, dim3(kBlock), 0, st, a, n_scans);
    } else {
        const unsigned nb = (unsigned)((n_scans + 255) / 256);
        const int levels = a.term == UWB_TERM_WB ? a.depth + 1 : a.depth;
        const int nact = a.g.dims[2] > 1 ? 3 : 2;
        const int cnt[3] = {a.coarse, a.coarse, nact == 3 ? a.coarse : 1};
        // the fused kernel sets up and finishes the walk itself
        const bool fused = levels >= 1 && fuse_levels(a, n_scans);
        if (!fused) hipLaunchKernelGGL(k_pl_init, dim3(nb), dim3(256), 0, st, a, n_scans);
        if (fused) {
            Grid64Args g = grid_args(a, kGridBox);
            g.state = a.state;
            g.out64 = a.lat64;
            g.out_stride = a.lat_stride;
            if ((rc = launch_pl_fused(g, a, levels, n_scans, st))) return rc;
        }
        for (int lev = 0; !fused && lev < levels; ++lev) {
            Grid64Args g = grid_args(a, kGridBox);
            g.lev = lev;
            g.step = (a.g.dims[0] >> lev) / a.coarse;
            g.state = a.state;
            g.out64 = a.lat64;
            g.out_stride = a.lat_stride;
            g.out_offset = (int64_t)lev * cnt[0] * cnt[1] * cnt[2];
            if ((rc = launch_grid64(g, cnt, g.step, n_scans, st))) return rc;
            // octree lattices of more than kWaveStatsPoints points: a workgroup per scan (chosen by the lattice
            // alone, so that a scan's walk does not depend on its batch; planar lattices keep one wavefront per
            // scan, as the learned walk's metric fallback does, whose scores equal the metric walk's bit for bit)
            if (nact == 3 && (int64_t)cnt[0] * cnt[1] * cnt[2] > kWaveStatsPoints) {
                hipLaunchKernelGGL(k_pl_level_wg<3>, dim3((unsigned)n_scans), dim3(kBlock), 0, st, a, lev);
            } else {
                const dim3 gw((unsigned)((n_scans + kWaves - 1) / kWaves));
                if (nact == 3) hipLaunchKernelGGL(k_pl_level<3>, gw, dim3(kBlock), 0, st, a, lev, n_scans);
                else hipLaunchKernelGGL(k_pl_level<2>, gw, dim3(kBlock), 0, st, a, lev, n_scans);
            }
        }
        if (!fused) hipLaunchKernelGGL(k_pl_finish, dim3(nb), dim3(256), 0, st, a, n_scans);
    }
    if ((rc = launch_roi(a, a.bf, n_scans, st))) return rc;
    return hipGetLastError() == hipSuccess ? UWB_OK : UWB_EHIP;
}

}  // namespace uwb


namespace uwb {

int launch_learned(const WalkArgs &a, int n_scans, uwb_cnn *cnn, float threshold, uint16_t *xin, float *probs,
                   int *fb_child, int roi_bf, hipStream_t st) {
    WalkArgs levels = a;
    levels.bf = UWB_DAS;     // the proposer and the fallback metric look at the coarse DAS image
    const unsigned nb = (unsigned)((n_scans + 255) / 256);
    hipLaunchKernelGGL(k_pl_init, dim3(nb), dim3(256), 0, st, levels, n_scans);
    const int cnt[3] = {kLearnG, kLearnG, 1};
    int rc;
    for (int lev = 0; lev < a.depth; ++lev) {
        Grid64Args g = grid_args(levels, kGridBox);
        g.lev = lev;
        g.step = (a.g.dims[0] >> lev) / kLearnG;
        g.out64 = a.lat64;
        g.out_stride = a.lat_stride;
        g.out_offset = (int64_t)lev * kLearnG * kLearnG;
        if ((rc = launch_grid64(g, cnt, g.step, n_scans, st))) return rc;
        hipLaunchKernelGGL(k_learn_level, dim3((unsigned)((n_scans + kWaves - 1) / kWaves)), dim3(kBlock), 0, st,
                           levels, lev, n_scans, xin, fb_child);
        if (hipGetLastError() != hipSuccess) return UWB_EHIP;
        const int s = uwb_cnn_forward(cnn, xin, n_scans, probs, (void *)st);
        if (s) return s;
        hipLaunchKernelGGL(k_learn_decide, dim3((n_scans + 255) / 256), dim3(256), 0, st, levels, lev, n_scans, probs,
                           fb_child, threshold);
    }
    hipLaunchKernelGGL(k_learn_finish, dim3((n_scans + 255) / 256), dim3(256), 0, st, levels, a.depth, n_scans);
    if ((rc = launch_roi(a, roi_bf, n_scans, st))) return rc;
    return hipGetLastError() == hipSuccess ? UWB_OK : UWB_EHIP;
}

int launch_cnn_inputs(const WalkArgs &a, int n_scans, const uwb_peak *targets, uint16_t *xin, int *labels,
                      hipStream_t st) {
    WalkArgs w = a;
    w.bf = UWB_DAS;
    hipLaunchKernelGGL(k_cnn_inputs, dim3(a.depth, n_scans), dim3(kBlock), a.lds_walk, st, w, targets, a.depth, xin,
                       labels);
    return hipGetLastError() == hipSuccess ? UWB_OK : UWB_EHIP;
}

}  // namespace uwb
