// Per-level statistics and decisions of the segment walk (Section III), shared by the
// level-synchronous kernels (walk.hip) and the fused per-level walk (walk_grid.hip).
#pragma once

#include <cmath>

#include "walk_internal.h"

namespace uwb {

// ----------------------------------------------------------------------------
// sample sets: a lattice of points with values, and membership in boxes
// ----------------------------------------------------------------------------
struct Lattice {
    int x0[3];      // finest index of lattice point k = 0 along each axis
    int step;       // D
    int cnt[3];     // points per axis
    __device__ int count() const { return cnt[0] * cnt[1] * cnt[2]; }
    __device__ void coord(int p, int &x, int &y, int &z) const {
        const int kx = p % cnt[0], ky = (p / cnt[0]) % cnt[1], kz = p / (cnt[0] * cnt[1]);
        x = x0[0] + step * kx;
        y = x0[1] + step * ky;
        z = x0[2] + step * kz;
    }
};

// The points p, p + stride, p + 2 stride, ... of a lattice in order, their finest indices
// formed by carries instead of a division per point (the divisions are done once).
struct LatticeCursor {
    int kx, ky, kz, dx, dy, dz, cx, cy;
    __device__ LatticeCursor(const Lattice &L, int p, int stride) {
        cx = L.cnt[0];
        cy = L.cnt[1];
        kx = p % cx; ky = (p / cx) % cy; kz = p / (cx * cy);
        dx = stride % cx; dy = (stride / cx) % cy; dz = stride / (cx * cy);
    }
    __device__ void coord(const Lattice &L, int &x, int &y, int &z) const {
        x = L.x0[0] + L.step * kx;
        y = L.x0[1] + L.step * ky;
        z = L.x0[2] + L.step * kz;
    }
    // dx < cx and dy < cy: at most one carry into each next index
    __device__ void advance() {
        kx += dx;
        const int c0 = kx >= cx;
        kx -= c0 ? cx : 0;
        ky += dy + c0;
        const int c1 = ky >= cy;
        ky -= c1 ? cy : 0;
        kz += dz + c1;
    }
};

__device__ __forceinline__ bool in_box(const int *b, int x, int y, int z) {
    return x >= b[0] && x < b[1] && y >= b[2] && y < b[3] && z >= b[4] && z < b[5];
}

// child c of box b, split at lo + floor(side/2) along the active axes (Morton bits)
__device__ __forceinline__ void split_box(const int *b, int c, int nact, int *out) {
    for (int i = 0; i < 6; ++i) out[i] = b[i];
    for (int d = 0; d < nact; ++d) {
        const int lo = b[2 * d], hi = b[2 * d + 1];
        const int mid = lo + (hi - lo) / 2;
        if ((c >> d) & 1) out[2 * d] = mid;
        else out[2 * d + 1] = mid;
    }
}

// widen each active side by floor(frac * side) on both ends, clipped to the grid
__device__ __forceinline__ void expand_box(const int *b, double frac, int nact, const int *dims, int *out) {
    for (int i = 0; i < 6; ++i) out[i] = b[i];
    for (int d = 0; d < nact; ++d) {
        const int lo = b[2 * d], hi = b[2 * d + 1];
        const int e = (int)floor(frac * (double)(hi - lo));
        out[2 * d] = max(0, lo - e);
        out[2 * d + 1] = min(dims[d], hi + e);
    }
}

// Decision metric of Section III on one child set (stats of raw and normalised values).
__device__ inline double metric_value(int metric, double n, double mean, double m2, double mx, double nmean, double nvar,
                               double pnvar) {
    switch (metric) {
        case UWB_MEAN: return mean;
        case UWB_VAR: return m2 / n;
        case UWB_MAX: return mx;
        case UWB_MAX_OVER_MEAN: return mean != 0.0 ? mx / mean : 0.0;
        case UWB_EQ5:
        case UWB_EQ5_CLAMPED: {
            double a = nvar > 0.0 ? (nvar - pnvar) / nvar : 0.0;
            if (metric == UWB_EQ5_CLAMPED) a = fmin(fmax(a, 0.0), 1.0);
            return (1.0 - a) * nmean + a * nvar;
        }
    }
    return 0.0;
}

struct LevelStats {
    double pn, pmean, pm2;
    double count[8];
};

// Largest octree lattice whose level statistics one wavefront takes; larger ones are split
// over the workgroup's four wavefronts (k_pl_level_wg).
constexpr int kWaveStatsPoints = 256;

// Combines each wavefront's reduced values v[0..n) over the WAVES wavefronts of the
// workgroup through LDS (red: WAVES x n doubles), in wavefront order: sums for the first
// nsum values, maxima for the rest.  Every thread of the workgroup calls it.
template <int WAVES>
__device__ __forceinline__ void combine_waves(double *v, int n, int nsum, double *red) {
    if constexpr (WAVES > 1) {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0)
            for (int i = 0; i < n; ++i) red[w * n + i] = v[i];
        __syncthreads();
        for (int i = 0; i < n; ++i) {
            double t = red[i];
            for (int k = 1; k < WAVES; ++k) t = i < nsum ? t + red[k * n + i] : fmax(t, red[k * n + i]);
            v[i] = t;
        }
        __syncthreads();   // red is free for the next combine
    }
}

// The same statistics for one scan on one wavefront (WAVES = 1, no workgroup barriers),
// or on a whole workgroup (WAVES = 4: wavefront w takes the points p with (p / 64) % 4 = w,
// and the wavefronts' sums are combined in wavefront order; red: LDS for the combine):
// for the per-level walk, whose every level's lattice lies inside its box, and for the
// paper walk (paper = true), whose samples are the decimated lattice points inside
// the current box.  Passes 2 and 3 run only when the metric or the W/B stop needs
// them.  Every lane returns the result.
template <int NACT, int WAVES = 1>
__device__ LevelStats wave_level_stats(const WalkArgs &a, const Lattice &L, const double *src, const int *box,
                                       int side, bool paper, int cbox[8][6], double sc8[8], double *red = nullptr) {
    constexpr int NCH = 1 << NACT;
    const int lane = threadIdx.x & 63;
    const int first = lane + 64 * (WAVES > 1 ? (int)(threadIdx.x >> 6) : 0), stride = 64 * WAVES;
    int sbx[NCH][6];
    const int half = side / 2;
    // the per-level walk scores each child on its box widened by the level frame; the
    // paper walk on the child's own samples
    const int efr = paper ? 0 : (int)floor(a.frame_level * (double)half);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        split_box(box, c, NACT, cbox[c]);
        for (int i = 0; i < 6; ++i) sbx[c][i] = cbox[c][i];
        for (int d = 0; d < NACT; ++d) {
            sbx[c][2 * d] = max(box[2 * d], cbox[c][2 * d] - efr);
            sbx[c][2 * d + 1] = min(box[2 * d + 1], cbox[c][2 * d + 1] + efr);
        }
    }
    const bool need2 = a.term == UWB_TERM_WB || a.metric == UWB_VAR || a.metric == UWB_EQ5 ||
                       a.metric == UWB_EQ5_CLAMPED;
    const bool need3 = a.metric == UWB_EQ5 || a.metric == UWB_EQ5_CLAMPED;
    // pass 1: counts, sums, maxima
    double pn = 0.0, psum = 0.0, pmax = -INFINITY;
    double cn[NCH], csum[NCH], cmx[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) { cn[c] = 0.0; csum[c] = 0.0; cmx[c] = -INFINITY; }
    for (LatticeCursor cur(L, first, stride); cur.kz < L.cnt[2]; cur.advance()) {
        const int p = (cur.kz * L.cnt[1] + cur.ky) * L.cnt[0] + cur.kx;
        int x, y, z;
        cur.coord(L, x, y, z);
        if (!in_box(box, x, y, z)) continue;
        const double v = src[p];
        pn += 1.0; psum += v; pmax = fmax(pmax, v);
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (in_box(sbx[c], x, y, z)) { cn[c] += 1.0; csum[c] += v; cmx[c] = fmax(cmx[c], v); }
    }
    pn = wave_sum(pn);
    psum = wave_sum(psum);
    pmax = wave_max(pmax);
#pragma unroll
    for (int c = 0; c < NCH; ++c) { cn[c] = wave_sum(cn[c]); csum[c] = wave_sum(csum[c]); cmx[c] = wave_max(cmx[c]); }
    if constexpr (WAVES > 1) {
        // the sums (counts, sums) lead, the maxima follow
        double w[3 * NCH + 3];
#pragma unroll
        for (int c = 0; c < NCH; ++c) { w[c] = cn[c]; w[NCH + c] = csum[c]; w[2 * NCH + 2 + c] = cmx[c]; }
        w[2 * NCH] = pn;
        w[2 * NCH + 1] = psum;
        w[3 * NCH + 2] = pmax;
        combine_waves<WAVES>(w, 3 * NCH + 3, 2 * NCH + 2, red);
#pragma unroll
        for (int c = 0; c < NCH; ++c) { cn[c] = w[c]; csum[c] = w[NCH + c]; cmx[c] = w[2 * NCH + 2 + c]; }
        pn = w[2 * NCH];
        psum = w[2 * NCH + 1];
        pmax = w[3 * NCH + 2];
    }
    const double pmean = psum / pn;
    const double scale = pmax > 0.0 ? pmax : 1.0;    // Eq. (5) normalisation
    // (the divisions below are taken only where the metric or a later pass uses them)
    const bool need_mean = need2 || a.metric == UWB_MEAN || a.metric == UWB_MAX_OVER_MEAN;
    double cmean[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) cmean[c] = need_mean ? csum[c] / cn[c] : 0.0;
    // pass 2: raw squared deviations and normalised sums
    double pm2 = 0.0, pnsum = 0.0, cm2[NCH], cnsum[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) { cm2[c] = 0.0; cnsum[c] = 0.0; }
    if (need2) {
        for (LatticeCursor cur(L, first, stride); cur.kz < L.cnt[2]; cur.advance()) {
            const int p = (cur.kz * L.cnt[1] + cur.ky) * L.cnt[0] + cur.kx;
            int x, y, z;
            cur.coord(L, x, y, z);
            if (!in_box(box, x, y, z)) continue;
            const double v = src[p];
            const double vn = pmax > 0.0 ? v / scale : v;
            pm2 += (v - pmean) * (v - pmean);
            pnsum += vn;
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (in_box(sbx[c], x, y, z)) { cm2[c] += (v - cmean[c]) * (v - cmean[c]); cnsum[c] += vn; }
        }
        pm2 = wave_sum(pm2);
        pnsum = wave_sum(pnsum);
#pragma unroll
        for (int c = 0; c < NCH; ++c) { cm2[c] = wave_sum(cm2[c]); cnsum[c] = wave_sum(cnsum[c]); }
        if constexpr (WAVES > 1) {
            double w[2 * NCH + 2];
#pragma unroll
            for (int c = 0; c < NCH; ++c) { w[c] = cm2[c]; w[NCH + c] = cnsum[c]; }
            w[2 * NCH] = pm2;
            w[2 * NCH + 1] = pnsum;
            combine_waves<WAVES>(w, 2 * NCH + 2, 2 * NCH + 2, red);
#pragma unroll
            for (int c = 0; c < NCH; ++c) { cm2[c] = w[c]; cnsum[c] = w[NCH + c]; }
            pm2 = w[2 * NCH];
            pnsum = w[2 * NCH + 1];
        }
    }
    const double pnmean = need2 ? pnsum / pn : 0.0;
    double cnmean[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) cnmean[c] = need2 ? cnsum[c] / cn[c] : 0.0;
    // pass 3: normalised squared deviations (Eq. 5 variances)
    double pv = 0.0, cv[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) cv[c] = 0.0;
    if (need3) {
        for (LatticeCursor cur(L, first, stride); cur.kz < L.cnt[2]; cur.advance()) {
            const int p = (cur.kz * L.cnt[1] + cur.ky) * L.cnt[0] + cur.kx;
            int x, y, z;
            cur.coord(L, x, y, z);
            if (!in_box(box, x, y, z)) continue;
            const double vn = pmax > 0.0 ? src[p] / scale : src[p];
            pv += (vn - pnmean) * (vn - pnmean);
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (in_box(sbx[c], x, y, z)) cv[c] += (vn - cnmean[c]) * (vn - cnmean[c]);
        }
        pv = wave_sum(pv);
#pragma unroll
        for (int c = 0; c < NCH; ++c) cv[c] = wave_sum(cv[c]);
        if constexpr (WAVES > 1) {
            double w[NCH + 1];
#pragma unroll
            for (int c = 0; c < NCH; ++c) w[c] = cv[c];
            w[NCH] = pv;
            combine_waves<WAVES>(w, NCH + 1, NCH + 1, red);
#pragma unroll
            for (int c = 0; c < NCH; ++c) cv[c] = w[c];
            pv = w[NCH];
        }
    }
    LevelStats out;
    out.pn = pn;
    out.pmean = pmean;
    out.pm2 = pm2;
    const double pnvar = need3 ? pv / pn : 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        out.count[c] = cn[c];
        sc8[c] = metric_value(a.metric, cn[c], cmean[c], cm2[c], cmx[c], cnmean[c], need3 ? cv[c] / cn[c] : 0.0,
                              pnvar);
    }
    return out;
}


// One level of the per-level walk for one scan, on one whole wavefront: the level's
// statistics over its lattice values (src), the W/B test of Eqs. (6)-(7), and the choice
// of the child (the first of the children within the tie band of the best score),
// carrying the previous level's figures in st.  box holds the level's box and receives
// the chosen child's.  Every lane computes the same state; lane 0 writes the result
// record (child, scores, W/B, next box), which nothing in the walk reads back.
// With WAVES = 4 the whole workgroup takes the statistics (red: LDS for their combine) and
// thread 0 writes the record.
template <int NACT, int WAVES = 1>
__device__ void pl_level_core(const WalkArgs &a, int lev, int scan, PLState &st, const double *src, int (&box)[6],
                              double *red = nullptr) {
    constexpr int NCH = 1 << NACT;
    uwb_segment_result &R = a.out[scan];
    const bool writer = WAVES > 1 ? threadIdx.x == 0 : (threadIdx.x & 63) == 0;
    const int side = a.g.dims[0] >> lev;
    const int step = side / a.coarse;
    Lattice L;
    for (int d = 0; d < 3; ++d) {
        L.x0[d] = d < NACT ? box[2 * d] + step / 2 : 0;
        L.cnt[d] = d < NACT ? a.coarse : 1;
    }
    L.step = step;
    const int P = L.count();
    int cbox[8][6];
    double sc8[8];
    const LevelStats ls = wave_level_stats<NACT, WAVES>(a, L, src, box, side, false, cbox, sc8, red);
    st.nvox += P;
    bool stop = false;
    if (a.term == UWB_TERM_WB && lev >= 1) {
        const double pooled = (st.prev_n * st.prev_mean + ls.pn * ls.pmean) / (st.prev_n + ls.pn);
        const double W = st.prev_m2 + ls.pm2;
        const double B = st.prev_n * (st.prev_mean - pooled) * (st.prev_mean - pooled) +
                         ls.pn * (ls.pmean - pooled) * (ls.pmean - pooled);
        if (writer) {
            R.wb[st.n_wb][0] = W;
            R.wb[st.n_wb][1] = B;
        }
        ++st.n_wb;
        if (lev >= 2 && (B <= st.prev_b || W >= st.prev_w)) { st.n_kept = lev - 1; stop = true; }
        st.prev_w = W;
        st.prev_b = B;
    }
    if (!stop) {
        st.prev_n = ls.pn;
        st.prev_mean = ls.pmean;
        st.prev_m2 = ls.pm2;
        if (lev == a.depth) {
            st.n_kept = a.depth;
            stop = true;
        } else {
            double best = -INFINITY;
#pragma unroll
            for (int c = 0; c < NCH; ++c) best = fmax(best, sc8[c]);
            const double thr = best - kTieRel * fabs(best);
            int sel = 0;
#pragma unroll
            for (int c = NCH - 1; c >= 0; --c)
                if (sc8[c] >= thr) sel = c;
            // the chosen child's box formed again rather than read from cbox[sel]: a runtime index into the
            // child arrays would place them in scratch memory
            int nb[6];
            split_box(box, sel, NACT, nb);
            if (writer) {
                R.child[st.made] = sel;
#pragma unroll
                for (int c = 0; c < 8; ++c) R.score[st.made][c] = c < NCH ? sc8[c] : 0.0;
                for (int i = 0; i < 6; ++i) R.box[lev + 1][i] = nb[i];
            }
            ++st.made;
            for (int i = 0; i < 6; ++i) box[i] = nb[i];
        }
    }
    if (stop) st.active = 0;
}

// The same level with the state, the box and the lattice values in global memory (the
// level-synchronous walk: one wavefront per scan, after the level's lattice kernel).
template <int NACT>
__device__ void pl_level_step(const WalkArgs &a, int lev, int scan) {
    PLState st = a.state[scan];
    if (!st.active) return;                    // uniform per wavefront; no workgroup barriers below
    int box[6];
    for (int i = 0; i < 6; ++i) box[i] = a.out[scan].box[lev][i];
    const int P = NACT == 3 ? a.coarse * a.coarse * a.coarse : a.coarse * a.coarse;
    const double *src = a.lat64 + (int64_t)scan * a.lat_stride + (int64_t)lev * P;
    pl_level_core<NACT>(a, lev, scan, st, src, box);
    if ((threadIdx.x & 63) == 0) a.state[scan] = st;
}

// Initial state of a scan's per-level walk: level 0's box is the whole grid.
__device__ inline void pl_init_state(const WalkArgs &a, PLState &S) {
    S.prev_n = S.prev_mean = S.prev_m2 = S.prev_w = S.prev_b = 0.0;
    S.nvox = 0;
    S.active = 1;
    S.n_kept = a.depth;
    S.made = 0;
    S.n_wb = 0;
}

// A finished per-level walk's record: the ROI (the last kept box widened by the final
// frame), the counts, and the detection fields cleared for the ROI phase.
__device__ inline void pl_finish_record(const WalkArgs &a, const PLState &st, uwb_segment_result &R) {
    const int nact = a.g.dims[2] > 1 ? 3 : 2;
    const int dims[3] = {a.g.dims[0], a.g.dims[1], a.g.dims[2]};
    int roi[6];
    expand_box(R.box[st.n_kept], a.frame_final, nact, dims, roi);
    R.n_levels = st.n_kept;
    R.term_level = st.made;
    R.decimation = 0;
    R.n_samples_level0 = (int)(nact == 3 ? a.coarse * a.coarse * a.coarse : a.coarse * a.coarse);
    R.n_wb = st.n_wb;
    for (int i = 0; i < 6; ++i) R.roi[i] = roi[i];
    const int64_t rv = (int64_t)(roi[1] - roi[0]) * (roi[3] - roi[2]) * (roi[5] - roi[4]);
    R.voxels_evaluated = st.nvox + rv;
    R.argmax = -1;
    R.peak = 0.0;
    R.learned_mask = 0;
    R.guard_hits = 0;
}

}  // namespace uwb
