// Final-imaging phase of the walks (Section III): the full-resolution image of
// every scan's region of interest and its maximal-energy voxel (the detection).
//
// k_roi32   images the ROI (box read from the scan's result) with the tile body of
//           the full-resolution FP32 kernel (one voxel per lane: tiles, or bands of
//           256 consecutive voxels for a ragged ROI), the ROI as a grid of its own -> roi32
// k_roi_pick one workgroup per scan: decides the detection in FP64, as for the
//           full image -- every ROI voxel whose FP32 energy is within kCandRel of
//           the ROI's FP32 maximum is re-evaluated in FP64 (a whole wave per voxel,
//           channels over the lanes, four voxels at a time), and the winner is the
//           lowest finest-grid index within the FP64 tie band kTieRel of the largest
//           of those values; it also copies the ROI image to the caller's buffer
//                                                            -> result, roi_img
// FP32 rounding moves an energy by about 1e-5 of the peak, far inside kCandRel, so
// the FP64 maximum is always among the candidates: the decision is the one a
// double-precision evaluation of the whole ROI would take.
#include <algorithm>
#include <climits>
#include <cmath>

#include "image32.h"
#include "walk_internal.h"

namespace uwb {
namespace {

constexpr int kRoiWaves = kBlock / 64;

struct RoiArgs {
    ScanSet ss;
    GridView g;                  // finest grid
    uwb_segment_result *res;     // [n_scans]: ROI box in, detection out
    float *roi32;                // [n_scans][roi_cap]
    int64_t roi_cap;
    float *roi_img;              // optional copy, scan s at s * roi_img_stride
    int64_t roi_img_stride;
    int lds_bytes;               // staging space of a workgroup
    int bf, window;
};

// Grid: x = scan, y = group of 256 voxels of the scan's own ROI -- a tile when the ROI
// is a whole number of tiles, else a band of consecutive voxels (x fastest), so that a
// ragged ROI idles only part of its last band (as 16 x 16 tiles, a 37 x 37 ROI idles
// 41 % of the lanes).  The groups with work -- every scan's first ones -- are dispatched
// before the ones past a scan's ROI, which only the largest possible ROI needs.  Each
// group's staging stride follows from its own bounding box.
template <int BF, int W, bool D3, bool MS>
__global__ __launch_bounds__(kBlock) void k_roi32(const RoiArgs a) {
    extern __shared__ float smem[];
    const int scan = blockIdx.x;
    const int *roi = a.res[scan].roi;
    TileJob j;
    for (int d = 0; d < 3; ++d) {   // the ROI as a grid of its own
        j.g.dims[d] = roi[2 * d + 1] - roi[2 * d];
        j.g.pitch[d] = a.g.pitch[d];
        j.g.origin[d] = a.g.origin[d] + roi[2 * d] * a.g.pitch[d];
    }
    const int64_t n = (int64_t)j.g.dims[0] * j.g.dims[1] * j.g.dims[2];
    // a ROI larger than its slot (never, for a planned walk) is not imaged
    if (n > a.roi_cap) return;
    // tiles of 16 x 16 (2D) or 8 x 8 x 4 when the ROI is a whole number of them (compact spans),
    // else bands: either way kBlock voxels per workgroup, as many groups
    int tx, ty, tz;
    TileShape<D3, 1>::get(tx, ty, tz);
    const bool tiled = j.g.dims[0] % tx == 0 && j.g.dims[1] % ty == 0 && j.g.dims[2] % tz == 0;
    const int64_t ngroups = (n + kBlock - 1) / kBlock;
    if ((int64_t)blockIdx.y >= ngroups) return;   // uniform per workgroup
    const ScanConst sc = scan_const(a.ss, scan);
    j.pos = sc.pos;
    j.tr = sc.tr;
    j.img = a.roi32 + (int64_t)scan * a.roi_cap;
    j.M = a.ss.n_ant;
    j.T = a.ss.n_samp;
    j.s = sc.s;
    j.t0s = sc.t0s;
    j.ms = a.ss.ms;
    const int ntx = j.g.dims[0] / tx, nty = j.g.dims[1] / ty;
    // (more groups than the grid's 65535 rows: the rows stride over them)
    for (int64_t b = blockIdx.y; b < ngroups; b += gridDim.y) {
        int x0, x1, y0, y1, z0, z1;
        if (tiled) {
            j.tx0 = x0 = (int)(b % ntx) * tx;
            j.ty0 = y0 = (int)((b / ntx) % nty) * ty;
            j.tz0 = z0 = (int)(b / ((int64_t)ntx * nty)) * tz;
            x1 = x0 + tx - 1; y1 = y0 + ty - 1; z1 = z0 + tz - 1;
        } else {
            j.tx0 = j.ty0 = j.tz0 = 0;
            j.p0 = b * kBlock;
            band_box(j.p0, min(j.p0 + kBlock, n) - 1, j.g.dims[0], j.g.dims[1], x0, x1, y0, y1, z0, z1);
        }
        // staging stride and channels per pass for this group (uniform: kept in scalar registers)
        j.rs = __builtin_amdgcn_readfirstlane(staged_samples(sc.s, (x1 - x0) * a.g.pitch[0], (y1 - y0) * a.g.pitch[1],
                                                             (z1 - z0) * a.g.pitch[2], W, a.ss.n_samp));
        j.chunk = __builtin_amdgcn_readfirstlane(min(a.lds_bytes / (j.rs * 16 + (MS ? 32 : 16)), min(j.M, kBlock)));
        if (j.chunk < 1) continue;   // never: the host sizes the LDS for the widest group
        if (tiled) image_tile<BF, W, D3, 1, MS, false>(j, smem);
        else image_tile<BF, W, D3, 1, MS, true>(j, smem);
    }
}

__device__ __forceinline__ void roi_pos(const RoiArgs &a, const int *roi, int rnx, int rny, int64_t p, double &rx,
                                        double &ry, double &rz) {
    const int64_t kx = p % rnx, ky = (p / rnx) % rny, kz = p / ((int64_t)rnx * rny);
    rx = a.g.origin[0] + (double)(roi[0] + kx) * a.g.pitch[0];
    ry = a.g.origin[1] + (double)(roi[2] + ky) * a.g.pitch[1];
    rz = a.g.origin[2] + (double)(roi[4] + kz) * a.g.pitch[2];
}

// The winner among a ROI's FP32 candidates, on one wavefront: candidates evaluated in
// index order, lane l remembering the l-th, so the tie band needs no second evaluation
// unless there are more than 64.  Every lane returns the same (index, value).
template <bool MV>
__device__ void pick_serial(const RoiArgs &a, const ScanConst &sc, const int *roi, int rnx, int rny, int64_t n,
                            const float *v, float thr32, int lane, long long &b, double &pv) {
    const int M = a.ss.n_ant, T = a.ss.n_samp;
    double best = -INFINITY;
    int count = 0;
    int64_t my_idx = 0;
    double my_val = 0.0;
    for (int64_t p0 = 0; p0 < n; p0 += 64) {
        const int64_t p = p0 + lane;
        unsigned long long mask = __ballot(p < n && v[p] >= thr32);
        while (mask) {
            const int l = __builtin_ctzll(mask);
            mask &= mask - 1;
            const int64_t pp = p0 + l;
            double rx, ry, rz;
            roi_pos(a, roi, rnx, rny, pp, rx, ry, rz);
            const double e = energy64_bf<MV>(a.bf, sc, M, T, a.window, rx, ry, rz, lane, 64);   // on every lane
            best = fmax(best, e);
            if (lane == count) { my_idx = pp; my_val = e; }
            ++count;
        }
    }
    const double thr64 = best - kTieRel * fabs(best);
    b = LLONG_MAX;
    pv = __builtin_nan("");
    if (count <= 64) {
        long long mine = lane < count && my_val >= thr64 ? my_idx : LLONG_MAX;
        b = wave_min_ll(mine);
        const unsigned long long owner = __ballot(mine == b && b != LLONG_MAX);
        if (owner) pv = __shfl(my_val, __builtin_ctzll(owner), 64);
    } else {   // more candidates than lanes: evaluate them again, the first in the band wins
        for (int64_t p0 = 0; p0 < n && b == LLONG_MAX; p0 += 64) {
            const int64_t p = p0 + lane;
            unsigned long long mask = __ballot(p < n && v[p] >= thr32);
            while (mask) {
                const int l = __builtin_ctzll(mask);
                mask &= mask - 1;
                const int64_t pp = p0 + l;
                double rx, ry, rz;
                roi_pos(a, roi, rnx, rny, pp, rx, ry, rz);
                const double e = energy64_bf<MV>(a.bf, sc, M, T, a.window, rx, ry, rz, lane, 64);
                if (e >= thr64) { b = pp; pv = e; break; }
            }
        }
    }
}

constexpr int kPickCap = 512;   // candidates listed in LDS per scan

// One workgroup per scan.  The FP32 maximum over all 256 lanes; the candidates listed in
// index order in LDS; the four wavefronts evaluate them in parallel (each candidate on a
// whole wavefront, channels over the lanes, so a candidate's FP64 value does not depend
// on which wavefront takes it); the winner is the lowest listed candidate within the tie
// band.  More candidates than the list holds (a flat image) go to the serial pick.
template <bool MV>
__global__ __launch_bounds__(kBlock) void k_roi_pick(const RoiArgs a) {
    __shared__ int cand[kPickCap];
    __shared__ double cval[kPickCap];
    __shared__ float redf[kRoiWaves];
    __shared__ double redd[kRoiWaves];
    __shared__ long long redl[kRoiWaves];
    __shared__ int redi[kRoiWaves];
    const int scan = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uwb_segment_result &R = a.res[scan];
    const int *roi = R.roi;
    const int rnx = roi[1] - roi[0], rny = roi[3] - roi[2], rnz = roi[5] - roi[4];
    const int64_t n = min((int64_t)rnx * rny * rnz, a.roi_cap);
    const float *v = a.roi32 + (int64_t)scan * a.roi_cap;
    float *copy = a.roi_img ? a.roi_img + (int64_t)scan * a.roi_img_stride : nullptr;

    // FP32 maximum (and the caller's copy of the image)
    float m = -INFINITY;
    for (int64_t p = tid; p < n; p += kBlock) {
        const float x = v[p];
        m = fmaxf(m, x);
        if (copy) copy[p] = x;
    }
    m = wave_maxf(m);
    if (lane == 0) redf[wave] = m;
    __syncthreads();
    m = fmaxf(fmaxf(redf[0], redf[1]), fmaxf(redf[2], redf[3]));
    const float thr32 = m - (float)kCandRel * fabsf(m);

    // candidates (FP32 energy within kCandRel of the maximum) in index order
    int count = 0;   // uniform
    for (int64_t p0 = 0; p0 < n; p0 += kBlock) {
        const int64_t p = p0 + tid;
        const bool c = p < n && v[p] >= thr32;
        const unsigned long long mask = __ballot(c);
        if (lane == 0) redi[wave] = __popcll(mask);
        __syncthreads();
        int slot = count + __popcll(mask & ((1ull << lane) - 1));
        for (int w = 0; w < wave; ++w) slot += redi[w];
        if (c && slot < kPickCap) cand[slot] = (int)p;
        count += redi[0] + redi[1] + redi[2] + redi[3];
        __syncthreads();   // redi read by every lane before the next round writes it
    }

    const ScanConst sc = scan_const(a.ss, scan);
    long long b = LLONG_MAX;
    double pv = __builtin_nan("");
    if (count > kPickCap || n > INT_MAX) {   // uniform over the workgroup
        if (wave == 0) pick_serial<MV>(a, sc, roi, rnx, rny, n, v, thr32, lane, b, pv);
    } else {
        for (int c = wave; c < count; c += kRoiWaves) {   // uniform per wavefront
            double rx, ry, rz;
            roi_pos(a, roi, rnx, rny, cand[c], rx, ry, rz);
            const double e = energy64_bf<MV>(a.bf, sc, a.ss.n_ant, a.ss.n_samp, a.window, rx, ry, rz, lane, 64);
            if (lane == 0) cval[c] = e;
        }
        __syncthreads();
        double best = -INFINITY;
        for (int c = tid; c < count; c += kBlock) best = fmax(best, cval[c]);
        best = wave_max(best);
        if (lane == 0) redd[wave] = best;
        __syncthreads();
        best = fmax(fmax(redd[0], redd[1]), fmax(redd[2], redd[3]));
        const double thr64 = best - kTieRel * fabs(best);
        long long first = LLONG_MAX;   // each lane's lowest list position in the band
        for (int c = tid; c < count; c += kBlock)
            if (cval[c] >= thr64) { first = c; break; }
        first = wave_min_ll(first);
        if (lane == 0) redl[wave] = first;
        __syncthreads();
        first = min(min(redl[0], redl[1]), min(redl[2], redl[3]));
        if (first != LLONG_MAX) { b = cand[first]; pv = cval[first]; }
    }
    if (tid != 0) return;
    R.guard_hits = count;   // FP32 candidates re-evaluated in FP64
    if (b == LLONG_MAX) {   // no finite candidate (e.g. a NaN image)
        R.argmax = -1;
        R.peak = __builtin_nan("");
        return;
    }
    const int64_t kx = b % rnx, ky = (b / rnx) % rny, kz = b / ((int64_t)rnx * rny);
    R.argmax = (roi[0] + kx) + (int64_t)a.g.dims[0] * ((roi[2] + ky) + (int64_t)a.g.dims[1] * (roi[4] + kz));
    R.peak = pv;
}

template <int BF, int W>
void launch_w(bool d3, dim3 grid, size_t lds, hipStream_t st, const RoiArgs &a) {
    if (a.ss.ms) {
        if (d3) hipLaunchKernelGGL((k_roi32<BF, W, true, true>), grid, dim3(kBlock), lds, st, a);
        else hipLaunchKernelGGL((k_roi32<BF, W, false, true>), grid, dim3(kBlock), lds, st, a);
    } else {
        if (d3) hipLaunchKernelGGL((k_roi32<BF, W, true, false>), grid, dim3(kBlock), lds, st, a);
        else hipLaunchKernelGGL((k_roi32<BF, W, false, false>), grid, dim3(kBlock), lds, st, a);
    }
}

template <int BF>
bool launch_bf(int window, bool d3, dim3 grid, size_t lds, hipStream_t st, const RoiArgs &a) {
    switch (window) {
#define UWB_W(w) case w: launch_w<BF, w>(d3, grid, lds, st, a); return true;
        UWB_WINDOWS(UWB_W)
#undef UWB_W
    }
    return false;
}

template <>
bool launch_bf<UWB_MVDR>(int window, bool d3, dim3 grid, size_t lds, hipStream_t st, const RoiArgs &a) {
    switch (window) {
#define UWB_W(w) case w: launch_w<UWB_MVDR, w>(d3, grid, lds, st, a); return true;
        UWB_MVDR_WINDOWS(UWB_W)
#undef UWB_W
    }
    return false;
}

}  // namespace

int launch_roi(const WalkArgs &w, int bf, int n_scans, hipStream_t st) {
    if (n_scans < 1) return UWB_OK;
    const bool d3 = w.g.dims[2] > 1;
    RoiArgs a;
    a.ss = w.ss;
    a.g = w.g;
    a.res = w.out;
    a.roi32 = w.roi32;
    a.roi_cap = w.roi_cap;
    a.roi_img = w.roi_img;
    a.roi_img_stride = w.roi_img_stride;
    a.bf = bf;
    a.window = w.window;
    const int64_t bands = (w.roi_cap + kBlock - 1) / kBlock;   // of the largest ROI
    if (bands < 1) return UWB_EUNSUPPORTED;
    // LDS: every channel at the widest span a band can have (the whole largest ROI), within
    // the budget; the kernel sizes each band's own stride and chunk to it
    const double s_max = 2.0 / (w.ss.v * w.ss.dt);
    const int rs_max = staged_samples(s_max, (w.roi_side[0] - 1) * w.g.pitch[0], (w.roi_side[1] - 1) * w.g.pitch[1],
                                      (w.roi_side[2] - 1) * w.g.pitch[2], w.window, w.ss.n_samp);
    const int per_ch = rs_max * 16 + (w.ss.ms ? 32 : 16);   // staged records of 4 samples + table entries
    if (per_ch > kLdsBudget) return UWB_EUNSUPPORTED;
    a.lds_bytes = (int)std::min<int64_t>((int64_t)per_ch * std::min(w.ss.n_ant, kBlock), kLdsBudget);
    const size_t lds = (size_t)a.lds_bytes;
    const dim3 grid((unsigned)n_scans, (unsigned)(bands < 65535 ? bands : 65535));
    const bool ok = bf == UWB_DMAS   ? launch_bf<UWB_DMAS>(w.window, d3, grid, lds, st, a)
                    : bf == UWB_MVDR ? launch_bf<UWB_MVDR>(w.window, d3, grid, lds, st, a)
                                     : launch_bf<UWB_DAS>(w.window, d3, grid, lds, st, a);
    if (!ok) return UWB_EINVAL;
    if (hipGetLastError() != hipSuccess) return UWB_EHIP;
    if (bf == UWB_MVDR) hipLaunchKernelGGL(k_roi_pick<true>, dim3((unsigned)n_scans), dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL(k_roi_pick<false>, dim3((unsigned)n_scans), dim3(kBlock), 0, st, a);
    return hipGetLastError() == hipSuccess ? UWB_OK : UWB_EHIP;
}

}  // namespace uwb
