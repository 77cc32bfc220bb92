// FP64 energies on regular lattices of focal points, for the segment walk:
// the g^d lattice of every scan's current box (per-level walk), the decimated
// lattice of the whole grid (paper walk) and the full-resolution ROI.
//
// The kernel mirrors the FP32 imaging kernel's structure in double precision.
// A workgroup evaluates 256 lattice points of one scan at a time, one point per
// lane: a tile of 16 x 16 (2D) or 8 x 8 x 4 (3D) points when the scan's lattice
// is a whole number of such tiles, else a band of 256 consecutive points in
// lattice order, so that a ragged lattice (a ROI) idles at most part of its last
// band instead of the edges of every tile row.  For a chunk of channels it
// derives (in FP64) the interval of samples any of its points can reach, stages
// those intervals from HBM into LDS, and then every lane computes its delay for
// each channel once (Eq. (1), or Eq. (2) for a bistatic channel, whose
// transmitter distance is kept while consecutive channels share the
// transmitter), reads the W+1 staged samples around it and accumulates the
// linearly interpolated window into W FP64 accumulators (Eq. (3) DAS, or the
// prefix form P_k += s_k S_k, S_k += s_k of the Section II-B pairwise DMAS sum, or
// for the Capon / MVDR beamformer the window sums and their W x W Gram matrix,
// solved per point).
// Positions are formed exactly as the rest of the walk forms them (origin +
// index * pitch on the finest grid), channels are taken in order, and every
// point's energy is written once: the values depend neither on the tiling nor on
// the staging.
#include <algorithm>
#include <atomic>
#include <cmath>

#include "image32.h"
#include "walk_internal.h"
#include "walk_level.h"

namespace uwb {
namespace {

constexpr int kTabBytes = 64;          // per staged channel: transmitter and receiver positions, first staged sample
constexpr int kLdsPerCu = 160 * 1024;  // LDS of one CU
constexpr int kGridLdsMax = 64 * 1024; // staging budget of one workgroup, at most

template <bool D3> struct Tile64 {
    static constexpr int X = D3 ? 8 : 16, Y = D3 ? 8 : 16, Z = D3 ? 4 : 1;
};

struct Lat {
    int x0[3], step, cnt[3];
};

// Square root of a squared distance (finite, >= 0): the hardware reciprocal square root
// refined by one step of Goldschmidt's coupled iteration for sqrt(x) and 1/(2 sqrt(x)),
// then two Newton corrections of the residual x - g^2 -- the steps of the compiler's
// general double-precision expansion, whose result it equals for x >= 2^-767, without
// that expansion's rescaling of tiny inputs and its zero and infinity cases (7 of its 18
// instructions).  x is raised to 1e-300 first, so a point on an antenna is 1e-150 m from it.
__device__ __forceinline__ double sqrt_dist(double x) {
    x = fmax(x, 1e-300);
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    return fma(d, h, g);
}

// One group of up to 256 points of the lattice L: lane point k (lattice indices,
// valid or not), the group's bounding box lo..hi (lattice indices) and the
// output offset of the lane's point.
struct Group {
    int k[3], lo[3], hi[3];
    int64_t p;
    bool valid;
};

template <int BF, int W, bool MS>
__device__ void grid64_group(const Grid64Args &a, const Lat &L, int scan, const ScanConst &sc, const Group &G,
                             unsigned char *dsm, int64_t out_offset, double *lat_lds);

// Group t of a c0 x c1 x c2 lattice as lane tid sees it: a tile when the lattice is a whole
// number of tiles (tiled), else the band of points t * 256 .. in lattice order.
template <bool D3>
__device__ __forceinline__ Group make_group(int c0, int c1, int c2, bool tiled, int64_t t, int tid) {
    using TS = Tile64<D3>;
    const int64_t n = (int64_t)c0 * c1 * c2;
    Group G;
    if (tiled) {
        const int ntx = c0 / TS::X, nty = c1 / TS::Y;
        G.lo[0] = (int)(t % ntx) * TS::X;
        G.lo[1] = (int)((t / ntx) % nty) * TS::Y;
        G.lo[2] = (int)(t / ((int64_t)ntx * nty)) * TS::Z;
        G.hi[0] = G.lo[0] + TS::X - 1;
        G.hi[1] = G.lo[1] + TS::Y - 1;
        G.hi[2] = G.lo[2] + TS::Z - 1;
        if (!D3) { G.k[0] = G.lo[0] + (tid & 15); G.k[1] = G.lo[1] + (tid >> 4); G.k[2] = 0; }
        else { G.k[0] = G.lo[0] + (tid & 7); G.k[1] = G.lo[1] + ((tid >> 3) & 7); G.k[2] = G.lo[2] + (tid >> 6); }
        G.valid = true;
        G.p = ((int64_t)G.k[2] * c1 + G.k[1]) * c0 + G.k[0];
    } else {
        const int64_t p0 = t * kBlock, p1 = min(p0 + kBlock, n) - 1;
        G.valid = p0 + tid <= p1;
        G.p = min(p0 + tid, p1);
        const int64_t s01 = (int64_t)c0 * c1;
        G.k[0] = (int)(G.p % c0); G.k[1] = (int)((G.p / c0) % c1); G.k[2] = (int)(G.p / s01);
        const int ax = (int)(p0 % c0), ay = (int)((p0 / c0) % c1), az = (int)(p0 / s01);
        const int bx = (int)(p1 % c0), by = (int)((p1 / c0) % c1), bz = (int)(p1 / s01);
        // a band within one row spans its own columns; across rows, whole rows; across slabs, whole slabs
        G.lo[2] = az; G.hi[2] = bz;
        G.lo[1] = az == bz ? ay : 0; G.hi[1] = az == bz ? by : c1 - 1;
        G.lo[0] = (az == bz && ay == by) ? ax : 0; G.hi[0] = (az == bz && ay == by) ? bx : c0 - 1;
    }
    return G;
}

// MS: the scans' channels are the transmitter-receiver pairs of a multistatic array.
// DAS with windows up to 13 samples fits five waves per SIMD without spilling: asked of
// the register allocator, which otherwise settles one wave lower.
template <int BF, int W, bool D3, bool MS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(BF == UWB_DAS && W <= 13 ? 5 : 1)))
void k_grid64(const Grid64Args a) {
    using TS = Tile64<D3>;
    extern __shared__ __align__(16) unsigned char dsm[];
    const int scan = blockIdx.y;
    const int tid = threadIdx.x;

    // this scan's lattice
    Lat L;
    if (a.mode == kGridBox) {
        if (a.state && !a.state[scan].active) return;
        const int *box = a.res[scan].box[a.lev];
        for (int d = 0; d < 3; ++d) {
            const bool act = d < 2 || D3;
            L.x0[d] = act ? box[2 * d] + a.step / 2 : 0;
            L.cnt[d] = act ? a.coarse : 1;
        }
        L.step = a.step;
    } else if (a.mode == kGridRoi) {
        const int *roi = a.res[scan].roi;
        for (int d = 0; d < 3; ++d) {
            L.x0[d] = roi[2 * d];
            L.cnt[d] = roi[2 * d + 1] - roi[2 * d];
        }
        L.step = 1;
    } else {
        for (int d = 0; d < 3; ++d) { L.x0[d] = a.x0[d]; L.cnt[d] = a.cnt[d]; }
        L.step = a.step;
    }
    const int c0 = L.cnt[0], c1 = L.cnt[1], c2 = L.cnt[2];
    const int64_t n = (int64_t)c0 * c1 * c2;
    // a lattice larger than its output slot (never, for a planned walk) is not written
    if (n < 1 || n + a.out_offset > a.out_stride) return;
    const bool tiled = c0 % TS::X == 0 && c1 % TS::Y == 0 && c2 % TS::Z == 0;
    const int64_t ngroups = (n + kBlock - 1) / kBlock;   // tiles or bands: the same count when tiled
    const int64_t t = blockIdx.x;   // the launch holds enough workgroups for the largest lattice
    if (t >= ngroups) return;       // uniform per workgroup
    const Group G = make_group<D3>(c0, c1, c2, tiled, t, tid);
    grid64_group<BF, W, MS>(a, L, scan, scan_const(a.ss, scan), G, dsm, a.out_offset, nullptr);
}

// The per-level walk in one launch, one workgroup per scan: the workgroup sets up the
// walk, then at every level images the coarse^d lattice of the scan's box (as k_grid64
// does, the energies also kept in LDS), and its first wavefront takes the level's
// statistics and decision; finally it writes the walk's record for the ROI phase.  The
// walk's state stays in the first wavefront's registers and the box and the lattice in
// LDS (barriers publish them), so a level reads nothing back from global memory.  Values
// and decisions are those of the level-synchronous kernels.
template <int BF, int W, bool D3, bool MS>
__global__ __launch_bounds__(kBlock) void k_pl_fused(const Grid64Args a, const WalkArgs w, int levels) {
    using TS = Tile64<D3>;
    extern __shared__ __align__(16) unsigned char dsm[];
    __shared__ double lat[kBlock];   // this level's lattice energies (at most kBlock points)
    __shared__ int sbox[6], sactive;
    const int scan = blockIdx.x;
    const int c0 = w.coarse, c1 = w.coarse, c2 = D3 ? w.coarse : 1;
    const int64_t n = (int64_t)c0 * c1 * c2;
    const bool tiled = c0 % TS::X == 0 && c1 % TS::Y == 0 && c2 % TS::Z == 0;
    const ScanConst sc = scan_const(a.ss, scan);
    uwb_segment_result &R = w.out[scan];
    PLState st;                                                          // first wavefront
    int box[6] = {0, w.g.dims[0], 0, w.g.dims[1], 0, w.g.dims[2]};      // first wavefront
    if (threadIdx.x < 64) pl_init_state(w, st);
    if (threadIdx.x < 6) sbox[threadIdx.x] = box[threadIdx.x];
    if (threadIdx.x == 0) {   // every record field the finishing step reads back is written by this thread
        for (int i = 0; i < 6; ++i) R.box[0][i] = box[i];
        sactive = 1;
    }
    __syncthreads();
    for (int lev = 0; lev < levels; ++lev) {
        if (!sactive) break;   // uniform: published by the barrier closing the previous level
        const int step = (w.g.dims[0] >> lev) / w.coarse;
        Lat L;
        for (int d = 0; d < 3; ++d) {
            const bool act = d < 2 || D3;
            L.x0[d] = act ? sbox[2 * d] + step / 2 : 0;
            L.cnt[d] = act ? w.coarse : 1;
        }
        L.step = step;
        const int64_t off = (int64_t)lev * n;
        if (n <= kBlock && n + off <= a.out_stride)   // always, for a planned walk
            grid64_group<BF, W, MS>(a, L, scan, sc, make_group<D3>(c0, c1, c2, tiled, 0, threadIdx.x), dsm, off, lat);
        __syncthreads();
        if (threadIdx.x < 64) {
            pl_level_core<D3 ? 3 : 2>(w, lev, scan, st, lat, box);
            if (threadIdx.x < 6) sbox[threadIdx.x] = box[threadIdx.x];
            if (threadIdx.x == 0) sactive = st.active;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        w.state[scan] = st;
        pl_finish_record(w, st, R);
    }
}

// Window taps K0 .. K1-1 of one channel at one point: the linearly interpolated samples
// (window starting at p, fraction f) into the DAS sums S_k and the DMAS prefix sums P_k.
// The lattice arithmetic is written as explicit fused operations, so that the kernels
// that instantiate it (k_grid64, k_pl_fused) take the same roundings and give the same
// values bit for bit, whatever the compiler would contract in each context.
template <int BF, int W, int K0, int K1>
__device__ __forceinline__ void taps64(const float *p, double f, double (&S)[W], double (&P)[BF == UWB_DMAS ? W : 1]) {
    float y[K1 - K0 + 1];
#pragma unroll
    for (int k = K0; k <= K1; ++k) y[k - K0] = p[k];
    const double g = 1.0 - f;
#pragma unroll
    for (int k = K0; k < K1; ++k) {
        const double s = fma(f, (double)y[k - K0 + 1], g * (double)y[k - K0]);
        if constexpr (BF == UWB_DMAS) P[k] = fma(s, S[k], P[k]);
        S[k] += s;
    }
}

// MVDR: the window sums and the Gram matrix (packed lower triangle) of the same samples.
template <int W>
__device__ __forceinline__ void taps64_mvdr(const float *p, double f, double (&S)[W], double (&gram)[W * (W + 1) / 2]) {
    float y[W + 1];
#pragma unroll
    for (int k = 0; k <= W; ++k) y[k] = p[k];
    const double g = 1.0 - f;
    double sv[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        sv[k] = fma(f, (double)y[k + 1], g * (double)y[k]);
        S[k] += sv[k];
    }
#pragma unroll
    for (int k = 0; k < W; ++k)
#pragma unroll
        for (int l = 0; l <= k; ++l) gram[tri(k, l)] = fma(sv[k], sv[l], gram[tri(k, l)]);
}

// lat_lds (optional): the energies written to LDS as well, at the points' lattice offsets.
template <int BF, int W, bool MS>
__device__ void grid64_group(const Grid64Args &a, const Lat &L, int scan, const ScanConst &sc, const Group &G,
                             unsigned char *dsm, int64_t out_offset, double *lat_lds) {
    constexpr int H = (W - 1) / 2;
    const int tid = threadIdx.x;
    const int M = a.ss.n_ant, T = a.ss.n_samp;
    double *tab = reinterpret_cast<double *>(dsm);   // [chunk][8]

    // lane point -> finest indices -> position
    const double rx = fma((double)(L.x0[0] + L.step * G.k[0]), a.g.pitch[0], a.g.origin[0]);
    const double ry = fma((double)(L.x0[1] + L.step * G.k[1]), a.g.pitch[1], a.g.origin[1]);
    const double rz = fma((double)(L.x0[2] + L.step * G.k[2]), a.g.pitch[2], a.g.origin[2]);

    // the group's bounding box (metres); its staging stride and the channels per chunk follow from it
    double blo[3], bhi[3];
    for (int d = 0; d < 3; ++d) {
        blo[d] = a.g.origin[d] + (L.x0[d] + L.step * G.lo[d]) * a.g.pitch[d];
        bhi[d] = a.g.origin[d] + (L.x0[d] + L.step * G.hi[d]) * a.g.pitch[d];
    }
    // (uniform, but computed on the vector unit: kept in scalar registers, so that the
    // channel loop's counters stay scalar)
    const int rs = __builtin_amdgcn_readfirstlane(
        staged_samples(sc.s, bhi[0] - blo[0], bhi[1] - blo[1], bhi[2] - blo[2], W, T));
    const int chunk = __builtin_amdgcn_readfirstlane(min(a.lds_bytes / (kTabBytes + 4 * rs), min(M, kBlock)));
    float *stage = reinterpret_cast<float *>(dsm + (size_t)kTabBytes * chunk);   // [chunk][rs]

    constexpr int NG = BF == UWB_MVDR ? W * (W + 1) / 2 : 1;
    double S[W], P[BF == UWB_DMAS ? W : 1], gram[NG];
#pragma unroll
    for (int k = 0; k < W; ++k) S[k] = 0.0;
#pragma unroll
    for (int k = 0; k < (BF == UWB_DMAS ? W : 1); ++k) P[k] = 0.0;
#pragma unroll
    for (int q = 0; q < NG; ++q) gram[q] = 0.0;

    double dtx = 0.0;   // bistatic: the current transmitter's distance
    for (int a0 = 0; chunk > 0 && a0 < M; a0 += chunk) {
        const int nch = min(chunk, M - a0);
        __syncthreads();   // previous chunk (or group) consumed
        if (tid < nch) {
            const int i = a0 + tid;
            // transmitter and receiver of the channel (the same antenna when monostatic)
            const float *at = sc.pos + 3 * (MS ? i / sc.ms : i), *ar = sc.pos + 3 * (MS ? i % sc.ms : i);
            double dmin = 0.0;
            for (int leg = 0; leg < 2; ++leg) {
                const float *ap = leg == 0 ? at : ar;
                const double ax = (double)ap[0], ay = (double)ap[1], az = (double)ap[2];
                // nearest point of the group's box to the antenna: earliest delay of the group
                const double nx = fmin(fmax(ax, blo[0]), bhi[0]) - ax;
                const double ny = fmin(fmax(ay, blo[1]), bhi[1]) - ay;
                const double nz = fmin(fmax(az, blo[2]), bhi[2]) - az;
                dmin += sqrt(nx * nx + ny * ny + nz * nz);
                tab[8 * tid + 3 * leg + 0] = ax;
                tab[8 * tid + 3 * leg + 1] = ay;
                tab[8 * tid + 3 * leg + 2] = az;
            }
            const double tmin = 0.5 * sc.s * dmin - sc.t0s;
            // first staged sample: one below the lowest window start, clamped so that a
            // window wholly outside the trace still reads a run of zeros
            double lo = floor(tmin) - (H + 1);
            lo = fmin(fmax(lo, -(double)(W + 1)), (double)(T + W + 1 - rs));
            tab[8 * tid + 6] = lo;
        }
        __syncthreads();
        stage_spans(stage, rs, nch, sc.tr + (int64_t)a0 * T, T, [&](int jj) { return (int)tab[8 * jj + 6]; });
        __syncthreads();
        // bistatic: receiver of the chunk's first channel (channels run in order, so a
        // transmitter's distance carries over a chunk boundary)
        int rxi = MS ? a0 % sc.ms : 0;
        for (int jj = 0; jj < nch; ++jj) {
            double tau;
            // (explicit fused operations, as in taps64)
            if (MS) {   // Eq. (2): both legs; the transmitter's leg is shared by its receivers
                if (rxi == 0) {   // a new transmitter (uniform over the workgroup)
                    const double dx = rx - tab[8 * jj + 0];
                    const double dy = ry - tab[8 * jj + 1];
                    const double dz = rz - tab[8 * jj + 2];
                    dtx = sqrt_dist(fma(dz, dz, fma(dy, dy, dx * dx)));
                }
                rxi = rxi + 1 == sc.ms ? 0 : rxi + 1;
                const double ux = rx - tab[8 * jj + 3];
                const double uy = ry - tab[8 * jj + 4];
                const double uz = rz - tab[8 * jj + 5];
                tau = fma(0.5 * sc.s, dtx + sqrt_dist(fma(uz, uz, fma(uy, uy, ux * ux))), -sc.t0s);
            } else {    // Eq. (1)
                const double dx = rx - tab[8 * jj + 0];
                const double dy = ry - tab[8 * jj + 1];
                const double dz = rz - tab[8 * jj + 2];
                tau = fma(sc.s, sqrt_dist(fma(dz, dz, fma(dy, dy, dx * dx))), -sc.t0s);
            }
            const double fl = floor(tau);
            const double f = tau - fl;
            // window samples n-H .. n+H+1 sit at stage offsets n-H-lo .. ; the clamp only
            // guards non-finite inputs (every span fits by construction)
            const double off = fmin(fmax(fl - H - tab[8 * jj + 6], 0.0), (double)(rs - (W + 1)));
            const float *p = stage + jj * rs + (int)off;
            if constexpr (BF == UWB_MVDR) taps64_mvdr<W>(p, f, S, gram);
            else taps64<BF, W, 0, W>(p, f, S, P);
        }
    }
    double e = 0.0;
    if constexpr (BF == UWB_MVDR) {
        e = mvdr_energy<double, W>(gram, S, M);
    } else {
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const double q = BF == UWB_DMAS ? P[k] : S[k];
            e = fma(q, q, e);
        }
    }
    if (chunk < 1) e = __builtin_nan("");   // a span longer than the staging space (rejected on the host)
    if (G.valid) {
        a.out64[(int64_t)scan * a.out_stride + out_offset + G.p] = e;
        if (lat_lds) lat_lds[G.p] = e;
        if (a.out32) a.out32[(int64_t)scan * a.out32_stride + G.p] = (float)e;
    }
}

// Staging budget per workgroup: the CU's LDS shared by as many workgroups as the
// kernel's registers let run at once (queried once per instantiation), less the kernel's
// own static LDS, at most kGridLdsMax in all.
int lds_budget(const void *kern, int block, std::atomic<int> &cache) {
    int b = cache.load(std::memory_order_relaxed);
    if (b > 0) return b;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, block, 0) != hipSuccess || nb < 1) nb = 5;
    hipFuncAttributes fa;
    const int stat = hipFuncGetAttributes(&fa, kern) == hipSuccess ? (int)fa.sharedSizeBytes : 4096;
    b = (std::min(kGridLdsMax, kLdsPerCu / nb) - stat) & ~255;
    cache.store(b, std::memory_order_relaxed);
    return b;
}

// w: null for k_grid64 (grid from the caller), else the walk of the fused per-level kernel
// (one workgroup per scan, levels levels).
template <int BF, int W, bool D3, bool MS>
int launch_k(dim3 grid, Grid64Args a, int rs_max, const WalkArgs *w, int levels, hipStream_t st) {
    static std::atomic<int> budget, budget_fused;
    const void *kern = w ? reinterpret_cast<const void *>(&k_pl_fused<BF, W, D3, MS>)
                         : reinterpret_cast<const void *>(&k_grid64<BF, W, D3, MS>);
    const int lim = lds_budget(kern, kBlock, w ? budget_fused : budget);
    if (kTabBytes + 4 * rs_max > lim) return UWB_EUNSUPPORTED;   // not even one channel's span fits
    a.lds_bytes = (int)std::min<int64_t>((int64_t)(kTabBytes + 4 * rs_max) * std::min(a.ss.n_ant, kBlock), lim);
    if (w) hipLaunchKernelGGL((k_pl_fused<BF, W, D3, MS>), grid, dim3(kBlock), a.lds_bytes, st, a, *w, levels);
    else hipLaunchKernelGGL((k_grid64<BF, W, D3, MS>), grid, dim3(kBlock), a.lds_bytes, st, a);
    return hipGetLastError() == hipSuccess ? UWB_OK : UWB_EHIP;
}

// rs_max: staged samples per channel of the widest group of the launch.
template <int BF, int W>
int launch_w(bool d3, dim3 grid, const Grid64Args &a, int rs_max, const WalkArgs *w, int levels, hipStream_t st) {
    if (a.ss.ms)
        return d3 ? launch_k<BF, W, true, true>(grid, a, rs_max, w, levels, st)
                  : launch_k<BF, W, false, true>(grid, a, rs_max, w, levels, st);
    return d3 ? launch_k<BF, W, true, false>(grid, a, rs_max, w, levels, st)
              : launch_k<BF, W, false, false>(grid, a, rs_max, w, levels, st);
}

template <int BF>
int launch_bf(int window, bool d3, dim3 grid, const Grid64Args &a, int rs_max, const WalkArgs *w, int levels,
              hipStream_t st) {
    switch (window) {
#define UWB_W(w_) case w_: return launch_w<BF, w_>(d3, grid, a, rs_max, w, levels, st);
        UWB_WINDOWS(UWB_W)
#undef UWB_W
    }
    return UWB_EINVAL;
}

template <>
int launch_bf<UWB_MVDR>(int window, bool d3, dim3 grid, const Grid64Args &a, int rs_max, const WalkArgs *w,
                        int levels, hipStream_t st) {
    switch (window) {
#define UWB_W(w_) case w_: return launch_w<UWB_MVDR, w_>(d3, grid, a, rs_max, w, levels, st);
        UWB_MVDR_WINDOWS(UWB_W)
#undef UWB_W
    }
    return UWB_EUNSUPPORTED;
}

template <typename... A>
int launch_any(int bf, int window, A... args) {
    return bf == UWB_DMAS   ? launch_bf<UWB_DMAS>(window, args...)
           : bf == UWB_MVDR ? launch_bf<UWB_MVDR>(window, args...)
                            : launch_bf<UWB_DAS>(window, args...);
}

// Largest bounding box (lattice steps per axis) of the groups the kernel forms on a
// cnt[0] x cnt[1] x cnt[2] lattice: a tile, or the bands of 256 consecutive points.
void group_extent(const int *cnt, bool d3, int64_t ext[3]) {
    const int tx = d3 ? 8 : 16, ty = d3 ? 8 : 16, tz = d3 ? 4 : 1;
    if (cnt[0] % tx == 0 && cnt[1] % ty == 0 && cnt[2] % tz == 0) {
        ext[0] = tx - 1; ext[1] = ty - 1; ext[2] = tz - 1;
        return;
    }
    const int64_t c0 = cnt[0], c1 = cnt[1], n = c0 * c1 * cnt[2];
    ext[0] = ext[1] = ext[2] = 0;
    for (int64_t p0 = 0; p0 < n; p0 += kBlock) {
        const int64_t p1 = std::min<int64_t>(p0 + kBlock, n) - 1;
        const int64_t az = p0 / (c0 * c1), bz = p1 / (c0 * c1);
        const int64_t ay = (p0 / c0) % c1, by = (p1 / c0) % c1;
        ext[2] = std::max(ext[2], bz - az);
        ext[1] = std::max(ext[1], az == bz ? by - ay : c1 - 1);
        ext[0] = std::max(ext[0], (az == bz && ay == by) ? p1 % c0 - p0 % c0 : c0 - 1);
    }
}

}  // namespace

// max_cnt: lattice points per axis (an upper bound over the scans for ROIs);
// max_step: finest voxels between neighbouring points.
int launch_grid64(Grid64Args a, const int *max_cnt, int max_step, int n_scans, hipStream_t st) {
    const bool d3 = a.g.dims[2] > 1;
    const int64_t points = (int64_t)max_cnt[0] * max_cnt[1] * max_cnt[2];
    if (points < 1 || n_scans < 1) return UWB_OK;
    const int64_t wgs = (points + kBlock - 1) / kBlock;
    if (wgs > 0x7fffffff || n_scans > 65535) return UWB_EUNSUPPORTED;
    // LDS: every channel of the widest group's span, within the kernel's budget (the kernel
    // sizes each group's own chunk of channels to it). A ROI's own size is known only on the
    // device: its groups lie within the bounding lattice.
    int64_t ext[3] = {max_cnt[0] - 1, max_cnt[1] - 1, max_cnt[2] - 1};
    if (a.mode != kGridRoi && points <= (int64_t)kBlock * 4096) group_extent(max_cnt, d3, ext);
    const double s_max = 2.0 / (a.ss.v * a.ss.dt);
    const int rs_max = staged_samples(s_max, (double)ext[0] * max_step * a.g.pitch[0],
                                      (double)ext[1] * max_step * a.g.pitch[1],
                                      (double)ext[2] * max_step * a.g.pitch[2], a.window, a.ss.n_samp);
    const dim3 grid((unsigned)wgs, (unsigned)n_scans);
    return launch_any(a.bf, a.window, d3, grid, a, rs_max, (const WalkArgs *)nullptr, 0, st);
}

// The per-level walk's levels in one launch (a: the kGridBox arguments of its lattices).
int launch_pl_fused(Grid64Args a, const WalkArgs &w, int levels, int n_scans, hipStream_t st) {
    if (n_scans < 1 || levels < 1) return UWB_OK;
    const bool d3 = a.g.dims[2] > 1;
    const int cnt[3] = {w.coarse, w.coarse, d3 ? w.coarse : 1};
    // LDS: sized for level 0, whose groups span the widest boxes
    const int step0 = a.g.dims[0] / w.coarse;
    int64_t ext[3];
    group_extent(cnt, d3, ext);
    const double s_max = 2.0 / (a.ss.v * a.ss.dt);
    const int rs_max = staged_samples(s_max, (double)ext[0] * step0 * a.g.pitch[0], (double)ext[1] * step0 * a.g.pitch[1],
                                      (double)ext[2] * step0 * a.g.pitch[2], a.window, a.ss.n_samp);
    const dim3 grid((unsigned)n_scans);
    return launch_any(a.bf, a.window, d3, grid, a, rs_max, &w, levels, st);
}

}  // namespace uwb
