// FP64 energies on regular lattices of focal points, for the segment walk:
// the g^d lattice of every scan's current box (per-level walk), the decimated
// lattice of the whole grid (paper walk) and the full-resolution ROI.
//
// The kernel mirrors the FP32 imaging kernel's structure in double precision.
// A workgroup owns a tile of 16 x 16 (2D) or 8 x 8 x 4 (3D) lattice points, one
// point per lane.  For a chunk of antennas it derives (in FP64) the interval of
// samples any point of the tile can reach, stages those intervals from HBM into
// LDS, and then every lane computes its delay for each antenna once (Eq. (1)),
// reads the W+1 staged samples around it and accumulates the linearly
// interpolated window into W FP64 accumulators (Eq. (3) DAS, or the prefix form
// P_k += s_k S_k, S_k += s_k of the Section II-B pairwise DMAS sum).  Positions
// are formed exactly as the rest of the walk forms them (origin + index * pitch
// on the finest grid), antennas are taken in order, and every point's energy is
// written once: the values do not depend on the tile shape.
#include <cmath>

#include "image32.h"
#include "walk_internal.h"

namespace uwb {
namespace {

constexpr int kTabBytes = 64;   // per staged channel: transmitter and receiver positions, first staged sample

template <bool D3> struct Tile64 {
    static constexpr int X = D3 ? 8 : 16, Y = D3 ? 8 : 16, Z = D3 ? 4 : 1;
};

struct Lat {
    int x0[3], step, cnt[3];
};

template <int BF, int W, bool D3>
__global__ __launch_bounds__(kBlock) void k_grid64(const Grid64Args a) {
    using TS = Tile64<D3>;
    constexpr int H = (W - 1) / 2;
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
    // a lattice larger than its output slot (never, for a planned walk) is not written
    if ((int64_t)L.cnt[0] * L.cnt[1] * L.cnt[2] + a.out_offset > a.out_stride) return;
    const int t = blockIdx.x;
    const int tx0 = (t % a.tiles[0]) * TS::X;
    const int ty0 = ((t / a.tiles[0]) % a.tiles[1]) * TS::Y;
    const int tz0 = (t / (a.tiles[0] * a.tiles[1])) * TS::Z;
    if (tx0 >= L.cnt[0] || ty0 >= L.cnt[1] || tz0 >= L.cnt[2]) return;   // uniform per workgroup

    const ScanConst sc = scan_const(a.ss, scan);
    const int M = a.ss.n_ant, T = a.ss.n_samp;
    const int rs = a.rs, chunk = a.chunk;
    double *tab = reinterpret_cast<double *>(dsm);                        // [chunk][8]
    float *stage = reinterpret_cast<float *>(dsm + (size_t)kTabBytes * chunk);   // [chunk][rs]

    // lane -> lattice point -> finest indices -> position
    int kx, ky, kz;
    if (!D3) { kx = tx0 + (tid & 15); ky = ty0 + (tid >> 4); kz = 0; }
    else { kx = tx0 + (tid & 7); ky = ty0 + ((tid >> 3) & 7); kz = tz0 + (tid >> 6); }
    const bool valid = kx < L.cnt[0] && ky < L.cnt[1] && kz < L.cnt[2];
    const int ix = L.x0[0] + L.step * min(kx, L.cnt[0] - 1);
    const int iy = L.x0[1] + L.step * min(ky, L.cnt[1] - 1);
    const int iz = L.x0[2] + L.step * min(kz, L.cnt[2] - 1);
    const double rx = a.g.origin[0] + ix * a.g.pitch[0];
    const double ry = a.g.origin[1] + iy * a.g.pitch[1];
    const double rz = a.g.origin[2] + iz * a.g.pitch[2];

    // the tile's bounding box (metres) and whether this scan's spans fit the staging stride
    double blo[3], bhi[3];
    {
        const int k0[3] = {tx0, ty0, tz0};
        const int ext[3] = {TS::X, TS::Y, TS::Z};
        for (int d = 0; d < 3; ++d) {
            const int k1 = min(k0[d] + ext[d], L.cnt[d]) - 1;
            blo[d] = a.g.origin[d] + (L.x0[d] + L.step * k0[d]) * a.g.pitch[d];
            bhi[d] = a.g.origin[d] + (L.x0[d] + L.step * k1) * a.g.pitch[d];
        }
    }
    const double ex = bhi[0] - blo[0], ey = bhi[1] - blo[1], ez = bhi[2] - blo[2];
    const bool fits = ceil(sc.s * sqrt(ex * ex + ey * ey + ez * ez)) + W + 6 <= (double)rs || rs >= T + 2 * W + 2;

    double S[W], P[BF == UWB_DMAS ? W : 1];
#pragma unroll
    for (int k = 0; k < W; ++k) S[k] = 0.0;
#pragma unroll
    for (int k = 0; k < (BF == UWB_DMAS ? W : 1); ++k) P[k] = 0.0;

    for (int a0 = 0; a0 < M; a0 += chunk) {
        const int nch = min(chunk, M - a0);
        __syncthreads();   // previous chunk consumed
        if (tid < nch) {
            const int i = a0 + tid;
            // transmitter and receiver of the channel (the same antenna when monostatic)
            const float *at = sc.pos + 3 * (sc.ms ? i / sc.ms : i), *ar = sc.pos + 3 * (sc.ms ? i % sc.ms : i);
            double dmin = 0.0;
            for (int leg = 0; leg < 2; ++leg) {
                const float *ap = leg == 0 ? at : ar;
                const double ax = (double)ap[0], ay = (double)ap[1], az = (double)ap[2];
                // nearest point of the tile's box to the antenna: earliest delay of the tile
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
        const int wave = tid >> 6, lane = tid & 63;
        for (int jj = wave; jj < nch; jj += kBlock / 64) {
            const int ilo = (int)tab[8 * jj + 6];
            const float *tr = sc.tr + (int64_t)(a0 + jj) * T;
            float *dst = stage + jj * rs;
            for (int m = lane; m < rs; m += 64) {
                const int gi = ilo + m;
                dst[m] = (gi >= 0 && gi < T) ? tr[gi] : 0.f;
            }
        }
        __syncthreads();
        for (int jj = 0; jj < nch; ++jj) {
            const double dx = rx - tab[8 * jj + 0];
            const double dy = ry - tab[8 * jj + 1];
            const double dz = rz - tab[8 * jj + 2];
            double tau;
            if (sc.ms) {   // Eq. (2): both legs
                const double ux = rx - tab[8 * jj + 3];
                const double uy = ry - tab[8 * jj + 4];
                const double uz = rz - tab[8 * jj + 5];
                tau = 0.5 * sc.s * (sqrt(dx * dx + dy * dy + dz * dz) + sqrt(ux * ux + uy * uy + uz * uz)) - sc.t0s;
            } else {
                tau = sc.s * sqrt(dx * dx + dy * dy + dz * dz) - sc.t0s;
            }
            const double fl = floor(tau);
            const double f = tau - fl;
            // window samples n-H .. n+H+1 sit at stage offsets n-H-lo .. ; the clamp only
            // guards non-finite inputs (every span fits by construction)
            const double off = fmin(fmax(fl - H - tab[8 * jj + 6], 0.0), (double)(rs - (W + 1)));
            const float *p = stage + jj * rs + (int)off;
            float y[W + 1];
#pragma unroll
            for (int k = 0; k <= W; ++k) y[k] = p[k];
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const double s = (1.0 - f) * (double)y[k] + f * (double)y[k + 1];
                if (BF == UWB_DMAS) P[k] += s * S[k];
                S[k] += s;
            }
        }
    }
    double e = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const double q = BF == UWB_DMAS ? P[k] : S[k];
        e += q * q;
    }
    if (!fits) e = __builtin_nan("");
    if (valid) {
        const int64_t p = ((int64_t)kz * L.cnt[1] + ky) * L.cnt[0] + kx;
        a.out64[(int64_t)scan * a.out_stride + a.out_offset + p] = e;
        if (a.out32) a.out32[(int64_t)scan * a.out32_stride + p] = (float)e;
    }
}

template <int BF, int W>
hipError_t launch_w(bool d3, dim3 grid, size_t lds, hipStream_t st, const Grid64Args &a) {
    if (d3) hipLaunchKernelGGL((k_grid64<BF, W, true>), grid, dim3(kBlock), lds, st, a);
    else hipLaunchKernelGGL((k_grid64<BF, W, false>), grid, dim3(kBlock), lds, st, a);
    return hipGetLastError();
}

template <int BF>
hipError_t launch_bf(int window, bool d3, dim3 grid, size_t lds, hipStream_t st, const Grid64Args &a) {
    switch (window) {
#define UWB_W(w) case w: return launch_w<BF, w>(d3, grid, lds, st, a);
        UWB_WINDOWS(UWB_W)
#undef UWB_W
    }
    return hipErrorInvalidValue;
}

}  // namespace

// max_cnt: lattice points per axis (an upper bound over the scans for ROIs);
// max_step: finest voxels between neighbouring points.
int launch_grid64(Grid64Args a, const int *max_cnt, int max_step, int n_scans, hipStream_t st) {
    const bool d3 = a.g.dims[2] > 1;
    const int tx = d3 ? 8 : 16, ty = d3 ? 8 : 16, tz = d3 ? 4 : 1;
    a.tiles[0] = (max_cnt[0] + tx - 1) / tx;
    a.tiles[1] = (max_cnt[1] + ty - 1) / ty;
    a.tiles[2] = (max_cnt[2] + tz - 1) / tz;
    const int64_t tiles = (int64_t)a.tiles[0] * a.tiles[1] * a.tiles[2];
    if (tiles < 1 || n_scans < 1) return UWB_OK;
    if (tiles > 0x7fffffff || n_scans > 65535) return UWB_EUNSUPPORTED;
    // staging stride from the largest samples-per-metre of the batch and the largest tile extent
    const double s_max = 2.0 / (a.ss.v * a.ss.dt);
    a.rs = staged_samples(s_max, (double)(tx - 1) * max_step * a.g.pitch[0], (double)(ty - 1) * max_step * a.g.pitch[1],
                          (double)(tz - 1) * max_step * a.g.pitch[2], a.window, a.ss.n_samp);
    const int per_ant = a.rs * 4 + kTabBytes;
    if (per_ant > kLdsBudget) return UWB_EUNSUPPORTED;
    a.chunk = kLdsBudget / per_ant;
    if (a.chunk > kBlock) a.chunk = kBlock;
    if (a.chunk > a.ss.n_ant) a.chunk = a.ss.n_ant;
    const size_t lds = (size_t)a.chunk * per_ant;
    const dim3 grid((unsigned)tiles, (unsigned)n_scans);
    const hipError_t e = a.bf == UWB_DMAS ? launch_bf<UWB_DMAS>(a.window, d3, grid, lds, st, a)
                                          : launch_bf<UWB_DAS>(a.window, d3, grid, lds, st, a);
    return e == hipSuccess ? UWB_OK : UWB_EHIP;
}

}  // namespace uwb
