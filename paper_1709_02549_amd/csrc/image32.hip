// Full-resolution FP32 DAS / DMAS imaging (Eq. (1) delay, Eq. (3) DAS, the
// pairwise DMAS of Section II-B) for gfx950.
//
// A workgroup (256 lanes = 4 wave64) owns a tile of voxels; every lane owns
// kVpl voxels.  For a chunk of antennas the workgroup first derives, per
// antenna, the interval of samples that any voxel of its tile can touch (the
// delay range over the tile's bounding box, computed in FP64, plus the window
// and one sample of margin) and stages those intervals from HBM into LDS with
// coalesced loads (zero outside the recorded trace).  Each lane then, per
// antenna, computes the round-trip delay in registers (one sqrt), reads the
// W+1 consecutive staged samples around it and accumulates the linearly
// interpolated window into W FP32 accumulators:
//   DAS : S_k += s_k
//   DMAS: P_k += s_k * A_k ; A_k += s_k   (A_k = sum of earlier antennas), which
//         regroups sum_{i<j} s_i s_j exactly and keeps the direct sum's error bound.
// The energy sum_k S_k^2 (or P_k^2) is written once per voxel.  No atomics,
// fixed summation order: results are bitwise reproducible.

#include "uwb_internal.h"

namespace uwb {
namespace {

constexpr int kLdsBudget = 40 * 1024;   // bytes of staged samples per workgroup

// Tile geometry.  2D: 16 (x) by 16*kVpl (y); lane (tx, ty) owns y = ty + 16 v.
//                 3D: 8 x 8 x 4*kVpl;     lane (tx, ty, tz) owns z = tz + 4 v.
template <bool D3> struct Tile;
template <> struct Tile<false> { static constexpr int X = 16, Y = 16, Z = 1; };
template <> struct Tile<true>  { static constexpr int X = 8, Y = 8, Z = 4; };
constexpr int kVpl = 2;

struct Args {
    ScanSet ss;
    GridView g;
    float *img;
    int64_t img_stride;     // elements between scans
    int tiles_x, tiles_y;   // tiles along x and y (z = rest)
    int rs;                 // staged samples per antenna (stride in LDS)
    int chunk;              // antennas staged per pass
};

template <int BF, int W, bool D3>
__global__ __launch_bounds__(kBlock) void k_image32(const Args a) {
    using TL = Tile<D3>;
    constexpr int H = (W - 1) / 2;
    constexpr int TX = TL::X, TY = D3 ? TL::Y : TL::Y * kVpl, TZ = D3 ? TL::Z * kVpl : 1;

    extern __shared__ float smem[];
    const int chunk = a.chunk, rs = a.rs;
    float4 *tab = reinterpret_cast<float4 *>(smem);          // [chunk]
    float *stage = smem + 4 * chunk;                          // [chunk][rs]

    const int tid = threadIdx.x;
    const int scan = blockIdx.y;
    const int tile = blockIdx.x;
    const int tx0 = (tile % a.tiles_x) * TX;
    const int ty0 = ((tile / a.tiles_x) % a.tiles_y) * TY;
    const int tz0 = (tile / (a.tiles_x * a.tiles_y)) * TZ;
    const int nx = a.g.dims[0], ny = a.g.dims[1], nz = a.g.dims[2];
    const int T = a.ss.n_samp, M = a.ss.n_ant;

    const ScanConst sc = scan_const(a.ss, scan);
    const float qx = (float)(sc.s * a.g.pitch[0]);
    const float qy = (float)(sc.s * a.g.pitch[1]);
    const float qz = (float)(sc.s * a.g.pitch[2]);
    const float t0s = (float)sc.t0s;
    // this scan's own staging need must fit the launch's (sized for the batch's bound)
    const double ex = (TX - 1) * a.g.pitch[0], ey = (TY - 1) * a.g.pitch[1], ez = (TZ - 1) * a.g.pitch[2];
    const double need = ceil(sc.s * sqrt(ex * ex + ey * ey + ez * ez)) + W + 6;
    const bool fits = need <= (double)rs || rs >= T + 2 * W + 2;

    // lane -> voxels
    int vx, vy[kVpl], vz[kVpl];
    if (!D3) {
        vx = tx0 + (tid & 15);
#pragma unroll
        for (int v = 0; v < kVpl; ++v) { vy[v] = ty0 + (tid >> 4) + 16 * v; vz[v] = 0; }
    } else {
        vx = tx0 + (tid & 7);
#pragma unroll
        for (int v = 0; v < kVpl; ++v) { vy[v] = ty0 + ((tid >> 3) & 7); vz[v] = tz0 + (tid >> 6) + 4 * v; }
    }
    const float fx = (float)vx;
    float fy[kVpl], fz[kVpl];
#pragma unroll
    for (int v = 0; v < kVpl; ++v) { fy[v] = (float)vy[v]; fz[v] = (float)vz[v]; }

    // bounding box of the tile's voxels (inclusive finest indices)
    const int bx1 = min(tx0 + TX, nx) - 1, by1 = min(ty0 + TY, ny) - 1, bz1 = min(tz0 + TZ, nz) - 1;

    float acc[kVpl][W];
    float pre[BF == UWB_DMAS ? kVpl : 1][BF == UWB_DMAS ? W : 1];
#pragma unroll
    for (int v = 0; v < kVpl; ++v)
#pragma unroll
        for (int k = 0; k < W; ++k) acc[v][k] = 0.f;
    if (BF == UWB_DMAS) {
#pragma unroll
        for (int v = 0; v < (BF == UWB_DMAS ? kVpl : 1); ++v)
#pragma unroll
            for (int k = 0; k < (BF == UWB_DMAS ? W : 1); ++k) pre[v][k] = 0.f;
    }

    for (int a0 = 0; a0 < M; a0 += chunk) {
        const int nch = min(chunk, M - a0);
        __syncthreads();   // previous chunk fully consumed
        if (tid < nch) {
            const int i = a0 + tid;
            const double ax = (double)sc.pos[3 * i + 0];
            const double ay = (double)sc.pos[3 * i + 1];
            const double az = (double)sc.pos[3 * i + 2];
            // antenna-relative offsets in sample units: c + idx * q
            const double cx = sc.s * (a.g.origin[0] - ax);
            const double cy = sc.s * (a.g.origin[1] - ay);
            const double cz = sc.s * (a.g.origin[2] - az);
            const double dqx = sc.s * a.g.pitch[0], dqy = sc.s * a.g.pitch[1], dqz = sc.s * a.g.pitch[2];
            const double lx = cx + tx0 * dqx, hx = cx + bx1 * dqx;
            const double ly = cy + ty0 * dqy, hy = cy + by1 * dqy;
            const double lz = cz + tz0 * dqz, hz = cz + bz1 * dqz;
            // nearest point of the tile's box to the antenna (the antenna is at 0 here)
            const double mx = fmin(fmax(0.0, lx), hx), my = fmin(fmax(0.0, ly), hy), mz = fmin(fmax(0.0, lz), hz);
            const double tmin = sqrt(mx * mx + my * my + mz * mz) - sc.t0s;
            // first staged sample: one below the lowest window start; clamped so that
            // a window outside the trace still reads a run of zeros
            double lo = floor(tmin) - (H + 1);
            lo = fmin(fmax(lo, -(double)(W + 1)), (double)(T + W + 1 - rs));
            const int ilo = (int)lo;
            float4 e;
            e.x = (float)cx;
            e.y = (float)cy;
            e.z = D3 ? (float)cz : (float)(cz * cz);
            e.w = __int_as_float(tid * rs - ilo - H);   // window start = floor(tau) + this
            tab[tid] = e;
        }
        __syncthreads();
        // stage [lo, lo + rs) of every antenna of the chunk
        const int wave = tid >> 6, lane = tid & 63;
        for (int j = wave; j < nch; j += kBlock / 64) {
            const int ilo = j * rs - H - __float_as_int(tab[j].w);
            const float *tr = sc.tr + (int64_t)(a0 + j) * T;
            float *dst = stage + j * rs;
            for (int m = lane; m < rs; m += 64) {
                const int gidx = ilo + m;
                dst[m] = (gidx >= 0 && gidx < T) ? tr[gidx] : 0.f;
            }
        }
        __syncthreads();

        for (int j = 0; j < nch; ++j) {
            const float4 e = tab[j];
            const int base = __float_as_int(e.w);
            const int lob = j * rs, hib = j * rs + rs - (W + 1);
            const float dx = fmaf(fx, qx, e.x);
            float part;
            if (!D3) {
                part = fmaf(dx, dx, e.z);
            } else {
                const float dy = fmaf(fy[0], qy, e.y);
                part = fmaf(dy, dy, dx * dx);
            }
#pragma unroll
            for (int v = 0; v < kVpl; ++v) {
                float d2;
                if (!D3) {
                    const float dy = fmaf(fy[v], qy, e.y);
                    d2 = fmaf(dy, dy, part);
                } else {
                    const float dz = fmaf(fz[v], qz, e.z);
                    d2 = fmaf(dz, dz, part);
                }
                const float tau = __builtin_amdgcn_sqrtf(d2) - t0s;
                const float fl = floorf(tau);
                const float f = tau - fl;
                const float g = 1.f - f;
                int idx = (int)fl + base;
                idx = min(max(idx, lob), hib);
                const float *p = stage + idx;
                float y[W + 1];
#pragma unroll
                for (int k = 0; k <= W; ++k) y[k] = p[k];
                if (BF == UWB_DAS) {
#pragma unroll
                    for (int k = 0; k < W; ++k) acc[v][k] = fmaf(f, y[k + 1], fmaf(g, y[k], acc[v][k]));
                } else {
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        const float s = fmaf(f, y[k + 1], g * y[k]);
                        pre[v][k] = fmaf(s, acc[v][k], pre[v][k]);
                        acc[v][k] += s;
                    }
                }
            }
        }
    }

    float *out = a.img + (int64_t)scan * a.img_stride;
#pragma unroll
    for (int v = 0; v < kVpl; ++v) {
        float en = 0.f;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const float q = (BF == UWB_DMAS) ? pre[v][k] : acc[v][k];
            en = fmaf(q, q, en);
        }
        if (!fits) en = __builtin_nanf("");
        if (vx < nx && vy[v] < ny && vz[v] < nz)
            out[((int64_t)vz[v] * ny + vy[v]) * nx + vx] = en;
    }
}

template <int BF, int W>
hipError_t launch_w(bool d3, dim3 grid, size_t lds, hipStream_t st, const Args &a) {
    if (d3) hipLaunchKernelGGL((k_image32<BF, W, true>), grid, dim3(kBlock), lds, st, a);
    else hipLaunchKernelGGL((k_image32<BF, W, false>), grid, dim3(kBlock), lds, st, a);
    return hipGetLastError();
}

template <int BF>
hipError_t launch_bf(int window, bool d3, dim3 grid, size_t lds, hipStream_t st, const Args &a) {
    switch (window) {
#define UWB_W(w) case w: return launch_w<BF, w>(d3, grid, lds, st, a);
        UWB_W(1) UWB_W(3) UWB_W(5) UWB_W(7) UWB_W(9) UWB_W(11) UWB_W(13) UWB_W(15)
        UWB_W(17) UWB_W(19) UWB_W(21) UWB_W(23) UWB_W(25) UWB_W(27) UWB_W(29) UWB_W(31)
#undef UWB_W
    }
    return hipErrorInvalidValue;
}

}  // namespace

// Staged samples per antenna for a tile: the delay range over any box is at most
// s * |box diagonal| (triangle inequality); add the window and margins.
static int staged_samples(const GridView &g, double s_max, int window, int T, bool d3) {
    const int tx = d3 ? Tile<true>::X : Tile<false>::X;
    const int ty = d3 ? Tile<true>::Y : Tile<false>::Y * kVpl;
    const int tz = d3 ? Tile<true>::Z * kVpl : 1;
    const double ex = (tx - 1) * g.pitch[0], ey = (ty - 1) * g.pitch[1], ez = (tz - 1) * g.pitch[2];
    const double span = s_max * sqrt(ex * ex + ey * ey + ez * ez);
    double rs = ceil(span) + window + 6;
    const double cap = (double)T + 2.0 * window + 2.0;
    if (!(rs <= cap)) rs = cap;
    return (int)rs;
}

int launch_image32(int bf, const ScanSet &ss, int n_scans, const GridView &g, int window, float *img,
                   hipStream_t stream) {
    const bool d3 = g.dims[2] > 1;
    const int tx = d3 ? Tile<true>::X : Tile<false>::X;
    const int ty = d3 ? Tile<true>::Y : Tile<false>::Y * kVpl;
    const int tz = d3 ? Tile<true>::Z * kVpl : 1;
    Args a;
    a.ss = ss;
    a.g = g;
    a.img = img;
    a.img_stride = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    a.tiles_x = (g.dims[0] + tx - 1) / tx;
    a.tiles_y = (g.dims[1] + ty - 1) / ty;
    const int tiles_z = (g.dims[2] + tz - 1) / tz;
    // inside a batch the speed may vary per scan: ss.v and ss.dt hold lower bounds
    // over the batch, so this sizes the staging for the largest samples-per-metre
    const double s_max = 2.0 / (ss.v * ss.dt);
    a.rs = staged_samples(g, s_max, window, ss.n_samp, d3);
    const int per_ant = a.rs * 4 + 16;
    if (per_ant > kLdsBudget) return UWB_EUNSUPPORTED;
    a.chunk = kLdsBudget / per_ant;
    if (a.chunk > kBlock) a.chunk = kBlock;
    if (a.chunk > ss.n_ant) a.chunk = ss.n_ant;
    const size_t lds = (size_t)a.chunk * per_ant;
    const int64_t tiles = (int64_t)a.tiles_x * a.tiles_y * tiles_z;
    if (tiles > 0x7fffffff || n_scans > 65535) return UWB_EUNSUPPORTED;
    dim3 grid((unsigned)tiles, (unsigned)n_scans);
    hipError_t e = bf == UWB_DMAS ? launch_bf<UWB_DMAS>(window, d3, grid, lds, stream, a)
                                  : launch_bf<UWB_DAS>(window, d3, grid, lds, stream, a);
    return e == hipSuccess ? UWB_OK : UWB_EHIP;
}

}  // namespace uwb
