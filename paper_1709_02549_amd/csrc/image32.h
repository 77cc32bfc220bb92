// FP32 tile body of the full-resolution DAS / DMAS kernels (shared by the
// grid-mapped kernel in image32.hip and the persistent batch kernel in
// batch.hip).  Internal header.
#pragma once

#include "uwb_internal.h"

namespace uwb {

constexpr int kLdsBudget = 40 * 1024;   // bytes of staged samples per workgroup (default)

// Every odd window 1..31 is compiled.
#define UWB_WINDOWS(X) X(1) X(3) X(5) X(7) X(9) X(11) X(13) X(15) X(17) X(19) X(21) X(23) X(25) X(27) X(29) X(31)
// MVDR: windows up to UWB_MVDR_MAX_WINDOW.
#define UWB_MVDR_WINDOWS(X) X(1) X(3) X(5) X(7) X(9) X(11)

// Staged samples per channel for a tile spanning (ex, ey, ez) metres: the delay
// range over any box is at most s * |box diagonal| (triangle inequality; for a
// bistatic channel each leg contributes s/2 of it); add the window and margins;
// never more than the whole zero-padded trace.
__host__ __device__ inline int staged_samples(double s, double ex, double ey, double ez, int window, int T) {
    const double span = s * sqrt(ex * ex + ey * ey + ez * ez);
    double rs = ceil(span) + window + 6;
    const double cap = (double)T + 2.0 * window + 2.0;
    if (!(rs <= cap)) rs = cap;
    return (int)rs;
}
void tile_shape(bool d3, int vpl, int *tx, int *ty, int *tz);

constexpr int kStageBatch = 8;   // rows of 64 samples a wavefront loads before writing them
constexpr int kMaxSubtiles = 4;  // tiles a workgroup may image from one staging (TileJob::subtiles)

// Windows shorter than this take the delay in FP64.  The FP32 delay carries an absolute error of about
// 2e-5 samples (an ulp of a delay of ~200 samples); an energy summed over 5 or more taps spans a good part
// of a pulse period and moves by ~1e-5 of itself, but the one or three taps of a short window can sit on a
// pulse flank where |slope| / |sample| reaches ~8 per sample at a voxel of 1 % of the peak, which would put
// the relative error of such a voxel at ~3e-4.  In FP64 the delay error is ~1e-13 samples and the only
// FP32 roundings left are those of the fraction, the interpolation and the sums (~1e-7 relative).
constexpr int kExactDelayWindow = 5;

// Copies the staged span [first(j), first(j) + rs) of channels j = 0 .. nch-1 (trace j at
// tr + j * T) to stage + j * rs, zero outside [0, T).  The workgroup's NW wavefronts take
// the channels in turn, a row of 64 samples per load; each wavefront issues kStageBatch rows'
// loads before their LDS writes, so that many loads are in flight instead of one.
template <int NW = kBlock / 64, typename First>
__device__ __forceinline__ void stage_spans(float *stage, int rs, int nch, const float *tr, int T, First first) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nrow = (rs + 63) >> 6;
    const int total = (nch > wave ? (nch - wave + NW - 1) / NW : 0) * nrow;   // this wavefront's rows
    int q = 0, row = 0;   // the batch's first row: channel wave + NW q, samples 64 row ..
    for (int r0 = 0; r0 < total; r0 += kStageBatch) {
        float v[kStageBatch];
        int dst[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int jj = wave + NW * q, m = 64 * row + lane;
            dst[u] = -1;
            v[u] = 0.f;
            if (r0 + u < total && m < rs) {
                dst[u] = jj * rs + m;
                const int gidx = first(jj) + m;
                if (gidx >= 0 && gidx < T) v[u] = tr[(int64_t)jj * T + gidx];
            }
            if (++row == nrow) { row = 0; ++q; }
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u)
            if (dst[u] >= 0) stage[dst[u]] = v[u];
    }
}

// Staged samples are read as 16-byte records (one ds_read_b128 each): 16-byte LDS reads stream at
// about twice the bytes per clock of 4- and 8-byte ones.  Record m of a channel holds either
//   plain (DIFF = false): (y_m, y_m+1, y_m+2, y_m+3), the window of W + 1 samples from sample n
//       in records n, n + 4, ... (ceil((W + 1) / 4) reads; three for W = 11), or
//   DIFF: (y_m, y_m+1 - y_m, y_m+1, y_m+2 - y_m+1), the W taps from n in records n, n + 2, ...
//       ((W + 1) / 2 reads; six for W = 11), so that each tap's linear interpolation
//       y + f (y' - y) is one FMA.
// Every record index read stays inside the channel's staged span: the window start n is at most
// rs - W - 1, and the last record read starts 4 (N - 1) <= W (plain) or W - 1 (DIFF) samples
// past it.
template <int W, bool DIFF> struct Rec {
    static constexpr int N = DIFF ? (W + 1) / 2 : (W + 1 + 3) / 4;   // records per window
    static constexpr int STEP = DIFF ? 2 : 4;                        // samples per record step
    static_assert(STEP * (N - 1) <= W, "record reads past the window");
};

// Copies the records (see Rec) of samples first(j) + m, m = 0 .. rs-1, of channels
// j = 0 .. nch-1 (trace j at tr + j * T) to rec[j * rs + m], samples outside [0, T) being zero.
// The workgroup's NW wavefronts take the channels in turn, a row of 64 records per step
// (overlapping, coalesced loads per lane); each wavefront issues kStageBatch rows' loads before
// their LDS writes, so that many loads are in flight instead of one.
template <bool DIFF, int NW = kBlock / 64, typename First>
__device__ __forceinline__ void stage_records(float4 *rec, int rs, int nch, const float *tr, int T, First first) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nrow = (rs + 63) >> 6;
    const int total = (nch > wave ? (nch - wave + NW - 1) / NW : 0) * nrow;   // this wavefront's rows
    int q = 0, row = 0;   // the batch's first row: channel wave + NW q, records 64 row ..
    for (int r0 = 0; r0 < total; r0 += kStageBatch) {
        float4 v[kStageBatch];
        int dst[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int jj = wave + NW * q, m = 64 * row + lane;
            dst[u] = -1;
            v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r0 + u < total && m < rs) {
                dst[u] = jj * rs + m;
                const int gidx = first(jj) + m;
                const float *t = tr + (int64_t)jj * T;
                float y[4];
#pragma unroll
                for (int e = 0; e < (DIFF ? 3 : 4); ++e) y[e] = (gidx + e >= 0 && gidx + e < T) ? t[gidx + e] : 0.f;
                if (DIFF) v[u] = make_float4(y[0], y[1] - y[0], y[1], y[2] - y[1]);
                else v[u] = make_float4(y[0], y[1], y[2], y[3]);
            }
            if (++row == nrow) { row = 0; ++q; }
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u)
            if (dst[u] >= 0) rec[dst[u]] = v[u];
    }
}

// One tile of one scan.
struct TileJob {
    const float *pos;     // [M][3]
    const float *tr;      // [M][T]
    float *img;           // [nz][ny][nx]
    int M, T;
    double s, t0s;        // samples per metre of path (2 / (v dt)) and t0 / dt
    GridView g;
    int tx0, ty0, tz0;    // first voxel of the tile
    int rs;               // staged samples per channel (LDS stride)
    int chunk;            // channels staged per pass
    int ms;               // multistatic: antennas per side (channel i*ms + j), 0: monostatic
    int64_t p0;           // band form: first voxel (linear, x fastest) of the band
    float *img_das = nullptr;   // DMAS only, optional: the DAS image of the same voxels
    float *tmax = nullptr;      // optional: the tile's FP32 maximum of img (of img_das: tmax_das)
    float *tmax_das = nullptr;
    int subtiles = 1;           // tiles along x imaged from one staging (then every channel fits one chunk)
};

// Tile geometry.  2D: 16 (x) by 16*VPL (y); lane (tx, ty) owns y = ty + 16 v.
//                 3D: 8 x 8 x 4*VPL;     lane (tx, ty, tz) owns z = tz + 4 v.
// A wave covers a 16 x 4 (2D) or 8 x 8 (3D) patch per v, so its delays -- and
// its LDS addresses -- stay within a few samples of each other.
template <bool D3, int VPL> struct TileShape {
    static constexpr int X = D3 ? 8 : 16, Y = D3 ? 8 : 16 * VPL, Z = D3 ? 4 * VPL : 1;
    __device__ static void get(int &x, int &y, int &z) { x = X; y = Y; z = Z; }
};

// floor(x) as an int in one instruction (x finite and within the int range; the
// compiler fuses floor and conversion only under finite-math flags)
__device__ __forceinline__ int floor_to_int(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Bounding box (inclusive finest indices) of the voxels p0 .. p1 of an nx x ny x nz grid
// in linear order: within one row its own columns; across rows whole rows; across
// slabs whole slabs.
__host__ __device__ inline void band_box(int64_t p0, int64_t p1, int nx, int ny, int &x0, int &x1, int &y0, int &y1,
                                         int &z0, int &z1) {
    const int64_t sxy = (int64_t)nx * ny;
    const int ax = (int)(p0 % nx), ay = (int)((p0 / nx) % ny), az = (int)(p0 / sxy);
    const int bx = (int)(p1 % nx), by = (int)((p1 / nx) % ny), bz = (int)(p1 / sxy);
    z0 = az; z1 = bz;
    y0 = az == bz ? ay : 0; y1 = az == bz ? by : ny - 1;
    x0 = (az == bz && ay == by) ? ax : 0; x1 = (az == bz && ay == by) ? bx : nx - 1;
}

// Monostatic (MS = false): channel i is antenna i, delay s |r - a_i| - t0s (Eq. (1)).
// Multistatic (MS = true): channel i*M + j, delay (s/2)(|r - a_i| + |r - a_j|) - t0s
// (Eq. (2)); the table then holds the transmitter's and the receiver's offsets.
// BAND (one voxel per lane only): the workgroup images the 256 consecutive voxels
// from j.p0 (x fastest) instead of a tile -- for small, ragged grids, whose tiles
// would idle many lanes; j.rs must cover the band's bounding box (band_box).
// T0Z: the scan's t0 is zero (sample 0 at the excitation peak, as in the workloads), so the monostatic delay
// is the scaled distance itself and its subtraction of t0 / dt, one instruction per voxel·antenna, is left
// out; subtracting zero is exact, so the energies are those of the general form bit for bit.
template <int BF, int W, bool D3, int VPL, bool MS = false, bool BAND = false, bool T0Z = false>
__device__ __forceinline__ void image_tile(const TileJob &j, float *smem) {
    static_assert(!BAND || VPL == 1, "a band holds one voxel per lane");
    using TS = TileShape<D3, VPL>;
    constexpr int H = (W - 1) / 2;
    constexpr int TX = TS::X, TY = TS::Y, TZ = TS::Z;
    constexpr int TE = MS ? 2 : 1;                            // table entries per channel
    // DMAS and MVDR interpolate from difference records (one FMA per tap); DAS, bound by the LDS
    // reads rather than by arithmetic, from plain ones (half the bytes)
    constexpr bool DIFF = BF != UWB_DAS;
    constexpr int NR = Rec<W, DIFF>::N;                       // records read per window
    constexpr int NY = DIFF ? 2 * NR : 4 * NR;                // floats gathered per window
    const int chunk = j.chunk, rs = j.rs;
    float4 *tab = reinterpret_cast<float4 *>(smem);          // [chunk][TE]
    float4 *recs = tab + TE * chunk;                          // [chunk][rs] records of 4 samples
    const double sc = MS ? 0.5 * j.s : j.s;                   // samples per metre of each leg
    const int tid = threadIdx.x;
    const int nx = j.g.dims[0], ny = j.g.dims[1], nz = j.g.dims[2];
    const int T = j.T, M = j.M;
    const int tx0 = j.tx0, ty0 = j.ty0, tz0 = j.tz0;
    // S tiles side by side along x share one staging of the traces: the staged span covers their union,
    // which is only a few samples longer than one tile's, and the table and the staging pass (global-memory
    // latency between two barriers) are paid once for S tiles.  The host sets S > 1 when every channel fits
    // one chunk; with several chunks each sub-tile stages them again.
    const int S = BAND ? 1 : j.subtiles;

    const float qx = (float)(sc * j.g.pitch[0]);
    const float qy = (float)(sc * j.g.pitch[1]);
    const float qz = (float)(sc * j.g.pitch[2]);
    const float t0s = (float)j.t0s;

    // lane -> voxels, and the bounding box of the workgroup's voxels (inclusive finest indices)
    // a lane's voxels differ only in y (2D) or z (3D), by a constant stride: one base each
    int vx, vy0, vz0;
    int bx0, by0, bz0, bx1, by1, bz1;
    bool live = true;   // band form: the lane's voxel exists
    if (BAND) {
        const int64_t n = (int64_t)nx * ny * nz, sxy = (int64_t)nx * ny;
        const int64_t p = j.p0 + tid, p1 = min(j.p0 + kBlock, n) - 1, pc = min(p, p1);
        live = p <= p1;
        vx = (int)(pc % nx);
        vy0 = (int)((pc / nx) % ny);
        vz0 = (int)(pc / sxy);
        band_box(j.p0, p1, nx, ny, bx0, bx1, by0, by1, bz0, bz1);
    } else if (!D3) {
        vx = tx0 + (tid & 15);
        vy0 = ty0 + (tid >> 4);
        vz0 = 0;
    } else {
        vx = tx0 + (tid & 7);
        vy0 = ty0 + ((tid >> 3) & 7);
        vz0 = tz0 + (tid >> 6);
    }
    if (!BAND) {
        bx0 = tx0; by0 = ty0; bz0 = tz0;
        bx1 = min(tx0 + S * TX, nx) - 1; by1 = min(ty0 + TY, ny) - 1; bz1 = min(tz0 + TZ, nz) - 1;
    }
    // this scan's own staging need must fit the launch's (a batch is sized for its bound)
    const double ex = (BAND ? bx1 - bx0 : S * TX - 1) * j.g.pitch[0], ey = (BAND ? by1 - by0 : TY - 1) * j.g.pitch[1],
                 ez = (BAND ? bz1 - bz0 : TZ - 1) * j.g.pitch[2];
    const double need = ceil(j.s * sqrt(ex * ex + ey * ey + ez * ez)) + W + 6;
    const bool fits = need <= (double)rs || rs >= T + 2 * W + 2;
    // voxel v of the lane: y = vy0 + 16 v (2D) or z = vz0 + 4 v (3D)
    auto VY = [&](int v) { return D3 ? vy0 : vy0 + 16 * v; };
    auto VZ = [&](int v) { return D3 ? vz0 + 4 * v : vz0; };
    // the coordinate in which the lane's voxels differ, as FP32, converted once for all channels
    // (DMAS and MVDR up to W = 11: 1.5-2 % faster); the DAS kernel, at four waves, and the wider
    // windows, whose accumulators already spill, keep converting it per channel
    constexpr bool kHoistCoord = BF != UWB_DAS && W <= 11;
    float fvv[VPL];
    if constexpr (kHoistCoord) {
#pragma unroll
        for (int v = 0; v < VPL; ++v) fvv[v] = (float)(D3 ? VZ(v) : VY(v));
    }
    auto FV = [&](int v) { return kHoistCoord ? fvv[v] : (float)(D3 ? VZ(v) : VY(v)); };

    // per sub-tile and wavefront: the maxima of the image and of the DAS image (tile maxima)
    __shared__ float tile_red[kMaxSubtiles][2][kBlock / 64];
    int n_sub = 0;   // sub-tiles imaged (those inside the grid)
    for (int st = 0; st < S; ++st, vx += TX) {
    if (!BAND && vx - (tid & (TX - 1)) >= nx) break;   // uniform: this sub-tile lies past the grid
    const float fx = (float)vx;

    // MVDR: one voxel per lane, whose window sums (acc) and Gram matrix (packed lower triangle) feed
    // the W x W solve of mvdr_energy
    constexpr bool MV = BF == UWB_MVDR;
    static_assert(!MV || VPL == 1, "the MVDR statistics of one voxel fill a lane's registers");
    constexpr int NG = MV ? W * (W + 1) / 2 : 1;
    float acc[VPL][W];
    float pre[BF == UWB_DMAS ? VPL : 1][BF == UWB_DMAS ? W : 1];
    float gram[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) gram[q] = 0.f;
#pragma unroll
    for (int v = 0; v < VPL; ++v)
#pragma unroll
        for (int k = 0; k < W; ++k) acc[v][k] = 0.f;
    if (BF == UWB_DMAS) {
#pragma unroll
        for (int v = 0; v < (BF == UWB_DMAS ? VPL : 1); ++v)
#pragma unroll
            for (int k = 0; k < (BF == UWB_DMAS ? W : 1); ++k) pre[v][k] = 0.f;
    }

    float dtx[MS ? VPL : 1];   // bistatic: current transmitter's leg (sample units) minus t0s, per voxel
#pragma unroll
    for (int v = 0; v < (MS ? VPL : 1); ++v) dtx[v] = 0.f;

    for (int a0 = 0; a0 < M; a0 += chunk) {
        const int nch = min(chunk, M - a0);
        if (st == 0 || chunk < M) {   // one chunk: its table and records serve every sub-tile
        __syncthreads();   // previous chunk (or previous tile) fully consumed
        if (tid < nch) {
            const int i = a0 + tid;
            // The box products below are the same in every chunk; hoisted out of the chunk loop they would
            // stay live (six doubles) across the voxel loop and be spilled to scratch memory, once per lane.
            // An empty asm statement on copies of the bounds (and of a zero the scale is offset by) keeps them
            // inside this branch.
            int b0x = bx0, b1x = bx1, b0y = by0, b1y = by1, b0z = bz0, b1z = bz1, zero = 0;
            asm volatile("" : "+v"(b0x), "+v"(b1x), "+v"(b0y), "+v"(b1y), "+v"(b0z), "+v"(b1z), "+v"(zero));
            const double scl = sc + (double)zero, t0s_d = j.t0s + (double)zero;
            const double dqx = scl * j.g.pitch[0], dqy = scl * j.g.pitch[1], dqz = scl * j.g.pitch[2];
            double tmin = -t0s_d;
            float4 e[TE];
#pragma unroll
            for (int leg = 0; leg < TE; ++leg) {
                const int ant = MS ? (leg == 0 ? i / j.ms : i % j.ms) : i;
                const double ax = (double)j.pos[3 * ant + 0];
                const double ay = (double)j.pos[3 * ant + 1];
                const double az = (double)j.pos[3 * ant + 2];
                // antenna-relative offsets in sample units: c + idx * q
                const double cx = scl * (j.g.origin[0] - ax);
                const double cy = scl * (j.g.origin[1] - ay);
                const double cz = scl * (j.g.origin[2] - az);
                const double lx = cx + b0x * dqx, hx = cx + b1x * dqx;
                const double ly = cy + b0y * dqy, hy = cy + b1y * dqy;
                const double lz = cz + b0z * dqz, hz = cz + b1z * dqz;
                // nearest point of the tile's box to the antenna (the antenna is at 0 here)
                const double mx = fmin(fmax(0.0, lx), hx), my = fmin(fmax(0.0, ly), hy), mz = fmin(fmax(0.0, lz), hz);
                tmin += sqrt(mx * mx + my * my + mz * mz);
                e[leg].x = (float)cx;
                e[leg].y = (float)cy;
                e[leg].z = D3 ? (float)cz : (float)(cz * cz);
                e[leg].w = 0.f;
            }
            // first staged sample: one below the lowest window start; clamped so that
            // a window outside the trace still reads a run of zeros
            double lo = floor(tmin) - (H + 1);
            lo = fmin(fmax(lo, -(double)(W + 1)), (double)(T + W + 1 - rs));
            const int ilo = (int)lo;
            e[0].w = __int_as_float(tid * rs - ilo - H);   // window start = floor(tau) + this
#pragma unroll
            for (int leg = 0; leg < TE; ++leg) tab[TE * tid + leg] = e[leg];
        }
        __syncthreads();
        // stage the records of [lo, lo + rs) of every antenna of the chunk
        stage_records<DIFF>(recs, rs, nch, j.tr + (int64_t)a0 * T, T,
                            [&](int jj) { return jj * rs - H - __float_as_int(tab[TE * jj].w); });
        __syncthreads();
        }

        // bistatic: receiver of the chunk's first channel (channels run in order, so a
        // transmitter's distances carry over a chunk boundary)
        int rxi = MS ? a0 % j.ms : 0;
        for (int jj = 0; jj < nch; ++jj) {
            const float4 e = tab[TE * jj];
            const float4 er = tab[TE * jj + (MS ? 1 : 0)];
            // window start in the stage = floor(tau) + base, kept within the channel's span
            // [jj rs, jj rs + rs - W - 1]: tau is clamped to the equivalent integer bounds
            // [lof, hif] before the floor (same index; a clamped window lies wholly in the
            // staged zero padding, so its fraction does not matter)
            const int base = __builtin_amdgcn_readfirstlane(__float_as_int(e.w));
            const float4 *sb = recs + base;
            const float lof = (float)(jj * rs - base), hif = lof + (float)(rs - (W + 1));
            // squared distance from the lane's voxels to one leg's antenna: leg_d2 forms the part
            // shared by the lane's voxels, leg_v adds voxel v's own coordinate
            auto leg_d2 = [&](const float4 &t, float &part) {
                const float dx = fmaf(fx, qx, t.x);
                if (!D3) part = fmaf(dx, dx, t.z);
                else { const float dy = fmaf((float)vy0, qy, t.y); part = fmaf(dy, dy, dx * dx); }
            };
            auto leg_v = [&](const float4 &t, float part, int v) {
                if (!D3) { const float dy = fmaf(FV(v), qy, t.y); return fmaf(dy, dy, part); }
                const float dz = fmaf(FV(v), qz, t.z);
                return fmaf(dz, dz, part);
            };
            float part, partr = 0.f;
            if (MS) {
                if (rxi == 0) {   // a new transmitter (uniform over the workgroup): its leg per voxel
                    leg_d2(e, part);
#pragma unroll
                    for (int v = 0; v < VPL; ++v) dtx[v] = __builtin_amdgcn_sqrtf(leg_v(e, part, v)) - t0s;
                }
                rxi = rxi + 1 == j.ms ? 0 : rxi + 1;
                leg_d2(er, partr);
            } else {
                leg_d2(e, part);
            }
            // software-pipelined over the lane's voxels: voxel v + 1's delay and window reads are
            // issued before voxel v's taps, so their LDS latency overlaps arithmetic
            auto locate = [&](int v, float &f, const float4 *&p) {
                if constexpr (W < kExactDelayWindow) {
                    // FP64 delay from the positions themselves (Eq. (1) / Eq. (2)); the window start is
                    // clamped to the same integer bounds as below
                    const int ch = a0 + jj;
                    const float *at = j.pos + 3 * (MS ? ch / j.ms : ch), *ar = j.pos + 3 * (MS ? ch % j.ms : ch);
                    const double rx = j.g.origin[0] + (double)vx * j.g.pitch[0];
                    const double ry = j.g.origin[1] + (double)VY(v) * j.g.pitch[1];
                    const double rz = j.g.origin[2] + (double)VZ(v) * j.g.pitch[2];
                    double dist = 0.0;
#pragma unroll
                    for (int leg = 0; leg < TE; ++leg) {
                        const float *ap = leg == 0 ? at : ar;
                        const double dx = rx - (double)ap[0], dy = ry - (double)ap[1], dz = rz - (double)ap[2];
                        dist += sqrt(dx * dx + dy * dy + dz * dz);
                    }
                    const double tau = sc * dist - j.t0s;
                    const double fl = floor(tau);
                    const double n = fmin(fmax(fl, (double)lof), (double)hif);
                    f = (float)(tau - fl);
                    p = sb + (int)n;
                } else {
                    float tau;
                    if (MS) tau = dtx[v] + __builtin_amdgcn_sqrtf(leg_v(er, partr, v));
                    else if constexpr (T0Z) tau = __builtin_amdgcn_sqrtf(leg_v(e, part, v));
                    else tau = __builtin_amdgcn_sqrtf(leg_v(e, part, v)) - t0s;
                    tau = __builtin_amdgcn_fmed3f(tau, lof, hif);
                    f = __builtin_amdgcn_fractf(tau);
                    p = sb + floor_to_int(tau);
                }
            };
            // the window from NR records: plain, y[k] = sample n + k (k <= W); DIFF, y[2k] = sample
            // n + k and y[2k + 1] = its forward difference (k < W)
            auto gather = [&](const float4 *p, float *y) {
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const float4 q = p[Rec<W, DIFF>::STEP * r];
                    y[4 * r] = q.x; y[4 * r + 1] = q.y; y[4 * r + 2] = q.z; y[4 * r + 3] = q.w;
                }
            };
            float fc, yc[4 * NR];
            {
                const float4 *p;
                locate(0, fc, p);
                gather(p, yc);
            }
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                float fn = 0.f, yn[4 * NR];
                static_assert(NY <= 4 * NR, "gathered floats");
                if (v + 1 < VPL) {
                    const float4 *p;
                    locate(v + 1, fn, p);
                    gather(p, yn);
                }
                __builtin_amdgcn_sched_barrier(0);   // keep those reads ahead of this voxel's taps
                const float f = fc, g = 1.f - fc;
                if (BF == UWB_DAS) {
#pragma unroll
                    for (int k = 0; k < W; ++k) acc[v][k] = fmaf(f, yc[k + 1], fmaf(g, yc[k], acc[v][k]));
                } else if (MV) {
                    float sv[W];
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        sv[k] = fmaf(f, yc[2 * k + 1], yc[2 * k]);
                        acc[v][k] += sv[k];
                    }
#pragma unroll
                    for (int k = 0; k < W; ++k)
#pragma unroll
                        for (int l = 0; l <= k; ++l) gram[tri(k, l)] = fmaf(sv[k], sv[l], gram[tri(k, l)]);
                } else {
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        const float s = fmaf(f, yc[2 * k + 1], yc[2 * k]);
                        pre[v][k] = fmaf(s, acc[v][k], pre[v][k]);
                        acc[v][k] += s;
                    }
                }
                if (v + 1 < VPL) {
                    fc = fn;
#pragma unroll
                    for (int k = 0; k < 4 * NR; ++k) yc[k] = yn[k];
                }
            }
        }
    }

    // the DMAS running sums acc_k = sum of s_k over every antenna are the DAS window sums
    // (Eq. (3)): a DMAS tile writes the DAS image too when asked, at no extra reads
    float *const das = BF == UWB_DMAS ? j.img_das : nullptr;
    float tm = -INFINITY, tmd = -INFINITY;   // this lane's maxima of its voxels (NaN ignored, as fmaxf does)
    // the voxels' row offsets are the same in every sub-tile; computed here from a laundered zero, they are
    // not hoisted out of the sub-tile loop (kept live across it they would be spilled to scratch memory)
    int zrow = 0;
    asm volatile("" : "+v"(zrow));
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        float en = 0.f, ed = 0.f;
        if constexpr (MV) {
            en = mvdr_energy<float, W>(gram, acc[0], M);
        } else {
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const float q = (BF == UWB_DMAS) ? pre[v][k] : acc[v][k];
                en = fmaf(q, q, en);
                if (BF == UWB_DMAS) ed = fmaf(acc[v][k], acc[v][k], ed);
            }
        }
        if (!fits) en = ed = __builtin_nanf("");
        if (live && vx < nx && VY(v) < ny && VZ(v) < nz) {
            const int64_t o = ((int64_t)(VZ(v) + zrow) * ny + (VY(v) + zrow)) * nx + (vx + zrow);
            j.img[o] = en;
            if (das) das[o] = ed;
            tm = fmaxf(tm, en);
            tmd = fmaxf(tmd, ed);
        }
    }
    // the tile's maxima, for a detection that reads them instead of the image (uniform branch): each
    // wavefront's maxima per sub-tile go to LDS, combined once after the last sub-tile
    if (!MV && j.tmax) {
        tm = wave_maxf(tm);
        tmd = wave_maxf(tmd);
        if ((tid & 63) == 0) { tile_red[st][0][tid >> 6] = tm; tile_red[st][1][tid >> 6] = tmd; }
    }
    ++n_sub;
    }   // sub-tiles
    if (BF != UWB_MVDR && j.tmax) {
        __syncthreads();
        if (tid < n_sub) {   // the sub-tiles' tiles are consecutive in tile order
            float m = tile_red[tid][0][0], md = tile_red[tid][1][0];
            for (int w = 1; w < kBlock / 64; ++w) { m = fmaxf(m, tile_red[tid][0][w]); md = fmaxf(md, tile_red[tid][1][w]); }
            j.tmax[tid] = m;
            if (j.tmax_das) j.tmax_das[tid] = md;
        }
    }
}

}  // namespace uwb
