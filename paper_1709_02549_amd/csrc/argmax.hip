// Detection by maximal synthesized energy (Section II-A), decided in FP64.
//
// The FP32 image locates the candidates; the decision is re-taken in FP64 so it
// does not depend on FP32 rounding.  Pipeline per scan (stream-ordered, no host
// synchronisation, no floating-point atomics, deterministic):
//   A  per 4096-voxel chunk: FP32 maximum                         -> cmax32[c]
//   B  one workgroup: thr32 = max32 - kCandRel |max32|, and the list of the chunks
//      whose maximum reaches it (in chunk order)
//   C  per listed chunk: every voxel with I32 >= thr32 is re-evaluated in FP64 by a
//      whole wave (antennas split over the 64 lanes, the chunk's four waves taking
//      the candidates in turn); chunk maximum and a short list of (index, value)
//                                                                 -> cmax64[c], list
//   D  one workgroup: thr64 = max64 - 1e-12 |max64| over the listed chunks
//   E  per listed chunk: lowest index among candidates with FP64 value >= thr64 (from
//      the list, or re-evaluated when the chunk had more candidates than it holds)
//   F  one workgroup: lowest index over chunks -> uwb_peak
// Stages C and E run kChunkCap workgroups per scan over the listed chunks (usually
// one to three hold candidates), not one per chunk.
// Tile mode: the chunks are the tiles of the full-resolution DAS / DMAS launch, whose
// FP32 maxima that launch wrote (uwb_das_dmas_batch_tilemax), and stage A is skipped:
// the image is read only where a tile holds candidates.  Within a tile, voxels in
// tile order have increasing linear indices, so both modes list and compare
// candidates in index order and give the same uwb_peak.
#include <climits>
#include <cstdint>
#include <cmath>
#include <mutex>

#include "uwb_internal.h"

namespace uwb {
namespace {

constexpr int kPerThread = 16;
constexpr int kChunkVox = kBlock * kPerThread;    // 4096 voxels per workgroup
constexpr int kList = 8;                          // candidates remembered per chunk
constexpr int kChunkCap = 8;                      // listed chunks per scan (stages C, E workgroups)

struct ChunkRec {           // one per (scan, chunk)
    float max32;
    int32_t count;          // FP64-evaluated candidates in the chunk
    double max64;
    int64_t idx[kList];
    double val[kList];
    int64_t best_idx;       // stage E result (INT64_MAX: none)
    double best_val;
};
struct ScanRec {            // one per scan
    float thr32;
    float max32;
    double thr64;
    double max64;
};

struct Args {
    ScanSet ss;
    GridView g;
    int window, bf;
    const float *img;
    int64_t nvox;
    int nchunks;
    int per_thread;         // voxels per lane of a chunk (chunk voxels / kBlock)
    ChunkRec *chunks;       // [scan][nchunks]
    ScanRec *scans;         // [scan]
    int *clist;             // [scan][1 + kChunkCap]: number of chunks reaching thr32, then the first ones
    uwb_peak *out;
    const float *tmax;      // tile mode: [scan][nchunks] FP32 tile maxima; null: chunk mode
    int tx, ty, tz, tiles_x, tiles_y;   // tile mode: tile shape and tiles along x, y
};

// Linear index of voxel `off` of chunk c, or -1 past the grid.
__device__ __forceinline__ int64_t chunk_voxel(const Args &a, int c, int off) {
    if (!a.tmax) {
        const int64_t v = (int64_t)c * kChunkVox + off;
        return v < a.nvox ? v : -1;
    }
    const int x = (c % a.tiles_x) * a.tx + off % a.tx;
    const int y = ((c / a.tiles_x) % a.tiles_y) * a.ty + (off / a.tx) % a.ty;
    const int z = (c / (a.tiles_x * a.tiles_y)) * a.tz + off / (a.tx * a.ty);
    if (x >= a.g.dims[0] || y >= a.g.dims[1] || z >= a.g.dims[2]) return -1;
    return ((int64_t)z * a.g.dims[1] + y) * a.g.dims[0] + x;
}

// The i-th chunk a stage C / E workgroup takes (i = blockIdx.x, blockIdx.x + gridDim.x, ...), -1 when
// done: the listed chunks, or every chunk when more reached thr32 than the list holds (the stages then
// skip those below it).
__device__ __forceinline__ int listed_chunk(const Args &a, int scan, int i) {
    const int *L = a.clist + (int64_t)scan * (1 + kChunkCap);
    const int cnt = L[0];
    if (cnt <= kChunkCap) return i < cnt ? L[1 + i] : -1;
    return i < a.nchunks ? i : -1;
}

__device__ __forceinline__ void voxel_pos(const GridView &g, int64_t idx, double &rx, double &ry, double &rz) {
    const int64_t nx = g.dims[0], ny = g.dims[1];
    const int64_t ix = idx % nx, iy = (idx / nx) % ny, iz = idx / (nx * ny);
    rx = g.origin[0] + (double)ix * g.pitch[0];
    ry = g.origin[1] + (double)iy * g.pitch[1];
    rz = g.origin[2] + (double)iz * g.pitch[2];
}

__device__ __forceinline__ float block_maxf(float x, float *red) {
    x = wave_maxf(x);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = x;
    __syncthreads();
    float r = red[0];
    for (int i = 1; i < kBlock / 64; ++i) r = fmaxf(r, red[i]);
    return r;
}

// 16-byte loads when every scan's image starts 16-byte aligned (voxels per scan a
// multiple of 4) and the chunk is whole: four float4 per lane, all issued before use.
__global__ __launch_bounds__(kBlock) void k_chunk_max32(const Args a) {
    __shared__ float red[kBlock / 64];
    const int scan = blockIdx.y, c = blockIdx.x;
    const float *img = a.img + (int64_t)scan * a.nvox;
    const int64_t c0 = (int64_t)c * kChunkVox;
    float m = -INFINITY;
    if ((a.nvox & 3) == 0 && c0 + kChunkVox <= a.nvox && (reinterpret_cast<uintptr_t>(a.img) & 15) == 0) {
        const float4 *v4 = reinterpret_cast<const float4 *>(img + c0);
        float4 x[kPerThread / 4];
#pragma unroll
        for (int k = 0; k < kPerThread / 4; ++k) x[k] = v4[k * kBlock + threadIdx.x];
#pragma unroll
        for (int k = 0; k < kPerThread / 4; ++k) m = fmaxf(m, fmaxf(fmaxf(x[k].x, x[k].y), fmaxf(x[k].z, x[k].w)));
    } else {
        for (int k = 0; k < kPerThread; ++k) {
            const int64_t v = c0 + k * kBlock + threadIdx.x;
            if (v < a.nvox) m = fmaxf(m, img[v]);
        }
    }
    m = block_maxf(m, red);
    if (threadIdx.x == 0) a.chunks[(int64_t)scan * a.nchunks + c].max32 = m;
}

__global__ __launch_bounds__(kBlock) void k_reduce32(const Args a) {
    __shared__ float red[kBlock / 64];
    __shared__ int wcnt[kBlock / 64];
    const int scan = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    ChunkRec *recs = a.chunks + (int64_t)scan * a.nchunks;
    float m = -INFINITY;
    for (int c = threadIdx.x; c < a.nchunks; c += kBlock) {
        float x;
        if (a.tmax) {   // tile mode: the imaging launch's tile maxima become the chunk maxima
            x = a.tmax[(int64_t)scan * a.nchunks + c];
            recs[c].max32 = x;
        } else {
            x = recs[c].max32;
        }
        m = fmaxf(m, x);
    }
    m = block_maxf(m, red);
    const float thr = m - (float)kCandRel * fabsf(m);
    // the chunks reaching thr32, in chunk order (every lane read its own chunks' maxima above)
    int *L = a.clist + (int64_t)scan * (1 + kChunkCap);
    int count = 0;   // uniform
    for (int c0 = 0; c0 < a.nchunks; c0 += kBlock) {
        const int c = c0 + threadIdx.x;
        const bool hit = c < a.nchunks && recs[c].max32 >= thr;
        const unsigned long long mask = __ballot(hit);
        if (lane == 0) wcnt[wave] = __popcll(mask);
        __syncthreads();
        int slot = count + __popcll(mask & ((1ull << lane) - 1));
        for (int w = 0; w < wave; ++w) slot += wcnt[w];
        if (hit && slot < kChunkCap) L[1 + slot] = c;
        for (int w = 0; w < kBlock / 64; ++w) count += wcnt[w];
        __syncthreads();   // wcnt read by every lane before the next round writes it
    }
    if (threadIdx.x == 0) {
        a.scans[scan].max32 = m;
        a.scans[scan].thr32 = thr;
        L[0] = count;
    }
}

constexpr int kEvalCap = 512;   // candidates of a chunk listed in LDS for stage C

// Stage C: FP64 evaluation of the chunk's candidates.  They are listed in index order in
// LDS and the four wavefronts evaluate them four at a time (each candidate on a whole
// wavefront, so its value does not depend on which one takes it); a chunk with more
// candidates than the list holds has every wavefront evaluate its own in turn.
template <bool MV>
__global__ __launch_bounds__(kBlock) void k_chunk_eval64(const Args a) {
    __shared__ double wmax[kBlock / 64];
    __shared__ int wcnt[kBlock / 64];
    __shared__ int lcount;
    __shared__ int64_t lidx[kList];
    __shared__ double lval[kList];
    __shared__ int cidx[kEvalCap];
    __shared__ double cval[kEvalCap];
    const int scan = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float thr = a.scans[scan].thr32;
    for (int it = blockIdx.x;; it += gridDim.x) {
        const int c = listed_chunk(a, scan, it);   // uniform
        if (c < 0) break;
        ChunkRec &rec = a.chunks[(int64_t)scan * a.nchunks + c];
        if (threadIdx.x == 0) lcount = 0;
        __syncthreads();
        double best = -INFINITY;
        if (rec.max32 >= thr) {   // uniform over the workgroup
            const ScanConst sc = scan_const(a.ss, scan);
            const float *img = a.img + (int64_t)scan * a.nvox;
            int count = 0;        // uniform
            for (int k = 0; k < a.per_thread; ++k) {
                const int off = k * kBlock + threadIdx.x;
                const int64_t v = chunk_voxel(a, c, off);
                const bool cand = v >= 0 && img[v] >= thr;
                const unsigned long long mask = __ballot(cand);
                if (lane == 0) wcnt[wave] = __popcll(mask);
                __syncthreads();
                int slot = count + __popcll(mask & ((1ull << lane) - 1));
                for (int w = 0; w < wave; ++w) slot += wcnt[w];
                if (cand && slot < kEvalCap) cidx[slot] = off;
                for (int w = 0; w < kBlock / 64; ++w) count += wcnt[w];
                __syncthreads();   // wcnt read by every lane before the next round writes it
            }
            if (count <= kEvalCap) {
                for (int i = wave; i < count; i += kBlock / 64) {   // uniform per wavefront
                    const int64_t vv = chunk_voxel(a, c, cidx[i]);
                    double rx, ry, rz;
                    voxel_pos(a.g, vv, rx, ry, rz);
                    const double e = energy64_bf<MV>(a.bf, sc, a.ss.n_ant, a.ss.n_samp, a.window, rx, ry, rz, lane, 64);
                    best = fmax(best, e);
                    if (lane == 0) cval[i] = e;
                }
                __syncthreads();
                if (threadIdx.x == 0) {   // the first kList candidates in index order
                    lcount = count;
                    for (int i = 0; i < count && i < kList; ++i) {
                        lidx[i] = chunk_voxel(a, c, cidx[i]);
                        lval[i] = cval[i];
                    }
                }
            } else {
                for (int k = 0; k < a.per_thread; ++k) {
                    const int64_t v = chunk_voxel(a, c, k * kBlock + threadIdx.x);
                    const bool cand = v >= 0 && img[v] >= thr;
                    unsigned long long mask = __ballot(cand);
                    while (mask) {
                        const int l = __builtin_ctzll(mask);
                        mask &= mask - 1;
                        const int64_t vv = chunk_voxel(a, c, k * kBlock + wave * 64 + l);
                        double rx, ry, rz;
                        voxel_pos(a.g, vv, rx, ry, rz);
                        const double e =
                            energy64_bf<MV>(a.bf, sc, a.ss.n_ant, a.ss.n_samp, a.window, rx, ry, rz, lane, 64);
                        best = fmax(best, e);
                        if (lane == 0) {
                            const int slot = atomicAdd(&lcount, 1);
                            if (slot < kList) { lidx[slot] = vv; lval[slot] = e; }
                        }
                    }
                }
            }
        }
        if (lane == 0) wmax[wave] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = wmax[0];
            for (int i = 1; i < kBlock / 64; ++i) m = fmax(m, wmax[i]);
            rec.max64 = m;
            rec.count = lcount;
            const int n = lcount < kList ? lcount : kList;
            for (int i = 0; i < n; ++i) { rec.idx[i] = lidx[i]; rec.val[i] = lval[i]; }
        }
        __syncthreads();   // the shared lists are free for the next chunk
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce64(const Args a) {
    __shared__ double red[kBlock / 64];
    const int scan = blockIdx.x;
    double m = -INFINITY;
    const float thr32 = a.scans[scan].thr32;
    for (int c = threadIdx.x; c < a.nchunks; c += kBlock) {
        const ChunkRec &r = a.chunks[(int64_t)scan * a.nchunks + c];
        if (r.max32 >= thr32) m = fmax(m, r.max64);   // stage C wrote the chunks that reach thr32
    }
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0];
        for (int i = 1; i < kBlock / 64; ++i) r = fmax(r, red[i]);
        a.scans[scan].max64 = r;
        a.scans[scan].thr64 = r - kTieRel * fabs(r);
    }
}

// Stage E: lowest index within the FP64 tie band, per chunk.
template <bool MV>
__global__ __launch_bounds__(kBlock) void k_chunk_select(const Args a) {
    __shared__ long long wbest[kBlock / 64];
    __shared__ double wval[kBlock / 64];
    const int scan = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double thr64 = a.scans[scan].thr64;
    const float thr32 = a.scans[scan].thr32;
    for (int it = blockIdx.x;; it += gridDim.x) {
        const int c = listed_chunk(a, scan, it);   // uniform
        if (c < 0) break;
        ChunkRec &rec = a.chunks[(int64_t)scan * a.nchunks + c];
        if (rec.max32 < thr32) continue;           // not evaluated by stage C (list overflow only)
        long long best = LLONG_MAX;
        double bval = 0.0;
        if (rec.count > 0 && rec.max64 >= thr64) {
            if (rec.count <= kList) {
                if (threadIdx.x == 0) {
                    for (int i = 0; i < rec.count; ++i)
                        if (rec.val[i] >= thr64 && rec.idx[i] < best) { best = rec.idx[i]; bval = rec.val[i]; }
                }
            } else {
                const ScanConst sc = scan_const(a.ss, scan);
                const float *img = a.img + (int64_t)scan * a.nvox;
                for (int k = 0; k < a.per_thread; ++k) {
                    const int64_t v = chunk_voxel(a, c, k * kBlock + threadIdx.x);
                    const bool cand = v >= 0 && img[v] >= thr32;
                    unsigned long long mask = __ballot(cand);
                    while (mask) {
                        const int l = __builtin_ctzll(mask);
                        mask &= mask - 1;
                        const int64_t vv = chunk_voxel(a, c, k * kBlock + wave * 64 + l);
                        if (vv >= best) continue;     // wave-uniform: indices only grow within a wave
                        double rx, ry, rz;
                        voxel_pos(a.g, vv, rx, ry, rz);
                        const double e =
                            energy64_bf<MV>(a.bf, sc, a.ss.n_ant, a.ss.n_samp, a.window, rx, ry, rz, lane, 64);
                        if (e >= thr64) { best = vv; bval = e; }
                    }
                }
            }
        }
        if (lane == 0) { wbest[wave] = best; wval[wave] = bval; }
        __syncthreads();
        if (threadIdx.x == 0) {
            long long b = wbest[0];
            double bv = wval[0];
            for (int i = 1; i < kBlock / 64; ++i)
                if (wbest[i] < b) { b = wbest[i]; bv = wval[i]; }
            rec.best_idx = b;
            rec.best_val = bv;
        }
        __syncthreads();   // wbest / wval are free for the next chunk
    }
}

__global__ __launch_bounds__(kBlock) void k_final(const Args a) {
    __shared__ long long sb[kBlock / 64];
    __shared__ double sv[kBlock / 64];
    __shared__ int sn[kBlock / 64];
    const int scan = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    long long b = LLONG_MAX;
    double bv = 0.0;
    int n = 0;
    for (int c = threadIdx.x; c < a.nchunks; c += kBlock) {
        const ChunkRec &r = a.chunks[(int64_t)scan * a.nchunks + c];
        n += r.max32 >= a.scans[scan].thr32 ? r.count : 0;
        if (r.max32 >= a.scans[scan].thr32 && r.count > 0 && r.max64 >= a.scans[scan].thr64 && r.best_idx < b) {
            b = r.best_idx;
            bv = r.best_val;
        }
    }
    // lowest index over the workgroup, with its value (indices are distinct across chunks)
    const long long wb = wave_min_ll(b);
    const unsigned long long owner = __ballot(b == wb && wb != LLONG_MAX);
    const double wv = owner ? __shfl(bv, __builtin_ctzll(owner), 64) : 0.0;
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    if (lane == 0) { sb[wave] = wb; sv[wave] = wv; sn[wave] = n; }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long best = LLONG_MAX;
        double val = 0.0;
        int cnt = 0;
        for (int i = 0; i < kBlock / 64; ++i) {
            cnt += sn[i];
            if (sb[i] < best) { best = sb[i]; val = sv[i]; }
        }
        uwb_peak p;
        if (best == LLONG_MAX) {   // no finite candidate (e.g. a NaN image)
            p.index = 0;
            p.value = __builtin_nan("");
            p.value32 = a.img[(int64_t)scan * a.nvox];
        } else {
            p.index = best;
            p.value = val;
            p.value32 = a.img[(int64_t)scan * a.nvox + best];
        }
        p.candidates = cnt;
        a.out[scan] = p;
    }
}

}  // namespace

// Chunks per scan: 4096-voxel runs, or (tile mode) the tiles of the full-resolution DAS / DMAS launch.
static int64_t chunk_count(const GridView &g, bool tiles, int *tx = nullptr, int *ty = nullptr, int *tz = nullptr,
                           int *tiles_x = nullptr, int *tiles_y = nullptr) {
    if (!tiles) return ((int64_t)g.dims[0] * g.dims[1] * g.dims[2] + kChunkVox - 1) / kChunkVox;
    int x, y, z;
    full_tile_shape(g.dims[2] > 1, &x, &y, &z);
    const int64_t nx = (g.dims[0] + x - 1) / x, ny = (g.dims[1] + y - 1) / y, nz = (g.dims[2] + z - 1) / z;
    if (tx) { *tx = x; *ty = y; *tz = z; *tiles_x = (int)nx; *tiles_y = (int)ny; }
    return nx * ny * nz;
}

size_t argmax_ws_bytes(const GridView &g, int n_scans, bool tiles) {
    const int64_t nchunks = chunk_count(g, tiles);
    return (size_t)n_scans * ((size_t)nchunks * sizeof(ChunkRec) + sizeof(ScanRec) + (1 + kChunkCap) * sizeof(int)) +
           256;
}

int64_t full_tile_count(const GridView &g) { return chunk_count(g, true); }

int launch_argmax(int bf, const ScanSet &ss, int n_scans, const GridView &g, int window, const float *img,
                  uwb_peak *out, void *ws, hipStream_t st, const float *tmax) {
    Args a;
    a.ss = ss;
    a.g = g;
    a.window = window;
    a.bf = bf;
    a.img = img;
    a.nvox = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    a.tmax = tmax;
    a.tx = a.ty = a.tz = a.tiles_x = a.tiles_y = 1;
    const int64_t nchunks = chunk_count(g, tmax != nullptr, &a.tx, &a.ty, &a.tz, &a.tiles_x, &a.tiles_y);
    if (nchunks > 0x7fffffff || n_scans > 65535) return UWB_EUNSUPPORTED;
    a.nchunks = (int)nchunks;
    a.per_thread = tmax ? a.tx * a.ty * a.tz / kBlock : kPerThread;
    if (tmax && a.per_thread * kBlock != a.tx * a.ty * a.tz) return UWB_EUNSUPPORTED;
    uintptr_t p = ((uintptr_t)ws + 255) & ~(uintptr_t)255;
    a.chunks = reinterpret_cast<ChunkRec *>(p);
    p += (size_t)n_scans * nchunks * sizeof(ChunkRec);
    a.scans = reinterpret_cast<ScanRec *>(p);
    p += (size_t)n_scans * sizeof(ScanRec);
    a.clist = reinterpret_cast<int *>(p);
    a.out = out;
    const dim3 gc((unsigned)nchunks, (unsigned)n_scans), gl((unsigned)kChunkCap, (unsigned)n_scans),
        gs((unsigned)n_scans);
    if (!tmax) hipLaunchKernelGGL(k_chunk_max32, gc, dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_reduce32, gs, dim3(kBlock), 0, st, a);
    if (bf == UWB_MVDR) hipLaunchKernelGGL(k_chunk_eval64<true>, gl, dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL(k_chunk_eval64<false>, gl, dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_reduce64, gs, dim3(kBlock), 0, st, a);
    if (bf == UWB_MVDR) hipLaunchKernelGGL(k_chunk_select<true>, gl, dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL(k_chunk_select<false>, gl, dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_final, gs, dim3(kBlock), 0, st, a);
    return hipGetLastError() == hipSuccess ? UWB_OK : UWB_EHIP;
}

// Scratch of the allocation-free detection (uwb_argmax_batch_noalloc): the chunk and scan records of
// stages A-F, in a device array that every GPU the library runs on holds once, until the process ends.
// Every record is written by the stage that produces it before a later stage reads it, so nothing has to
// start at zero.  Host code never passes the array's name to a kernel (on the host it stands for a
// host-side shadow, not a device address): it takes each device's address once from
// hipGetSymbolAddress and hands that pointer to the kernels like any workspace.
namespace {
static __device__ __align__(256) unsigned char scratch[UWB_ARGMAX_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
}  // namespace

int argmax_scratch(void **ptr) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return UWB_EHIP;
    if (dev >= kMaxDevices) return UWB_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return UWB_EHIP;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return UWB_OK;
}

}  // namespace uwb
