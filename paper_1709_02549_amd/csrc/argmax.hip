// Detection by maximal synthesized energy (Section II-A), decided in FP64.
//
// The FP32 image locates the candidates; the decision is re-taken in FP64 so it
// does not depend on FP32 rounding.  Pipeline per scan (stream-ordered, no host
// synchronisation, no floating-point atomics, deterministic):
//   A  per 4096-voxel chunk: FP32 maximum                         -> cmax32[c]
//   B  one workgroup: thr32 = max32 - kCandRel |max32|
//   C  per chunk: every voxel with I32 >= thr32 is re-evaluated in FP64 by a whole
//      wave (antennas split over the 64 lanes, the chunk's four waves taking the
//      candidates in turn); chunk maximum and a short list of (index, value)
//                                                                 -> cmax64[c], list
//   D  one workgroup: thr64 = max64 - 1e-12 |max64|
//   E  per chunk: lowest index among candidates with FP64 value >= thr64 (from the
//      list, or re-evaluated when the chunk had more candidates than the list holds)
//   F  one workgroup: lowest index over chunks -> uwb_peak
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
    ChunkRec *chunks;       // [scan][nchunks]
    ScanRec *scans;         // [scan]
    uwb_peak *out;
};

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
    const int scan = blockIdx.x;
    float m = -INFINITY;
    for (int c = threadIdx.x; c < a.nchunks; c += kBlock) m = fmaxf(m, a.chunks[(int64_t)scan * a.nchunks + c].max32);
    m = block_maxf(m, red);
    if (threadIdx.x == 0) {
        a.scans[scan].max32 = m;
        a.scans[scan].thr32 = m - (float)kCandRel * fabsf(m);
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
    const int scan = blockIdx.y, c = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    ChunkRec &rec = a.chunks[(int64_t)scan * a.nchunks + c];
    const float thr = a.scans[scan].thr32;
    const int64_t c0 = (int64_t)c * kChunkVox;
    if (threadIdx.x == 0) lcount = 0;
    __syncthreads();
    double best = -INFINITY;
    if (rec.max32 >= thr) {   // uniform over the workgroup
        const ScanConst sc = scan_const(a.ss, scan);
        const float *img = a.img + (int64_t)scan * a.nvox;
        int count = 0;        // uniform
        for (int k = 0; k < kPerThread; ++k) {
            const int off = k * kBlock + threadIdx.x;
            const bool cand = c0 + off < a.nvox && img[c0 + off] >= thr;
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
                const int64_t vv = c0 + cidx[i];
                double rx, ry, rz;
                voxel_pos(a.g, vv, rx, ry, rz);
                const double e = energy64_bf<MV>(a.bf, sc, a.ss.n_ant, a.ss.n_samp, a.window, rx, ry, rz, lane, 64);
                best = fmax(best, e);
                if (lane == 0) cval[i] = e;
            }
            __syncthreads();
            if (threadIdx.x == 0) {   // the first kList candidates in index order
                lcount = count;
                for (int i = 0; i < count && i < kList; ++i) { lidx[i] = c0 + cidx[i]; lval[i] = cval[i]; }
            }
        } else {
            for (int k = 0; k < kPerThread; ++k) {
                const int64_t v = c0 + k * kBlock + threadIdx.x;
                const bool cand = v < a.nvox && img[v] >= thr;
                unsigned long long mask = __ballot(cand);
                while (mask) {
                    const int l = __builtin_ctzll(mask);
                    mask &= mask - 1;
                    const int64_t vv = c0 + k * kBlock + wave * 64 + l;
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
}

__global__ __launch_bounds__(kBlock) void k_reduce64(const Args a) {
    __shared__ double red[kBlock / 64];
    const int scan = blockIdx.x;
    double m = -INFINITY;
    for (int c = threadIdx.x; c < a.nchunks; c += kBlock) m = fmax(m, a.chunks[(int64_t)scan * a.nchunks + c].max64);
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
    const int scan = blockIdx.y, c = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    ChunkRec &rec = a.chunks[(int64_t)scan * a.nchunks + c];
    const double thr64 = a.scans[scan].thr64;
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
            const float thr = a.scans[scan].thr32;
            for (int k = 0; k < kPerThread; ++k) {
                const int64_t v = (int64_t)c * kChunkVox + k * kBlock + threadIdx.x;
                const bool cand = v < a.nvox && img[v] >= thr;
                unsigned long long mask = __ballot(cand);
                while (mask) {
                    const int l = __builtin_ctzll(mask);
                    mask &= mask - 1;
                    const int64_t vv = (int64_t)c * kChunkVox + k * kBlock + wave * 64 + l;
                    if (vv >= best) continue;     // wave-uniform: indices only grow within a wave
                    double rx, ry, rz;
                    voxel_pos(a.g, vv, rx, ry, rz);
                    const double e = energy64_bf<MV>(a.bf, sc, a.ss.n_ant, a.ss.n_samp, a.window, rx, ry, rz, lane, 64);
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

size_t argmax_ws_bytes(const GridView &g, int n_scans) {
    const int64_t nvox = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    const int64_t nchunks = (nvox + kChunkVox - 1) / kChunkVox;
    return (size_t)n_scans * ((size_t)nchunks * sizeof(ChunkRec) + sizeof(ScanRec)) + 256;
}

int launch_argmax(int bf, const ScanSet &ss, int n_scans, const GridView &g, int window, const float *img,
                  uwb_peak *out, void *ws, hipStream_t st) {
    Args a;
    a.ss = ss;
    a.g = g;
    a.window = window;
    a.bf = bf;
    a.img = img;
    a.nvox = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    const int64_t nchunks = (a.nvox + kChunkVox - 1) / kChunkVox;
    if (nchunks > 0x7fffffff || n_scans > 65535) return UWB_EUNSUPPORTED;
    a.nchunks = (int)nchunks;
    uintptr_t p = ((uintptr_t)ws + 255) & ~(uintptr_t)255;
    a.chunks = reinterpret_cast<ChunkRec *>(p);
    a.scans = reinterpret_cast<ScanRec *>(p + (size_t)n_scans * nchunks * sizeof(ChunkRec));
    a.out = out;
    const dim3 gc((unsigned)nchunks, (unsigned)n_scans), gs((unsigned)n_scans);
    hipLaunchKernelGGL(k_chunk_max32, gc, dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_reduce32, gs, dim3(kBlock), 0, st, a);
    if (bf == UWB_MVDR) hipLaunchKernelGGL(k_chunk_eval64<true>, gc, dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL(k_chunk_eval64<false>, gc, dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_reduce64, gs, dim3(kBlock), 0, st, a);
    if (bf == UWB_MVDR) hipLaunchKernelGGL(k_chunk_select<true>, gc, dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL(k_chunk_select<false>, gc, dim3(kBlock), 0, st, a);
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
