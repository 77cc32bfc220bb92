// LDS read-bandwidth probe: the on-chip resource that bounds the gather of the
// imaging kernels (each voxel-antenna reads W + 1 staged samples from LDS).
//
// Every workgroup (256 lanes) fills a 32 KiB LDS array (N elements of `width`
// bytes), then each lane streams `iters` (a multiple of 8) reads of `width` bytes
// (ds_read_b32 / _b64 / _b128).  A step issues eight reads, two groups of four: a
// group reads elements off + lane + 256 u (u = 0..3), so a wave's 64 reads fall on
// consecutive elements (no bank conflicts) and the four reads differ by immediate
// address offsets.  off = (step * stride) & (N/2 - 1) with stride a kernel argument
// (0 in the launches below): with compile-time addresses the compiler sees that the
// reads repeat and hoists them out of the loop.  Every index is at most
// N/2 - 1 + 3*256 + 255 < N, inside the array, whatever the stride.
// The values are folded into one integer per lane (three-input XORs, about two VALU
// instructions per 16-byte read, far below the read rate) and written out, so no
// read can be dropped.  The first lane records the shader-clock and the constant
// 100 MHz counters around its loop; the host derives the clock from them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "uwb_internal.h"

namespace uwb {
namespace {

constexpr int kProbeBytes = 32 * 1024;   // a power of two: five workgroups fit a CU's LDS

__device__ __forceinline__ unsigned fold(unsigned a, unsigned b) { return a ^ b; }
__device__ __forceinline__ unsigned fold(uint2 a, unsigned b) { return a.x ^ a.y ^ b; }
__device__ __forceinline__ unsigned fold(uint4 a, unsigned b) { return (a.x ^ a.y ^ a.z) ^ (a.w ^ b); }

template <int WIDTH>
__global__ __launch_bounds__(kBlock) void k_lds_read(int iters, int stride, unsigned *sink, long long *clk) {
    using V = typename std::conditional<WIDTH == 4, unsigned,
              typename std::conditional<WIDTH == 8, uint2, uint4>::type>::type;
    constexpr int N = kProbeBytes / WIDTH;          // elements of the array
    static_assert(N / 2 - 1 + 3 * kBlock + kBlock - 1 < N, "probe reads must stay inside the array");
    __shared__ V buf[N];
    for (int i = threadIdx.x; i < N; i += kBlock) {
        V v;
        unsigned *w = reinterpret_cast<unsigned *>(&v);
        for (int k = 0; k < WIDTH / 4; ++k) w[k] = (unsigned)(i * 7 + k);
        buf[i] = v;
    }
    __syncthreads();
    const long long c0 = clock64(), r0 = wall_clock64();
    unsigned acc = 0;
    for (int it = 0; it < iters; it += 8) {
        const V *p0 = buf + ((it * stride) & (N / 2 - 1)) + threadIdx.x;
        const V *p1 = buf + (((it + 4) * stride) & (N / 2 - 1)) + threadIdx.x;
        V v[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[u] = p0[u * kBlock];
            v[4 + u] = p1[u * kBlock];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fold(v[u], acc);
    }
    __syncthreads();
    const long long c1 = clock64(), r1 = wall_clock64();
    sink[(size_t)blockIdx.x * kBlock + threadIdx.x] = acc;
    if (threadIdx.x == 0) {
        clk[4 * blockIdx.x + 0] = c0;
        clk[4 * blockIdx.x + 1] = c1;
        clk[4 * blockIdx.x + 2] = r0;
        clk[4 * blockIdx.x + 3] = r1;
    }
}

}  // namespace
}  // namespace uwb

extern "C" int uwb_probe_lds_read(int32_t width, int32_t iters, int32_t n_groups, double *bytes_per_s,
                                  double *clock_hz, void *stream) {
    using namespace uwb;
    if (!bytes_per_s || !clock_hz || iters < 8 || iters % 8 || n_groups < 1 || n_groups > 65536) return UWB_EINVAL;
    if (width != 4 && width != 8 && width != 16) return UWB_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    unsigned *sink = nullptr;
    long long *clk = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = UWB_OK;
    if (hipMalloc(&sink, sizeof(unsigned) * (size_t)n_groups * kBlock) != hipSuccess ||
        hipMalloc(&clk, sizeof(long long) * 4 * (size_t)n_groups) != hipSuccess) {
        rc = UWB_ENOMEM;
    } else if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = UWB_EHIP;
    } else {
        auto launch = [&]() {
            const int stride = 0;   // runtime value: the reads cannot be hoisted (every stride stays in bounds)
            if (width == 4)
                hipLaunchKernelGGL(k_lds_read<4>, dim3(n_groups), dim3(kBlock), 0, st, iters, stride, sink, clk);
            else if (width == 8)
                hipLaunchKernelGGL(k_lds_read<8>, dim3(n_groups), dim3(kBlock), 0, st, iters, stride, sink, clk);
            else
                hipLaunchKernelGGL(k_lds_read<16>, dim3(n_groups), dim3(kBlock), 0, st, iters, stride, sink, clk);
        };
        launch();   // warm-up
        hipEventRecord(e0, st);
        launch();
        hipEventRecord(e1, st);
        float ms = 0.f;
        std::vector<long long> h(4 * (size_t)n_groups);
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
            hipMemcpy(h.data(), clk, h.size() * sizeof(long long), hipMemcpyDeviceToHost) != hipSuccess) {
            rc = UWB_EHIP;
        } else {
            *bytes_per_s = (double)n_groups * kBlock * (double)iters * width / (ms * 1e-3);
            std::vector<double> f;
            for (int g = 0; g < n_groups; ++g) {
                const double dc = (double)(h[4 * g + 1] - h[4 * g]), dr = (double)(h[4 * g + 3] - h[4 * g + 2]);
                if (dr > 0) f.push_back(dc / dr * 100e6);   // wall_clock64 ticks at 100 MHz
            }
            std::sort(f.begin(), f.end());
            *clock_hz = f.empty() ? 0.0 : f[f.size() / 2];
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (sink) hipFree(sink);
    if (clk) hipFree(clk);
    return rc;
}
