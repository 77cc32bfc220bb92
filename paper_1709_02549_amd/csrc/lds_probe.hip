// LDS read-bandwidth probe: the on-chip resource that bounds the gather of the
// imaging kernels (each voxel-antenna reads W + 1 staged samples from LDS).
//
// Every workgroup (256 lanes) fills a 64 KiB LDS array, then each lane streams
// `iters` (a multiple of 8) reads of `width` bytes (ds_read_b32 / _b64 / _b128) at addresses that
// walk the array with a stride of one read per lane, so a wave's 64 reads fall
// on consecutive dwords (no bank conflicts) and every read is inside the array.
// The values are folded into one integer per lane and written out, so no read
// can be dropped.  The first lane records the shader-clock and the constant
// 100 MHz counters around its loop; the host derives the clock from them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "uwb_internal.h"

namespace uwb {
namespace {

constexpr int kProbeBytes = 32 * 1024;   // a power of two: five workgroups fit a CU's LDS

template <int WIDTH>
__global__ __launch_bounds__(kBlock) void k_lds_read(int iters, unsigned *sink, long long *clk) {
    using V = typename std::conditional<WIDTH == 4, unsigned,
              typename std::conditional<WIDTH == 8, uint2, uint4>::type>::type;
    constexpr int N = kProbeBytes / WIDTH;          // elements of the array
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
    // eight independent reads in flight per lane per step; the addresses depend on the loop counter only
    for (int it = 0; it < iters; it += 8) {
        V v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = buf[(threadIdx.x + (it + u) * kBlock) & (N - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const unsigned *w = reinterpret_cast<const unsigned *>(&v[u]);
#pragma unroll
            for (int k = 0; k < WIDTH / 4; ++k) acc ^= w[k];
        }
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
            if (width == 4) hipLaunchKernelGGL(k_lds_read<4>, dim3(n_groups), dim3(kBlock), 0, st, iters, sink, clk);
            else if (width == 8) hipLaunchKernelGGL(k_lds_read<8>, dim3(n_groups), dim3(kBlock), 0, st, iters, sink, clk);
            else hipLaunchKernelGGL(k_lds_read<16>, dim3(n_groups), dim3(kBlock), 0, st, iters, sink, clk);
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
