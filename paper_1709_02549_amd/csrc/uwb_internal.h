// Internal definitions shared by the HIP sources of libuwb (device-side views,
// launch helpers).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/uwb.h"

namespace uwb {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kMaxWindow = UWB_MAX_WINDOW;
constexpr double kTieRel = 1e-12;    // relative band of the maximum-selection rule
constexpr double kCandRel = 1e-3;    // FP32 candidates for the FP64 argmax re-evaluation

// A set of same-shaped scans in device memory.  Scan s uses
//   ant_pos + s*pos_stride, traces + s*tr_stride, and (dt, t0, v) either from
//   params[3*s..] (device) or, when params == nullptr, from the inline values.
struct ScanSet {
    const float *ant_pos;
    const float *traces;
    const double *params;
    int64_t pos_stride, tr_stride;
    int32_t n_ant, n_samp;
    double dt, t0, v;
};

struct GridView {
    double origin[3];
    double pitch[3];
    int32_t dims[3];
};

// Per-scan constants in sample units: tau = s * |r - a| - t0s.
struct ScanConst {
    const float *pos;
    const float *tr;
    double s;     // 2 / (v dt)
    double t0s;   // t0 / dt
};

__device__ __forceinline__ ScanConst scan_const(const ScanSet &ss, int scan) {
    ScanConst c;
    c.pos = ss.ant_pos + (int64_t)scan * ss.pos_stride;
    c.tr = ss.traces + (int64_t)scan * ss.tr_stride;
    double dt = ss.dt, t0 = ss.t0, v = ss.v;
    if (ss.params) {
        dt = ss.params[3 * scan + 0];
        t0 = ss.params[3 * scan + 1];
        v = ss.params[3 * scan + 2];
    }
    c.s = 2.0 / (v * dt);
    c.t0s = t0 / dt;
    return c;
}

// Wave-level reductions (wave64).
__device__ __forceinline__ double wave_sum(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ __forceinline__ double wave_max(double x) {
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
    return x;
}
__device__ __forceinline__ float wave_maxf(float x) {
    for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
    return x;
}
__device__ __forceinline__ long long wave_min_ll(long long x) {
    for (int o = 32; o > 0; o >>= 1) {
        long long y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    return x;
}

// ------------------------------------------------------------------------------
// FP64 energy of one focal point, evaluated cooperatively by a group of G lanes
// (G a power of two <= 64, lanes of one group contiguous in the wave).  Lane
// `gl` of the group takes antennas gl, gl+G, ...  The window is processed in
// register chunks of kChunk offsets, so any window up to kMaxWindow works with
// a fixed register budget.  Partial sums of the group are combined with
//   (S, P) (+) (S', P') = (S + S', P + P' + S S'),
// which is the exact decomposition of sum_{i<j} s_i s_j over two antenna sets.
// Every lane of the group returns the energy.
// ------------------------------------------------------------------------------
constexpr int kChunk = 8;

__device__ __forceinline__ double trace64(const float *tr, int T, long long m) {
    return (m >= 0 && m < T) ? (double)tr[m] : 0.0;
}

template <int BF>
__device__ double energy64_group(const ScanConst &sc, int M, int T, int window, double rx, double ry,
                                 double rz, int gl, int G) {
    const int h = (window - 1) / 2;
    double energy = 0.0;
    for (int k0 = -h; k0 <= h; k0 += kChunk) {
        double S[kChunk], P[kChunk];
#pragma unroll
        for (int j = 0; j < kChunk; ++j) { S[j] = 0.0; P[j] = 0.0; }
        for (int i = gl; i < M; i += G) {
            const double ax = (double)sc.pos[3 * i + 0];
            const double ay = (double)sc.pos[3 * i + 1];
            const double az = (double)sc.pos[3 * i + 2];
            const double dx = rx - ax, dy = ry - ay, dz = rz - az;
            const double tau = sc.s * sqrt(dx * dx + dy * dy + dz * dz) - sc.t0s;
            const double fl = floor(tau);
            const double f = tau - fl;
            // clamp keeps the index arithmetic finite for absurd inputs; such
            // positions are far outside the trace, where samples are zero anyway
            const double flc = fmin(fmax(fl, -1.0e9), 1.0e9);
            const long long n = (long long)flc;
            const float *tr = sc.tr + (int64_t)i * T;
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                const int k = k0 + j;
                if (k <= h) {
                    const double y0 = trace64(tr, T, n + k);
                    const double y1 = trace64(tr, T, n + k + 1);
                    const double s = (1.0 - f) * y0 + f * y1;
                    if (BF == UWB_DMAS) P[j] += s * S[j];
                    S[j] += s;
                }
            }
        }
        for (int o = 1; o < G; o <<= 1) {
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                const double So = __shfl_xor(S[j], o, 64);
                if (BF == UWB_DMAS) {
                    const double Po = __shfl_xor(P[j], o, 64);
                    P[j] = P[j] + Po + S[j] * So;
                }
                S[j] += So;
            }
        }
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            if (k0 + j <= h) {
                const double q = (BF == UWB_DMAS) ? P[j] : S[j];
                energy += q * q;
            }
        }
    }
    return energy;
}

__device__ __forceinline__ double energy64_dispatch(int bf, const ScanConst &sc, int M, int T, int window,
                                                    double rx, double ry, double rz, int gl, int G) {
    return bf == UWB_DMAS ? energy64_group<UWB_DMAS>(sc, M, T, window, rx, ry, rz, gl, G)
                          : energy64_group<UWB_DAS>(sc, M, T, window, rx, ry, rz, gl, G);
}

}  // namespace uwb

// Host-side launchers implemented in the .hip files.
namespace uwb {
int launch_image32(int bf, const ScanSet &ss, int n_scans, const GridView &g, int window, float *img,
                   hipStream_t stream);
int launch_argmax(int bf, const ScanSet &ss, int n_scans, const GridView &g, int window, const float *img,
                  uwb_peak *out, void *ws, hipStream_t stream);
size_t argmax_ws_bytes(const GridView &g, int n_scans);
}  // namespace uwb
