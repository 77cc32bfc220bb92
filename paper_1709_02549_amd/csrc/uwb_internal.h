// Internal definitions shared by the HIP sources of libuwb (device-side views,
// launch helpers).  Not part of the public ABI.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/uwb.h"

namespace uwb {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kMaxWindow = UWB_MAX_WINDOW;
constexpr double kTieRel = 1e-12;    // relative band of the maximum-selection rule
constexpr double kCandRel = 1e-3;    // FP32 candidates for the FP64 argmax re-evaluation
constexpr int kMaxMultistaticAnt = 256;   // antennas of a multistatic scan (M^2 channels)

// A set of same-shaped scans in device memory.  Scan s uses
//   ant_pos + s*pos_stride, traces + s*tr_stride, and (dt, t0, v) either from
//   params[3*s..] (device) or, when params == nullptr, from the inline values.
// n_ant counts channels.  Monostatic (ms == 0): channel i is antenna i.
// Multistatic (ms == M > 0): M antennas, n_ant = M^2 channels, channel i*M + j
// transmits from antenna i and receives on antenna j (Eq. (2)).
struct ScanSet {
    const float *ant_pos;
    const float *traces;
    const double *params;
    int64_t pos_stride, tr_stride;
    int32_t n_ant, n_samp;
    int32_t ms;
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
    int ms;       // multistatic: antennas per side (0: monostatic)
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
    c.ms = ss.ms;
    return c;
}

// BF16 <-> FP32 (BF16 stored as its 16-bit pattern).
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);   // NaN
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

// Wave-level reductions (wave64).
// Wave-wide FP64 sum and maximum, the same value in every lane: a butterfly whose
// first four stages stay inside rows of 16 lanes and run as data-parallel-primitive
// moves (lanes paired at distance 1 and 2 by quad permutations, then quads by the
// half-row mirror and half-rows by the row mirror) instead of LDS-crossbar permutations;
// the last two stages pair rows 16 and 32 lanes apart.  Every stage adds two values
// that are the same in both lanes of a pair, so all lanes hold the same bits throughout,
// which are those of the xor butterfly over 1, 2, 4, 8, 16, 32.
template <int CTRL>
__device__ __forceinline__ double dpp_row64(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror: lane i <-> 7 - i within each 8
constexpr int kDppMirror = 0x140;      // row_mirror: lane i <-> 15 - i within each row
// One stage of a butterfly over aligned groups of lanes that starts at distance 1: the
// value of the partner o lanes away (lane ^ o).  For o < 16 the partner sits in the same
// row, and once the previous stages have made every aligned group of o lanes agree, the
// quad permutations and the (half-)row mirrors pair the same values as the xor does, so
// those stages run as DPP moves; o >= 16 goes through the LDS crossbar.
template <int O>
__device__ __forceinline__ double bfly64(double x) {
    if constexpr (O == 1) return dpp_row64<kDppXor1>(x);
    else if constexpr (O == 2) return dpp_row64<kDppXor2>(x);
    else if constexpr (O == 4) return dpp_row64<kDppHalfMirror>(x);
    else if constexpr (O == 8) return dpp_row64<kDppMirror>(x);
    else return __shfl_xor(x, O, 64);
}
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_row64<kDppXor1>(x);
    x += dpp_row64<kDppXor2>(x);
    x += dpp_row64<kDppHalfMirror>(x);
    x += dpp_row64<kDppMirror>(x);
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
}
__device__ __forceinline__ double wave_max(double x) {
    x = fmax(x, dpp_row64<kDppXor1>(x));
    x = fmax(x, dpp_row64<kDppXor2>(x));
    x = fmax(x, dpp_row64<kDppHalfMirror>(x));
    x = fmax(x, dpp_row64<kDppMirror>(x));
    x = fmax(x, __shfl_xor(x, 16, 64));
    x = fmax(x, __shfl_xor(x, 32, 64));
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
// Staging of trace samples for the FP64 evaluations (walk, ROI, argmax guard).
// For a box of focal points, every antenna's samples that any point of the box
// can touch are copied once into LDS (zero outside the recorded trace); the
// per-point loops then gather from LDS instead of issuing dependent HBM loads.
// ------------------------------------------------------------------------------
constexpr int kStageMaxAnt = 1024;

struct Stage {
    float *buf;      // staged samples, antenna i at buf[off[i] .. off[i] + len[i])
    int *lo;         // first staged sample index of antenna i
    int *off;
    int *len;
    int cap;         // floats available in buf
};

// Exclusive prefix sum of one int per thread over the workgroup; returns the total.
__device__ __forceinline__ int block_exclusive_scan(int x, int *out, int *tmp /* [kBlock/64] */) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = x;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    __syncthreads();
    if (lane == 63) tmp[w] = inc;
    __syncthreads();
    int base = 0, total = 0;
    for (int k = 0; k < kBlock / 64; ++k) {
        if (k < w) base += tmp[k];
        total += tmp[k];
    }
    *out = base + inc - x;
    return total;
}

// Stage the samples a box of focal points [blo, bhi] (inclusive finest indices) can
// touch.  Returns false (uniformly) when they do not fit; the caller then reads HBM.
__device__ bool stage_box(const Stage &st, int *tmp, const ScanConst &sc, int M, int T, int window,
                          const GridView &g, const int *blo, const int *bhi) {
    if (M > kStageMaxAnt || sc.ms) return false;   // monostatic spans only
    const int h = (window - 1) / 2;
    const int tid = threadIdx.x;
    for (int i = tid; i < M; i += kBlock) {
        double dn2 = 0.0, df2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double a = (double)sc.pos[3 * i + d];
            const double l = g.origin[d] + blo[d] * g.pitch[d] - a;
            const double u = g.origin[d] + bhi[d] * g.pitch[d] - a;
            const double n = fmin(fmax(0.0, l), u);
            const double f = fmax(fabs(l), fabs(u));
            dn2 += n * n;
            df2 += f * f;
        }
        const double tmin = sc.s * sqrt(dn2) - sc.t0s, tmax = sc.s * sqrt(df2) - sc.t0s;
        double lo = fmin(fmax(floor(tmin) - h - 1, -(double)(window + 1)), (double)T);
        double hi = fmin(fmax(floor(tmax) + h + 2, lo + window), (double)(T + window));
        st.lo[i] = (int)lo;
        st.len[i] = (int)(hi - lo) + 1;
    }
    __syncthreads();
    // prefix sum of the lengths: thread t owns antennas [t*c, (t+1)*c)
    const int c = (M + kBlock - 1) / kBlock;
    int mine = 0;
    for (int i = tid * c; i < min(M, (tid + 1) * c); ++i) mine += st.len[i];
    int base;
    const int total = block_exclusive_scan(mine, &base, tmp);
    if (total > st.cap) return false;
    for (int i = tid * c; i < min(M, (tid + 1) * c); ++i) {
        st.off[i] = base;
        base += st.len[i];
    }
    __syncthreads();
    const int lane = tid & 63;
    for (int i = tid >> 6; i < M; i += kBlock / 64) {
        const float *tr = sc.tr + (int64_t)i * T;
        const int l0 = st.lo[i], n = st.len[i], o = st.off[i];
        for (int m = lane; m < n; m += 64) {
            const int gi = l0 + m;
            st.buf[o + m] = (gi >= 0 && gi < T) ? tr[gi] : 0.f;
        }
    }
    __syncthreads();
    return true;
}

// ------------------------------------------------------------------------------
// Capon / MVDR energy of one focal point from its window statistics (header: the
// beamformer's definition).  gram: the packed lower triangle of G = X^T X,
// entry (k, l <= k) at k (k + 1) / 2 + l; b: X^T 1; M: channels.  Through the
// Woodbury identity, R_l^-1 1 = (1/delta) (1 - X c) with c = A^-1 b and
// A = G + W delta I, so the output samples are y = W delta c / (M - b^T c).  The
// statistics are first divided by tr = trace(G) = |X|^2 (the energy scales as
// |X|^2), which leaves A' = G / tr + (loading / M) I, whose eigenvalues lie in
// [loading / M, 1 + loading / M]: the system is well conditioned at any signal
// level.  Cholesky A' = L L^T (in place), L z = b / sqrt(tr), L^T c = z; then
// b^T c = |z|^2 and I = tr (loading / M)^2 |c|^2 / (M - |z|^2)^2.
// tr = 0 (no signal) gives 0; a non-finite tr gives NaN.
// ------------------------------------------------------------------------------
constexpr int tri(int k, int l) { return k * (k + 1) / 2 + l; }

template <typename Real, int W>
__device__ __forceinline__ Real mvdr_energy(Real (&gram)[W * (W + 1) / 2], const Real (&b)[W], int M) {
    Real tr = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) tr += gram[tri(k, k)];
    if (!(tr > Real(0))) return tr == Real(0) ? Real(0) : static_cast<Real>(__builtin_nan(""));
    const Real inv = Real(1) / tr, load = Real(UWB_MVDR_LOADING) / Real(M);
#pragma unroll
    for (int q = 0; q < W * (W + 1) / 2; ++q) gram[q] *= inv;
#pragma unroll
    for (int k = 0; k < W; ++k) gram[tri(k, k)] += load;
    Real rd[W];   // 1 / L_jj
#pragma unroll
    for (int j = 0; j < W; ++j) {
        Real d = gram[tri(j, j)];
#pragma unroll
        for (int p = 0; p < j; ++p) d -= gram[tri(j, p)] * gram[tri(j, p)];
        const Real ljj = sqrt(d);
        gram[tri(j, j)] = ljj;
        rd[j] = Real(1) / ljj;
#pragma unroll
        for (int i = j + 1; i < W; ++i) {
            Real t = gram[tri(i, j)];
#pragma unroll
            for (int p = 0; p < j; ++p) t -= gram[tri(i, p)] * gram[tri(j, p)];
            gram[tri(i, j)] = t * rd[j];
        }
    }
    const Real sb = sqrt(inv);
    Real z[W], zz = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        Real t = b[i] * sb;
#pragma unroll
        for (int p = 0; p < i; ++p) t -= gram[tri(i, p)] * z[p];
        z[i] = t * rd[i];
        zz += z[i] * z[i];
    }
    Real c[W], cc = 0;
#pragma unroll
    for (int i = W - 1; i >= 0; --i) {
        Real t = z[i];
#pragma unroll
        for (int p = i + 1; p < W; ++p) t -= gram[tri(p, i)] * c[p];
        c[i] = t * rd[i];
        cc += c[i] * c[i];
    }
    const Real den = Real(M) - zz;
    return tr * load * load * cc / (den * den);
}

// ------------------------------------------------------------------------------
// FP64 energy of one focal point, evaluated cooperatively by a group of G lanes
// (G a power of two <= 64, lanes of one group contiguous in the wave).  Lane
// `gl` of the group takes antennas gl, gl+G, ...  The window is processed in
// register chunks of kChunk offsets, so any window up to kMaxWindow works with
// a fixed register budget.  Partial sums of the group are combined with
//   (S, P) (+) (S', P') = (S + S', P + P' + S S'),
// which is the exact decomposition of sum_{i<j} s_i s_j over two antenna sets.
// Samples come from a Stage (LDS) when `st` is non-null, else from HBM.
// Every lane of the group returns the energy.
// ------------------------------------------------------------------------------
constexpr int kChunk = 8;

// FP64 delay in samples of channel i at r: Eq. (1) (monostatic) or Eq. (2) (multistatic).
__device__ __forceinline__ double delay64(const ScanConst &sc, int i, double rx, double ry, double rz) {
    if (sc.ms) {
        const float *at = sc.pos + 3 * (i / sc.ms), *ar = sc.pos + 3 * (i % sc.ms);
        const double tx = rx - (double)at[0], ty = ry - (double)at[1], tz = rz - (double)at[2];
        const double ux = rx - (double)ar[0], uy = ry - (double)ar[1], uz = rz - (double)ar[2];
        return 0.5 * sc.s * (sqrt(tx * tx + ty * ty + tz * tz) + sqrt(ux * ux + uy * uy + uz * uz)) - sc.t0s;
    }
    const double dx = rx - (double)sc.pos[3 * i + 0];
    const double dy = ry - (double)sc.pos[3 * i + 1];
    const double dz = rz - (double)sc.pos[3 * i + 2];
    return sc.s * sqrt(dx * dx + dy * dy + dz * dz) - sc.t0s;
}

__device__ __forceinline__ double trace64(const float *tr, int T, long long m) {
    return (m >= 0 && m < T) ? (double)tr[m] : 0.0;
}

template <int BF>
__device__ double energy64_group(const ScanConst &sc, int M, int T, int window, double rx, double ry,
                                 double rz, int gl, int G, const Stage *st) {
    const int h = (window - 1) / 2;
    double energy = 0.0;
    for (int k0 = -h; k0 <= h; k0 += kChunk) {
        double S[kChunk], P[kChunk];
#pragma unroll
        for (int j = 0; j < kChunk; ++j) { S[j] = 0.0; P[j] = 0.0; }
        for (int i = gl; i < M; i += G) {
            const double tau = delay64(sc, i, rx, ry, rz);
            const double fl = floor(tau);
            const double f = tau - fl;
            if (st) {
                // window [n-h, n+h+1] lies inside the staged span by construction;
                // the clamp only guards non-finite inputs
                const int l0 = st->lo[i], ln = st->len[i];
                const double nc = fmin(fmax(fl, (double)(l0 + h)), (double)(l0 + ln - h - 2));
                const float *p = st->buf + st->off[i] + ((int)nc - l0);
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    const int k = k0 + j;
                    if (k <= h) {
                        const double y0 = (double)p[k];
                        const double y1 = (double)p[k + 1];
                        const double s = (1.0 - f) * y0 + f * y1;
                        if (BF == UWB_DMAS) P[j] += s * S[j];
                        S[j] += s;
                    }
                }
            } else {
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
        }
        // the group's butterfly over 1, 2, 4, ... < G: both lanes of a pair form the same sums
        auto stage = [&](auto oc) {
            constexpr int O = decltype(oc)::value;
            if (O < G) {   // uniform
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    const double So = bfly64<O>(S[j]);
                    if (BF == UWB_DMAS) {
                        const double Po = bfly64<O>(P[j]);
                        P[j] = P[j] + Po + S[j] * So;
                    }
                    S[j] += So;
                }
            }
        };
        stage(std::integral_constant<int, 1>{});
        stage(std::integral_constant<int, 2>{});
        stage(std::integral_constant<int, 4>{});
        stage(std::integral_constant<int, 8>{});
        stage(std::integral_constant<int, 16>{});
        stage(std::integral_constant<int, 32>{});
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

// The Capon / MVDR energy of one focal point in FP64 by a group of G lanes: every lane
// accumulates the window sums and the Gram matrix of its channels (gl, gl + G, ...), the
// group adds them up with a butterfly (each pair of lanes forms the same sums, so every
// lane ends with identical values), and every lane solves the W x W system.
template <int W>
__device__ double energy64_mvdr(const ScanConst &sc, int M, int T, double rx, double ry, double rz, int gl, int G,
                                const Stage *st) {
    constexpr int H = (W - 1) / 2, NG = W * (W + 1) / 2;
    double gram[NG], b[W];
#pragma unroll
    for (int q = 0; q < NG; ++q) gram[q] = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) b[k] = 0.0;
    for (int i = gl; i < M; i += G) {
        const double tau = delay64(sc, i, rx, ry, rz);
        const double fl = floor(tau);
        const double f = tau - fl;
        double y[W + 1];
        if (st) {
            // window [n-h, n+h+1] lies inside the staged span by construction; the clamp only
            // guards non-finite inputs
            const int l0 = st->lo[i], ln = st->len[i];
            const double nc = fmin(fmax(fl, (double)(l0 + H)), (double)(l0 + ln - H - 2));
            const float *p = st->buf + st->off[i] + ((int)nc - l0);
#pragma unroll
            for (int k = 0; k <= W; ++k) y[k] = (double)p[k - H];
        } else {
            const long long n = (long long)fmin(fmax(fl, -1.0e9), 1.0e9);
            const float *tr = sc.tr + (int64_t)i * T;
#pragma unroll
            for (int k = 0; k <= W; ++k) y[k] = trace64(tr, T, n + k - H);
        }
        double sv[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            sv[k] = (1.0 - f) * y[k] + f * y[k + 1];
            b[k] += sv[k];
        }
#pragma unroll
        for (int k = 0; k < W; ++k)
#pragma unroll
            for (int l = 0; l <= k; ++l) gram[tri(k, l)] += sv[k] * sv[l];
    }
    auto stage = [&](auto oc) {
        constexpr int O = decltype(oc)::value;
        if (O < G) {   // uniform
#pragma unroll
            for (int q = 0; q < NG; ++q) gram[q] += bfly64<O>(gram[q]);
#pragma unroll
            for (int k = 0; k < W; ++k) b[k] += bfly64<O>(b[k]);
        }
    };
    stage(std::integral_constant<int, 1>{});
    stage(std::integral_constant<int, 2>{});
    stage(std::integral_constant<int, 4>{});
    stage(std::integral_constant<int, 8>{});
    stage(std::integral_constant<int, 16>{});
    stage(std::integral_constant<int, 32>{});
    return mvdr_energy<double, W>(gram, b, M);
}

// DAS or DMAS.
__device__ __forceinline__ double energy64_dispatch(int bf, const ScanConst &sc, int M, int T, int window,
                                                    double rx, double ry, double rz, int gl, int G,
                                                    const Stage *st = nullptr) {
    return bf == UWB_DMAS ? energy64_group<UWB_DMAS>(sc, M, T, window, rx, ry, rz, gl, G, st)
                          : energy64_group<UWB_DAS>(sc, M, T, window, rx, ry, rz, gl, G, st);
}

// Any beamformer: MV selects the MVDR energy, whose W x W statistics take about 160 more VGPRs than
// DAS / DMAS, so the kernels that evaluate candidates are instantiated once for MVDR and once for the
// others, and the DAS / DMAS instantiation keeps its occupancy.
template <bool MV>
__device__ __forceinline__ double energy64_bf(int bf, const ScanConst &sc, int M, int T, int window, double rx,
                                             double ry, double rz, int gl, int G, const Stage *st = nullptr) {
    if constexpr (MV) {
        switch (window) {
            case 1: return energy64_mvdr<1>(sc, M, T, rx, ry, rz, gl, G, st);
            case 3: return energy64_mvdr<3>(sc, M, T, rx, ry, rz, gl, G, st);
            case 5: return energy64_mvdr<5>(sc, M, T, rx, ry, rz, gl, G, st);
            case 7: return energy64_mvdr<7>(sc, M, T, rx, ry, rz, gl, G, st);
            case 9: return energy64_mvdr<9>(sc, M, T, rx, ry, rz, gl, G, st);
            case 11: return energy64_mvdr<11>(sc, M, T, rx, ry, rz, gl, G, st);
        }
        return __builtin_nan("");   // rejected on the host
    } else {
        return energy64_dispatch(bf, sc, M, T, window, rx, ry, rz, gl, G, st);
    }
}

}  // namespace uwb

// Host-side launchers implemented in the .hip files.
namespace uwb {
// img_das (DMAS only, optional): the DAS images of the same scans, from the same launch.
// tmax, tmax_das (DAS / DMAS only, optional): each workgroup tile's FP32 maximum of img (and of img_das),
// [n_scans][full_tile_count(g)], for the detection's tile mode.
int launch_image32(int bf, const ScanSet &ss, int n_scans, const GridView &g, int window, float *img,
                   hipStream_t stream, float *img_das = nullptr, float *tmax = nullptr, float *tmax_das = nullptr);
// tmax (optional): the FP32 tile maxima the full-resolution DAS / DMAS launch wrote for img; the detection
// then skips its own pass over the image (tile mode, whose workspace is argmax_ws_bytes(g, n, true)).
int launch_argmax(int bf, const ScanSet &ss, int n_scans, const GridView &g, int window, const float *img,
                  uwb_peak *out, void *ws, hipStream_t stream, const float *tmax = nullptr);
size_t argmax_ws_bytes(const GridView &g, int n_scans, bool tiles = false);
// Tiles per scan of the full-resolution DAS / DMAS launch, and their shape.
int64_t full_tile_count(const GridView &g);
void full_tile_shape(bool d3, int *tx, int *ty, int *tz);
// This device's scratch of the allocation-free detection (UWB_ARGMAX_SCRATCH_BYTES bytes), its address
// taken once per device; UWB_EHIP if the runtime cannot give it.
int argmax_scratch(void **ptr);
}  // namespace uwb
