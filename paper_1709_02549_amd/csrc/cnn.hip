// Learned segment proposer: a small CNN scoring the four children of a quadtree
// box from the box's 32 x 32 coarse DAS energy image (normalised by its maximum).
//
//   conv3x3(1->32, s1) ReLU -> 3 x [conv3x3(32->32, s2) ReLU]  (32 -> 16 -> 8 -> 4)
//   child c = bx + 2 by: mean of the 2 x 2 cells of quadrant (bx, by) -> 32 features
//   shared linear 32 -> 1 -> 4 logits -> softmax
//
// Weights and activations are stored in BF16, every product is accumulated in
// FP32; gradients, Adam moments and the master weights are FP32.  Tensors are
// NCHW.  All reductions run in a fixed order (no floating-point atomics), so a
// training run is bitwise reproducible.
//
// Kernels: forward convolution (+bias, ReLU, BF16 store); readout forward and
// backward with softmax cross-entropy; backward-data convolution fused with the
// ReLU derivative of its input; backward-weight convolution (one workgroup per
// (output channel, input channel), 9 taps, block reduction); Adam.
#include <cmath>
#include <cstring>
#include <vector>

#include "uwb_internal.h"

namespace uwb {
namespace {

constexpr int C = 32;          // channels of every hidden layer
constexpr int IN = 32;         // input side
constexpr int NPARAM = 28097;  // 288 + 3*9216 + 4*32 + 32 + 1

// offsets of each tensor in the flat parameter vector (the oracle's order:
// conv weights 1..4, conv biases 1..4, readout weight, readout bias)
constexpr int OFF_W[4] = {0, 288, 288 + 9216, 288 + 2 * 9216};
constexpr int OFF_B = 288 + 3 * 9216;          // 27936
constexpr int OFF_WL = OFF_B + 4 * C;          // 28064
constexpr int OFF_BL = OFF_WL + C;             // 28096


// ------------------------------------------------------------------------------
// forward convolution: X [N][CIN][HIN][HIN] bf16 -> Y [N][32][HO][HO] bf16 (ReLU)
// Workgroup: one sample, RB output rows; lane: one output pixel, 16 channels.
// ------------------------------------------------------------------------------
template <int CIN, int HIN, int S, int RB>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t *__restrict__ X, const uint16_t *__restrict__ Wb,
                                                 const uint16_t *__restrict__ Bb, uint16_t *__restrict__ Y) {
    constexpr int HO = HIN / S;
    constexpr int NR = S * (RB - 1) + 3;     // input rows needed (with padding)
    constexpr int WP = HIN + 2;
    constexpr int PIX = RB * HO;             // output pixels per workgroup
    constexpr int GROUPS = 256 / PIX;        // channel groups
    constexpr int CPG = C / GROUPS;          // channels per lane
    static_assert(PIX * GROUPS == 256 && CPG * GROUPS == C, "tile shape");
    __shared__ float w[CIN * 9][C];          // [ci*9 + k][co]
    __shared__ uint16_t xin[CIN][NR][WP];
    const int n = blockIdx.y, r0 = blockIdx.x * RB, tid = threadIdx.x;
    for (int e = tid; e < CIN * 9 * C; e += 256) {
        const int co = e / (CIN * 9), r = e % (CIN * 9);
        w[r][co] = bf2f(Wb[e]);
    }
    const uint16_t *xs = X + (size_t)n * CIN * HIN * HIN;
    for (int e = tid; e < CIN * NR * WP; e += 256) {
        const int ci = e / (NR * WP), rr = (e / WP) % NR, cc = e % WP;
        const int yi = S * r0 - 1 + rr, xi = cc - 1;
        xin[ci][rr][cc] = (yi >= 0 && yi < HIN && xi >= 0 && xi < HIN) ? xs[(ci * HIN + yi) * HIN + xi] : (uint16_t)0;
    }
    __syncthreads();
    const int p = tid % PIX, g = tid / PIX;
    const int oy = p / HO, ox = p % HO;
    float acc[CPG];
#pragma unroll
    for (int j = 0; j < CPG; ++j) acc[j] = bf2f(Bb[g * CPG + j]);
    for (int ci = 0; ci < CIN; ++ci) {
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const float xv = bf2f(xin[ci][S * oy + ky][S * ox + kx]);
                const float *wr = &w[ci * 9 + ky * 3 + kx][g * CPG];
#pragma unroll
                for (int j = 0; j < CPG; ++j) acc[j] = fmaf(wr[j], xv, acc[j]);
            }
    }
    uint16_t *ys = Y + (size_t)n * C * HO * HO;
    if (r0 + oy < HO) {
#pragma unroll
        for (int j = 0; j < CPG; ++j) ys[((g * CPG + j) * HO + r0 + oy) * HO + ox] = f2bf(fmaxf(acc[j], 0.f));
    }
}

// ------------------------------------------------------------------------------
// forward convolution 32 -> 32 channels, stride 2 (+bias, ReLU), on BF16 MFMA.
// An implicit GEMM: rows = output pixels, columns = the 32 output channels,
// K = 288 ordered (tap, input channel), so a 16-wide K step is one tap and 16
// consecutive input channels.  A workgroup takes units of 128 output pixels
// (NS samples x RB output rows); it stages their input rows into LDS as
// [sample][row][column][channel] (channel stride padded to 40), and each wave
// runs 18 v_mfma_f32_32x32x16_bf16 for its 32 pixels x 32 channels.  The weight
// fragments are loaded into registers once per workgroup.  Lane layouts:
//   A (32 x 16): lane l holds row l % 32, k = 8 (l / 32) .. + 7
//   B (16 x 32): lane l holds column l % 32, k = 8 (l / 32) .. + 7
//   D (32 x 32): lane l holds column l % 32, rows 8 (v / 4) + 4 (l / 32) + v % 4
// ------------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

template <int HIN, int NS, int RB>
__global__ __launch_bounds__(256) void k_conv_mfma(const uint16_t *__restrict__ X, const uint16_t *__restrict__ Wb,
                                                  const uint16_t *__restrict__ Bb, uint16_t *__restrict__ Y, int n) {
    constexpr int HO = HIN / 2;
    constexpr int NR = 2 * RB + 1;     // staged input rows per sample (top padding row included)
    constexpr int WP = HIN + 1;        // staged columns: input columns -1 .. HIN-1
    constexpr int CP = 40;             // channel stride of a staged pixel (bf16 elements)
    constexpr int UPS = HO / RB;       // units per sample
    static_assert(NS * RB * HO == 128 && HO % RB == 0 && HO % 4 == 0, "unit shape");
    __shared__ __align__(16) uint16_t xs[NS * NR * WP * CP];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int co = lane & 31, kh = lane >> 5;
    bf16x8_t bfr[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int ci = 16 * h + 8 * kh + j;
                bfr[t][h][j] = __builtin_bit_cast(__bf16, Wb[(co * C + ci) * 9 + t]);
            }
    const float bias = bf2f(Bb[co]);
    // the left padding column is zero for every unit
    for (int e = tid; e < NS * NR * C; e += 256) xs[(e / C) * WP * CP + e % C] = 0;
    constexpr int VPR = HIN / 8;       // 16-byte vectors per input row
    const int units = ((n + NS - 1) / NS) * UPS;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int n0 = (u / UPS) * NS, r0 = (u % UPS) * RB;
        __syncthreads();   // the previous unit's tile is consumed
        // each task: 8 consecutive input pixels of one (sample, channel, row), one 16-byte load,
        // transposed into the [pixel][channel] staging layout
        for (int task = tid; task < NS * C * NR * VPR; task += 256) {
            const int vx = task % VPR, yr = (task / VPR) % NR, ci = (task / (VPR * NR)) % C;
            const int sm = task / (VPR * NR * C);
            const int yi = 2 * r0 - 1 + yr, nn = n0 + sm;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (nn < n && yi >= 0 && yi < HIN)
                v = *reinterpret_cast<const uint4 *>(X + (((size_t)nn * C + ci) * HIN + yi) * HIN + 8 * vx);
            uint16_t *dst = xs + ((sm * NR + yr) * WP + 1 + 8 * vx) * CP + ci;
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                dst[(2 * j) * CP] = (uint16_t)(w[j] & 0xffffu);
                dst[(2 * j + 1) * CP] = (uint16_t)(w[j] >> 16);
            }
        }
        __syncthreads();
        const int m = 32 * wave + (lane & 31);
        const int sm = m / (RB * HO), oy = (m % (RB * HO)) / HO, ox = m % HO;
        f32x16_t acc;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ky = t / 3, kx = t % 3;
            const uint16_t *pa = xs + ((sm * NR + 2 * oy + ky) * WP + 2 * ox + kx) * CP + 8 * kh;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const bf16x8_t a = *reinterpret_cast<const bf16x8_t *>(pa + 16 * h);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bfr[t][h], acc, 0, 0, 0);
            }
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int mm = 32 * wave + 8 * g + 4 * kh;        // first of 4 consecutive pixels (same row)
            const int s2 = mm / (RB * HO), oy2 = (mm % (RB * HO)) / HO, ox2 = mm % HO;
            const int nn = n0 + s2;
            if (nn < n) {
                uint2 packed;
                packed.x = (uint32_t)f2bf(fmaxf(acc[4 * g + 0] + bias, 0.f)) |
                           ((uint32_t)f2bf(fmaxf(acc[4 * g + 1] + bias, 0.f)) << 16);
                packed.y = (uint32_t)f2bf(fmaxf(acc[4 * g + 2] + bias, 0.f)) |
                           ((uint32_t)f2bf(fmaxf(acc[4 * g + 3] + bias, 0.f)) << 16);
                *reinterpret_cast<uint2 *>(Y + (((size_t)nn * C + co) * HO + r0 + oy2) * HO + ox2) = packed;
            }
        }
    }
}

template <int HIN, int NS, int RB>
void launch_conv_mfma(const uint16_t *X, const uint16_t *Wb, const uint16_t *Bb, uint16_t *Y, int n, hipStream_t st) {
    constexpr int UPS = (HIN / 2) / RB;
    const int units = ((n + NS - 1) / NS) * UPS;
    const int grid = units < 2048 ? units : 2048;
    hipLaunchKernelGGL((k_conv_mfma<HIN, NS, RB>), dim3(grid), dim3(256), 0, st, X, Wb, Bb, Y, n);
}

// ------------------------------------------------------------------------------
// readout: A4 [N][32][4][4] -> logits, softmax, (loss and gradients)
// One workgroup processes all samples in a fixed order; per-sample terms are
// summed per lane and reduced across the block in a fixed order.
// ------------------------------------------------------------------------------
__device__ __forceinline__ void quad_feats(const uint16_t *a4, float feat[4][C]) {
    for (int c = 0; c < 4; ++c) {
        const int bx = c & 1, by = c >> 1;
        for (int k = 0; k < C; ++k) {
            const uint16_t *m = a4 + k * 16;
            feat[c][k] = 0.25f * (bf2f(m[(2 * by) * 4 + 2 * bx]) + bf2f(m[(2 * by) * 4 + 2 * bx + 1]) +
                                  bf2f(m[(2 * by + 1) * 4 + 2 * bx]) + bf2f(m[(2 * by + 1) * 4 + 2 * bx + 1]));
        }
    }
}

__global__ __launch_bounds__(256) void k_readout(const uint16_t *__restrict__ A4, const uint16_t *__restrict__ Wb,
                                                 const int *__restrict__ labels, int n, float *__restrict__ probs,
                                                 float *__restrict__ dZ4, float *__restrict__ grad,
                                                 float *__restrict__ loss) {
    __shared__ float red[256];
    const uint16_t *wl = Wb + OFF_WL;
    const float bl = bf2f(Wb[OFF_BL]);
    float dwl[C];
    for (int k = 0; k < C; ++k) dwl[k] = 0.f;
    float dbl = 0.f, lsum = 0.f;
    // inference runs on many workgroups; with labels a single workgroup keeps the reductions' order fixed
    for (int s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256) {
        const uint16_t *a4 = A4 + (size_t)s * C * 16;
        float feat[4][C];
        quad_feats(a4, feat);
        float z[4], mx = -INFINITY;
        for (int c = 0; c < 4; ++c) {
            float t = bl;
            for (int k = 0; k < C; ++k) t = fmaf(feat[c][k], bf2f(wl[k]), t);
            z[c] = t;
            mx = fmaxf(mx, t);
        }
        float e[4], se = 0.f;
        for (int c = 0; c < 4; ++c) { e[c] = expf(z[c] - mx); se += e[c]; }
        float pr[4];
        for (int c = 0; c < 4; ++c) {
            pr[c] = e[c] / se;
            if (probs) probs[4 * s + c] = pr[c];
        }
        if (labels) {
            const int lab = labels[s];
            const bool valid = lab >= 0 && lab < 4;    // other labels mask the sample out
            float zl = z[0];
            for (int c = 1; c < 4; ++c) zl = c == lab ? z[c] : zl;
            if (valid) lsum += -(zl - mx - logf(se));
            float dl[4];
            for (int c = 0; c < 4; ++c) dl[c] = valid ? (pr[c] - (c == lab ? 1.f : 0.f)) / (float)n : 0.f;
            for (int c = 0; c < 4; ++c) {
                dbl += dl[c];
                for (int k = 0; k < C; ++k) dwl[k] = fmaf(dl[c], feat[c][k], dwl[k]);
            }
            // d(activation) = dl[c] * wl[k] / 4 on quadrant c, masked by ReLU' (a4 > 0)
            float *dz = dZ4 + (size_t)s * C * 16;
            for (int k = 0; k < C; ++k)
                for (int q = 0; q < 16; ++q) {
                    const int y = q >> 2, x = q & 3;
                    const int c = (x >> 1) + 2 * (y >> 1);
                    const float v = dl[c] * bf2f(wl[k]) * 0.25f;
                    dz[k * 16 + q] = bf2f(a4[k * 16 + q]) > 0.f ? v : 0.f;
                }
        }
    }
    if (!labels) return;
    // fixed-order block reductions of dwl[k], dbl and the loss
    for (int k = 0; k < C + 2; ++k) {
        const float v = k < C ? dwl[k] : (k == C ? dbl : lsum);
        red[threadIdx.x] = v;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (k < C) grad[OFF_WL + k] = red[0];
            else if (k == C) grad[OFF_BL] = red[0];
            else *loss = red[0] / (float)n;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------
// backward data: dZ [N][32][HO][HO] fp32, W -> dX [N][CIN][HIN][HIN] masked by
// ReLU'(A_in > 0), fp32.  Workgroup: one sample, RB input rows; lane: one input
// pixel, 16 input channels.
// ------------------------------------------------------------------------------
template <int HIN, int S, int RB>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const float *__restrict__ dZ, const uint16_t *__restrict__ Wb,
                                                      const uint16_t *__restrict__ Ain, float *__restrict__ dX) {
    constexpr int CIN = C;
    constexpr int HO = HIN / S;
    constexpr int PIX = RB * HIN;
    constexpr int GROUPS = 256 / PIX;
    constexpr int CPG = CIN / GROUPS;
    constexpr int NR = RB / S + 2;           // output rows that touch RB input rows
    static_assert(PIX * GROUPS == 256 && CPG * GROUPS == CIN, "tile shape");
    __shared__ float w[C * 9][CIN];          // [co*9 + k][ci]
    __shared__ float dz[C][NR][HO];
    const int n = blockIdx.y, r0 = blockIdx.x * RB, tid = threadIdx.x;
    for (int e = tid; e < C * CIN * 9; e += 256) {
        const int co = e / (CIN * 9), ci = (e / 9) % CIN, k = e % 9;
        w[co * 9 + k][ci] = bf2f(Wb[e]);
    }
    const int oy0 = (r0 + 1 - 2) / S < 0 ? 0 : (r0 + 1 - 2) / S;   // first output row touching r0
    const float *dzs = dZ + (size_t)n * C * HO * HO;
    for (int e = tid; e < C * NR * HO; e += 256) {
        const int co = e / (NR * HO), rr = (e / HO) % NR, xo = e % HO;
        const int yo = oy0 + rr;
        dz[co][rr][xo] = yo < HO ? dzs[(co * HO + yo) * HO + xo] : 0.f;
    }
    __syncthreads();
    const int p = tid % PIX, g = tid / PIX;
    const int yi = r0 + p / HIN, xi = p % HIN;
    float acc[CPG];
#pragma unroll
    for (int j = 0; j < CPG; ++j) acc[j] = 0.f;
    for (int ky = 0; ky < 3; ++ky) {
        const int ty = yi + 1 - ky;
        if (ty < 0 || ty % S) continue;
        const int yo = ty / S;
        if (yo >= HO) continue;
        for (int kx = 0; kx < 3; ++kx) {
            const int tx = xi + 1 - kx;
            if (tx < 0 || tx % S) continue;
            const int xo = tx / S;
            if (xo >= HO) continue;
            for (int co = 0; co < C; ++co) {
                const float d = dz[co][yo - oy0][xo];
                const float *wr = &w[co * 9 + ky * 3 + kx][g * CPG];
#pragma unroll
                for (int j = 0; j < CPG; ++j) acc[j] = fmaf(wr[j], d, acc[j]);
            }
        }
    }
    if (yi < HIN) {
        const uint16_t *as = Ain + (size_t)n * CIN * HIN * HIN;
        float *dxs = dX + (size_t)n * CIN * HIN * HIN;
#pragma unroll
        for (int j = 0; j < CPG; ++j) {
            const int ci = g * CPG + j;
            const size_t o = ((size_t)ci * HIN + yi) * HIN + xi;
            dxs[o] = bf2f(as[o]) > 0.f ? acc[j] : 0.f;
        }
    }
}

// ------------------------------------------------------------------------------
// backward weight: dW[co][ci][k] = sum_n sum_pixels dZ[n][co][p] * X[n][ci][shifted p],
// db[co] = sum dZ.  Two deterministic stages: workgroup (co, ci, chunk) reduces a
// fixed chunk of the (sample, pixel) range into part[chunk][co][ci][10]; then
// k_reduce_parts sums the chunks in order.
// ------------------------------------------------------------------------------
constexpr int kMaxChunks = 64;
constexpr int kChunkElems = 4096;

template <int CIN, int HIN, int S>
__global__ __launch_bounds__(256) void k_conv_bwd_weight(const float *__restrict__ dZ, const uint16_t *__restrict__ X,
                                                        int n, int chunk_len, float *__restrict__ part) {
    constexpr int HO = HIN / S;
    __shared__ float red[256];
    const int co = blockIdx.x, ci = blockIdx.y, ch = blockIdx.z;
    float acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = 0.f;
    const int total = n * HO * HO;
    const int e0 = ch * chunk_len, e1 = min(total, e0 + chunk_len);
    for (int e = e0 + threadIdx.x; e < e1; e += 256) {
        const int s = e / (HO * HO), p = e % (HO * HO);
        const int yo = p / HO, xo = p % HO;
        const float d = dZ[((size_t)s * C + co) * HO * HO + p];
        if (d == 0.f) continue;
        const uint16_t *xs = X + ((size_t)s * CIN + ci) * HIN * HIN;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const int yi = S * yo + ky - 1;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int xi = S * xo + kx - 1;
                const float xv = (yi >= 0 && yi < HIN && xi >= 0 && xi < HIN) ? bf2f(xs[yi * HIN + xi]) : 0.f;
                acc[ky * 3 + kx] = fmaf(d, xv, acc[ky * 3 + kx]);
            }
        }
        acc[9] += d;
    }
    for (int k = 0; k < 10; ++k) {
        red[threadIdx.x] = acc[k];
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(((size_t)ch * C + co) * CIN + ci) * 10 + k] = red[0];
        __syncthreads();
    }
}

__global__ void k_reduce_parts(const float *__restrict__ part, int nch, int cin, float *__restrict__ dW,
                               float *__restrict__ db) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;   // (co, ci, k)
    if (i >= C * cin * 10) return;
    const int k = i % 10, ci = (i / 10) % cin, co = i / (10 * cin);
    float sum = 0.f;
    for (int ch = 0; ch < nch; ++ch) sum += part[(size_t)ch * C * cin * 10 + i];
    if (k < 9) dW[(co * cin + ci) * 9 + k] = sum;
    else if (ci == 0) db[co] = sum;
}

template <int CIN, int HIN, int S>
void launch_bwd_weight(const float *dZ, const uint16_t *X, int n, float *part, float *dW, float *db, hipStream_t st) {
    constexpr int HO = HIN / S;
    const int total = n * HO * HO;
    int nch = (total + kChunkElems - 1) / kChunkElems;
    nch = nch < 1 ? 1 : (nch > kMaxChunks ? kMaxChunks : nch);
    const int chunk_len = (total + nch - 1) / nch;
    hipLaunchKernelGGL((k_conv_bwd_weight<CIN, HIN, S>), dim3(C, CIN, nch), dim3(256), 0, st, dZ, X, n, chunk_len,
                       part);
    hipLaunchKernelGGL(k_reduce_parts, dim3((C * CIN * 10 + 255) / 256), dim3(256), 0, st, part, nch, CIN, dW, db);
}

// Adam on FP32 masters, then the BF16 compute copy.
__global__ void k_adam(float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, uint16_t *__restrict__ wb, int np, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float t = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    theta[i] = t;
    wb[i] = f2bf(t);
}

__global__ void k_to_bf16(const float *__restrict__ a, uint16_t *__restrict__ b, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = f2bf(a[i]);
}

}  // namespace
}  // namespace uwb

using namespace uwb;

struct uwb_cnn {
    int max_batch = 0;
    int64_t step = 0;
    // device buffers
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
    float *part = nullptr;   // per-chunk partial weight gradients
    uint16_t *wb = nullptr;
    uint16_t *a[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // a[0] = input copy not kept: a[1..4]
    float *dz[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};     // dZ of layers 1..4
    std::vector<void *> owned;
};

namespace uwb {
namespace {

constexpr int kSide[5] = {32, 32, 16, 8, 4};   // spatial side of a[i]

template <typename T>
bool dalloc(uwb_cnn *h, T **p, size_t count) {
    if (hipMalloc((void **)p, sizeof(T) * (count ? count : 1)) != hipSuccess) return false;
    h->owned.push_back(*p);
    return true;
}

hipError_t forward(uwb_cnn *h, const uint16_t *x, int n, hipStream_t st) {
    hipLaunchKernelGGL((k_conv_fwd<1, 32, 1, 8>), dim3(4, n), dim3(256), 0, st, x, h->wb + OFF_W[0],
                       h->wb + OFF_B + 0 * C, h->a[1]);
    launch_conv_mfma<32, 1, 8>(h->a[1], h->wb + OFF_W[1], h->wb + OFF_B + 1 * C, h->a[2], n, st);
    launch_conv_mfma<16, 2, 8>(h->a[2], h->wb + OFF_W[2], h->wb + OFF_B + 2 * C, h->a[3], n, st);
    launch_conv_mfma<8, 8, 4>(h->a[3], h->wb + OFF_W[3], h->wb + OFF_B + 3 * C, h->a[4], n, st);
    return hipGetLastError();
}

hipError_t backward(uwb_cnn *h, const uint16_t *x, const int *labels, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_readout, dim3(1), dim3(256), 0, st, h->a[4], h->wb, labels, n, (float *)nullptr, h->dz[4],
                       h->grad, h->loss);
    // layer 4 (8 -> 4), layer 3 (16 -> 8), layer 2 (32 -> 16): weight grads, then data grads
    launch_bwd_weight<C, 8, 2>(h->dz[4], h->a[3], n, h->part, h->grad + OFF_W[3], h->grad + OFF_B + 3 * C, st);
    hipLaunchKernelGGL((k_conv_bwd_data<8, 2, 8>), dim3(1, n), dim3(256), 0, st, h->dz[4], h->wb + OFF_W[3], h->a[3],
                       h->dz[3]);
    launch_bwd_weight<C, 16, 2>(h->dz[3], h->a[2], n, h->part, h->grad + OFF_W[2], h->grad + OFF_B + 2 * C, st);
    hipLaunchKernelGGL((k_conv_bwd_data<16, 2, 4>), dim3(4, n), dim3(256), 0, st, h->dz[3], h->wb + OFF_W[2],
                       h->a[2], h->dz[2]);
    launch_bwd_weight<C, 32, 2>(h->dz[2], h->a[1], n, h->part, h->grad + OFF_W[1], h->grad + OFF_B + 1 * C, st);
    hipLaunchKernelGGL((k_conv_bwd_data<32, 2, 2>), dim3(16, n), dim3(256), 0, st, h->dz[2], h->wb + OFF_W[1],
                       h->a[1], h->dz[1]);
    launch_bwd_weight<1, 32, 1>(h->dz[1], x, n, h->part, h->grad + OFF_W[0], h->grad + OFF_B + 0 * C, st);
    return hipGetLastError();
}

}  // namespace
}  // namespace uwb

namespace uwb {
int cnn_max_batch(const uwb_cnn *h) { return h ? h->max_batch : 0; }
}  // namespace uwb

extern "C" {

int uwb_cnn_param_count(void) { return NPARAM; }

int uwb_cnn_create(uwb_cnn **out, int32_t max_batch, const float *init_params) {
    if (!out || !init_params || max_batch < 1) return UWB_EINVAL;
    if (max_batch > 65535) return UWB_EUNSUPPORTED;   // one grid row per sample
    *out = nullptr;
    uwb_cnn *h = new (std::nothrow) uwb_cnn();
    if (!h) return UWB_ENOMEM;
    h->max_batch = max_batch;
    const size_t nb = (size_t)max_batch;
    bool ok = dalloc(h, &h->theta, NPARAM) && dalloc(h, &h->m, NPARAM) && dalloc(h, &h->v, NPARAM) &&
              dalloc(h, &h->grad, NPARAM) && dalloc(h, &h->loss, 1) && dalloc(h, &h->wb, NPARAM) &&
              dalloc(h, &h->part, (size_t)kMaxChunks * C * C * 10);
    for (int i = 1; i <= 4 && ok; ++i) {
        ok = dalloc(h, &h->a[i], nb * C * kSide[i] * kSide[i]) && dalloc(h, &h->dz[i], nb * C * kSide[i] * kSide[i]);
    }
    if (!ok) { uwb_cnn_destroy(h); return UWB_ENOMEM; }
    if (hipMemcpy(h->theta, init_params, sizeof(float) * NPARAM, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(h->m, 0, sizeof(float) * NPARAM) != hipSuccess ||
        hipMemset(h->v, 0, sizeof(float) * NPARAM) != hipSuccess) {
        uwb_cnn_destroy(h);
        return UWB_EHIP;
    }
    hipLaunchKernelGGL(k_to_bf16, dim3((NPARAM + 255) / 256), dim3(256), 0, nullptr, h->theta, h->wb, NPARAM);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        uwb_cnn_destroy(h);
        return UWB_EHIP;
    }
    *out = h;
    return UWB_OK;
}

int uwb_cnn_destroy(uwb_cnn *h) {
    if (!h) return UWB_EINVAL;
    for (void *p : h->owned) hipFree(p);
    delete h;
    return UWB_OK;
}

int uwb_cnn_forward(uwb_cnn *h, const uint16_t *x, int32_t n, float *probs, void *stream) {
    if (!h || !x || !probs || n < 1) return UWB_EINVAL;
    if (n > h->max_batch) return UWB_ERANGE;
    const hipStream_t st = (hipStream_t)stream;
    if (forward(h, x, n, st) != hipSuccess) return UWB_EHIP;
    hipLaunchKernelGGL(k_readout, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, h->a[4], h->wb,
                       (const int *)nullptr, n, probs, (float *)nullptr, (float *)nullptr, (float *)nullptr);
    return hipGetLastError() == hipSuccess ? UWB_OK : UWB_EHIP;
}

int uwb_cnn_gradients(uwb_cnn *h, const uint16_t *x, const int32_t *labels, int32_t n, float *grad_out,
                      float *loss_out, void *stream) {
    if (!h || !x || !labels || n < 1) return UWB_EINVAL;
    if (n > h->max_batch) return UWB_ERANGE;
    const hipStream_t st = (hipStream_t)stream;
    if (forward(h, x, n, st) != hipSuccess || backward(h, x, labels, n, st) != hipSuccess) return UWB_EHIP;
    if (grad_out && hipMemcpyAsync(grad_out, h->grad, sizeof(float) * NPARAM, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return UWB_EHIP;
    if (loss_out && hipMemcpyAsync(loss_out, h->loss, sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return UWB_EHIP;
    return UWB_OK;
}

int uwb_cnn_train_step(uwb_cnn *h, const uint16_t *x, const int32_t *labels, int32_t n, float lr, float *loss_out,
                       void *stream) {
    if (!h || !x || !labels || n < 1 || !(lr > 0.f) || !std::isfinite(lr)) return UWB_EINVAL;
    if (n > h->max_batch) return UWB_ERANGE;
    const hipStream_t st = (hipStream_t)stream;
    if (forward(h, x, n, st) != hipSuccess || backward(h, x, labels, n, st) != hipSuccess) return UWB_EHIP;
    h->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)h->step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)h->step));
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, h->theta, h->m, h->v, h->grad, h->wb,
                       NPARAM, lr, b1, b2, 1e-8f, c1, c2);
    if (loss_out && hipMemcpyAsync(loss_out, h->loss, sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return UWB_EHIP;
    return hipGetLastError() == hipSuccess ? UWB_OK : UWB_EHIP;
}

// Checkpoint: host buffers of NPARAM floats each (any may be NULL), and the step count.
int uwb_cnn_get_state(uwb_cnn *h, float *theta, float *m, float *v, int64_t *step, void *stream) {
    if (!h) return UWB_EINVAL;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return UWB_EHIP;
    if (theta && hipMemcpy(theta, h->theta, sizeof(float) * NPARAM, hipMemcpyDeviceToHost) != hipSuccess) return UWB_EHIP;
    if (m && hipMemcpy(m, h->m, sizeof(float) * NPARAM, hipMemcpyDeviceToHost) != hipSuccess) return UWB_EHIP;
    if (v && hipMemcpy(v, h->v, sizeof(float) * NPARAM, hipMemcpyDeviceToHost) != hipSuccess) return UWB_EHIP;
    if (step) *step = h->step;
    return UWB_OK;
}

int uwb_cnn_set_state(uwb_cnn *h, const float *theta, const float *m, const float *v, int64_t step, void *stream) {
    if (!h || !theta || !m || !v || step < 0) return UWB_EINVAL;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return UWB_EHIP;
    if (hipMemcpy(h->theta, theta, sizeof(float) * NPARAM, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->m, m, sizeof(float) * NPARAM, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->v, v, sizeof(float) * NPARAM, hipMemcpyHostToDevice) != hipSuccess)
        return UWB_EHIP;
    h->step = step;
    hipLaunchKernelGGL(k_to_bf16, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, h->theta, h->wb,
                       NPARAM);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return UWB_EHIP;
    return UWB_OK;
}

// Device pointer to the BF16 compute weights (NPARAM values, flat order), for the learned walk.
const uint16_t *uwb_cnn_weights_bf16(const uwb_cnn *h) { return h ? h->wb : nullptr; }

}  // extern "C"
