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
// Kernels: forward convolution (+bias, ReLU, BF16 store; the 32-channel layers on
// BF16 MFMA); readout, and its training form with softmax cross-entropy; for the
// 32-channel layers, backward-data (fused with the ReLU derivative of its input)
// and backward-weight convolutions, and the first layer's backward weight, on
// BF16 MFMA, FP32 operands entering as two BF16 parts; Adam.
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
// readout (inference): A4 [N][32][4][4] -> four quadrant features of 32 channels,
// the shared linear score of each, softmax.  One thread per sample.
// ------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_readout(const uint16_t *__restrict__ A4, const uint16_t *__restrict__ Wb,
                                                 int n, float *__restrict__ probs) {
    const uint16_t *wl = Wb + OFF_WL;
    const float bl = bf2f(Wb[OFF_BL]);
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const uint16_t *a4 = A4 + (size_t)s * C * 16;
    float z[4], mx = -INFINITY;
    for (int c = 0; c < 4; ++c) {
        const int bx = c & 1, by = c >> 1;
        float t = bl;
        for (int k = 0; k < C; ++k) {
            const uint16_t *m = a4 + k * 16;
            const float f = 0.25f * (bf2f(m[(2 * by) * 4 + 2 * bx]) + bf2f(m[(2 * by) * 4 + 2 * bx + 1]) +
                                     bf2f(m[(2 * by + 1) * 4 + 2 * bx]) + bf2f(m[(2 * by + 1) * 4 + 2 * bx + 1]));
            t = fmaf(f, bf2f(wl[k]), t);
        }
        z[c] = t;
        mx = fmaxf(mx, t);
    }
    float e[4], se = 0.f;
    for (int c = 0; c < 4; ++c) { e[c] = expf(z[c] - mx); se += e[c]; }
    for (int c = 0; c < 4; ++c) probs[4 * s + c] = e[c] / se;
}

// ------------------------------------------------------------------------------
// training readout: softmax cross-entropy of the four quadrant scores, its
// gradients with respect to the readout weights, bias and the last activations
// (masked by their ReLU derivative), one wavefront per sample.  Lane l takes channel k = l % 32 and quadrants 2 (l / 32), 2 (l / 32) + 1
// (the bottom or top half of the 4 x 4 map); the logits are wavefront sums.  Each
// workgroup (4 samples) sums its samples' readout-weight, bias and loss terms in
// wave order into part[wg][C + 2]; k_readout_reduce adds the workgroups in order.
// ------------------------------------------------------------------------------
constexpr int kReadoutTerms = C + 2;   // d wl[0..31], d bl, loss

__global__ __launch_bounds__(256) void k_readout_train(const uint16_t *__restrict__ A4, const uint16_t *__restrict__ Wb,
                                                       const int *__restrict__ labels, int n, float *__restrict__ dZ4,
                                                       float *__restrict__ part) {
    __shared__ float red[4][kReadoutTerms];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int k = lane & 31, by = lane >> 5;
    const int s = 4 * blockIdx.x + wave;
    const float wlk = bf2f(Wb[OFF_WL + k]);
    const float bl = bf2f(Wb[OFF_BL]);
    float dwl = 0.f, dbl = 0.f, ls = 0.f;
    if (s < n) {
        const uint16_t *m = A4 + ((size_t)s * C + k) * 16;
        float feat[2];
#pragma unroll
        for (int bx = 0; bx < 2; ++bx)
            feat[bx] = 0.25f * (bf2f(m[(2 * by) * 4 + 2 * bx]) + bf2f(m[(2 * by) * 4 + 2 * bx + 1]) +
                                bf2f(m[(2 * by + 1) * 4 + 2 * bx]) + bf2f(m[(2 * by + 1) * 4 + 2 * bx + 1]));
        // logits of quadrants c = bx + 2 by: sums over the 32 channels of each half-wave
        float z2[2];
#pragma unroll
        for (int bx = 0; bx < 2; ++bx) {
            float t = feat[bx] * wlk;
#pragma unroll
            for (int o = 1; o < 32; o <<= 1) t += __shfl_xor(t, o, 64);
            z2[bx] = t + bl;
        }
        float z[4];
        z[0] = __shfl(z2[0], 0, 64);
        z[1] = __shfl(z2[1], 0, 64);
        z[2] = __shfl(z2[0], 32, 64);
        z[3] = __shfl(z2[1], 32, 64);
        float mx = z[0];
        for (int c = 1; c < 4; ++c) mx = fmaxf(mx, z[c]);
        float e[4], se = 0.f;
        for (int c = 0; c < 4; ++c) { e[c] = expf(z[c] - mx); se += e[c]; }
        const int lab = labels[s];
        const bool valid = lab >= 0 && lab < 4;   // other labels mask the sample out
        float zl = z[0];
        for (int c = 1; c < 4; ++c) zl = c == lab ? z[c] : zl;
        ls = valid ? -(zl - mx - logf(se)) : 0.f;
        float dl[4];
        for (int c = 0; c < 4; ++c) dl[c] = valid ? (e[c] / se - (c == lab ? 1.f : 0.f)) / (float)n : 0.f;
        dbl = dl[0] + dl[1] + dl[2] + dl[3];
        // d wl[k]: this half's two quadrants, plus the other half's
        const float mine = fmaf(dl[2 * by + 1], feat[1], dl[2 * by] * feat[0]);
        const float other = __shfl_xor(mine, 32, 64);
        dwl = by == 0 ? mine + other : other + mine;
        // d(activation) on this lane's 8 positions (rows 2 by, 2 by + 1), masked by ReLU'(a4 > 0)
        float *dz = dZ4 + ((size_t)s * C + k) * 16 + 8 * by;
        const uint16_t *a = m + 8 * by;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int c = ((q & 3) >> 1) + 2 * by;
            const float v = dl[c] * wlk * 0.25f;
            dz[q] = bf2f(a[q]) > 0.f ? v : 0.f;
        }
    }
    if (lane < C) red[wave][lane] = dwl;
    if (lane == 0) { red[wave][C] = dbl; red[wave][C + 1] = ls; }
    __syncthreads();
    if (threadIdx.x < kReadoutTerms) {
        const int t = threadIdx.x;
        part[(size_t)blockIdx.x * kReadoutTerms + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    }
}

__global__ void k_readout_reduce(const float *__restrict__ part, int nwg, int n, float *__restrict__ grad,
                                 float *__restrict__ loss) {
    const int t = threadIdx.x;
    if (t >= kReadoutTerms) return;
    float sum = 0.f;
    for (int b = 0; b < nwg; b += 16) {   // in workgroup order, loaded 16 at a time
        float v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = b + j < nwg ? part[(size_t)(b + j) * kReadoutTerms + t] : 0.f;
#pragma unroll
        for (int j = 0; j < 16; ++j) sum += v[j];
    }
    if (t < C) grad[OFF_WL + t] = sum;
    else if (t == C) grad[OFF_BL] = sum;
    else *loss = sum / (float)n;
}

// FP32 value as the sum of two BF16 values: its rounding, and the rounding of the
// remainder (exact in FP32): together within 2^-17 of the value, relative.
__device__ __forceinline__ void split_bf16(float x, uint16_t &hi, uint16_t &lo) {
    hi = f2bf(x);
    lo = f2bf(x - bf2f(hi));
}

// ------------------------------------------------------------------------------
// backward data of a 32 -> 32 channel, stride-2 convolution, on BF16 MFMA, fused
// with the ReLU derivative of its input:
//   dX[ci][yi][xi] = [A_in > 0] * sum over co and the taps (ky, kx) with
//                    yi = 2 yo + ky - 1, xi = 2 xo + kx - 1 of W[co][ci][ky][kx] dZ[co][yo][xo].
// Input pixel (2 a + py, 2 b + px) of parity class (py, px) takes its taps at fixed
// offsets: along y, py = 0 has ky = 1 (yo = a), py = 1 has ky = 0 (yo = a + 1) and
// ky = 2 (yo = a); x likewise.  So per class it is a GEMM over K = (tap, co) with
// rows = the "super-pixels" (a, b), columns = ci: A = dZ shifted by (dy, dx) in
// {0, 1}^2 (FP32 as two BF16 operands, split_bf16), B = W at that tap.  A workgroup
// takes units of 128 super-pixels (NS samples x RA super-rows), 32 per wave; it
// stages dZ rows a0 .. a0 + RA (the last one zero past the edge) and columns
// 0 .. HO (likewise) as [pixel][co] with a padded channel stride, so each A fragment
// (8 consecutive co) is one 16-byte LDS read, shared by every class that uses its
// shift.  W is staged once per workgroup as [tap][ci][co] for its fragments.
// ------------------------------------------------------------------------------
template <int HIN, int NS, int RA>
struct BwddShape {
    static constexpr int HO = HIN / 2;
    static constexpr int CP = 40;                                  // channel stride of a staged pixel (bf16)
    static constexpr int PIX = NS * (RA + 1) * (HO + 1);           // staged dZ pixels per unit
    static constexpr int LDS_DZ = 2 * PIX * CP;                    // [hi | lo][pixel][co]
    static constexpr int LDS_W = 9 * C * CP;                       // [tap][ci][co]
    static constexpr int LDS = LDS_DZ > LDS_W ? LDS_DZ : LDS_W;
    static constexpr int UPS = HO / RA;
    static_assert(NS * RA * HO == 128 && HO % RA == 0 && HO % 4 == 0, "unit shape");
};

template <int HIN, int NS, int RA>
__global__ __launch_bounds__(256) void k_bwdd_mfma(const float *__restrict__ dZ, const uint16_t *__restrict__ Wb,
                                                  const uint16_t *__restrict__ Ain, float *__restrict__ dX, int n) {
    using SH = BwddShape<HIN, NS, RA>;
    constexpr int HO = SH::HO, CP = SH::CP, PIX = SH::PIX, UPS = SH::UPS;
    __shared__ __align__(16) uint16_t lds[SH::LDS];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int col = lane & 31, kh = lane >> 5;
    // W as [tap][ci][co], then this lane's B fragments: column ci = col, k = co = 16 h + 8 kh .. + 7
    for (int e = tid; e < C * C * 9; e += 256) {
        const int co = e / (C * 9), ci = (e / 9) % C, t = e % 9;
        lds[(t * C + ci) * CP + co] = Wb[e];
    }
    __syncthreads();
    bf16x8_t bfr[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) bfr[t][h] = *reinterpret_cast<const bf16x8_t *>(lds + (t * C + col) * CP + 16 * h + 8 * kh);

    const int units = ((n + NS - 1) / NS) * UPS;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int n0 = (u / UPS) * NS, a0 = (u % UPS) * RA;
        __syncthreads();   // the weights (first unit) or the previous unit are consumed
        // dZ: one task = 4 channels of one staged pixel (zero past the edges and the batch);
        // consecutive lanes take consecutive pixels, so the loads of a channel coalesce
        for (int task = tid; task < PIX * (C / 4); task += 256) {
            const int pix = task % PIX, c4 = task / PIX;
            const int bb = pix % (HO + 1), ar = (pix / (HO + 1)) % (RA + 1), sm = pix / ((HO + 1) * (RA + 1));
            const int a = a0 + ar, nn = n0 + sm;
            uint16_t hi[4], lo[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int co = 4 * c4 + j;
                const float v = (nn < n && a < HO && bb < HO) ? dZ[(((size_t)nn * C + co) * HO + a) * HO + bb] : 0.f;
                split_bf16(v, hi[j], lo[j]);
            }
            uint2 ph, pl;
            ph.x = (uint32_t)hi[0] | ((uint32_t)hi[1] << 16);
            ph.y = (uint32_t)hi[2] | ((uint32_t)hi[3] << 16);
            pl.x = (uint32_t)lo[0] | ((uint32_t)lo[1] << 16);
            pl.y = (uint32_t)lo[2] | ((uint32_t)lo[3] << 16);
            *reinterpret_cast<uint2 *>(lds + pix * CP + 4 * c4) = ph;
            *reinterpret_cast<uint2 *>(lds + PIX * CP + pix * CP + 4 * c4) = pl;
        }
        __syncthreads();
        // this lane's super-pixel (A row): m = 32 wave + col
        const int m = 32 * wave + col;
        const int sm = m / (RA * HO), al = (m / HO) % RA, b = m % HO;
        f32x16_t acc[4];   // class (py, px) = 2 py + px
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[c][v] = 0.f;
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int pix = (sm * (RA + 1) + al + dy) * (HO + 1) + b + dx;
                    const bf16x8_t ah = *reinterpret_cast<const bf16x8_t *>(lds + pix * CP + 16 * h + 8 * kh);
                    const bf16x8_t alo = *reinterpret_cast<const bf16x8_t *>(lds + PIX * CP + pix * CP + 16 * h + 8 * kh);
                    // classes and taps at this shift: along y, dy = 0 serves (py 0, ky 1) and (py 1, ky 2),
                    // dy = 1 serves (py 1, ky 0); along x likewise
#pragma unroll
                    for (int py = 0; py < 2; ++py) {
                        if (dy == 1 && py == 0) continue;
                        const int ky = dy == 1 ? 0 : (py == 0 ? 1 : 2);
#pragma unroll
                        for (int px = 0; px < 2; ++px) {
                            if (dx == 1 && px == 0) continue;
                            const int kx = dx == 1 ? 0 : (px == 0 ? 1 : 2);
                            const int c = 2 * py + px, t = 3 * ky + kx;
                            acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bfr[t][h], acc[c], 0, 0, 0);
                            acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bfr[t][h], acc[c], 0, 0, 0);
                        }
                    }
                }
        // D: column ci = col, rows (super-pixels) 8 (v / 4) + 4 kh + v % 4; the two x-classes of a
        // super-pixel are adjacent columns: one 8-byte store each, masked by ReLU'(A_in)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int mm = 32 * wave + 8 * (v / 4) + 4 * kh + v % 4;
            const int s2 = mm / (RA * HO), a2 = a0 + (mm / HO) % RA, b2 = mm % HO;
            const int nn = n0 + s2;
            if (nn >= n) continue;
#pragma unroll
            for (int py = 0; py < 2; ++py) {
                const size_t o = (((size_t)nn * C + col) * HIN + 2 * a2 + py) * HIN + 2 * b2;
                const uint32_t am = *reinterpret_cast<const uint32_t *>(Ain + o);
                float2 r;
                r.x = bf2f((uint16_t)(am & 0xffffu)) > 0.f ? acc[2 * py][v] : 0.f;
                r.y = bf2f((uint16_t)(am >> 16)) > 0.f ? acc[2 * py + 1][v] : 0.f;
                *reinterpret_cast<float2 *>(dX + o) = r;
            }
        }
    }
}

template <int HIN, int NS, int RA>
void launch_bwdd_mfma(const float *dZ, const uint16_t *Wb, const uint16_t *Ain, float *dX, int n, hipStream_t st) {
    constexpr int UPS = BwddShape<HIN, NS, RA>::UPS;
    const int units = ((n + NS - 1) / NS) * UPS;
    const int grid = units < 1024 ? units : 1024;
    hipLaunchKernelGGL((k_bwdd_mfma<HIN, NS, RA>), dim3(grid), dim3(256), 0, st, dZ, Wb, Ain, dX, n);
}

constexpr int kMaxChunks = 256;   // workgroups (partials) of a backward-weight launch, at most

// dW and db from the per-workgroup partials part[chunk][co][ci][10], summed in chunk
// order: thread (output i, group g) adds its quarter of the chunks (loaded 16 at a
// time), then the four group sums are added in group order.
constexpr int kReduceOut = 64;   // outputs per workgroup of k_reduce_parts

__global__ __launch_bounds__(256) void k_reduce_parts(const float *__restrict__ part, int nch, int cin,
                                                      float *__restrict__ dW, float *__restrict__ db) {
    __shared__ float red[4][kReduceOut];
    const int tx = threadIdx.x % kReduceOut, g = threadIdx.x / kReduceOut;
    const int total = C * cin * 10;
    const int i = blockIdx.x * kReduceOut + tx;   // (co, ci, k)
    const int len = (nch + 3) / 4, c0 = g * len, c1 = min(nch, c0 + len);
    float sum = 0.f;
    if (i < total) {
        for (int ch = c0; ch < c1; ch += 16) {
            float v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = ch + j < c1 ? part[(size_t)(ch + j) * total + i] : 0.f;
#pragma unroll
            for (int j = 0; j < 16; ++j) sum += v[j];
        }
    }
    red[g][tx] = sum;
    __syncthreads();
    if (g != 0 || i >= total) return;
    sum = ((red[0][tx] + red[1][tx]) + red[2][tx]) + red[3][tx];
    const int k = i % 10, ci = (i / 10) % cin, co = i / (10 * cin);
    if (k < 9) dW[(co * cin + ci) * 9 + k] = sum;
    else if (ci == 0) db[co] = sum;
}

void launch_reduce_parts(const float *part, int nch, int cin, float *dW, float *db, hipStream_t st) {
    const int total = C * cin * 10;
    hipLaunchKernelGGL(k_reduce_parts, dim3((total + kReduceOut - 1) / kReduceOut), dim3(256), 0, st, part, nch, cin,
                       dW, db);
}

// ------------------------------------------------------------------------------
// backward weight of a 32 -> 32 channel, stride-2 convolution, on BF16 MFMA.  Per
// tap t = (ky, kx):
//   dW_t[co][ci] = sum over samples and output pixels (yo, xo) of
//                  dZ[co][yo][xo] * X[ci][2 yo + ky - 1][2 xo + kx - 1],
//   db[co]       = sum of dZ[co][yo][xo],
// i.e. GEMMs with K = (sample, output pixel): A = dZ (32 co x 16 pixels), B = the
// input at tap t (16 pixels x 32 ci), or ones for the bias.  dZ is FP32 and enters
// as two BF16 operands (split_bf16), so the products keep FP32 accuracy; X is BF16
// already.  Accumulation is FP32 in the MFMA.  A workgroup takes units of 64 output
// pixels (NS samples x RBO output rows) in a fixed sequence and stages, per unit,
// dZ as [co][pixel] (high and low parts) and the input rows as three column arrays
// per (ci, row) -- X[2 xo], X[2 xo - 1], X[2 xo + 1] for xo = 0 .. HO-1 -- so that
// each fragment is a contiguous LDS read.  Wave w accumulates taps w, w + 4, w + 8
// (wave 1: the bias in place of tap 9) over the workgroup's units and writes one
// partial per workgroup; k_reduce_parts sums the partials in workgroup order.
// Lane layouts as in k_conv_mfma (A: row l % 32, k = 8 (l / 32) .. + 7; B: column
// l % 32, same k; D: column l % 32, rows 8 (v / 4) + 4 (l / 32) + v % 4).
// ------------------------------------------------------------------------------
constexpr int kBwdUnitPix = 64;   // output pixels per unit of the MFMA backward-weight kernel

template <int HIN, int NS, int RBO>
struct BwdwShape {
    static constexpr int HO = HIN / 2;
    static constexpr int P = NS * RBO * HO;          // output pixels per unit
    static constexpr int NR = 2 * RBO + 1;           // staged input rows per sample (2 r0 - 1 .. 2 r0 + 2 RBO - 1)
    static constexpr int PA = P + 8;                 // dZ row stride (bf16)
    // per-(sample, ci) stride of the staged input: 2 (mod 64) dwords apart, so the 32
    // channels of a fragment read fall in distinct LDS banks
    static constexpr int XCI = ((NR * 3 * HO + 127) / 128) * 128 + 4;
    static constexpr int LDS_X = NS * C * XCI;       // bf16 elements
    static constexpr int LDS_DZ = 2 * C * PA;
    static constexpr int UPS = HO / RBO;             // units per sample group
    static_assert(P == kBwdUnitPix && HO % 4 == 0 && HO % RBO == 0, "unit shape");
};

template <int HIN, int NS, int RBO>
__global__ __launch_bounds__(256) void k_bwdw_mfma(const float *__restrict__ dZ, const uint16_t *__restrict__ X, int n,
                                                  float *__restrict__ part) {
    using SH = BwdwShape<HIN, NS, RBO>;
    constexpr int HO = SH::HO, P = SH::P, NR = SH::NR, PA = SH::PA, XCI = SH::XCI, UPS = SH::UPS;
    __shared__ __align__(16) uint16_t xs[SH::LDS_X];
    __shared__ __align__(16) uint16_t dzs[SH::LDS_DZ];   // [hi | lo][co][pixel]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int col = lane & 31, kh = lane >> 5;
    const int ntap = wave < 2 ? 3 : 2;                   // taps w, w + 4, w + 8 (wave 1: 1, 5, bias)
    f32x16_t acc[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[j][v] = 0.f;
    bf16x8_t ones;
#pragma unroll
    for (int j = 0; j < 8; ++j) ones[j] = __builtin_bit_cast(__bf16, (uint16_t)0x3f80);

    const int units = ((n + NS - 1) / NS) * UPS;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int n0 = (u / UPS) * NS, r0 = (u % UPS) * RBO;
        __syncthreads();   // the previous unit is consumed
        // input rows: one task = 8 consecutive columns of one (sample, ci, row)
        constexpr int VPR = HIN / 8;
        for (int task = tid; task < NS * C * NR * VPR; task += 256) {
            const int vx = task % VPR, r = (task / VPR) % NR, ci = (task / (VPR * NR)) % C, sm = task / (VPR * NR * C);
            const int yi = 2 * r0 - 1 + r, nn = n0 + sm;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (nn < n && yi >= 0 && yi < HIN)
                v = *reinterpret_cast<const uint4 *>(X + (((size_t)nn * C + ci) * HIN + yi) * HIN + 8 * vx);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            uint16_t *row = xs + (sm * C + ci) * XCI + r * 3 * HO;   // [E | O0 | O2][HO]
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int xo = 4 * vx + j;                              // columns 2 xo (even), 2 xo + 1 (odd)
                row[xo] = (uint16_t)(w[j] & 0xffffu);                   // E[xo]  = X[2 xo]
                row[2 * HO + xo] = (uint16_t)(w[j] >> 16);              // O2[xo] = X[2 xo + 1]
                if (xo + 1 < HO) row[HO + xo + 1] = (uint16_t)(w[j] >> 16);   // O0[xo + 1] = X[2 xo + 1]
            }
            if (vx == 0) row[HO] = 0;                                   // O0[0] = X[-1] (padding)
        }
        // dZ: one task = 4 consecutive pixels of one (sample, co); a sample's unit rows are contiguous
        for (int task = tid; task < C * P / 4; task += 256) {
            const int q = task % (P / 4), co = task / (P / 4);
            const int p = 4 * q, sm = p / (RBO * HO), pr = p % (RBO * HO);
            const int nn = n0 + sm;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (nn < n) v = *reinterpret_cast<const float4 *>(dZ + ((size_t)nn * C + co) * HO * HO + r0 * HO + pr);
            const float f[4] = {v.x, v.y, v.z, v.w};
            uint16_t hi[4], lo[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) split_bf16(f[j], hi[j], lo[j]);
            uint2 ph, pl;
            ph.x = (uint32_t)hi[0] | ((uint32_t)hi[1] << 16);
            ph.y = (uint32_t)hi[2] | ((uint32_t)hi[3] << 16);
            pl.x = (uint32_t)lo[0] | ((uint32_t)lo[1] << 16);
            pl.y = (uint32_t)lo[2] | ((uint32_t)lo[3] << 16);
            *reinterpret_cast<uint2 *>(dzs + co * PA + p) = ph;
            *reinterpret_cast<uint2 *>(dzs + C * PA + co * PA + p) = pl;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < P / 16; ++ks) {
            const int p0 = 16 * ks + 8 * kh;   // this lane's 8 pixels: p0 .. p0 + 7 (two quads, one row each)
            const bf16x8_t ah = *reinterpret_cast<const bf16x8_t *>(dzs + col * PA + p0);
            const bf16x8_t al = *reinterpret_cast<const bf16x8_t *>(dzs + C * PA + col * PA + p0);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                if (j >= ntap) break;
                const int t = wave + 4 * j;   // 9 = bias
                bf16x8_t b;
                if (t == 9) {
                    b = ones;
                } else {
                    const int ky = t / 3, kx = t % 3;
                    const int arr = kx == 1 ? 0 : (kx == 0 ? 1 : 2);
#pragma unroll
                    for (int hq = 0; hq < 2; ++hq) {
                        const int p = p0 + 4 * hq;
                        const int sm = p / (RBO * HO), yl = (p / HO) % RBO, xo = p % HO;
                        const uint2 w = *reinterpret_cast<const uint2 *>(
                            xs + (sm * C + col) * XCI + ((2 * yl + ky) * 3 + arr) * HO + xo);
                        b[4 * hq + 0] = __builtin_bit_cast(__bf16, (uint16_t)(w.x & 0xffffu));
                        b[4 * hq + 1] = __builtin_bit_cast(__bf16, (uint16_t)(w.x >> 16));
                        b[4 * hq + 2] = __builtin_bit_cast(__bf16, (uint16_t)(w.y & 0xffffu));
                        b[4 * hq + 3] = __builtin_bit_cast(__bf16, (uint16_t)(w.y >> 16));
                    }
                }
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, b, acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b, acc[j], 0, 0, 0);
            }
        }
    }
    // this workgroup's partial: part[wg][co][ci][10] (the bias in every ci slot of entry 9)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (j >= ntap) break;
        const int t = wave + 4 * j;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int co = 8 * (v / 4) + 4 * kh + v % 4;
            part[(((size_t)blockIdx.x * C + co) * C + col) * 10 + t] = acc[j][v];
        }
    }
}

template <int HIN, int NS, int RBO>
void launch_bwdw_mfma(const float *dZ, const uint16_t *X, int n, float *part, float *dW, float *db, hipStream_t st) {
    constexpr int UPS = BwdwShape<HIN, NS, RBO>::UPS;
    const int units = ((n + NS - 1) / NS) * UPS;
    const int nch = units < kMaxChunks ? units : kMaxChunks;
    hipLaunchKernelGGL((k_bwdw_mfma<HIN, NS, RBO>), dim3(nch), dim3(256), 0, st, dZ, X, n, part);
    launch_reduce_parts(part, nch, C, dW, db, st);
}

// ------------------------------------------------------------------------------
// backward weight of the first convolution (1 -> 32 channels, stride 1) on BF16
// MFMA: dW[co][t] = sum over samples and pixels of dZ[co][y][x] x[y + ky - 1][x + kx - 1]
// and db[co] = sum of dZ, as one GEMM over K = (sample, pixel): A = dZ (32 co x 16
// pixels, as two BF16 parts), B = 16 pixels x 32 columns holding the input at tap t
// in column t < 9, ones in column 9 (the bias) and zeros beyond.  A unit is
// kL1Rows rows (128 pixels) of one sample; its input rows y0 - 1 .. y0 + kL1Rows are
// staged as three copies shifted by kx - 1 (zero outside), so that each lane's 8
// pixels at its tap are one aligned 16-byte read.  The four waves take alternate
// 16-pixel steps of every unit; their sums are added in wave order at the end,
// one partial per workgroup (part[wg][co][10]).
// ------------------------------------------------------------------------------
constexpr int kL1Rows = 4;

__global__ __launch_bounds__(256) void k_bwdw1_mfma(const float *__restrict__ dZ, const uint16_t *__restrict__ X, int n,
                                                    float *__restrict__ part) {
    constexpr int H = IN;
    constexpr int NRS = kL1Rows + 2;
    constexpr int UPS = H / kL1Rows;
    __shared__ __align__(16) uint16_t xs[NRS * 3 * H];   // [row][kx][x]
    __shared__ float red[4][C][10];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int col = lane & 31, kh = lane >> 5;
    f32x16_t acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
    bf16x8_t fixed;   // column 9: ones (bias); columns 10 .. 31: zeros
#pragma unroll
    for (int j = 0; j < 8; ++j) fixed[j] = __builtin_bit_cast(__bf16, (uint16_t)(col == 9 ? 0x3f80 : 0));
    const int units = n * UPS;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int nn = u / UPS, y0 = (u % UPS) * kL1Rows;
        __syncthreads();   // the previous unit's rows are consumed
        for (int e = tid; e < NRS * 3 * H; e += 256) {
            const int xi = e % H, kx = (e / H) % 3, r = e / (3 * H);
            const int yy = y0 - 1 + r, xx = xi + kx - 1;
            xs[e] = (yy >= 0 && yy < H && xx >= 0 && xx < H) ? X[((size_t)nn * H + yy) * H + xx] : (uint16_t)0;
        }
        __syncthreads();
        for (int ks = wave; ks < kL1Rows * H / 16; ks += 4) {
            const int p0 = 16 * ks + 8 * kh;   // this lane's 8 pixels, within one row
            const int yl = p0 / H, x0 = p0 % H;
            const float *src = dZ + (((size_t)nn * C + col) * H + y0 + yl) * H + x0;
            const float4 v0 = *reinterpret_cast<const float4 *>(src);
            const float4 v1 = *reinterpret_cast<const float4 *>(src + 4);
            const float f[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
            bf16x8_t ah, al;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                uint16_t hi, lo;
                split_bf16(f[j], hi, lo);
                ah[j] = __builtin_bit_cast(__bf16, hi);
                al[j] = __builtin_bit_cast(__bf16, lo);
            }
            bf16x8_t b = fixed;
            if (col < 9) b = *reinterpret_cast<const bf16x8_t *>(xs + ((yl + col / 3) * 3 + col % 3) * H + x0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, b, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b, acc, 0, 0, 0);
        }
    }
    // D: column col, rows co = 8 (v / 4) + 4 kh + v % 4
    if (col < 10) {
#pragma unroll
        for (int v = 0; v < 16; ++v) red[wave][8 * (v / 4) + 4 * kh + v % 4][col] = acc[v];
    }
    __syncthreads();
    for (int e = tid; e < C * 10; e += 256) {
        const int co = e / 10, t = e % 10;
        part[((size_t)blockIdx.x * C + co) * 10 + t] = ((red[0][co][t] + red[1][co][t]) + red[2][co][t]) + red[3][co][t];
    }
}

void launch_bwdw1_mfma(const float *dZ, const uint16_t *X, int n, float *part, float *dW, float *db, hipStream_t st) {
    const int units = n * (IN / kL1Rows);
    const int nch = units < kMaxChunks ? units : kMaxChunks;
    hipLaunchKernelGGL(k_bwdw1_mfma, dim3(nch), dim3(256), 0, st, dZ, X, n, part);
    launch_reduce_parts(part, nch, 1, dW, db, st);
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
    const int nro = (n + 3) / 4;   // readout workgroups (the partials fit the weight-gradient scratch)
    hipLaunchKernelGGL(k_readout_train, dim3(nro), dim3(256), 0, st, h->a[4], h->wb, labels, n, h->dz[4], h->part);
    hipLaunchKernelGGL(k_readout_reduce, dim3(1), dim3(64), 0, st, h->part, nro, n, h->grad, h->loss);
    // layer 4 (8 -> 4), layer 3 (16 -> 8), layer 2 (32 -> 16): weight grads, then data grads
    launch_bwdw_mfma<8, 4, 4>(h->dz[4], h->a[3], n, h->part, h->grad + OFF_W[3], h->grad + OFF_B + 3 * C, st);
    launch_bwdd_mfma<8, 8, 4>(h->dz[4], h->wb + OFF_W[3], h->a[3], h->dz[3], n, st);
    launch_bwdw_mfma<16, 1, 8>(h->dz[3], h->a[2], n, h->part, h->grad + OFF_W[2], h->grad + OFF_B + 2 * C, st);
    launch_bwdd_mfma<16, 2, 8>(h->dz[3], h->wb + OFF_W[2], h->a[2], h->dz[2], n, st);
    launch_bwdw_mfma<32, 1, 4>(h->dz[2], h->a[1], n, h->part, h->grad + OFF_W[1], h->grad + OFF_B + 1 * C, st);
    launch_bwdd_mfma<32, 1, 8>(h->dz[2], h->wb + OFF_W[1], h->a[1], h->dz[1], n, st);
    launch_bwdw1_mfma(h->dz[1], x, n, h->part, h->grad + OFF_W[0], h->grad + OFF_B + 0 * C, st);
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
    hipLaunchKernelGGL(k_readout, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, h->a[4], h->wb, n, probs);
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
