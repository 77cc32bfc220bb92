// Full-resolution FP32 DAS / DMAS imaging (Eq. (1) delay, Eq. (3) DAS, the
// pairwise DMAS of Section II-B) for gfx950, and the Capon / MVDR beamformer
// named in Section I on the same gather.
//
// A workgroup (256 lanes = 4 wave64) owns a tile of voxels; every lane owns
// VPL voxels.  For a chunk of antennas the workgroup first derives, per
// antenna, the interval of samples that any voxel of its tile can touch (the
// delay range over the tile's bounding box, computed in FP64, plus the window
// and a sample of margin) and stages those intervals from HBM into LDS with
// coalesced loads (zero outside the recorded trace).  Each lane then, per
// antenna, computes the round-trip delay in registers (one sqrt), reads the
// W+1 consecutive staged samples around it and accumulates the linearly
// interpolated window into W FP32 accumulators:
//   DAS : S_k += s_k
//   DMAS: P_k += s_k * A_k ; A_k += s_k   (A_k = sum of earlier antennas), which
//         regroups sum_{i<j} s_i s_j exactly and keeps the direct sum's error bound.
//   MVDR: S_k += s_k and the Gram matrix G_kl += s_k s_l (one voxel per lane),
//         solved per voxel through a W x W Cholesky factorisation (mvdr_energy).
// The energy sum_k S_k^2 (or P_k^2, or the MVDR output energy) is written once per voxel.  No atomics,
// fixed summation order: results are bitwise reproducible and independent of
// the tile shape.
//
// A DMAS launch can also write the DAS image: the running sums A_k are the DAS
// window sums, so it costs one more energy per voxel and no extra reads.
//
// The tile body is shared by two kernels: k_image32 maps blockIdx to (tile,
// scan) for same-shaped batches; k_batch32 is a persistent kernel that pulls
// (scan, tile) items of uneven scans from a work list (see batch.hip).
#include <algorithm>

#include "image32.h"

namespace uwb {

void tile_shape(bool d3, int vpl, int *tx, int *ty, int *tz) {
    if (d3) { *tx = 8; *ty = 8; *tz = 4 * vpl; }
    else { *tx = 16; *ty = 16 * vpl; *tz = 1; }
}

namespace {

// Voxels per lane of the grid-mapped kernel: 4 (tiles of 16 x 64 in 2D, 8 x 8 x 16 in 3D)
// measured a few per cent faster than 2 for DAS and DMAS on the 512 x 512 batch.
constexpr int kImageVpl = 4;

// Tiles along x a workgroup images from one staging of the traces, when every channel fits one chunk and
// the launch keeps at least kGroupMinWorkgroups workgroups (a few per CU slot): the staging pass, about
// 7 % of a 512 x 512 DMAS launch with one tile per workgroup, is then paid once per four tiles.
constexpr int kGroupTiles = kMaxSubtiles;
constexpr int64_t kGroupMinWorkgroups = 4096;

}  // namespace

void full_tile_shape(bool d3, int *tx, int *ty, int *tz) { tile_shape(d3, kImageVpl, tx, ty, tz); }

namespace {

struct Args {
    ScanSet ss;
    GridView g;
    float *img;
    float *img_das;         // DMAS launch, optional: the DAS images too (same layout)
    int64_t img_stride;     // elements between scans
    float *tmax, *tmax_das; // optional: each tile's FP32 maximum of img / img_das, [scan][tiles]
    int tiles;              // tiles per scan
    int tiles_x, tiles_y;   // tiles along x and y (z = rest)
    int rs;                 // staged samples per antenna (stride in LDS)
    int chunk;              // antennas staged per pass
    int subtiles;           // tiles along x per workgroup, imaged from one staging
    int groups_x;           // workgroups along x: ceil(tiles_x / subtiles)
};

// Voxels per lane of a beamformer: MVDR keeps a W x W Gram matrix per voxel, one voxel per lane.
template <int BF> constexpr int image_vpl() { return BF == UWB_MVDR ? 1 : kImageVpl; }

// Waves per SIMD asked of the register allocator: DMAS three (168 VGPRs), DAS four (the
// multistatic DAS kernel otherwise settles at three, 9 % slower), MVDR two.
template <int BF, int W, bool D3, bool MS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(BF == UWB_MVDR ? 2 : BF == UWB_DAS ? 4 : 3)))
void k_image32(const Args a) {
    constexpr int VPL = image_vpl<BF>();
    extern __shared__ __align__(16) float smem[];
    const int scan = blockIdx.y;
    const ScanConst sc = scan_const(a.ss, scan);
    int tx, ty, tz;
    TileShape<D3, VPL>::get(tx, ty, tz);
    TileJob j;
    j.pos = sc.pos;
    j.tr = sc.tr;
    j.img = a.img + (int64_t)scan * a.img_stride;
    j.img_das = a.img_das ? a.img_das + (int64_t)scan * a.img_stride : nullptr;
    const int g = blockIdx.x, gx = g % a.groups_x, gyz = g / a.groups_x;   // gyz = tile row (y, z)
    const int64_t slot = (int64_t)scan * a.tiles + (int64_t)gyz * a.tiles_x + gx * a.subtiles;   // first sub-tile's
    j.tmax = a.tmax ? a.tmax + slot : nullptr;
    j.tmax_das = a.tmax_das ? a.tmax_das + slot : nullptr;
    j.M = a.ss.n_ant;
    j.T = a.ss.n_samp;
    j.s = sc.s;
    j.t0s = sc.t0s;
    j.g = a.g;
    j.tx0 = gx * a.subtiles * tx;
    j.ty0 = (gyz % a.tiles_y) * ty;
    j.tz0 = (gyz / a.tiles_y) * tz;
    j.subtiles = a.subtiles;
    j.rs = a.rs;
    j.chunk = a.chunk;
    j.ms = a.ss.ms;
    if (!MS && j.t0s == 0.0) image_tile<BF, W, D3, VPL, MS, false, true>(j, smem);   // uniform per workgroup
    else image_tile<BF, W, D3, VPL, MS>(j, smem);
}

template <int BF, int W>
hipError_t launch_w(bool d3, dim3 grid, size_t lds, hipStream_t st, const Args &a) {
    if (a.ss.ms) {
        if (d3) hipLaunchKernelGGL((k_image32<BF, W, true, true>), grid, dim3(kBlock), lds, st, a);
        else hipLaunchKernelGGL((k_image32<BF, W, false, true>), grid, dim3(kBlock), lds, st, a);
    } else {
        if (d3) hipLaunchKernelGGL((k_image32<BF, W, true, false>), grid, dim3(kBlock), lds, st, a);
        else hipLaunchKernelGGL((k_image32<BF, W, false, false>), grid, dim3(kBlock), lds, st, a);
    }
    return hipGetLastError();
}

template <int BF>
hipError_t launch_bf(int window, bool d3, dim3 grid, size_t lds, hipStream_t st, const Args &a) {
    switch (window) {
#define UWB_W(w) case w: return launch_w<BF, w>(d3, grid, lds, st, a);
        UWB_WINDOWS(UWB_W)
#undef UWB_W
    }
    return hipErrorInvalidValue;
}

template <>
hipError_t launch_bf<UWB_MVDR>(int window, bool d3, dim3 grid, size_t lds, hipStream_t st, const Args &a) {
    switch (window) {
#define UWB_W(w) case w: return launch_w<UWB_MVDR, w>(d3, grid, lds, st, a);
        UWB_MVDR_WINDOWS(UWB_W)
#undef UWB_W
    }
    return hipErrorInvalidValue;
}

}  // namespace

int launch_image32(int bf, const ScanSet &ss, int n_scans, const GridView &g, int window, float *img,
                   hipStream_t stream, float *img_das, float *tmax, float *tmax_das) {
    if (img_das && bf != UWB_DMAS) return UWB_EINVAL;
    if ((tmax || tmax_das) && bf == UWB_MVDR) return UWB_EINVAL;
    if (tmax_das && !img_das) return UWB_EINVAL;
    if (bf == UWB_MVDR && window > UWB_MVDR_MAX_WINDOW) return UWB_EUNSUPPORTED;
    const bool d3 = g.dims[2] > 1;
    int tx, ty, tz;
    tile_shape(d3, bf == UWB_MVDR ? image_vpl<UWB_MVDR>() : kImageVpl, &tx, &ty, &tz);
    Args a;
    a.ss = ss;
    a.g = g;
    a.img = img;
    a.img_das = img_das;
    a.img_stride = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    a.tiles_x = (g.dims[0] + tx - 1) / tx;
    a.tiles_y = (g.dims[1] + ty - 1) / ty;
    const int tiles_z = (g.dims[2] + tz - 1) / tz;
    // inside a batch the speed may vary per scan: ss.v and ss.dt hold lower bounds
    // over the batch, so this sizes the staging for the largest samples-per-metre
    const double s_max = 2.0 / (ss.v * ss.dt);
    const int64_t tiles = (int64_t)a.tiles_x * a.tiles_y * tiles_z;
    if (tiles > 0x7fffffff || n_scans > 65535) return UWB_EUNSUPPORTED;
    // staging for S tiles side by side along x: S = kGroupTiles when every channel then fits one chunk and
    // the launch still holds enough workgroups to fill the device several times over, else S = 1
    auto plan = [&](int S, int &rs, int &chunk) {
        rs = staged_samples(s_max, (S * tx - 1) * g.pitch[0], (ty - 1) * g.pitch[1], (tz - 1) * g.pitch[2], window,
                            ss.n_samp);
        const int per_ant = rs * 16 + (ss.ms ? 32 : 16);   // staged records of 4 samples + table entries
        if (per_ant > kLdsBudget) return false;
        chunk = std::min(std::min(kLdsBudget / per_ant, kBlock), ss.n_ant);
        return true;
    };
    int S = 1;
    if (a.tiles_x >= kGroupTiles && (tiles / kGroupTiles) * n_scans >= kGroupMinWorkgroups &&
        plan(kGroupTiles, a.rs, a.chunk) && a.chunk >= ss.n_ant)
        S = kGroupTiles;
    else if (!plan(1, a.rs, a.chunk))
        return UWB_EUNSUPPORTED;
    a.subtiles = S;
    a.groups_x = (a.tiles_x + S - 1) / S;
    const size_t lds = (size_t)a.chunk * (a.rs * 16 + (ss.ms ? 32 : 16));
    a.tiles = (int)tiles;
    a.tmax = tmax;
    a.tmax_das = tmax_das;
    const int64_t groups = (int64_t)a.groups_x * a.tiles_y * tiles_z;
    dim3 grid((unsigned)groups, (unsigned)n_scans);
    hipError_t e = bf == UWB_DMAS   ? launch_bf<UWB_DMAS>(window, d3, grid, lds, stream, a)
                   : bf == UWB_MVDR ? launch_bf<UWB_MVDR>(window, d3, grid, lds, stream, a)
                                    : launch_bf<UWB_DAS>(window, d3, grid, lds, stream, a);
    return e == hipSuccess ? UWB_OK : UWB_EHIP;
}

}  // namespace uwb
