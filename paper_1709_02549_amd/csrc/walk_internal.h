// Internal arguments of the segment-walk kernels (not part of the public ABI).
#pragma once

#include "uwb_internal.h"

namespace uwb {

constexpr int kMaxCoarsePoints = 4096;   // g^d lattice values held in LDS per level
constexpr double kMinChildSamples = 4;   // paper walk: stop when a child holds fewer samples

// Per-scan state of the level-synchronous per-level walk (workspace).
struct PLState {
    double prev_n, prev_mean, prev_m2, prev_w, prev_b;   // previous level's samples and W/B
    int64_t nvox;                                       // focal points evaluated so far
    int active, n_kept, made, n_wb;
};

struct WalkArgs {
    ScanSet ss;
    GridView g;
    int window, bf;
    int walk, coarse, metric, term, depth;
    double frame_level, frame_final;
    // paper walk: decimated lattice (D, first point, points per axis)
    int decimation;
    int dec_x0[3], dec_cnt[3];
    int64_t dec_count;
    double *dec64;             // [n_scans][dec_count]
    // ROI
    int64_t roi_cap;           // ROI bound: stride of roi32
    int roi_side[3];           // largest ROI side per axis
    float *roi32;              // [n_scans][roi_cap]: FP32 ROI images
    float *roi_img;            // optional, scan s at s * roi_img_stride
    int64_t roi_img_stride;
    uwb_segment_result *out;   // [n_scans]
    // per-level walk: lattice values of the current level and per-scan state
    double *lat64;             // [n_scans][depth + 1][coarse^d]: every level's lattice is kept
    int64_t lat_stride;        // doubles per scan in lat64
    PLState *state;            // [n_scans]
    // dynamic LDS layout: [coarse values: pmax doubles][stage tables: 3 * stage_ant ints][stage: stage_cap floats]
    int pmax, stage_ant, stage_cap;
    size_t lds_walk, lds_lattice;
    int lattice_stage_cap;
};

// FP64 energies on regular lattices (walk_grid.hip).
enum { kGridBox = 0, kGridRoi = 1, kGridFixed = 2 };
struct Grid64Args {
    ScanSet ss;
    GridView g;
    int window, bf;
    int mode;
    int lev, coarse, step;             // kGridBox: coarse^d lattice of res[s].box[lev], step D; kGridFixed: step
    int x0[3], cnt[3];                 // kGridFixed: first point (finest indices) and points per axis
    const uwb_segment_result *res;     // kGridBox, kGridRoi
    const PLState *state;              // kGridBox: inactive scans are skipped (null: none)
    double *out64;                     // scan s at s * out_stride + out_offset, lattice order (x fastest)
    int64_t out_stride, out_offset;
    float *out32;                      // optional FP32 copy
    int64_t out32_stride;
    int lds_bytes;                     // filled by launch_grid64
};
int launch_grid64(Grid64Args a, const int *max_cnt, int max_step, int n_scans, hipStream_t st);
// Every level of the per-level walk in one launch, one workgroup per scan (walk_grid.hip).
int launch_pl_fused(Grid64Args a, const WalkArgs &w, int levels, int n_scans, hipStream_t st);

// Points the workspace pointers of a planned walk into ws (size from plan_walk).
void assign_walk_ws(WalkArgs *a, void *ws, int n_scans);

int launch_walk(const WalkArgs &a, int n_scans, hipStream_t st);
// Final imaging of every scan's ROI (box from its result) with beamformer bf, in FP32 into
// roi32 (and roi_img), and its detection decided in FP64 into the result (walk_roi.hip).
int launch_roi(const WalkArgs &a, int bf, int n_scans, hipStream_t st);
// agree[i] = 1 when the final ROIs of ra[i] and rb[i] intersect.
int launch_roi_overlap(const uwb_segment_result *ra, const uwb_segment_result *rb, int32_t *agree, int n,
                       hipStream_t st);
// Mixed-resolution image [n_scans][nz][ny][nx] from a finished walk's results and workspace.
int launch_composite(const WalkArgs &a, int n_scans, float *img, hipStream_t st);
int launch_learned(const WalkArgs &a, int n_scans, uwb_cnn *cnn, float threshold, uint16_t *xin, float *probs,
                   int *fb_child, int roi_bf, hipStream_t st);
int launch_cnn_inputs(const WalkArgs &a, int n_scans, const uwb_peak *targets, uint16_t *xin, int *labels,
                      hipStream_t st);
void size_walk_lds(WalkArgs *a, int n_ant);

// Host planning of a walk: validates the tree against the grid and fills the
// mode fields of WalkArgs (depth, decimated lattice) plus the ROI bound and the
// workspace size for n_scans.
int plan_walk(const GridView &g, const uwb_segment_tree *t, int n_scans, WalkArgs *a, int64_t *roi_bound,
              size_t *ws_bytes);

}  // namespace uwb
