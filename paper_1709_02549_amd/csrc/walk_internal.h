// Internal arguments of the segment-walk kernels (not part of the public ABI).
#pragma once

#include "uwb_internal.h"

namespace uwb {

constexpr int kMaxCoarsePoints = 4096;   // g^d lattice values held in LDS per level
constexpr double kMinChildSamples = 4;   // paper walk: stop when a child holds fewer samples

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
    int64_t roi_cap;           // ROI bound: stride of roi64
    double *roi64;             // [n_scans][roi_cap]
    float *roi_img;            // optional, scan s at s * roi_img_stride
    int64_t roi_img_stride;
    uwb_segment_result *out;   // [n_scans]
    // dynamic LDS layout: [coarse values: pmax doubles][stage tables: 3 * stage_ant ints][stage: stage_cap floats]
    int pmax, stage_ant, stage_cap;
    size_t lds_walk, lds_lattice;
    int lattice_stage_cap;
};

int launch_walk(const WalkArgs &a, int n_scans, hipStream_t st);
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
