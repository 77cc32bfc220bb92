/*
 * uwb.h -- C ABI of the MI355X (gfx950) library for confocal microwave imaging
 * with a coarse-to-fine segment walk (Ettefagh, Moghaddam, Vahidian, "A Novel
 * Low-Complexity Framework in Ultra-Wideband Imaging for Breast Cancer
 * Detection", arXiv:1709.02549).
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless the comment says "host".  The caller
 *    owns every buffer.  Nothing here allocates device memory, except the plan
 *    objects of the batch interface (which own what they allocate).
 *  - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *    enqueued asynchronously on it; results are ready when the stream is.
 *  - The return value is a status: UWB_OK (0) or a negative UWB_E* code.  All
 *    arguments are validated before anything is enqueued, so an error never
 *    leaves partial work in flight.  No call throws or aborts.
 *  - Traces are not scanned for NaN/Inf: non-finite samples propagate into the
 *    affected voxels.  Antenna positions live in device memory and are not
 *    scanned either; a non-finite position yields non-finite energies, never
 *    an out-of-bounds access.
 *  - Calls are stateless and reentrant; plan objects are not thread-safe.
 */
#ifndef UWB_H
#define UWB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum uwb_status {
    UWB_OK = 0,
    UWB_EINVAL = -1,        /* null pointer, size or value out of its domain */
    UWB_ERANGE = -2,        /* output or workspace too small, too many levels */
    UWB_ENOMEM = -3,        /* allocation inside a plan failed */
    UWB_EHIP = -4,          /* HIP launch or runtime error */
    UWB_EUNSUPPORTED = -5   /* valid request outside what the library handles */
};

enum uwb_beamformer { UWB_DAS = 0, UWB_DMAS = 1, UWB_MVDR = 2 };

/*
 * UWB_MVDR: the Capon (minimum-variance distortionless-response) beamformer that
 * Section I names among the data-adaptive methods (minimum output power with a
 * distortionless response toward the focal point); the paper gives no formula
 * and leaves better beamformers inside its framework to Section V.  At a focal
 * point r, with x_i(k) the aligned window sample of channel i at offset
 * k = -h..h (the same gather as DAS / DMAS) and X = [x_i(k)] (M channels x W):
 *   R   = (1/W) sum_k x(k) x(k)^T          sample covariance over the W offsets
 *   R_l = R + delta I,  delta = UWB_MVDR_LOADING * trace(R) / M   (diagonal loading)
 *   w   = R_l^-1 1 / (1^T R_l^-1 1)         steering vector all ones after alignment
 *   I(r) = sum_k (w^T x(k))^2,   and I = 0 where trace(R) = 0.
 * Computed through the W x W system of the Woodbury identity (the same weights
 * up to rounding): with G = X^T X, b = X^T 1 (the DAS window sums) and
 * A = G + W delta I, c = A^-1 b gives I = (W delta)^2 |c|^2 / (M - b^T c)^2.
 * Windows up to UWB_MVDR_MAX_WINDOW samples (the W x W system lives in registers).
 */
#define UWB_MVDR_LOADING 3.0
#define UWB_MVDR_MAX_WINDOW 11

/* Largest supported energy window (samples) and trace length. */
#define UWB_MAX_WINDOW 31
#define UWB_MAX_SAMPLES 65536

/*
 * One monostatic scan (Section II-A): M antennas at r_i, each recording Y_i.
 *   ant_pos  device [n_ant][3] fp32, metres (z = 0 for a planar setup)
 *   traces   device [n_ant][n_samp] fp32, antenna-major, row stride n_samp;
 *            sample m was taken at time t0 + m*dt
 *   dt       sampling period, s (> 0)
 *   t0       time of sample 0 relative to the excitation peak, s (finite)
 *   v        propagation speed in the medium, m/s (> 0)
 * Requires n_ant >= 1 and 2 <= n_samp <= UWB_MAX_SAMPLES.
 */
typedef struct {
    int32_t n_ant, n_samp;
    const float *ant_pos;
    const float *traces;
    double dt, t0, v;
} uwb_scan;

/*
 * A batch of same-shaped scans, e.g. many acquisitions imaged on one grid.
 *   ant_pos  device [n_scans][n_ant][3] fp32
 *   traces   device [n_scans][n_ant][n_samp] fp32
 *   params   device [n_scans][3] fp64: (dt, t0, v) per scan
 *   v_min, dt_min  host lower bounds of v and dt over the batch (> 0), used to
 *            size on-chip staging; a scan below them gets NaN energies
 */
typedef struct {
    int32_t n_scans, n_ant, n_samp;
    const float *ant_pos;
    const float *traces;
    const double *params;
    double v_min, dt_min;
} uwb_scan_batch;

/*
 * Focal points "according to the desired resolution" (Section II-A): a regular
 * grid of voxel centres  r(ix,iy,iz) = origin + (ix,iy,iz) * pitch.
 * dims = (nx, ny, nz), each >= 1; nz == 1 is a planar (2D) image.  Images are
 * stored [nz][ny][nx] fp32, x fastest.  pitch must be finite and > 0.
 */
typedef struct {
    double origin[3];
    double pitch[3];
    int32_t dims[3];
} uwb_grid;

/*
 * DAS energy image, Eq. (3) with the Eq. (1) delay:
 *   tau_i(r) = (2 |r - r_i| / v - t0) / dt            (round trip, in samples)
 *   s_i(r,k) = Y_i at fractional sample tau_i(r) + k (linear interpolation,
 *              zero outside [0, n_samp)),  k = -h..h,  window = 2h+1
 *   I(r)     = sum_k ( sum_i s_i(r,k) )^2
 * window: odd, 1 <= window <= UWB_MAX_WINDOW (11 in the reference workloads).
 * img: device [nz][ny][nx] fp32, written entirely.  FP32 arithmetic.
 */
int uwb_das(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img, void *stream);

/*
 * DMAS energy image (Section II-B): the aligned signals are multiplied in
 * pairs and the products summed before the windowed energy,
 *   I(r) = sum_k ( sum_{i<j} s_i(r,k) s_j(r,k) )^2 .
 * Same arguments and layout as uwb_das.  FP32 arithmetic; the pairwise sum is
 * regrouped as sum_j s_j * (sum_{i<j} s_i), which is exact in real arithmetic.
 */
int uwb_dmas(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img, void *stream);

/* Batched forms: img is device [n_scans][nz][ny][nx]. */
int uwb_das_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img,
                  void *stream);
int uwb_dmas_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img,
                   void *stream);

/*
 * Both images in one pass.  The DMAS sum is accumulated as sum_j s_j A_j with
 * A_j = sum_{i<j} s_i (Section II-B); once every antenna is in, A is the DAS
 * window sum of Eq. (3).  These calls write the DMAS image (img_dmas, as
 * uwb_dmas) and the DAS image (img_das, I = sum_k A_k^2) of the same scans from
 * one launch, at the cost of the DMAS image alone.  The DAS values are those of
 * uwb_das up to FP32 rounding (the interpolated sample is formed once and then
 * added, where uwb_das folds it into the sum directly); the DMAS values equal
 * uwb_dmas's bit for bit.  img_das and img_dmas: device, the uwb_das layout
 * ([n_scans][nz][ny][nx] for the batch forms), caller-owned, not overlapping
 * (else UWB_EINVAL); other arguments and errors as uwb_das / uwb_das_batch.
 */
/*
 * Capon / MVDR energy image (UWB_MVDR above): the same gather as uwb_das, the
 * weights adapted per focal point.  window: odd, 1 <= window <= UWB_MVDR_MAX_WINDOW
 * (UWB_EUNSUPPORTED beyond).  img: device, the uwb_das layout, written entirely.
 * FP32 arithmetic (the W x W solve too: its system is normalised, see above).
 * The _batch form images same-shaped scans as uwb_das_batch; the _multistatic
 * forms take the M^2 channels of uwb_das_multistatic (M counts channels there).
 * Detection and the segment walk accept UWB_MVDR as their beamformer.
 */
int uwb_mvdr(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img, void *stream);
int uwb_mvdr_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img, void *stream);
int uwb_mvdr_multistatic(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img, void *stream);
int uwb_mvdr_multistatic_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img,
                               void *stream);

int uwb_das_dmas(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img_das, float *img_dmas,
                 void *stream);
int uwb_das_dmas_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img_das,
                       float *img_dmas, void *stream);

/*
 * Detection (Section II-A): the tumour is at the voxel of maximal energy.
 * The decision is taken in FP64 so it does not depend on FP32 rounding:
 * every voxel whose FP32 energy is within 1e-3 (relative) of the FP32 maximum
 * is re-evaluated in FP64 from the scan, and the winner is the lowest linear
 * index (x fastest) among candidates whose FP64 energy is >= max - 1e-12*|max|.
 *   img      the image produced by uwb_das / uwb_dmas for the same scan
 *   out      device uwb_peak (one per scan for the batch form)
 *   workspace/workspace_bytes  device scratch of at least
 *            uwb_argmax_workspace_bytes(grid, n_scans) bytes
 */
typedef struct {
    int64_t index;          /* linear voxel index, x fastest */
    double value;           /* FP64 energy of that voxel */
    float value32;          /* its FP32 image value */
    int32_t candidates;     /* voxels re-evaluated in FP64 */
} uwb_peak;

size_t uwb_argmax_workspace_bytes(const uwb_grid *grid, int32_t n_scans);
int uwb_argmax(const uwb_scan *scan, const uwb_grid *grid, int32_t window, int32_t beamformer,
               const float *img, uwb_peak *out, void *workspace, size_t workspace_bytes, void *stream);
int uwb_argmax_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window,
                     int32_t beamformer, const float *img, uwb_peak *out, void *workspace,
                     size_t workspace_bytes, void *stream);

/*
 * Imaging and detection without a second pass over the images (Section II-A
 * detection fused with the Eq. (3) / Section II-B images).  The full-resolution
 * DAS / DMAS launch works in tiles of voxels (16 x 64 in 2D, 8 x 8 x 16 in 3D);
 * uwb_das_dmas_batch_tilemax is uwb_das_dmas_batch that also writes every
 * tile's FP32 maximum of each image, and uwb_argmax_batch_tilemax is
 * uwb_argmax_batch that takes the maxima from those instead of reading the
 * whole image for them: it reads the image only in the tiles whose maximum
 * comes within 1e-3 of the scan's.  The uwb_peak records are identical to
 * uwb_argmax_batch's on the same image (same candidates, same FP64 decision).
 *   uwb_image_tiles(grid)   tiles per scan (the length of one scan's maxima);
 *                           negative status for an invalid grid
 *   tmax_das, tmax_dmas     device [n_scans][uwb_image_tiles(grid)] fp32,
 *                           caller-owned, overlapping neither each other nor
 *                           the images (else UWB_EINVAL)
 *   tmax (detection)        the maxima written for img by the imaging call on
 *                           the same scans, grid and window; beamformer
 *                           UWB_DAS or UWB_DMAS only (else UWB_EINVAL)
 *   workspace               device, >= uwb_argmax_tilemax_workspace_bytes(grid,
 *                           n_scans) bytes (else UWB_ERANGE)
 * Other arguments and errors as uwb_das_dmas_batch / uwb_argmax_batch.
 */
int64_t uwb_image_tiles(const uwb_grid *grid);
int uwb_das_dmas_batch_tilemax(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img_das,
                               float *img_dmas, float *tmax_das, float *tmax_dmas, void *stream);
size_t uwb_argmax_tilemax_workspace_bytes(const uwb_grid *grid, int32_t n_scans);
int uwb_argmax_batch_tilemax(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, int32_t beamformer,
                             const float *img, const float *tmax, uwb_peak *out, void *workspace,
                             size_t workspace_bytes, void *stream);

/*
 * Allocation-free detection, for callers that cannot allocate device memory
 * while they run: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The same computation and result as uwb_argmax_batch
 * (same kernels, same rule, bit-identical uwb_peak records), with its scratch
 * taken from a device array the library holds instead of a workspace argument.
 *   scans, grid, window, beamformer, img, out   as uwb_argmax_batch (device
 *            img and out, caller-owned)
 *   Limit: uwb_argmax_workspace_bytes(grid, n_scans) must not exceed
 *          UWB_ARGMAX_SCRATCH_BYTES (4 MiB: e.g. 256 scans of 512 x 512, or one
 *          256^3 volume); a larger request returns UWB_ERANGE before anything
 *          is launched.
 *   The array is one per GPU (the current device, hipGetDevice, whose queue
 *   `stream` must be), held from the first call on that device until the
 *   process ends.  Calls on one GPU share it: calls that overlap on that GPU
 *   (concurrent streams, or host threads) race and may return wrong results;
 *   serialise them (one stream, or events).  Calls no hipMalloc / hipFree.
 *   Errors: as uwb_argmax_batch; UWB_ERANGE as above; UWB_EHIP if the device
 *   address of the array cannot be obtained.
 */
#define UWB_ARGMAX_SCRATCH_BYTES (4u << 20)
int uwb_argmax_batch_noalloc(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window,
                             int32_t beamformer, const float *img, uwb_peak *out, void *stream);

/*
 * Coarse-to-fine segment walk (Section III).
 *
 * walk = UWB_WALK_PAPER follows the three phases as written: one image of the
 *   whole grid on a lattice decimated by D (points at D*k + floor(D/2) along each
 *   axis; D manual, or automatic from the smallest tumour to detect, see
 *   uwb_auto_decimation); then ROI selection: split the current box into 4
 *   (8 in 3D) at x0 + floor(side/2), score each child on the decimated samples
 *   inside it, keep the best, widen it by the sliding frame
 *   floor(frame_level * child side) on each end (clipped to the grid), repeat;
 *   stop when a child would hold fewer than 4 samples, after max_depth
 *   splits, or by the W/B rule.
 * walk = UWB_WALK_PER_LEVEL re-images every box on a g^d lattice (step
 *   side/g); boxes stay aligned (grid side = g * 2^L), frame_level only widens
 *   each child's scoring set, and the walk ends at box side g.
 * In both modes the final ROI is the last box widened by
 *   floor(frame_final * side) on each end, imaged at full resolution; the
 *   detection is its maximal-energy voxel (same rule as uwb_argmax).
 *
 * Metrics (Section III, decision metric): mean, population variance, max,
 *   max/mean, and Eq. (5): M = (1 - a) mu_c + a var_c with
 *   a = (var_c - var_p) / var_c (a = 0 if var_c = 0), var_p being the variance
 *   of the parent box's samples; Eq. (5) values are divided by the parent's
 *   sample maximum first.  UWB_EQ5_CLAMPED clamps a to [0, 1].
 * term = UWB_TERM_WB adds the Eq. (6)-(7) stop: with the previous and the
 *   current box's samples as the two classes, W = sum of squared deviations
 *   from the class means, B = sum_class n (class mean - pooled mean)^2; the first
 *   split always proceeds, a later one stops the walk unless B grows and W
 *   shrinks, and that split is undone.
 * Ties among children (and voxels): lowest index among values
 *   >= max - 1e-12*|max|.  All decisions are taken in FP64.
 */
typedef enum { UWB_MEAN = 0, UWB_VAR = 1, UWB_EQ5 = 2, UWB_MAX = 3, UWB_MAX_OVER_MEAN = 4,
               UWB_EQ5_CLAMPED = 5 } uwb_metric;
typedef enum { UWB_TERM_FIXED_DEPTH = 0, UWB_TERM_WB = 1 } uwb_term;
typedef enum { UWB_WALK_PER_LEVEL = 0, UWB_WALK_PAPER = 1 } uwb_walk;

typedef struct {
    int32_t beamformer;     /* UWB_DAS, UWB_DMAS or UWB_MVDR (window <= UWB_MVDR_MAX_WINDOW) */
    int32_t walk;           /* uwb_walk */
    int32_t coarse;         /* g, even, 2..64 (PER_LEVEL); g^d <= 4096 */
    int32_t decimation;     /* D >= 1 (PAPER); 0 = automatic from min_tumour */
    double min_tumour;      /* metres, automatic D */
    int32_t max_depth;      /* 0 = as deep as the mode allows; <= UWB_MAX_LEVELS */
    int32_t metric;         /* uwb_metric */
    int32_t term;           /* uwb_term */
    double frame_level;     /* >= 0 */
    double frame_final;     /* >= 0 */
} uwb_segment_tree;

#define UWB_MAX_LEVELS 16

typedef struct {
    int32_t n_levels;                       /* splits kept */
    int32_t term_level;                     /* splits made (n_levels + 1 if W/B undid one) */
    int32_t decimation;                     /* D used (PAPER), 0 otherwise */
    int32_t n_samples_level0;               /* lattice points of the first image */
    int32_t child[UWB_MAX_LEVELS];          /* Morton child (bx + 2 by + 4 bz) per split made */
    int32_t box[UWB_MAX_LEVELS + 1][6];     /* finest-voxel [x0,x1,y0,y1,z0,z1) before/after each split */
    double score[UWB_MAX_LEVELS][8];        /* child metrics per split made */
    double wb[UWB_MAX_LEVELS + 1][2];       /* (W, B) of iterations 1, 2, ... */
    int32_t n_wb;                           /* entries of wb written */
    int32_t roi[6];                         /* final ROI box */
    int64_t argmax;                         /* finest-grid linear index, x fastest */
    double peak;                            /* FP64 energy there */
    int64_t voxels_evaluated;               /* focal points beamformed in total */
    int32_t learned_mask;                   /* learned walk: bit l set if the CNN decided split l */
    int32_t guard_hits;                     /* ROI voxels whose FP32 energy came within 1e-3 of the
                                               ROI's FP32 maximum and were re-evaluated in FP64 to
                                               decide the detection (>= 1 when argmax >= 0) */
} uwb_segment_result;

/*
 * Multistatic imaging (Eq. (2) and Eq. (4)): every one of the M antennas
 * transmits and every one receives.  scan->n_ant = M (<= 256), scan->ant_pos
 * [M][3], scan->traces [M * M][n_samp] fp32 with channel i * M + j the signal
 * sent by antenna i and received on antenna j.  The delay of channel (i, j) is
 * the transmitter-to-point plus point-to-receiver path,
 *   n_ij(r) = ((|r - a_i| + |r - a_j|) / v - t0) / dt
 * (Eq. (1) when i = j).  DAS is Eq. (4), the sum over all M^2 channels; DMAS
 * takes the pairwise products of Section II-B over all pairs of distinct
 * channels.  Batch forms: n_ant = M, traces [n_scans][M * M][n_samp].
 * Everything else (images, workspace sizes, argmax rule, walk semantics and
 * errors) as the monostatic calls; the learned walk and batch plans are
 * monostatic only.
 */
int uwb_das_multistatic(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img, void *stream);
int uwb_dmas_multistatic(const uwb_scan *scan, const uwb_grid *grid, int32_t window, float *img, void *stream);
int uwb_das_multistatic_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img,
                              void *stream);
int uwb_dmas_multistatic_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window, float *img,
                               void *stream);
/* Both multistatic images in one pass (as uwb_das_dmas_batch, Eq. (2) delays). */
int uwb_das_dmas_multistatic_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window,
                                   float *img_das, float *img_dmas, void *stream);
int uwb_argmax_multistatic(const uwb_scan *scan, const uwb_grid *grid, int32_t window, int32_t beamformer,
                           const float *img, uwb_peak *out, void *workspace, size_t workspace_bytes, void *stream);
int uwb_argmax_multistatic_batch(const uwb_scan_batch *scans, const uwb_grid *grid, int32_t window,
                                 int32_t beamformer, const float *img, uwb_peak *out, void *workspace,
                                 size_t workspace_bytes, void *stream);
int uwb_segment_refine_multistatic(const uwb_scan *scan, const uwb_grid *finest, int32_t window,
                                   const uwb_segment_tree *tree, uwb_segment_result *out, float *roi_img,
                                   int64_t roi_capacity, void *workspace, size_t workspace_bytes, void *stream);
int uwb_segment_refine_multistatic_batch(const uwb_scan_batch *scans, const uwb_grid *finest, int32_t window,
                                         const uwb_segment_tree *tree, uwb_segment_result *out, float *roi_img,
                                         int64_t roi_capacity, void *workspace, size_t workspace_bytes,
                                         void *stream);

/* Largest ROI (voxels) the walk can end with for this grid and tree: the
   minimum roi_capacity.  Negative status on invalid arguments. */
int64_t uwb_segment_roi_capacity(const uwb_grid *finest, const uwb_segment_tree *tree);
/* Device workspace bytes needed by uwb_segment_refine(_batch) for n_scans. */
size_t uwb_segment_workspace_bytes(const uwb_grid *finest, const uwb_segment_tree *tree, int32_t n_scans);

/*
 * out:       device uwb_segment_result (one per scan for the batch form)
 * roi_img:   device fp32 [roi_capacity] per scan (batch: scan s at
 *            s * roi_capacity), the final ROI image [z][y][x] of the ROI box,
 *            imaged in FP32 (the detection in out is decided in FP64 over the
 *            voxels within 1e-3 of its maximum, as for a full image); may be NULL
 * roi_capacity: >= uwb_segment_roi_capacity(...), else UWB_ERANGE
 */
int uwb_segment_refine(const uwb_scan *scan, const uwb_grid *finest, int32_t window,
                       const uwb_segment_tree *tree, uwb_segment_result *out, float *roi_img,
                       int64_t roi_capacity, void *workspace, size_t workspace_bytes, void *stream);
int uwb_segment_refine_batch(const uwb_scan_batch *scans, const uwb_grid *finest, int32_t window,
                             const uwb_segment_tree *tree, uwb_segment_result *out, float *roi_img,
                             int64_t roi_capacity, void *workspace, size_t workspace_bytes,
                             void *stream);

/*
 * The check the paper proposes for scans that may hold no tumour (Section IV,
 * last paragraph): run the three-phase walk (tree->walk must be
 * UWB_WALK_PAPER) with two different decimation factors d1 != d2 (>= 1); the
 * detection is confirmed when the two final ROIs point to the same place,
 * read here as: the two ROI boxes intersect.
 *   out      device uwb_segment_result [2][n_scans]: the d1 walks, then the d2 walks
 *   agree    device int32 [n_scans]: 1 = ROIs intersect (confirmed), 0 = they do not
 *            (the walks followed artifacts: no tumour)
 * Workspace: uwb_tumour_check_workspace_bytes (0 for invalid arguments).
 */
size_t uwb_tumour_check_workspace_bytes(const uwb_grid *finest, const uwb_segment_tree *tree, int32_t d1, int32_t d2,
                                        int32_t n_scans);
int uwb_tumour_check_batch(const uwb_scan_batch *scans, const uwb_grid *finest, int32_t window,
                           const uwb_segment_tree *tree, int32_t d1, int32_t d2, uwb_segment_result *out,
                           int32_t *agree, void *workspace, size_t workspace_bytes, void *stream);

/*
 * The walk of uwb_segment_refine_batch plus its mixed-resolution image (the
 * final-imaging phase of Section III: one region at full resolution, the rest
 * at low resolution).  composite: device [n_scans][nz][ny][nx] fp32.  Inside
 * each scan's ROI it holds the full-resolution energy; elsewhere every voxel
 * holds the coarse sample whose block contains it: the decimated lattice of the
 * paper walk (block [D k, D k + D) per axis, the last block running to the
 * grid's end), or, for the per-level walk, the deepest imaged level whose box
 * contains the voxel (block [x0 + D_l k, x0 + D_l (k + 1)) of that box).
 * Other arguments, sizes and errors as uwb_segment_refine_batch.
 */
int uwb_segment_composite_batch(const uwb_scan_batch *scans, const uwb_grid *finest, int32_t window,
                                const uwb_segment_tree *tree, uwb_segment_result *out, float *roi_img,
                                int64_t roi_capacity, void *workspace, size_t workspace_bytes, float *composite,
                                void *stream);

/*
 * Batched serving of uneven scans: many scans, each with its own antenna
 * count, trace length and grid, imaged (DAS or DMAS, as uwb_das / uwb_dmas)
 * by one persistent launch that is captured once into a HIP graph.
 *
 * uwb_batch_plan_create copies per-scan descriptors and the (scan, tile) work
 * list to device memory it owns and captures the graph.  The item array is
 * host memory and is not kept; the scans' traces, positions and output
 * images are device buffers that must stay valid while the plan is run.
 * All scans of a plan are planar (nz == 1) or all volumetric.
 * uwb_batch_run enqueues one replay on `stream`.
 * uwb_batch_autotune times every candidate configuration on this batch
 * (`reps` replays each, on `stream`, synchronising) and keeps, among those
 * within 2 % of the fastest, the one whose median scan completes first (the
 * serving latency); if the environment variable UWB_TUNE_CACHE names a file, it
 * records the choice there, and a later plan of the same batch shape created
 * with cfg == NULL reuses it.
 * uwb_batch_timestamps synchronises `stream` and returns, per scan, the time
 * from the start of the last replay to the moment its last tile finished
 * (ns, device clock; -1 if not finished).
 * uwb_batch_set_config / uwb_batch_autotune rebuild the plan's device state:
 * no replay of the plan may be in flight.
 */
typedef struct {
    uwb_scan scan;
    uwb_grid grid;
    float *img;             /* device [nz][ny][nx] fp32 */
} uwb_batch_item;

typedef struct {
    int32_t vpl;            /* voxels per lane: 1, 2 or 4 (planar tile 16 x 16*vpl; volumetric uses 2) */
    int32_t wgs_per_cu;     /* resident workgroups per compute unit, 1..32 */
    int32_t lds_kb;         /* LDS staging budget per workgroup in KiB, 4..60 (sets the antenna chunk) */
    int32_t order;          /* 0: scans by decreasing cost (tiles x antennas); 1: as given */
} uwb_batch_config;

typedef struct uwb_batch_plan uwb_batch_plan;

int uwb_batch_plan_create(uwb_batch_plan **plan, const uwb_batch_item *items, int32_t n_scans,
                          int32_t beamformer, int32_t window, const uwb_batch_config *cfg);
int uwb_batch_run(uwb_batch_plan *plan, void *stream);
int uwb_batch_autotune(uwb_batch_plan *plan, int32_t reps, void *stream, uwb_batch_config *best);
int uwb_batch_get_config(const uwb_batch_plan *plan, uwb_batch_config *cfg);
int uwb_batch_set_config(uwb_batch_plan *plan, const uwb_batch_config *cfg);
int uwb_batch_timestamps(uwb_batch_plan *plan, int64_t *done_ns, void *stream);
int uwb_batch_plan_destroy(uwb_batch_plan *plan);

/*
 * Learned segment proposer (extension): a small CNN that scores the four
 * children of a quadtree box from the box's 32 x 32 coarse DAS energy image,
 * normalised by its maximum.
 *   conv3x3(1->32, stride 1) ReLU -> 3 x [conv3x3(32->32, stride 2) ReLU]
 *   child c = bx + 2 by: mean of the 2 x 2 cells of quadrant (bx, by) -> 32
 *   features -> shared linear 32 -> 1 -> 4 logits -> softmax.
 * Zero padding 1.  BF16 weights and activations, FP32 accumulation; FP32
 * master weights, gradients and Adam moments (beta 0.9 / 0.999, eps 1e-8).
 * Parameters (uwb_cnn_param_count() = 28097 floats) are flat, in the order
 * conv weights 1..4 ([32][Cin][3][3] each), conv biases 1..4 ([32] each),
 * readout weight [32], readout bias.
 *   x        device [n][32][32] BF16 (uint16 bit patterns), n <= max_batch
 *   labels   device [n] int32 in 0..3 (the child holding the target); a sample
 *            with any other label is masked out (no loss, no gradient; the
 *            mean still divides by n)
 *   probs    device [n][4] fp32
 *   grad_out device [28097] fp32 (may be NULL); loss_out device fp32 (may be NULL)
 * The handle owns its device buffers.  Calls on one handle must not overlap.
 * uwb_cnn_get_state / set_state move the checkpoint (masters, moments, step)
 * through host buffers of 28097 floats each, synchronising `stream`.
 */
typedef struct uwb_cnn uwb_cnn;
int uwb_cnn_param_count(void);
int uwb_cnn_create(uwb_cnn **cnn, int32_t max_batch, const float *init_params /* host */);
int uwb_cnn_destroy(uwb_cnn *cnn);
int uwb_cnn_forward(uwb_cnn *cnn, const uint16_t *x, int32_t n, float *probs, void *stream);
int uwb_cnn_gradients(uwb_cnn *cnn, const uint16_t *x, const int32_t *labels, int32_t n, float *grad_out,
                      float *loss_out, void *stream);
int uwb_cnn_train_step(uwb_cnn *cnn, const uint16_t *x, const int32_t *labels, int32_t n, float lr,
                       float *loss_out, void *stream);
int uwb_cnn_get_state(uwb_cnn *cnn, float *theta, float *m, float *v, int64_t *step, void *stream);
int uwb_cnn_set_state(uwb_cnn *cnn, const float *theta, const float *m, const float *v, int64_t step,
                      void *stream);
const uint16_t *uwb_cnn_weights_bf16(const uwb_cnn *cnn);

/*
 * Learned walk: the per-level quadtree walk (planar grid, g = 32, fixed depth)
 * in which, at every split, the CNN scores the children from the box's coarse
 * DAS lattice; its child is kept when its probability is >= threshold,
 * otherwise the tree's metric decides (on the same FP64 lattice).  The final
 * ROI is imaged with the tree's beamformer as in uwb_segment_refine.
 * learned_mask bit l of each result tells which splits the CNN decided.
 * Requires n_scans <= the CNN's max_batch.  Workspace: uwb_learned_workspace_bytes.
 */
size_t uwb_learned_workspace_bytes(const uwb_grid *finest, const uwb_segment_tree *tree, int32_t n_scans);
int uwb_learned_refine_batch(const uwb_scan_batch *scans, const uwb_grid *finest, int32_t window,
                             const uwb_segment_tree *tree, uwb_cnn *cnn, float threshold,
                             uwb_segment_result *out, float *roi_img, int64_t roi_capacity, void *workspace,
                             size_t workspace_bytes, void *stream);

/*
 * Training inputs of the proposer: for every scan and every level l of the
 * per-level walk (g = 32) the aligned box of side N / 2^l holding targets[scan]
 * (e.g. the full-resolution DMAS detection) is imaged on its 32 x 32 lattice
 * (DAS, FP64, normalised by its maximum) into x [scan * L + l] (BF16), and
 * labels[scan * L + l] receives the child that holds the target.  A target
 * index outside the grid yields zero inputs and label -1 for that scan (masked
 * out by the training calls).
 * L = uwb_cnn_input_levels(finest) = log2(N / 32).
 */
int32_t uwb_cnn_input_levels(const uwb_grid *finest);
int uwb_cnn_training_inputs(const uwb_scan_batch *scans, const uwb_grid *finest, int32_t window,
                            const uwb_peak *targets, uint16_t *x, int32_t *labels, void *stream);

/*
 * GPU generator of seeded synthetic planar scans (training data of the learned
 * proposer): one tumour and n_clutter point scatterers in a disc of `radius`
 * around the origin, echoes of the pulse sin(2 pi f0 t) exp(-t^2/2 sigma^2) /
 * pulse_peak (|t| <= 6 sigma) with 1/r^2 amplitude (1 at 1 cm), white noise at
 * snr_db.  Scene parameters come from SplitMix64(seed ^ (salt << 56)), noise
 * from Philox4x32-10 keyed by the seed, so the host generator draws the same
 * scan for the same seed.
 *   ant_pos  device [n_ant][3] fp32 (shared by every scan)
 *   seeds    device [n] uint64
 *   traces   device [n][n_ant][n_samp] fp32 (n_samp <= 2048)
 *   tumours  device [n][3] fp64 tumour positions, or NULL
 */
typedef struct {
    int32_t n_ant, n_samp, n_clutter;
    double v, dt, t0, radius, snr_db;
    double pulse_f0, pulse_sigma, pulse_peak;
    uint64_t salt;
} uwb_gen_recipe;
int uwb_generate_disc_scans(const uwb_gen_recipe *recipe, const float *ant_pos, const uint64_t *seeds, int32_t n,
                            float *traces, double *tumours, void *stream);

/*
 * Automatic spatial decimation factor (Section III; worked example in
 * Section IV): one focal point per square inscribed in the smallest tumour,
 * D = floor(min_tumour / (sqrt(2) * pitch)), at least 1.  Host-only, pure.
 * Returns D >= 1, or UWB_EINVAL for non-finite or non-positive arguments.
 */
int uwb_auto_decimation(double min_tumour, double pitch);

/* Static description of a status code (never NULL). */
/*
 * Machine probe: the LDS read bandwidth of the device, the on-chip resource the
 * gather of the imaging kernels draws on (W + 1 staged samples per voxel-antenna,
 * Eq. (3)).  Launches n_groups workgroups of 256 lanes, each streaming `iters`
 * reads of `width` bytes (4, 8 or 16: ds_read_b32 / _b64 / _b128) per lane from a
 * 32 KiB LDS array with conflict-free addresses, and times the launch with HIP
 * events.  Synchronous: returns after the stream has drained.
 *   iters       >= 8, a multiple of 8
 *   n_groups    1 .. 65536 (use many per CU to fill the device)
 *   bytes_per_s host out: LDS bytes read per second over the whole device
 *   clock_hz    host out: the shader clock measured during the loop (median over
 *               workgroups of the cycle counter against the constant 100 MHz counter)
 * Allocates and frees a small device buffer (the values read are written out so
 * that no read is dropped).  Errors: UWB_EINVAL for out-of-range arguments,
 * UWB_ENOMEM, UWB_EHIP.
 */
int uwb_probe_lds_read(int32_t width, int32_t iters, int32_t n_groups, double *bytes_per_s, double *clock_hz,
                       void *stream);

const char *uwb_status_string(int status);

/* Library version string, e.g. "uwb 0.1 gfx950". */
const char *uwb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* UWB_H */
