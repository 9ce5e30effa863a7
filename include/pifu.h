/*
 * pifu.h -- C ABI of libpifu, the MI355X (gfx950) implementation of hierarchical
 * surface localization and mesh-free rendering for a pixel-aligned implicit
 * function (Li et al., "Monocular Real-Time Volumetric Performance Capture",
 * ECCV 2020, Sec. 3.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - A grid with 2^L cells per axis has 2^L + 1 nodes per axis.  Node (i, j, k)
 *    sits at NDC (-1 + 2i/2^Lx, -1 + 2j/2^Ly, -1 + 2k/2^Lz); i runs along x,
 *    j along y, k along z.  Linear node index n = (i * ny + j) * nz + k (z fastest).
 *  - Feature maps are HWC float32 in device memory: F[h][w][c], row h along y,
 *    column w along x.  Pixel coordinates are u = (x+1)/2 (W-1), v = (y+1)/2 (H-1);
 *    texels outside the map contribute 0 (the bilinear sampler of Eq. 1).
 *  - label = [logit > 0]; occupancy p = sigmoid(logit) (the 0.5 level set of Sec. 3).
 *  - Every pointer documented "device" must point to memory of the current HIP
 *    device, owned by the caller.  "host" pointers are read during the call only.
 *  - Every call validates its arguments on the host before any launch and
 *    returns a negative status without touching device memory on failure.
 *    No C++ exception crosses this boundary.
 *  - pifu_occupancy_grid, pifu_render_view and pifu_grid_and_render block until
 *    their work on their streams is complete (the conflict loop's trip count is
 *    read back between waves); results are then visible to later work on any
 *    stream.  The *_async forms enqueue the same work without any host read-back
 *    (graph-capturable) and keep every count in device memory.
 *  - The library never allocates device memory during a call: scratch comes
 *    from the caller's workspace, sized by the matching *_workspace_size query.
 */
#ifndef PIFU_H
#define PIFU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define PIFU_OK 0
#define PIFU_ERR_INVALID_ARGUMENT (-1)   /* null/misaligned pointer, size out of range */
#define PIFU_ERR_WORKSPACE_TOO_SMALL (-2)
#define PIFU_ERR_UNSUPPORTED (-3)        /* device is not gfx950, or unsupported shape */
#define PIFU_ERR_HIP (-4)                /* a HIP runtime call or launch failed */
#define PIFU_ERR_SCRATCH_TOO_SMALL (-5)  /* the options need more workspace than the fixed
                                            scratch of pifu_occupancy_grid_async_noalloc */

/* ---------------------------------------------------------------- enums */
#define PIFU_FIELD_MLP 0          /* Eq. 1: MLP over bilinearly sampled features */
#define PIFU_FIELD_ELLIPSOIDS 1   /* analytic stand-in: k (1 - min_i |M_i (P - c_i)|^2) */
#define PIFU_FIELD_PLANE 2        /* analytic stand-in: a x + b y + c z + d */
#define PIFU_FIELD_CBN 3          /* the appendix's lifting network: soft one-hot depth code and
                                     conditional batch norm on the sampled feature (pifu_cbn) */

#define PIFU_ACT_RELU 1
#define PIFU_ACT_LRELU 2          /* LeakyReLU, negative slope 0.01 */
#define PIFU_ACT_SIGMOID 3
#define PIFU_ACT_TANH 4

#define PIFU_PREC_FP32 0          /* MFMA f32 inputs, f32 accumulation */
#define PIFU_PREC_BF16 1          /* MFMA bf16 inputs, f32 accumulation */
#define PIFU_PREC_FP8 2           /* MFMA OCP e4m3 inputs with per-layer scales, f32 accumulation */
#define PIFU_PREC_FP16 3          /* MFMA IEEE binary16 inputs, f32 accumulation; a value outside
                                     the binary16 range sends the call's evaluations to FP32 */

#define PIFU_MAX_LAYERS 8
#define PIFU_MAX_ELLIPSOIDS 32

typedef void* pifu_stream;        /* a hipStream_t; NULL means the null stream */
typedef struct pifu_ctx pifu_ctx;

/*
 * Fully connected network (the occupancy MLP f_O of Eq. 1, the colour MLP f_T
 * of Eq. 2, or a distilled surrogate).  Layer 0 reads [f; extras] where f is the
 * sampled feature (feat_dim values) and extras are z (n_extra = 1) or z and the
 * occupancy value (n_extra = 2).  Layer l >= 1 reads [h_{l-1}; f] when skip[l]
 * is non-zero, else h_{l-1}.  Hidden layers use hidden_act; the last layer
 * (1 or 3 outputs) is followed by out_act.
 * W[l] is device float32 row-major [widths[l]][in_width(l)], 16-byte aligned;
 * b[l] device float32.  A null or misaligned pointer is INVALID_ARGUMENT.
 * Supported: feat_dim % 32 == 0, hidden widths % 64 == 0, last width <= 4.
 * fp8_amax[l] (host value) is the calibrated max |input| of layer l, used for the
 * static FP8 activation scale; 0 selects the default amax 16.
 */
typedef struct pifu_mlp {
  int32_t n_layers;
  int32_t feat_dim;
  int32_t n_extra;
  int32_t hidden_act;
  int32_t out_act;
  int32_t widths[PIFU_MAX_LAYERS];
  int32_t skip[PIFU_MAX_LAYERS];
  const float* W[PIFU_MAX_LAYERS];
  const float* b[PIFU_MAX_LAYERS];
  float fp8_amax[PIFU_MAX_LAYERS];
} pifu_mlp;

/*
 * The conditional-batch-norm lifting network with soft one-hot depth (appendix, "Depth
 * Representation" and "Pixel-aligned 3D Lifting"; Tab. 2, HRNet-CBN-SoftZ).  With
 * c = Phi(P_xy) the sampled feature (feat_dim channels) and Z the soft one-hot code of
 * P_z (n_z channels: with s = (n_z - 1)(P_z + 1)/2, Z[floor s] = 1 + floor s - s,
 * Z[floor s + 1] = s - floor s; the code is defined for -1 <= P_z <= 1 and a depth
 * outside is clamped to that interval):
 *   h_0 = Wp Z + bp;  for block i = 0 .. n_blocks-1 (h_i = W[i-1] a_{i-1} + b[i-1] for
 *   i >= 1):  a_i = relu(gamma_i(c) (h_i - mean[i]) / sqrt(var[i] + eps) + beta_i(c)),
 *   gamma_i(c) = Wg[i] c + bg[i], beta_i(c) = Wb[i] c + bb[i];  logit = Wo a_last + bo.
 * (Batch norm with its running statistics.)  Device float32 arrays, row-major
 * [out][in], 16-byte aligned: Wp [width][n_z], W[i] [width][width], Wg[i] and Wb[i]
 * [width][feat_dim], Wo [1][width]; vectors of width (bo: 1).  Supported: width % 64 == 0
 * and <= 512, feat_dim % 32 == 0 and <= 512, 2 <= n_z <= 256, 1 <= n_blocks <= 8.
 */
#define PIFU_CBN_MAX_BLOCKS 8
typedef struct pifu_cbn {
  int32_t feat_dim, n_z, width, n_blocks;
  float eps;
  const float* Wp;
  const float* bp;
  const float* W[PIFU_CBN_MAX_BLOCKS];
  const float* b[PIFU_CBN_MAX_BLOCKS];
  const float* Wg[PIFU_CBN_MAX_BLOCKS];
  const float* bg[PIFU_CBN_MAX_BLOCKS];
  const float* Wb[PIFU_CBN_MAX_BLOCKS];
  const float* bb[PIFU_CBN_MAX_BLOCKS];
  const float* mean[PIFU_CBN_MAX_BLOCKS];
  const float* var[PIFU_CBN_MAX_BLOCKS];
  const float* Wo;
  const float* bo;
} pifu_cbn;

/*
 * An occupancy (or colour) field.  For PIFU_FIELD_MLP: feat (device, HWC float32,
 * H x W x C with C == mlp->feat_dim) and mlp (host struct) are required;
 * surrogate (host struct, nullable) is a cheaper MLP over the same features used
 * on coarse levels (see pifu_grid_opts).  For PIFU_FIELD_ELLIPSOIDS: ell (host)
 * holds n_ell records of 12 floats: centre c (3) then M = diag(1/a) R^T row-major
 * (9); logit = sharpness * (1 - min_i |M_i (P - c_i)|^2).  For PIFU_FIELD_PLANE:
 * logit = plane[0] x + plane[1] y + plane[2] z + plane[3].  Analytic fields are
 * evaluated in float64.
 */
typedef struct pifu_field {
  int32_t kind;
  int32_t H, W, C;
  const float* feat;
  const pifu_mlp* mlp;
  const pifu_mlp* surrogate;
  int32_t n_ell;
  float sharpness;
  const float* ell;
  float plane[4];
  const pifu_cbn* cbn;      /* PIFU_FIELD_CBN (host struct): the network; feat as for MLP fields.
                               Supported by pifu_occupancy_grid, pifu_octree_grid and
                               pifu_eval_points in PIFU_PREC_FP32 */
} pifu_field;

/* Per-level counters (Sec. 3.2 steps), written to host memory by the calls. */
typedef struct pifu_level_stats {
  int32_t level;            /* log2 of the x cell count of this level */
  uint32_t nodes;           /* nodes of the level lattice (render last level: output columns x (D+1)) */
  uint32_t b0;              /* boundary candidates: interpolated value neither 0 nor 1 */
  uint32_t dilated;         /* nodes of the 1-ring dilation not evaluated before */
  uint32_t evaluated;       /* nodes evaluated at this level (all waves) */
  uint32_t waves;           /* conflict waves that added nodes */
  uint32_t conflicts;       /* conflict nodes summed over waves */
  uint32_t mlp_points;      /* points pushed through the MLP (incl. clipped render points) */
  uint32_t band_fp32;       /* points re-run in FP32 by the precision band */
  uint32_t guard_fp64;      /* points re-run in FP64 by the FP32 guard band */
  uint32_t surrogate_fallback; /* surrogate points re-run with the full MLP */
  uint32_t shadow;          /* render last level: shadow nodes (never evaluated) */
  uint32_t hits;            /* render last level: pixels with a surface hit */
  uint32_t reserved[3];
} pifu_level_stats;

/*
 * Options of pifu_occupancy_grid.
 *   log2_final in [1, 10], log2_coarse in [1, log2_final]: the final grid has
 *   2^log2_final cells per axis and the coarsest (densely evaluated) level
 *   2^log2_coarse.  dense != 0 evaluates every final node instead (the
 *   brute-force baseline) and ignores log2_coarse.
 *   precision: PIFU_PREC_*.  band_delta: for BF16/FP16/FP8, points with
 *   |p - 0.5| < band_delta are re-run with FP32 accuracy (FP8 runs: FP32 MFMA; BF16 and
 *   FP16 runs: FP32-accurate products of binary16 hi / lo operand splits, three FP16
 *   MFMAs per step).  FP16 runs check every converted operand (feature, weight, hidden
 *   activation) against the binary16 range; once one falls outside it, every evaluation
 *   of the call from then on (including the one that overflowed) is re-run in FP32 and
 *   counted in band_fp32.  BF16 runs check the split operands (binary16 weight copies,
 *   the band's features and activations) and, once one falls outside the range, re-run
 *   that band and every later band of the call in FP32.  guard_logit: points whose FP32
 *   logit has |logit| < guard_logit are re-run in FP64 so that labels are decided
 *   exactly (0 disables).  surrogate_max_log2: levels with at most this log2
 *   size use field->surrogate when present (points with |p_s - 0.5| <
 *   surrogate_delta go to the full MLP); -1 disables.  tile_m: MLP point tile
 *   (0 = chosen per launch: autotuned, else by size; 32 (FP32 only, else 64), 64,
 *   96 (FP32: 128 points x 64 outputs, else 128), 128 or 256).  Every tile gives
 *   bit-identical results.  max_waves: cap on
 *   conflict waves per level
 *   (0 = none).
 */
typedef struct pifu_grid_opts {
  int32_t log2_final;
  int32_t log2_coarse;
  int32_t dense;
  int32_t precision;
  float band_delta;
  float guard_logit;
  int32_t surrogate_max_log2;
  float surrogate_delta;
  int32_t tile_m;
  int32_t max_waves;
} pifu_grid_opts;

/*
 * Options of pifu_render_view.  The target-view lattice has 2^log2_w cells in x
 * and y and 2^log2_d cells in z; the coarsest level has 2^log2_coarse_w cells in
 * x and y (and 2^(log2_d - log2_w + log2_coarse_w) in z).  The image is W x H with
 * W = H = 2^log2_w; pixel (row v, column u) is node column (u, v).  Other fields
 * as in pifu_grid_opts; precision applies to the occupancy network, and the colour
 * network runs in FP32, or (BF16 and FP16 renders) with FP32-accurate products of
 * binary16 hi / lo operand splits, re-run in FP32 if an operand leaves the binary16
 * range.
 */
typedef struct pifu_render_opts {
  int32_t log2_w;
  int32_t log2_d;
  int32_t log2_coarse_w;
  int32_t precision;
  float band_delta;
  float guard_logit;
  int32_t surrogate_max_log2;
  float surrogate_delta;
  int32_t tile_m;
  int32_t max_waves;
} pifu_render_opts;

/* ---------------------------------------------------------------- handle */

/* Creates a handle bound to the current HIP device (must be gfx950).  The
 * handle owns about 1 KB of mapped pinned host memory for count read-back (and
 * the same again for the companion state that pifu_grid_and_render's second
 * thread uses) and never allocates device memory.  One handle must not be used
 * by two threads at once. */
int32_t pifu_create(pifu_ctx** out);
void pifu_destroy(pifu_ctx* ctx);
const char* pifu_status_string(int32_t status);

/* ---------------------------------------------------------------- occupancy grid */

/* Bytes of device workspace pifu_occupancy_grid needs for these options/field. */
int32_t pifu_occupancy_grid_workspace_size(const pifu_field* field, const pifu_grid_opts* opts,
                                           size_t* bytes);

/*
 * Hierarchical surface localization on the input-view grid (Sec. 3.2,
 * "Octree-based Robust Surface Localization"; evaluation by Eq. 1).
 * Outputs (device, (2^L+1)^3 entries, z fastest):
 *   occ     float32: p where the network was evaluated, else the culled value 0/1.
 *   labels  uint8 0/1.
 *   eval_level (nullable) uint8: level (log2 size) at which each node was
 *           evaluated, 255 if never.
 * cells (device, cells_cap entries): sorted indices (i*R + j)*R + k of the cells
 * whose 8 corner labels differ; *n_cells (host) receives the true count, which
 * may exceed cells_cap (then only cells_cap entries are written).
 * stats (host, nullable): log2_final - log2_coarse + 1 records, coarsest first.
 */
int32_t pifu_occupancy_grid(pifu_ctx* ctx, const pifu_field* field, const pifu_grid_opts* opts,
                            float* occ, uint8_t* labels, uint8_t* eval_level,
                            uint32_t* cells, uint32_t cells_cap, uint32_t* n_cells,
                            pifu_level_stats* stats, void* workspace, size_t workspace_bytes,
                            pifu_stream stream);

/* ---------------------------------------------------------------- octree baselines */

#define PIFU_OCTREE_BINARIZED 0   /* subdivide cells whose corner labels [p > 0.5] differ */
#define PIFU_OCTREE_THRESHOLD 1   /* subdivide cells whose corner occupancies deviate from their
                                     mean by more than a threshold */

/*
 * The octree subdivisions that Sec. 3.2 ("Octree-based Robust Surface Localization")
 * compares its localization with (the trade-off of Fig. 3), on the input-view grid:
 * the coarsest level is evaluated densely; each finer level subdivides the coarse cells
 * selected by `mode` and evaluates every node of them not evaluated before (no dilation,
 * no conflict search).  Other nodes take the trilinear interpolation of the coarse
 * values -- of the corner labels for PIFU_OCTREE_BINARIZED (so 0 or 1), of the corner
 * occupancies for PIFU_OCTREE_THRESHOLD, with label [value > 0.5].
 * PIFU_OCTREE_THRESHOLD subdivides a cell when max_i |p_i - mean(p)| > threshold over
 * its 8 corner occupancy values p_i; the decision reads the stored float32 occupancies
 * and takes mean and deviations in float64 (corner sum over (di, dj, dk), dk fastest),
 * and interpolation is separable in float64 (x, then y, then z; 0.5 (lo + hi) per step).
 * threshold is ignored for PIFU_OCTREE_BINARIZED.
 * opts, outputs, workspace (pifu_occupancy_grid_workspace_size) and errors as for
 * pifu_occupancy_grid; opts->dense must be 0; the surrogate and max_waves are not used.
 * stats (host, nullable, one record per level): nodes, b0 = cells subdivided from the
 * coarser level, dilated = evaluated = nodes evaluated at the level, and the
 * evaluation counters.  Blocks until done.
 */
int32_t pifu_octree_grid(pifu_ctx* ctx, const pifu_field* field, const pifu_grid_opts* opts,
                         int32_t mode, double threshold, float* occ, uint8_t* labels,
                         uint8_t* eval_level, uint32_t* cells, uint32_t cells_cap,
                         uint32_t* n_cells, pifu_level_stats* stats, void* workspace,
                         size_t workspace_bytes, pifu_stream stream);

/* ---------------------------------------------------------------- several frames */

/* Outputs of one frame of pifu_occupancy_grid_batched (device buffers as in
 * pifu_occupancy_grid; n_cells is written by the call; stats host, nullable,
 * log2_final - log2_coarse + 1 records). */
typedef struct pifu_grid_out {
  float* occ;
  uint8_t* labels;
  uint32_t* cells;
  uint32_t cells_cap;
  uint32_t n_cells;
  pifu_level_stats* stats;
} pifu_grid_out;

int32_t pifu_occupancy_grid_batched_workspace_size(int32_t n, const pifu_field* const* fields,
                                                   const pifu_grid_opts* const* opts,
                                                   size_t* bytes);

/*
 * Hierarchical localization of n <= 16 independent frames in one pass: frames are
 * processed independently in the paper (Sec. 3), so their levels run in lockstep
 * and every conflict wave evaluates all frames' points with one set of MLP GEMMs
 * (the network is shared; feature maps and analytic shapes differ per frame).
 * Frames may differ in log2_final; every other option, the field kind and the
 * network must be equal (else PIFU_ERR_INVALID_ARGUMENT).  Results are identical
 * to n calls of pifu_occupancy_grid.  The combined point list holds at most 2^28
 * points per wave (PIFU_ERR_WORKSPACE_TOO_SMALL beyond).  Blocks until done.
 */
int32_t pifu_occupancy_grid_batched(pifu_ctx* ctx, int32_t n, const pifu_field* const* fields,
                                    const pifu_grid_opts* const* opts, pifu_grid_out* outs,
                                    void* workspace, size_t workspace_bytes, pifu_stream stream);

/* ---------------------------------------------------------------- render */

int32_t pifu_render_view_workspace_size(const pifu_field* occ_field, const pifu_field* color_field,
                                        const pifu_render_opts* opts, size_t* bytes);

/*
 * Mesh-free rendering of a target view (Sec. 3.2, "Mesh-free Rendering"; Eq. 3).
 * view (host, 12 floats): row-major 3x4 [A | t] mapping target-view NDC to
 * input-view NDC; points mapped outside [-1,1]^3 have logit -inf.  bg (host, 3).
 * Outputs (device, image row-major, H = W = 2^log2_w):
 *   rgb   float32 H*W*3: tanh output of the colour MLP at the hit point
 *         (Eq. 2 with extras z' and the occupancy of the hit node), bg elsewhere.
 *   depth float32 H*W: target-view z of the hit point, NaN where no hit.
 *   hit   uint8 H*W: 1 where the ray meets the surface.
 * stats (host, nullable): (log2_w - log2_coarse_w + 1) records; the last one is
 * the final render level (shadow, evaluated, hits).
 * color_field must be PIFU_FIELD_MLP with an MLP of n_extra == 2 and 3 outputs.
 */
int32_t pifu_render_view(pifu_ctx* ctx, const pifu_field* occ_field, const pifu_field* color_field,
                         const float* view, const pifu_render_opts* opts, const float* bg,
                         float* rgb, float* depth, uint8_t* hit, pifu_level_stats* stats,
                         void* workspace, size_t workspace_bytes, pifu_stream stream);

/*
 * Optional per-node record of a render, for inspection and testing (the steps of
 * Sec. 3.2, "Mesh-free Rendering").  Every pointer is device memory or null.
 *   kstar  int32 H*W (row v, column u): the first argmax k* (nearest node from the
 *          observer whose interpolated value is 1), -1 where there is none.
 *   k1     int32 H*W: the second argmax after evaluation (the node whose occupancy and
 *          that of k1 + 1 give the surface point), -1 where there is no hit.
 *   eval_level uint8 over the finest target lattice, (W+1)*(W+1)*(D+1) nodes, z fastest:
 *          log2 of the x cell count of the level at which each node was evaluated by
 *          the network, 255 if never.
 *   logit  float32 over the same lattice: the logit of every evaluated node (other
 *          entries are left as they were).
 */
typedef struct pifu_render_trace {
  int32_t* kstar;
  int32_t* k1;
  uint8_t* eval_level;
  float* logit;
} pifu_render_trace;

/* pifu_render_view with the record above written as well (trace must not be null). */
int32_t pifu_render_view_traced(pifu_ctx* ctx, const pifu_field* occ_field,
                                const pifu_field* color_field, const float* view,
                                const pifu_render_opts* opts, const float* bg, float* rgb,
                                float* depth, uint8_t* hit, pifu_level_stats* stats,
                                void* workspace, size_t workspace_bytes, pifu_stream stream,
                                const pifu_render_trace* trace);

/* ---------------------------------------------------------------- one frame */

/* The arguments of one pifu_occupancy_grid call, as one record. */
typedef struct pifu_grid_call {
  const pifu_field* field;
  const pifu_grid_opts* opts;
  float* occ;
  uint8_t* labels;
  uint8_t* eval_level;          /* nullable */
  uint32_t* cells;
  uint32_t cells_cap;
  uint32_t* n_cells;            /* host */
  pifu_level_stats* stats;      /* host, nullable */
  void* workspace;
  size_t workspace_bytes;
  pifu_stream stream;
} pifu_grid_call;

/* The arguments of one pifu_render_view call, as one record. */
typedef struct pifu_render_call {
  const pifu_field* occ_field;
  const pifu_field* color_field;
  const float* view;            /* host, 12 floats */
  const pifu_render_opts* opts;
  const float* bg;              /* host, 3 floats */
  float* rgb;
  float* depth;
  uint8_t* hit;
  pifu_level_stats* stats;      /* host, nullable */
  void* workspace;
  size_t workspace_bytes;
  pifu_stream stream;
} pifu_render_call;

/*
 * One frame of the method (Sec. 3.2): the surface localized on the input-view grid
 * and a target view rendered without a mesh.  The two are independent (the render
 * localizes the surface along its own rays, Eq. 3), so they run concurrently: the
 * grid on the calling thread and grid->stream, the render on a second host thread
 * with the handle's companion state and render->stream.  Many launches of either
 * are too small to fill the GPU, and the other's work fills the gaps.  Every
 * output, including the stats, is identical to pifu_occupancy_grid followed by
 * pifu_render_view with the same arguments.  When the two streams are the same
 * (or a second thread cannot be started) the calls run one after the other.
 * Each call's arguments are validated as by its own entry point; the two
 * workspaces and all outputs must not overlap.  Returns the grid's status if it
 * failed, else the render's.  Kernel profiling (pifu_profile_enable on ctx)
 * covers both.  Blocks until both are done.
 */
int32_t pifu_grid_and_render(pifu_ctx* ctx, const pifu_grid_call* grid,
                             const pifu_render_call* render);

/* ---------------------------------------------------------------- device-driven calls */

/* Status bits of the device-driven calls (written to *status_dev). */
#define PIFU_STATUS_LIST_OVER 1u    /* a point list exceeded max_points: results are invalid */
#define PIFU_STATUS_WAVES_LEFT 2u   /* conflicts remained after the wave budget: results are
                                       those of a capped conflict loop */
#define PIFU_STATUS_GUARD_OVER 4u   /* more FP64-guard points than one guard pass holds: some
                                       labels were decided in FP32 only */
#define PIFU_STATUS_CELLS_OVER 8u   /* more surface cells than cells_cap (truncated list) */

/*
 * Asynchronous pifu_occupancy_grid (Sec. 3.2, "Octree-based Robust Surface Localization"):
 * the same method and results, enqueued on `stream` without any host read-back or
 * synchronization, so the call can be captured into a HIP graph and replayed.  Every
 * count stays in device memory:
 *   n_cells_dev  (device uint32) the true number of surface cells (cells holds
 *                min(*n_cells_dev, cells_cap) of them);
 *   stats_dev    (device, log2_final - log2_coarse + 1 records, 4-byte aligned);
 *   status_dev   (device uint32) PIFU_STATUS_* bits, 0 when the results are complete.
 * max_points bounds the points of one network evaluation (0: min(largest level, 2^20));
 * the workspace holds the activations of that many points, so a larger bound trades
 * memory for range.  The conflict loop runs a fixed ladder of waves per level:
 * opts->max_waves when non-zero (the cap of the blocking call), else 12 waves with
 * PIFU_STATUS_WAVES_LEFT set if a level still has conflicts after them.  Waves past the
 * last conflict launch kernels that find empty lists.  Unsupported: PIFU_PREC_FP8 (its
 * weight scales are read back on the host).  Argument errors are returned before
 * anything is enqueued; device-side conditions arrive in *status_dev.  The workspace
 * and outputs must stay valid until the stream (or graph) has run.
 */
int32_t pifu_occupancy_grid_async_workspace_size(const pifu_field* field,
                                                 const pifu_grid_opts* opts, uint32_t max_points,
                                                 size_t* bytes);
int32_t pifu_occupancy_grid_async(pifu_ctx* ctx, const pifu_field* field,
                                  const pifu_grid_opts* opts, uint32_t max_points, float* occ,
                                  uint8_t* labels, uint8_t* eval_level, uint32_t* cells,
                                  uint32_t cells_cap, uint32_t* n_cells_dev,
                                  pifu_level_stats* stats_dev, uint32_t* status_dev,
                                  void* workspace, size_t workspace_bytes, pifu_stream stream);

/*
 * Asynchronous pifu_render_view (Sec. 3.2, "Mesh-free Rendering"; Eq. 3): as above, with
 * stats_dev holding log2_w - log2_coarse_w + 1 device records.  max_points is raised to
 * at least W * W (the colour network's points).
 */
int32_t pifu_render_view_async_workspace_size(const pifu_field* occ_field,
                                              const pifu_field* color_field,
                                              const pifu_render_opts* opts, uint32_t max_points,
                                              size_t* bytes);
int32_t pifu_render_view_async(pifu_ctx* ctx, const pifu_field* occ_field,
                               const pifu_field* color_field, const float* view,
                               const pifu_render_opts* opts, uint32_t max_points, const float* bg,
                               float* rgb, float* depth, uint8_t* hit, pifu_level_stats* stats_dev,
                               uint32_t* status_dev, void* workspace, size_t workspace_bytes,
                               pifu_stream stream);

/*
 * pifu_occupancy_grid_async without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The workspace is a fixed scratch array of
 * PIFU_NOALLOC_SCRATCH_MIB MiB in the library's device memory, one per GPU, held until
 * the process ends; its address is looked up once per device by pifu_create.  The call
 * allocates nothing.  Arguments, outputs, results and device-side status are those of
 * pifu_occupancy_grid_async.  Options whose workspace
 * (pifu_occupancy_grid_async_workspace_size) exceeds the scratch return
 * PIFU_ERR_SCRATCH_TOO_SMALL before anything is enqueued; a smaller max_points lowers
 * the need.  Every call on one GPU shares that GPU's array and finds the previous
 * call's contents in it (the call clears what it needs cleared): calls that overlap on
 * one GPU -- on two streams, two threads, or two handles -- race and must not be made.
 */
#define PIFU_NOALLOC_SCRATCH_MIB 128
size_t pifu_noalloc_scratch_bytes(void);
int32_t pifu_occupancy_grid_async_noalloc(pifu_ctx* ctx, const pifu_field* field,
                                          const pifu_grid_opts* opts, uint32_t max_points,
                                          float* occ, uint8_t* labels, uint8_t* eval_level,
                                          uint32_t* cells, uint32_t cells_cap,
                                          uint32_t* n_cells_dev, pifu_level_stats* stats_dev,
                                          uint32_t* status_dev, pifu_stream stream);

/* Outputs of one frame of pifu_occupancy_grid_batched_async (device buffers as in
 * pifu_occupancy_grid_async). */
typedef struct pifu_grid_out_dev {
  float* occ;
  uint8_t* labels;
  uint32_t* cells;
  uint32_t cells_cap;
  uint32_t* n_cells_dev;          /* device uint32: the frame's true surface-cell count */
  pifu_level_stats* stats_dev;    /* device, log2_final - log2_coarse + 1 records */
} pifu_grid_out_dev;

/*
 * Device-driven pifu_occupancy_grid_batched (frames are processed independently in the
 * paper, Sec. 3, so their levels run in lockstep): every level and conflict wave is one
 * set of launches over all frames' combined work list -- one pass of the network's
 * persistent GEMMs, the precision band and the FP64 guard over every frame's points --
 * with all counts in device memory and nothing read back, so the whole call can be
 * captured into one HIP graph and replayed.  Frames, options and restrictions as in
 * pifu_occupancy_grid_batched (n <= 16; one network; frames may differ in log2_final);
 * the conflict loop runs the wave ladder of pifu_occupancy_grid_async (opts->max_waves,
 * else 12 waves with PIFU_STATUS_WAVES_LEFT).  max_points bounds the combined points of
 * one pass (0: min(largest combined level, 2^21)); the workspace holds that many points'
 * activations.  Per-frame statistics are tallied on the device.  *status_dev receives the
 * PIFU_STATUS_* bits of all frames.  Results equal pifu_occupancy_grid_batched's and n
 * pifu_occupancy_grid calls'.  Unsupported: PIFU_PREC_FP8, PIFU_FIELD_PLANE, and the
 * surrogate on any level.
 */
int32_t pifu_occupancy_grid_batched_async_workspace_size(int32_t n, const pifu_field* const* fields,
                                                         const pifu_grid_opts* const* opts,
                                                         uint32_t max_points, size_t* bytes);
int32_t pifu_occupancy_grid_batched_async(pifu_ctx* ctx, int32_t n, const pifu_field* const* fields,
                                          const pifu_grid_opts* const* opts, uint32_t max_points,
                                          const pifu_grid_out_dev* outs, uint32_t* status_dev,
                                          void* workspace, size_t workspace_bytes,
                                          pifu_stream stream);

/* ---------------------------------------------------------------- mesh hand-off */

/*
 * Marching Cubes over the surface cells of an occupancy grid -- the mesh extraction of
 * the PIFu baseline (Sec. 1; Sec. 3.2, "Inference for Human Reconstruction") -- with
 * vertex colours (the texture paragraph of Sec. 3.1).
 * Inputs (device): occ and labels over the (2^log2_final + 1)^3 nodes (z fastest), as
 * written by pifu_occupancy_grid; cells, the sorted surface-cell list (n_cells entries).
 * Vertices: one per lattice edge whose end labels differ, at the 0.5 crossing of the
 * linear interpolation of the two end occupancies (t clipped to [0, 1]), sorted by edge
 * id 3 * node + axis; verts (device float32 vert_cap x 3, NDC).  Triangles: per cell in
 * list order, from a 256-case table derived from the contour on the cube faces (an
 * ambiguous face keeps its inside corners apart, so neighbouring cells agree and the
 * mesh is closed); normals (right-hand rule) point from label 1 to label 0; tris
 * (device uint32 tri_cap x 3, vertex indices).  *n_verts and *n_tris (host) receive the
 * true counts; only the first vert_cap / tri_cap are written (a triangle whose vertex
 * lies past vert_cap is then meaningless).
 * colors (device float32 vert_cap x 3, nullable; requires color_field): a vertex seen by
 * the input camera (orthographic, at z = +1: no label-1 node above the edge's k in the
 * columns of its two nodes) takes the input pixel -- bilinear over image (device HWC
 * float32, img_h x img_w x 3, texels outside 0; nullable: then every vertex uses the
 * network); the others take Eq. 2's colour network (PIFU_FIELD_MLP, n_extra 2, 3
 * outputs) at [Phi(g_T, P_xy); P_z; 0.5], in FP32.  Workspace: pifu_mesh_workspace_size.
 * Blocks until done.
 */
int32_t pifu_mesh_workspace_size(int32_t log2_final, uint32_t n_cells, uint32_t vert_cap,
                                 const pifu_field* color_field, size_t* bytes);
int32_t pifu_mesh(pifu_ctx* ctx, int32_t log2_final, const float* occ, const uint8_t* labels,
                  const uint32_t* cells, uint32_t n_cells, const pifu_field* color_field,
                  const float* image, int32_t img_h, int32_t img_w, float* verts, float* colors,
                  uint32_t vert_cap, uint32_t* n_verts, uint32_t* tris, uint32_t tri_cap,
                  uint32_t* n_tris, void* workspace, size_t workspace_bytes, pifu_stream stream);

/* ---------------------------------------------------------------- point evaluation */

int32_t pifu_eval_points_workspace_size(const pifu_field* field, int32_t precision, uint32_t n,
                                        size_t* bytes);

/*
 * Evaluates a field at n input-view NDC points (Eq. 1) with the same kernels the
 * grid path uses.  pts: device float32 n x 4 (x, y, z, unused).  logit: device
 * float32 n.  labels (device uint8 n, nullable) receives the label decided with
 * the guard band.  occ (device float32 n, nullable) receives the occupancy value
 * p = 1 / (1 + exp(-logit)) in float32, as the grid computes it.  precision /
 * band_delta / guard_logit as in pifu_grid_opts.  Blocks until done.
 */
int32_t pifu_eval_points(pifu_ctx* ctx, const pifu_field* field, int32_t precision,
                         float band_delta, float guard_logit, const float* pts, uint32_t n,
                         float* logit, uint8_t* labels, float* occ, void* workspace,
                         size_t workspace_bytes, pifu_stream stream);

/*
 * Static FP8 activation scales (the per-layer scale of the precision ladder): runs
 * field->mlp in FP32 over n input-view points (device float32 n x 4, as for
 * pifu_eval_points) and writes, for every hidden layer l, the largest |value| of that
 * layer's quantized input (layer 0: the sampled feature; layer l >= 1: the previous
 * layer's output and, with a skip, the feature) to amax[l] (host, n_layers - 1 values).
 * These are the values pifu_mlp.fp8_amax expects.  Workspace as
 * pifu_eval_points_workspace_size(field, PIFU_PREC_FP32, n).  Blocks until done.
 */
int32_t pifu_fp8_calibrate(pifu_ctx* ctx, const pifu_field* field, const float* pts, uint32_t n,
                           float* amax, void* workspace, size_t workspace_bytes,
                           pifu_stream stream);

/* ---------------------------------------------------------------- surrogate training */

/* Bytes of workspace pifu_mlp_grad needs for batches of up to max_batch points. */
int32_t pifu_mlp_train_workspace_size(const pifu_field* field, uint32_t max_batch, size_t* bytes);

/*
 * Gradient of the mean soft-target binary cross entropy (the occupancy loss of
 * Sec. 3.1, with soft teacher targets) of field->mlp over a batch:
 *   loss = mean_m [softplus(s_m) - t_m s_m],  s_m = logit of point m.
 * field: PIFU_FIELD_MLP (feat = the frame's feature map, mlp = the network being
 * trained, float32 weights).  pts: device float32 n x 4 (x, y, z in input NDC,
 * teacher occupancy t in [0,1]).  dW[l], db[l]: device float32 outputs shaped like
 * mlp->W[l], mlp->b[l].  loss: device float (nullable).  Reductions over the batch
 * run in a fixed order, so results are bit-reproducible.  Asynchronous on stream.
 */
int32_t pifu_mlp_grad(pifu_ctx* ctx, const pifu_field* field, const float* pts, uint32_t n,
                      float* const* dW, float* const* db, float* loss, void* workspace,
                      size_t workspace_bytes, pifu_stream stream);

/* pifu_mlp_grad that also writes every point's loss softplus(s_m) - t_m s_m to
 * point_loss (device float32 n, nullable) -- the per-point BCE that point-OHEM reads. */
int32_t pifu_mlp_grad_ex(pifu_ctx* ctx, const pifu_field* field, const float* pts, uint32_t n,
                         float* const* dW, float* const* db, float* loss, float* point_loss,
                         void* workspace, size_t workspace_bytes, pifu_stream stream);

/*
 * Point-OHEM sampling (Sec. 3.3, Eq. 6 right): draws `batch` training points with
 * replacement, with probability proportional to their stored inverse probabilities
 * weights[0 .. n) (device float32, >= 0, not all 0; n <= 2^27).  Each weight w is taken
 * as the integer floor(w * 2^16) and the prefix sums are exact 64-bit integers; draw b
 * uses r = output number counter * batch + b of SplitMix64 (Steele, Lea and Flood 2014)
 * started from state seed, the target t = floor(r * S / 2^64) with S the weights' total,
 * and picks the first point whose inclusive prefix sum exceeds t.  idx (device uint32,
 * batch) receives the drawn indices; batch_pts (device float32 batch x 4, 16-byte
 * aligned, nullable) receives pool[idx] (pool: device n x 4, the training points).
 * Workspace: pifu_ohem_sample_workspace_size.  Asynchronous on stream.
 */
int32_t pifu_ohem_sample_workspace_size(uint32_t n, size_t* bytes);
int32_t pifu_ohem_sample(pifu_ctx* ctx, const float* weights, uint32_t n, const float* pool,
                         uint32_t batch, uint64_t seed, uint64_t counter, uint32_t* idx,
                         float* batch_pts, void* workspace, size_t workspace_bytes,
                         pifu_stream stream);

/*
 * The stored inverse probabilities of the drawn points from their losses (Eq. 6 right):
 * weights[idx[b]] = min(1 / (exp(-point_loss[b] / alpha) + beta), 2^20) for b < batch
 * (device pointers; alpha > 0, beta >= 0).  The cap keeps the inverse probability finite.
 * Asynchronous on stream.
 */
int32_t pifu_ohem_update(pifu_ctx* ctx, const float* point_loss, const uint32_t* idx,
                         uint32_t batch, float alpha, float beta, float* weights,
                         pifu_stream stream);

/*
 * One RMSProp step on every parameter of net (the optimizer the paper trains the
 * shape network with, appendix A1.2):  v = alpha v + (1 - alpha) g^2,
 * w -= lr g / (sqrt(v) + eps).  net->W / net->b are updated in place (device);
 * vW / vb hold the running averages (device, zero-initialised by the caller).
 */
int32_t pifu_rmsprop_step(pifu_ctx* ctx, const pifu_mlp* net, const float* const* dW,
                          const float* const* db, float* const* vW, float* const* vb, float lr,
                          float alpha, float eps, pifu_stream stream);

/* ---------------------------------------------------------------- tile autotuner */

/*
 * Times every hidden layer of field->mlp (and field->surrogate, in BF16) with point
 * tiles 64, 128 and 256 on m lattice points, and records the fastest tile per
 * (precision, layer shape, batch-size bucket <= 8192 / <= 32768 / larger) in ctx;
 * later calls with tile_m == 0 use it.  A tile within 3% of the fastest loses to
 * 128, then to 64 (deterministic ties).  All tiles produce bit-identical results.
 * chosen (host, nullable) receives one tile per timed layer.  Workspace as
 * pifu_eval_points_workspace_size(field, precision, m).  Blocks until done.
 */
int32_t pifu_autotune_mlp(pifu_ctx* ctx, const pifu_field* field, int32_t precision, uint32_t m,
                          int32_t* chosen, void* workspace, size_t workspace_bytes,
                          pifu_stream stream);
/* Forgets every autotuned tile of ctx. */
int32_t pifu_autotune_clear(pifu_ctx* ctx);

/*
 * The library's operand conversions applied to n float32 values (device in/out):
 * PIFU_PREC_BF16 -> uint16 bfloat16 bits (round to nearest even);
 * PIFU_PREC_FP16 -> uint16 IEEE binary16 bits (round to nearest even, overflow to
 * infinity);
 * PIFU_PREC_FP8 -> uint8 OCP e4m3fn codes (nearest even, saturating at +-448, no
 * scaling).  The MLP kernels use exactly these conversions.  Blocks until done.
 */
int32_t pifu_convert_f32(pifu_ctx* ctx, const float* in, uint32_t n, int32_t precision, void* out,
                         pifu_stream stream);

/* ---------------------------------------------------------------- kernel profiling */

/* Kernel families timed by the built-in profiler (index into pifu_profile_read's array). */
#define PIFU_KERN_GEMM_F32 0      /* MLP hidden layer, FP32 MFMA */
#define PIFU_KERN_GEMM_BF16 1     /* MLP hidden layer, BF16 MFMA */
#define PIFU_KERN_GEMM_FP8 2      /* MLP hidden layer, FP8 MFMA */
#define PIFU_KERN_GATHER 3        /* point projection + bilinear feature gather */
#define PIFU_KERN_HEAD 4          /* last MLP layer + output rule */
#define PIFU_KERN_GEMM_F16 5      /* MLP hidden layer, FP16 MFMA */
#define PIFU_KERN_GEMM_F16X3 6    /* FP32-accurate hidden layer from three FP16 MFMA products
                                     (the FP32-accurate band of a BF16 or FP16
                                     run, the colour MLP of their renders) */
#define PIFU_KERN_COUNT 8

/* Accumulated over the launches of one kernel family since the last enable. flops
 * and bytes are algorithmic counts (2*M*N*K for a GEMM; texels read + features
 * written for the gather), not hardware counters. */
typedef struct pifu_kernel_profile {
  uint64_t launches;
  double total_ms;
  double flops;
  double bytes;
} pifu_kernel_profile;

/* on != 0: every later call records HIP events around each launch of the families
 * above, on the stream the launch uses, and accumulates durations when the call
 * completes.  Enabling (or disabling) resets the accumulators. */
int32_t pifu_profile_enable(pifu_ctx* ctx, int32_t on);
/* Copies PIFU_KERN_COUNT records into out (host). */
int32_t pifu_profile_read(pifu_ctx* ctx, pifu_kernel_profile* out);

#ifdef __cplusplus
}
#endif
#endif /* PIFU_H */
