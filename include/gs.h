/*
 * gs.h — C ABI of libgsmi: one partition's 3D Gaussian Splatting training
 * step on an MI355X (gfx950).
 *
 * The paper (Han et al., "Distributed 3D Gaussian Splatting for
 * High-Resolution Isosurface Visualization", Sec. II, "Parallel Training")
 * trains each data partition independently with the 3D-GS method of Kerbl
 * et al.; the calls below are the steps of that training step:
 *
 *   gs_project     -> 3D Gaussian to 2D conic (EWA splatting Jacobian)
 *   gs_bin_sort    -> tile binning + stable radix sort on (image, tile, depth)
 *   gs_raster_fwd  -> front-to-back alpha compositing per pixel
 *   gs_loss        -> background-masked L1 + D-SSIM loss and its image gradient
 *                     (masks: Sec. II "Image Rendering and Masking", Sec. III-A)
 *   gs_raster_bwd  -> reverse-order replay of the compositing (gradients)
 *   gs_project_bwd -> chain rule back to the Gaussian parameters
 *   gs_adam        -> Adam update of all parameters
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns gs_status (GS_OK = 0, negative = error) and never
 *   aborts.  gs_last_error() returns a thread-local message for the last
 *   failure on the calling thread.
 * - Argument validation happens on the host before anything is enqueued: a
 *   call that returns GS_ERR_ARG has launched nothing.
 * - All buffers marked "device" are caller-owned device memory.  The library
 *   allocates no device memory in any call; calls that need scratch space
 *   take a caller-owned workspace sized by the matching *_workspace_bytes().
 * - Every call enqueues its kernels on `stream` (a hipStream_t; NULL = the
 *   null stream) and returns without synchronising.  Only gs_check_status()
 *   synchronises the stream.
 * - Float arrays are fp32.  Per-Gaussian arrays are planar SoA "[C][n]":
 *   component c of Gaussian i lives at ptr[c*n + i].
 * - Images are planar [S][3][H][W] fp32, masks [S][H][W] u8 (0 = background),
 *   per-pixel state [S][H][W].  Pixel (x, y) has its centre at (x+0.5, y+0.5).
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GS_OK = 0,
  GS_ERR_ARG = -1,         /* invalid argument; nothing was enqueued            */
  GS_ERR_HIP = -2,         /* a HIP runtime call or kernel launch failed        */
  GS_ERR_CAPACITY = -3,    /* the duplicate list outgrew dup_capacity           */
  GS_ERR_NONFINITE = -4,   /* a loss value or parameter update was not finite   */
  GS_ERR_UNSUPPORTED = -5  /* the request is valid but not implemented          */
} gs_status;

/* Pinhole camera in OpenCV axes (x right, y down, z forward).
 * A world point X maps to camera space as x_c = R X + t (R row-major).
 * Pixel coordinates: u = fx x_c/z_c + cx, v = fy y_c/z_c + cy.          */
typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float znear;              /* points with z_c <= znear are culled          */
  int32_t width, height;    /* must equal the call's gs_tiling width/height */
  int32_t reserved;
} gs_camera;                /* 80 bytes */

/* The Gaussians of one or more partitions, planar SoA, read-only.
 *   mean [3][n], log_scale [3][n], quat [4][n] as (w, x, y, z) (any norm > 0),
 *   opacity_logit [n], color [3 (D+1)^2][n]: real spherical-harmonic
 *   coefficients of degree D = sh_degree (0..GS_SH_MAX_DEGREE), coefficient k
 *   (index l*l + l + m, Condon-Shortley phase) of channel c in row 3k + c.
 * The colour a camera sees is max(0, sum_k Y_k(d) color_k + 1/2) with d the
 * unit vector from the camera centre -R^T t to the mean (the view-dependent
 * colour of 3D-GS, whose images the paper fits, Sec. I); at D = 0 this is
 * max(0, C0 color + 1/2), C0 = 1/(2 sqrt(pi)).  Arrays stored at a higher
 * degree may be drawn at a lower one: the rows are coefficient-major, so
 * the first 3 (D+1)^2 rows are the lower-degree model.                     */
#define GS_SH_MAX_DEGREE 3
typedef struct {
  const float* mean;
  const float* log_scale;
  const float* quat;
  const float* opacity_logit;
  const float* color;
  int64_t n;
  int32_t sh_degree;
  int32_t reserved;
} gs_gaussians;

/* Gradients with respect to the gs_gaussians fields, same layout (color:
 * the 3 (D+1)^2 rows of the call's degree).                              */
typedef struct {
  float* mean;
  float* log_scale;
  float* quat;
  float* opacity_logit;
  float* color;
  int64_t n;
} gs_grads;

/* The images ("slots") one call renders.  Slot s draws Gaussians
 * [gauss_offset[s], gauss_offset[s] + pair_offset[s+1] - pair_offset[s])
 * through camera cams[s]; its (Gaussian, slot) pairs are numbered
 * pair_offset[s] .. pair_offset[s+1]-1.  One partition seen from V views is
 * pair_offset = {0, n, 2n, ..., Vn}, gauss_offset = {0, ..., 0}.  Several
 * partitions of one concatenated Gaussian array batch by giving each slot its
 * partition's offset.  All three arrays live in device memory; n_slots is
 * at most GS_MAX_SLOTS and total_pairs must equal pair_offset[n_slots].   */
#define GS_MAX_SLOTS 1024
typedef struct {
  int32_t n_slots;
  int64_t total_pairs;
  const int64_t* pair_offset;   /* device [n_slots + 1], pair_offset[0] = 0 */
  const int64_t* gauss_offset;  /* device [n_slots]                         */
  const gs_camera* cams;        /* device [n_slots]                         */
} gs_views;

/* Image geometry of a call: every slot is width x height pixels, binned in
 * tile_w x tile_h tiles (tile_w * tile_h <= 1024; tiles_x = ceil(W/tile_w)).*/
typedef struct {
  int32_t width, height;
  int32_t tile_w, tile_h;
} gs_tiling;

/* Projected record of one (Gaussian, slot) pair, 12 fp32 per pair
 * ("rec[m][12]", 48 bytes, 16-byte aligned):
 *   [0..1] mean2d (pixels)     [2..4] conic Q11, Q12, Q22 (inverse of the
 *   dilated 2D covariance)     [5] opacity   [6..8] rgb   [9] depth (z_c)
 *   [10] slot index (int32 bits)              [11] reserved (0)
 * tile_bbox [m][4] u16 holds the inclusive tile range (tx0, ty0, tx1, ty1);
 * n_tiles [m] is (tx1-tx0+1)(ty1-ty0+1), or 0 for a culled pair.           */
#define GS_REC_STRIDE 12
typedef struct {
  float* rec;
  uint16_t* tile_bbox;
  int32_t* n_tiles;
  int64_t m;
} gs_projected;

/* Gradient of the loss with respect to each pair's projected record,
 * 9 fp32 per pair ("d_rec[m][9]"): d mean2d (2), d conic (3) in the same
 * Q11, Q12, Q22 parameterisation, d opacity, d rgb (3).                    */
#define GS_DREC_STRIDE 9

/* Device status block written by gs_bin_sort / gs_loss / gs_adam:
 *   status[0]  bit flags: 1 = duplicate overflow, 2 = non-finite loss
 *   status[1]  duplicates required by the last gs_bin_sort
 *   status[2..3] reserved.  The caller zeroes it once (gs_zero).           */
#define GS_STATUS_WORDS 4
#define GS_FLAG_CAPACITY 1
#define GS_FLAG_NONFINITE 2

/* ------------------------------------------------------------------------ */

/* Project every (Gaussian, slot) pair of `views` (3D-GS method cited in
 * Sec. I/II; EWA splatting).  Per pair:
 *   s = exp(log_scale), q^ = q/|q|, o = sigmoid(opacity_logit),
 *   rgb = max(0, C0 color + 1/2);  Sigma = R(q^) diag(s)^2 R(q^)^T;
 *   t = R_v mu + t_v (culled if t_z <= znear);  mean2d = (fx t_x/t_z + cx,
 *   fy t_y/t_z + cy);  Jacobian J of the perspective map with t_x/t_z and
 *   t_y/t_z clamped to 1.3 * W/(2 fx) resp. 1.3 * H/(2 fy);
 *   Sigma2 = J R_v Sigma R_v^T J^T + 0.3 I;  conic = Sigma2^{-1};
 *   support = {d : d^T conic d <= 2 ln(255 o)} (where alpha >= 1/255),
 *   culled if 255 o <= 1;  pixel bbox = [floor(m -/+ h) -/+ 1] clamped to
 *   the image, h = sqrt(2 ln(255 o) diag(Sigma2));  tile bbox from it.
 * out->m must equal views->total_pairs.  Culled pairs get n_tiles = 0.     */
gs_status gs_project(const gs_gaussians* g, const gs_views* views,
                     const gs_tiling* tiling, gs_projected* out, void* stream);

/* Workspace for gs_bin_sort with m pairs and room for dup_capacity
 * duplicates (one per (pair, overlapped tile)).                            */
size_t gs_bin_sort_workspace_bytes(int64_t m, int64_t dup_capacity,
                                   const gs_tiling* tiling, int32_t n_slots);

/* Tile binning and sorting (the 3D-GS per-tile, depth-ordered lists).  Each
 * pair emits one entry per listed tile with key ((slot * tiles_per_slot +
 * ty * tiles_x + tx) << 32) | bits(depth) and value = pair index; entries
 * are sorted stably by key, so equal keys keep ascending pair index.  The
 * listed tiles of a pair with n_tiles > 0 are those of its tile bbox whose
 * pixel-centre rectangle [tx tile_w + 1/2, tx tile_w + tile_w - 1/2] x
 * [ty tile_h + 1/2, ty tile_h + tile_h - 1/2] meets its support widened by a
 * rounding margin: d^T conic d <= 2 ln(255 o) + 0.02 + 1e-5 M, with M =
 * a X^2 + 2|b| X Y + c Y^2 for the largest |dx| = X and |dy| = Y from the
 * mean to the bbox's pixel-centre extents (conic (a, b, c), opacity o and
 * mean read from rec).  No pixel centre of another bbox tile reaches
 * alpha >= 1/255, so images do not depend on it.  A bbox of more than 64
 * tiles is listed whole.  Outputs (device):
 *   keys_out [dup_capacity] u64 (optional, may be NULL: the sort then
 *   carries 32-bit tile indices instead of the 64-bit keys, with the same
 *   ids_out and tile_ranges), ids_out [dup_capacity] u32 (sorted),
 *   tile_ranges [n_slots * tiles_per_slot][2] u32: [start, end) into ids_out
 *   (start = end = 0 for an empty tile),
 *   pair_first [m][2] u32 (optional, may be NULL): per pair, the emission
 *   index of its first entry and its entry count.  Entries are emitted pair
 *   by pair in ascending (depth bits, pair index) order, each pair's tiles
 *   row-major over its tile bbox, so pair p's entries are emission indices
 *   pair_first[p][0] .. pair_first[p][0] + pair_first[p][1] - 1 (word 0 is
 *   unspecified when the count is 0),
 *   emit_out [dup_capacity] u32 (optional, may be NULL): the emission index
 *   of each sorted entry (aligned with ids_out).
 * The true duplicate count is written to status[1]; when it exceeds
 * dup_capacity, GS_FLAG_CAPACITY is set, the list is truncated to the first
 * dup_capacity entries in emission order and the ranges are NOT meaningful:
 * the caller detects it with gs_check_status, grows the buffers and reruns. */
gs_status gs_bin_sort(const gs_projected* proj, const gs_views* views,
                      const gs_tiling* tiling, int64_t dup_capacity,
                      void* ws, size_t ws_bytes, uint64_t* keys_out,
                      uint32_t* ids_out, uint32_t* tile_ranges,
                      uint32_t* pair_first, uint32_t* emit_out, int64_t* status,
                      void* stream);

/* How the rasterisers walk the tiles of a call (optional; NULL = one
 * work-group per tile in an XCD-aware order).
 *   tile_order       device [S * tiles] permutation of the tiles (e.g. the
 *                    longest-first order from gs_tile_order), or NULL
 *   queue            device u32 work counter: when set, a persistent grid of
 *                    persistent_waves work-groups (0 = 16 per CU) pulls tiles
 *                    atomically in tile_order order; the call resets it.
 * Chunked backward (STORED mode only): with chunk > 0 (a multiple of 64) the
 * backward cuts every tile list into `chunk`-entry work items that run in
 * parallel; the forward then stores, for each pixel and every `chunk`
 * entries, the transmittance there and the (transmittance-normalised) colour
 * still to come behind it into checkpoints [max_items][tile_w*tile_h] float4,
 * and the backward starts each item from them.
 *   chunk_offset [n_tiles + 1], chunk_items [max_items]: from gs_chunk_items
 *   after gs_bin_sort (the same plan must be passed to both raster calls).
 * fwd_waves: waves per tile in the forward (0 or 1 = one wave per tile; 2 or
 * 4 split the tile's pixels over that many waves of one work-group, which
 * shortens the longest tiles; must divide tile_w * tile_h / 64; not with a
 * queue).
 * Split forward (fwd_split = 1, chunked STORED mode only): the forward
 * composites every chunk item in parallel from a local transmittance of 1
 * (one wave per item; chunk_last [max_items][tile_w*tile_h] u16 device
 * workspace receives each item's chunk-local position of the last blend per
 * pixel), then one wave per tile joins its chunks in list order, composites
 * again with the stop rule the chunk in which a pixel's transmittance
 * reaches the cut-off, and writes the image, T_final, n_contrib and the
 * backward's checkpoints.  Long tile lists then no longer run on one wave
 * each; the results equal the sequential forward's up to FP32 rounding of
 * the transmittance products and colour sums.
 * Deterministic gradients: with dup_grads ([dup_capacity][9] f32 device
 * workspace; dup_capacity as passed to gs_bin_sort), pair_first ([m][2]) and
 * emit_idx (pair_first and emit_out of gs_bin_sort of the same step) set,
 * the backward writes each (tile, pair) entry's 9 gradient components into
 * the slot of its emission index instead of adding them atomically, then
 * sums every pair's slots in emission order into d_rec: no atomics, and
 * gradients are bitwise reproducible.
 * Images do not depend on the plan; gradients only up to FP32 summation
 * order.                                                                   */
typedef struct {
  const uint32_t* tile_order;
  uint32_t* queue;
  int32_t persistent_waves;
  int32_t chunk;
  const uint32_t* chunk_offset;
  const uint32_t* chunk_items;
  float* checkpoints;
  int64_t max_items;
  int32_t fwd_waves;
  int32_t fwd_split;
  float* dup_grads;
  const uint32_t* pair_first;
  int64_t dup_capacity;
  const uint32_t* emit_idx;
  uint16_t* chunk_last;
} gs_raster_plan;

/* Upper bound on the work items of gs_chunk_items for a duplicate capacity. */
int64_t gs_chunk_max_items(int64_t n_tiles, int64_t dup_capacity, int32_t chunk);

/* Work items of the chunked backward: chunk_offset[t] = first item of tile t
 * (chunk_offset[n_tiles] = item count = sum of ceil(len_t / chunk)),
 * chunk_items[i] = tile of item i.  Device arrays, no host sync.  Entries of
 * chunk_items past the item count are unspecified (above 16384 tiles the
 * call keeps per-block sums there while it scans).                         */
gs_status gs_chunk_items(const uint32_t* tile_ranges, int64_t n_tiles, int32_t chunk,
                         int64_t max_items, uint32_t* chunk_offset, uint32_t* chunk_items,
                         void* stream);

size_t gs_tile_order_workspace_bytes(int64_t n_tiles);

/* Longest-first order of the tiles of a call by list length (bucketed by
 * floor(log2(length + 1)), descending), for load balance of batched,
 * uneven partitions.  tile_ranges as written by gs_bin_sort; order [n_tiles]
 * device output.  The order inside a bucket is unspecified.                */
gs_status gs_tile_order(const uint32_t* tile_ranges, int64_t n_tiles, void* ws,
                        size_t ws_bytes, uint32_t* order, void* stream);

/* Front-to-back compositing (3D-GS rasteriser).  For each pixel p of each
 * slot, over its tile's sorted list: power = -1/2 d^T conic d with
 * d = p - mean2d (skipped if power > 0); alpha = min(0.99, o e^power),
 * skipped if alpha < 1/255; the loop stops before a Gaussian whose blend
 * would take the transmittance T below 1e-4; C += rgb alpha T,
 * T *= (1 - alpha).  image = C + T bg.
 * Outputs (device): image [S][3][H][W]; T_final [S][H][W] and n_contrib
 * [S][H][W] (list position after the last blended entry), both optional
 * (NULL) when the backward will run in recompute mode.  bg: 3 host floats. */
gs_status gs_raster_fwd(const gs_projected* proj, const gs_views* views,
                        const gs_tiling* tiling, const uint32_t* ids,
                        const uint32_t* tile_ranges, const float bg[3],
                        float* image, float* T_final, int32_t* n_contrib,
                        const gs_raster_plan* plan, void* stream);

#define GS_BWD_STORED 0     /* use T_final / n_contrib from the forward      */
#define GS_BWD_RECOMPUTE 1  /* replay the forward per tile to recover them   */

/* Reverse-order replay of the compositing: the exact derivative of
 * gs_raster_fwd with every skip/stop/clamp decision held fixed (the
 * derivative through a clamped alpha is zero).  d_image [S][3][H][W] is
 * dL/d(image).  Accumulates (+=) into d_rec [m][9] (caller zeroes it).
 * mode GS_BWD_STORED needs T_final and n_contrib; GS_BWD_RECOMPUTE ignores
 * them (may be NULL).                                                      */
gs_status gs_raster_bwd(const gs_projected* proj, const gs_views* views,
                        const gs_tiling* tiling, const uint32_t* ids,
                        const uint32_t* tile_ranges, const float bg[3],
                        const float* T_final, const int32_t* n_contrib,
                        const float* d_image, int32_t mode, float* d_rec,
                        const gs_raster_plan* plan, void* stream);

/* Measurement helper, not part of the training step: per pixel, the number
 * of list entries the front-to-back compositing of gs_raster_fwd blends
 * (alpha test passed, transmittance still at or above 1e-4 after it), with
 * the same FP32 decisions.  These (pixel, Gaussian) pairs are the work an
 * exact rasteriser cannot avoid, which prices the rasteriser's roofline.
 * n_blend [S][H][W] int32 (device, caller-owned, fully written).  Tiles of
 * at most 512 pixels.  Errors as gs_raster_fwd.                            */
gs_status gs_raster_count(const gs_projected* proj, const gs_views* views,
                          const gs_tiling* tiling, const uint32_t* ids,
                          const uint32_t* tile_ranges, int32_t* n_blend, void* stream);

/* Chain rule from d_rec back to the Gaussian parameters (sum over every
 * slot that draws the Gaussian), accumulating (+=) into grads.  Depth, the
 * support and the bboxes carry no gradient.  Deterministic (no atomics).   */
gs_status gs_project_bwd(const gs_gaussians* g, const gs_views* views,
                         const gs_tiling* tiling, const gs_projected* proj,
                         const float* d_rec, gs_grads* grads, void* stream);

size_t gs_loss_workspace_bytes(int32_t S, int32_t H, int32_t W);

/* Background-masked photometric loss per image s (Sec. II masks):
 *   I^ = M image, G^ = M target (M broadcast over rgb; mask NULL = all 1),
 *   L1 = mean |I^ - G^| over 3HW,  SSIM = mean over 3HW of the SSIM map with
 *   an 11x11 Gaussian window (sigma 1.5), zero padding, C1 = 0.01^2,
 *   C2 = 0.03^2;  loss[s] = (1 - lambda) L1 + lambda (1 - SSIM).
 * Writes loss_out [S] (device) and d_image [S][3][H][W] = grad_scale *
 * dloss[s]/d(image) (sign(0) = 0 in the L1 subgradient).  A non-finite loss
 * sets GS_FLAG_NONFINITE in status (may be NULL).                          */
gs_status gs_loss(const float* image, const float* target,
                  const uint8_t* mask, int32_t S, int32_t H, int32_t W,
                  float lambda_dssim, float grad_scale, void* ws,
                  size_t ws_bytes, float* loss_out, float* d_image,
                  int64_t* status, void* stream);

/* gs_loss without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, outputs and errors as gs_loss, minus
 * ws / ws_bytes: the partial sums live in a 4 MiB array inside the library,
 * one per device, held until the process ends (S x ceil(H/32) x ceil(W/32)
 * x 24 bytes must fit: e.g. up to 85 images of 1920x1080).  Larger requests
 * fail with GS_ERR_ARG and enqueue nothing.  The call allocates nothing.
 * Every call on a device shares that device's array, so calls that overlap
 * on one device (other streams, other threads) race; calls ordered on one
 * stream do not.                                                           */
gs_status gs_loss_noalloc(const float* image, const float* target,
                          const uint8_t* mask, int32_t S, int32_t H, int32_t W,
                          float lambda_dssim, float grad_scale, float* loss_out,
                          float* d_image, int64_t* status, void* stream);

/* Workspace for gs_masked_psnr on S images of H x W.                      */
size_t gs_psnr_workspace_bytes(int32_t S, int32_t H, int32_t W);

/* Masked PSNR of each image s, the reconstruction metric the trainers stop
 * on (PSNR, Sec. III; restricted to the object by the background mask of
 * Sec. II "Image Rendering and Masking"):
 *   se = sum over pixels p with mask[s][p] != 0 of
 *        sum_c (clamp(image[s][c][p], 0, 1) - target[s][c][p])^2,
 *   cnt = 3 x (number of such pixels),
 *   psnr_out[s] = 10 log10(cnt / se)  (images in [0, 1], peak 1),
 *   +inf when se = 0 < cnt, NaN when cnt = 0 (an empty mask).
 * image, target [S][3][H][W] f32, mask [S][H][W] u8 (NULL = all pixels),
 * psnr_out [S] f32: device.  Sums in FP64 in a fixed order (reproducible).
 * ws: gs_psnr_workspace_bytes, 8-byte aligned.                             */
gs_status gs_masked_psnr(const float* image, const float* target, const uint8_t* mask,
                         int32_t S, int32_t H, int32_t W, void* ws, size_t ws_bytes,
                         float* psnr_out, void* stream);

/* x[r][i] *= scale[r] for rows r < rows and i < row_len (device arrays): the
 * chain rule of the per-image loss of gs_loss through an upstream gradient
 * (autograd).                                                              */
gs_status gs_scale_rows(float* x, const float* scale, int64_t rows, int64_t row_len,
                        void* stream);

/* One parameter group of gs_adam: count fp32 elements at param/grad/m/v.  */
typedef struct {
  float* param;
  float* grad;
  float* m;
  float* v;
  int64_t count;
  float lr;
} gs_adam_group;
#define GS_MAX_ADAM_GROUPS 8

/* Adam with bias correction, dense over every element (step counts from 1):
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   param -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * groups: host array of n_groups (<= GS_MAX_ADAM_GROUPS).  zero_grad != 0
 * clears each grad after reading it.                                      */
gs_status gs_adam(const gs_adam_group* groups, int32_t n_groups, float beta1,
                  float beta2, float eps, int32_t step, int32_t zero_grad,
                  void* stream);

/* Workspace for gs_knn on n points.                                         */
size_t gs_knn_workspace_bytes(int64_t n, int32_t k);

/* Exact k nearest neighbours of every point among the other points
 * (Euclidean, FP32), used by the initialisation: the plain one sets a
 * Gaussian's isotropic scale to the mean distance to its 3 nearest
 * neighbours, the learned one reads 16-NN offsets (isosurface points,
 * Sec. II "Isosurface Extraction").
 *   pts [3][n] device (planar x, y, z); idx [n][k] i32 and dist [n][k] f32
 *   device outputs sorted by (distance, index); missing neighbours (n <= k)
 *   are -1 / +inf.  mean_dist [n] f32 device output: the arithmetic mean of
 *   the distances to the neighbours found, summed nearest first (0 when
 *   n = 1).  Each of idx, dist and mean_dist may be NULL (not written); at
 *   least one must be given.  1 <= k <= 32, n < 2^31.  ws:
 *   gs_knn_workspace_bytes, 256-byte aligned.  Uniform grid + shell search
 *   with an exact stopping bound; no host synchronisation.                 */
gs_status gs_knn(const float* pts, int64_t n, int32_t k, void* ws, size_t ws_bytes,
                 int32_t* idx, float* dist, float* mean_dist, void* stream);

/* Workspace for gs_plain_init on n points.                                 */
size_t gs_plain_init_workspace_bytes(int64_t n);

/* The plain initialisation of the Gaussians of n isosurface points (one
 * Gaussian per extracted point, Sec. II "Isosurface Extraction"; shape from
 * the 3D-GS default the paper trains with):
 *   mean = pts, color [3][n] = sqrt(pi) normals (degree-0 colour (n+1)/2
 *   for unit normals), and, when log_scale is not NULL:
 *   log_scale [3][n] = log(max(d, 1e-6)) with d the mean distance to the 3
 *   nearest other points (gs_knn), quat [4][n] = (1, 0, 0, 0),
 *   opacity_logit [n] = log(opacity / (1 - opacity)), 0 < opacity < 1.
 * With log_scale NULL only mean and colour are written (ws, quat and
 * opacity_logit unused): the learned initialisation takes the shape from
 * gs_mlp_apply.  pts, normals [3][n] device; outputs planar device arrays.
 * ws: gs_plain_init_workspace_bytes(n), 256-byte aligned.                  */
gs_status gs_plain_init(const float* pts, const float* normals, int64_t n, float opacity,
                        void* ws, size_t ws_bytes, float* mean, float* log_scale, float* quat,
                        float* opacity_logit, float* color, void* stream);

/* gs_adam with the step count on the device, so that a captured HIP graph
 * can replay training steps unchanged: the kernels use t = step_dev[0] + 1
 * for the bias corrections and, for group g with lr_final[g] > 0 (host
 * array, may be NULL), the log-linear decay lr_g (lr_final[g]/lr_g)^min(t /
 * decay_steps, 1) (the 3D-GS position schedule); a last kernel stores
 * step_dev[0] = t.  step_dev: one device int32, 0 before the first step.   */
gs_status gs_adam_dev(const gs_adam_group* groups, int32_t n_groups, const float* lr_final,
                      int32_t decay_steps, float beta1, float beta2, float eps,
                      int32_t* step_dev, int32_t zero_grad, void* stream);

/* gs_project_bwd into zeroed gradients followed by gs_adam_dev, in one pass
 * over the Gaussians (the 3D-GS step's last two stages): each Gaussian's
 * gradient, summed over its pairs of `views`, stays in registers and updates
 * its parameters (11 + the colour rows), m and v in place at once, so the
 * gradient arrays are neither written nor read.  Bitwise equal to the two
 * calls.
 *   groups: 5 groups in the order mean, log_scale, quat, opacity_logit,
 *   color whose param arrays are g's (counts 3n, 3n, 4n, n, rows x n) with
 *   their m, v and lr; rows is a multiple of 3 from 3 (D+1)^2 (D =
 *   g->sh_degree) to 48: stored rows past the active degree are updated with
 *   a zero gradient, as a dense gs_adam_dev would.  grad pointers are not
 *   used.  n_groups = 6 gives the colour rows from 3 on their own learning
 *   rate (3D-GS steps the higher spherical-harmonic bands at 1/20 of the
 *   plain colour's): group 4 is then the first 3 rows (count 3n) and group
 *   5 the rest of the same arrays (param, m and v at group 4's plus 3n,
 *   count (rows - 3) x n); lr_final has n_groups entries.
 *   visible_only != 0: sparse Adam, the optimiser form that updates only the
 *   Gaussians a step draws: a Gaussian with no pair of `views` whose n_tiles
 *   is > 0 keeps its parameters, m and v unchanged (and none of them is
 *   read); the step count and its bias corrections stay global.  With 0,
 *   every Gaussian is updated (dense, the 3D-GS default).  lr_final (5 or NULL),
 *   decay_steps, betas, eps and step_dev as gs_adam_dev (step_dev is
 *   incremented).  Gaussians drawn by no pair get a zero gradient.         */
gs_status gs_project_bwd_adam(const gs_gaussians* g, const gs_views* views,
                              const gs_tiling* tiling, const gs_projected* proj,
                              const float* d_rec, const gs_adam_group* groups,
                              int32_t n_groups, const float* lr_final,
                              int32_t decay_steps, float beta1,
                              float beta2, float eps, int32_t visible_only, int32_t* step_dev,
                              void* stream);

/* ------------------------------------------------------------------------
 * Microbenchmarks of the units the rooflines price (measurement helpers, not
 * part of the training step).  The caller times each launch with events on
 * `stream`; all buffers are device memory it owns.
 *   gs_peak_copy:   dst = src, `bytes` (multiple of 16, 16-byte aligned): HBM
 *                   bandwidth = 2 bytes / time.
 *   gs_peak_fma:    blocks x 256 lanes x iters x 16 FP32 fused multiply-adds
 *                   (no packed FP32 instructions); out [blocks * 256].
 *   gs_peak_exp:    the same count of hardware base-2 exponentials.
 *   gs_peak_lds:    blocks x 256 lanes x iters x 4 LDS reads of 16 bytes.
 *   gs_peak_atomic: blocks x 256 lanes x iters FP32 atomic adds of 1 to
 *                   hashed addresses of dst [n_addr >= 64]: one hash per
 *                   lane, or (contiguous != 0) one per wave with its lanes
 *                   on 64 consecutive floats.
 *   gs_peak_mfma:   blocks x 4 waves x iters x 8 BF16 16x16x32 matrix
 *                   multiply-accumulates (16384 flops each); out [blocks*256].
 * Errors: GS_ERR_ARG on NULL buffers or non-positive counts.               */
gs_status gs_peak_copy(const void* src, void* dst, int64_t bytes, void* stream);
gs_status gs_peak_fma(float* out, int32_t blocks, int32_t iters, void* stream);
gs_status gs_peak_exp(float* out, int32_t blocks, int32_t iters, void* stream);
gs_status gs_peak_lds(float* out, int32_t blocks, int32_t iters, void* stream);
gs_status gs_peak_atomic(float* dst, int64_t n_addr, int32_t blocks, int32_t iters,
                         int32_t contiguous, void* stream);
gs_status gs_peak_mfma(float* out, int32_t blocks, int32_t iters, void* stream);

/* ------------------------------------------------------------------------
 * Adaptive density control of the 3D-GS method each partition is trained
 * with (Sec. II "Parallel Training"; the paper keeps its defaults): every
 * few hundred steps, Gaussians whose mean screen-space position gradient is
 * large are cloned (small ones) or split in two (large ones), faint or
 * oversized ones are pruned, and opacities are periodically clamped.
 *   per step:   gs_densify_stats after gs_raster_bwd
 *   densify:    gs_densify_select -> (host reads n_out) -> gs_densify_apply
 *               into arrays of n_out Gaussians; the caller resets the
 *               statistics (gs_zero)
 * A Gaussian's state: parameters in the planar layouts of gs_gaussians and
 * its Adam moments in the same layouts, in the order mean, log_scale, quat,
 * opacity_logit, color (m and v of a group may both be NULL).             */
typedef struct {
  float* param[5];
  float* m[5];
  float* v[5];
  int64_t n;
  int32_t color_rows;   /* rows of the colour arrays, 3 (D+1)^2; 0 means 3 */
  int32_t reserved;
} gs_gaussian_state;

/* accum[g] += sum over g's visible pairs (n_tiles > 0) of |(dL/dmean2d_x W/2,
 * dL/dmean2d_y H/2)| (the gradient of the projected mean in normalised
 * device coordinates; FP32, one correctly rounded operation at a time);
 * denom[g] += their count.  d_rec as gs_raster_bwd writes it; accum, denom [n] device.      */
gs_status gs_densify_stats(const gs_views* views, const gs_tiling* tiling,
                           const gs_projected* proj, const float* d_rec, int64_t n,
                           float* accum, float* denom, void* stream);

size_t gs_densify_workspace_bytes(int64_t n);

/* Per Gaussian (FP32 comparisons of the inputs with the thresholds):
 * faint = opacity_logit < min_opacity_logit; grow = denom > 0 and
 * accum >= grad_threshold x denom (exact); L = max log-scale.  Action:
 *   faint                              -> dropped
 *   grow, L <= max_log_scale_clone     -> kept and cloned (2 outputs)
 *   grow, L >  max_log_scale_clone     -> split into 2 children with
 *                                         log-scales minus log_split
 *   otherwise                          -> kept
 * and any output whose largest log-scale exceeds max_log_scale is dropped.
 * action [n] i32 device (0 drop, 1 keep, 2 clone, 3 split); n_out: one
 * device i64, the number of outputs; ws (gs_densify_workspace_bytes, 8-byte
 * aligned) keeps the per-block output offsets for gs_densify_apply.        */
gs_status gs_densify_select(const gs_gaussian_state* state, const float* accum,
                            const float* denom, float grad_threshold,
                            float max_log_scale_clone, float min_opacity_logit,
                            float max_log_scale, float log_split, void* ws,
                            size_t ws_bytes, int32_t* action, int64_t* n_out,
                            void* stream);

/* Writes the outputs in input order: a kept Gaussian once with its moments;
 * a clone twice, the copy with zero moments; a split Gaussian as two
 * children c = 0, 1 at mean + R(q/|q|) (exp(log_scale) * z[g][c]) with
 * log_scale - log_split, the rest of its parameters copied, zero moments.
 * z [n][2][3] device standard normal samples (the random draws of the
 * split, passed in).  in / action / ws from gs_densify_select; out->n must
 * be its n_out (outputs past out->n are not written).  in and out must not
 * overlap.                                                                  */
gs_status gs_densify_apply(const gs_gaussian_state* in, const int32_t* action,
                           const void* ws, const float* z, float log_split,
                           gs_gaussian_state* out, void* stream);

/* opacity_logit = min(opacity_logit, max_opacity_logit); the opacity
 * group's moments (if given) are cleared.                                   */
gs_status gs_opacity_reset(gs_gaussian_state* state, float max_opacity_logit, void* stream);

/* ------------------------------------------------------------------------
 * Learned initialisation.  The paper places one Gaussian at every point of
 * the extracted isosurface (Sec. II, "Isosurface Extraction") and leaves its
 * starting shape to the 3D-GS default (isotropic, scale from the 3 nearest
 * neighbours, see gs_knn).  These calls add a small network that predicts
 * the starting log-scale, rotation and opacity of each Gaussian from its 16
 * nearest isosurface points, trained on Gaussians the training step itself
 * has fitted:
 *   inference: gs_knn(k=16) -> gs_mlp_features -> gs_mlp_fwd -> gs_mlp_apply
 *   training:  gs_mlp_targets (once) then per step gs_mlp_fwd ->
 *              gs_mlp_loss -> gs_mlp_bwd -> gs_adam
 * Network: y = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3, 96 -> 64 -> 64 -> 8,
 * bf16 MFMA products with fp32 accumulation.  The bf16 roundings are:
 * x (stored bf16), the weights (rounded from the fp32 masters when loaded),
 * both hidden activations after bias + ReLU; in the backward also dy, dZ2
 * and dZ1 (after the ReLU mask).  Biases, pre-activations and outputs fp32.
 * Per point: y[0:3] log-scale offset, y[3:7] quaternion (w, x, y, z) in the
 * point's local frame (unnormalised), y[7] opacity logit.
 *
 * Local frame of a point with unit normal n: z = n, x = normalise(n x e)
 * with e the world axis least aligned with n (lowest index on ties),
 * y = z x x.  F = the 3x3 matrix whose rows are x, y, z (world -> local).
 * ------------------------------------------------------------------------ */

/* fp32 master weights, all device, row-major (input index first):
 *   w1 [96][64], w2 [64][64], w3 [64][8], b1 [64], b2 [64], b3 [8].         */
typedef struct {
  const float* w1;
  const float* w2;
  const float* w3;
  const float* b1;
  const float* b2;
  const float* b3;
} gs_mlp;

/* Gradient outputs of gs_mlp_bwd, same shapes as gs_mlp; they are ADDED to.
 * dx: [n][96] fp32 gradient of the features, overwritten; may be NULL.   */
typedef struct {
  float* dw1;
  float* dw2;
  float* dw3;
  float* db1;
  float* db2;
  float* db3;
  float* dx;
} gs_mlp_grads;

/* Features of n isosurface points from their 16 nearest neighbours
 * (gs_knn with k = 16: idx/dist [n][16], sorted, -1 = missing).
 *   pts, normals [3][n] device (normals need not be unit length).
 *   x_bf16 [n][96] device out, 16-byte aligned: for neighbour k,
 *     x[6k..6k+2] = F (p_j - p) / dbar,  x[6k+3..6k+5] = F n_j
 *     (zero for a missing neighbour), rounded to bf16 (nearest even).
 *   dbar [n] device out: mean distance over the present neighbours (1 if
 *     none).  n < 2^31.                                                   */
gs_status gs_mlp_features(const float* pts, const float* normals, int64_t n,
                          const int32_t* knn_idx, const float* knn_dist,
                          uint16_t* x_bf16, float* dbar, void* stream);

/* Forward: y [n][8] fp32 device out for x_bf16 [n][96] (16-byte aligned).
 * w: host struct of device pointers.  n = 0 is a no-op.                   */
gs_status gs_mlp_fwd(const uint16_t* x_bf16, int64_t n, const gs_mlp* w,
                     float* y, void* stream);

/* Workspace for gs_mlp_bwd on n points (per-work-group partial sums).     */
size_t gs_mlp_bwd_workspace_bytes(int64_t n);

/* Backward for upstream dy [n][8] fp32: recomputes the forward and adds the
 * parameter gradients to g (host struct of device pointers); writes g->dx
 * if it is not NULL.  ws: gs_mlp_bwd_workspace_bytes(n), 256-byte aligned.
 * The reduction order is fixed: results are deterministic.                */
gs_status gs_mlp_bwd(const uint16_t* x_bf16, int64_t n, const gs_mlp* w,
                     const float* dy, gs_mlp_grads* g, void* ws,
                     size_t ws_bytes, void* stream);

/* Training targets from fitted Gaussians (same identity as the points):
 *   target[i][0:3] = log_scale[:, i] - log dbar[i],
 *   target[i][3:7] = unit quaternion of F R(quat[:, i]) with w >= 0,
 *   target[i][7]   = opacity_logit[i].
 * log_scale [3][n], quat [4][n], opacity_logit [n], normals [3][n],
 * dbar [n] device in; target [n][8] device out.                            */
gs_status gs_mlp_targets(const float* log_scale, const float* quat,
                         const float* opacity_logit, const float* normals,
                         const float* dbar, int64_t n, float* target,
                         void* stream);

/* Workspace for gs_mlp_loss on n points.                                   */
size_t gs_mlp_loss_workspace_bytes(int64_t n);

/* Loss = (1/n) sum_i [ sum_{a<3} (y_a - t_a)^2 + (y_7 - t_7)^2
 *                      + 1 - |<y[3:7]/|y[3:7]|, t[3:7]>| ]
 * (the rotation term is blind to the sign of the quaternion).  Writes
 * dy = dLoss/dy [n][8] and the loss to loss_out (one device float).  n >= 1.
 * ws: gs_mlp_loss_workspace_bytes(n).                                      */
gs_status gs_mlp_loss(const float* y, const float* target, int64_t n, float* dy,
                      void* ws, size_t ws_bytes, float* loss_out, void* stream);

/* Initial Gaussians from network outputs y [n][8]:
 *   log_scale[a][i] = log dbar[i] + y[i][a],
 *   quat[:, i] = unit quaternion (w >= 0) of F^T R(y[i][3:7]),
 *   opacity_logit[i] = y[i][7].
 * The inverse of gs_mlp_targets.  All device; outputs planar SoA.          */
gs_status gs_mlp_apply(const float* y, const float* normals, const float* dbar,
                       int64_t n, float* log_scale, float* quat,
                       float* opacity_logit, void* stream);

/* Fill `bytes` bytes at device pointer `ptr` with zero using a kernel (safe
 * to capture in a HIP graph).  bytes must be a multiple of 4.             */
gs_status gs_zero(void* ptr, size_t bytes, void* stream);

/* Synchronise `stream`, read the status block and report:
 * GS_ERR_CAPACITY (required duplicates in *required_out), GS_ERR_NONFINITE,
 * or GS_OK.  required_out may be NULL.                                    */
gs_status gs_check_status(const int64_t* status, void* stream,
                          int64_t* required_out);

/* HIP-graph handles of a whole training step (the batched, persistent step
 * of one or more partitions and views that Sec. II "Parallel Training" runs
 * per partition, replayed so the step costs one launch).
 *
 * gs_graph_begin starts capturing `stream` (a created stream, not the null
 * stream; thread-local capture mode, so an unsafe call such as a device
 * allocation made by this thread during the capture invalidates it).  The
 * library's calls enqueued on `stream` until gs_graph_end are recorded, not
 * run.  Every library call is capturable: data-dependent sizes stay on the
 * device and clears are kernels (gs_zero), never memset nodes.
 * gs_graph_end stops the capture, instantiates it and returns a
 * library-owned handle in *out (NULL on failure: GS_ERR_HIP when the capture
 * was invalidated or instantiation failed).
 * gs_graph_launch enqueues one replay on `stream` (any stream, the null
 * stream included).  A replay reads the device buffers the captured calls
 * named, at their current contents, so those buffers must stay allocated
 * while the handle is used.  gs_graph_destroy frees the handle (NULL is a
 * no-op); work already launched is unaffected.                            */
typedef struct gs_graph gs_graph;
gs_status gs_graph_begin(void* stream);
gs_status gs_graph_end(void* stream, gs_graph** out);
gs_status gs_graph_launch(gs_graph* graph, void* stream);
void gs_graph_destroy(gs_graph* graph);

/* Thread-local text of the last error ("" if none).                        */
const char* gs_last_error(void);

/* Library version string.                                                  */
const char* gs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GS_H */
