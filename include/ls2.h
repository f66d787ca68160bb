/*
 * ls2.h -- C ABI of libls2, the MI355X (gfx950) sparse-coefficient Gaussian
 * splatting library (LangSplatV2, arXiv 2507.07136).
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless marked (host).  Arrays are
 *     row-major and contiguous.  The caller owns all memory; the library
 *     never allocates or frees (scratch comes in through a caller-sized
 *     workspace where one is needed).  The one exception is
 *     ls2_splat_decode_query_noalloc, which uses a fixed scratch array the
 *     library holds per GPU.
 *   - Calls are asynchronous on `stream` unless documented otherwise.  Apart
 *     from that scratch array and the check mode's flag word, there is no
 *     global state: calls on different streams do not interact.
 *   - Invalid sizes or null required pointers return LS2_ERR_ARG before any
 *     work is enqueued.  Shapes outside the compiled kernel set return
 *     LS2_ERR_UNSUPPORTED.  A HIP launch failure returns LS2_ERR_DEVICE.
 *   - Pixel (px, py) is sampled at (px + 0.5, py + 0.5).  Screen tiles are
 *     16 x 16 pixels, numbered row-major: tile = ty * ceil(W/16) + tx.
 *   - Code indices (topk_idx) must lie in [0, L).  By default they are taken
 *     modulo L (L is a power of two), so a bad index never reads or writes
 *     out of bounds but lands on another atom.  With the environment variable
 *     LS2_CHECK=1, or after ls2_set_check(1), every entry point that reads
 *     topk_idx first scans it and returns LS2_ERR_ARG if any index is out of
 *     range; the scan synchronises the stream once (a debugging mode, not for
 *     stream capture, and concurrent checking calls on one device share one
 *     flag word).
 */
#ifndef LS2_H
#define LS2_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LS2_TILE 16

enum {
    LS2_OK = 0,
    LS2_ERR_ARG = -1,          /* invalid argument (null pointer, negative size, K > L, ...) */
    LS2_ERR_CAPACITY = -2,     /* more pairs than max_pairs (ls2_bin_sort); shape beyond the fixed scratch (_noalloc) */
    LS2_ERR_UNSUPPORTED = -3,  /* shape outside the compiled set */
    LS2_ERR_DEVICE = -4        /* HIP runtime error */
};

enum { LS2_F32 = 0, LS2_BF16 = 1 };

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  world_to_cam is
 * the 3x4 row-major [R | t]; a world point X maps to p = R X + t.  Passed by
 * (host) pointer. */
typedef struct ls2_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float world_to_cam[12];
    float znear;               /* Gaussians with camera z <= znear are culled */
} ls2_camera;
/* Every entry point taking a camera returns LS2_ERR_ARG unless width and
 * height are in [1, 32768], the intrinsics and world_to_cam are finite and
 * znear is finite and > 0. */

/* Human-readable text for a status code (static storage). */
const char* ls2_status_string(int status);

/* Library version, major * 10000 + minor * 100 + patch. */
int ls2_version(void);

/* Fingerprint of the sources the library was built from (16 hex digits, or
 * "unknown"); the Python binding refuses a library whose fingerprint differs
 * from the sources beside it.  Static storage. */
const char* ls2_source_hash(void);

/* Turns the code-index check on (enabled != 0) or off for the whole process,
 * overriding LS2_CHECK; returns the previous setting (0 or 1). */
int ls2_set_check(int enabled);

/*
 * ls2_project -- per-Gaussian projection to the image plane.
 *
 * Section 3.1, Eqs. 1-2: Sigma = R S S^T R^T with R from the unit quaternion
 * q = (w, x, y, z) (normalised here) and S = diag(scales).  The paper cites
 * EWA splatting for the projection; this library uses the local affine
 * Jacobian J of the perspective map at the camera-space mean p = (x, y, z),
 * J = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]], the screen covariance
 * Sigma2D = J R_wc Sigma R_wc^T J^T + 0.3 I, and a radius of
 * ceil(3 sqrt(lambda_max(Sigma2D))) pixels.
 *
 * In:  means [n,3], scales [n,3] (> 0), quats [n,4] (w, x, y, z).
 * Out: mean2d [n,2] = (fx x/z + cx, fy y/z + cy); conic [n,3] = the inverse of
 *      Sigma2D as (A, B, C) with Sigma2D^-1 = [[A, B], [B, C]]; depth [n] = z;
 *      radius [n]; tiles_touched [n] = number of 16x16 tiles in the rectangle
 *      [floor((u-r)/16), floor((u+r)/16)] x [floor((v-r)/16), floor((v+r)/16)]
 *      clipped to the grid (evaluated in float32).
 * A Gaussian is culled (radius = 0, tiles_touched = 0, other outputs 0) if
 * z <= znear, any value is non-finite, det(Sigma2D) <= 0, or its rectangle
 * is empty.  n = 0 is a no-op.
 */
int ls2_project(const ls2_camera* cam, int32_t n, const float* means, const float* scales,
                const float* quats, float* mean2d, float* conic, float* depth, int32_t* radius,
                int32_t* tiles_touched, hipStream_t stream);

/*
 * ls2_bin_sort -- tile binning and per-tile depth order.
 *
 * Eq. 3 composites each tile's Gaussians in front-to-back order: every visible
 * Gaussian contributes one (tile, Gaussian) pair per tile of its rectangle
 * (same float32 rule as ls2_project), and each tile's pairs are ordered by
 * float32 depth, ties broken by Gaussian id (a unique, total order).
 *
 * In:  mean2d [n,2], radius [n], depth [n] from ls2_project.
 * Out: ids [P] (Gaussian id of each pair, grouped by tile, depth-ordered);
 *      keys [P] = (tile << 32) | float32 bits of depth (optional: may be NULL);
 *      tile_ranges [tiles,2] = [start, end) of each tile's list in ids (tiles
 *      row-major).  The lists are stored superblock by superblock: the tile
 *      grid is cut into superblocks of S x S tiles (S = 4, or the smallest
 *      larger power of two that keeps the superblocks within 4096),
 *      superblocks in row-major order and the tiles of one superblock
 *      row-major inside it; start is the number of pairs of all tiles before
 *      it in this order (an empty tile has start = end).  P is at most
 *      max_pairs.  If P > max_pairs every range is [0, 0).
 * workspace: device scratch of at least ls2_bin_sort_workspace() bytes,
 *      256-byte aligned, owned by the caller, not shared between concurrent
 *      calls.
 * num_pairs (host, optional): if non-NULL the call synchronises the stream
 *      once and stores P; if P > max_pairs it returns LS2_ERR_CAPACITY (grow
 *      the buffers and call again).  If NULL the call does not synchronise;
 *      on overflow every tile range is left empty and P can be read later
 *      with ls2_bin_sort_count().
 */
int ls2_bin_sort_workspace(const ls2_camera* cam, int32_t n, int64_t max_pairs, size_t* bytes);
int ls2_bin_sort(const ls2_camera* cam, int32_t n, const float* mean2d, const int32_t* radius,
                 const float* depth, int64_t max_pairs, uint64_t* keys, uint32_t* ids,
                 uint32_t* tile_ranges, int64_t* num_pairs, void* workspace, size_t workspace_bytes,
                 hipStream_t stream);
/* P of the last ls2_bin_sort (or ls2_project_bin_sort) that used this
 * workspace (synchronises stream). */
int ls2_bin_sort_count(const void* workspace, int64_t* num_pairs, hipStream_t stream);

/*
 * ls2_project_bin_sort -- ls2_project followed by ls2_bin_sort (Section 3.1,
 * Eqs. 1-2, then the depth-ordered tile lists of Eq. 3) with one launch fewer:
 * the binning's first pass projects each Gaussian itself, with the same
 * instructions as ls2_project, writes the projection's outputs and takes the
 * tile rectangle from the results in registers.  Every output equals that of
 * the two calls bit for bit.  Arguments as in ls2_project (mean2d, conic,
 * depth, radius out; tiles_touched optional) and ls2_bin_sort (the same
 * workspace, from ls2_bin_sort_workspace).
 */
int ls2_project_bin_sort(const ls2_camera* cam, int32_t n, const float* means, const float* scales,
                         const float* quats, float* mean2d, float* conic, float* depth, int32_t* radius,
                         int32_t* tiles_touched, int64_t max_pairs, uint64_t* keys, uint32_t* ids,
                         uint32_t* tile_ranges, int64_t* num_pairs, void* workspace, size_t workspace_bytes,
                         hipStream_t stream);

/*
 * ls2_splat_sparse -- efficient sparse coefficient splatting.
 *
 * Section 3.4 and Appendix A (Algorithm 1), with the compositing rule of
 * Eq. 3: for each pixel v, walk its tile's ordered list front to back with
 * alpha_i = min(0.99, o_i exp(-0.5 d^T conic_i d)), d = mean2d_i - v; skip
 * alpha_i < 1/255; stop (without blending) once T (1 - alpha_i) < 1e-4;
 * otherwise for every level l and each of the K stored pairs (j, w_ilj):
 *     coef_l(v)[j] += w_ilj * alpha_i * T,   then T *= 1 - alpha_i.
 * Only the K non-zero coefficients are touched (O(K) per Gaussian, not O(L)).
 * Levels share alpha and T (each level's pass takes the same decisions).
 * Repeated indices within one Gaussian's K pairs add their weights.
 *
 * In:  tile_ranges, ids from ls2_bin_sort; mean2d [n,2], conic [n,3] from
 *      ls2_project; opacity [n] in (0,1); topk_idx [n,levels,K] int32 in
 *      [0, L); topk_w [n,levels,K].
 * Out: coef [levels,H,W,L], accumulated in float32 and stored as float32
 *      (coef_dtype LS2_F32) or bfloat16 (LS2_BF16, rounded nearest-even: the
 *      values ls2_dict_decode's bf16 compute rounds a float32 map to, so the
 *      feature map is the same either way); 16-byte aligned.
 *      final_T [H,W] (optional) = transmittance after the last blended
 *      Gaussian; last [H,W] (optional) = 1 + position in the tile list of
 *      the last blended Gaussian (0 if none).
 * Supported: L in {32, 64, 128}, 1 <= K <= 8, levels in {1, 2, 3} with
 * levels * L <= 192.  Out-of-range indices are wrapped modulo L (garbage
 * result, never out-of-bounds access).
 */
int ls2_splat_sparse(const ls2_camera* cam, int32_t n, int32_t levels, int32_t K, int32_t L,
                     const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                     const float* conic, const float* opacity, const int32_t* topk_idx,
                     const float* topk_w, void* coef, int32_t coef_dtype, float* final_T, int32_t* last,
                     hipStream_t stream);

/*
 * ls2_splat_decode -- ls2_splat_sparse followed by Eq. 7's decode F = W S in
 * one pass: each pixel's coefficients, once composited, are rounded to
 * bfloat16 (nearest even) and multiplied by the bfloat16-rounded dictionary on
 * the matrix cores (float32 accumulation), and only the feature map is
 * written.  The features equal ls2_splat_sparse (LS2_BF16 map) followed by
 * ls2_dict_decode (LS2_BF16 compute and output) bit for bit; final_T, last
 * and the optional map equal ls2_splat_sparse's.
 *
 * In:  as ls2_splat_sparse; dict [L,D] f32.
 * Out: feat [levels,H,W,D] bfloat16, 16-byte aligned; coef [levels,H,W,L]
 *      bfloat16 (optional: NULL skips the map), 16-byte aligned; final_T,
 *      last (optional) as ls2_splat_sparse.
 * workspace: at least ls2_splat_decode_workspace() bytes (the dictionary in
 *      bfloat16, repacked by the call), 16-byte aligned, owned by the caller,
 *      not shared between concurrent calls.
 * Supported: as ls2_splat_sparse, and D a multiple of 64 up to 1024.
 */
int ls2_splat_decode_workspace(int32_t L, int32_t D, size_t* bytes);
int ls2_splat_decode(const ls2_camera* cam, int32_t n, int32_t levels, int32_t K, int32_t L, int32_t D,
                     const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                     const float* conic, const float* opacity, const int32_t* topk_idx,
                     const float* topk_w, const float* dict, void* feat, void* coef, float* final_T,
                     int32_t* last, void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * ls2_splat_decode_query -- ls2_splat_decode with the relevancy of Section
 * 3.2 (LERF form, as ls2_query) formed in the same pass: while each chunk of
 * a wave's features is on chip it is scored against the bfloat16-rounded
 * texts on the matrix cores (dot products and squared norms accumulated over
 * the features in increasing order), so the relevancy equals ls2_query on
 * the bfloat16 feature map bit for bit.  The feature map is written only if
 * feat is given.
 *
 * In:  as ls2_splat_decode; pos [D], neg [n_neg,D] f32; tau.
 * Out: relevancy [levels,H,W] f32; feat [levels,H,W,D] bfloat16 (optional,
 *      16-byte aligned); coef, final_T, last (optional) as ls2_splat_decode.
 * workspace: at least ls2_splat_decode_query_workspace() bytes (the repacked
 *      dictionary, the bfloat16 texts and their norms), 16-byte aligned,
 *      owned by the caller, not shared between concurrent calls.
 * Supported: as ls2_splat_decode, and 1 <= n_neg <= 8.
 */
int ls2_splat_decode_query_workspace(int32_t L, int32_t D, int32_t n_neg, size_t* bytes);
int ls2_splat_decode_query(const ls2_camera* cam, int32_t n, int32_t levels, int32_t K, int32_t L, int32_t D,
                           const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                           const float* conic, const float* opacity, const int32_t* topk_idx,
                           const float* topk_w, const float* dict, const float* pos, int32_t n_neg,
                           const float* neg, float tau, float* relevancy, void* feat, void* coef,
                           float* final_T, int32_t* last, void* workspace, size_t workspace_bytes,
                           hipStream_t stream);

/*
 * ls2_splat_decode_query_noalloc -- ls2_splat_decode_query for callers that
 * cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc).  It takes no workspace and calls
 * no allocating routine: the repacked dictionary and texts go to a scratch
 * array of 160 KiB that the library holds on each GPU it runs on until the
 * process ends.  The caller still passes inputs and outputs, with the same
 * meaning, layout and ownership as ls2_splat_decode_query; the outputs are
 * bit-identical to it.
 *
 * Limit: the scratch must hold ls2_splat_decode_query_workspace(L, D, n_neg)
 * bytes (for example L = 128 with D <= 512, or L = 64 with D <= 1024);
 * larger shapes return LS2_ERR_CAPACITY before any device call.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one
 * GPU (concurrent streams or host threads) race and must be serialised by
 * the caller.  The first call on a device looks up its scratch address
 * (LS2_ERR_DEVICE if that fails).
 */
int ls2_splat_decode_query_noalloc(const ls2_camera* cam, int32_t n, int32_t levels, int32_t K, int32_t L,
                                   int32_t D, const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                                   const float* conic, const float* opacity, const int32_t* topk_idx,
                                   const float* topk_w, const float* dict, const float* pos, int32_t n_neg,
                                   const float* neg, float tau, float* relevancy, void* feat, void* coef,
                                   float* final_T, int32_t* last, hipStream_t stream);

/*
 * ls2_splat_dense -- the dense form of the coefficient splatting: every
 * Gaussian blends all L coefficients of each level (the rendering that
 * Section 3.4 avoids by blending only the K non-zero ones; Table 9 times both).
 * Same lists, alpha rule, culling and outputs as ls2_splat_sparse; weights are
 * dense [n,levels,L].  With the stored pairs scattered into dense weights
 * (repeated indices summed in slot order) the result equals ls2_splat_sparse
 * bit for bit: both blend with one fused multiply-add per coefficient in list
 * order.  Kept as the ablation baseline and as a cross-check.
 * Supported: L in {32, 64}, levels in {1, 2, 3}, levels * L <= 192.
 */
int ls2_splat_dense(const ls2_camera* cam, int32_t n, int32_t levels, int32_t L, const uint32_t* tile_ranges,
                    const uint32_t* ids, const float* mean2d, const float* conic, const float* opacity,
                    const float* weights, float* coef, float* final_T, int32_t* last, hipStream_t stream);

/*
 * ls2_dict_decode -- feature map F = W S (Eq. 7: rendering the sparse
 * coefficients and multiplying by the global codebook S equals rendering
 * the D-dimensional features).  One product shared by all levels.
 *
 * In:  coef [m,L] (m = levels*H*W rows), float32 (coef_dtype LS2_F32) or
 *      bfloat16 (LS2_BF16, only with LS2_BF16 compute); dict [L,D] f32.
 *      coef and feat 16-byte aligned.
 * compute: LS2_F32 (float32 products and accumulation) or LS2_BF16 (both
 *      operands rounded to bfloat16, nearest-even; float32 accumulation on
 *      the matrix cores).
 * Out: feat [m,D], float32 (out_dtype LS2_F32) or bfloat16 (LS2_BF16,
 *      rounded nearest-even from the float32 accumulator).
 * Supported: L in {32, 64, 128}; D in {128, 256, 384, 512, 1024}.
 */
int ls2_dict_decode(int64_t m, int32_t L, int32_t D, const void* coef, int32_t coef_dtype, const float* dict,
                    int32_t compute, int32_t out_dtype, void* feat, hipStream_t stream);

/*
 * ls2_dict_decode_query -- ls2_dict_decode (LS2_BF16 compute, bfloat16
 * feature map) with the relevancy of ls2_query computed in the decode's
 * epilogue, while each 32-row tile of F is still on chip (the decode ->
 * relevancy fusion of Eq. 7 followed by the Section 3.2 score).  The
 * relevancy equals ls2_query on the bfloat16 feature map bit for bit (same
 * matrix-core dot products with the bf16-rounded texts, same norms, same
 * formula), without reading the map back.
 *
 * In:  coef [m,L] float32 or bfloat16 (coef_dtype); dict [L,D] f32;
 *      pos [D]; neg [n_neg,D] f32; tau.
 * Out: feat [m,D] bfloat16, or NULL to skip writing the feature map;
 *      relevancy [m] f32.  coef and feat 16-byte aligned.
 * Supported: L in {32, 64, 128}; D in {128, 256, 384, 512}; 1 <= n_neg <= 8.
 */
int ls2_dict_decode_query(int64_t m, int32_t L, int32_t D, const void* coef, int32_t coef_dtype, const float* dict,
                          void* feat, const float* pos, int32_t n_neg, const float* neg, float tau,
                          float* relevancy, hipStream_t stream);

/*
 * ls2_query -- relevancy of each feature to a text query.
 *
 * Section 3.2 scores relevancy as LERF does: with cosine similarities
 * s_q = cos(F, pos), s_j = cos(F, neg_j) against n_neg canonical negatives,
 *     r = min_j exp(tau s_q) / (exp(tau s_q) + exp(tau s_j))
 *       = sigmoid(tau (s_q - max_j s_j)).
 * Norms are guarded below by 1e-12 (a zero feature scores 0.5).
 *
 * In:  feat [m,D] f32 or bf16 (feat_dtype); pos [D]; neg [n_neg,D] f32.
 * Out: relevancy [m] f32.  Arithmetic is float32.
 * Supported: D a multiple of 64 up to 1024, 1 <= n_neg <= 8.
 */
int ls2_query(int64_t m, int32_t D, const void* feat, int32_t feat_dtype, const float* pos,
              int32_t n_neg, const float* neg, float tau, float* relevancy, hipStream_t stream);

/*
 * ls2_query_coef -- the relevancy of ls2_query computed from the coefficient
 * map, without forming the feature map.  Eq. 7 gives F = W S, so
 * F . e = W . (S e) and |F|^2 = W^T (S S^T) W; the cosine similarities and
 * r = sigmoid(tau (s_q - max_j s_j)) follow exactly (up to float32 rounding)
 * from the L coefficients of each pixel.
 *
 * In:  coef [m,L] f32 (m = levels*H*W rows of ls2_splat_sparse's output),
 *      dict [L,D], pos [D], neg [n_neg,D] f32.
 * Out: relevancy [m] f32.
 * workspace: at least ls2_query_coef_workspace() bytes (projected embeddings
 *      and the L x L Gram matrix, rebuilt by every call), 16-byte aligned.
 * Supported: L in {32, 64, 128}, 1 <= n_neg <= 8, any D >= 1.
 */
int ls2_query_coef_workspace(int32_t L, int32_t n_neg, size_t* bytes);
int ls2_query_coef(int64_t m, int32_t L, int32_t D, const float* coef, const float* dict, const float* pos,
                   int32_t n_neg, const float* neg, float tau, float* relevancy, void* workspace,
                   size_t workspace_bytes, hipStream_t stream);

/*
 * ls2_postprocess -- relevancy post-processing (Section 3.2: a mean filter on
 * each level's relevancy map, then one semantic level is selected; the
 * evaluation appendix: the localization point is the argmax of the smoothed
 * map, the mask is the normalised smoothed map above a threshold, the blend
 * 0.5 (M + Avg(M)) and selection by the mean relevancy inside the mask are
 * the variant used for some datasets).
 *
 * In:  relevancy [levels,H,W] f32; kernel: odd box size (the mean runs over
 *      the kernel x kernel window clipped to the image); smooth_mode
 *      LS2_SMOOTH_AVG (Avg(M)) or LS2_SMOOTH_HALF (0.5 (M + Avg(M)));
 *      select_mode LS2_SELECT_MAX (level with the largest smoothed maximum)
 *      or LS2_SELECT_MASK_MEAN (level with the largest mean smoothed value
 *      inside its own mask; an empty mask counts as -inf); threshold on the
 *      normalised map (s - min) / (max - min) (0 when max == min), mask =
 *      normalised > threshold.  Ties go to the lowest level / first pixel in
 *      row-major order.
 * Out: smoothed [levels,H,W] f32; mask [H,W] u8 (0/1) of the selected level;
 *      result [4] int32 = selected level, x, y, y * W + x of the argmax;
 *      level_stats [levels,4] f32 (optional) = max, min, mask mean, mask count.
 * workspace: at least ls2_postprocess_workspace() bytes, 256-byte aligned.
 * Every reduction runs in a fixed order (deterministic).
 * Supported: levels <= 8, H * W < 2^31.
 */
enum { LS2_SMOOTH_AVG = 0, LS2_SMOOTH_HALF = 1 };
enum { LS2_SELECT_MAX = 0, LS2_SELECT_MASK_MEAN = 1 };
int ls2_postprocess_workspace(int32_t levels, int32_t H, int32_t W, size_t* bytes);
int ls2_postprocess(int32_t levels, int32_t H, int32_t W, const float* relevancy, int32_t kernel,
                    int32_t smooth_mode, int32_t select_mode, float threshold, float* smoothed,
                    uint8_t* mask, int32_t* result, float* level_stats, void* workspace,
                    size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Backward pass.  The sparse coefficients and the codebook are learned
 * jointly (Section 3.3); these entry points give the gradients of every
 * forward stage, in reverse order: feature loss -> decode -> splat ->
 * project (or query -> decode -> ...).  All arithmetic is float32.  Gradient
 * outputs are OVERWRITTEN (the library clears what it accumulates into).
 * Gradients are taken with respect to the activated values the forward
 * consumes (scales > 0, opacity in (0,1), normalised-in-kernel quaternions).
 * ---------------------------------------------------------------------- */

/*
 * ls2_feature_loss -- training objective between the rendered feature map
 * and a target feature map Y (the 2D feature maps the field is fitted to,
 * Section 4.1; the paper does not print the loss, this library uses
 *     loss = mean_{v,d} |F - Y| + mean_v (1 - cos(F(v), Y(v))),
 * norms guarded below by 1e-12, sign(0) = 0).
 *
 * In:  feat [m,D] f32, target [m,D] f32.
 * Out: loss (device, one double); d_feat [m,D] f32 = dloss/dF (optional:
 *      NULL computes the loss only).
 * workspace: at least ls2_feature_loss_workspace() bytes, 8-byte aligned.
 * The loss is reduced in a fixed order (deterministic).
 * Supported: D a multiple of 64 up to 1024; m >= 1.
 */
int ls2_feature_loss_workspace(int64_t m, size_t* bytes);
int ls2_feature_loss(int64_t m, int32_t D, const float* feat, const float* target, double* loss,
                     float* d_feat, void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * ls2_decode_feature_loss -- ls2_dict_decode (LS2_F32 compute, float32
 * output) fused with ls2_feature_loss: F = W S (Eq. 7) is formed tile by tile
 * on the matrix cores and consumed in place, so the feature map itself need
 * not travel through HBM.  F, d_feat and the loss equal those of decoding and
 * then calling ls2_feature_loss up to float32 rounding (same formulas, same
 * per-row reduction order; the loss is summed in a different fixed order).
 *
 * In:  coef [m,L], dict [L,D], target [m,D], all f32.
 * Out: loss (device, one double); d_feat [m,D]; feat [m,D] f32 (optional).
 * workspace: at least ls2_decode_feature_loss_workspace() bytes, 8-byte
 *      aligned.
 * Supported: L in {32, 64}; D in {128, 256, 384, 512}; m >= 1.
 */
int ls2_decode_feature_loss_workspace(int64_t m, int32_t D, size_t* bytes);
int ls2_decode_feature_loss(int64_t m, int32_t L, int32_t D, const float* coef, const float* dict,
                            const float* target, double* loss, float* d_feat, float* feat, void* workspace,
                            size_t workspace_bytes, hipStream_t stream);

/*
 * ls2_decode_loss_backward -- ls2_decode_feature_loss and
 * ls2_dict_decode_backward in one pass (float32): F = W S (Eq. 7), the loss
 * of ls2_feature_loss against the target (Section 4.1), dL/dF, and both
 * gradients of the decode, d_coef = dL/dF S^T and d_dict = coef^T dL/dF,
 * with dL/dF kept on the chip (never written to memory).  Each product takes
 * the same operands in the same order as the two-call chain, so d_coef and
 * d_dict equal that chain's bit for bit; the loss, whose partial sums follow
 * the workgroups, does too when ls2_decode_feature_loss launches the same
 * number of them (one per compute unit at D = 512) and is otherwise a few
 * float32 roundings of its compensated total away.
 *
 * In:  coef [m,L], dict [L,D], target [m,D], all f32, 16-byte aligned.
 * Out: loss (device, one double); d_coef [m,L]; d_dict [L,D] (both
 *      overwritten).
 * workspace: at least ls2_decode_loss_backward_workspace() bytes, 16-byte
 *      aligned (dS partial sums and the loss partials).
 * Supported: L in {32, 64}; D in {128, 256, 384, 512}; m >= 1.
 */
int ls2_decode_loss_backward_workspace(int64_t m, int32_t L, int32_t D, size_t* bytes);
int ls2_decode_loss_backward(int64_t m, int32_t L, int32_t D, const float* coef, const float* dict,
                             const float* target, double* loss, float* d_coef, float* d_dict, void* workspace,
                             size_t workspace_bytes, hipStream_t stream);

/*
 * ls2_query_backward -- d_feat = d_rel * dr/dF for the relevancy of
 * ls2_query (Section 3.2, LERF form).  The minimum over negatives selects the
 * first negative of largest similarity; its (sub)gradient is used.
 *
 * In:  feat [m,D] f32 or bf16 (feat_dtype), pos [D], neg [n_neg,D], tau,
 *      d_rel [m] f32.
 * Out: d_feat [m,D] f32.
 * Supported: D a multiple of 64 up to 1024, 1 <= n_neg <= 8.
 */
int ls2_query_backward(int64_t m, int32_t D, const void* feat, int32_t feat_dtype, const float* pos,
                       int32_t n_neg, const float* neg, float tau, const float* d_rel, float* d_feat,
                       hipStream_t stream);

/*
 * ls2_dict_decode_backward -- gradients of F = W S (Eq. 7):
 *     d_coef = d_feat S^T  [m,L],     d_dict = coef^T d_feat  [L,D]
 * (all levels share S, so their rows are summed into one d_dict).
 *
 * In:  coef [m,L], dict [L,D], d_feat [m,D], all f32.
 * compute: LS2_F32 (float32 matrix-core products; the only form built).
 * Out: d_coef [m,L] (optional), d_dict [L,D] (optional; at least one of the
 *      two must be requested).  d_dict is reduced in a fixed order
 *      (deterministic).
 * workspace: at least ls2_dict_decode_backward_workspace() bytes when d_dict
 *      is requested (partial sums over pixel ranges), 16-byte aligned.
 * coef, dict, d_feat and d_coef must be 16-byte aligned (LS2_ERR_ARG
 *      otherwise).  With L <= 64, D <= 512 and both outputs requested, one
 *      kernel forms both products from a single read of d_feat.
 * Supported: L in {32, 64, 128}; D in {128, 256, 384, 512, 1024}.
 */
int ls2_dict_decode_backward_workspace(int64_t m, int32_t L, int32_t D, size_t* bytes);
int ls2_dict_decode_backward(int64_t m, int32_t L, int32_t D, const float* coef, const float* dict,
                             int32_t compute, const float* d_feat, float* d_coef, float* d_dict,
                             void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * ls2_splat_sparse_backward -- gradients of ls2_splat_sparse (Algorithm 1,
 * Eq. 3) from d_coef = dL/dcoef.  For one pixel with contributors i (front
 * to back), e_i = alpha_i T_i and c_i = sum_{l,k} d_coef_l[idx_ilk] w_ilk:
 *     d topk_w_ilk += d_coef_l[idx_ilk] e_i,
 *     dL/dalpha_i   = T_i c_i - (sum_{m>i} c_m e_m) / (1 - alpha_i),
 * then through alpha = o exp(-0.5 d^T conic d) (no gradient where alpha is
 * clamped at 0.99) to opacity, mean2d and conic.  The pixel's contributors
 * and T_i are recovered from the forward's final_T and last, with alpha
 * evaluated by the same instructions as the forward.
 *
 * In:  the forward's inputs (tile_ranges .. topk_w) and outputs final_T [H,W]
 *      and last [H,W] (both required); d_coef [levels,H,W,L].
 * Out: d_mean2d [n,2], d_conic [n,3] (A, B, C as in ls2_project),
 *      d_opacity [n], d_topk_w [n,levels,K].  Accumulated with float atomics:
 *      the summation order (and the last bits) may vary between runs.
 * Supported: as ls2_splat_sparse.
 */
int ls2_splat_sparse_backward(const ls2_camera* cam, int32_t n, int32_t levels, int32_t K, int32_t L,
                              const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                              const float* conic, const float* opacity, const int32_t* topk_idx,
                              const float* topk_w, const float* final_T, const int32_t* last,
                              const float* d_coef, float* d_mean2d, float* d_conic, float* d_opacity,
                              float* d_topk_w, hipStream_t stream);

/*
 * ls2_sparse_codes -- the sparse coefficient parametrisation (Section 3.3): a
 * Gaussian's L-dimensional parameter z is normalised by a softmax, its K
 * largest values are kept and renormalised to sum 1, which equals the softmax
 * of the K kept logits.  Indices come in descending order of the logit, ties
 * to the smaller index.  ls2_sparse_codes_backward gives dL/dz from dL/dw with
 * the selection held fixed: dz_j = w_j (dw_j - sum_k w_k dw_k) for kept j, 0
 * otherwise (d_logits is overwritten).
 *
 * In:  logits [rows,L] f32 (rows = n * levels).
 * Out: topk_idx [rows,K] int32, topk_w [rows,K] f32 (the layout
 *      ls2_splat_sparse consumes).
 * Supported: L a multiple of 4 up to 1024, 1 <= K <= 8.
 */
int ls2_sparse_codes(int64_t rows, int32_t L, int32_t K, const float* logits, int32_t* topk_idx, float* topk_w,
                     hipStream_t stream);
int ls2_sparse_codes_backward(int64_t rows, int32_t L, int32_t K, const int32_t* topk_idx, const float* topk_w,
                              const float* d_topk_w, float* d_logits, hipStream_t stream);

/*
 * ls2_project_backward -- gradients of ls2_project (Section 3.1, Eqs. 1-2,
 * EWA projection as in ls2_project) from d_mean2d [n,2] and d_conic [n,3]
 * to d_means [n,3], d_scales [n,3] and d_quats [n,4] (through the
 * normalisation q / |q|).  Depth and radius carry no gradient.  Culled
 * Gaussians (radius [n] from the forward is 0) get zeros.
 */
int ls2_project_backward(const ls2_camera* cam, int32_t n, const float* means, const float* scales,
                         const float* quats, const int32_t* radius, const float* d_mean2d,
                         const float* d_conic, float* d_means, float* d_scales, float* d_quats,
                         hipStream_t stream);

/*
 * ls2_accumulate -- dst[i] += src[i] for i < n (f32): sums the gradients of
 * the views of one training step (the batch of camera views is one step).
 * Both pointers 16-byte aligned.
 */
int ls2_accumulate(int64_t n, const float* src, float* dst, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LS2_H */
