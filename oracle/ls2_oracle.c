/*
 * ls2_oracle.c -- plain, slow, obviously-correct FP64 CPU reference for the
 * sparse-coefficient Gaussian splatting path of LangSplatV2 (arXiv 2507.07136).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header, table or constant generator with
 * the HIP library.
 *
 * What is computed, and where the paper defines it:
 *   - Gaussian kernel and covariance Sigma = R S S^T R^T: Section 3.1, Eqs. 1-2.
 *   - Projection to the image plane: Section 3.1 cites EWA splatting
 *     (Zwicker et al. 2001) and 3D Gaussian Splatting without restating the
 *     formula; this file uses the local-affine Jacobian of the perspective map
 *     at the mean, a 0.3 px^2 low-pass dilation and a 3-sigma radius (the
 *     readings are listed in the design notes).
 *   - Front-to-back alpha compositing over the depth-ordered Gaussians of a
 *     tile: Section 3.1, Eq. 3, with alpha_i = o_i G2D_i(v).
 *   - Sparse coefficient field and the blend of only the K non-zero
 *     coefficients: Section 3.3 Eq. 5, Section 3.4 and Appendix A (Algorithm 1):
 *     W[j] += w_ij * alpha_i * prod_{m<i}(1 - alpha_m).
 *   - Dense D-dim rendering of f_i = w_i S (Eq. 6) for the linearity identity
 *     of Eq. 7: sum_i e_i w_i S = (sum_i e_i w_i) S.
 *   - Decode as one matrix product with the global codebook: Section 3.3, Eq. 7.
 *   - Relevancy: Section 3.2 says it follows LERF; LERF's score is the minimum
 *     over canonical negatives of the pairwise softmax between the query and
 *     the negative cosine similarities.
 *
 * Parity status per function is stated in the header comment of each.
 * All arithmetic is double precision except where a floating-point value
 * decides an integer (tile rectangle, depth order): there the float32 value is
 * used, as the GPU kernel does.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TILE 16

/* thresholds of the compositing rule, as float32 constants promoted to double */
static const double ALPHA_MAX = (double)0.99f;
static const double ALPHA_MIN = (double)(1.0f / 255.0f);
static const double T_MIN = (double)1e-4f;
static const double DILATION = (double)0.3f;

/* camera array: [W, H, fx, fy, cx, cy, R00..R22, t0..t2, znear] */
typedef struct {
    int W, H, tx, ty;
    double fx, fy, cx, cy;
    double R[9], t[3];
    double znear;
} cam_t;

static cam_t cam_from(const double* c) {
    cam_t k;
    k.W = (int)c[0];
    k.H = (int)c[1];
    k.fx = c[2]; k.fy = c[3]; k.cx = c[4]; k.cy = c[5];
    for (int i = 0; i < 9; ++i) k.R[i] = c[6 + i];
    for (int i = 0; i < 3; ++i) k.t[i] = c[15 + i];
    k.znear = c[18];
    k.tx = (k.W + ORC_TILE - 1) / ORC_TILE;
    k.ty = (k.H + ORC_TILE - 1) / ORC_TILE;
    return k;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Eq. 2: rotation matrix from a quaternion (w, x, y, z), normalised.  */
/* ------------------------------------------------------------------ */
static void quat_to_rot(const double q_in[4], double R[9]) {
    double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
    double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void matmul3(const double A[9], const double B[9], double C[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

static void transpose3(const double A[9], double B[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[3 * j + i] = A[3 * i + j];
}

/* Tile rectangle of a projected Gaussian, evaluated in float32 exactly as the
 * kernel does: tiles [floor((u - r)/16), floor((u + r)/16)] clipped to the
 * grid.  Returns 0 if empty. */
static int rect_f32(float u, float v, int r, int tx, int ty, int* x0, int* y0, int* x1, int* y1) {
    float rf = (float)r;
    float lox = floorf((u - rf) * 0.0625f), hix = floorf((u + rf) * 0.0625f);
    float loy = floorf((v - rf) * 0.0625f), hiy = floorf((v + rf) * 0.0625f);
    if (lox < 0.0f) lox = 0.0f;
    if (loy < 0.0f) loy = 0.0f;
    if (hix > (float)(tx - 1)) hix = (float)(tx - 1);
    if (hiy > (float)(ty - 1)) hiy = (float)(ty - 1);
    if (!(lox <= hix) || !(loy <= hiy)) return 0;
    *x0 = (int)lox; *x1 = (int)hix; *y0 = (int)loy; *y1 = (int)hiy;
    return 1;
}

/* ------------------------------------------------------------------ */
/* Projection (Eqs. 1-2 and the EWA reading).                          */
/* Outputs per Gaussian i:                                             */
/*   mean2d[2i..]  pixel-space mean (u, v)                             */
/*   cov2d[3i..]   dilated screen covariance (a, b, c)                 */
/*   conic[3i..]   its inverse (A, B, C) = (c, -b, a) / det            */
/*   depth[i]      camera-space z                                      */
/*   extent[i]     3 * sqrt(lambda_max) (radius before ceil)           */
/*   radius[i]     ceil(extent), 0 if culled                           */
/*   rect[4i..]    x0, y0, x1, y1 tile rectangle (inclusive)           */
/*   touched[i]    number of tiles in the rectangle                    */
/* Culled (radius 0, zeros elsewhere): z <= znear, non-finite values,  */
/* det <= 0, or an empty tile rectangle.                               */
/* Parity pinned by closed forms (on-axis / axis-aligned Gaussians),   */
/* the image-edge pixel of the 60-degree field of view and a numerical */
/* Jacobian of the perspective map.                                    */
/* ------------------------------------------------------------------ */
static void project_one(const cam_t* cam, const double mu[3], const double s3[3], const double q[4], int i,
                        double* mean2d, double* cov2d, double* conic, double* depth, double* extent,
                        int32_t* radius, int32_t* rect, int32_t* touched) {
    mean2d[2 * i] = mean2d[2 * i + 1] = 0;
    cov2d[3 * i] = cov2d[3 * i + 1] = cov2d[3 * i + 2] = 0;
    conic[3 * i] = conic[3 * i + 1] = conic[3 * i + 2] = 0;
    depth[i] = 0; extent[i] = 0; radius[i] = 0; touched[i] = 0;
    rect[4 * i] = rect[4 * i + 1] = rect[4 * i + 2] = rect[4 * i + 3] = 0;

    double p[3];
    for (int r = 0; r < 3; ++r)
        p[r] = cam->R[3 * r] * mu[0] + cam->R[3 * r + 1] * mu[1] + cam->R[3 * r + 2] * mu[2] + cam->t[r];
    double x = p[0], y = p[1], z = p[2];
    if (!(z > cam->znear) || !isfinite(x) || !isfinite(y)) return;

    /* Eq. 2: Sigma = R S S^T R^T */
    double Rq[9];
    quat_to_rot(q, Rq);
    double M[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * s3[c];
    double Mt[9], Sig[9];
    transpose3(M, Mt);
    matmul3(M, Mt, Sig);

    /* world -> camera covariance */
    double Rt[9], tmp[9], Sc[9];
    transpose3(cam->R, Rt);
    matmul3(cam->R, Sig, tmp);
    matmul3(tmp, Rt, Sc);

    /* EWA: local affine approximation of the perspective map at the mean */
    double J[6] = {cam->fx / z, 0.0, -cam->fx * x / (z * z),
                   0.0, cam->fy / z, -cam->fy * y / (z * z)};
    double JS[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += J[3 * r + k] * Sc[3 * k + c];
            JS[3 * r + c] = acc;
        }
    double cv[4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += JS[3 * r + k] * J[3 * c + k];
            cv[2 * r + c] = acc;
        }
    double a = cv[0] + DILATION, b = cv[1], c = cv[3] + DILATION;
    double det = a * c - b * b;
    if (!(det > 0) || !isfinite(det)) return;

    double mid = 0.5 * (a + c);
    double disc = mid * mid - det;
    double lam = mid + sqrt(disc > 0 ? disc : 0);
    double ext = 3.0 * sqrt(lam);
    if (!isfinite(ext) || ext > 1e7) return;
    int r = (int)ceil(ext);

    double u = cam->fx * x / z + cam->cx;
    double v = cam->fy * y / z + cam->cy;
    int x0, y0, x1, y1;
    if (!rect_f32((float)u, (float)v, r, cam->tx, cam->ty, &x0, &y0, &x1, &y1)) return;

    mean2d[2 * i] = u; mean2d[2 * i + 1] = v;
    cov2d[3 * i] = a; cov2d[3 * i + 1] = b; cov2d[3 * i + 2] = c;
    conic[3 * i] = c / det; conic[3 * i + 1] = -b / det; conic[3 * i + 2] = a / det;
    depth[i] = z; extent[i] = ext; radius[i] = r;
    rect[4 * i] = x0; rect[4 * i + 1] = y0; rect[4 * i + 2] = x1; rect[4 * i + 3] = y1;
    touched[i] = (x1 - x0 + 1) * (y1 - y0 + 1);
}

void orc_project(const double* cam_arr, int n, const float* means, const float* scales,
                 const float* quats, double* mean2d, double* cov2d, double* conic,
                 double* depth, double* extent, int32_t* radius, int32_t* rect, int32_t* touched) {
    cam_t cam = cam_from(cam_arr);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double mu[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
        double s3[3] = {scales[3 * i], scales[3 * i + 1], scales[3 * i + 2]};
        double q[4] = {quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]};
        project_one(&cam, mu, s3, q, i, mean2d, cov2d, conic, depth, extent, radius, rect, touched);
    }
}

/* Same projection on float64 inputs (finite-difference checks). */
void orc_project_f64(const double* cam_arr, int n, const double* means, const double* scales,
                     const double* quats, double* mean2d, double* cov2d, double* conic,
                     double* depth, double* extent, int32_t* radius, int32_t* rect, int32_t* touched) {
    cam_t cam = cam_from(cam_arr);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        project_one(&cam, means + 3 * i, scales + 3 * i, quats + 4 * i, i, mean2d, cov2d, conic, depth, extent,
                    radius, rect, touched);
}

/* ------------------------------------------------------------------ */
/* Tile binning and depth order (Eq. 3 composites each tile's          */
/* Gaussians front to back).  One (tile, Gaussian) pair per tile of the */
/* rectangle; pairs ordered by tile, then float32 depth, then id.       */
/* Outputs keys = tile << 32 | float32 bits of depth, ids, and per-tile */
/* [start, end) ranges.  Returns 0, or -2 when cap < P (num_pairs = P). */
/* Parity pinned against numpy's lexsort of the same triples and a    */
/* brute-force per-pixel renderer.                                     */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t tile, dbits, id; } pair_t;

static int pair_cmp(const void* a, const void* b) {
    const pair_t* p = (const pair_t*)a;
    const pair_t* q = (const pair_t*)b;
    if (p->tile != q->tile) return p->tile < q->tile ? -1 : 1;
    if (p->dbits != q->dbits) return p->dbits < q->dbits ? -1 : 1;
    if (p->id != q->id) return p->id < q->id ? -1 : 1;
    return 0;
}

static uint32_t f32_bits(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

int orc_tile_lists(const double* cam_arr, int n, const float* mean2d, const int32_t* radius,
                   const float* depth, int64_t cap, uint64_t* keys, uint32_t* ids,
                   uint32_t* ranges, int64_t* num_pairs) {
    cam_t cam = cam_from(cam_arr);
    int64_t P = 0;
    for (int i = 0; i < n; ++i) {
        int x0, y0, x1, y1;
        if (radius[i] <= 0) continue;
        if (!rect_f32(mean2d[2 * i], mean2d[2 * i + 1], radius[i], cam.tx, cam.ty, &x0, &y0, &x1, &y1))
            continue;
        P += (int64_t)(x1 - x0 + 1) * (y1 - y0 + 1);
    }
    *num_pairs = P;
    int ntiles = cam.tx * cam.ty;
    if (P > cap) return -2;
    pair_t* pairs = (pair_t*)malloc(sizeof(pair_t) * (size_t)(P > 0 ? P : 1));
    int64_t k = 0;
    for (int i = 0; i < n; ++i) {
        int x0, y0, x1, y1;
        if (radius[i] <= 0) continue;
        if (!rect_f32(mean2d[2 * i], mean2d[2 * i + 1], radius[i], cam.tx, cam.ty, &x0, &y0, &x1, &y1))
            continue;
        for (int ty = y0; ty <= y1; ++ty)
            for (int tx = x0; tx <= x1; ++tx) {
                pairs[k].tile = (uint32_t)(ty * cam.tx + tx);
                pairs[k].dbits = f32_bits(depth[i]);
                pairs[k].id = (uint32_t)i;
                ++k;
            }
    }
    qsort(pairs, (size_t)P, sizeof(pair_t), pair_cmp);
    for (int64_t j = 0; j < P; ++j) {
        if (keys) keys[j] = ((uint64_t)pairs[j].tile << 32) | pairs[j].dbits;
        ids[j] = pairs[j].id;
    }
    /* ranges: [start, end) of each tile; start = number of pairs in the tiles
     * before it (so an empty tile has start = end = that count) */
    for (int t = 0; t < ntiles; ++t) ranges[2 * t + 1] = 0;
    for (int64_t j = 0; j < P; ++j) ranges[2 * pairs[j].tile + 1] += 1;
    uint32_t acc = 0;
    for (int t = 0; t < ntiles; ++t) {
        uint32_t c = ranges[2 * t + 1];
        ranges[2 * t] = acc;
        acc += c;
        ranges[2 * t + 1] = acc;
    }
    free(pairs);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Per-pixel front-to-back walk (Eq. 3).  For the ordered list of the  */
/* pixel's tile, compute the blending weights e_i = alpha_i prod_{j<i}  */
/* (1 - alpha_j) of Eq. 7 for the Gaussians that contribute.           */
/*   alpha = min(0.99, o * exp(-0.5 d^T conic d)); skip alpha < 1/255;  */
/*   stop (without blending) once T (1 - alpha) < 1e-4.                 */
/* Writes contributing list positions and their e_i; returns count.    */
/* *T_out = final transmittance, *last_out = 1 + position of the last   */
/* contributing entry relative to the tile start (0 if none),          */
/* *margin = smallest relative distance of an alpha decision (clamp,    */
/* skip) to its threshold, *margin_T = the same for the stop decision   */
/* (transmittance against 1e-4) divided by the transmittance's condition */
/* number c = 1 + sum (alpha_j / (1 - alpha_j) + 0.02) over the Gaussians */
/* blended so far and the current one: a relative perturbation e of     */
/* every alpha moves T by about e (c - 1) relatively (the 0.02 per term */
/* covers the rounding of each product).                                */
/* ------------------------------------------------------------------ */
static int walk_pixel(double pxc, double pyc, uint32_t start, uint32_t end, const uint32_t* ids,
                      const double* mean2d, const double* conic, const double* opacity,
                      int32_t* pos_out, double* e_out, double* T_before_out, double* alpha_out,
                      double* T_out, int32_t* last_out, double* margin, double* margin_T) {
    double T = 1.0;
    int cnt = 0;
    int32_t last = 0;
    double mg = INFINITY, mgT = INFINITY;
    double cond = 1.0;
    for (uint32_t pos = start; pos < end; ++pos) {
        uint32_t i = ids[pos];
        double dx = mean2d[2 * i] - pxc;
        double dy = mean2d[2 * i + 1] - pyc;
        double A = conic[3 * i], B = conic[3 * i + 1], C = conic[3 * i + 2];
        double power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy;
        if (power > 0) continue;
        double g = opacity[i] * exp(power);
        double m1 = fabs(g - ALPHA_MAX) / ALPHA_MAX;
        if (m1 < mg) mg = m1;
        double alpha = g < ALPHA_MAX ? g : ALPHA_MAX;
        double m2 = fabs(alpha - ALPHA_MIN) / ALPHA_MIN;
        if (m2 < mg) mg = m2;
        if (alpha < ALPHA_MIN) continue;
        double testT = T * (1.0 - alpha);
        double m3 = fabs(testT - T_MIN) / T_MIN / (cond + alpha / (1.0 - alpha) + 0.02);
        if (m3 < mgT) mgT = m3;
        if (testT < T_MIN) break;
        cond += alpha / (1.0 - alpha) + 0.02;
        if (pos_out) pos_out[cnt] = (int32_t)(pos - start);
        if (e_out) e_out[cnt] = alpha * T;
        if (T_before_out) T_before_out[cnt] = T;
        if (alpha_out) alpha_out[cnt] = alpha;
        ++cnt;
        T = testT;
        last = (int32_t)(pos - start + 1);
    }
    *T_out = T;
    *last_out = last;
    *margin = mg;
    if (margin_T) *margin_T = mgT;
    return cnt;
}

/* ------------------------------------------------------------------ */
/* The same walk with chosen alternatives at its near decisions.       */
/* A float32 evaluation of a decision whose float64 value lies within   */
/* rounding of its threshold may legitimately come out the other way,  */
/* so a parity check compares the kernel with every outcome the walk    */
/* can take when such decisions are flipped.  Three decisions of Eq. 3  */
/* are discontinuous in the inputs and can flip:                       */
/*   - the skip of a non-positive-definite exponent (power > 0), near   */
/*     when |power| <= thr * (|A| dx^2 / 2 + |B dx dy| + |C| dy^2 / 2);   */
/*   - the skip of alpha < 1/255, near when |alpha - 1/255| <= thr/255;   */
/*   - the stop once T (1 - alpha) < 1e-4, near when its condition-     */
/*     scaled margin (as in walk_pixel) is below thr.                   */
/* The clamp at 0.99 is continuous in the inputs and is not flipped.    */
/* Bit b of `flips` takes the b-th near decision met along this walk    */
/* the other way (bits past the last near decision are ignored);        */
/* *n_near = the number of near decisions met.  With flips = 0 the walk */
/* is walk_pixel's.                                                     */
/* ------------------------------------------------------------------ */
static int walk_pixel_alt(double pxc, double pyc, uint32_t start, uint32_t end, const uint32_t* ids,
                          const double* mean2d, const double* conic, const double* opacity, double thr,
                          uint32_t flips, int32_t* pos_out, double* e_out, double* T_out, int32_t* last_out,
                          int* n_near) {
    double T = 1.0;
    int cnt = 0, near = 0;
    int32_t last = 0;
    double cond = 1.0;
    for (uint32_t pos = start; pos < end; ++pos) {
        uint32_t i = ids[pos];
        double dx = mean2d[2 * i] - pxc;
        double dy = mean2d[2 * i + 1] - pyc;
        double A = conic[3 * i], B = conic[3 * i + 1], C = conic[3 * i + 2];
        double power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy;
        int skip = power > 0;
        double scale = 0.5 * fabs(A) * dx * dx + fabs(B * dx * dy) + 0.5 * fabs(C) * dy * dy;
        if (fabs(power) <= thr * scale) {
            if ((flips >> near) & 1u) skip = !skip;
            ++near;
        }
        if (skip) continue;
        double g = opacity[i] * exp(power);
        double alpha = g < ALPHA_MAX ? g : ALPHA_MAX;
        skip = alpha < ALPHA_MIN;
        if (fabs(alpha - ALPHA_MIN) <= thr * ALPHA_MIN) {
            if ((flips >> near) & 1u) skip = !skip;
            ++near;
        }
        if (skip) continue;
        double testT = T * (1.0 - alpha);
        int stop = testT < T_MIN;
        if (fabs(testT - T_MIN) / T_MIN / (cond + alpha / (1.0 - alpha) + 0.02) < thr) {
            if ((flips >> near) & 1u) stop = !stop;
            ++near;
        }
        if (stop) break;
        cond += alpha / (1.0 - alpha) + 0.02;
        if (pos_out) pos_out[cnt] = (int32_t)(pos - start);
        if (e_out) e_out[cnt] = alpha * T;
        ++cnt;
        T = testT;
        last = (int32_t)(pos - start + 1);
    }
    *T_out = T;
    *last_out = last;
    *n_near = near;
    return cnt;
}

static uint32_t max_range(const uint32_t* ranges, int ntiles) {
    uint32_t m = 0;
    for (int t = 0; t < ntiles; ++t) {
        uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
        if (len > m) m = len;
    }
    return m;
}

/* ------------------------------------------------------------------ */
/* Sparse coefficient splatting (Section 3.4, Algorithm 1): for every   */
/* level l and pixel v, W_l(v)[j] = sum_i e_i(v) w_{i,l,j}, blending    */
/* only the K stored (index, coefficient) pairs of each Gaussian.      */
/* coef: [levels, H, W, L]; final_T, margin: [H, W]; last: [H, W].      */
/* Parity pinned by closed forms (one and two Gaussians, the T stop    */
/* rule), invariants (T in [1e-4, 1] non-increasing, sum W + T = 1),    */
/* the dense-L and dense-D (Eq. 6/7) renderers and a brute-force       */
/* per-pixel binning.                                                  */
/* ------------------------------------------------------------------ */
void orc_composite(const double* cam_arr, int levels, int K, int L, const uint32_t* ranges,
                   const uint32_t* ids, const double* mean2d, const double* conic,
                   const double* opacity, const int32_t* topk_idx, const double* topk_w,
                   double* coef, double* final_T, int32_t* last, double* margin, double* margin_T) {
    cam_t cam = cam_from(cam_arr);
    int ntiles = cam.tx * cam.ty;
    size_t HW = (size_t)cam.W * cam.H;
    memset(coef, 0, sizeof(double) * (size_t)levels * HW * L);
    uint32_t maxlen = max_range(ranges, ntiles);
    #pragma omp parallel
    {
        int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (maxlen + 1));
        double* e = (double*)malloc(sizeof(double) * (maxlen + 1));
        #pragma omp for schedule(dynamic, 1)
        for (int t = 0; t < ntiles; ++t) {
            int tx = t % cam.tx, ty = t / cam.tx;
            for (int py = ty * ORC_TILE; py < (ty + 1) * ORC_TILE && py < cam.H; ++py)
                for (int px = tx * ORC_TILE; px < (tx + 1) * ORC_TILE && px < cam.W; ++px) {
                    size_t pix = (size_t)py * cam.W + px;
                    double T;
                    int32_t lst;
                    double mg, mgT;
                    int cnt = walk_pixel(px + 0.5, py + 0.5, ranges[2 * t], ranges[2 * t + 1], ids,
                                         mean2d, conic, opacity, pos, e, NULL, NULL, &T, &lst, &mg, &mgT);
                    for (int c = 0; c < cnt; ++c) {
                        uint32_t i = ids[ranges[2 * t] + pos[c]];
                        for (int lv = 0; lv < levels; ++lv) {
                            double* W = coef + ((size_t)lv * HW + pix) * L;
                            for (int k = 0; k < K; ++k) {
                                size_t o = ((size_t)i * levels + lv) * K + k;
                                W[topk_idx[o]] += topk_w[o] * e[c];
                            }
                        }
                    }
                    final_T[pix] = T;
                    last[pix] = lst;
                    margin[pix] = mg;
                    margin_T[pix] = mgT;
                }
        }
        free(pos);
        free(e);
    }
}

/* Dense renderer (Eqs. 4 and 6): out(v) = sum_i e_i(v) feat_i for a dense  */
/* per-Gaussian vector of C channels.  With feat_i = w_i S it is the   */
/* D-dimensional rendering of Eq. 6; with feat_i = the dense L-vector w_i */
/* it is the unsparsified coefficient rendering.  out: [H, W, C].       */
void orc_composite_dense(const double* cam_arr, int C, const uint32_t* ranges, const uint32_t* ids,
                         const double* mean2d, const double* conic, const double* opacity,
                         const double* feat, double* out) {
    cam_t cam = cam_from(cam_arr);
    int ntiles = cam.tx * cam.ty;
    memset(out, 0, sizeof(double) * (size_t)cam.W * cam.H * C);
    uint32_t maxlen = max_range(ranges, ntiles);
    #pragma omp parallel
    {
        int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (maxlen + 1));
        double* e = (double*)malloc(sizeof(double) * (maxlen + 1));
        #pragma omp for schedule(dynamic, 1)
        for (int t = 0; t < ntiles; ++t) {
            int tx = t % cam.tx, ty = t / cam.tx;
            for (int py = ty * ORC_TILE; py < (ty + 1) * ORC_TILE && py < cam.H; ++py)
                for (int px = tx * ORC_TILE; px < (tx + 1) * ORC_TILE && px < cam.W; ++px) {
                    double T, mg;
                    int32_t lst;
                    int cnt = walk_pixel(px + 0.5, py + 0.5, ranges[2 * t], ranges[2 * t + 1], ids,
                                         mean2d, conic, opacity, pos, e, NULL, NULL, &T, &lst, &mg, NULL);
                    double* o = out + ((size_t)py * cam.W + px) * C;
                    for (int c = 0; c < cnt; ++c) {
                        const double* f = feat + (size_t)ids[ranges[2 * t] + pos[c]] * C;
                        for (int ch = 0; ch < C; ++ch) o[ch] += e[c] * f[ch];
                    }
                }
        }
        free(pos);
        free(e);
    }
}

/* Composite only the listed pixels (flat indices py * W + px), for     */
/* sampled parity checks at full size.  coef: [npix, levels, L].        */
void orc_composite_pixels(const double* cam_arr, int levels, int K, int L, const uint32_t* ranges,
                          const uint32_t* ids, const double* mean2d, const double* conic,
                          const double* opacity, const int32_t* topk_idx, const double* topk_w,
                          int64_t npix, const int64_t* pix, double* coef, double* final_T,
                          int32_t* last, double* margin, double* margin_T) {
    cam_t cam = cam_from(cam_arr);
    uint32_t maxlen = max_range(ranges, cam.tx * cam.ty);
    memset(coef, 0, sizeof(double) * (size_t)npix * levels * L);
    #pragma omp parallel
    {
        int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (maxlen + 1));
        double* e = (double*)malloc(sizeof(double) * (maxlen + 1));
        #pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < npix; ++q) {
            int px = (int)(pix[q] % cam.W), py = (int)(pix[q] / cam.W);
            int t = (py / ORC_TILE) * cam.tx + px / ORC_TILE;
            double T, mg, mgT;
            int32_t lst;
            int cnt = walk_pixel(px + 0.5, py + 0.5, ranges[2 * t], ranges[2 * t + 1], ids, mean2d,
                                 conic, opacity, pos, e, NULL, NULL, &T, &lst, &mg, &mgT);
            for (int c = 0; c < cnt; ++c) {
                uint32_t i = ids[ranges[2 * t] + pos[c]];
                for (int lv = 0; lv < levels; ++lv) {
                    double* W = coef + ((size_t)q * levels + lv) * L;
                    for (int k = 0; k < K; ++k) {
                        size_t o = ((size_t)i * levels + lv) * K + k;
                        W[topk_idx[o]] += topk_w[o] * e[c];
                    }
                }
            }
            final_T[q] = T;
            last[q] = lst;
            margin[q] = mg;
            margin_T[q] = mgT;
        }
        free(pos);
        free(e);
    }
}

/* orc_composite_pixels with the near decisions of pixel q taken as     */
/* flips[q] selects (walk_pixel_alt); n_near[q] = the number of near    */
/* decisions that pixel's walk met.  coef: [npix, levels, L].           */
void orc_composite_pixels_alt(const double* cam_arr, int levels, int K, int L, const uint32_t* ranges,
                              const uint32_t* ids, const double* mean2d, const double* conic,
                              const double* opacity, const int32_t* topk_idx, const double* topk_w,
                              int64_t npix, const int64_t* pix, const uint32_t* flips, double thr, double* coef,
                              double* final_T, int32_t* last, int32_t* n_near) {
    cam_t cam = cam_from(cam_arr);
    uint32_t maxlen = max_range(ranges, cam.tx * cam.ty);
    memset(coef, 0, sizeof(double) * (size_t)npix * levels * L);
    #pragma omp parallel
    {
        int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (maxlen + 1));
        double* e = (double*)malloc(sizeof(double) * (maxlen + 1));
        #pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < npix; ++q) {
            int px = (int)(pix[q] % cam.W), py = (int)(pix[q] / cam.W);
            int t = (py / ORC_TILE) * cam.tx + px / ORC_TILE;
            double T;
            int32_t lst;
            int nn;
            int cnt = walk_pixel_alt(px + 0.5, py + 0.5, ranges[2 * t], ranges[2 * t + 1], ids, mean2d, conic,
                                     opacity, thr, flips[q], pos, e, &T, &lst, &nn);
            for (int c = 0; c < cnt; ++c) {
                uint32_t i = ids[ranges[2 * t] + pos[c]];
                for (int lv = 0; lv < levels; ++lv) {
                    double* W = coef + ((size_t)q * levels + lv) * L;
                    for (int k = 0; k < K; ++k) {
                        size_t o = ((size_t)i * levels + lv) * K + k;
                        W[topk_idx[o]] += topk_w[o] * e[c];
                    }
                }
            }
            final_T[q] = T;
            last[q] = lst;
            n_near[q] = nn;
        }
        free(pos);
        free(e);
    }
}

/* Brute-force renderer: for every pixel, gather all Gaussians whose tile */
/* rectangle (float32 rule) contains the pixel's tile, order them by     */
/* (float32 depth, id) and composite.  No tile lists involved; used to   */
/* pin the binning.  coef: [levels, H, W, L].                           */
typedef struct { uint32_t dbits, id; } dkey_t;
static int dkey_cmp(const void* a, const void* b) {
    const dkey_t* p = (const dkey_t*)a;
    const dkey_t* q = (const dkey_t*)b;
    if (p->dbits != q->dbits) return p->dbits < q->dbits ? -1 : 1;
    return p->id < q->id ? -1 : (p->id > q->id ? 1 : 0);
}

void orc_composite_bruteforce(const double* cam_arr, int n, int levels, int K, int L,
                              const float* mean2d_f32, const int32_t* radius, const float* depth_f32,
                              const double* mean2d, const double* conic, const double* opacity,
                              const int32_t* topk_idx, const double* topk_w, double* coef,
                              double* final_T) {
    cam_t cam = cam_from(cam_arr);
    size_t HW = (size_t)cam.W * cam.H;
    memset(coef, 0, sizeof(double) * (size_t)levels * HW * L);
    #pragma omp parallel
    {
        dkey_t* list = (dkey_t*)malloc(sizeof(dkey_t) * (size_t)(n > 0 ? n : 1));
        #pragma omp for schedule(dynamic, 1)
        for (int py = 0; py < cam.H; ++py)
            for (int px = 0; px < cam.W; ++px) {
                int tx = px / ORC_TILE, ty = py / ORC_TILE;
                int cnt = 0;
                for (int i = 0; i < n; ++i) {
                    int x0, y0, x1, y1;
                    if (radius[i] <= 0) continue;
                    if (!rect_f32(mean2d_f32[2 * i], mean2d_f32[2 * i + 1], radius[i], cam.tx, cam.ty,
                                  &x0, &y0, &x1, &y1))
                        continue;
                    if (tx < x0 || tx > x1 || ty < y0 || ty > y1) continue;
                    list[cnt].dbits = f32_bits(depth_f32[i]);
                    list[cnt].id = (uint32_t)i;
                    ++cnt;
                }
                qsort(list, (size_t)cnt, sizeof(dkey_t), dkey_cmp);
                double T = 1.0;
                size_t pix = (size_t)py * cam.W + px;
                for (int c = 0; c < cnt; ++c) {
                    uint32_t i = list[c].id;
                    double dx = mean2d[2 * i] - (px + 0.5), dy = mean2d[2 * i + 1] - (py + 0.5);
                    double power = -0.5 * (conic[3 * i] * dx * dx + conic[3 * i + 2] * dy * dy)
                                   - conic[3 * i + 1] * dx * dy;
                    if (power > 0) continue;
                    double alpha = fmin(ALPHA_MAX, opacity[i] * exp(power));
                    if (alpha < ALPHA_MIN) continue;
                    if (T * (1.0 - alpha) < T_MIN) break;
                    for (int lv = 0; lv < levels; ++lv)
                        for (int k = 0; k < K; ++k) {
                            size_t o = ((size_t)i * levels + lv) * K + k;
                            coef[((size_t)lv * HW + pix) * L + topk_idx[o]] += topk_w[o] * alpha * T;
                        }
                    T *= 1.0 - alpha;
                }
                final_T[pix] = T;
            }
        free(list);
    }
}

/* ------------------------------------------------------------------ */
/* Decode (Eq. 7): F = W S, one plain triple loop per pixel row.        */
/* coef [M, L], dict [L, D], out [M, D].  Pinned against a library      */
/* float64 matrix product.                                             */
/* ------------------------------------------------------------------ */
void orc_decode(int64_t M, int L, int D, const double* coef, const double* dict, double* out) {
    #pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < M; ++m) {
        double* o = out + m * D;
        for (int d = 0; d < D; ++d) o[d] = 0.0;
        for (int l = 0; l < L; ++l) {
            double c = coef[m * L + l];
            const double* s = dict + (size_t)l * D;
            for (int d = 0; d < D; ++d) o[d] += c * s[d];
        }
    }
}

/* float32 -> bfloat16 -> float32, round to nearest, ties to even (IEEE).  */
static float round_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) {          /* inf / nan */
        if (u & 0x007fffffu) u |= 0x00400000u;        /* keep nan quiet */
        u &= 0xffff0000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7fffu + lsb;
        u &= 0xffff0000u;
    }
    float r;
    memcpy(&r, &u, 4);
    return r;
}

void orc_round_bf16(int64_t n, const float* in, float* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = round_bf16(in[i]);
}

/* Decode with both operands rounded to bfloat16 first (the precision form:
 * bf16 inputs, exact products, wide accumulation).  If round_out, the
 * result is rounded to float32 and then to bfloat16.  Pinned by the
 * rounding routine against a library bf16 conversion and by reduction to
 * orc_decode when inputs are already bf16-representable. */
void orc_decode_bf16(int64_t M, int L, int D, const float* coef, const float* dict, int round_out,
                     double* out) {
    float* sb = (float*)malloc(sizeof(float) * (size_t)L * D);
    for (size_t j = 0; j < (size_t)L * D; ++j) sb[j] = round_bf16(dict[j]);
    #pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < M; ++m) {
        double* o = out + m * D;
        for (int d = 0; d < D; ++d) o[d] = 0.0;
        for (int l = 0; l < L; ++l) {
            double c = (double)round_bf16(coef[m * L + l]);
            const float* s = sb + (size_t)l * D;
            for (int d = 0; d < D; ++d) o[d] += c * (double)s[d];
        }
        if (round_out)
            for (int d = 0; d < D; ++d) o[d] = (double)round_bf16((float)o[d]);
    }
    free(sb);
}

/* ------------------------------------------------------------------ */
/* Relevancy (Section 3.2, which takes LERF's score): with cosine      */
/* s_q = cos(F, q) and s_j = cos(F, c_j) against the canonical          */
/* negatives, r = min_j exp(tau s_q) / (exp(tau s_q) + exp(tau s_j)).  */
/* A zero feature (norm below 1e-12) has cosine 0 with everything.     */
/* Pinned by the closed form sigmoid(tau (s_q - max_j s_j)), F = q and  */
/* F = 0 special cases.                                                 */
/* ------------------------------------------------------------------ */
static double cosine(const double* f, const float* e, int D) {
    double fe = 0, ff = 0, ee = 0;
    for (int d = 0; d < D; ++d) {
        fe += f[d] * (double)e[d];
        ff += f[d] * f[d];
        ee += (double)e[d] * (double)e[d];
    }
    double nf = sqrt(ff), ne = sqrt(ee);
    if (nf < 1e-12) nf = 1e-12;
    if (ne < 1e-12) ne = 1e-12;
    return fe / (nf * ne);
}

void orc_query(int64_t M, int D, const double* feat, const float* pos, int n_neg, const float* neg,
               double tau, double* out) {
    #pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < M; ++m) {
        const double* f = feat + m * D;
        double sq = cosine(f, pos, D);
        double r = INFINITY;
        for (int j = 0; j < n_neg; ++j) {
            double sj = cosine(f, neg + (size_t)j * D, D);
            double eq = exp(tau * sq), ej = exp(tau * sj);
            double pj = eq / (eq + ej);
            if (pj < r) r = pj;
        }
        out[m] = r;
    }
}

/* ================================================================== */
/* Backward pass.  The paper learns the sparse coefficients and the    */
/* codebook jointly (Section 3.3) but prints no backward formulas; the */
/* functions below are the chain rule of the forward definitions above, */
/* derived by hand in float64.  Every one is pinned by central finite  */
/* differences of the corresponding forward function.  Discrete        */
/* decisions (culling, tile rectangles, depth order, the alpha clamp,  */
/* the 1/255 skip and the transmittance stop) are held fixed: they     */
/* have zero derivative almost everywhere.                             */
/* ================================================================== */

/* Training loss on a feature map F against a target Y (M rows of D):
 *   loss = mean_{m,d} |F - Y| + mean_m (1 - cos(F_m, Y_m)),
 * cos(a, b) = a.b / (max(|a|, 1e-12) max(|b|, 1e-12)), sign(0) = 0.
 * Writes the loss and dloss/dF. */
void orc_loss_l1cos(int64_t M, int D, const double* F, const double* Y, double* loss, double* dF) {
    double l1 = 0.0, lc = 0.0;
    const double inv_md = 1.0 / ((double)M * D), inv_m = 1.0 / (double)M;
    #pragma omp parallel for schedule(static) reduction(+ : l1, lc)
    for (int64_t m = 0; m < M; ++m) {
        const double* f = F + m * D;
        const double* y = Y + m * D;
        double* g = dF + m * D;
        double fy = 0, ff = 0, yy = 0;
        for (int d = 0; d < D; ++d) {
            double e = f[d] - y[d];
            l1 += fabs(e);
            g[d] = (e > 0 ? 1.0 : (e < 0 ? -1.0 : 0.0)) * inv_md;
            fy += f[d] * y[d];
            ff += f[d] * f[d];
            yy += y[d] * y[d];
        }
        double nf = sqrt(ff), ny = sqrt(yy);
        double gf = nf > 1e-12 ? nf : 1e-12, gy = ny > 1e-12 ? ny : 1e-12;
        double c = fy / (gf * gy);
        lc += 1.0 - c;
        /* d(-c)/df = -(y / (gf gy) - [nf > eps] fy f / (nf^3 gy)) */
        for (int d = 0; d < D; ++d) {
            double dc = y[d] / (gf * gy);
            if (nf > 1e-12) dc -= fy * f[d] / (nf * nf * nf * gy);
            g[d] -= dc * inv_m;
        }
    }
    *loss = l1 * inv_md + lc * inv_m;
}

/* Relevancy backward: r = min_j sigmoid(tau (s_q - s_j)) = sigmoid(tau (s_q -
 * s_j*)) with j* the first negative of largest similarity.  Writes
 * dF = d_rel * dr/dF.  ``margin`` (per row, may be NULL) is the gap between
 * the two largest negative similarities (the subgradient choice flips there). */
static void cos_grad(const double* f, const float* e, int D, double* out_scale_e, double* out_scale_f,
                     double* s_out) {
    /* s = f.e / (gf ge); ds/df = e / (gf ge) - [nf > eps] (f.e) f / (nf^3 ge) */
    double fe = 0, ff = 0, ee = 0;
    for (int d = 0; d < D; ++d) {
        fe += f[d] * (double)e[d];
        ff += f[d] * f[d];
        ee += (double)e[d] * (double)e[d];
    }
    double nf = sqrt(ff), ne = sqrt(ee);
    double gf = nf > 1e-12 ? nf : 1e-12, ge = ne > 1e-12 ? ne : 1e-12;
    *s_out = fe / (gf * ge);
    *out_scale_e = 1.0 / (gf * ge);
    *out_scale_f = nf > 1e-12 ? -fe / (nf * nf * nf * ge) : 0.0;
}

void orc_query_backward(int64_t M, int D, const double* feat, const float* pos, int n_neg, const float* neg,
                        double tau, const double* d_rel, double* d_feat, double* margin) {
    #pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < M; ++m) {
        const double* f = feat + m * D;
        double* g = d_feat + m * D;
        double aq, bq, sq;
        cos_grad(f, pos, D, &aq, &bq, &sq);
        int jstar = 0;
        double smax = -INFINITY, s2 = -INFINITY;
        double aj = 0, bj = 0;
        for (int j = 0; j < n_neg; ++j) {
            double a_, b_, s_;
            cos_grad(f, neg + (size_t)j * D, D, &a_, &b_, &s_);
            if (s_ > smax) {
                s2 = smax;
                smax = s_;
                jstar = j;
                aj = a_;
                bj = b_;
            } else if (s_ > s2) {
                s2 = s_;
            }
        }
        if (margin) margin[m] = n_neg > 1 ? smax - s2 : INFINITY;
        double r = 1.0 / (1.0 + exp(-tau * (sq - smax)));
        double dr = d_rel[m] * tau * r * (1.0 - r); /* dr/d(s_q - s_j*) */
        const float* ej = neg + (size_t)jstar * D;
        for (int d = 0; d < D; ++d)
            g[d] = dr * ((aq * pos[d] + bq * f[d]) - (aj * ej[d] + bj * f[d]));
    }
}

/* Decode backward (Eq. 7 is linear): d_coef = d_feat S^T, d_dict = coef^T d_feat. */
void orc_decode_backward(int64_t M, int L, int D, const double* coef, const double* dict, const double* d_feat,
                         double* d_coef, double* d_dict) {
    #pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < M; ++m)
        for (int l = 0; l < L; ++l) {
            double s = 0;
            for (int d = 0; d < D; ++d) s += d_feat[m * D + d] * dict[(size_t)l * D + d];
            d_coef[m * L + l] = s;
        }
    #pragma omp parallel for schedule(static)
    for (int l = 0; l < L; ++l) {
        for (int d = 0; d < D; ++d) d_dict[(size_t)l * D + d] = 0.0;
        for (int64_t m = 0; m < M; ++m) {
            double c = coef[m * L + l];
            if (c == 0.0) continue;
            for (int d = 0; d < D; ++d) d_dict[(size_t)l * D + d] += c * d_feat[m * D + d];
        }
    }
}

/* Compositing backward.  For one pixel with contributors i = 1..n (front to
 * back), blend weights e_i = alpha_i T_i, T_i = prod_{j<i} (1 - alpha_j):
 *   W_l[j] = sum_i e_i w_{i,l,j}.
 * With g_l = dL/dW_l and c_i = sum_l sum_k g_l[idx_ilk] w_ilk:
 *   dL/dw_ilk  += g_l[idx_ilk] e_i
 *   dL/dalpha_i = T_i c_i - (1 / (1 - alpha_i)) sum_{m > i} c_m e_m
 * (e_m for m > i contains the factor 1 - alpha_i once).  Then
 *   alpha_i = o_i exp(power_i) (unclamped; 0 gradient where clamped at 0.99),
 *   dalpha/do = exp(power), dalpha/dpower = alpha,
 *   power = -0.5 (A dx^2 + C dy^2) - B dx dy with (dx, dy) = mean2d - pixel:
 *   dpower/du = -(A dx + B dy), dpower/dv = -(C dy + B dx),
 *   dpower/dA = -dx^2 / 2, dpower/dB = -dx dy, dpower/dC = -dy^2 / 2.
 * The forward walk is re-run here and its contributors stored; the suffix
 * sums are formed directly.  Gradient outputs are overwritten. */
/* One pixel's share of the splat gradients: g0 points at the pixel's     */
/* dL/dcoef of level 0 and level lv sits lv_stride doubles further.  The   */
/* scratch arrays hold maxlen + 1 entries.                                */
static void backward_pixel(const cam_t* cam, int px, int py, int levels, int K, const uint32_t* ranges,
                           const uint32_t* ids, const double* mean2d, const double* conic, const double* opacity,
                           const int32_t* topk_idx, const double* topk_w, const double* g0, size_t lv_stride,
                           int32_t* pos, double* e, double* Tb, double* al, double* cc, double* d_mean2d,
                           double* d_conic, double* d_opacity, double* d_w) {
    int t = (py / ORC_TILE) * cam->tx + px / ORC_TILE;
    double T, mg;
    int32_t lst;
    int cnt = walk_pixel(px + 0.5, py + 0.5, ranges[2 * t], ranges[2 * t + 1], ids, mean2d, conic, opacity, pos,
                         e, Tb, al, &T, &lst, &mg, NULL);
    for (int c = 0; c < cnt; ++c) {
        uint32_t i = ids[ranges[2 * t] + pos[c]];
        double s = 0;
        for (int lv = 0; lv < levels; ++lv) {
            const double* g = g0 + (size_t)lv * lv_stride;
            for (int k = 0; k < K; ++k) {
                size_t o = ((size_t)i * levels + lv) * K + k;
                s += g[topk_idx[o]] * topk_w[o];
                d_w[o] += g[topk_idx[o]] * e[c];
            }
        }
        cc[c] = s;
    }
    double suffix = 0.0; /* sum_{m > i} c_m e_m */
    for (int c = cnt - 1; c >= 0; --c) {
        uint32_t i = ids[ranges[2 * t] + pos[c]];
        double dalpha = Tb[c] * cc[c] - suffix / (1.0 - al[c]);
        suffix += cc[c] * e[c];
        double dx = mean2d[2 * i] - (px + 0.5), dy = mean2d[2 * i + 1] - (py + 0.5);
        double A = conic[3 * i], B = conic[3 * i + 1], C = conic[3 * i + 2];
        double power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy;
        double G = exp(power);
        if (opacity[i] * G >= ALPHA_MAX) continue; /* clamped: no gradient */
        double dpow = dalpha * opacity[i] * G;
        d_opacity[i] += dalpha * G;
        d_mean2d[2 * i] += dpow * (-(A * dx + B * dy));
        d_mean2d[2 * i + 1] += dpow * (-(C * dy + B * dx));
        d_conic[3 * i] += dpow * (-0.5 * dx * dx);
        d_conic[3 * i + 1] += dpow * (-dx * dy);
        d_conic[3 * i + 2] += dpow * (-0.5 * dy * dy);
    }
}

static void zero_splat_grads(int n, int levels, int K, double* d_mean2d, double* d_conic, double* d_opacity,
                             double* d_w) {
    memset(d_mean2d, 0, sizeof(double) * 2 * (size_t)n);
    memset(d_conic, 0, sizeof(double) * 3 * (size_t)n);
    memset(d_opacity, 0, sizeof(double) * (size_t)n);
    memset(d_w, 0, sizeof(double) * (size_t)n * levels * K);
}

void orc_composite_backward(const double* cam_arr, int n, int levels, int K, int L, const uint32_t* ranges,
                            const uint32_t* ids, const double* mean2d, const double* conic, const double* opacity,
                            const int32_t* topk_idx, const double* topk_w, const double* d_coef,
                            double* d_mean2d, double* d_conic, double* d_opacity, double* d_w) {
    cam_t cam = cam_from(cam_arr);
    int ntiles = cam.tx * cam.ty;
    size_t HW = (size_t)cam.W * cam.H;
    zero_splat_grads(n, levels, K, d_mean2d, d_conic, d_opacity, d_w);
    uint32_t maxlen = max_range(ranges, ntiles);
    /* sequential over pixels: gradient accumulation into shared per-Gaussian
     * slots stays deterministic and obviously race-free */
    int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (maxlen + 1));
    double* e = (double*)malloc(sizeof(double) * (maxlen + 1));
    double* Tb = (double*)malloc(sizeof(double) * (maxlen + 1));
    double* al = (double*)malloc(sizeof(double) * (maxlen + 1));
    double* cc = (double*)malloc(sizeof(double) * (maxlen + 1));
    for (int t = 0; t < ntiles; ++t) {
        int tx = t % cam.tx, ty = t / cam.tx;
        for (int py = ty * ORC_TILE; py < (ty + 1) * ORC_TILE && py < cam.H; ++py)
            for (int px = tx * ORC_TILE; px < (tx + 1) * ORC_TILE && px < cam.W; ++px)
                backward_pixel(&cam, px, py, levels, K, ranges, ids, mean2d, conic, opacity, topk_idx, topk_w,
                               d_coef + ((size_t)py * cam.W + px) * L, HW * L, pos, e, Tb, al, cc, d_mean2d,
                               d_conic, d_opacity, d_w);
    }
    free(pos);
    free(e);
    free(Tb);
    free(al);
    free(cc);
}

/* The same gradients when dL/dcoef is zero outside the listed pixels (flat */
/* indices py * W + px, each listed once): a pixel with zero upstream       */
/* gradient adds nothing to any Gaussian, so only the listed pixels are     */
/* walked.  d_coef: [npix, levels, L], row q for pixel pix[q].             */
void orc_composite_backward_pixels(const double* cam_arr, int n, int levels, int K, int L,
                                   const uint32_t* ranges, const uint32_t* ids, const double* mean2d,
                                   const double* conic, const double* opacity, const int32_t* topk_idx,
                                   const double* topk_w, int64_t npix, const int64_t* pix, const double* d_coef,
                                   double* d_mean2d, double* d_conic, double* d_opacity, double* d_w) {
    cam_t cam = cam_from(cam_arr);
    zero_splat_grads(n, levels, K, d_mean2d, d_conic, d_opacity, d_w);
    uint32_t maxlen = max_range(ranges, cam.tx * cam.ty);
    int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (maxlen + 1));
    double* e = (double*)malloc(sizeof(double) * (maxlen + 1));
    double* Tb = (double*)malloc(sizeof(double) * (maxlen + 1));
    double* al = (double*)malloc(sizeof(double) * (maxlen + 1));
    double* cc = (double*)malloc(sizeof(double) * (maxlen + 1));
    for (int64_t q = 0; q < npix; ++q)
        backward_pixel(&cam, (int)(pix[q] % cam.W), (int)(pix[q] / cam.W), levels, K, ranges, ids, mean2d, conic,
                       opacity, topk_idx, topk_w, d_coef + (size_t)q * levels * L, L, pos, e, Tb, al, cc, d_mean2d,
                       d_conic, d_opacity, d_w);
    free(pos);
    free(e);
    free(Tb);
    free(al);
    free(cc);
}

/* Projection backward: from dL/d(mean2d) and dL/d(conic) to dL/d(means),
 * dL/d(scales), dL/d(quats) through
 *   p = R_wc mu + t,  (u, v) = (fx x/z + cx, fy y/z + cy),
 *   Sigma = M M^T, M = R(q / |q|) diag(s),  Sigma_c = R_wc Sigma R_wc^T,
 *   Sigma2D = J Sigma_c J^T + 0.3 I, J = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]],
 *   conic = Sigma2D^-1 as (A, B, C) = (c, -b, a) / (ac - b^2).
 * Culled Gaussians (radius 0) get zero gradients.  Outputs overwritten. */
static void quat_rot_grad(const double q_in[4], const double dR[9], double dq[4]) {
    /* dL/dq for R(q/|q|): first dL/dqhat from the rotation formula, then the
     * projection through the normalisation. */
    double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
    double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
    double g[4];
    /* R00 = 1 - 2(y^2 + z^2)  R01 = 2(xy - wz)  R02 = 2(xz + wy)
     * R10 = 2(xy + wz)  R11 = 1 - 2(x^2 + z^2)  R12 = 2(yz - wx)
     * R20 = 2(xz - wy)  R21 = 2(yz + wx)  R22 = 1 - 2(x^2 + y^2) */
    g[0] = 2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    g[1] = 2 * (y * dR[1] + z * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                2 * x * dR[8]);
    g[2] = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                2 * y * dR[8]);
    g[3] = 2 * (-2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * z * dR[4] + y * dR[5] + x * dR[6] +
                y * dR[7]);
    double qh[4] = {w, x, y, z};
    double dot = g[0] * qh[0] + g[1] * qh[1] + g[2] * qh[2] + g[3] * qh[3];
    for (int k = 0; k < 4; ++k) dq[k] = (g[k] - dot * qh[k]) / n;
}

static void project_backward_one(const cam_t* cam, const double mu[3], const double s[3], const double q[4],
                                 const double* d_mean2d, const double* d_conic, int i, double* d_means,
                                 double* d_scales, double* d_quats) {
    double p[3];
    for (int r = 0; r < 3; ++r)
        p[r] = cam->R[3 * r] * mu[0] + cam->R[3 * r + 1] * mu[1] + cam->R[3 * r + 2] * mu[2] + cam->t[r];
    double x = p[0], y = p[1], z = p[2];
    double Rq[9], M[9], Mt[9], Sig[9], Rt[9], tmp[9], Sc[9];
    quat_to_rot(q, Rq);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * s[c];
    transpose3(M, Mt);
    matmul3(M, Mt, Sig);
    transpose3(cam->R, Rt);
    matmul3(cam->R, Sig, tmp);
    matmul3(tmp, Rt, Sc);
    double J[6] = {cam->fx / z, 0.0, -cam->fx * x / (z * z), 0.0, cam->fy / z, -cam->fy * y / (z * z)};
    /* Sigma2D entries */
    double cv[4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += J[3 * r + k] * Sc[3 * k + l] * J[3 * c + l];
            cv[2 * r + c] = acc;
        }
    double a = cv[0] + DILATION, b = cv[1], c = cv[3] + DILATION;
    double det = a * c - b * b;
    /* conic (A, B, C) = (c, -b, a) / det: derivatives w.r.t. (a, b, c) */
    double gA = d_conic[3 * i], gB = d_conic[3 * i + 1], gC = d_conic[3 * i + 2];
    double d2 = det * det;
    double ga = gA * (-c * c / d2) + gB * (b * c / d2) + gC * (1.0 / det - a * c / d2);
    double gb = gA * (2.0 * b * c / d2) + gB * (-1.0 / det - 2.0 * b * b / d2) + gC * (2.0 * a * b / d2);
    double gc = gA * (1.0 / det - a * c / d2) + gB * (a * b / d2) + gC * (-a * a / d2);
    /* symmetric gradient matrix of Sigma2D: dL = ga da + gb db + gc dc with
     * b appearing twice in the matrix */
    double G2[4] = {ga, 0.5 * gb, 0.5 * gb, gc};
    /* dL/dSigma_c = J^T G2 J; dL/dJ = 2 G2 J Sigma_c */
    double GS[9];
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            double acc = 0;
            for (int r = 0; r < 2; ++r)
                for (int cc2 = 0; cc2 < 2; ++cc2) acc += J[3 * r + k] * G2[2 * r + cc2] * J[3 * cc2 + l];
            GS[3 * k + l] = acc;
        }
    double GJ[6];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) {
            double acc = 0;
            for (int cc2 = 0; cc2 < 2; ++cc2)
                for (int l = 0; l < 3; ++l) acc += G2[2 * r + cc2] * J[3 * cc2 + l] * Sc[3 * l + k];
            GJ[3 * r + k] = 2.0 * acc;
        }
    /* J depends on p: J00 = fx/z, J02 = -fx x/z^2, J11 = fy/z, J12 = -fy y/z^2 */
    double dp[3] = {0, 0, 0};
    dp[0] += GJ[2] * (-cam->fx / (z * z));
    dp[1] += GJ[5] * (-cam->fy / (z * z));
    dp[2] += GJ[0] * (-cam->fx / (z * z)) + GJ[2] * (2.0 * cam->fx * x / (z * z * z)) +
             GJ[4] * (-cam->fy / (z * z)) + GJ[5] * (2.0 * cam->fy * y / (z * z * z));
    /* mean2d */
    double gu = d_mean2d[2 * i], gv = d_mean2d[2 * i + 1];
    dp[0] += gu * cam->fx / z;
    dp[1] += gv * cam->fy / z;
    dp[2] += gu * (-cam->fx * x / (z * z)) + gv * (-cam->fy * y / (z * z));
    /* p = R_wc mu + t */
    for (int k = 0; k < 3; ++k)
        d_means[3 * i + k] = cam->R[k] * dp[0] + cam->R[3 + k] * dp[1] + cam->R[6 + k] * dp[2];
    /* Sigma_c = R_wc Sigma R_wc^T -> dL/dSigma = R_wc^T GS R_wc */
    double t1[9], GSig[9];
    matmul3(Rt, GS, t1);
    matmul3(t1, cam->R, GSig);
    /* Sigma = M M^T -> dL/dM = (GSig + GSig^T) M */
    double GSs[9], dM[9];
    for (int k = 0; k < 9; ++k) GSs[k] = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int cc2 = 0; cc2 < 3; ++cc2) GSs[3 * r + cc2] = GSig[3 * r + cc2] + GSig[3 * cc2 + r];
    matmul3(GSs, M, dM);
    /* M = Rq diag(s) */
    double dR[9];
    for (int r = 0; r < 3; ++r)
        for (int cc2 = 0; cc2 < 3; ++cc2) dR[3 * r + cc2] = dM[3 * r + cc2] * s[cc2];
    for (int cc2 = 0; cc2 < 3; ++cc2) {
        double acc = 0;
        for (int r = 0; r < 3; ++r) acc += dM[3 * r + cc2] * Rq[3 * r + cc2];
        d_scales[3 * i + cc2] = acc;
    }
    quat_rot_grad(q, dR, d_quats + 4 * i);
}

void orc_project_backward(const double* cam_arr, int n, const float* means, const float* scales, const float* quats,
                          const int32_t* radius, const double* d_mean2d, const double* d_conic, double* d_means,
                          double* d_scales, double* d_quats) {
    cam_t cam = cam_from(cam_arr);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k) d_means[3 * i + k] = d_scales[3 * i + k] = 0.0;
        for (int k = 0; k < 4; ++k) d_quats[4 * i + k] = 0.0;
        if (radius[i] <= 0) continue;
        double mu[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
        double s3[3] = {scales[3 * i], scales[3 * i + 1], scales[3 * i + 2]};
        double q[4] = {quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]};
        project_backward_one(&cam, mu, s3, q, d_mean2d, d_conic, i, d_means, d_scales, d_quats);
    }
}

/* Same on float64 inputs (finite-difference checks). */
void orc_project_backward_f64(const double* cam_arr, int n, const double* means, const double* scales,
                              const double* quats, const int32_t* radius, const double* d_mean2d,
                              const double* d_conic, double* d_means, double* d_scales, double* d_quats) {
    cam_t cam = cam_from(cam_arr);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k) d_means[3 * i + k] = d_scales[3 * i + k] = 0.0;
        for (int k = 0; k < 4; ++k) d_quats[4 * i + k] = 0.0;
        if (radius[i] <= 0) continue;
        project_backward_one(&cam, means + 3 * i, scales + 3 * i, quats + 4 * i, d_mean2d, d_conic, i, d_means,
                             d_scales, d_quats);
    }
}

