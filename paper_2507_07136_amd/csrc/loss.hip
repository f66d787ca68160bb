// ls2_feature_loss: a feature-map objective for fitting the sparse
// coefficient field and codebook to 2D feature maps Y (Section 4.1 trains the
// field for 10,000 iterations with the Gaussian geometry fixed; the paper does
// not print the loss).  This library reads it as an equal-weight L1 plus
// cosine term:
//   loss = mean_{v,d} |F - Y| + mean_v (1 - cos(F(v), Y(v))),
// with cos(a, b) = a.b / (|a|_g |b|_g), |x|_g = max(|x|, 1e-12), sign(0) = 0,
// and its gradient
//   dF = sign(F - Y) / (m D) - (Y / (|F|_g |Y|_g) - [|F| > eps] (F.Y) F / (|F|^3 |Y|_g)) / m.
//
// One wave per row.  Each workgroup writes its partial sums (in double) to the
// workspace and a one-workgroup kernel adds them in a fixed order, so the
// loss is deterministic.
#include "ls2_internal.h"

namespace ls2 {

constexpr int kLossBlocks = 2048;
constexpr int kLossMaxV = 4;  // float4s per lane: D <= 1024

__device__ __forceinline__ float sgn(float e) { return e > 0.f ? 1.f : (e < 0.f ? -1.f : 0.f); }

__global__ __launch_bounds__(256) void k_feature_loss(long long m, int D, const float* __restrict__ F,
                                                      const float* __restrict__ Y, float* __restrict__ dF,
                                                      double* __restrict__ partial) {
    __shared__ double red[2][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nv4 = D / 4;
    const float inv_md = (float)(1.0 / ((double)m * D)), inv_m = (float)(1.0 / (double)m);
    double l1_acc = 0.0, lc_acc = 0.0;
    const long long wstride = (long long)gridDim.x * 4;
    for (long long row = (long long)blockIdx.x * 4 + wave; row < m; row += wstride) {
        float4 f[kLossMaxV], y[kLossMaxV];
        float l1 = 0.f, fy = 0.f, ff = 0.f, yy = 0.f;
#pragma unroll
        for (int q = 0; q < kLossMaxV; ++q) {
            const int v = lane + 64 * q;
            f[q] = y[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (v < nv4) {
                f[q] = reinterpret_cast<const float4*>(F + row * D)[v];
                y[q] = reinterpret_cast<const float4*>(Y + row * D)[v];
            }
            l1 += fabsf(f[q].x - y[q].x) + fabsf(f[q].y - y[q].y) + fabsf(f[q].z - y[q].z) + fabsf(f[q].w - y[q].w);
            fy = fmaf(f[q].x, y[q].x, fmaf(f[q].y, y[q].y, fmaf(f[q].z, y[q].z, fmaf(f[q].w, y[q].w, fy))));
            ff = fmaf(f[q].x, f[q].x, fmaf(f[q].y, f[q].y, fmaf(f[q].z, f[q].z, fmaf(f[q].w, f[q].w, ff))));
            yy = fmaf(y[q].x, y[q].x, fmaf(y[q].y, y[q].y, fmaf(y[q].z, y[q].z, fmaf(y[q].w, y[q].w, yy))));
        }
        l1 = wave_allsum(l1);
        fy = wave_allsum(fy);
        ff = wave_allsum(ff);
        yy = wave_allsum(yy);
        const float nf = sqrtf(ff), ny = sqrtf(yy);
        const float gf = fmaxf(nf, 1e-12f), gy = fmaxf(ny, 1e-12f);
        const float c = fy / (gf * gy);
        l1_acc += (double)l1;
        lc_acc += (double)(1.0f - c);
        if (dF) {
            const float ay = inv_m / (gf * gy);
            const float bf = nf > 1e-12f ? inv_m * fy / (nf * nf * nf * gy) : 0.f;
#pragma unroll
            for (int q = 0; q < kLossMaxV; ++q) {
                const int v = lane + 64 * q;
                if (v < nv4) {
                    float4 o;
                    o.x = sgn(f[q].x - y[q].x) * inv_md - ay * y[q].x + bf * f[q].x;
                    o.y = sgn(f[q].y - y[q].y) * inv_md - ay * y[q].y + bf * f[q].y;
                    o.z = sgn(f[q].z - y[q].z) * inv_md - ay * y[q].z + bf * f[q].z;
                    o.w = sgn(f[q].w - y[q].w) * inv_md - ay * y[q].w + bf * f[q].w;
                    reinterpret_cast<float4*>(dF + row * D)[v] = o;
                }
            }
        }
    }
    if (lane == 0) {
        red[0][wave] = l1_acc;
        red[1][wave] = lc_acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        partial[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

__global__ __launch_bounds__(64) void k_feature_loss_final(const double* __restrict__ partial, int nblocks,
                                                  long long m, int D, double* __restrict__ loss) {
    // lane t adds the partials t, t + 64, ... in order; lane 0 then adds the
    // 64 lane sums in order: a fixed summation order, so the loss is
    // reproducible
    __shared__ double s[2][64];
    const int t = threadIdx.x;
    double l1 = 0.0, lc = 0.0;
    for (int b = t; b < nblocks; b += 64) {
        l1 += partial[2 * b];
        lc += partial[2 * b + 1];
    }
    s[0][t] = l1;
    s[1][t] = lc;
    __syncthreads();
    if (t == 0) {
        double a = 0.0, c = 0.0;
        for (int k = 0; k < 64; ++k) {
            a += s[0][k];
            c += s[1][k];
        }
        *loss = a / ((double)m * D) + c / (double)m;
    }
}

static int loss_blocks(long long m) {
    const long long b = (m + 3) / 4;
    return (int)(b < kLossBlocks ? (b < 1 ? 1 : b) : kLossBlocks);
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_feature_loss_workspace(int64_t m, size_t* bytes) {
    if (!bytes || m < 0) return LS2_ERR_ARG;
    *bytes = (size_t)loss_blocks(m) * 2 * sizeof(double);
    return LS2_OK;
}

extern "C" int ls2_feature_loss(int64_t m, int32_t D, const float* feat, const float* target, double* loss,
                                float* d_feat, void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (m < 1 || D < 1 || !feat || !target || !loss || !workspace) return LS2_ERR_ARG;
    if (D % 64 != 0 || D > 1024) return LS2_ERR_UNSUPPORTED;
    const int nb = loss_blocks(m);
    if (workspace_bytes < (size_t)nb * 2 * sizeof(double)) return LS2_ERR_ARG;
    double* partial = static_cast<double*>(workspace);
    hipLaunchKernelGGL(k_feature_loss, dim3(nb), dim3(256), 0, stream, m, D, feat, target, d_feat, partial);
    LS2_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_feature_loss_final, dim3(1), dim3(64), 0, stream, partial, nb, m, D, loss);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}
