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
// One wave per row.  The row sums are accumulated in compensated float32
// (CSum); each workgroup writes its partial sums to the workspace and a
// one-workgroup kernel adds them in a fixed order, so the loss is
// deterministic.  Only the final scalar is widened to double.
#include "ls2_internal.h"

namespace ls2 {

constexpr int kLossBlocks = 2048;
constexpr int kLossMaxV = 4;  // float4s per lane: D <= 1024

__device__ __forceinline__ float sgn(float e) { return e > 0.f ? 1.f : (e < 0.f ? -1.f : 0.f); }

__global__ __launch_bounds__(256) void k_feature_loss(long long m, int D, float inv_md, float inv_m,
                                                      const float* __restrict__ F, const float* __restrict__ Y,
                                                      float* __restrict__ dF, CSum* __restrict__ partial) {
    __shared__ CSum red[2][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nv4 = D / 4;
    CSum l1_acc{}, lc_acc{};
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
        l1_acc.add(l1);
        lc_acc.add(1.0f - c);
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
        CSum a = red[0][0], b = red[1][0];
        for (int w = 1; w < 4; ++w) {
            a.add(red[0][w]);
            b.add(red[1][w]);
        }
        partial[2 * blockIdx.x] = a;
        partial[2 * blockIdx.x + 1] = b;
    }
}

// Adds the per-workgroup partials of the two loss terms in a fixed order
// (lane t the partials t, t + 64, ..., then lane 0 the 64 lane sums), so the
// loss is reproducible, and writes mean |F - Y| + mean (1 - cos).
__global__ __launch_bounds__(64) void k_loss_final(const CSum* __restrict__ partial, int nblocks, float inv_md,
                                                   float inv_m, double* __restrict__ loss) {
    __shared__ CSum s[2][64];
    const int t = threadIdx.x;
    CSum l1{}, lc{};
    for (int b = t; b < nblocks; b += 64) {
        l1.add(partial[2 * b]);
        lc.add(partial[2 * b + 1]);
    }
    s[0][t] = l1;
    s[1][t] = lc;
    __syncthreads();
    if (t == 0) {
        CSum a{}, c{};
        for (int k = 0; k < 64; ++k) {
            a.add(s[0][k]);
            c.add(s[1][k]);
        }
        *loss = (double)(a.value() * inv_md + c.value() * inv_m);
    }
}

int launch_loss_final(const CSum* partial, int nblocks, long long m, int D, double* loss, hipStream_t stream) {
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, stream, partial, nblocks, loss_inv_md(m, D),
                       loss_inv_m(m), loss);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}

static int loss_blocks(long long m) {
    const long long b = (m + 3) / 4;
    return (int)(b < kLossBlocks ? (b < 1 ? 1 : b) : kLossBlocks);
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_feature_loss_workspace(int64_t m, size_t* bytes) {
    if (!bytes || m < 0) return LS2_ERR_ARG;
    *bytes = (size_t)loss_blocks(m) * 2 * sizeof(CSum);
    return LS2_OK;
}

extern "C" int ls2_feature_loss(int64_t m, int32_t D, const float* feat, const float* target, double* loss,
                                float* d_feat, void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (m < 1 || D < 1 || !feat || !target || !loss || !workspace) return LS2_ERR_ARG;
    if (D % 64 != 0 || D > 1024) return LS2_ERR_UNSUPPORTED;
    const int nb = loss_blocks(m);
    if (workspace_bytes < (size_t)nb * 2 * sizeof(CSum)) return LS2_ERR_ARG;
    CSum* partial = static_cast<CSum*>(workspace);
    hipLaunchKernelGGL(k_feature_loss, dim3(nb), dim3(256), 0, stream, m, D, loss_inv_md(m, D), loss_inv_m(m),
                       feat, target, d_feat, partial);
    LS2_LAUNCH_CHECK();
    return launch_loss_final(partial, nb, m, D, loss, stream);
}
