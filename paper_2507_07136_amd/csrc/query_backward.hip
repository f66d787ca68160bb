// ls2_query_backward: gradient of the relevancy score with respect to the
// feature map.  The score (the LERF relevancy the method follows for
// open-vocabulary queries, Section 3.2) is
//   r = min_j sigmoid(tau (s_q - s_j)) = sigmoid(tau (s_q - s_j*)),
// with s = cos(F, e) and j* the first negative of largest similarity, so
//   dF = d_r tau r (1 - r) (ds_q/dF - ds_j*/dF),
//   ds/dF = e / (|F|_g |e|_g) - [|F| > eps] (F.e) F / (|F|^3 |e|_g),
// where |x|_g = max(|x|, 1e-12).
//
// One wave per feature row: each lane holds D/64 features as float4s, the
// 2 + n_neg dot products are reduced across the wave, the text vectors and
// their norms sit in LDS for the workgroup's lifetime.
#include "ls2_internal.h"

namespace ls2 {

constexpr int kQbMaxNeg = 8;
constexpr int kQbMaxV = 4;  // float4s per lane: D <= 1024

template <bool BF16>
__global__ __launch_bounds__(256) void k_query_backward(long long m, int D, const void* __restrict__ feat,
                                                        const float* __restrict__ pos, int n_neg,
                                                        const float* __restrict__ neg, float tau,
                                                        const float* __restrict__ d_rel,
                                                        float* __restrict__ d_feat) {
    __shared__ float4 text4[(1 + kQbMaxNeg) * 256];
    __shared__ float tnorm[1 + kQbMaxNeg];
    float* text = reinterpret_cast<float*>(text4);
    const int nt = 1 + n_neg;
    for (int i = threadIdx.x; i < nt * D; i += blockDim.x) {
        const int t = i / D, d = i - t * D;
        text[t * D + d] = t == 0 ? pos[d] : neg[(size_t)(t - 1) * D + d];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave == 0) {
        for (int t = 0; t < nt; ++t) {
            float s = 0.f;
            for (int d = lane; d < D; d += 64) s = fmaf(text[t * D + d], text[t * D + d], s);
            s = wave_allsum(s);
            if (lane == 0) tnorm[t] = fmaxf(sqrtf(s), 1e-12f);
        }
    }
    __syncthreads();
    const int nv4 = D / 4;
    const long long wstride = (long long)gridDim.x * (blockDim.x >> 6);
    for (long long row = (long long)blockIdx.x * (blockDim.x >> 6) + wave; row < m; row += wstride) {
        float4 f[kQbMaxV];
#pragma unroll
        for (int q = 0; q < kQbMaxV; ++q) {
            const int v = lane + 64 * q;
            f[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (v < nv4) {
                if (BF16) {
                    const uint2 raw = reinterpret_cast<const uint2*>(static_cast<const unsigned short*>(feat) +
                                                                     row * D)[v];
                    f[q] = make_float4(__uint_as_float(raw.x << 16), __uint_as_float(raw.x & 0xffff0000u),
                                       __uint_as_float(raw.y << 16), __uint_as_float(raw.y & 0xffff0000u));
                } else {
                    f[q] = reinterpret_cast<const float4*>(static_cast<const float*>(feat) + row * D)[v];
                }
            }
        }
        float ff = 0.f;
        float dots[1 + kQbMaxNeg];
#pragma unroll
        for (int t = 0; t < 1 + kQbMaxNeg; ++t) dots[t] = 0.f;
#pragma unroll
        for (int q = 0; q < kQbMaxV; ++q) {
            const int v = lane + 64 * q;
            if (v < nv4) {
                ff = fmaf(f[q].x, f[q].x, fmaf(f[q].y, f[q].y, fmaf(f[q].z, f[q].z, fmaf(f[q].w, f[q].w, ff))));
#pragma unroll
                for (int t = 0; t < 1 + kQbMaxNeg; ++t) {
                    if (t < nt) {
                        const float4 e = text4[t * nv4 + v];
                        dots[t] = fmaf(f[q].x, e.x, fmaf(f[q].y, e.y, fmaf(f[q].z, e.z, fmaf(f[q].w, e.w, dots[t]))));
                    }
                }
            }
        }
        ff = wave_allsum(ff);
#pragma unroll
        for (int t = 0; t < 1 + kQbMaxNeg; ++t)
            if (t < nt) dots[t] = wave_allsum(dots[t]);
        const float nf = sqrtf(ff);
        const float gf = fmaxf(nf, 1e-12f);
        const float sq = dots[0] / (gf * tnorm[0]);
        int js = 0;
        float smax = -INFINITY;
#pragma unroll
        for (int t = 1; t < 1 + kQbMaxNeg; ++t) {
            if (t < nt) {
                const float sj = dots[t] / (gf * tnorm[t]);
                if (sj > smax) {
                    smax = sj;
                    js = t;
                }
            }
        }
        float fej = 0.f, tnj = 1.f;
#pragma unroll
        for (int t = 1; t < 1 + kQbMaxNeg; ++t)
            if (t == js) {
                fej = dots[t];
                tnj = tnorm[t];
            }
        const float r = 1.0f / (1.0f + expf(-tau * (sq - smax)));
        const float dr = d_rel[row] * tau * r * (1.0f - r);
        // ds/dF = a e + b F for s = F.e / (|F|_g |e|_g)
        const float aq = dr / (gf * tnorm[0]), aj = dr / (gf * tnj);
        const float inv3 = nf > 1e-12f ? 1.0f / (nf * nf * nf) : 0.0f;
        const float bcoef = dr * inv3 * (fej / tnj - dots[0] / tnorm[0]);  // b_q - b_j, times dr
#pragma unroll
        for (int q = 0; q < kQbMaxV; ++q) {
            const int v = lane + 64 * q;
            if (v < nv4) {
                const float4 eq = text4[v], ej = text4[js * nv4 + v];
                float4 o;
                o.x = aq * eq.x - aj * ej.x + bcoef * f[q].x;
                o.y = aq * eq.y - aj * ej.y + bcoef * f[q].y;
                o.z = aq * eq.z - aj * ej.z + bcoef * f[q].z;
                o.w = aq * eq.w - aj * ej.w + bcoef * f[q].w;
                reinterpret_cast<float4*>(d_feat + row * D)[v] = o;
            }
        }
    }
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_query_backward(int64_t m, int32_t D, const void* feat, int32_t feat_dtype, const float* pos,
                                  int32_t n_neg, const float* neg, float tau, const float* d_rel, float* d_feat,
                                  hipStream_t stream) {
    if (m < 0 || D < 1 || n_neg < 1 || !pos || !neg || !(tau > 0.0f)) return LS2_ERR_ARG;
    if (feat_dtype != LS2_F32 && feat_dtype != LS2_BF16) return LS2_ERR_ARG;
    if (m > 0 && (!feat || !d_rel || !d_feat)) return LS2_ERR_ARG;
    if (D % 64 != 0 || D > 1024 || n_neg > kQbMaxNeg) return LS2_ERR_UNSUPPORTED;
    if (m == 0) return LS2_OK;
    long long blocks = (m + 3) / 4;
    if (blocks > 4096) blocks = 4096;
    if (feat_dtype == LS2_BF16)
        hipLaunchKernelGGL(k_query_backward<true>, dim3((unsigned)blocks), dim3(256), 0, stream, m, D, feat, pos,
                           n_neg, neg, tau, d_rel, d_feat);
    else
        hipLaunchKernelGGL(k_query_backward<false>, dim3((unsigned)blocks), dim3(256), 0, stream, m, D, feat, pos,
                           n_neg, neg, tau, d_rel, d_feat);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}
