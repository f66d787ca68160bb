// ls2_sparse_codes / ls2_sparse_codes_backward: the sparse coefficient
// parametrisation of Section 3.3 -- a Gaussian's L-dimensional parameter is
// normalised by a softmax, its K largest values are kept and renormalised.
// All softmax values share one denominator, so the kept weights are the
// softmax of the K kept logits; the backward treats the selection as fixed:
// dz_j = w_j (dw_j - sum_k w_k dw_k) for kept j, 0 for the others.
//
// One thread per row (a Gaussian's level): the row is read as float4s and the
// K largest logits are kept in a register list sorted by (value descending,
// index ascending).
#include "ls2_internal.h"

namespace ls2 {

template <int KMAX>
__global__ __launch_bounds__(256) void k_sparse_codes(long long rows, int L, int K, const float* __restrict__ z,
                                                      int* __restrict__ idx, float* __restrict__ w) {
    const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (r >= rows) return;
    float tv[KMAX];
    int ti[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        tv[k] = -INFINITY;
        ti[k] = 0x7fffffff;
    }
    const float4* row = reinterpret_cast<const float4*>(z + r * L);
    for (int q = 0; q < L / 4; ++q) {
        const float4 v4 = row[q];
        const float vs[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float v = vs[e];
            int i = 4 * q + e;
            // insert (v, i) into the sorted list; later indices lose ties
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                if (k < K && (v > tv[k] || (v == tv[k] && i < ti[k]))) {
                    const float sv = tv[k];
                    const int si = ti[k];
                    tv[k] = v;
                    ti[k] = i;
                    v = sv;
                    i = si;
                }
            }
        }
    }
    float s = 0.0f, e[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        e[k] = k < K ? expf(tv[k] - tv[0]) : 0.0f;
        s += e[k];
    }
    const float inv = 1.0f / s;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k < K) {
            idx[r * K + k] = ti[k];
            w[r * K + k] = e[k] * inv;
        }
    }
}

__global__ __launch_bounds__(256) void k_sparse_codes_backward(long long rows, int L, int K, const int* __restrict__ idx,
                                                               const float* __restrict__ w,
                                                               const float* __restrict__ dw,
                                                               float* __restrict__ dz) {
    const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (r >= rows) return;
    float s = 0.0f;
    for (int k = 0; k < K; ++k) s = fmaf(w[r * K + k], dw[r * K + k], s);
    float4* out = reinterpret_cast<float4*>(dz + r * L);
    for (int q = 0; q < L / 4; ++q) out[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int k = 0; k < K; ++k) {
        const int j = idx[r * K + k];
        if (j >= 0 && j < L) dz[r * L + j] = w[r * K + k] * (dw[r * K + k] - s);
    }
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_sparse_codes(int64_t rows, int32_t L, int32_t K, const float* logits, int32_t* topk_idx,
                                float* topk_w, hipStream_t stream) {
    if (rows < 0 || L < 1 || K < 1 || K > L) return LS2_ERR_ARG;
    if (rows > 0 && (!logits || !topk_idx || !topk_w)) return LS2_ERR_ARG;
    if (L % 4 != 0 || L > 1024 || K > 8) return LS2_ERR_UNSUPPORTED;
    if (rows == 0) return LS2_OK;
    const unsigned blocks = (unsigned)((rows + 255) / 256);
    if (K <= 4)
        hipLaunchKernelGGL(k_sparse_codes<4>, dim3(blocks), dim3(256), 0, stream, rows, L, K, logits, topk_idx, topk_w);
    else
        hipLaunchKernelGGL(k_sparse_codes<8>, dim3(blocks), dim3(256), 0, stream, rows, L, K, logits, topk_idx, topk_w);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}

extern "C" int ls2_sparse_codes_backward(int64_t rows, int32_t L, int32_t K, const int32_t* topk_idx,
                                         const float* topk_w, const float* d_topk_w, float* d_logits,
                                         hipStream_t stream) {
    if (rows < 0 || L < 1 || K < 1 || K > L) return LS2_ERR_ARG;
    if (rows > 0 && (!topk_idx || !topk_w || !d_topk_w || !d_logits)) return LS2_ERR_ARG;
    if (L % 4 != 0 || L > 1024 || K > 8) return LS2_ERR_UNSUPPORTED;
    if (rows == 0) return LS2_OK;
    const unsigned blocks = (unsigned)((rows + 255) / 256);
    hipLaunchKernelGGL(k_sparse_codes_backward, dim3(blocks), dim3(256), 0, stream, rows, L, K, topk_idx, topk_w,
                       d_topk_w, d_logits);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}
