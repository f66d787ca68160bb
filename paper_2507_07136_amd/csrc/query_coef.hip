// ls2_query_coef: the relevancy of ls2_query evaluated directly on the
// coefficient map.  By Eq. 7 the feature of a pixel is F = W S, so for any
// text embedding e
//     F . e   = W . (S e)            (an L-term dot product),
//     |F|^2   = W^T (S S^T) W        (an L x L quadratic form),
// and the cosine similarities, hence the LERF relevancy
// sigmoid(tau (s_q - max_j s_j)) (Section 3.2), follow without forming the
// D-dimensional feature map: the pass reads 4 L bytes per pixel instead of
// 2-4 D, and the feature map never has to exist.
//
// k_qc_prep (one workgroup per codebook row) forms S e_t for the positive and
// negative embeddings, the Gram matrix G = S S^T and the embedding norms in a
// small workspace.  For L <= 64 the quadratic form runs on the matrix cores
// (k_qc_mfma); for L = 128, k_qc_main gives each lane one pixel: its L
// coefficients in registers, G and the projected embeddings broadcast from
// LDS.
#include "ls2_internal.h"

namespace ls2 {

constexpr int kQcMaxText = 9;  // 1 positive + up to 8 negatives

struct QcLayout {
    int L, nt;
    size_t proj, norms, gram, total;  // float offsets
};

__host__ __device__ inline QcLayout qc_layout(int L, int nt) {
    QcLayout q;
    q.L = L;
    q.nt = nt;
    q.proj = 0;                           // [nt][L]: S e_t
    q.norms = q.proj + (size_t)nt * L;    // [16]: |e_t|
    q.gram = q.norms + 16;                // [L][L]
    q.total = q.gram + (size_t)L * L;
    return q;
}

// One workgroup per codebook row i, four waves: each wave forms some of the
// dot products of row i (with every row j, and with every embedding) from
// coalesced loads and a wave reduction.
__global__ __launch_bounds__(256) void k_qc_prep(int L, int D, const float* __restrict__ dict,
                                                 const float* __restrict__ pos, int n_neg,
                                                 const float* __restrict__ neg, float* __restrict__ ws) {
    const QcLayout q = qc_layout(L, 1 + n_neg);
    const int i = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float* si = dict + (size_t)i * D;
    // rows j = 0 .. L-1, then embeddings t = 0 .. nt-1, spread over the waves
    for (int job = wave; job < L + q.nt; job += 4) {
        const float* v = job < L ? dict + (size_t)job * D
                                 : (job == L ? pos : neg + (size_t)(job - L - 1) * D);
        float acc = 0.0f, ee = 0.0f;
        for (int d = lane; d < D; d += 64) {
            acc = fmaf(si[d], v[d], acc);
            ee = fmaf(v[d], v[d], ee);
        }
        acc = wave_allsum(acc);
        if (job < L) {
            if (lane == 0) ws[q.gram + (size_t)i * L + job] = acc;
        } else {
            const int t = job - L;
            if (lane == 0) ws[q.proj + (size_t)t * L + i] = acc;
            if (i == 0) {
                ee = wave_allsum(ee);
                if (lane == 0) ws[q.norms + t] = fmaxf(sqrtf(ee), 1e-12f);
            }
        }
    }
}

template <int L>
__global__ __launch_bounds__(256) void k_qc_main(long long m, const float* __restrict__ coef, int n_neg,
                                                 const float* __restrict__ ws, float tau,
                                                 float* __restrict__ out) {
    __shared__ float4 sh4[(L * L + kQcMaxText * L + 16) / 4];
    float* sh = reinterpret_cast<float*>(sh4);
    const QcLayout q = qc_layout(L, 1 + n_neg);
    // LDS: G [L][L], then the projections [nt][L], then the norms
    float* G = sh;
    float* P = sh + L * L;
    float* N = P + kQcMaxText * L;
    for (int i = threadIdx.x; i < L * L; i += blockDim.x) G[i] = ws[q.gram + i];
    for (int i = threadIdx.x; i < q.nt * L; i += blockDim.x) P[i] = ws[q.proj + i];
    if (threadIdx.x < q.nt) N[threadIdx.x] = ws[q.norms + threadIdx.x];
    __syncthreads();
    const float4* G4 = reinterpret_cast<const float4*>(G);
    const float4* P4 = reinterpret_cast<const float4*>(P);
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < m;
         p += (long long)gridDim.x * blockDim.x) {
        float w[L];
        const float4* src = reinterpret_cast<const float4*>(coef + p * L);
#pragma unroll
        for (int c = 0; c < L / 4; ++c) {
            const float4 v = src[c];
            w[4 * c] = v.x; w[4 * c + 1] = v.y; w[4 * c + 2] = v.z; w[4 * c + 3] = v.w;
        }
        // |F|^2 = sum_j w_j (G w)_j: a runtime loop over the rows of G (LDS
        // broadcasts), each row dotted with the register-resident w; w_j
        // itself is re-read from the (cached) coefficient row
        float nn = 0.0f;
        const float* wrow = coef + p * L;
        for (int j = 0; j < L; ++j) {
            float u = 0.0f;
#pragma unroll
            for (int c = 0; c < L / 4; ++c) {
                const float4 g = G4[j * (L / 4) + c];
                u = fmaf(g.x, w[4 * c], fmaf(g.y, w[4 * c + 1], fmaf(g.z, w[4 * c + 2], fmaf(g.w, w[4 * c + 3], u))));
            }
            nn = fmaf(wrow[j], u, nn);
        }
        const float nf = sqrtf(fmaxf(nn, 0.0f));
        const float gf = fmaxf(nf, 1e-12f);
        float sq = 0.0f, smax = -INFINITY;
        for (int t = 0; t < q.nt; ++t) {
            float dot = 0.0f;
#pragma unroll
            for (int c = 0; c < L / 4; ++c) {
                const float4 e = P4[(t * L) / 4 + c];
                dot = fmaf(w[4 * c], e.x, fmaf(w[4 * c + 1], e.y, fmaf(w[4 * c + 2], e.z, fmaf(w[4 * c + 3], e.w, dot))));
            }
            const float s = dot / (gf * N[t]);
            if (t == 0) sq = s;
            else smax = fmaxf(smax, s);
        }
        out[p] = 1.0f / (1.0f + expf(-tau * (sq - smax)));
    }
}

// Matrix-core form for L <= 64: per 32-pixel block a wave forms
// T = G W^T [L x 32] with v_mfma_f32_32x32x2_f32 (A = G rows, lane l: row
// l%32, k = l/32; B = W^T, lane l: pixel l%32; the reduction index is
// permuted so half h covers k in [h L/2, (h+1) L/2), i.e. each lane reads
// its pixel's coefficients as contiguous float4s).  The lane then holds T for
// rows 8 g + 4 h + i of its pixel, multiplies by the matching coefficients
// and the two lane halves are added: |F|^2 = sum_L W_L T_L.  G's operands stay
// in VGPRs for the whole kernel.
typedef float f32x16q __attribute__((ext_vector_type(16)));

template <int L>
__global__ __launch_bounds__(256) void k_qc_mfma(long long m, const float* __restrict__ coef, int n_neg,
                                                 const float* __restrict__ ws, float tau,
                                                 float* __restrict__ out) {
    constexpr int TL = L / 32, KS = L / 2;
    __shared__ float P[kQcMaxText * L];
    __shared__ float N[16];
    const QcLayout q = qc_layout(L, 1 + n_neg);
    for (int i = threadIdx.x; i < q.nt * L; i += blockDim.x) P[i] = ws[q.proj + i];
    if (threadIdx.x < q.nt) N[threadIdx.x] = ws[q.norms + threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, col = lane & 31, half = lane >> 5;
    float ga[TL][KS];
#pragma unroll
    for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int s = 0; s < KS; ++s) ga[tl][s] = ws[q.gram + (size_t)(32 * tl + col) * L + half * KS + s];
    const long long nblk = (m + 31) / 32;
    const long long wstride = (long long)gridDim.x * (blockDim.x >> 6);
    for (long long blk = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); blk < nblk;
         blk += wstride) {
        const long long p = blk * 32 + col;
        const bool valid = p < m;
        const float* row = coef + (valid ? p : m - 1) * L;
        float wv[KS];
#pragma unroll
        for (int c = 0; c < KS / 4; ++c) {
            const float4 v = reinterpret_cast<const float4*>(row + half * KS)[c];
            wv[4 * c] = v.x; wv[4 * c + 1] = v.y; wv[4 * c + 2] = v.z; wv[4 * c + 3] = v.w;
        }
        f32x16q acc[TL];
#pragma unroll
        for (int tl = 0; tl < TL; ++tl) {
            acc[tl] = (f32x16q){};
#pragma unroll
            for (int s = 0; s < KS; ++s) acc[tl] = __builtin_amdgcn_mfma_f32_32x32x2f32(ga[tl][s], wv[s], acc[tl], 0, 0, 0);
        }
        float part = 0.0f;
#pragma unroll
        for (int tl = 0; tl < TL; ++tl)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const float4 w4 = reinterpret_cast<const float4*>(row + 32 * tl + 8 * g + 4 * half)[0];
                part = fmaf(acc[tl][4 * g], w4.x, fmaf(acc[tl][4 * g + 1], w4.y,
                            fmaf(acc[tl][4 * g + 2], w4.z, fmaf(acc[tl][4 * g + 3], w4.w, part))));
            }
        const float nn = part + __shfl_xor(part, 32);
        const float gf = fmaxf(sqrtf(fmaxf(nn, 0.0f)), 1e-12f);
        float sq = 0.0f, smax = -INFINITY;
        for (int t = 0; t < q.nt; ++t) {
            const float* pt = P + t * L + half * KS;
            float d = 0.0f;
#pragma unroll
            for (int s = 0; s < KS; ++s) d = fmaf(wv[s], pt[s], d);
            d += __shfl_xor(d, 32);
            const float sv = d / (gf * N[t]);
            if (t == 0) sq = sv;
            else smax = fmaxf(smax, sv);
        }
        if (valid && half == 0) out[p] = 1.0f / (1.0f + expf(-tau * (sq - smax)));
    }
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_query_coef_workspace(int32_t L, int32_t n_neg, size_t* bytes) {
    if (!bytes || L < 1 || n_neg < 1) return LS2_ERR_ARG;
    if (!(L == 32 || L == 64 || L == 128) || n_neg > kQcMaxText - 1) return LS2_ERR_UNSUPPORTED;
    *bytes = qc_layout(L, 1 + n_neg).total * sizeof(float);
    return LS2_OK;
}

extern "C" int ls2_query_coef(int64_t m, int32_t L, int32_t D, const float* coef, const float* dict,
                              const float* pos, int32_t n_neg, const float* neg, float tau, float* relevancy,
                              void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (m < 0 || L < 1 || D < 1 || n_neg < 1 || !dict || !pos || !neg || !(tau > 0.0f) || !workspace)
        return LS2_ERR_ARG;
    if (m > 0 && (!coef || !relevancy)) return LS2_ERR_ARG;
    if (!(L == 32 || L == 64 || L == 128) || n_neg > kQcMaxText - 1) return LS2_ERR_UNSUPPORTED;
    const QcLayout q = qc_layout(L, 1 + n_neg);
    if (workspace_bytes < q.total * sizeof(float)) return LS2_ERR_ARG;
    float* ws = static_cast<float*>(workspace);
    hipLaunchKernelGGL(k_qc_prep, dim3(L), dim3(256), 0, stream, L, D, dict, pos, n_neg, neg, ws);
    LS2_LAUNCH_CHECK();
    if (m == 0) return LS2_OK;
    if (L <= 64) {
        // 4 waves per workgroup, one 32-pixel block per wave and step
        long long blocks = ((m + 31) / 32 + 3) / 4;
        if (blocks > 2048) blocks = 2048;
        if (L == 32)
            hipLaunchKernelGGL(k_qc_mfma<32>, dim3((unsigned)blocks), dim3(256), 0, stream, m, coef, n_neg, ws, tau,
                               relevancy);
        else
            hipLaunchKernelGGL(k_qc_mfma<64>, dim3((unsigned)blocks), dim3(256), 0, stream, m, coef, n_neg, ws, tau,
                               relevancy);
    } else {
        long long blocks = (m + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_qc_main<128>, dim3((unsigned)blocks), dim3(256), 0, stream, m, coef, n_neg, ws, tau,
                           relevancy);
    }
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}
