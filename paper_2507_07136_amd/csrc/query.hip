// ls2_query: LERF relevancy (followed by Section 3.2) per feature row:
//   r = min_j exp(tau s_q) / (exp(tau s_q) + exp(tau s_j)) = sigmoid(tau (s_q - max_j s_j))
// with cosine similarities against one positive and n_neg canonical negative
// text embeddings.
//
// The feature map is read once (HBM-bound).  Each wave scores 16 rows at a
// time: the dot products with the text embeddings run on the matrix cores
// (rows x D times D x 16 text columns, unused columns zero), so every lane
// loads 16 contiguous bytes of one row per step and no cross-lane reductions
// are needed for the dots.  Squared norms come from the diagonal of F F^T
// (bf16 input, one more MFMA on the same registers) or from a per-lane FMA
// chain (f32 input).
#include "ls2_internal.h"

namespace ls2 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct QueryArgs {
    long long m;
    int D, ntext;  // ntext = 1 + n_neg
    const void* feat;
    const float* pos;   // [D]
    const float* neg;   // [ntext - 1, D]
    float tau;
    float* out;
    long long nblocks;  // 16-row blocks
};

constexpr int kQWaves = 4;

// Orders this wave's LDS writes before its subsequent LDS reads (the waves of
// the workgroup iterate independently, so no workgroup barrier is used).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS: text rows (f32 or bf16, padded), text norms, per-wave dot tiles.
template <bool BF16>
__global__ __launch_bounds__(kQWaves * 64) void k_query(QueryArgs a) {
    extern __shared__ float4 smem4[];
    char* smem = reinterpret_cast<char*>(smem4);
    const int D = a.D, ntext = a.ntext;
    const int tstride = BF16 ? (D + 8) * 2 : (D + 4) * 4;  // bytes per padded text row
    char* text_s = smem;
    float* tnorm_s = reinterpret_cast<float*>(smem + ntext * tstride);
    float* dots_s = tnorm_s + 16;                    // [waves][16 rows][17]
    float* nrm_s = dots_s + kQWaves * 16 * 17;       // [waves][4][16]

    // stage text (rounded to bf16 for the bf16 path) and its float32 norms
    for (int i = threadIdx.x; i < ntext * D; i += blockDim.x) {
        const int j = i / D, d = i - j * D;
        const float v = j == 0 ? a.pos[d] : a.neg[(size_t)(j - 1) * D + d];
        if (BF16) reinterpret_cast<__bf16*>(text_s + j * tstride)[d] = (__bf16)v;
        else reinterpret_cast<float*>(text_s + j * tstride)[d] = v;
    }
    if (threadIdx.x < 64) {
        for (int j = 0; j < ntext; ++j) {
            float s = 0.f;
            const float* t = j == 0 ? a.pos : a.neg + (size_t)(j - 1) * D;
            for (int d = threadIdx.x; d < D; d += 64) s += t[d] * t[d];
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            if (threadIdx.x == 0) tnorm_s[j] = fmaxf(sqrtf(s), 1e-12f);
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const bool tcol = r16 < ntext;
    float* dots_w = dots_s + wave * 16 * 17;
    float* nrm_w = nrm_s + wave * 64;

    for (long long blk = (long long)blockIdx.x * kQWaves + wave; blk < a.nblocks;
         blk += (long long)gridDim.x * kQWaves) {
        const long long p = blk * 16 + r16;
        const bool valid = p < a.m;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        float nrm = 0.f;
        if (BF16) {
            f32x4 gram = {0.f, 0.f, 0.f, 0.f};
            const bf16x8* row = reinterpret_cast<const bf16x8*>(reinterpret_cast<const __bf16*>(a.feat) + p * D);
            const bf16x8 zero8 = {};
            for (int ks = 0; ks < D / 32; ++ks) {
                const bf16x8 fa = valid ? row[ks * 4 + g] : zero8;
                const bf16x8 tb = tcol ? *reinterpret_cast<const bf16x8*>(text_s + r16 * tstride + (ks * 32 + g * 8) * 2)
                                       : zero8;
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, tb, acc, 0, 0, 0);
                gram = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fa, gram, 0, 0, 0);
            }
            // diagonal of the Gram tile: row (g*4 + i) == column r16
            const int i = r16 - g * 4;
            if (i >= 0 && i < 4) nrm_w[r16] = gram[i];
        } else {
            const float4* row = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(a.feat) + p * D);
            const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
            for (int k4 = 0; k4 < D / 16; ++k4) {
                const float4 fa = valid ? row[k4 * 4 + g] : z4;
                const float4 tb = tcol ? *reinterpret_cast<const float4*>(text_s + r16 * tstride + (k4 * 16 + g * 4) * 4)
                                       : z4;
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.x, tb.x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.y, tb.y, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.z, tb.z, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.w, tb.w, acc, 0, 0, 0);
                nrm = fmaf(fa.x, fa.x, nrm);
                nrm = fmaf(fa.y, fa.y, nrm);
                nrm = fmaf(fa.z, fa.z, nrm);
                nrm = fmaf(fa.w, fa.w, nrm);
            }
            nrm_w[g * 16 + r16] = nrm;
        }
        // dots: lane holds text column r16, rows g*4 + i
#pragma unroll
        for (int i = 0; i < 4; ++i) dots_w[(g * 4 + i) * 17 + r16] = acc[i];
        wave_lds_sync();
        if (lane < 16) {
            const long long q = blk * 16 + lane;
            if (q < a.m) {
                const float n2 = BF16 ? nrm_w[lane]
                                      : (nrm_w[lane] + nrm_w[16 + lane]) + (nrm_w[32 + lane] + nrm_w[48 + lane]);
                a.out[q] = lerf_relevancy(dots_w + lane * 17, n2, tnorm_s, ntext, a.tau);
            }
        }
        wave_lds_sync();
    }
}

static int num_cus_q() {
    static int n = 0;
    if (n == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        n = v;
    }
    return n;
}

template <bool BF16>
static int launch_query(const QueryArgs& a, hipStream_t stream) {
    const int tstride = BF16 ? (a.D + 8) * 2 : (a.D + 4) * 4;
    const size_t lds = (size_t)a.ntext * tstride + sizeof(float) * (16 + kQWaves * 16 * 17 + kQWaves * 64);
    long long grid = (long long)num_cus_q() * 4;
    const long long need = (a.nblocks + kQWaves - 1) / kQWaves;
    if (grid > need) grid = need;
    hipLaunchKernelGGL((k_query<BF16>), dim3((unsigned)grid), dim3(kQWaves * 64), lds, stream, a);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_query(int64_t m, int32_t D, const void* feat, int32_t feat_dtype, const float* pos, int32_t n_neg,
                         const float* neg, float tau, float* relevancy, hipStream_t stream) {
    if (m < 0 || D < 1 || n_neg < 1 || !feat || !pos || !neg || !relevancy) return LS2_ERR_ARG;
    if (feat_dtype != LS2_F32 && feat_dtype != LS2_BF16) return LS2_ERR_ARG;
    if (D % 64 != 0 || D > 1024 || n_neg > 8) return LS2_ERR_UNSUPPORTED;
    if (m == 0) return LS2_OK;
    QueryArgs a;
    a.m = m;
    a.D = D;
    a.ntext = 1 + n_neg;
    a.feat = feat;
    a.pos = pos;
    a.neg = neg;
    a.tau = tau;
    a.out = relevancy;
    a.nblocks = (m + 15) / 16;
    return feat_dtype == LS2_BF16 ? launch_query<true>(a, stream) : launch_query<false>(a, stream);
}
