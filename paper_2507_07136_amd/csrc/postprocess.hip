// ls2_postprocess: the relevancy post-processing stage (Section 3.2: a mean
// filter over each level's relevancy map, then the selection of one level; the
// evaluation appendix gives the localization point as the argmax of the
// smoothed map, the segmentation mask as the normalised smoothed map above a
// threshold, the blend 0.5 (M + Avg(M)) used on some datasets, and the two
// level-selection rules).
//
//   k_pp_rows, k_pp_cols  separable k x k box mean over the window clipped to
//                         the image (then the optional blend with M);
//   k_pp_minmax(+final)   per level max (first index on ties) and min, block
//                         partials reduced in a fixed order;
//   k_pp_maskstats(+final) per level sum and count of the smoothed values
//                         whose normalised value exceeds the threshold, and
//                         the level selection;
//   k_pp_mask             the selected level's mask.
// Every reduction runs in a fixed order, so results are reproducible.
#include "ls2_internal.h"

namespace ls2 {

constexpr int kPpBlocks = 256;
constexpr int kPpMaxLevels = 8;

struct PpLayout {
    size_t tmp, pmax, parg, pmin, psum, pcnt, stats, total;  // bytes
};

inline PpLayout pp_layout(int levels, int H, int W) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    PpLayout l;
    size_t off = 0;
    l.tmp = off; off = al(off + sizeof(float) * (size_t)levels * H * W);
    l.pmax = off; off = al(off + sizeof(float) * kPpBlocks * levels);
    l.parg = off; off = al(off + sizeof(int) * kPpBlocks * levels);
    l.pmin = off; off = al(off + sizeof(float) * kPpBlocks * levels);
    l.psum = off; off = al(off + sizeof(CSum) * kPpBlocks * levels);
    l.pcnt = off; off = al(off + sizeof(int) * kPpBlocks * levels);
    l.stats = off; off = al(off + sizeof(float) * 4 * kPpMaxLevels + sizeof(int) * 2 * kPpMaxLevels);
    l.total = off;
    return l;
}

__global__ void k_pp_rows(int levels, int H, int W, int r, const float* __restrict__ M, float* __restrict__ tmp) {
    const long long n = (long long)levels * H * W;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % W);
        const long long row = i - x;
        const int x0 = max(0, x - r), x1 = min(W - 1, x + r);
        float s = 0.0f;
        for (int xx = x0; xx <= x1; ++xx) s += M[row + xx];
        tmp[i] = s;
    }
}

__global__ void k_pp_cols(int levels, int H, int W, int r, int mode, const float* __restrict__ M,
                          const float* __restrict__ tmp, float* __restrict__ S) {
    const long long n = (long long)levels * H * W;
    const long long HW = (long long)H * W;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long l = i / HW;
        const long long rem = i - l * HW;
        const int y = (int)(rem / W), x = (int)(rem - (long long)y * W);
        const int y0 = max(0, y - r), y1 = min(H - 1, y + r);
        const int x0 = max(0, x - r), x1 = min(W - 1, x + r);
        float s = 0.0f;
        for (int yy = y0; yy <= y1; ++yy) s += tmp[l * HW + (long long)yy * W + x];
        float v = s / (float)((y1 - y0 + 1) * (x1 - x0 + 1));
        if (mode == LS2_SMOOTH_HALF) v = 0.5f * (M[i] + v);
        S[i] = v;
    }
}

// (value, index) with the larger value winning and the smaller index on ties
__device__ __forceinline__ void better(float& v, int& i, float v2, int i2) {
    if (v2 > v || (v2 == v && i2 < i)) {
        v = v2;
        i = i2;
    }
}

__global__ __launch_bounds__(256) void k_pp_minmax(int levels, long long HW, const float* __restrict__ S,
                                                   float* __restrict__ pmax, int* __restrict__ parg,
                                                   float* __restrict__ pmin) {
    __shared__ float smax[4], smin[4];
    __shared__ int sarg[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int l = 0; l < levels; ++l) {
        const float* s = S + l * HW;
        float mx = -INFINITY, mn = INFINITY;
        int ai = 0x7fffffff;
        for (long long p = blockIdx.x * 256LL + threadIdx.x; p < HW; p += (long long)gridDim.x * 256) {
            const float v = s[p];
            better(mx, ai, v, (int)p);
            mn = fminf(mn, v);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float v2 = __shfl_xor(mx, off);
            const int i2 = __shfl_xor(ai, off);
            better(mx, ai, v2, i2);
            mn = fminf(mn, __shfl_xor(mn, off));
        }
        if (lane == 0) {
            smax[wave] = mx;
            sarg[wave] = ai;
            smin[wave] = mn;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < 4; ++w) {
                better(mx, ai, smax[w], sarg[w]);
                mn = fminf(mn, smin[w]);
            }
            pmax[l * gridDim.x + blockIdx.x] = mx;
            parg[l * gridDim.x + blockIdx.x] = ai;
            pmin[l * gridDim.x + blockIdx.x] = mn;
        }
        __syncthreads();
    }
}

// one thread per level: partials in block order
__global__ void k_pp_minmax_final(int levels, int nb, const float* __restrict__ pmax, const int* __restrict__ parg,
                                  const float* __restrict__ pmin, float* __restrict__ stats, int* __restrict__ sarg) {
    const int l = threadIdx.x;
    if (l >= levels) return;
    float mx = -INFINITY, mn = INFINITY;
    int ai = 0x7fffffff;
    for (int b = 0; b < nb; ++b) {
        better(mx, ai, pmax[l * nb + b], parg[l * nb + b]);
        mn = fminf(mn, pmin[l * nb + b]);
    }
    stats[4 * l] = mx;
    stats[4 * l + 1] = mn;
    sarg[l] = ai;
}

__device__ __forceinline__ bool in_mask(float s, float mn, float mx, float thr) {
    const float norm = mx > mn ? (s - mn) / (mx - mn) : 0.0f;
    return norm > thr;
}

__global__ __launch_bounds__(256) void k_pp_maskstats(int levels, long long HW, const float* __restrict__ S,
                                                      const float* __restrict__ stats, float thr,
                                                      CSum* __restrict__ psum, int* __restrict__ pcnt) {
    __shared__ CSum ssum[4];
    __shared__ int scnt[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int l = 0; l < levels; ++l) {
        const float* s = S + l * HW;
        const float mx = stats[4 * l], mn = stats[4 * l + 1];
        CSum sum{};
        int cnt = 0;
        for (long long p = blockIdx.x * 256LL + threadIdx.x; p < HW; p += (long long)gridDim.x * 256) {
            const float v = s[p];
            if (in_mask(v, mn, mx, thr)) {
                sum.add(v);
                ++cnt;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            CSum o;
            o.s = __shfl_xor(sum.s, off);
            o.c = __shfl_xor(sum.c, off);
            sum.add(o);
            cnt += __shfl_xor(cnt, off);
        }
        if (lane == 0) {
            ssum[wave] = sum;
            scnt[wave] = cnt;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            CSum t = ssum[0];
            for (int w = 1; w < 4; ++w) t.add(ssum[w]);
            psum[l * gridDim.x + blockIdx.x] = t;
            pcnt[l * gridDim.x + blockIdx.x] = scnt[0] + scnt[1] + scnt[2] + scnt[3];
        }
        __syncthreads();
    }
}

__global__ void k_pp_select(int levels, int nb, int W, int select_mode, const CSum* __restrict__ psum,
                            const int* __restrict__ pcnt, float* __restrict__ stats, const int* __restrict__ sarg,
                            int* __restrict__ sel, int32_t* __restrict__ result, float* __restrict__ level_stats) {
    if (threadIdx.x != 0) return;
    int best = 0;
    float bestv = -INFINITY;
    for (int l = 0; l < levels; ++l) {
        CSum sum{};
        long long cnt = 0;
        for (int b = 0; b < nb; ++b) {
            sum.add(psum[l * nb + b]);
            cnt += pcnt[l * nb + b];
        }
        stats[4 * l + 2] = cnt > 0 ? sum.value() / (float)cnt : -INFINITY;
        stats[4 * l + 3] = (float)cnt;
        const float key = select_mode == LS2_SELECT_MAX ? stats[4 * l] : stats[4 * l + 2];
        if (l == 0 || key > bestv) {
            bestv = key;
            best = l;
        }
        if (level_stats)
            for (int q = 0; q < 4; ++q) level_stats[4 * l + q] = stats[4 * l + q];
    }
    *sel = best;
    const int idx = sarg[best];
    result[0] = best;
    result[1] = idx % W;
    result[2] = idx / W;
    result[3] = idx;
}

__global__ void k_pp_mask(long long HW, const float* __restrict__ S, const float* __restrict__ stats,
                          const int* __restrict__ sel, float thr, uint8_t* __restrict__ mask) {
    const int l = *sel;
    const float mx = stats[4 * l], mn = stats[4 * l + 1];
    const float* s = S + l * HW;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < HW; p += (long long)gridDim.x * blockDim.x)
        mask[p] = in_mask(s[p], mn, mx, thr) ? 1 : 0;
}

static unsigned grid_for(long long n) {
    long long b = (n + 255) / 256;
    return (unsigned)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_postprocess_workspace(int32_t levels, int32_t H, int32_t W, size_t* bytes) {
    if (!bytes || levels < 1 || H < 1 || W < 1) return LS2_ERR_ARG;
    if (levels > kPpMaxLevels) return LS2_ERR_UNSUPPORTED;
    *bytes = pp_layout(levels, H, W).total;
    return LS2_OK;
}

extern "C" int ls2_postprocess(int32_t levels, int32_t H, int32_t W, const float* relevancy, int32_t kernel,
                               int32_t smooth_mode, int32_t select_mode, float threshold, float* smoothed,
                               uint8_t* mask, int32_t* result, float* level_stats, void* workspace,
                               size_t workspace_bytes, hipStream_t stream) {
    if (levels < 1 || H < 1 || W < 1 || !relevancy || !smoothed || !mask || !result || !workspace) return LS2_ERR_ARG;
    if (kernel < 1 || (kernel & 1) == 0) return LS2_ERR_ARG;
    if ((smooth_mode != LS2_SMOOTH_AVG && smooth_mode != LS2_SMOOTH_HALF) ||
        (select_mode != LS2_SELECT_MAX && select_mode != LS2_SELECT_MASK_MEAN) || !(threshold == threshold))
        return LS2_ERR_ARG;
    if (levels > kPpMaxLevels || (long long)H * W > 0x7fffffffLL) return LS2_ERR_UNSUPPORTED;
    const PpLayout lay = pp_layout(levels, H, W);
    if (workspace_bytes < lay.total || ((uintptr_t)workspace & 255) != 0) return LS2_ERR_ARG;
    char* ws = static_cast<char*>(workspace);
    float* tmp = reinterpret_cast<float*>(ws + lay.tmp);
    float* pmax = reinterpret_cast<float*>(ws + lay.pmax);
    int* parg = reinterpret_cast<int*>(ws + lay.parg);
    float* pmin = reinterpret_cast<float*>(ws + lay.pmin);
    CSum* psum = reinterpret_cast<CSum*>(ws + lay.psum);
    int* pcnt = reinterpret_cast<int*>(ws + lay.pcnt);
    float* stats = reinterpret_cast<float*>(ws + lay.stats);
    int* sarg = reinterpret_cast<int*>(stats + 4 * kPpMaxLevels);
    int* sel = sarg + kPpMaxLevels;
    const long long HW = (long long)H * W, n = (long long)levels * HW;
    const int r = kernel / 2;
    hipLaunchKernelGGL(k_pp_rows, dim3(grid_for(n)), dim3(256), 0, stream, levels, H, W, r, relevancy, tmp);
    LS2_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_pp_cols, dim3(grid_for(n)), dim3(256), 0, stream, levels, H, W, r, smooth_mode, relevancy,
                       tmp, smoothed);
    LS2_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_pp_minmax, dim3(kPpBlocks), dim3(256), 0, stream, levels, HW, smoothed, pmax, parg, pmin);
    LS2_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_pp_minmax_final, dim3(1), dim3(64), 0, stream, levels, kPpBlocks, pmax, parg, pmin, stats,
                       sarg);
    LS2_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_pp_maskstats, dim3(kPpBlocks), dim3(256), 0, stream, levels, HW, smoothed, stats, threshold,
                       psum, pcnt);
    LS2_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_pp_select, dim3(1), dim3(64), 0, stream, levels, kPpBlocks, W, select_mode, psum, pcnt,
                       stats, sarg, sel, result, level_stats);
    LS2_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_pp_mask, dim3(grid_for(HW)), dim3(256), 0, stream, HW, smoothed, stats, sel, threshold, mask);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}
