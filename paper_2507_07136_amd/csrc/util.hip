// ls2_accumulate: dst += src over n floats (gradient accumulation over the
// views of a training step).  Grid-stride, float4 where aligned.
#include "ls2_internal.h"

namespace ls2 {

__global__ __launch_bounds__(256) void k_accumulate(long long n, const float* __restrict__ src,
                                                    float* __restrict__ dst) {
    const long long n4 = n / 4;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n4; i += stride) {
        const float4 a = reinterpret_cast<const float4*>(src)[i];
        float4 b = reinterpret_cast<float4*>(dst)[i];
        b.x += a.x; b.y += a.y; b.z += a.z; b.w += a.w;
        reinterpret_cast<float4*>(dst)[i] = b;
    }
    for (long long i = 4 * n4 + blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) dst[i] += src[i];
}

}  // namespace ls2

extern "C" int ls2_accumulate(int64_t n, const float* src, float* dst, hipStream_t stream) {
    if (n < 0 || (n > 0 && (!src || !dst))) return LS2_ERR_ARG;
    if (!ls2::aligned16(src) || !ls2::aligned16(dst)) return LS2_ERR_ARG;
    if (n == 0) return LS2_OK;
    long long blocks = (n / 4 + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(ls2::k_accumulate, dim3((unsigned)blocks), dim3(256), 0, stream, n, src, dst);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}
