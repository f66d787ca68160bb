// ls2_project: per-Gaussian EWA projection (Section 3.1, Eqs. 1-2; EWA
// splatting as cited there).  One thread per Gaussian, float32 throughout.
#include "project_common.h"

namespace ls2 {

__global__ __launch_bounds__(256) void k_project(CamK cam, int n, const float* __restrict__ means,
                                                 const float* __restrict__ scales,
                                                 const float* __restrict__ quats,
                                                 float* __restrict__ mean2d, float* __restrict__ conic,
                                                 float* __restrict__ depth, int* __restrict__ radius,
                                                 int* __restrict__ touched) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    store_proj(project_one(cam, means, scales, quats, i), i, mean2d, conic, depth, radius, touched);
}

}  // namespace ls2

extern "C" int ls2_project(const ls2_camera* cam, int32_t n, const float* means, const float* scales,
                           const float* quats, float* mean2d, float* conic, float* depth, int32_t* radius,
                           int32_t* tiles_touched, hipStream_t stream) {
    if (!ls2::cam_valid(cam) || n < 0) return LS2_ERR_ARG;
    if (n == 0) return LS2_OK;
    if (!means || !scales || !quats || !mean2d || !conic || !depth || !radius) return LS2_ERR_ARG;
    const ls2::CamK k = ls2::cam_k(*cam);
    const int blocks = (n + 255) / 256;
    hipLaunchKernelGGL(ls2::k_project, dim3(blocks), dim3(256), 0, stream, k, n, means, scales, quats, mean2d,
                       conic, depth, radius, tiles_touched);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}
