// ls2_splat_dense: the dense reference form of the coefficient splatting --
// every Gaussian blends all L coefficients of each level (the rendering that
// Section 3.4 replaces by blending only the K non-zero ones; Table 9 compares
// the two).  Same quadrant mapping, culling, staging and alpha arithmetic as
// ls2_splat_sparse; the per-pixel accumulators live in VGPRs (the coefficient
// index is static here), the Gaussian's weights are read with wave-uniform
// loads.  As in the sparse splat, one wave renders one level of one quadrant.  With weights that are zero outside a Gaussian's K stored indices
// the result equals ls2_splat_sparse bit for bit (an added exact zero leaves
// every float unchanged).
#include "splat_common.h"

namespace ls2 {

struct SplatDenseArgs {
    CamK cam;
    int n, levels, L;
    const unsigned* ranges;
    const unsigned* ids;
    const float* mean2d;
    const float* conic;
    const float* opacity;
    const float* weights;  // [n, levels, L]
    float* coef;
    float* final_T;
    int* last;
};

template <int L>
__global__ __launch_bounds__(64) void k_splat_dense(SplatDenseArgs a) {
    constexpr int STRIDE = 8;  // u, v, A2, B2, C2, o, position, id
    __shared__ float4 stage4[64 * STRIDE / 4];
    float* stage = reinterpret_cast<float*>(stage4);
    const CamK& cam = a.cam;
    const int ntiles = cam.tx * cam.ty;
    int tile, slot;
    xcd_remap(blockIdx.x, gridDim.x, 4 * a.levels, tile, slot);
    if (tile >= ntiles) return;
    const int quad = slot & 3, lv0 = slot >> 2;
    const int lane = threadIdx.x;
    const int tx = tile % cam.tx, ty = tile / cam.tx;
    const int qx0 = tx * kTile + (quad & 1) * 8, qy0 = ty * kTile + (quad >> 1) * 8;
    if (qx0 >= cam.W || qy0 >= cam.H) return;
    const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
    const bool inside = px < cam.W && py < cam.H;
    const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
    const float bx0 = (float)qx0 + 0.5f, by0 = (float)qy0 + 0.5f;
    const float bx1 = (float)min(qx0 + 7, cam.W - 1) + 0.5f, by1 = (float)min(qy0 + 7, cam.H - 1) + 0.5f;
    const unsigned start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const unsigned long long lt = (1ull << lane) - 1ull;

    float acc[L];
#pragma unroll
    for (int c = 0; c < L; ++c) acc[c] = 0.0f;
    float T = 1.0f;
    int last = 0;
    bool active = inside;

    for (unsigned b = start; b < end; b += 64) {
        if (__builtin_amdgcn_ballot_w64(active) == 0) break;
        const unsigned pos = b + lane;
        unsigned id = 0xffffffffu;
        float mu = 0.f, mv = 0.f, cA = 0.f, cB = 0.f, cC = 0.f, op = 0.f;
        if (pos < end) {
            id = a.ids[pos];
            if (id < (unsigned)a.n) {
                const float2 m = reinterpret_cast<const float2*>(a.mean2d)[id];
                mu = m.x;
                mv = m.y;
                cA = a.conic[3 * id];
                cB = a.conic[3 * id + 1];
                cC = a.conic[3 * id + 2];
                op = a.opacity[id];
            }
        }
        const bool keep = pos < end && id < (unsigned)a.n && may_touch(mu, mv, cA, cB, cC, op, bx0, bx1, by0, by1);
        const unsigned long long kmask = __builtin_amdgcn_ballot_w64(keep);
        const int nkeep = __builtin_popcountll(kmask);
        wave_lds_order();
        if (keep) {
            float* r = stage + __builtin_popcountll(kmask & lt) * STRIDE;
            r[0] = mu;
            r[1] = mv;
            r[2] = -0.5f * kLog2e * cA;
            r[3] = -kLog2e * cB;
            r[4] = -0.5f * kLog2e * cC;
            r[5] = op;
            reinterpret_cast<unsigned*>(r)[6] = b - start + lane;
            reinterpret_cast<unsigned*>(r)[7] = id;
        }
        wave_lds_order();
        for (int j = 0; j < nkeep; ++j) {
            const float* r = stage + j * STRIDE;
            const float4 h0 = *reinterpret_cast<const float4*>(r);
            const float4 h1 = *reinterpret_cast<const float4*>(r + 4);
            const float dx = h0.x - pxc, dy = h0.y - pyc;
            const float p2 = gauss_power2(h0.z, h0.w, h1.x, dx, dy);
            const float g = h1.y * fast_exp2(p2);
            const float alpha = fminf(0.99f, g);
            const float c = alpha * T;
            const float testT = T - c;
            const bool hit = active && p2 <= 0.0f && alpha >= (1.0f / 255.0f);
            const bool stop = hit && testT < 1e-4f;
            const bool contrib = hit && !stop;
            active = active && !stop;
            if (__builtin_amdgcn_ballot_w64(contrib) != 0) {
                // the Gaussian's dense weights: a wave-uniform address
                const unsigned gid = __builtin_amdgcn_readfirstlane(__float_as_uint(h1.w));
                const float* w = a.weights + ((size_t)gid * a.levels + lv0) * L;
                const float cc = contrib ? c : 0.0f;
#pragma unroll
                for (int q = 0; q < L; ++q) acc[q] = contrib ? fmaf(w[q], cc, acc[q]) : acc[q];
                if (contrib) {
                    T = testT;
                    last = __float_as_int(h1.z) + 1;
                }
            }
            if ((j & 7) == 7 && __builtin_amdgcn_ballot_w64(active) == 0) break;
        }
    }
    if (!inside) return;
    const size_t HW = (size_t)cam.W * cam.H;
    const size_t pix = (size_t)py * cam.W + px;
    float4* dst = reinterpret_cast<float4*>(a.coef + ((size_t)lv0 * HW + pix) * L);
#pragma unroll
    for (int q = 0; q < L / 4; ++q) dst[q] = make_float4(acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]);
    if (lv0 == 0) {
        if (a.final_T) a.final_T[pix] = T;
        if (a.last) a.last[pix] = last;
    }
}

template <int L>
static int launch_dense(const SplatDenseArgs& a, hipStream_t stream) {
    const int grid = round_up8(a.cam.tx * a.cam.ty * 4 * a.levels);
    hipLaunchKernelGGL((k_splat_dense<L>), dim3(grid), dim3(64), 0, stream, a);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_splat_dense(const ls2_camera* cam, int32_t n, int32_t levels, int32_t L,
                               const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                               const float* conic, const float* opacity, const float* weights, float* coef,
                               float* final_T, int32_t* last, hipStream_t stream) {
    if (!cam_valid(cam) || n < 0 || levels < 1 || L < 1) return LS2_ERR_ARG;
    if (!tile_ranges || !coef) return LS2_ERR_ARG;
    if (n > 0 && (!ids || !mean2d || !conic || !opacity || !weights)) return LS2_ERR_ARG;
    if (!(L == 32 || L == 64) || levels > 3 || levels * L > 192) return LS2_ERR_UNSUPPORTED;
    SplatDenseArgs a;
    a.cam = cam_k(*cam);
    a.n = n;
    a.levels = levels;
    a.L = L;
    a.ranges = tile_ranges;
    a.ids = ids;
    a.mean2d = mean2d;
    a.conic = conic;
    a.opacity = opacity;
    a.weights = weights;
    a.coef = coef;
    a.final_T = final_T;
    a.last = last;
    return L == 32 ? launch_dense<32>(a, stream) : launch_dense<64>(a, stream);
}
