// ls2_splat_sparse: efficient sparse coefficient splatting (Section 3.4,
// Appendix A Algorithm 1) with the front-to-back rule of Eq. 3.
//
// Mapping on CDNA4:
//   - one wavefront (64 lanes) per 8x8 pixel quadrant of a 16x16 tile, one
//     pixel per lane; the four quadrant waves of a tile walk the same list
//     independently (no workgroup barriers), so each stops as soon as all of
//     its own pixels are saturated (ballot over the lanes);
//   - the wave stages 64 list entries at a time into its own LDS slice (one
//     entry per lane: a gather of the Gaussian's 2D mean, conic, opacity and
//     K (index, weight) pairs per level), then every lane reads each entry
//     back as a broadcast;
//   - the K indices of the current Gaussian are wave-uniform, so they live in
//     scalar registers and select a register of the per-lane accumulator
//     vectors through the VGPR index mode: the L-dim coefficient vector of
//     each pixel stays in VGPRs (32 floats per vector; L/32 vectors per
//     level) and each blend touches only the K selected registers.
#include "ls2_internal.h"

namespace ls2 {

typedef float v32f __attribute__((ext_vector_type(32)));

struct SplatArgs {
    CamK cam;
    int n, levels, K, L;
    const unsigned* ranges;
    const unsigned* ids;
    const float* mean2d;
    const float* conic;
    const float* opacity;
    const int* topk_idx;
    const float* topk_w;
    float* coef;
    float* final_T;
    int* last;
};

constexpr float kLog2e = 1.4426950408889634f;

// Record layout in LDS (dwords): u, v, A2, B2, C2, o, idx words, weights.
// A2 = -0.5 A log2(e), B2 = -B log2(e), C2 = -0.5 C log2(e), so that the
// Gaussian exponent in base 2 is A2 dx^2 + B2 dx dy + C2 dy^2.
template <int KMAX, int LVMAX>
struct Rec {
    static constexpr int KW = (KMAX + 3) / 4;          // packed u8 index words per level
    static constexpr int IDX = 6;
    static constexpr int W = IDX + LVMAX * KW;
    static constexpr int RAW = W + LVMAX * KMAX;
    static constexpr int STRIDE = (RAW + 3) & ~3;      // 16-byte aligned records
};

// exponent (base 2) of the Gaussian at offset (dx, dy); shared by forward and
// backward so both take the same decisions bit for bit.
__device__ __forceinline__ float gauss_power2(float A2, float B2, float C2, float dx, float dy) {
    return fmaf(dx, fmaf(A2, dx, B2 * dy), C2 * dy * dy);
}

template <int NV, int KMAX, int LVMAX>
__global__ __launch_bounds__(64) void k_splat_sparse(SplatArgs a) {
    using R = Rec<KMAX, LVMAX>;
    __shared__ float4 stage4[64 * R::STRIDE / 4];
    float* stage = reinterpret_cast<float*>(stage4);

    const CamK& cam = a.cam;
    const int ntiles = cam.tx * cam.ty;
    int tile, quad;
    xcd_remap(blockIdx.x, gridDim.x, 4, tile, quad);
    if (tile >= ntiles) return;
    const int lane = threadIdx.x;
    const int tx = tile % cam.tx, ty = tile / cam.tx;
    const int qx0 = tx * kTile + (quad & 1) * 8, qy0 = ty * kTile + (quad >> 1) * 8;
    if (qx0 >= cam.W || qy0 >= cam.H) return;  // quadrant fully outside the image
    const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
    const bool inside = px < cam.W && py < cam.H;
    const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;

    const unsigned start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const int levels = a.levels, K = a.K;
    const int lmask = a.L - 1;

    v32f acc[LVMAX][NV];
#pragma unroll
    for (int lv = 0; lv < LVMAX; ++lv)
#pragma unroll
        for (int h = 0; h < NV; ++h) acc[lv][h] = (v32f){};

    float T = 1.0f;
    int last = 0;
    bool active = inside;

    for (unsigned b = start; b < end; b += 64) {
        if (__builtin_amdgcn_ballot_w64(active) == 0) break;
        const int nb = (int)min(64u, end - b);
        // ---- stage: lane j gathers entry b + j
        if (lane < nb) {
            unsigned id = a.ids[b + lane];
            float* r = stage + lane * R::STRIDE;
            // an id outside [0, n) can only come from a corrupted list; read
            // Gaussian 0 instead and make the entry transparent
            const bool bad = id >= (unsigned)a.n;
            if (bad) id = 0;
            const float2 m = reinterpret_cast<const float2*>(a.mean2d)[id];
            const float cA = a.conic[3 * id], cB = a.conic[3 * id + 1], cC = a.conic[3 * id + 2];
            r[0] = m.x;
            r[1] = m.y;
            r[2] = -0.5f * kLog2e * cA;
            r[3] = -kLog2e * cB;
            r[4] = -0.5f * kLog2e * cC;
            r[5] = bad ? 0.0f : a.opacity[id];
#pragma unroll
            for (int lv = 0; lv < LVMAX; ++lv) {
                if (lv < levels) {
                    const size_t base = ((size_t)id * levels + lv) * K;
                    unsigned wd[R::KW];
#pragma unroll
                    for (int q = 0; q < R::KW; ++q) wd[q] = 0;
#pragma unroll
                    for (int k = 0; k < KMAX; ++k) {
                        if (k < K) {
                            const unsigned ix = (unsigned)(a.topk_idx[base + k] & lmask);
                            wd[k >> 2] |= ix << (8 * (k & 3));
                            r[R::W + lv * KMAX + k] = a.topk_w[base + k];
                        }
                    }
#pragma unroll
                    for (int q = 0; q < R::KW; ++q) reinterpret_cast<unsigned*>(r)[R::IDX + lv * R::KW + q] = wd[q];
                }
            }
        }
        __syncthreads();  // single-wave workgroup: orders the LDS writes before the reads

        for (int j = 0; j < nb; ++j) {
            const float* r = stage + j * R::STRIDE;
            const float4 h0 = *reinterpret_cast<const float4*>(r);
            const float2 h1 = *reinterpret_cast<const float2*>(r + 4);
            const float dx = h0.x - pxc, dy = h0.y - pyc;
            const float p2 = gauss_power2(h0.z, h0.w, h1.x, dx, dy);
            const float g = h1.y * exp2f(p2);
            const float alpha = fminf(0.99f, g);
            const float testT = T * (1.0f - alpha);
            const bool hit = active && p2 <= 0.0f && alpha >= (1.0f / 255.0f);
            const bool stop = hit && testT < 1e-4f;
            const bool contrib = hit && !stop;
            active = active && !stop;
            const float c = contrib ? alpha * T : 0.0f;
            if (__builtin_amdgcn_ballot_w64(contrib) != 0) {
#pragma unroll
                for (int lv = 0; lv < LVMAX; ++lv) {
                    if (lv < levels) {
#pragma unroll
                        for (int k = 0; k < KMAX; ++k) {
                            if (k < K) {
                                const unsigned word = __builtin_amdgcn_readfirstlane(
                                    reinterpret_cast<const unsigned*>(r)[R::IDX + lv * R::KW + (k >> 2)]);
                                const unsigned ix = (word >> (8 * (k & 3))) & 0xffu;
                                const float w = __uint_as_float(__builtin_amdgcn_readfirstlane(
                                    __float_as_uint(r[R::W + lv * KMAX + k])));
                                const float x = w * c;
                                const unsigned jl = ix & 31u, jh = ix >> 5;
#pragma unroll
                                for (int h = 0; h < NV; ++h) acc[lv][h][jl] += (jh == (unsigned)h) ? x : 0.0f;
                            }
                        }
                    }
                }
                if (contrib) {
                    T = testT;
                    last = (int)(b - start) + j + 1;
                }
            }
            if (__builtin_amdgcn_ballot_w64(active) == 0) break;
        }
        __syncthreads();  // the next batch overwrites the stage
    }

    if (!inside) return;
    const size_t HW = (size_t)cam.W * cam.H;
    const size_t pix = (size_t)py * cam.W + px;
#pragma unroll
    for (int lv = 0; lv < LVMAX; ++lv) {
        if (lv < levels) {
            float4* dst = reinterpret_cast<float4*>(a.coef + ((size_t)lv * HW + pix) * (size_t)(NV * 32));
#pragma unroll
            for (int h = 0; h < NV; ++h)
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    dst[h * 8 + q] = make_float4(acc[lv][h][4 * q], acc[lv][h][4 * q + 1], acc[lv][h][4 * q + 2],
                                                 acc[lv][h][4 * q + 3]);
        }
    }
    if (a.final_T) a.final_T[pix] = T;
    if (a.last) a.last[pix] = last;
}

template <int NV, int KMAX, int LVMAX>
static int launch_splat(const SplatArgs& a, hipStream_t stream) {
    const int ntiles = a.cam.tx * a.cam.ty;
    const int grid = round_up8(ntiles * 4);
    hipLaunchKernelGGL((k_splat_sparse<NV, KMAX, LVMAX>), dim3(grid), dim3(64), 0, stream, a);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_splat_sparse(const ls2_camera* cam, int32_t n, int32_t levels, int32_t K, int32_t L,
                                const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                                const float* conic, const float* opacity, const int32_t* topk_idx,
                                const float* topk_w, float* coef, float* final_T, int32_t* last,
                                hipStream_t stream) {
    if (!cam_valid(cam) || n < 0 || levels < 1 || K < 1 || L < 1 || K > L) return LS2_ERR_ARG;
    if (!tile_ranges || !coef) return LS2_ERR_ARG;
    if (n > 0 && (!ids || !mean2d || !conic || !opacity || !topk_idx || !topk_w)) return LS2_ERR_ARG;
    if (!(L == 32 || L == 64 || L == 128) || K > 8 || levels > 3 || levels * L > 192) return LS2_ERR_UNSUPPORTED;
    SplatArgs a;
    a.cam = cam_k(*cam);
    a.n = n;
    a.levels = levels;
    a.K = K;
    a.L = L;
    a.ranges = tile_ranges;
    a.ids = ids;
    a.mean2d = mean2d;
    a.conic = conic;
    a.opacity = opacity;
    a.topk_idx = topk_idx;
    a.topk_w = topk_w;
    a.coef = coef;
    a.final_T = final_T;
    a.last = last;
    const bool k8 = K > 4;
    const bool l3 = levels > 1;
    if (L == 32) {
        if (l3) return k8 ? launch_splat<1, 8, 3>(a, stream) : launch_splat<1, 4, 3>(a, stream);
        return k8 ? launch_splat<1, 8, 1>(a, stream) : launch_splat<1, 4, 1>(a, stream);
    }
    if (L == 64) {
        if (l3) return k8 ? launch_splat<2, 8, 3>(a, stream) : launch_splat<2, 4, 3>(a, stream);
        return k8 ? launch_splat<2, 8, 1>(a, stream) : launch_splat<2, 4, 1>(a, stream);
    }
    return k8 ? launch_splat<4, 8, 1>(a, stream) : launch_splat<4, 4, 1>(a, stream);
}
