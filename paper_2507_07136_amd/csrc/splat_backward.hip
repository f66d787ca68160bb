// ls2_splat_sparse_backward: gradients of the sparse coefficient splatting
// (Section 3.4, Algorithm 1 with the compositing rule of Eq. 3) with respect
// to the 2D means, conics, opacities and the stored coefficients.
//
// For a pixel with contributors i (front to back), e_i = alpha_i T_i and
// W_l[j] = sum_i e_i w_{i,l,j}.  With g_l = dL/dW_l and
// c_i = sum_{l,k} g_l[idx_ilk] w_ilk:
//   dL/dw_ilk   = g_l[idx_ilk] e_i
//   dL/dalpha_i = T_i c_i - S_i / (1 - alpha_i),  S_i = sum_{m > i} c_m e_m,
// and through alpha = o exp(power) (no gradient where clamped at 0.99) to o,
// the 2D mean and the conic.
//
// Mapping: one wave per (8x8 quadrant, level).  The wave walks its tile list
// backwards from the largest `last` of its pixels, recovering each pixel's
// transmittance as T_i = T_{i+1} / (1 - alpha_i) from the stored final
// transmittance (no per-pixel lists are stored), with alpha recomputed by the
// same instructions as the forward.  Each lane holds its pixel's dL/dW vector
// of the level in registers, and the K wave-uniform indices select from it by
// register indexing; LDS holds only the staged records, so occupancy is set by
// registers.  dL/dalpha is a sum over levels of T_i c_il - S_il / (1 - alpha_i)
// (S_il: the level's share of S_i), so each level wave adds its own share of
// the mean / conic / opacity gradients; with one level per wave the L-float
// vector fits in registers with room for several waves per SIMD.  Per Gaussian the wave's 6 + K values are
// summed over its 64 pixels in one reduce-scatter and added with one atomic
// instruction (one lane per value).
#include "splat_common.h"

namespace ls2 {

typedef float v32f_bw __attribute__((ext_vector_type(32)));  // 32 lanes' worth of one pixel's dL/dW

struct SplatBwArgs {
    CamK cam;
    int n, levels, K, L;
    const unsigned* ranges;
    const unsigned* ids;
    const float* mean2d;
    const float* conic;
    const float* opacity;
    const int* topk_idx;
    const float* topk_w;
    const float* final_T;
    const int* last;
    const float* d_coef;
    float* d_mean2d;
    float* d_conic;
    float* d_opacity;
    float* d_topk_w;
};

// staged record (dwords): u, v, A2, B2, C2, o, position, id, A, B, C, idx words, weights
template <int KMAX>
struct BwRec {
    static constexpr int KW = (KMAX + 3) / 4;
    static constexpr int POS = 6, ID = 7, CA = 8;
    static constexpr int IDX = 11;
    static constexpr int W = IDX + KW;
    static constexpr int RAW = W + KMAX;
    static constexpr int STRIDE = (RAW + 3) & ~3;
};

template <int NV, int KMAX, bool EXACT>
__global__ __launch_bounds__(64, NV <= 2 ? 3 : 2) void k_splat_backward(SplatBwArgs a) {
    using R = BwRec<KMAX>;
    constexpr int NG = 6 + KMAX;    // gradient values per Gaussian
    __shared__ float4 stage4[64 * R::STRIDE / 4];
    float* stage = reinterpret_cast<float*>(stage4);

    const CamK& cam = a.cam;
    const int ntiles = cam.tx * cam.ty;
    const int levels = a.levels;
    int tile, slot;
    xcd_remap(blockIdx.x, gridDim.x, 4 * levels, tile, slot);
    if (tile >= ntiles) return;
    const int lv = slot >> 2, quad = slot & 3;
    const int lane = threadIdx.x;
    const int tx = tile % cam.tx, ty = tile / cam.tx;
    const int qx0 = tx * kTile + (quad & 1) * 8, qy0 = ty * kTile + (quad >> 1) * 8;
    if (qx0 >= cam.W || qy0 >= cam.H) return;
    const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
    const bool inside = px < cam.W && py < cam.H;
    const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
    const float bx0 = (float)qx0 + 0.5f, by0 = (float)qy0 + 0.5f;
    const float bx1 = (float)min(qx0 + 7, cam.W - 1) + 0.5f, by1 = (float)min(qy0 + 7, cam.H - 1) + 0.5f;
    const size_t HW = (size_t)cam.W * cam.H;
    const size_t pix = (size_t)py * cam.W + px;

    const unsigned start = a.ranges[2 * tile];
    const int list_len = (int)(a.ranges[2 * tile + 1] - start);
    const int K = EXACT ? KMAX : a.K, L = a.L;
    const int lmask = L - 1;
    const unsigned long long lt = (1ull << lane) - 1ull;

    float T = inside ? a.final_T[pix] : 1.0f;
    const int lastp = inside ? a.last[pix] : 0;
    int maxlast = lastp;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) maxlast = max(maxlast, __shfl_xor(maxlast, off));
    maxlast = min(maxlast, list_len);  // a forward state from another list cannot read past this one
    if (maxlast <= 0) return;  // no pixel of the quadrant blended anything

    // this lane's output after the reduce-scatter: value q of each Gaussian
    // goes to base[q] + stride[q] * id
    const TrSlot ts = tr_slot(NG, lane);
    float* out_base = nullptr;
    int out_stride = 0;
    bool out_on = ts.valid && ts.leader;
    if (ts.index < 2) {
        out_base = a.d_mean2d + ts.index;
        out_stride = 2;
    } else if (ts.index < 5) {
        out_base = a.d_conic + (ts.index - 2);
        out_stride = 3;
    } else if (ts.index == 5) {
        out_base = a.d_opacity;
        out_stride = 1;
    } else {
        const int k = ts.index - 6;
        out_on = out_on && k < K;
        out_base = a.d_topk_w + (size_t)lv * K + k;
        out_stride = levels * K;
    }

    // dL/dW of this lane's pixel at this level, in registers: the K
    // wave-uniform indices of a Gaussian select from it by register indexing
    v32f_bw gv[NV];
#pragma unroll
    for (int h = 0; h < NV; ++h) gv[h] = (v32f_bw){};
    if (inside) {
        const float4* src = reinterpret_cast<const float4*>(a.d_coef + ((size_t)lv * HW + pix) * (size_t)(NV * 32));
#pragma unroll
        for (int h = 0; h < NV; ++h)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float4 v = src[h * 8 + q];
                gv[h][4 * q] = v.x;
                gv[h][4 * q + 1] = v.y;
                gv[h][4 * q + 2] = v.z;
                gv[h][4 * q + 3] = v.w;
            }
    }

    float S = 0.0f;  // this level's sum over later contributors of c_m e_m
    // Software pipeline over the 64-entry batches (walked backwards): while
    // a batch is processed, the records and codes of the batch before it in
    // the list are in flight.
    struct Rc {
        unsigned id;
        float mu, mv, cA, cB, cC, op;
        int ix[KMAX];
        float w[KMAX];
    };
    auto fetch = [&](int bend_) {
        Rc q;
        q.id = 0xffffffffu;
        q.mu = q.mv = q.cA = q.cB = q.cC = q.op = 0.0f;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            q.ix[k] = 0;
            q.w[k] = 0.0f;
        }
        const int b0_ = max(0, bend_ - 64);
        if (bend_ > 0 && lane < bend_ - b0_) {
            q.id = a.ids[start + b0_ + lane];
            if (q.id < (unsigned)a.n) {
                const unsigned i = q.id;
                const float2 m = reinterpret_cast<const float2*>(a.mean2d)[i];
                q.mu = m.x;
                q.mv = m.y;
                q.cA = a.conic[3 * i];
                q.cB = a.conic[3 * i + 1];
                q.cC = a.conic[3 * i + 2];
                q.op = a.opacity[i];
                const size_t base = ((size_t)i * levels + lv) * K;
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    q.ix[k] = k < K ? a.topk_idx[base + k] : 0;
                    q.w[k] = k < K ? a.topk_w[base + k] : 0.0f;
                }
            }
        }
        return q;
    };
    Rc nxt = fetch(maxlast);
    for (int bend = maxlast; bend > 0; bend -= 64) {
        const int b0 = max(0, bend - 64), nb = bend - b0;
        const Rc cur = nxt;
        nxt = fetch(bend - 64);  // the batch before this one in the list
        const unsigned id = cur.id;
        const float mu = cur.mu, mv = cur.mv, cA = cur.cA, cB = cur.cB, cC = cur.cC, op = cur.op;
        const bool keep = lane < nb && id < (unsigned)a.n && may_touch(mu, mv, cA, cB, cC, op, bx0, bx1, by0, by1);
        const unsigned long long kmask = __builtin_amdgcn_ballot_w64(keep);
        const int nkeep = __builtin_popcountll(kmask);
        wave_lds_order();  // single-wave workgroup: previous batch's reads done
        if (keep) {
            float* r = stage + __builtin_popcountll(kmask & lt) * R::STRIDE;
            r[0] = mu;
            r[1] = mv;
            r[2] = -0.5f * kLog2e * cA;
            r[3] = -kLog2e * cB;
            r[4] = -0.5f * kLog2e * cC;
            r[5] = op;
            reinterpret_cast<unsigned*>(r)[R::POS] = b0 + lane;
            reinterpret_cast<unsigned*>(r)[R::ID] = id;
            r[R::CA] = cA;
            r[R::CA + 1] = cB;
            r[R::CA + 2] = cC;
            unsigned wd[R::KW];
#pragma unroll
            for (int q = 0; q < R::KW; ++q) wd[q] = 0u;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const unsigned ix = k < K ? (unsigned)(cur.ix[k] & lmask) : 0u;
                wd[k >> 2] |= ix << (8 * (k & 3));
                r[R::W + k] = k < K ? cur.w[k] : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < R::KW; ++q) reinterpret_cast<unsigned*>(r)[R::IDX + q] = wd[q];
        }
        wave_lds_order();

        for (int j = nkeep - 1; j >= 0; --j) {
            const float* r = stage + j * R::STRIDE;
            const float4 h0 = *reinterpret_cast<const float4*>(r);
            const float4 h1 = *reinterpret_cast<const float4*>(r + 4);
            const int pos = __float_as_int(h1.z);
            const float dx = h0.x - pxc, dy = h0.y - pyc;
            const float p2 = gauss_power2(h0.z, h0.w, h1.x, dx, dy);
            const float G = fast_exp2(p2);
            const float g = h1.y * G;
            const float alpha = fminf(0.99f, g);
            const bool hit = pos < lastp && p2 <= 0.0f && alpha >= (1.0f / 255.0f);
            if (__builtin_amdgcn_ballot_w64(hit) == 0) continue;
            float vals[NG];
#pragma unroll
            for (int q = 0; q < NG; ++q) vals[q] = 0.0f;
            unsigned words[R::KW];
#pragma unroll
            for (int q = 0; q < R::KW; ++q)
                words[q] = __builtin_amdgcn_readfirstlane(reinterpret_cast<const unsigned*>(r)[R::IDX + q]);
            if (hit) {
                const float inv_one_m = __builtin_amdgcn_rcpf(1.0f - alpha);  // 1 ulp; 1 - alpha >= 0.01
                T = T * inv_one_m;  // transmittance in front of this Gaussian
                const float e = alpha * T;
                float c = 0.0f;
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    if (k < K) {
                        const unsigned ix = (words[k >> 2] >> (8 * (k & 3))) & 0xffu;  // < L, wave-uniform
                        float gk = 0.0f;
#pragma unroll
                        for (int h = 0; h < NV; ++h)
                            if ((int)(ix >> 5) == h) gk = gv[h][ix & 31u];
                        c = fmaf(gk, r[R::W + k], c);
                        vals[6 + k] = gk * e;
                    }
                }
                const float dalpha = T * c - S * inv_one_m;
                S = fmaf(c, e, S);
                if (g < 0.99f) {  // unclamped: alpha = o exp(power)
                    const float dpow = dalpha * alpha;  // dL/dpower (natural log units)
                    const float A = r[R::CA], B = r[R::CA + 1], C = r[R::CA + 2];
                    vals[0] = dpow * -(A * dx + B * dy);  // d mean2d.x
                    vals[1] = dpow * -(C * dy + B * dx);  // d mean2d.y
                    vals[2] = dpow * (-0.5f * dx * dx);   // d conic A
                    vals[3] = dpow * (-dx * dy);          // d conic B
                    vals[4] = dpow * (-0.5f * dy * dy);   // d conic C
                    vals[5] = dalpha * G;                 // d opacity
                }
            }
            // sums over the wave's pixels, one value per lane, one atomic instruction
            const float tot = tr_reduce<5, NG>(vals, lane);
            const unsigned gid = reinterpret_cast<const unsigned*>(r)[R::ID];
            if (out_on && tot != 0.0f) atomicAdd(out_base + (size_t)out_stride * gid, tot);
        }
    }
}

__global__ void k_zero_f32(float* __restrict__ p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

static int zero_f32(float* p, long long n, hipStream_t stream) {
    if (n <= 0) return LS2_OK;
    const long long b = (n + 255) / 256;
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)(b < 2048 ? b : 2048)), dim3(256), 0, stream, p, n);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}

template <int NV, int KMAX>
static int launch_splat_bw(const SplatBwArgs& a, hipStream_t stream) {
    const int ntiles = a.cam.tx * a.cam.ty;
    const int grid = round_up8(ntiles * 4 * a.levels);
    if (a.K == KMAX)
        hipLaunchKernelGGL((k_splat_backward<NV, KMAX, true>), dim3(grid), dim3(64), 0, stream, a);
    else
        hipLaunchKernelGGL((k_splat_backward<NV, KMAX, false>), dim3(grid), dim3(64), 0, stream, a);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_splat_sparse_backward(const ls2_camera* cam, int32_t n, int32_t levels, int32_t K, int32_t L,
                                         const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                                         const float* conic, const float* opacity, const int32_t* topk_idx,
                                         const float* topk_w, const float* final_T, const int32_t* last,
                                         const float* d_coef, float* d_mean2d, float* d_conic, float* d_opacity,
                                         float* d_topk_w, hipStream_t stream) {
    if (!cam_valid(cam) || n < 0 || levels < 1 || K < 1 || L < 1 || K > L) return LS2_ERR_ARG;
    if (!tile_ranges || !final_T || !last || !d_coef) return LS2_ERR_ARG;
    if (n > 0 && (!ids || !mean2d || !conic || !opacity || !topk_idx || !topk_w || !d_mean2d || !d_conic ||
                  !d_opacity || !d_topk_w))
        return LS2_ERR_ARG;
    if (!(L == 32 || L == 64 || L == 128) || K > 8 || levels > 3 || levels * L > 192) return LS2_ERR_UNSUPPORTED;
    if (n == 0) return LS2_OK;
    if (const int st = check_code_indices((long long)n * levels * K, L, topk_idx, stream)) return st;
    int st;
    if ((st = zero_f32(d_mean2d, 2LL * n, stream)) != LS2_OK) return st;
    if ((st = zero_f32(d_conic, 3LL * n, stream)) != LS2_OK) return st;
    if ((st = zero_f32(d_opacity, (long long)n, stream)) != LS2_OK) return st;
    if ((st = zero_f32(d_topk_w, (long long)n * levels * K, stream)) != LS2_OK) return st;
    SplatBwArgs a;
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
    a.final_T = final_T;
    a.last = last;
    a.d_coef = d_coef;
    a.d_mean2d = d_mean2d;
    a.d_conic = d_conic;
    a.d_opacity = d_opacity;
    a.d_topk_w = d_topk_w;
    const bool k8 = K > 4;
    if (L == 32) return k8 ? launch_splat_bw<1, 8>(a, stream) : launch_splat_bw<1, 4>(a, stream);
    if (L == 64) return k8 ? launch_splat_bw<2, 8>(a, stream) : launch_splat_bw<2, 4>(a, stream);
    return k8 ? launch_splat_bw<4, 8>(a, stream) : launch_splat_bw<4, 4>(a, stream);
}
