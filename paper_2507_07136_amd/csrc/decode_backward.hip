// ls2_dict_decode_backward: gradients of F = W S (Eq. 7) given G = dL/dF:
//   dW = G S^T   [m x L]   (contraction over the D features),
//   dS = W^T G   [L x D]   (contraction over the m pixels; with several
//                           levels sharing S, their rows are simply more
//                           pixels of the same product).
// Both are float32 products on the matrix cores (v_mfma_f32_32x32x2_f32):
// at 2 m L D flops each they are bound by the fp32 MFMA rate, not by the
// one read of G they each need.
//
// dW: persistent workgroups of 8 waves; S (or a column chunk of it) lives in
//     LDS, each wave computes [L x 32 MT] tiles of dW^T for its pixels with
//     the reduction over D permuted so every lane reads its pixel's gradient
//     as contiguous 64-byte runs.
// dS: split-K over pixels.  Workgroup (part, column chunk) accumulates its
//     [L x chunk] slice over a contiguous pixel range in registers and writes
//     it to the workspace; a second kernel sums the parts in a fixed order,
//     so the result is deterministic.
#include "ls2_internal.h"

namespace ls2 {

typedef float f32x16b __attribute__((ext_vector_type(16)));

struct DecodeBwArgs {
    long long m;
    int L, D;
    const float* coef;
    const float* dict;
    const float* d_feat;
    float* d_coef;
    float* ws;       // [nparts][L][D]
    float* d_dict;
    int DC;          // dict columns per LDS chunk (dW kernel)
    int nparts;      // pixel parts (dS kernel)
    int DWG;         // columns per dS workgroup
    long long part_len;  // pixels per part (multiple of 32)
};

constexpr int kDcoefWaves = 8;

// dW^T tile [L x 32] per pixel tile: C = A B with A = S rows (32 x 2, lane l:
// row l%32, k = l/32) and B = G^T (2 x 32, lane l: pixel l%32, k = l/32).
// Step j of a 32-column group pairs column c0 + j (half 0) with c0 + 16 + j
// (half 1), so each lane reads 16 consecutive floats of its row.
template <int L, int MT>
__global__ __launch_bounds__(kDcoefWaves * 64, 1) void k_dcoef(DecodeBwArgs a) {
    constexpr int TL = L / 32;
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    const int DC = a.DC, D = a.D;
    const int sstride = DC + 4;
    const int nch = D / DC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 31, half = lane >> 5;
    const long long wg_pix = (long long)kDcoefWaves * 32 * MT;
    const long long nblk = (a.m + wg_pix - 1) / wg_pix;

    auto load_chunk = [&](int ch) {
        const int f4_row = DC / 4;
        for (int i = threadIdx.x; i < L * f4_row; i += blockDim.x) {
            const int r = i / f4_row, c4 = i - r * f4_row;
            const float4 v = reinterpret_cast<const float4*>(a.dict + (size_t)r * D + (size_t)ch * DC)[c4];
            *reinterpret_cast<float4*>(lds + r * sstride + 4 * c4) = v;
        }
    };
    if (nch == 1) {
        load_chunk(0);
        __syncthreads();
    }
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long pw = blk * wg_pix + (long long)wave * 32 * MT;  // the wave's first pixel
        f32x16b acc[TL][MT];
#pragma unroll
        for (int tl = 0; tl < TL; ++tl)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[tl][mt] = (f32x16b){};
        const float* grow[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            long long p = pw + mt * 32 + col;
            if (p >= a.m) p = a.m - 1;  // clamped rows are computed but not stored
            grow[mt] = a.d_feat + p * D + half * 16;
        }
        // column groups of 32 over the whole row; the next group's gradient
        // loads are issued before the current group's matrix-core work
        const int ngroups = D / 32;
        float4 g[MT][4], gn[MT][4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) g[mt][q] = reinterpret_cast<const float4*>(grow[mt])[q];
        for (int cg = 0; cg < ngroups; ++cg) {
            const int col0 = cg * 32;
            const int c0 = col0 % DC;
            if (nch > 1 && c0 == 0) {
                lds_barrier();
                load_chunk(col0 / DC);
                lds_barrier();
            }
            if (cg + 1 < ngroups) {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int q = 0; q < 4; ++q) gn[mt][q] = reinterpret_cast<const float4*>(grow[mt] + col0 + 32)[q];
            }
            float4 s[TL][4];
#pragma unroll
            for (int tl = 0; tl < TL; ++tl)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    s[tl][q] = *reinterpret_cast<const float4*>(lds + (32 * tl + col) * sstride + c0 + half * 16 + 4 * q);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int tl = 0; tl < TL; ++tl)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) {
                            const float sv = e == 0 ? s[tl][q].x : e == 1 ? s[tl][q].y : e == 2 ? s[tl][q].z : s[tl][q].w;
                            const float gv = e == 0 ? g[mt][q].x : e == 1 ? g[mt][q].y : e == 2 ? g[mt][q].z : g[mt][q].w;
                            acc[tl][mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(sv, gv, acc[tl][mt], 0, 0, 0);
                        }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int q = 0; q < 4; ++q) g[mt][q] = gn[mt][q];
        }
        // C[row, pixel]: lane holds rows 8 g + 4 half + i of pixel col
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const long long p = pw + mt * 32 + col;
            if (p < a.m) {
#pragma unroll
                for (int tl = 0; tl < TL; ++tl)
#pragma unroll
                    for (int gq = 0; gq < 4; ++gq)
                        *reinterpret_cast<float4*>(a.d_coef + p * L + 32 * tl + 8 * gq + 4 * half) =
                            make_float4(acc[tl][mt][4 * gq], acc[tl][mt][4 * gq + 1], acc[tl][mt][4 * gq + 2],
                                        acc[tl][mt][4 * gq + 3]);
            }
        }
    }
}

// dS partial [L x 32 TD] per wave: C = A B with A = W^T (32 x 2, lane l:
// atom row l%32, pixel k = l/32) and B = G (2 x 32, lane l: feature l%32,
// pixel k = l/32).  Step j of a 32-pixel group pairs pixel j (half 0) with
// pixel 16 + j (half 1).
template <int L, int TD>
__global__ __launch_bounds__(512) void k_ddict_partial(DecodeBwArgs a) {
    constexpr int TL = L / 32;
    const int D = a.D;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 31, half = lane >> 5;
    const int nchunk = D / a.DWG;
    const int part = blockIdx.x / nchunk, chunk = blockIdx.x - part * nchunk;
    const int d0 = chunk * a.DWG + wave * 32 * TD;
    const long long p_begin = (long long)part * a.part_len;
    long long p_end = p_begin + a.part_len;
    if (p_end > a.m) p_end = a.m;

    f32x16b acc[TL][TD];
#pragma unroll
    for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int td = 0; td < TD; ++td) acc[tl][td] = (f32x16b){};

    for (long long p0 = p_begin; p0 < p_end; p0 += 32) {
        // fully unrolled: the group's operand loads are all issued ahead of
        // its matrix-core work
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const long long p = p0 + half * 16 + j;
            const bool ok = p < p_end;
            float w[TL], g[TD];
#pragma unroll
            for (int tl = 0; tl < TL; ++tl) w[tl] = ok ? a.coef[p * L + 32 * tl + col] : 0.0f;
#pragma unroll
            for (int td = 0; td < TD; ++td) g[td] = ok ? a.d_feat[p * D + d0 + 32 * td + col] : 0.0f;
#pragma unroll
            for (int tl = 0; tl < TL; ++tl)
#pragma unroll
                for (int td = 0; td < TD; ++td)
                    acc[tl][td] = __builtin_amdgcn_mfma_f32_32x32x2f32(w[tl], g[td], acc[tl][td], 0, 0, 0);
        }
    }
    float* out = a.ws + (size_t)part * L * D;
#pragma unroll
    for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int td = 0; td < TD; ++td)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 32 * tl + 8 * (r >> 2) + 4 * half + (r & 3);
                out[(size_t)row * D + d0 + 32 * td + col] = acc[tl][td][r];
            }
}

// d_dict[e] = sum over parts of ws[part][e].  A workgroup takes 64
// consecutive elements; its 16 waves each add a contiguous slice of the parts
// (eight loads in flight per lane), then wave 0 adds the 16 slice sums in
// order: a fixed order, so the result is reproducible.
__global__ __launch_bounds__(1024) void k_ddict_reduce(const float* __restrict__ ws, int nparts, int LD,
                                                       float* __restrict__ d_dict) {
    __shared__ float part_sum[16][64];
    const int lane = threadIdx.x & 63, slice = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    const int per = (nparts + 15) / 16;
    const int p0 = slice * per, p1 = min(nparts, p0 + per);
    float acc = 0.0f;
    if (e < LD) {
        int p = p0;
        for (; p + 8 <= p1; p += 8) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = ws[(size_t)(p + k) * LD + e];
#pragma unroll
            for (int k = 0; k < 8; ++k) acc += v[k];
        }
        for (; p < p1; ++p) acc += ws[(size_t)p * LD + e];
    }
    part_sum[slice][lane] = acc;
    __syncthreads();
    if (slice == 0 && e < LD) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < 16; ++k) s += part_sum[k][lane];
        d_dict[e] = s;
    }
}

// Both products in one pass over G (L <= 64, D a multiple of 64, D <= 512):
// a workgroup of D / 64 waves walks 32-pixel tiles; wave w owns features
// [64 w, 64 w + 64).  Per tile:
//   1. each wave copies its 32 x 64 slice of G, and the workgroup the tile's
//      32 x L coefficients W, into LDS (both loaded coalesced during the
//      previous tile), then issues the loads of the next tile;
//   2. each wave forms its dW^T partial [L x 32] = S[:, its features]
//      G[tile, its features]^T (S in registers) and writes it to LDS;
//   3. after a barrier each wave accumulates dS[:, its features] += W^T G in
//      registers and then takes its share of summing the D / 64 partials (in
//      wave order) into the tile's dW rows, so the sums overlap the other
//      waves' matrix-core work.
// At the end each workgroup writes its dS partial; k_ddict_reduce sums the
// partials in a fixed order.  G is read from HBM once instead of twice.
constexpr int kFusedRow = 68;  // G staging / partial row stride (floats)

template <int L, int WPT>
__global__ __launch_bounds__(512, 1) void k_decode_bw_fused(DecodeBwArgs a) {
    constexpr int TL = L / 32;
    constexpr int PROW = L + 4;
    constexpr int WROW = L + 4;
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    const int D = a.D;
    const int nwaves = blockDim.x >> 6;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 31, half = lane >> 5;
    const int f_wave = wave * 64;
    float* stage = lds + wave * (32 * kFusedRow);                  // [32 px][68], this wave's G slice
    float* part = lds + nwaves * (32 * kFusedRow);                 // [nwaves][32 px][L + 4]
    float* wt = part + nwaves * (32 * PROW);                       // [32 px][L + 4], the tile's W
    const long long nblk = (a.m + 31) / 32;

    // S in the dW layout: sb[tl][j] = S[32 tl + col][f_wave + 32 half + j]
    float sb[TL][32];
#pragma unroll
    for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int j = 0; j < 32; ++j) sb[tl][j] = a.dict[(size_t)(32 * tl + col) * D + f_wave + 32 * half + j];

    f32x16b accd[TL][2];
#pragma unroll
    for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) accd[tl][mt] = (f32x16b){};

    // coalesced G slice loads: instruction i covers rows 4 i .. 4 i + 3, lane
    // l row 4 i + l / 16, float4 column l % 16.  W: float4 number
    // threadIdx.x + k blockDim.x of the tile (row-major), k < WPT
    const int lrow = lane >> 4, lc4 = lane & 15;
    constexpr int W4 = 32 * L / 4;   // float4s in a W tile; WPT >= W4 / blockDim.x
    float4 gr[8], wreg[WPT];
    auto load_tile = [&](long long blk) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const long long p = blk * 32 + 4 * i + lrow;
            gr[i] = (blk < nblk && p < a.m) ? reinterpret_cast<const float4*>(a.d_feat + p * D + f_wave)[lc4]
                                            : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const int idx = threadIdx.x + k * blockDim.x;
            const int wr = idx / (L / 4), wc4 = idx - wr * (L / 4);
            const long long p = blk * 32 + wr;
            wreg[k] = (idx < W4 && blk < nblk && p < a.m) ? reinterpret_cast<const float4*>(a.coef + p * L)[wc4]
                                                          : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    long long blk = blockIdx.x;
    load_tile(blk);
    for (; blk < nblk; blk += gridDim.x) {
        const long long p0 = blk * 32;
        // 1. LDS copies (every read of the previous tile's copies ended before
        //    the barrier that closed it)
#pragma unroll
        for (int i = 0; i < 8; ++i) *reinterpret_cast<float4*>(stage + (4 * i + lrow) * kFusedRow + 4 * lc4) = gr[i];
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const int idx = threadIdx.x + k * blockDim.x;
            const int wr = idx / (L / 4), wc4 = idx - wr * (L / 4);
            if (idx < W4) *reinterpret_cast<float4*>(wt + wr * WROW + 4 * wc4) = wreg[k];
        }
        wave_lds_order();
        load_tile(blk + gridDim.x);
        // 2. dW^T partial over this wave's 64 features
        f32x16b accc[TL];
#pragma unroll
        for (int tl = 0; tl < TL; ++tl) accc[tl] = (f32x16b){};
#pragma unroll
        for (int j4 = 0; j4 < 8; ++j4) {
            const float4 g4 = *reinterpret_cast<const float4*>(stage + col * kFusedRow + 32 * half + 4 * j4);
            const float gv[4] = {g4.x, g4.y, g4.z, g4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int tl = 0; tl < TL; ++tl)
                    accc[tl] = __builtin_amdgcn_mfma_f32_32x32x2f32(sb[tl][4 * j4 + e], gv[e], accc[tl], 0, 0, 0);
        }
        // lane holds atoms 32 tl + 8 g + 4 half + i of pixel col
        float* pw = part + wave * (32 * PROW) + col * PROW;
#pragma unroll
        for (int tl = 0; tl < TL; ++tl)
#pragma unroll
            for (int g = 0; g < 4; ++g)
                *reinterpret_cast<float4*>(pw + 32 * tl + 8 * g + 4 * half) =
                    make_float4(accc[tl][4 * g], accc[tl][4 * g + 1], accc[tl][4 * g + 2], accc[tl][4 * g + 3]);
        lds_barrier();
        // 3a. dS += W^T G: step s pairs pixel q(s) (half 0) with q(s) + 8 (half 1)
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int q = (s >> 3) * 16 + (s & 7) + 8 * half;
            float w[TL], g[2];
#pragma unroll
            for (int tl = 0; tl < TL; ++tl) w[tl] = wt[q * WROW + 32 * tl + col];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) g[mt] = stage[q * kFusedRow + 32 * mt + col];
#pragma unroll
            for (int tl = 0; tl < TL; ++tl)
#pragma unroll
                for (int mt = 0; mt < 2; ++mt)
                    accd[tl][mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(w[tl], g[mt], accd[tl][mt], 0, 0, 0);
        }
        // 3b. this thread's share of the tile's dW rows
        for (int t = threadIdx.x; t < W4; t += blockDim.x) {
            const int px = t / (L / 4), a4 = t - px * (L / 4);
            float4 s4 = *reinterpret_cast<const float4*>(part + px * PROW + 4 * a4);
            for (int w = 1; w < nwaves; ++w) {
                const float4 v = *reinterpret_cast<const float4*>(part + w * (32 * PROW) + px * PROW + 4 * a4);
                s4.x += v.x;
                s4.y += v.y;
                s4.z += v.z;
                s4.w += v.w;
            }
            const long long p = p0 + px;
            if (p < a.m) *reinterpret_cast<float4*>(a.d_coef + p * L + 4 * a4) = s4;
        }
        lds_barrier();
    }
    float* out = a.ws + (size_t)blockIdx.x * L * D;
#pragma unroll
    for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 32 * tl + 8 * (r >> 2) + 4 * half + (r & 3);
                out[(size_t)row * D + f_wave + 32 * mt + col] = accd[tl][mt][r];
            }
}

static int decode_bw_plan(long long m, int L, int D, DecodeBwArgs& a) {
    a.m = m;
    a.L = L;
    a.D = D;
    // LDS chunk of S: at most 128 KB, a multiple of 32 columns dividing D
    a.DC = 32768 / L < D ? 32768 / L : D;
    while (D % a.DC != 0) a.DC -= 32;
    a.DWG = D < 512 ? D : 512;
    const int nchunk = D / a.DWG;
    const long long nblk32 = (m + 31) / 32;
    long long nparts = 512 / nchunk;
    if (nparts > nblk32) nparts = nblk32;
    if (nparts < 1) nparts = 1;
    a.part_len = ((nblk32 + nparts - 1) / nparts) * 32;
    a.nparts = (int)((m + a.part_len - 1) / a.part_len);
    if (a.nparts < 1) a.nparts = 1;
    return LS2_OK;
}

static int td_for(int L, int D) {
    if (L == 32) return D % 256 == 0 ? 8 : 4;
    if (L == 64) return 4;
    return 2;
}

static bool fused_bw_ok(int L, int D) { return (L == 32 || L == 64) && D % 64 == 0 && D <= 512; }

static size_t fused_bw_lds(int L, int D) {
    const int nw = D / 64;
    return ((size_t)nw * 32 * kFusedRow + (size_t)nw * 32 * (L + 4) + (size_t)32 * (L + 4)) * sizeof(float);
}

template <int L>
static int launch_decode_bw(DecodeBwArgs a, hipStream_t stream) {
    constexpr int MT = L <= 64 ? 2 : 1;
    static int num_cus = 0;
    if (num_cus == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        num_cus = n;
    }
    if constexpr (L <= 64) {
        if (a.d_coef && a.d_dict && fused_bw_ok(L, a.D)) {
            const size_t lds = fused_bw_lds(L, a.D);
            const int threads = (a.D / 64) * 64;
            const int wpt_need = (32 * L / 4 + threads - 1) / threads;
            const void* kern = wpt_need <= 1   ? (const void*)k_decode_bw_fused<L, 1>
                               : wpt_need <= 2 ? (const void*)k_decode_bw_fused<L, 2>
                                               : (const void*)k_decode_bw_fused<L, 4>;
            static bool attr[3] = {false, false, false};
            const int ai = wpt_need <= 1 ? 0 : (wpt_need <= 2 ? 1 : 2);
            if (!attr[ai]) {
                if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(160 * 1024)) !=
                    hipSuccess)
                    return LS2_ERR_DEVICE;
                attr[ai] = true;
            }
            // one workgroup per CU (the partial products fill the LDS), at most
            // one dS partial per workspace slot
            const long long nblk = (a.m + 31) / 32;
            long long grid = num_cus;
            if (grid > a.nparts) grid = a.nparts;
            if (grid > nblk) grid = nblk;
            if (ai == 0)
                hipLaunchKernelGGL((k_decode_bw_fused<L, 1>), dim3((unsigned)grid), dim3(threads), lds, stream, a);
            else if (ai == 1)
                hipLaunchKernelGGL((k_decode_bw_fused<L, 2>), dim3((unsigned)grid), dim3(threads), lds, stream, a);
            else
                hipLaunchKernelGGL((k_decode_bw_fused<L, 4>), dim3((unsigned)grid), dim3(threads), lds, stream, a);
            LS2_LAUNCH_CHECK();
            const int LD = L * a.D;
            hipLaunchKernelGGL(k_ddict_reduce, dim3((LD + 63) / 64), dim3(1024), 0, stream, a.ws, (int)grid, LD,
                               a.d_dict);
            LS2_LAUNCH_CHECK();
            return LS2_OK;
        }
    }
    if (a.d_coef) {
        const size_t lds = (size_t)L * (a.DC + 4) * sizeof(float);
        static bool attr = false;
        if (!attr) {
            if (hipFuncSetAttribute((const void*)k_dcoef<L, MT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(136 * 1024)) != hipSuccess)
                return LS2_ERR_DEVICE;
            attr = true;
        }
        const long long wg_pix = (long long)kDcoefWaves * 32 * MT;
        long long grid = (a.m + wg_pix - 1) / wg_pix;
        if (grid > num_cus) grid = num_cus;
        hipLaunchKernelGGL((k_dcoef<L, MT>), dim3((unsigned)grid), dim3(kDcoefWaves * 64), lds, stream, a);
        LS2_LAUNCH_CHECK();
    }
    if (a.d_dict) {
        const int td = td_for(L, a.D);
        const int nw = a.DWG / (32 * td);
        const int nchunk = a.D / a.DWG;
        const dim3 grid((unsigned)(a.nparts * nchunk)), block((unsigned)(nw * 64));
        // accumulators per lane: L * 32 TD / 64 = 128 (or 64 for L = 32, D = 384)
        if constexpr (L == 32) {
            if (td == 8)
                hipLaunchKernelGGL((k_ddict_partial<32, 8>), grid, block, 0, stream, a);
            else
                hipLaunchKernelGGL((k_ddict_partial<32, 4>), grid, block, 0, stream, a);
        } else {
            hipLaunchKernelGGL((k_ddict_partial<L, 256 / L>), grid, block, 0, stream, a);
        }
        LS2_LAUNCH_CHECK();
        const int LD = L * a.D;
        hipLaunchKernelGGL(k_ddict_reduce, dim3((LD + 63) / 64), dim3(1024), 0, stream, a.ws, a.nparts, LD,
                           a.d_dict);
        LS2_LAUNCH_CHECK();
    }
    return LS2_OK;
}

static int num_cus_bw() {
    static int n_cus = 0;
    if (n_cus == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        n_cus = n;
    }
    return n_cus;
}

// ---------------------------------------------------------------------------
// Decode, feature loss and both decode gradients in one pass (L in {32, 64},
// D a multiple of 128 up to 512): the float32 training objective of Section
// 4.1 on F = W S (Eq. 7), with dL/dF consumed on the chip instead of being
// written and read back.  A workgroup of D / 64 waves walks 32-pixel blocks;
// wave w owns features [64 w, 64 w + 64), keeps its slice of S in the
// forward operand layout (the first feature tile in VGPRs, the second in LDS:
// the registers would not hold both) and its dS = W^T dL/dF partial in the
// matrix accumulators across blocks.  Per block:
//   1. F = W S over its slice (W from a double-buffered LDS tile loaded a
//      block ahead) while the block's target rows arrive;
//   2. the per-pixel sums of the loss (|F - Y|, F.Y, F.F, Y.Y over the slice),
//      exchanged between the waves through LDS;
//   3. dL/dF, in the accumulator registers and in the wave's LDS tile;
//   4. the dW partial dL/dF S^T over the slice, from the registers: one
//      v_permlane32_swap per register pair gives the B operands in which step
//      x pairs feature x with x + 32, as the separate backward reads them;
//      the A operands (S rows) stream from L2, the first half issued before
//      the exchange;
//   5. dS += W^T dL/dF from the tile;
//   6. the dW partials through the tiles, summed in wave order and stored.
// Every product takes the same operands in the same order as
// ls2_decode_feature_loss followed by ls2_dict_decode_backward (and the loss
// formulas are the same), so with the same workgroup count d_coef, d_dict and
// the loss equal that chain's bit for bit.
struct DecodeLossBwArgs {
    long long m, nblocks;
    int D;
    const float* coef;    // W [m, L]
    const float* dict;    // S [L, D]
    const float* target;  // Y [m, D]
    float* d_coef;        // [m, L]
    float* ws;            // [gridDim.x][L][D]: dS partials
    CSum* partial;        // [gridDim.x][2]: loss partials
    float inv_md, inv_m;
};

typedef float f32x4l __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float loss_sign(float e) { return e > 0.f ? 1.f : (e < 0.f ? -1.f : 0.f); }

constexpr int kLbRow = 68;  // row stride (floats) of the per-wave tiles and the W tiles

template <int L, int WPT>
__global__ __launch_bounds__(512, 1) void k_decode_loss_bw(DecodeLossBwArgs a) {
    constexpr int TL = L / 32;      // atom tiles of 32
    constexpr int KS = L / 2;       // forward k-steps
    constexpr int W4 = 32 * L / 4;  // float4s in a W tile
    extern __shared__ float4 lds4[];
    __shared__ float4 red[2][8][32];  // per block parity, wave, pixel: (l1, fy, ff, yy) over the wave's slice
    __shared__ CSum lred[2][64];
    float* lds = reinterpret_cast<float*>(lds4);
    const int D = a.D;
    const int nwaves = blockDim.x >> 6;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 31, half = lane >> 5;
    const int f_wave = wave * 64;
    float* tile = lds + wave * (32 * kLbRow);        // [32 px][kLbRow]: target, then dL/dF, then the dW partial
    float* wtiles = lds + nwaves * (32 * kLbRow);    // [2][32 px][kLbRow]: W of the current and the next block
    // the second feature tile's forward operands: [KS / 4][64 lanes] float4 per wave
    float4* sa1 = reinterpret_cast<float4*>(wtiles + 2 * (32 * kLbRow)) + wave * (KS / 4) * 64;
    const int sp = lane >> 4, su = lane & 15;        // row-segment access: rows 4 i + sp, 16-byte unit su
    const float inv_md = a.inv_md, inv_m = a.inv_m;
    CSum l1_acc{}, lc_acc{};

    // forward A operand S[half KS + s][f_wave + 32 mt + col]: the first
    // feature tile's in VGPRs, the second's in LDS (four k-steps per float4)
    float sa[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) sa[s] = a.dict[(size_t)(half * KS + s) * D + f_wave + col];
#pragma unroll
    for (int q = 0; q < KS / 4; ++q) {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = a.dict[(size_t)(half * KS + 4 * q + e) * D + f_wave + 32 + col];
        sa1[q * 64 + lane] = make_float4(v[0], v[1], v[2], v[3]);
    }
    // dW A operand rows: S[32 tl + col][f_wave + 32 half + x]
    const float* srow = a.dict + (size_t)col * D + f_wave + 32 * half;

    f32x16b accd[TL][2];
#pragma unroll
    for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) accd[tl][mt] = (f32x16b){};

    // W tile: float4 number threadIdx.x + k blockDim.x of the tile (row-major)
    auto load_w = [&](long long bk, float4 (&w)[WPT]) {
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const int idx = threadIdx.x + k * blockDim.x;
            const int wr = idx / (L / 4), wc4 = idx - wr * (L / 4);
            const long long p = bk * 32 + wr;
            w[k] = (idx < W4 && bk < a.nblocks && p < a.m) ? reinterpret_cast<const float4*>(a.coef + p * L)[wc4]
                                                           : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto store_w = [&](float* wt, const float4 (&w)[WPT]) {
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const int idx = threadIdx.x + k * blockDim.x;
            const int wr = idx / (L / 4), wc4 = idx - wr * (L / 4);
            if (idx < W4) *reinterpret_cast<float4*>(wt + wr * kLbRow + 4 * wc4) = w[k];
        }
    };

    long long blk = blockIdx.x;
    const long long bstep = gridDim.x;
    float4 wpf[WPT];
    load_w(blk, wpf);
    store_w(wtiles, wpf);
    load_w(blk + bstep, wpf);
    lds_barrier();
    int cur = 0;
    for (; blk < a.nblocks; blk += bstep) {
        const long long p0 = blk * 32;
        const float* wt = wtiles + cur * (32 * kLbRow);
        // 1. the block's target rows, then F = W S on the matrix cores
        f32x4l yr[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const long long row = p0 + 4 * i + sp;
            yr[i] = row < a.m
                        ? __builtin_nontemporal_load(reinterpret_cast<const f32x4l*>(a.target + row * D + f_wave) + su)
                        : (f32x4l){0.f, 0.f, 0.f, 0.f};
        }
        f32x16b acc[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) acc[mt] = (f32x16b){};
#pragma unroll
        for (int q = 0; q < KS / 4; ++q) {  // B operand: pixel col, atoms half KS + 4 q .. + 3
            const float4 w4 = *reinterpret_cast<const float4*>(wt + col * kLbRow + half * KS + 4 * q);
            const float4 s4 = sa1[q * 64 + lane];
            const float wq[4] = {w4.x, w4.y, w4.z, w4.w};
            const float s1[4] = {s4.x, s4.y, s4.z, s4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[4 * q + e], wq[e], acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(s1[e], wq[e], acc[1], 0, 0, 0);
            }
        }
        // the target through the tile into the accumulator layout
#pragma unroll
        for (int i = 0; i < 8; ++i) *reinterpret_cast<f32x4l*>(tile + (4 * i + sp) * kLbRow + 4 * su) = yr[i];
        // the first dW A operands, in flight during the exchange
        constexpr int SBA = 4;  // groups of four k-steps loaded ahead
        float4 sbq[8][TL];
#pragma unroll
        for (int j4 = 0; j4 < SBA; ++j4)
#pragma unroll
            for (int tl = 0; tl < TL; ++tl)
                sbq[j4][tl] = *reinterpret_cast<const float4*>(srow + (size_t)(32 * tl) * D + 4 * j4);
        wave_lds_order();
        // 2. per-pixel partial sums over the slice (lane: pixel col, features
        //    32 mt + 8 g + 4 half + [0, 4))
        auto ytile = [&](int mt, int g) -> float4* {
            return reinterpret_cast<float4*>(tile + col * kLbRow + mt * 32 + g * 8 + half * 4);
        };
        float l1 = 0.f, fy = 0.f, ff = 0.f, yy = 0.f;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const float f0 = acc[mt][4 * g], f1 = acc[mt][4 * g + 1], f2 = acc[mt][4 * g + 2], f3 = acc[mt][4 * g + 3];
                const float4 yv = *ytile(mt, g);
                l1 += fabsf(f0 - yv.x) + fabsf(f1 - yv.y) + fabsf(f2 - yv.z) + fabsf(f3 - yv.w);
                fy = fmaf(f0, yv.x, fmaf(f1, yv.y, fmaf(f2, yv.z, fmaf(f3, yv.w, fy))));
                ff = fmaf(f0, f0, fmaf(f1, f1, fmaf(f2, f2, fmaf(f3, f3, ff))));
                yy = fmaf(yv.x, yv.x, fmaf(yv.y, yv.y, fmaf(yv.z, yv.z, fmaf(yv.w, yv.w, yy))));
            }
        l1 += __shfl_xor(l1, 32);
        fy += __shfl_xor(fy, 32);
        ff += __shfl_xor(ff, 32);
        yy += __shfl_xor(yy, 32);
        if (half == 0) red[cur][wave][col] = make_float4(l1, fy, ff, yy);
        lds_barrier();
        // the next block's W tile: every wave finished reading that buffer
        // before the barrier that closed the previous block
        store_w(wtiles + (cur ^ 1) * (32 * kLbRow), wpf);
        load_w(blk + 2 * bstep, wpf);
        // 3. the row sums, the loss terms and dL/dF (registers and tile)
        float4 t = red[cur][0][col];
        for (int w = 1; w < nwaves; ++w) {
            const float4 u = red[cur][w][col];
            t.x += u.x; t.y += u.y; t.z += u.z; t.w += u.w;
        }
        const float nf = sqrtf(t.z), ny = sqrtf(t.w);
        const float gf = fmaxf(nf, 1e-12f), gy = fmaxf(ny, 1e-12f);
        const float cs = t.y / (gf * gy);
        if (wave == 0 && half == 0 && p0 + col < a.m) {
            l1_acc.add(t.x);
            lc_acc.add(1.0f - cs);
        }
        const float ay = inv_m / (gf * gy);
        const float bf = nf > 1e-12f ? inv_m * t.y / (nf * nf * nf * gy) : 0.f;
        const bool rok = p0 + col < a.m;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const float f0 = acc[mt][4 * g], f1 = acc[mt][4 * g + 1], f2 = acc[mt][4 * g + 2], f3 = acc[mt][4 * g + 3];
                const float4 yv = *ytile(mt, g);
                float4 o;
                o.x = loss_sign(f0 - yv.x) * inv_md - ay * yv.x + bf * f0;
                o.y = loss_sign(f1 - yv.y) * inv_md - ay * yv.y + bf * f1;
                o.z = loss_sign(f2 - yv.z) * inv_md - ay * yv.z + bf * f2;
                o.w = loss_sign(f3 - yv.w) * inv_md - ay * yv.w + bf * f3;
                if (!rok) o = make_float4(0.f, 0.f, 0.f, 0.f);  // rows past m: no gradient
                *ytile(mt, g) = o;  // in place: this lane alone reads and writes these 16 bytes
                acc[mt][4 * g] = o.x;
                acc[mt][4 * g + 1] = o.y;
                acc[mt][4 * g + 2] = o.z;
                acc[mt][4 * g + 3] = o.w;
            }
        // 4. dW partial: B operand of step x (ascending) = features x (half 0)
        //    and 32 + x (half 1) of pixel col.  After the swap, sw[0][r] holds
        //    x = 8 (r / 4) + r % 4 and sw[1][r] holds x = 8 (r / 4) + 4 + r % 4.
        float sw[2][16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const auto pr = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc[0][r]), __float_as_uint(acc[1][r]),
                                                             false, false);
            sw[0][r] = __uint_as_float(pr[0]);
            sw[1][r] = __uint_as_float(pr[1]);
        }
        f32x16b accc[TL];
#pragma unroll
        for (int tl = 0; tl < TL; ++tl) accc[tl] = (f32x16b){};
#pragma unroll
        for (int j4 = 0; j4 < 8; ++j4) {
            if (j4 + SBA < 8) {
#pragma unroll
                for (int tl = 0; tl < TL; ++tl)
                    sbq[j4 + SBA][tl] = *reinterpret_cast<const float4*>(srow + (size_t)(32 * tl) * D + 4 * (j4 + SBA));
            }
            const int g = j4 >> 1, c = j4 & 1;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float bx = sw[c][4 * g + e];
#pragma unroll
                for (int tl = 0; tl < TL; ++tl) {
                    const float4 s4 = sbq[j4][tl];
                    const float av = e == 0 ? s4.x : (e == 1 ? s4.y : (e == 2 ? s4.z : s4.w));
                    accc[tl] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bx, accc[tl], 0, 0, 0);
                }
            }
        }
        wave_lds_order();  // dL/dF in the tile before the dS reads
        // 5. dS += W^T dL/dF: step s pairs pixel q(s) (half 0) with q(s) + 8 (half 1)
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int q = (s >> 3) * 16 + (s & 7) + 8 * half;
            float w[TL], gv[2];
#pragma unroll
            for (int tl = 0; tl < TL; ++tl) w[tl] = wt[q * kLbRow + 32 * tl + col];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) gv[mt] = tile[q * kLbRow + 32 * mt + col];
#pragma unroll
            for (int tl = 0; tl < TL; ++tl)
#pragma unroll
                for (int mt = 0; mt < 2; ++mt)
                    accd[tl][mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(w[tl], gv[mt], accd[tl][mt], 0, 0, 0);
        }
        wave_lds_order();  // the tile's dS reads are done before the dW partial overwrites it
        // 6. the dW partial (lane: atoms 32 tl + 8 g + 4 half + [0, 4) of pixel col)
#pragma unroll
        for (int tl = 0; tl < TL; ++tl)
#pragma unroll
            for (int g = 0; g < 4; ++g)
                *reinterpret_cast<float4*>(tile + col * kLbRow + 32 * tl + 8 * g + 4 * half) =
                    make_float4(accc[tl][4 * g], accc[tl][4 * g + 1], accc[tl][4 * g + 2], accc[tl][4 * g + 3]);
        lds_barrier();
        for (int t4 = threadIdx.x; t4 < W4; t4 += blockDim.x) {
            const int px = t4 / (L / 4), a4 = t4 - px * (L / 4);
            float4 s4 = *reinterpret_cast<const float4*>(lds + px * kLbRow + 4 * a4);
            for (int w = 1; w < nwaves; ++w) {
                const float4 v = *reinterpret_cast<const float4*>(lds + w * (32 * kLbRow) + px * kLbRow + 4 * a4);
                s4.x += v.x;
                s4.y += v.y;
                s4.z += v.z;
                s4.w += v.w;
            }
            const long long p = p0 + px;
            if (p < a.m) *reinterpret_cast<float4*>(a.d_coef + p * L + 4 * a4) = s4;
        }
        lds_barrier();  // the tiles are free for the next block's target; its W tile is complete
        cur ^= 1;
    }
    float* out = a.ws + (size_t)blockIdx.x * L * D;
#pragma unroll
    for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 32 * tl + 8 * (r >> 2) + 4 * half + (r & 3);
                out[(size_t)row * D + f_wave + 32 * mt + col] = accd[tl][mt][r];
            }
    // per-pixel loss terms were added by the lanes of wave 0: sum them in lane order
    if (wave == 0) {
        lred[0][lane] = l1_acc;
        lred[1][lane] = lc_acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        CSum s0{}, s1{};
        for (int l = 0; l < 64; ++l) {
            s0.add(lred[0][l]);
            s1.add(lred[1][l]);
        }
        a.partial[2 * blockIdx.x] = s0;
        a.partial[2 * blockIdx.x + 1] = s1;
    }
}

constexpr int kLossBwMaxParts = 512;  // workgroups (dS and loss partials) at most

static size_t loss_bw_lds(int L, int D) {
    return (size_t)(D / 64 + 2) * 32 * kLbRow * sizeof(float) + (size_t)(D / 64) * (L / 8) * 64 * sizeof(float4);
}

static long long loss_bw_grid(long long m) {
    const long long nblk = (m + 31) / 32;
    long long grid = num_cus_bw();
    if (grid > kLossBwMaxParts) grid = kLossBwMaxParts;
    if (grid > nblk) grid = nblk;
    return grid < 1 ? 1 : grid;
}

static size_t loss_bw_dsum_bytes(long long m, int L, int D) {
    const long long nblk = (m + 31) / 32;
    const long long parts = nblk < kLossBwMaxParts ? nblk : kLossBwMaxParts;
    return (size_t)(parts < 1 ? 1 : parts) * L * D * sizeof(float);
}

template <int L>
static int launch_decode_loss_bw(DecodeLossBwArgs a, long long grid, hipStream_t stream) {
    const int threads = (a.D / 64) * 64;
    const int wpt = (32 * L / 4 + threads - 1) / threads;
    const size_t lds = loss_bw_lds(L, a.D);
    const void* kern = wpt <= 1 ? (const void*)k_decode_loss_bw<L, 1>
                                : (wpt <= 2 ? (const void*)k_decode_loss_bw<L, 2> : (const void*)k_decode_loss_bw<L, 4>);
    static bool attr[2][3] = {};
    bool& done = attr[L == 64][wpt <= 1 ? 0 : (wpt <= 2 ? 1 : 2)];
    if (!done) {
        if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(150 * 1024)) != hipSuccess)
            return LS2_ERR_DEVICE;
        done = true;
    }
    if (wpt <= 1)
        hipLaunchKernelGGL((k_decode_loss_bw<L, 1>), dim3((unsigned)grid), dim3(threads), lds, stream, a);
    else if (wpt <= 2)
        hipLaunchKernelGGL((k_decode_loss_bw<L, 2>), dim3((unsigned)grid), dim3(threads), lds, stream, a);
    else
        hipLaunchKernelGGL((k_decode_loss_bw<L, 4>), dim3((unsigned)grid), dim3(threads), lds, stream, a);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}

static bool decode_bw_supported(int L, int D) {
    return (L == 32 || L == 64 || L == 128) && D % 128 == 0 && D >= 128 && (D <= 512 || D == 1024);
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_dict_decode_backward_workspace(int64_t m, int32_t L, int32_t D, size_t* bytes) {
    if (!bytes || m < 0 || L < 1 || D < 1) return LS2_ERR_ARG;
    if (!decode_bw_supported(L, D)) return LS2_ERR_UNSUPPORTED;
    *bytes = 0;
    if (m == 0) return LS2_OK;
    DecodeBwArgs a;
    decode_bw_plan(m, L, D, a);
    *bytes = (size_t)a.nparts * L * D * sizeof(float);
    return LS2_OK;
}

extern "C" int ls2_dict_decode_backward(int64_t m, int32_t L, int32_t D, const float* coef, const float* dict,
                                        int32_t compute, const float* d_feat, float* d_coef, float* d_dict,
                                        void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (m < 0 || L < 1 || D < 1 || !dict || (m > 0 && !d_feat)) return LS2_ERR_ARG;
    if (compute != LS2_F32 && compute != LS2_BF16) return LS2_ERR_ARG;
    if (!d_coef && !d_dict) return LS2_ERR_ARG;
    if (d_dict && m > 0 && !coef) return LS2_ERR_ARG;
    if (!decode_bw_supported(L, D) || compute != LS2_F32) return LS2_ERR_UNSUPPORTED;
    if (!aligned16(coef) || !aligned16(dict) || !aligned16(d_feat) || !aligned16(d_coef)) return LS2_ERR_ARG;
    if (m == 0) {  // dS of an empty product: zeros (a fill kernel, no memset node)
        if (d_dict) {
            hipLaunchKernelGGL(k_ddict_reduce, dim3((L * D + 63) / 64), dim3(1024), 0, stream, (const float*)nullptr,
                               0, L * D, d_dict);
            LS2_LAUNCH_CHECK();
        }
        return LS2_OK;
    }
    DecodeBwArgs a;
    decode_bw_plan(m, L, D, a);
    if (d_dict) {
        const size_t need = (size_t)a.nparts * L * D * sizeof(float);
        if (!workspace || workspace_bytes < need) return LS2_ERR_ARG;
    }
    a.coef = coef;
    a.dict = dict;
    a.d_feat = d_feat;
    a.d_coef = d_coef;
    a.d_dict = d_dict;
    a.ws = static_cast<float*>(workspace);
    switch (L) {
        case 32: return launch_decode_bw<32>(a, stream);
        case 64: return launch_decode_bw<64>(a, stream);
        default: return launch_decode_bw<128>(a, stream);
    }
}

extern "C" int ls2_decode_loss_backward_workspace(int64_t m, int32_t L, int32_t D, size_t* bytes) {
    if (!bytes || m < 1 || L < 1 || D < 1) return LS2_ERR_ARG;
    if (!(L == 32 || L == 64) || D % 128 != 0 || D > 512) return LS2_ERR_UNSUPPORTED;
    *bytes = loss_bw_dsum_bytes(m, L, D) + (size_t)kLossBwMaxParts * 2 * sizeof(CSum);
    return LS2_OK;
}

extern "C" int ls2_decode_loss_backward(int64_t m, int32_t L, int32_t D, const float* coef, const float* dict,
                                        const float* target, double* loss, float* d_coef, float* d_dict,
                                        void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (m < 1 || L < 1 || D < 1 || !coef || !dict || !target || !loss || !d_coef || !d_dict || !workspace)
        return LS2_ERR_ARG;
    if (!(L == 32 || L == 64) || D % 128 != 0 || D > 512) return LS2_ERR_UNSUPPORTED;
    if (!aligned16(coef) || !aligned16(dict) || !aligned16(target) || !aligned16(d_coef) || !aligned16(workspace))
        return LS2_ERR_ARG;
    const size_t dsum = loss_bw_dsum_bytes(m, L, D);
    if (workspace_bytes < dsum + (size_t)kLossBwMaxParts * 2 * sizeof(CSum)) return LS2_ERR_ARG;
    DecodeLossBwArgs a;
    a.m = m;
    a.nblocks = (m + 31) / 32;
    a.D = D;
    a.coef = coef;
    a.dict = dict;
    a.target = target;
    a.d_coef = d_coef;
    a.ws = static_cast<float*>(workspace);
    a.partial = reinterpret_cast<CSum*>(static_cast<char*>(workspace) + dsum);
    a.inv_md = loss_inv_md(m, D);
    a.inv_m = loss_inv_m(m);
    const long long grid = loss_bw_grid(m);
    const int rc = L == 32 ? launch_decode_loss_bw<32>(a, grid, stream) : launch_decode_loss_bw<64>(a, grid, stream);
    if (rc != LS2_OK) return rc;
    const int LD = L * D;
    hipLaunchKernelGGL(k_ddict_reduce, dim3((LD + 63) / 64), dim3(1024), 0, stream, a.ws, (int)grid, LD, d_dict);
    LS2_LAUNCH_CHECK();
    return launch_loss_final(a.partial, (int)grid, m, D, loss, stream);
}
