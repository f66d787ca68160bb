// ls2_dict_decode: F = W S (Eq. 7), one dense [m x L] x [L x D] product per
// call, on the CDNA4 matrix cores.
//
// The product has only L = 32..128 terms per output, so it is bound by the
// HBM write of F (about 51 flop per byte in bf16), not by the matrix cores.
// The kernel is built around streaming F out at full bandwidth:
//   - persistent workgroups, one wave per D/(waves) feature slice; the wave's
//     slice of S stays in VGPRs for the whole kernel (read once);
//   - per block of 32 pixels each wave computes the transposed tile
//     F^T[features x pixels] so that every lane ends up holding 4 consecutive
//     features of one pixel, which it writes as one 8/16-byte LDS store;
//   - the workgroup then writes the 32 x D tile to HBM as contiguous rows
//     (every store instruction covers whole 1-2 KB rows).
// bf16 compute: v_mfma_f32_32x32x16_bf16 (operands rounded to nearest even).
// f32 compute:  v_mfma_f32_32x32x2_f32.
#include "ls2_internal.h"

namespace ls2 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4q __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

struct DecodeArgs {
    long long m;
    int D;
    int FC;        // features per workgroup chunk (min(D, 512))
    int nchunks;   // D / FC
    const float* coef;  // float32 map (bfloat16 map: coef16)
    const unsigned short* coef16;
    // relevancy epilogue (bf16 compute, one feature chunk): texts and output
    const float* pos = nullptr;
    const float* neg = nullptr;
    int ntext = 0;
    float tau = 1.0f;
    float* rel = nullptr;
    const float* dict;
    void* feat;
    long long nblocks;
};

__device__ __forceinline__ unsigned pack_bf16x2(float a, float b) { return bf16_pair(a, b); }

// Coefficient loads of one 32-pixel block (zeros past the end), issued ahead
// of use so they overlap the previous block's work.
// Unconditional variant: out-of-range blocks and rows read a valid row
// instead (their results are never stored), so every wave issues the same
// number of loads and the waits can be counted exactly.
template <int L>
__device__ __forceinline__ void load_coef_bf16path_clamped(const DecodeArgs& a, long long bk, int col, int half,
                                                           float4 (&raw)[L / 16][2]) {
    long long p = (bk < a.nblocks ? bk : 0) * 32 + col;
    if (p >= a.m) p = a.m - 1;
#pragma unroll
    for (int ks = 0; ks < L / 16; ++ks) {
        const float4* src = reinterpret_cast<const float4*>(a.coef + p * L + ks * 16 + half * 8);
        raw[ks][0] = src[0];
        raw[ks][1] = src[1];
    }
}

template <int L>
__device__ __forceinline__ void load_coef_bf16path(const DecodeArgs& a, long long bk, int col, int half,
                                                   float4 (&raw)[L / 16][2]) {
    const long long p = bk * 32 + col;
    const bool ok = bk < a.nblocks && p < a.m;
#pragma unroll
    for (int ks = 0; ks < L / 16; ++ks) {
        if (ok) {
            const float4* src = reinterpret_cast<const float4*>(a.coef + p * L + ks * 16 + half * 8);
            raw[ks][0] = src[0];
            raw[ks][1] = src[1];
        } else {
            raw[ks][0] = raw[ks][1] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
}

template <int L>
__device__ __forceinline__ void load_coef_f32path(const DecodeArgs& a, long long bk, int col, int half,
                                                  float4 (&raw)[L / 8]) {
    const long long p = bk * 32 + col;
    const bool ok = bk < a.nblocks && p < a.m;
#pragma unroll
    for (int q = 0; q < L / 8; ++q)
        raw[q] = ok ? reinterpret_cast<const float4*>(a.coef + p * L + half * (L / 2))[q]
                    : make_float4(0.f, 0.f, 0.f, 0.f);
}

// ---------------------------------------------------------------------------
// bf16 compute.  MFMA 32x32x16: A (32 x 16) lane l holds row l%32, k =
// (l/32)*8 + [0,8); B (16 x 32) lane l holds column l%32, same k; C (32 x 32)
// lane l holds column l%32, rows (r/4)*8 + (l/32)*4 + r%4 for register r.
// A = S^T slice (features x k), B = W^T (k x pixels), C = F^T tile.
// Each wave owns 64 features (2 row tiles of 32); a workgroup has FC/64
// waves.  The 32-pixel coefficient tile is loaded once per workgroup, rounded
// to bf16 into a double-buffered LDS tile, and read back as B operands; the
// next tile's loads (at most two float4 per thread) are in flight during the
// current tile's work.  Few registers per wave let 16 waves share a CU, which
// keeps the HBM write stream busy while single waves wait on their memory
// counters.  CB: the coefficient map is already bfloat16 (read as is, the
// same values the float32 map rounds to).
//
// QRY: relevancy epilogue (bf16 feature tile, D <= 512).  While the 32 x D
// tile of F sits in LDS, waves 0 and 1 score its two 16-row halves exactly as
// ls2_query scores a bf16 feature map (the same matrix-core dot products with
// the bf16-rounded texts, the same Gram diagonal for the squared norms, the
// same relevancy function), so the result equals ls2_query on the written map
// bit for bit, without reading the map back.  a.feat may be null: then F is
// not written at all.
constexpr int kTileRowBytes(int L) { return L * 2 + 16; }  // padded bf16 coefficient row
constexpr int kQryTextPad = 8;                             // bf16 text row padding

// LDS bytes of the relevancy epilogue: bf16 texts, text norms, dot tiles, norms
inline size_t qry_lds(int D, int ntext) {
    return (size_t)ntext * (D + kQryTextPad) * 2 + sizeof(float) * (16 + 2 * 16 * 17 + 2 * 16);
}

template <int L, bool OUT_BF16, bool CB, bool QRY>
__global__ __launch_bounds__(512) void k_decode_bf16(DecodeArgs a) {
    constexpr int KS = L / 16;   // k-steps
    constexpr int MT = 2;        // 32-feature tiles per wave
    constexpr int OSZ = OUT_BF16 ? 2 : 4;
    constexpr int TROW = kTileRowBytes(L);
    constexpr int TILE = 32 * TROW;  // bytes of one coefficient tile
    constexpr int F4 = 32 * L / 4;   // float4s in a tile
    extern __shared__ float4 smem4[];
    char* tiles = reinterpret_cast<char*>(smem4);  // two coefficient tiles
    char* smem = tiles + 2 * TILE;                 // output staging
    char* qry = smem + 32 * (a.FC * OSZ + 16);     // relevancy epilogue (QRY)

    const int D = a.D;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nthreads = blockDim.x;
    const int chunk = blockIdx.x % a.nchunks;
    const int row_bytes = a.FC * OSZ;
    const int srow = row_bytes + 16;
    const int col = lane & 31, half = lane >> 5;
    const int f_wave = chunk * a.FC + wave * (MT * 32);

    bf16x8 sa[MT][KS];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int f = f_wave + mt * 32 + col;
            bf16x8 v;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (__bf16)a.dict[(size_t)(ks * 16 + half * 8 + e) * D + f];
            sa[mt][ks] = v;
        }

    const int qtstride = (D + kQryTextPad) * 2;
    float* q_tnorm = reinterpret_cast<float*>(qry + a.ntext * qtstride);
    float* q_dots = q_tnorm + 16;         // [2][16 rows][17]
    float* q_nrm = q_dots + 2 * 16 * 17;  // [2][16]
    if (QRY) {
        // texts rounded to bf16 (the matrix-core operands) and their float32 norms
        for (int i = threadIdx.x; i < a.ntext * D; i += nthreads) {
            const int j = i / D, d = i - j * D;
            const float v = j == 0 ? a.pos[d] : a.neg[(size_t)(j - 1) * D + d];
            reinterpret_cast<__bf16*>(qry + j * qtstride)[d] = (__bf16)v;
        }
        if (threadIdx.x < 64) {
            for (int j = 0; j < a.ntext; ++j) {
                float sacc = 0.f;
                const float* t = j == 0 ? a.pos : a.neg + (size_t)(j - 1) * D;
                for (int d = threadIdx.x; d < D; d += 64) sacc += t[d] * t[d];
                for (int off = 32; off > 0; off >>= 1) sacc += __shfl_xor(sacc, off);
                if (threadIdx.x == 0) q_tnorm[j] = fmaxf(sqrtf(sacc), 1e-12f);
            }
        }
        // published by the barrier before the first tile's epilogue
    }
    const long long bstep = gridDim.x / a.nchunks;
    long long blk = blockIdx.x / a.nchunks;
    // cooperative tile loads: float4 number i = threadIdx.x + j * nthreads of
    // the tile (row i / (L/4), columns 4 (i % (L/4)) ..); rows past the end
    // read the last row (never stored)
    constexpr int PER = (F4 + 127) / 128;  // float4 per thread, at most (workgroups have >= 128 threads)
    float4 pre[PER];   // 4 float32 coefficients
    uint2 pre16[PER];  // 4 bfloat16 coefficients
    auto load_tile = [&](long long bk) {
        const long long b = bk < a.nblocks ? bk : 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = threadIdx.x + j * nthreads;
            if (i < F4) {
                long long p = b * 32 + i / (L / 4);
                if (p >= a.m) p = a.m - 1;
                if (CB)
                    pre16[j] = reinterpret_cast<const uint2*>(a.coef16 + p * L)[i % (L / 4)];
                else
                    pre[j] = reinterpret_cast<const float4*>(a.coef + p * L)[i % (L / 4)];
            }
        }
    };
    auto store_tile = [&](char* t) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = threadIdx.x + j * nthreads;
            if (i < F4) {
                uint2 v;
                if (CB) {
                    v = pre16[j];
                } else {
                    v.x = pack_bf16x2(pre[j].x, pre[j].y);
                    v.y = pack_bf16x2(pre[j].z, pre[j].w);
                }
                *reinterpret_cast<uint2*>(t + (i / (L / 4)) * TROW + (i % (L / 4)) * 8) = v;
            }
        }
    };
    load_tile(blk);
    store_tile(tiles);
    load_tile(blk + bstep);
    lds_barrier();
    int cur = 0;
    for (; blk < a.nblocks; blk += bstep) {
        const long long p0 = blk * 32;
        const char* t = tiles + cur * TILE;
        // B operands from the tile: pixel col, k = ks*16 + half*8 + [0,8)
        bf16x8 wb[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) wb[ks] = *reinterpret_cast<const bf16x8*>(t + col * TROW + (ks * 16 + half * 8) * 2);
        f32x16 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            acc[mt] = (f32x16){};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa[mt][ks], wb[ks], acc[mt], 0, 0, 0);
        }
        // stage: lane holds pixel col, features f_wave + mt*32 + g*8 + half*4 + [0,4)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int f = f_wave - chunk * a.FC + mt * 32 + g * 8 + half * 4;  // within the chunk
                char* dst = smem + col * srow + f * OSZ;
                if (OUT_BF16) {
                    uint2 v;
                    v.x = pack_bf16x2(acc[mt][4 * g], acc[mt][4 * g + 1]);
                    v.y = pack_bf16x2(acc[mt][4 * g + 2], acc[mt][4 * g + 3]);
                    *reinterpret_cast<uint2*>(dst) = v;
                } else {
                    *reinterpret_cast<float4*>(dst) =
                        make_float4(acc[mt][4 * g], acc[mt][4 * g + 1], acc[mt][4 * g + 2], acc[mt][4 * g + 3]);
                }
            }
        // the next tile goes to the other buffer (its last readers finished
        // before the previous barrier)
        store_tile(tiles + (cur ^ 1) * TILE);
        lds_barrier();
        load_tile(blk + 2 * bstep);
        // write the 32 x FC tile as contiguous rows: 32 rows x FC*OSZ/16
        // vectors over FC threads, exactly 2*OSZ per thread (unconditional: a
        // partial last block re-stores its final vector)
        const int chunks_per_row = row_bytes / 16;
        const long long rows = (a.m - p0) < 32 ? (a.m - p0) : 32;
        const int nvec = (int)rows * chunks_per_row;
        const long long out_row = (long long)D * OSZ;
        if (!QRY || a.feat) {
            char* out = reinterpret_cast<char*>(a.feat) + p0 * out_row + (long long)chunk * row_bytes;
#pragma unroll
            for (int it = 0; it < 2 * OSZ; ++it) {
                const int c = min((int)threadIdx.x + it * nthreads, nvec - 1);
                const int r = c / chunks_per_row, q = c - r * chunks_per_row;
                const f32x4v v = *reinterpret_cast<const f32x4v*>(smem + r * srow + q * 16);
                __builtin_nontemporal_store(v, reinterpret_cast<f32x4v*>(out + (long long)r * out_row + q * 16));
            }
        }
        if (QRY && wave < 2) {
            // rows 16 wave .. 16 wave + 15 of the tile: A = F rows (lane: row
            // r16, features ks*32 + g*8 ..), B = text columns (lane: text r16)
            const int r16 = lane & 15, g = lane >> 4;
            const bool tcol = r16 < a.ntext;
            const bf16x8 zero8 = {};
            f32x4q dacc = {0.f, 0.f, 0.f, 0.f}, gram = {0.f, 0.f, 0.f, 0.f};
            const char* frow = smem + (16 * wave + r16) * srow;
            for (int ks = 0; ks < D / 32; ++ks) {
                const bf16x8 fa = *reinterpret_cast<const bf16x8*>(frow + (ks * 32 + g * 8) * 2);
                const bf16x8 tb = tcol ? *reinterpret_cast<const bf16x8*>(qry + r16 * qtstride + (ks * 32 + g * 8) * 2)
                                       : zero8;
                dacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, tb, dacc, 0, 0, 0);
                gram = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fa, gram, 0, 0, 0);
            }
            float* dw = q_dots + wave * 16 * 17;
            float* nw = q_nrm + wave * 16;
            const int i = r16 - g * 4;  // diagonal of the Gram tile: row g*4 + i == column r16
            if (i >= 0 && i < 4) nw[r16] = gram[i];
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) dw[(g * 4 + ii) * 17 + r16] = dacc[ii];
            wave_lds_order();
            if (lane < 16) {
                const long long row = p0 + 16 * wave + lane;
                if (row < a.m) a.rel[row] = lerf_relevancy(dw + lane * 17, nw[lane], q_tnorm, a.ntext, a.tau);
            }
        }
        lds_barrier();
        cur ^= 1;
    }
}

// ---------------------------------------------------------------------------
// f32 compute.  MFMA 32x32x2 f32: A (32 x 2) lane l holds row l%32, k = l/32;
// B (2 x 32) lane l holds column l%32, k = l/32; C as above.  The reduction
// index is permuted so that lane half h covers k in [h*L/2, (h+1)*L/2): step s
// pairs k = s (half 0) with k = L/2 + s (half 1), letting each lane read its
// pixel's coefficients as contiguous float4s.
//
// Every wave works on its own: it owns one 64-feature slice of S (2 row
// tiles, in VGPRs) and walks its own sequence of 32-pixel blocks, staging
// each 32 x 64 result in a private LDS slice and writing it as 256-byte (128
// for bf16 output) row segments.  With no workgroup barrier the waves that
// share a SIMD drift into different phases, so one wave's matrix-core chain
// runs while another stages and stores: the matrix cores are the bound.
constexpr int kF32Waves = 8;  // waves per workgroup (independent)

template <int L, bool OUT_BF16>
__global__ __launch_bounds__(kF32Waves * 64) void k_decode_f32(DecodeArgs a) {
    constexpr int KS = L / 2;
    constexpr int MT = 2;
    constexpr int OSZ = OUT_BF16 ? 2 : 4;
    constexpr int SEG = 64 * OSZ;      // bytes of one pixel's slice
    constexpr int SROW = SEG + 16;     // LDS row (padded against bank conflicts)
    constexpr int U = SEG / 16;        // 16-byte units per pixel slice
    constexpr int PPI = 64 / U;        // pixels per store instruction
    extern __shared__ float4 smem4[];
    const int D = a.D;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    char* st = reinterpret_cast<char*>(smem4) + wave * 32 * SROW;
    const int col = lane & 31, half = lane >> 5;
    const int nfg = D / 64;
    const long long gw = (long long)blockIdx.x * kF32Waves + wave;
    const int fg = (int)(gw % nfg);
    const long long bstep = (long long)gridDim.x * kF32Waves / nfg;
    long long blk = gw / nfg;
    const int f0 = fg * 64;

    float sa[MT][KS];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int s = 0; s < KS; ++s) sa[mt][s] = a.dict[(size_t)(half * KS + s) * D + f0 + mt * 32 + col];

    // store phase: instruction i covers pixels PPI i + lane / U, unit lane % U
    const int sp = lane / U, su = lane % U;
    float4 raw[KS / 4];
    load_coef_f32path<L>(a, blk, col, half, raw);
    for (; blk < a.nblocks; blk += bstep) {
        const long long p0 = blk * 32;
        float wv[KS];
#pragma unroll
        for (int q = 0; q < KS / 4; ++q) {
            wv[4 * q] = raw[q].x; wv[4 * q + 1] = raw[q].y; wv[4 * q + 2] = raw[q].z; wv[4 * q + 3] = raw[q].w;
        }
        load_coef_f32path<L>(a, blk + bstep, col, half, raw);  // the next block's, during this one
        f32x16 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            acc[mt] = (f32x16){};
#pragma unroll
            for (int s = 0; s < KS; ++s) acc[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[mt][s], wv[s], acc[mt], 0, 0, 0);
        }
        // lane holds pixel col, features mt*32 + g*8 + half*4 + [0,4) of the slice
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                char* dst = st + col * SROW + (mt * 32 + g * 8 + half * 4) * OSZ;
                if (OUT_BF16) {
                    *reinterpret_cast<uint2*>(dst) = make_uint2(pack_bf16x2(acc[mt][4 * g], acc[mt][4 * g + 1]),
                                                                pack_bf16x2(acc[mt][4 * g + 2], acc[mt][4 * g + 3]));
                } else {
                    *reinterpret_cast<float4*>(dst) =
                        make_float4(acc[mt][4 * g], acc[mt][4 * g + 1], acc[mt][4 * g + 2], acc[mt][4 * g + 3]);
                }
            }
        wave_lds_order();
        f32x4v v[32 / PPI];
#pragma unroll
        for (int i = 0; i < 32 / PPI; ++i)
            v[i] = *reinterpret_cast<const f32x4v*>(st + (PPI * i + sp) * SROW + su * 16);
        char* out = reinterpret_cast<char*>(a.feat) + (p0 + sp) * (long long)D * OSZ + (long long)f0 * OSZ + su * 16;
#pragma unroll
        for (int i = 0; i < 32 / PPI; ++i)
            if (p0 + PPI * i + sp < a.m)
                __builtin_nontemporal_store(
                    v[i], reinterpret_cast<f32x4v*>(out + (long long)(PPI * i) * D * OSZ));
        wave_lds_order();  // the slice's reads are done before the next block overwrites it
    }
}

// Workgroups of `kernel` that fit on one CU at once (registers, LDS, waves):
// persistent grids are sized to exactly fill the chip, so no workgroup waits
// for a second round at reduced occupancy.
static int resident_per_cu(const void* kernel, int threads, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds) != hipSuccess || nb < 1) nb = 1;
    return nb;
}

static int g_num_cus = 0;

static int num_cus() {
    if (g_num_cus == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        g_num_cus = n;
    }
    return g_num_cus;
}

// ---------------------------------------------------------------------------
// Decode fused with the feature loss (float32 compute).  The workgroup's
// D/64 waves each own a 64-feature slice of S (in VGPRs) and compute the same
// 32-pixel block; F never leaves the matrix-core accumulators.  Each wave
// forms its slice's per-pixel partial sums (|F - Y|, F.Y, F.F, Y.Y), the
// waves exchange them through LDS (one barrier per block), and every wave
// then writes its slice of dL/dF.  The target comes in, and dL/dF goes out,
// as 256-byte row segments through a per-wave LDS tile (the accumulator
// layout would touch 32 rows per instruction).  The next block's matrix-core
// chain is issued in two halves around the barrier, so it runs while this
// block's sums, gradient and stores are formed; its coefficients and target
// rows are loaded a block ahead.  The row sums follow the loss's definition
// (ls2_feature_loss) in another summation order, so dL/dF matches decoding
// and then calling the loss up to float32 rounding.  F is written only if
// asked for.
struct DecodeLossArgs {
    DecodeArgs d;
    const float* target;
    float* d_feat;
    float* feat;        // optional
    CSum* partial;      // [gridDim.x][2]
    float inv_md, inv_m;
};

__device__ __forceinline__ float sgn_dl(float e) { return e > 0.f ? 1.f : (e < 0.f ? -1.f : 0.f); }

template <int L>
__global__ __launch_bounds__(512, 1) void k_decode_loss_f32(DecodeLossArgs la) {
    constexpr int KS = L / 2;
    constexpr int MT = 2;
    constexpr int SROW = 64 * 4 + 16;  // LDS row of a wave's tile: 64 floats, padded
    extern __shared__ float4 smem4[];
    __shared__ float4 red[2][8][32];  // per block parity, wave, pixel: (l1, fy, ff, yy) over the wave's 64 features
    __shared__ CSum lred[2][64];
    const DecodeArgs& a = la.d;
    const int D = a.D;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int col = lane & 31, half = lane >> 5;
    const int f_wave = wave * (MT * 32);
    const float inv_md = la.inv_md, inv_m = la.inv_m;
    char* const tile = reinterpret_cast<char*>(smem4) + wave * 32 * SROW;  // this wave's 32 x 64 staging tile
    const int sp = lane >> 4, su = lane & 15;  // row-segment access: rows 4 i + sp, 16-byte unit su
    CSum l1_acc{}, lc_acc{};

    float sa[MT][KS];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int s = 0; s < KS; ++s) sa[mt][s] = a.dict[(size_t)(half * KS + s) * D + f_wave + mt * 32 + col];

    auto load_coef = [&](long long bk, float (&wv)[KS]) {
        float4 raw[KS / 4];
        load_coef_f32path<L>(a, bk, col, half, raw);
#pragma unroll
        for (int q = 0; q < KS / 4; ++q) {
            wv[4 * q] = raw[q].x; wv[4 * q + 1] = raw[q].y; wv[4 * q + 2] = raw[q].z; wv[4 * q + 3] = raw[q].w;
        }
    };
    // the target's 32 x 64 slice of block bk as 256-byte row segments
    auto load_target_rows = [&](long long bk, f32x4v (&yr)[8]) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const long long row = bk * 32 + 4 * i + sp;
            yr[i] = (bk < a.nblocks && row < a.m)
                        ? __builtin_nontemporal_load(reinterpret_cast<const f32x4v*>(la.target + row * D + f_wave) + su)
                        : (f32x4v){0.f, 0.f, 0.f, 0.f};
        }
    };

    long long blk = blockIdx.x;
    const long long bstep = gridDim.x;
    float wv[KS];
    f32x16 acc[MT];
    load_coef(blk, wv);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        acc[mt] = (f32x16){};
#pragma unroll
        for (int s = 0; s < KS; ++s) acc[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[mt][s], wv[s], acc[mt], 0, 0, 0);
    }
    load_coef(blk + bstep, wv);
    f32x4v yr[8];
    load_target_rows(blk, yr);
    int cur = 0;
    for (; blk < a.nblocks; blk += bstep) {
        const long long row = blk * 32 + col;
        const bool rok = row < a.m;
        // the target rows through the tile into the accumulator layout
#pragma unroll
        for (int i = 0; i < 8; ++i) *reinterpret_cast<f32x4v*>(tile + (4 * i + sp) * SROW + su * 16) = yr[i];
        load_target_rows(blk + bstep, yr);  // the next block's rows: a whole block to arrive
        wave_lds_order();
        // the target is read from the tile where it is used (accumulator layout)
        auto ytile = [&](int mt, int g) -> float4* {
            return reinterpret_cast<float4*>(tile + col * SROW + (mt * 32 + g * 8 + half * 4) * 4);
        };
        f32x16 nacc[MT];
        // next block, first feature tile: its matrix-core chain overlaps this block's partial sums
        nacc[0] = (f32x16){};
#pragma unroll
        for (int s = 0; s < KS; ++s) nacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[0][s], wv[s], nacc[0], 0, 0, 0);
        float l1 = 0.f, fy = 0.f, ff = 0.f, yy = 0.f;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const float f0 = acc[mt][4 * g], f1 = acc[mt][4 * g + 1], f2 = acc[mt][4 * g + 2], f3 = acc[mt][4 * g + 3];
                const float4 yv = *ytile(mt, g);
                l1 += fabsf(f0 - yv.x) + fabsf(f1 - yv.y) + fabsf(f2 - yv.z) + fabsf(f3 - yv.w);
                fy = fmaf(f0, yv.x, fmaf(f1, yv.y, fmaf(f2, yv.z, fmaf(f3, yv.w, fy))));
                ff = fmaf(f0, f0, fmaf(f1, f1, fmaf(f2, f2, fmaf(f3, f3, ff))));
                yy = fmaf(yv.x, yv.x, fmaf(yv.y, yv.y, fmaf(yv.z, yv.z, fmaf(yv.w, yv.w, yy))));
            }
        // the two lane halves hold the same pixel's other 32 features
        l1 += __shfl_xor(l1, 32);
        fy += __shfl_xor(fy, 32);
        ff += __shfl_xor(ff, 32);
        yy += __shfl_xor(yy, 32);
        if (half == 0) red[cur][wave][col] = make_float4(l1, fy, ff, yy);
        __syncthreads();
        // next block, second feature tile: overlaps this block's gradient and stores
        nacc[1] = (f32x16){};
#pragma unroll
        for (int s = 0; s < KS; ++s) nacc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[1][s], wv[s], nacc[1], 0, 0, 0);
        load_coef(blk + 2 * bstep, wv);  // the operand registers are free once the chain has issued
        float4 t = red[cur][0][col];
        for (int w = 1; w < nwaves; ++w) {
            const float4 u = red[cur][w][col];
            t.x += u.x; t.y += u.y; t.z += u.z; t.w += u.w;
        }
        const float nf = sqrtf(t.z), ny = sqrtf(t.w);
        const float gf = fmaxf(nf, 1e-12f), gy = fmaxf(ny, 1e-12f);
        const float cs = t.y / (gf * gy);
        if (wave == 0 && half == 0 && rok) {
            l1_acc.add(t.x);
            lc_acc.add(1.0f - cs);
        }
        const float ay = inv_m / (gf * gy);
        const float bf = nf > 1e-12f ? inv_m * t.y / (nf * nf * nf * gy) : 0.f;
        // dL/dF into the tile (the target is in registers by now), out as row segments
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const float f0 = acc[mt][4 * g], f1 = acc[mt][4 * g + 1], f2 = acc[mt][4 * g + 2], f3 = acc[mt][4 * g + 3];
                const float4 yv = *ytile(mt, g);
                float4 o;
                o.x = sgn_dl(f0 - yv.x) * inv_md - ay * yv.x + bf * f0;
                o.y = sgn_dl(f1 - yv.y) * inv_md - ay * yv.y + bf * f1;
                o.z = sgn_dl(f2 - yv.z) * inv_md - ay * yv.z + bf * f2;
                o.w = sgn_dl(f3 - yv.w) * inv_md - ay * yv.w + bf * f3;
                *ytile(mt, g) = o;  // in place: this lane alone reads and writes these 16 bytes
            }
        wave_lds_order();
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const long long r = blk * 32 + 4 * i + sp;
            const f32x4v v = *reinterpret_cast<const f32x4v*>(tile + (4 * i + sp) * SROW + su * 16);
            if (r < a.m) __builtin_nontemporal_store(v, reinterpret_cast<f32x4v*>(la.d_feat + r * D + f_wave) + su);
        }
        if (la.feat) {  // F as well: the same way
            wave_lds_order();
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    *reinterpret_cast<float4*>(tile + col * SROW + (mt * 32 + g * 8 + half * 4) * 4) =
                        make_float4(acc[mt][4 * g], acc[mt][4 * g + 1], acc[mt][4 * g + 2], acc[mt][4 * g + 3]);
            wave_lds_order();
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const long long r = blk * 32 + 4 * i + sp;
                const f32x4v v = *reinterpret_cast<const f32x4v*>(tile + (4 * i + sp) * SROW + su * 16);
                if (r < a.m) __builtin_nontemporal_store(v, reinterpret_cast<f32x4v*>(la.feat + r * D + f_wave) + su);
            }
        }
        wave_lds_order();  // the tile's reads are done before the next target rows land in it
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = nacc[mt];
        cur ^= 1;  // red[cur] is rewritten two blocks later, after every wave passed the next barrier
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
        la.partial[2 * blockIdx.x] = s0;
        la.partial[2 * blockIdx.x + 1] = s1;
    }
}

constexpr int kDecodeLossMaxBlocks = 4096;

template <int L>
static int launch_decode_loss(DecodeLossArgs la, hipStream_t stream) {
    DecodeArgs& a = la.d;
    a.FC = a.D;
    a.nchunks = 1;
    const size_t lds = (size_t)(a.D / 64) * 32 * (64 * 4 + 16);  // one staging tile per wave
    static bool attr = false;
    if (!attr) {
        if (hipFuncSetAttribute((const void*)k_decode_loss_f32<L>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                150 * 1024) != hipSuccess)
            return LS2_ERR_DEVICE;
        attr = true;
    }
    const int threads = (a.D / 64) * 64;
    long long grid = (long long)num_cus() * resident_per_cu((const void*)k_decode_loss_f32<L>, threads, lds);
    if (grid > a.nblocks) grid = a.nblocks;
    if (grid > kDecodeLossMaxBlocks) grid = kDecodeLossMaxBlocks;
    hipLaunchKernelGGL((k_decode_loss_f32<L>), dim3((unsigned)grid), dim3(threads), lds, stream, la);
    LS2_LAUNCH_CHECK();
    return (int)grid;
}

template <int L, bool OB, bool CB, bool QRY = false>
static int launch_decode_bf16(const DecodeArgs& a, hipStream_t stream) {
    const int osz = OB ? 2 : 4;
    const size_t lds = (size_t)32 * (a.FC * osz + 16);
    const long long need = a.nblocks * a.nchunks;
    const int threads = (a.FC / 64) * 64;
    const size_t lds_b = lds + 2 * (size_t)32 * kTileRowBytes(L) + (QRY ? qry_lds(a.D, a.ntext) : 0);
    const void* kern = (const void*)k_decode_bf16<L, OB, CB, QRY>;
    static bool attr = false;
    if (!attr) {
        if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024) != hipSuccess)
            return LS2_ERR_DEVICE;
        attr = true;
    }
    long long grid = (long long)num_cus() * resident_per_cu(kern, threads, lds_b);
    grid -= grid % a.nchunks;
    if (grid < a.nchunks) grid = a.nchunks;
    if (grid > need) grid = need;
    hipLaunchKernelGGL((k_decode_bf16<L, OB, CB, QRY>), dim3((unsigned)grid), dim3(threads), lds_b, stream, a);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}

template <int L, bool OB>
static int launch_decode(const DecodeArgs& a0, int compute, bool cb, hipStream_t stream) {
    DecodeArgs a = a0;
    a.FC = a.D < 512 ? a.D : 512;
    a.nchunks = a.D / a.FC;
    const int osz = OB ? 2 : 4;
    const size_t lds = (size_t)32 * (a.FC * osz + 16);
    const long long need = a.nblocks * a.nchunks;
    auto grid_for = [&](const void* kernel, int threads) {
        long long grid = (long long)num_cus() * resident_per_cu(kernel, threads, lds);
        grid -= grid % a.nchunks;
        if (grid < a.nchunks) grid = a.nchunks;
        return grid > need ? need : grid;
    };
    if (compute == LS2_BF16) {
        return cb ? launch_decode_bf16<L, OB, true>(a, stream) : launch_decode_bf16<L, OB, false>(a, stream);
    } else {
        // independent waves: every wave owns a 64-feature slice and its own
        // 32-pixel blocks; the grid is a whole number of feature groups
        const int nfg = a.D / 64;
        const size_t lds32 = (size_t)kF32Waves * 32 * (64 * osz + 16);
        const void* kern = (const void*)k_decode_f32<L, OB>;
        long long grid = (long long)num_cus() * resident_per_cu(kern, kF32Waves * 64, lds32);
        long long waves = grid * kF32Waves;
        waves -= waves % nfg;
        if (waves < nfg) waves = nfg;
        if (waves > a.nblocks * nfg) waves = a.nblocks * nfg;
        // whole workgroups with a whole number of feature groups (nfg is a power of two)
        while ((waves % kF32Waves) != 0 || (waves % nfg) != 0) ++waves;
        grid = waves / kF32Waves;
        hipLaunchKernelGGL((k_decode_f32<L, OB>), dim3((unsigned)grid), dim3(kF32Waves * 64), lds32, stream, a);
    }
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_dict_decode(int64_t m, int32_t L, int32_t D, const void* coef, int32_t coef_dtype,
                               const float* dict, int32_t compute, int32_t out_dtype, void* feat, hipStream_t stream) {
    if (m < 0 || L < 1 || D < 1 || !dict || !feat || !coef) return LS2_ERR_ARG;
    if ((compute != LS2_F32 && compute != LS2_BF16) || (out_dtype != LS2_F32 && out_dtype != LS2_BF16) ||
        (coef_dtype != LS2_F32 && coef_dtype != LS2_BF16))
        return LS2_ERR_ARG;
    if (!(L == 32 || L == 64 || L == 128) || D % 128 != 0 || (D > 512 && D != 1024)) return LS2_ERR_UNSUPPORTED;
    if (coef_dtype == LS2_BF16 && compute != LS2_BF16) return LS2_ERR_UNSUPPORTED;
    if (!aligned16(coef) || !aligned16(feat)) return LS2_ERR_ARG;
    if (m == 0) return LS2_OK;
    const bool cb = coef_dtype == LS2_BF16;
    DecodeArgs a;
    a.m = m;
    a.D = D;
    a.coef = cb ? nullptr : static_cast<const float*>(coef);
    a.coef16 = cb ? static_cast<const unsigned short*>(coef) : nullptr;
    a.dict = dict;
    a.feat = feat;
    a.nblocks = (m + 31) / 32;
    const bool ob = out_dtype == LS2_BF16;
    switch (L) {
        case 32:
            return ob ? launch_decode<32, true>(a, compute, cb, stream) : launch_decode<32, false>(a, compute, cb, stream);
        case 64:
            return ob ? launch_decode<64, true>(a, compute, cb, stream) : launch_decode<64, false>(a, compute, cb, stream);
        default:
            return ob ? launch_decode<128, true>(a, compute, cb, stream)
                      : launch_decode<128, false>(a, compute, cb, stream);
    }
}


extern "C" int ls2_dict_decode_query(int64_t m, int32_t L, int32_t D, const void* coef, int32_t coef_dtype,
                                     const float* dict, void* feat, const float* pos, int32_t n_neg, const float* neg,
                                     float tau, float* relevancy, hipStream_t stream) {
    if (m < 0 || L < 1 || D < 1 || !coef || !dict || !pos || !neg || !relevancy || n_neg < 1) return LS2_ERR_ARG;
    if (coef_dtype != LS2_F32 && coef_dtype != LS2_BF16) return LS2_ERR_ARG;
    if (!(L == 32 || L == 64 || L == 128) || D % 128 != 0 || D > 512 || n_neg > 8) return LS2_ERR_UNSUPPORTED;
    if (!aligned16(coef) || !aligned16(feat)) return LS2_ERR_ARG;
    if (m == 0) return LS2_OK;
    const bool cb = coef_dtype == LS2_BF16;
    DecodeArgs a;
    a.m = m;
    a.D = D;
    a.FC = D;
    a.nchunks = 1;
    a.coef = cb ? nullptr : static_cast<const float*>(coef);
    a.coef16 = cb ? static_cast<const unsigned short*>(coef) : nullptr;
    a.dict = dict;
    a.feat = feat;
    a.nblocks = (m + 31) / 32;
    a.pos = pos;
    a.neg = neg;
    a.ntext = 1 + n_neg;
    a.tau = tau;
    a.rel = relevancy;
    switch (L) {
        case 32: return cb ? launch_decode_bf16<32, true, true, true>(a, stream) : launch_decode_bf16<32, true, false, true>(a, stream);
        case 64: return cb ? launch_decode_bf16<64, true, true, true>(a, stream) : launch_decode_bf16<64, true, false, true>(a, stream);
        default: return cb ? launch_decode_bf16<128, true, true, true>(a, stream) : launch_decode_bf16<128, true, false, true>(a, stream);
    }
}

extern "C" int ls2_decode_feature_loss_workspace(int64_t m, int32_t D, size_t* bytes) {
    if (!bytes || m < 0 || D < 1) return LS2_ERR_ARG;
    *bytes = (size_t)kDecodeLossMaxBlocks * 2 * sizeof(CSum);
    return LS2_OK;
}

extern "C" int ls2_decode_feature_loss(int64_t m, int32_t L, int32_t D, const float* coef, const float* dict,
                                       const float* target, double* loss, float* d_feat, float* feat,
                                       void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (m < 1 || L < 1 || D < 1 || !coef || !dict || !target || !loss || !d_feat || !workspace) return LS2_ERR_ARG;
    if (workspace_bytes < (size_t)kDecodeLossMaxBlocks * 2 * sizeof(CSum)) return LS2_ERR_ARG;
    if (!(L == 32 || L == 64) || D % 128 != 0 || D > 512) return LS2_ERR_UNSUPPORTED;
    DecodeLossArgs la;
    la.d.m = m;
    la.d.D = D;
    la.d.coef = coef;
    la.d.coef16 = nullptr;
    la.d.dict = dict;
    la.d.feat = nullptr;
    la.d.nblocks = (m + 31) / 32;
    la.target = target;
    la.d_feat = d_feat;
    la.feat = feat;
    la.partial = static_cast<CSum*>(workspace);
    la.inv_md = loss_inv_md(m, D);
    la.inv_m = loss_inv_m(m);
    int grid;
    grid = L == 32 ? launch_decode_loss<32>(la, stream) : launch_decode_loss<64>(la, stream);
    if (grid < 0) return grid;
    return launch_loss_final(la.partial, grid, m, D, loss, stream);
}
