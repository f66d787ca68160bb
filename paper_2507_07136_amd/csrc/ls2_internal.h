// Internal helpers of libls2 (device and host).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "ls2.h"

namespace ls2 {

constexpr int kTile = LS2_TILE;

// Camera passed to kernels by value.
struct CamK {
    int W, H, tx, ty;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float znear;
};

inline CamK cam_k(const ls2_camera& c) {
    CamK k;
    k.W = c.width;
    k.H = c.height;
    k.tx = (c.width + kTile - 1) / kTile;
    k.ty = (c.height + kTile - 1) / kTile;
    k.fx = c.fx; k.fy = c.fy; k.cx = c.cx; k.cy = c.cy;
    for (int r = 0; r < 3; ++r) {
        for (int j = 0; j < 3; ++j) k.R[3 * r + j] = c.world_to_cam[4 * r + j];
        k.t[r] = c.world_to_cam[4 * r + 3];
    }
    k.znear = c.znear;
    return k;
}

// A usable camera: image size in [1, 32768]^2, finite intrinsics, and a near
// plane that is finite and positive (sort keys are the bits of a positive
// float32 depth, and z near 0 would make the projection Jacobian blow up).
inline bool cam_valid(const ls2_camera* c) {
    if (!c || c->width <= 0 || c->height <= 0 || c->width > (1 << 15) || c->height > (1 << 15)) return false;
    if (!std::isfinite(c->fx) || !std::isfinite(c->fy) || !std::isfinite(c->cx) || !std::isfinite(c->cy))
        return false;
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(c->world_to_cam[i])) return false;
    return std::isfinite(c->znear) && c->znear > 0.0f;
}

// Tile rectangle [x0,x1] x [y0,y1] of a Gaussian with float32 mean (u, v) and
// integer radius r: [floor((u - r)/16), floor((u + r)/16)] clipped to the
// grid.  Every step is an explicit round-to-nearest float32 operation so the
// decision is identical wherever it is evaluated.  Returns false if empty.
__host__ __device__ inline bool tile_rect(float u, float v, int r, int tx, int ty, int& x0, int& y0,
                                          int& x1, int& y1) {
    const float rf = (float)r;
#if defined(__HIP_DEVICE_COMPILE__)
    float lox = floorf(__fmul_rn(__fsub_rn(u, rf), 0.0625f));
    float hix = floorf(__fmul_rn(__fadd_rn(u, rf), 0.0625f));
    float loy = floorf(__fmul_rn(__fsub_rn(v, rf), 0.0625f));
    float hiy = floorf(__fmul_rn(__fadd_rn(v, rf), 0.0625f));
#else
    float lox = floorf((u - rf) * 0.0625f);
    float hix = floorf((u + rf) * 0.0625f);
    float loy = floorf((v - rf) * 0.0625f);
    float hiy = floorf((v + rf) * 0.0625f);
#endif
    lox = lox < 0.0f ? 0.0f : lox;
    loy = loy < 0.0f ? 0.0f : loy;
    hix = hix > (float)(tx - 1) ? (float)(tx - 1) : hix;
    hiy = hiy > (float)(ty - 1) ? (float)(ty - 1) : hiy;
    if (!(lox <= hix) || !(loy <= hiy)) return false;
    x0 = (int)lox; x1 = (int)hix; y0 = (int)loy; y1 = (int)hiy;
    return true;
}

// Map a linear block index to (work item, slot).  Blocks are dispatched
// round-robin over the 8 XCDs, so block b runs on XCD b % 8.  The remap gives
// each XCD one contiguous range of the linear order: the `per` blocks of one
// work item share an XCD, and spatially adjacent tiles share its L2.  The
// grid must be a multiple of 8; linear indices past the work are returned as
// item >= the caller's item count.
__device__ inline void xcd_remap(int b, int grid, int per, int& item, int& slot) {
    const int per_xcd = grid >> 3;
    const int lin = (b & 7) * per_xcd + (b >> 3);
    item = lin / per;
    slot = lin - item * per;
}

inline int round_up8(int x) { return (x + 7) & ~7; }

// Sum over the 64 lanes of a wave with DPP moves (no LDS round trip).  xor 1
// and xor 2 inside quads, the half-row and row mirrors complete each 16-lane
// row, row broadcasts 15 and 31 add rows 0-2 into row 3: the total is exact
// in lane 63 only.  Every lane must be active.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_add(float v) {
    const int moved = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false);
    return v + __int_as_float(moved);
}

__device__ __forceinline__ float wave_sum_lane63(float v) {
    v = dpp_add<0xb1>(v);          // quad_perm [1,0,3,2]
    v = dpp_add<0x4e>(v);          // quad_perm [2,3,0,1]
    v = dpp_add<0x141>(v);         // row_half_mirror
    v = dpp_add<0x140>(v);         // row_mirror
    v = dpp_add<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
    return v;
}

// LERF relevancy of one feature from its dot products with the texts (index
// 0 the positive, 1.. the negatives), its squared norm and the texts' guarded
// norms: sigmoid(tau (s_q - max_j s_j)) on cosine similarities, the feature
// norm guarded below by 1e-12.
__device__ __forceinline__ float lerf_relevancy(const float* dots, float fnorm2, const float* tnorm, int ntext,
                                                float tau) {
    const float nf = fmaxf(sqrtf(fnorm2), 1e-12f);
    const float sq = dots[0] / (nf * tnorm[0]);
    float smax = -INFINITY;
    for (int j = 1; j < ntext; ++j) smax = fmaxf(smax, dots[j] / (nf * tnorm[j]));
    return 1.0f / (1.0f + expf(-tau * (sq - smax)));
}

// Two floats rounded to bfloat16 (nearest even), packed low / high: one
// v_cvt_pk_bf16_f32 (the same rounding as converting each on its own).
typedef __bf16 bf16x2_i __attribute__((ext_vector_type(2)));
typedef float f32x2_i __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned bf16_pair(float a, float b) {
    const f32x2_i v = {a, b};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2_i));
}

// Compensated float32 sum (Neumaier): s + c holds the running total to about
// twice float32's precision, so a sum over many rows or partials stays within
// a few float32 roundings of the exact sum whatever its length (scalar
// results such as the loss are accumulated this way, not in float64).
// Trivial (usable in LDS); start from CSum{} for zero.
struct CSum {
    float s, c;
    __device__ __forceinline__ void add(float x) {
        const float t = s + x;
        c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    __device__ __forceinline__ void add(const CSum& o) {
        add(o.s);
        c += o.c;
    }
    __device__ __forceinline__ float value() const { return s + c; }
};

// The loss's mean weights 1 / (m D) and 1 / m, rounded once on the host.
inline float loss_inv_md(long long m, int D) { return (float)(1.0 / ((double)m * (double)D)); }
inline float loss_inv_m(long long m) { return (float)(1.0 / (double)m); }

// Final sum of per-workgroup loss partials (two CSum per workgroup: the L1
// and the cosine term) into the scalar loss; defined with ls2_feature_loss.
int launch_loss_final(const CSum* partial, int nblocks, long long m, int D, double* loss, hipStream_t stream);

// LS2_CHECK mode (check.hip): whether it is on, and the scan of n levels K
// code indices against [0, L) that the entry points reading topk_idx run
// first when it is (LS2_ERR_ARG if any lies outside; synchronises stream).
bool check_mode();
int check_code_indices(long long count, int L, const int32_t* topk_idx, hipStream_t stream);

// Host-side check of the 16-byte alignment that float4 accesses need (a null
// pointer passes; null arguments are checked separately).
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// Reduce-scatter of V per-lane values over the 64 lanes of a wave.  Each step
// pairs lane l with the lane that differs in one bit: lanes with the bit
// clear keep the first ceil(n/2) of their n values, lanes with it set the
// rest, each adding its partner's copy.  Bits 5 and 4 use v_permlane32_swap /
// v_permlane16_swap (one swap exchanges a whole pair), bits 3..0 DPP moves
// (row_ror 8, row_half_mirror, quad_perm xor 2, xor 1).  Once one value is
// left the remaining bits are summed as a butterfly.  On return lane l holds
// the wave total of value tr_slot(V, l).index (see below); every lane must be
// active.
template <int BIT>
__device__ __forceinline__ float tr_exchange(float x, float y, int lane) {
    if constexpr (BIT == 5) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else if constexpr (BIT == 4) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else {
        constexpr int CTRL = BIT == 3 ? 0x128 : BIT == 2 ? 0x141 : BIT == 1 ? 0x4e : 0xb1;
        const bool hi = (lane >> BIT) & 1;
        const float send = hi ? x : y;
        const float recv = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), CTRL, 0xf, 0xf, false));
        return (hi ? y : x) + recv;
    }
}

template <int BIT, int V>
__device__ __forceinline__ float tr_reduce(const float (&v)[V], int lane) {
    static_assert(V >= 1 && V <= 64, "tr_reduce: 1..64 values");
    if constexpr (V == 1) {
        if constexpr (BIT >= 0) {
            const float nv[1] = {tr_exchange<BIT>(v[0], v[0], lane)};
            return tr_reduce<BIT - 1, 1>(nv, lane);
        } else {
            return v[0];
        }
    } else {
        static_assert(BIT >= 0, "tr_reduce: more values than lanes");
        constexpr int H = (V + 1) / 2;
        float nv[H];
#pragma unroll
        for (int i = 0; i < H; ++i) nv[i] = tr_exchange<BIT>(v[i], i + H < V ? v[i + H] : 0.0f, lane);
        return tr_reduce<BIT - 1, H>(nv, lane);
    }
}

// Which value lane l ends with after tr_reduce<5, V>: index, whether that
// slot holds a value (not padding), and whether l is the one lane (lowest
// of the butterfly group) that should use it.
struct TrSlot {
    int index;
    bool valid;
    bool leader;
};
__device__ __forceinline__ TrSlot tr_slot(int V, int lane) {
    int base = 0, cnt = V, size = V, bit = 5;
    for (; bit >= 0 && size > 1; --bit) {
        const int h = (size + 1) / 2;
        if ((lane >> bit) & 1) {
            base += h;
            cnt = cnt - h > 0 ? cnt - h : 0;
        } else {
            cnt = cnt < h ? cnt : h;
        }
        size = h;
    }
    // bits bit..0 were summed as a butterfly: every lane of the group holds
    // the total; the group's lowest lane is the leader
    const int rest = bit >= 0 ? ((1 << (bit + 1)) - 1) : 0;
    return TrSlot{base, cnt > 0, (lane & rest) == 0};
}

// The wave sum, broadcast to every lane (as a wave-uniform value).
__device__ __forceinline__ float wave_allsum(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_lane63(v)), 63));
}

// Workgroup barrier that orders LDS only: waits for this wave's outstanding
// LDS operations, then meets the other waves.  Unlike __syncthreads() it does
// not wait for global loads and stores in flight, so streaming stores of one
// tile overlap the work on the next.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// For single-wave workgroups: LDS operations of one wave complete in order,
// so only the compiler must not move LDS accesses across this point.
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

#define LS2_LAUNCH_CHECK()                                              \
    do {                                                                \
        if (hipGetLastError() != hipSuccess) return LS2_ERR_DEVICE;     \
    } while (0)

}  // namespace ls2
