// Per-Gaussian helpers shared by the compositing forward and backward kernels,
// so both evaluate alpha with the same instructions and take the same
// decisions.
#pragma once

#include "ls2_internal.h"

namespace ls2 {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// Exponent (base 2) of the Gaussian at offset (dx, dy) given the conic scaled
// to A2 = -0.5 A log2(e), B2 = -B log2(e), C2 = -0.5 C log2(e).
__device__ __forceinline__ float gauss_power2(float A2, float B2, float C2, float dx, float dy) {
    return fmaf(dx, fmaf(A2, dx, B2 * dy), C2 * dy * dy);
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Can a Gaussian with mean (u, v), conic (A, B, C) and opacity o reach
// alpha >= 1/255 at any pixel centre of the box [x0, x1] x [y0, y1]?
// alpha >= 1/255 <=> q(d) = d^T Q d <= t2 = 2 ln(255 o), Q = [[A, B], [B, C]].
// q is convex, so its minimum over the box is 0 if the mean lies inside and
// otherwise lies on an edge; on an edge with fixed dx the minimum over dy is
// at dy = -B dx / C clamped to the edge (symmetrically for fixed dy).  The
// test compares that exact minimum against t2 inflated by 2e-3 relative plus
// 0.02, far beyond the float32 error of the kernel's own alpha, so a dropped
// entry is one that every pixel of the box skips.  Degenerate values are kept.
__device__ __forceinline__ bool may_touch(float u, float v, float A, float B, float C, float o, float x0, float x1,
                                          float y0, float y1) {
    if (!(o >= 1.0f / 255.0f)) return o != o;  // o < 1/255 never blends (NaN kept)
    const float t2 = 2.0f * logf(255.0f * o);
    if (!(A > 0.0f) || !(C > 0.0f) || !(A * C - B * B > 0.0f) || !(t2 >= 0.0f)) return true;
    const float dx0 = x0 - u, dx1 = x1 - u, dy0 = y0 - v, dy1 = y1 - v;
    if (dx0 <= 0.0f && dx1 >= 0.0f && dy0 <= 0.0f && dy1 >= 0.0f) return true;  // mean inside the box
    const float bc = B / C, ba = B / A;
    auto q = [&](float dx, float dy) { return fmaf(A * dx, dx, fmaf(2.0f * B * dx, dy, C * dy * dy)); };
    auto on_x = [&](float dx) { return q(dx, fminf(fmaxf(-bc * dx, dy0), dy1)); };  // edge dx fixed
    auto on_y = [&](float dy) { return q(fminf(fmaxf(-ba * dy, dx0), dx1), dy); };  // edge dy fixed
    const float m = fminf(fminf(on_x(dx0), on_x(dx1)), fminf(on_y(dy0), on_y(dy1)));
    if (!(m == m)) return true;
    return m <= fmaf(t2, 1.002f, 0.02f);
}

}  // namespace ls2
