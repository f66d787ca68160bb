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
// alpha >= 1/255 <=> d^T Q d <= 2 ln(255 o), an ellipse whose bounding box
// has half-widths sqrt(2 ln(255 o) Sigma_xx) and sqrt(2 ln(255 o) Sigma_yy)
// with Sigma = Q^-1.  The box is inflated by 1e-3 relative + 0.01 px, far
// beyond the float32 error of the kernel's own alpha, so a dropped entry is
// one that every pixel of the box skips.  Degenerate values are kept.
__device__ __forceinline__ bool may_touch(float u, float v, float A, float B, float C, float o, float x0, float x1,
                                          float y0, float y1) {
    if (!(o >= 1.0f / 255.0f)) return o != o;  // o < 1/255 never blends (NaN kept)
    const float det = A * C - B * B;
    const float t2 = 2.0f * logf(255.0f * o);
    if (!(det > 0.0f) || !(t2 >= 0.0f)) return true;
    const float ex = sqrtf(t2 * C / det) * 1.001f + 0.01f;
    const float ey = sqrtf(t2 * A / det) * 1.001f + 0.01f;
    if (!(ex == ex) || !(ey == ey)) return true;
    return u + ex >= x0 && u - ex <= x1 && v + ey >= y0 && v - ey <= y1;
}

}  // namespace ls2
