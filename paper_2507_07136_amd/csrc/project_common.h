// EWA projection of one Gaussian (Section 3.1, Eqs. 1-2; EWA splatting as
// cited there), float32, shared by ls2_project and the projecting count pass
// of ls2_project_bin_sort so that both produce the same bits.
#pragma once

#include "ls2_internal.h"

namespace ls2 {

struct ProjOut {
    float u, v, A, B, C, z;
    int r, cnt;  // radius (0: culled) and the number of tiles its rectangle covers
};

// The inputs of one Gaussian, loaded apart from the arithmetic so that a
// thread can issue the loads of several Gaussians at once.
struct ProjIn {
    float mx, my, mz, s0, s1, s2, qw, qx, qy, qz;
};

__device__ __forceinline__ ProjIn load_proj(const float* __restrict__ means, const float* __restrict__ scales,
                                            const float* __restrict__ quats, int i) {
    return ProjIn{means[3 * i],     means[3 * i + 1],  means[3 * i + 2],  scales[3 * i],     scales[3 * i + 1],
                  scales[3 * i + 2], quats[4 * i],      quats[4 * i + 1],  quats[4 * i + 2],  quats[4 * i + 3]};
}

__device__ __forceinline__ ProjOut project_in(const CamK& cam, const ProjIn& g) {
    // multiply-adds are fused only inside one expression, never by the code
    // generator across statements: the result then does not depend on the
    // kernel this is inlined into, so every caller produces the same bits
#pragma clang fp contract(on)
    const float mx = g.mx, my = g.my, mz = g.mz;
    // camera-space mean p = R mu + t
    const float x = cam.R[0] * mx + cam.R[1] * my + cam.R[2] * mz + cam.t[0];
    const float y = cam.R[3] * mx + cam.R[4] * my + cam.R[5] * mz + cam.t[1];
    const float z = cam.R[6] * mx + cam.R[7] * my + cam.R[8] * mz + cam.t[2];

    float u = 0.f, v = 0.f, A = 0.f, B = 0.f, C = 0.f, zout = 0.f;
    int r = 0, cnt = 0;
    bool ok = (z > cam.znear) && isfinite(x) && isfinite(y);
    if (ok) {
        // Eq. 2: Sigma = R(q) S S^T R(q)^T; in camera space
        // Sigma_c = (Rc R(q) S)(Rc R(q) S)^T.
        float qw = g.qw, qx = g.qx, qy = g.qy, qz = g.qz;
        const float qn = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
        qw *= qn; qx *= qn; qy *= qn; qz *= qn;
        const float Rq[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                             2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                             2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
        const float s[3] = {g.s0, g.s1, g.s2};
        float T[9];  // Rc * Rq * diag(s)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                T[3 * a + b] = (cam.R[3 * a] * Rq[b] + cam.R[3 * a + 1] * Rq[3 + b] + cam.R[3 * a + 2] * Rq[6 + b]) * s[b];
        // EWA: local affine Jacobian of the perspective map at p; G = J T
        const float iz = 1.0f / z;
        const float j00 = cam.fx * iz, j02 = -cam.fx * x * iz * iz;
        const float j11 = cam.fy * iz, j12 = -cam.fy * y * iz * iz;
        float g0[3], g1[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            g0[b] = j00 * T[b] + j02 * T[6 + b];
            g1[b] = j11 * T[3 + b] + j12 * T[6 + b];
        }
        const float a = g0[0] * g0[0] + g0[1] * g0[1] + g0[2] * g0[2] + 0.3f;
        const float bb = g0[0] * g1[0] + g0[1] * g1[1] + g0[2] * g1[2];
        const float c = g1[0] * g1[0] + g1[1] * g1[1] + g1[2] * g1[2] + 0.3f;
        const float det = a * c - bb * bb;
        ok = det > 0.f && isfinite(det);
        if (ok) {
            const float mid = 0.5f * (a + c);
            const float disc = fmaxf(mid * mid - det, 0.f);
            const float ext = 3.0f * sqrtf(mid + sqrtf(disc));
            ok = ext <= 1e7f;
            if (ok) {
                r = (int)ceilf(ext);
                u = cam.fx * x * iz + cam.cx;
                v = cam.fy * y * iz + cam.cy;
                int x0, y0, x1, y1;
                ok = tile_rect(u, v, r, cam.tx, cam.ty, x0, y0, x1, y1);
                if (ok) {
                    const float idet = 1.0f / det;
                    A = c * idet;
                    B = -bb * idet;
                    C = a * idet;
                    zout = z;
                    cnt = (x1 - x0 + 1) * (y1 - y0 + 1);
                }
            }
        }
    }
    if (!ok) {
        u = v = A = B = C = zout = 0.f;
        r = 0;
        cnt = 0;
    }
    return ProjOut{u, v, A, B, C, zout, r, cnt};
}

__device__ __forceinline__ ProjOut project_one(const CamK& cam, const float* __restrict__ means,
                                               const float* __restrict__ scales, const float* __restrict__ quats,
                                               int i) {
    return project_in(cam, load_proj(means, scales, quats, i));
}

// The projection's outputs for Gaussian i (tiles_touched optional).
__device__ __forceinline__ void store_proj(const ProjOut& o, int i, float* __restrict__ mean2d,
                                           float* __restrict__ conic, float* __restrict__ depth,
                                           int* __restrict__ radius, int* __restrict__ touched) {
    reinterpret_cast<float2*>(mean2d)[i] = make_float2(o.u, o.v);
    conic[3 * i] = o.A;
    conic[3 * i + 1] = o.B;
    conic[3 * i + 2] = o.C;
    depth[i] = o.z;
    radius[i] = o.r;
    if (touched) touched[i] = o.cnt;
}

}  // namespace ls2
