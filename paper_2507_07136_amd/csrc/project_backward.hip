// ls2_project_backward: gradients of the EWA projection (Section 3.1,
// Eqs. 1-2) with respect to the 3D means, scales and quaternions, given the
// gradients of the 2D means and conics.  One thread per Gaussian, float32.
//
// The forward factors the camera-space covariance as T T^T with
// T = R_wc R(q) diag(s) and the screen covariance as G G^T + 0.3 I with
// G = J T.  The chain used here:
//   conic = Sigma2D^-1:   dSigma2D = -conic dConic conic (symmetric form),
//   Sigma2D = G G^T:      dG = 2 dSigma2D G,
//   G = J T:              dJ = dG T^T,  dT = J^T dG,
//   T = R_wc N, N = R(q) diag(s):  dN = R_wc^T dT,
//   N:                    dR(q) = dN diag(s),  ds_b = sum_a dN_ab R(q)_ab,
//   R(q/|q|):             quaternion partials, then the projection through
//                         the normalisation,
//   J(p) and (u, v)(p):   dp, then dmu = R_wc^T dp.
// Culled Gaussians (radius 0) receive zero gradients.
#include "ls2_internal.h"

namespace ls2 {

__global__ __launch_bounds__(256) void k_project_backward(CamK cam, int n, const float* __restrict__ means,
                                                          const float* __restrict__ scales,
                                                          const float* __restrict__ quats,
                                                          const int* __restrict__ radius,
                                                          const float* __restrict__ d_mean2d,
                                                          const float* __restrict__ d_conic,
                                                          float* __restrict__ d_means, float* __restrict__ d_scales,
                                                          float* __restrict__ d_quats) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gm[3] = {0.f, 0.f, 0.f}, gs[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
    if (radius[i] > 0) {
        const float mx = means[3 * i], my = means[3 * i + 1], mz = means[3 * i + 2];
        const float x = cam.R[0] * mx + cam.R[1] * my + cam.R[2] * mz + cam.t[0];
        const float y = cam.R[3] * mx + cam.R[4] * my + cam.R[5] * mz + cam.t[1];
        const float z = cam.R[6] * mx + cam.R[7] * my + cam.R[8] * mz + cam.t[2];

        const float q0 = quats[4 * i], q1 = quats[4 * i + 1], q2 = quats[4 * i + 2], q3 = quats[4 * i + 3];
        const float qn = 1.0f / sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
        const float w = q0 * qn, qx = q1 * qn, qy = q2 * qn, qz = q3 * qn;
        const float Rq[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - w * qz), 2.f * (qx * qz + w * qy),
                             2.f * (qx * qy + w * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - w * qx),
                             2.f * (qx * qz - w * qy), 2.f * (qy * qz + w * qx), 1.f - 2.f * (qx * qx + qy * qy)};
        const float s[3] = {scales[3 * i], scales[3 * i + 1], scales[3 * i + 2]};
        float T[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                T[3 * a + b] = (cam.R[3 * a] * Rq[b] + cam.R[3 * a + 1] * Rq[3 + b] + cam.R[3 * a + 2] * Rq[6 + b]) * s[b];
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
        const float idet = 1.0f / (a * c - bb * bb);
        const float A = c * idet, B = -bb * idet, C = a * idet;

        // conic -> Sigma2D = [[a, b], [b, c]]: d(Sigma^-1) = -Sigma^-1 dSigma Sigma^-1
        const float gA = d_conic[3 * i], gB = d_conic[3 * i + 1], gC = d_conic[3 * i + 2];
        const float ga = -(gA * A * A + gB * A * B + gC * B * B);
        const float gb = -(2.f * gA * A * B + gB * (A * C + B * B) + 2.f * gC * B * C);
        const float gc = -(gA * B * B + gB * B * C + gC * C * C);
        // Sigma2D = G G^T: a = g0.g0, b = g0.g1, c = g1.g1
        float dg0[3], dg1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            dg0[k] = 2.f * ga * g0[k] + gb * g1[k];
            dg1[k] = gb * g0[k] + 2.f * gc * g1[k];
        }
        // G = J T
        float dj00 = 0.f, dj02 = 0.f, dj11 = 0.f, dj12 = 0.f, dT[9];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            dj00 += dg0[k] * T[k];
            dj02 += dg0[k] * T[6 + k];
            dj11 += dg1[k] * T[3 + k];
            dj12 += dg1[k] * T[6 + k];
            dT[k] = j00 * dg0[k];
            dT[3 + k] = j11 * dg1[k];
            dT[6 + k] = j02 * dg0[k] + j12 * dg1[k];
        }
        // T = R_wc N
        float dR[9];
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const float dN = cam.R[m] * dT[b] + cam.R[3 + m] * dT[3 + b] + cam.R[6 + m] * dT[6 + b];
                dR[3 * m + b] = dN * s[b];
                gs[b] += dN * Rq[3 * m + b];
            }
        // R(w, x, y, z): partial derivatives of each entry
        const float dw = 2.f * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
        const float dx = 2.f * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.f * qx * dR[4] - w * dR[5] + qz * dR[6] +
                                w * dR[7] - 2.f * qx * dR[8]);
        const float dy = 2.f * (-2.f * qy * dR[0] + qx * dR[1] + w * dR[2] + qx * dR[3] + qz * dR[5] - w * dR[6] +
                                qz * dR[7] - 2.f * qy * dR[8]);
        const float dz = 2.f * (-2.f * qz * dR[0] - w * dR[1] + qx * dR[2] + w * dR[3] - 2.f * qz * dR[4] +
                                qy * dR[5] + qx * dR[6] + qy * dR[7]);
        // through q / |q|: remove the radial component, scale by 1 / |q|
        const float dot = dw * w + dx * qx + dy * qy + dz * qz;
        gq[0] = (dw - dot * w) * qn;
        gq[1] = (dx - dot * qx) * qn;
        gq[2] = (dy - dot * qy) * qn;
        gq[3] = (dz - dot * qz) * qn;

        // camera-space mean: through J and through (u, v)
        const float gu = d_mean2d[2 * i], gv = d_mean2d[2 * i + 1];
        const float iz2 = iz * iz, iz3 = iz2 * iz;
        const float dpx = dj02 * (-cam.fx * iz2) + gu * cam.fx * iz;
        const float dpy = dj12 * (-cam.fy * iz2) + gv * cam.fy * iz;
        const float dpz = dj00 * (-cam.fx * iz2) + dj02 * (2.f * cam.fx * x * iz3) + dj11 * (-cam.fy * iz2) +
                          dj12 * (2.f * cam.fy * y * iz3) - gu * cam.fx * x * iz2 - gv * cam.fy * y * iz2;
#pragma unroll
        for (int k = 0; k < 3; ++k) gm[k] = cam.R[k] * dpx + cam.R[3 + k] * dpy + cam.R[6 + k] * dpz;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d_means[3 * i + k] = gm[k];
        d_scales[3 * i + k] = gs[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) d_quats[4 * i + k] = gq[k];
}

}  // namespace ls2

extern "C" int ls2_project_backward(const ls2_camera* cam, int32_t n, const float* means, const float* scales,
                                    const float* quats, const int32_t* radius, const float* d_mean2d,
                                    const float* d_conic, float* d_means, float* d_scales, float* d_quats,
                                    hipStream_t stream) {
    if (!ls2::cam_valid(cam) || n < 0) return LS2_ERR_ARG;
    if (n == 0) return LS2_OK;
    if (!means || !scales || !quats || !radius || !d_mean2d || !d_conic || !d_means || !d_scales || !d_quats)
        return LS2_ERR_ARG;
    const ls2::CamK k = ls2::cam_k(*cam);
    hipLaunchKernelGGL(ls2::k_project_backward, dim3((n + 255) / 256), dim3(256), 0, stream, k, n, means, scales,
                       quats, radius, d_mean2d, d_conic, d_means, d_scales, d_quats);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}
