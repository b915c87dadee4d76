// Data generation: colours of rays through an analytic scene of soft-edged
// spheres, composited with the volume-rendering quadrature (paper
// Eq. volume_rendering) at midpoint samples.  Not part of the training step.
#include "common.hpp"

namespace {

constexpr int kMaxSpheres = 256;

__global__ __launch_bounds__(256) void scene_render_kernel(const float* __restrict__ rays_o,
                                                           const float* __restrict__ rays_d, int B, dvgo_box box,
                                                           const float* __restrict__ spheres, int ns, float edge,
                                                           float step, float bg0, float bg1, float bg2,
                                                           float* __restrict__ rgb) {
    __shared__ float sp[kMaxSpheres * 8];
    for (int i = threadIdx.x; i < ns * 8; i += blockDim.x) sp[i] = spheres[i];
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= B) return;
    float o[3], d[3];
    for (int i = 0; i < 3; ++i) {
        o[i] = rays_o[3 * r + i];
        d[i] = rays_d[3 * r + i];
    }
    float te = -INFINITY, tx = INFINITY;
    bool miss = false;
    for (int i = 0; i < 3; ++i) {
        if (d[i] == 0.0f) {
            if (o[i] < box.xyz_min[i] || o[i] > box.xyz_max[i]) miss = true;
        } else {
            const float inv = 1.0f / d[i];
            const float t0 = (box.xyz_min[i] - o[i]) * inv, t1 = (box.xyz_max[i] - o[i]) * inv;
            te = fmaxf(te, fminf(t0, t1));
            tx = fminf(tx, fmaxf(t0, t1));
        }
    }
    const float tn = fmaxf(te, 0.0f);
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    if (!miss && tn < tx) {
        const float inv_edge = 1.0f / edge;
        for (int k = 0;; ++k) {
            const float t = tn + (static_cast<float>(k) + 0.5f) * step;
            if (!(t < tx)) break;
            const float x0 = o[0] + t * d[0], x1 = o[1] + t * d[1], x2 = o[2] + t * d[2];
            float sig = 0.0f, s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
            for (int i = 0; i < ns; ++i) {
                const float* q = sp + 8 * i;
                const float dx = x0 - q[0], dy = x1 - q[1], dz = x2 - q[2];
                const float z = (q[3] - sqrtf(dx * dx + dy * dy + dz * dz)) * inv_edge;
                if (z < -30.0f) continue;
                const float si = q[4] / (1.0f + expf(-z));
                sig += si;
                s0 += si * q[5];
                s1 += si * q[6];
                s2 += si * q[7];
            }
            if (sig > 0.0f) {
                const float a = -expm1f(-sig * step);
                const float w = T * a / sig;
                c0 += w * s0;
                c1 += w * s1;
                c2 += w * s2;
                T *= 1.0f - a;
                if (T < 1e-7f) {
                    T = 0.0f;
                    break;
                }
            }
        }
    }
    rgb[3 * r + 0] = c0 + T * bg0;
    rgb[3 * r + 1] = c1 + T * bg1;
    rgb[3 * r + 2] = c2 + T * bg2;
}

}  // namespace

extern "C" int32_t dvgo_scene_render(const float* rays_o, const float* rays_d, int32_t B, const dvgo_box* box,
                                     const float* spheres, int32_t n_spheres, float edge, float step, const float* bg,
                                     float* rgb, void* stream) {
    if (B < 0 || !box || !bg || n_spheres < 0 || n_spheres > kMaxSpheres) return DVGO_E_ARG;
    if (!(edge > 0.0f) || !(step > 0.0f)) return DVGO_E_ARG;
    if (B > 0 && (!rays_o || !rays_d || !rgb || (n_spheres > 0 && !spheres))) return DVGO_E_ARG;
    if (B == 0) return DVGO_OK;
    DVGO_LAUNCH(K_SCENE, scene_render_kernel, dim3((B + 255) / 256), dim3(256), 0, dvgo::as_stream(stream), rays_o,
                       rays_d, B, *box, spheres, n_spheres, edge, step, bg[0], bg[1], bg[2], rgb);
    return dvgo::launch_status();
}
