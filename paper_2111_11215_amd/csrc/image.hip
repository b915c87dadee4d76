// Test-time rendering of a whole image (the paper renders 800 x 800 views
// at test time with the same sampler and forward as training, minus the
// jitter, and skips free space in testing too): per chunk of pixels, one
// kernel casts the pinhole rays, then the plain sampler (coarse mask and
// optional fine-density skip, no jitter, no proposal) and the forward
// render run on them through the library's own entry points.
#include "common.hpp"

namespace {

struct Cam {
    float R[9];   // camera-to-world rotation, row-major: world = R * camera
    float o[3];
    float focal;
    int H, W;
};

// Ray of pixel p = i*W + j through its centre: camera-space direction
// ((j + 1/2 - W/2)/focal, -(i + 1/2 - H/2)/focal, -1), rotated to world
// space and normalised; the origin is the camera centre.
__global__ __launch_bounds__(256) void cast_rays_kernel(Cam c, int64_t p0, int n, float* __restrict__ ro,
                                                        float* __restrict__ rd) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const int64_t p = p0 + k;
    const int i = static_cast<int>(p / c.W), j = static_cast<int>(p % c.W);
    const float x = (static_cast<float>(j) + 0.5f - 0.5f * static_cast<float>(c.W)) / c.focal;
    const float y = -(static_cast<float>(i) + 0.5f - 0.5f * static_cast<float>(c.H)) / c.focal;
    float d[3];
    for (int r = 0; r < 3; ++r) d[r] = c.R[3 * r + 0] * x + c.R[3 * r + 1] * y - c.R[3 * r + 2];
    const float inv = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int r = 0; r < 3; ++r) {
        rd[3 * static_cast<int64_t>(k) + r] = d[r] * inv;
        ro[3 * static_cast<int64_t>(k) + r] = c.o[r];
    }
}

struct ImageWs {
    size_t ro, rd, t_near, t_far, valid, n_uniform, perm, ray_offset, n_kept, sample_ray, sample_k, log_t, samp,
        render, total;
};

ImageWs image_ws(int32_t chunk, int32_t max_samples, const dvgo_box* grid) {
    ImageWs L{};
    const int64_t cap = static_cast<int64_t>(chunk) * max_samples;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = dvgo::align_up(off + bytes, 256);
        return o;
    };
    L.ro = take(static_cast<size_t>(chunk) * 12);
    L.rd = take(static_cast<size_t>(chunk) * 12);
    L.t_near = take(static_cast<size_t>(chunk) * 4);
    L.t_far = take(static_cast<size_t>(chunk) * 4);
    L.valid = take(static_cast<size_t>(chunk));
    L.n_uniform = take(static_cast<size_t>(chunk) * 4);
    L.perm = take(static_cast<size_t>(chunk) * 4);
    L.ray_offset = take(static_cast<size_t>(chunk + 1) * 4);
    L.n_kept = take(8);
    L.sample_ray = take(static_cast<size_t>(cap) * 4);
    L.sample_k = take(static_cast<size_t>(cap) * 4);
    L.log_t = take(static_cast<size_t>(chunk) * 4);
    L.samp = take(dvgo_sample_workspace_bytes(chunk));
    L.render = take(dvgo_render_fwd_workspace_bytes(chunk, cap, 12, grid));
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

size_t dvgo_render_image_workspace_bytes(int32_t chunk, int32_t max_samples, const dvgo_box* grid) {
    if (chunk < 1 || max_samples < 1 || !dvgo::box_ok(grid, 2)) return 0;
    if (static_cast<int64_t>(chunk) * max_samples >= (1LL << 31)) return 0;
    return image_ws(chunk, max_samples, grid).total;
}

int32_t dvgo_render_image(const dvgo_field* field, const dvgo_mlp* mlp, const dvgo_camera* cam, float step,
                          int32_t max_samples, const uint32_t* coarse_bits, const dvgo_box* coarse_box,
                          const dvgo_fine_filter* fine, const float* bg, int32_t chunk, float* rgb, float* depth, float* acc, float* rays_o,
                          float* rays_d, void* workspace, size_t workspace_bytes, void* stream) {
    if (!field || !mlp || !cam || !bg || !rgb || chunk < 1 || max_samples < 1 || !(step > 0.0f)) return DVGO_E_ARG;
    if (cam->H < 1 || cam->W < 1 || !(cam->focal > 0.0f)) return DVGO_E_ARG;
    if (static_cast<int64_t>(cam->H) * cam->W >= (1LL << 31)) return DVGO_E_UNSUPPORTED;
    const size_t need = dvgo_render_image_workspace_bytes(chunk, max_samples, &field->box);
    if (need == 0) return DVGO_E_ARG;
    if (!workspace || workspace_bytes < need) return DVGO_E_CAPACITY;
    const ImageWs L = image_ws(chunk, max_samples, &field->box);
    char* ws = static_cast<char*>(workspace);
    auto F = [&](size_t off) { return reinterpret_cast<float*>(ws + off); };
    auto I = [&](size_t off) { return reinterpret_cast<int32_t*>(ws + off); };
    Cam c;
    for (int k = 0; k < 9; ++k) c.R[k] = cam->c2w[k];
    for (int k = 0; k < 3; ++k) c.o[k] = cam->origin[k];
    c.focal = cam->focal;
    c.H = cam->H;
    c.W = cam->W;
    const int64_t npix = static_cast<int64_t>(cam->H) * cam->W;
    const int64_t cap = static_cast<int64_t>(chunk) * max_samples;
    hipStream_t s = dvgo::as_stream(stream);
    for (int64_t p0 = 0; p0 < npix; p0 += chunk) {
        const int n = static_cast<int>(npix - p0 < chunk ? npix - p0 : chunk);
        float* ro = rays_o ? rays_o + 3 * p0 : F(L.ro);
        float* rd = rays_d ? rays_d + 3 * p0 : F(L.rd);
        hipLaunchKernelGGL(cast_rays_kernel, dim3((n + 255) / 256), dim3(256), 0, s, c, p0, n, ro, rd);
        if (int32_t st = dvgo::launch_status()) return st;
        if (int32_t st = dvgo_sample_rays(ro, rd, nullptr, n, &field->box, step, max_samples, coarse_bits,
                                          coarse_box, nullptr, fine, 0, F(L.t_near), F(L.t_far),
                                          reinterpret_cast<uint8_t*>(ws + L.valid), I(L.n_uniform), I(L.perm),
                                          I(L.ray_offset), I(L.sample_ray), I(L.sample_k), cap,
                                          reinterpret_cast<int64_t*>(ws + L.n_kept), ws + L.samp,
                                          dvgo_sample_workspace_bytes(n), stream))
            return st;
        if (int32_t st = dvgo_render_fwd(field, mlp, ro, rd, nullptr, F(L.t_near), I(L.n_uniform), I(L.perm),
                                         I(L.ray_offset), I(L.sample_ray), I(L.sample_k),
                                         reinterpret_cast<int64_t*>(ws + L.n_kept), cap, n, step, bg, rgb + 3 * p0,
                                         depth ? depth + p0 : nullptr, acc ? acc + p0 : nullptr, F(L.log_t),
                                         nullptr, nullptr, ws + L.render,
                                         dvgo_render_fwd_workspace_bytes(n, cap, 12, &field->box), stream))
            return st;
    }
    return DVGO_OK;
}

}  // extern "C"
