// Image-fitting toy of the paper's Sec. 3 ("Sharp decision boundary via
// post-activation"): a gh x gw grid V, bilinearly interpolated at the pixel
// centres of an H x W image, predicts an alpha image with one of three
// orders of interpolation and activation (Eq. pre_activation,
// in_activation, post_activation; softplus without shift, alpha(s) =
// 1 - exp(-s delta)), fitted to a binary target by mean squared error.
//   pixel kernel   alpha per pixel; for the loss also dL/dalpha = 2(a - T)/N
//                  and per-workgroup sums of (a - T)^2
//   vertex kernel  dL/dV per vertex: one wavefront walks the pixels of its
//                  four cells and sums their contributions (no atomics,
//                  fixed order)
//   reduce         the loss from the per-workgroup sums, in a fixed order
#include "common.hpp"

namespace {

constexpr int kPix = 256;   // pixels per workgroup of the pixel kernel

struct ToyArgs {
    const float* V;
    int gh, gw, H, W, mode;
    float su, sv;   // (gh-1)/H and (gw-1)/W, rounded once to float32
    float delta;
};

__device__ __forceinline__ float softplus_t(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }
__device__ __forceinline__ float sigmoid_t(float x) { return 1.0f / (1.0f + expf(-x)); }
__device__ __forceinline__ float alpha_t(float s, float delta) { return -expm1f(-s * delta); }

// Cell and bilinear weights of pixel (i, j): corners (i0,j0), (i0,j0+1),
// (i0+1,j0), (i0+1,j0+1).
struct Bil {
    int i0, j0;
    float w[4];
};

__device__ __forceinline__ Bil bilinear(const ToyArgs& a, int i, int j) {
    const float u = (static_cast<float>(i) + 0.5f) * a.su;
    const float v = (static_cast<float>(j) + 0.5f) * a.sv;
    const float fi = fminf(fmaxf(floorf(u), 0.0f), static_cast<float>(a.gh - 2));
    const float fj = fminf(fmaxf(floorf(v), 0.0f), static_cast<float>(a.gw - 2));
    const float fu = fminf(fmaxf(u - fi, 0.0f), 1.0f), fv = fminf(fmaxf(v - fj, 0.0f), 1.0f);
    Bil b;
    b.i0 = static_cast<int>(fi);
    b.j0 = static_cast<int>(fj);
    b.w[0] = (1.0f - fu) * (1.0f - fv);
    b.w[1] = (1.0f - fu) * fv;
    b.w[2] = fu * (1.0f - fv);
    b.w[3] = fu * fv;
    return b;
}

__device__ __forceinline__ void corners(const ToyArgs& a, const Bil& b, float c[4]) {
    const int64_t base = static_cast<int64_t>(b.i0) * a.gw + b.j0;
    c[0] = a.V[base];
    c[1] = a.V[base + 1];
    c[2] = a.V[base + a.gw];
    c[3] = a.V[base + a.gw + 1];
}

// The pixel's alpha, and the scalar that multiplies dL/dalpha on the way
// to every corner (post: alpha'(softplus(vbar)) sigmoid(vbar); in:
// alpha'(sbar); pre: 1, the per-corner factor is taken at the vertex).
__device__ __forceinline__ float pixel_alpha(const ToyArgs& a, const Bil& b, const float c[4], float* chain) {
    if (a.mode == DVGO_TOY_PRE) {
        float s = 0.0f;
        for (int k = 0; k < 4; ++k) s += b.w[k] * alpha_t(softplus_t(c[k]), a.delta);
        *chain = 1.0f;
        return s;
    }
    if (a.mode == DVGO_TOY_IN) {
        float s = 0.0f;
        for (int k = 0; k < 4; ++k) s += b.w[k] * softplus_t(c[k]);
        *chain = a.delta * expf(-s * a.delta);
        return alpha_t(s, a.delta);
    }
    float v = 0.0f;
    for (int k = 0; k < 4; ++k) v += b.w[k] * c[k];
    const float sp = softplus_t(v);
    *chain = a.delta * expf(-sp * a.delta) * sigmoid_t(v);
    return alpha_t(sp, a.delta);
}

__global__ __launch_bounds__(kPix) void toy_pixel_kernel(ToyArgs a, const float* __restrict__ target,
                                                         float* __restrict__ image, float* __restrict__ dalpha,
                                                         float* __restrict__ part) {
    __shared__ float red[kPix];
    const int64_t n = static_cast<int64_t>(a.H) * a.W;
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kPix + threadIdx.x;
    float r2 = 0.0f;
    if (p < n) {
        const int i = static_cast<int>(p / a.W), j = static_cast<int>(p % a.W);
        const Bil b = bilinear(a, i, j);
        float c[4], chain;
        corners(a, b, c);
        const float al = pixel_alpha(a, b, c, &chain);
        if (image) image[p] = al;
        if (target) {
            const float r = al - target[p];
            dalpha[p] = 2.0f * r / static_cast<float>(n);
            r2 = r * r;
        }
    }
    if (!part) return;
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int st = kPix / 2; st > 0; st >>= 1) {
        if (static_cast<int>(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// dL/dV[a][b]: one wavefront per vertex.  The vertex's pixels are those of
// the rows and columns whose u, v lie within one cell of it (a margin of
// one pixel on each side; each pixel's own cell decides), dealt to the 64
// lanes in row-major order; each lane sums its pixels in order and the
// lanes' sums meet in a fixed butterfly, so the result does not depend on
// scheduling.
constexpr int kVertWaves = 4;   // vertices (wavefronts) per workgroup

__global__ __launch_bounds__(64 * kVertWaves) void toy_vertex_kernel(ToyArgs a, const float* __restrict__ dalpha,
                                                                     float* __restrict__ grad) {
    const int64_t nv = static_cast<int64_t>(a.gh) * a.gw;
    const int lane = threadIdx.x & 63;
    const int64_t vid = static_cast<int64_t>(blockIdx.x) * kVertWaves + (threadIdx.x >> 6);
    if (vid >= nv) return;
    const int va = static_cast<int>(vid / a.gw), vb = static_cast<int>(vid % a.gw);
    const float rows_per = static_cast<float>(a.H) / static_cast<float>(a.gh - 1);
    const float cols_per = static_cast<float>(a.W) / static_cast<float>(a.gw - 1);
    const int i_lo = max(0, static_cast<int>(floorf((va - 1) * rows_per)) - 1);
    const int i_hi = min(a.H - 1, static_cast<int>(ceilf((va + 1) * rows_per)) + 1);
    const int j_lo = max(0, static_cast<int>(floorf((vb - 1) * cols_per)) - 1);
    const int j_hi = min(a.W - 1, static_cast<int>(ceilf((vb + 1) * cols_per)) + 1);
    const int ncol = j_hi - j_lo + 1;
    const int npix = (i_hi - i_lo + 1) * ncol;
    const float mine = a.V[vid];
    // pre and in: the corner's own factor (alpha'(softplus(V)) sigmoid(V),
    // or sigmoid(V)) is common to every pixel
    const float own = a.mode == DVGO_TOY_PRE ? a.delta * expf(-softplus_t(mine) * a.delta) * sigmoid_t(mine)
                      : a.mode == DVGO_TOY_IN ? sigmoid_t(mine) : 1.0f;
    float g = 0.0f;
    for (int q = lane; q < npix; q += 64) {
        const int i = i_lo + q / ncol, j = j_lo + q % ncol;
        const Bil b = bilinear(a, i, j);
        const int di = va - b.i0, dj = vb - b.j0;
        if (di < 0 || di > 1 || dj < 0 || dj > 1) continue;
        float chain = 1.0f;
        if (a.mode != DVGO_TOY_PRE) {
            float c[4];
            corners(a, b, c);
            pixel_alpha(a, b, c, &chain);
        }
        g += dalpha[static_cast<int64_t>(i) * a.W + j] * chain * b.w[2 * di + dj];
    }
    for (int off = 32; off > 0; off >>= 1) g += __shfl_xor(g, off, 64);
    if (lane == 0) grad[vid] = g * own;
}

__global__ __launch_bounds__(256) void toy_reduce_kernel(const float* __restrict__ part, int n, float inv_n,
                                                         float* __restrict__ loss) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int k = threadIdx.x; k < n; k += 256) s += part[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (static_cast<int>(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] * inv_n;
}

int32_t toy_args(const float* V, int32_t gh, int32_t gw, int32_t H, int32_t W, int32_t mode, float delta,
                 ToyArgs* a) {
    if (!V || gh < 2 || gw < 2 || H < 1 || W < 1 || !(delta > 0.0f)) return DVGO_E_ARG;
    if (mode != DVGO_TOY_PRE && mode != DVGO_TOY_IN && mode != DVGO_TOY_POST) return DVGO_E_ARG;
    if (static_cast<int64_t>(H) * W >= (1LL << 31) || static_cast<int64_t>(gh) * gw >= (1LL << 31))
        return DVGO_E_UNSUPPORTED;
    a->V = V;
    a->gh = gh;
    a->gw = gw;
    a->H = H;
    a->W = W;
    a->mode = mode;
    volatile float nu = static_cast<float>(gh - 1), nv = static_cast<float>(gw - 1);
    a->su = nu / static_cast<float>(H);
    a->sv = nv / static_cast<float>(W);
    a->delta = delta;
    return DVGO_OK;
}

}  // namespace

extern "C" {

size_t dvgo_toy2d_workspace_bytes(int32_t H, int32_t W) {
    if (H < 1 || W < 1) return 0;
    const size_t n = static_cast<size_t>(H) * W;
    return dvgo::align_up(n * 4, 256) + dvgo::align_up((n + kPix - 1) / kPix * 4, 256);
}

int32_t dvgo_toy2d_forward(const float* V, int32_t gh, int32_t gw, int32_t H, int32_t W, int32_t mode, float delta,
                           float* image, void* stream) {
    ToyArgs a;
    if (int32_t st = toy_args(V, gh, gw, H, W, mode, delta, &a)) return st;
    if (!image) return DVGO_E_ARG;
    const int64_t n = static_cast<int64_t>(H) * W;
    DVGO_LAUNCH(K_TOY_PIXEL, toy_pixel_kernel, dim3(static_cast<unsigned>((n + kPix - 1) / kPix)), dim3(kPix), 0,
                dvgo::as_stream(stream), a, static_cast<const float*>(nullptr), image, static_cast<float*>(nullptr),
                static_cast<float*>(nullptr));
    return dvgo::launch_status();
}

int32_t dvgo_toy2d_loss_grad(const float* V, int32_t gh, int32_t gw, const float* target, int32_t H, int32_t W,
                             int32_t mode, float delta, float* grad, float* loss, void* workspace,
                             size_t workspace_bytes, void* stream) {
    ToyArgs a;
    if (int32_t st = toy_args(V, gh, gw, H, W, mode, delta, &a)) return st;
    if (!target || !grad || !loss) return DVGO_E_ARG;
    if (!workspace || workspace_bytes < dvgo_toy2d_workspace_bytes(H, W)) return DVGO_E_CAPACITY;
    const int64_t n = static_cast<int64_t>(H) * W;
    const int nblk = static_cast<int>((n + kPix - 1) / kPix);
    float* dalpha = static_cast<float*>(workspace);
    float* part = reinterpret_cast<float*>(static_cast<char*>(workspace) + dvgo::align_up(n * 4, 256));
    hipStream_t s = dvgo::as_stream(stream);
    DVGO_LAUNCH(K_TOY_PIXEL, toy_pixel_kernel, dim3(nblk), dim3(kPix), 0, s, a, target, static_cast<float*>(nullptr),
                dalpha, part);
    if (int32_t st = dvgo::launch_status()) return st;
    const int64_t nv = static_cast<int64_t>(gh) * gw;
    DVGO_LAUNCH(K_TOY_VERTEX, toy_vertex_kernel, dim3(static_cast<unsigned>((nv + kVertWaves - 1) / kVertWaves)),
                dim3(64 * kVertWaves), 0, s, a, dalpha, grad);
    if (int32_t st = dvgo::launch_status()) return st;
    DVGO_LAUNCH(K_TOY_REDUCE, toy_reduce_kernel, dim3(1), dim3(256), 0, s, part, nblk,
                1.0f / static_cast<float>(n), loss);
    return dvgo::launch_status();
}

}  // extern "C"
