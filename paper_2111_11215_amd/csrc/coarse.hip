// Coarse stage of the paper (Sec. 4.1, "Coarse geometry searching"): a
// density grid with post-activation and a view-invariant colour grid
// (Eq. coarse_queries, colour = sigmoid of the interpolated 3 channels),
// trained with the photometric loss, the per-point rgb loss and the
// background entropy loss, Adam with the view-count-based learning rate of
// Prior 2 on the density.
//   coarse_step_kernel  one wavefront per ray: the forward (gathers,
//                       prefix-scan compositing, the ray's loss terms),
//                       then the adjoint walked from the ray's end with the
//                       transmittance recomputed by prefix sums as in the
//                       forward, scattering the grid gradients with float
//                       atomics aggregated over the wavefront: consecutive
//                       samples of a ray in the same cell share its eight
//                       corners, so their contributions are summed across
//                       lanes first and the run's first lane adds them
//                       (100^3 grids: few samples per vertex)
//   loss_reduce         the per-ray losses summed in a fixed order
//   view_count / scale  Prior 2: per-vertex view counts and n_j / n_max
//   adam_scaled         Adam with a per-element learning-rate factor
#include "adam.hpp"
#include "common.hpp"
#include "scan.hpp"

using dvgo::GridArgs;
using namespace dvgo_dev;

namespace {

constexpr int kMaxSteps = 64;   // 64-sample steps per ray (4096 samples)

struct CoarseArgs {
    const float* rays_o;
    const float* rays_d;
    const float* jitter;
    const float* t_near;
    const int* perm;
    const int* ray_offset;
    const int* sample_k;
    const int64_t* n_kept;
    int64_t cap;
    int B;
    float step;
    GridArgs g;
    const float* density;
    const float* rgb;
    float act_shift;
    float bg[3];
    const float* target;
    float w_pt, w_bg;
    float* rgb_out;
    float* ray_loss;
    float* grad_density;
    float* grad_rgb;
};

__device__ __forceinline__ float softplus_c(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }
__device__ __forceinline__ float sigmoid_c(float x) { return 1.0f / (1.0f + expf(-x)); }

// One sample's interpolated raw density and colour pre-activation, with the
// corner indices and weights for the scatter.
struct CSample {
    int64_t corner[8];   // corner[0] is the cell's base vertex
    float w[8];
    float raw, pre[3], t;
};

// Sum of v over the lanes from this one to the end of its run of equal
// keys (runs are contiguous: a ray's samples in one cell are consecutive,
// and a lane without a sample has a key of its own).
__device__ __forceinline__ float run_suffix_sum(float v, int64_t key, int lane) {
    #pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const float ov = __shfl_down(v, off, 64);
        const int64_t ok = __shfl_down(key, off, 64);
        if (lane + off < 64 && ok == key) v += ov;
    }
    return v;
}

__device__ __forceinline__ void coarse_sample(const CoarseArgs& a, const float o[3], const float d[3], float tn, float p,
                                              int k, CSample& cs) {
    cs.t = recipe_tk(tn, p, k, a.step);
    float x[3];
    recipe_x(o, d, cs.t, x);
    int i0[3];
    float f[3];
    for (int i = 0; i < 3; ++i) {
        const float u = (x[i] - a.g.mn[i]) * a.g.scale[i];
        const float fl = fminf(fmaxf(floorf(u), 0.0f), static_cast<float>(a.g.n[i] - 2));
        i0[i] = static_cast<int>(fl);
        f[i] = fminf(fmaxf(u - fl, 0.0f), 1.0f);
    }
    const int64_t sx = static_cast<int64_t>(a.g.n[1]) * a.g.n[2], sy = a.g.n[2];
    const int64_t base = i0[0] * sx + i0[1] * sy + i0[2];
    cs.raw = 0.0f;
    cs.pre[0] = cs.pre[1] = cs.pre[2] = 0.0f;
    #pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int bx = (c >> 2) & 1, by = (c >> 1) & 1, bz = c & 1;
        cs.w[c] = (bx ? f[0] : 1.0f - f[0]) * (by ? f[1] : 1.0f - f[1]) * (bz ? f[2] : 1.0f - f[2]);
        cs.corner[c] = base + bx * sx + by * sy + bz;
        cs.raw += cs.w[c] * a.density[cs.corner[c]];
        for (int ch = 0; ch < 3; ++ch) cs.pre[ch] += cs.w[c] * a.rgb[3 * cs.corner[c] + ch];
    }
}

__global__ __launch_bounds__(256) void coarse_step_kernel(CoarseArgs a) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = blockIdx.x * 4 + wave;
    if (slot >= a.B) return;
    const int64_t n = *a.n_kept < a.cap ? *a.n_kept : a.cap;
    const int r = a.perm[slot];
    int64_t s0 = a.ray_offset[slot], s1 = a.ray_offset[slot + 1];
    s0 = s0 < n ? s0 : n;
    s1 = s1 < n ? s1 : n;
    float o[3], d[3], tgt[3];
    for (int i = 0; i < 3; ++i) {
        o[i] = a.rays_o[3 * r + i];
        d[i] = a.rays_d[3 * r + i];
        tgt[i] = a.target[3 * r + i];
    }
    const float tn = a.t_near[r];
    const float p = a.jitter ? a.jitter[r] : 0.0f;
    const int64_t nsteps = (s1 - s0 + 63) / 64;
    // ---- forward: prefix-scan compositing; lane j keeps log T at the start of step j
    float logT = 0.0f, start = 0.0f, C[3] = {0.0f, 0.0f, 0.0f}, pt = 0.0f;
    for (int64_t it = 0; it < nsteps; ++it) {
        if (lane == static_cast<int>(it)) start = logT;
        const int64_t s = s0 + it * 64 + lane;
        const bool ok = s < s1;
        float sd = 0.0f, alpha = 0.0f, c[3] = {0.0f, 0.0f, 0.0f};
        if (ok) {
            CSample cs;
            coarse_sample(a, o, d, tn, p, a.sample_k[s], cs);
            sd = softplus_c(cs.raw + a.act_shift) * a.step;
            alpha = -expm1f(-sd);
            for (int ch = 0; ch < 3; ++ch) c[ch] = sigmoid_c(cs.pre[ch]);
        }
        const float incl = wave_incl_scan(sd, lane);
        const float excl = dpp_wave<0x138>(incl);
        const float w = ok ? expf(logT - excl) * alpha : 0.0f;
        float e2 = 0.0f;
        for (int ch = 0; ch < 3; ++ch) {
            C[ch] += w * c[ch];
            const float dd = c[ch] - tgt[ch];
            e2 += dd * dd;
        }
        pt += w * e2;
        logT -= lane_value(incl, 63);
    }
    for (int ch = 0; ch < 3; ++ch) C[ch] = wave_sum(C[ch]);
    pt = wave_sum(pt);
    const float Tend = expf(logT);
    const float invB = 1.0f / static_cast<float>(a.B);
    float gC[3], photo = 0.0f;
    for (int ch = 0; ch < 3; ++ch) {
        C[ch] += Tend * a.bg[ch];
        const float dd = C[ch] - tgt[ch];
        gC[ch] = 2.0f * dd * invB;
        photo += dd * dd;
    }
    // background entropy of T_end, clamped to [1e-6, 1 - 1e-6]
    const float pb = fminf(fmaxf(Tend, 1e-6f), 1.0f - 1e-6f);
    const float ent = -pb * logf(pb) - (1.0f - pb) * log1pf(-pb);
    const bool inside = Tend > 1e-6f && Tend < 1.0f - 1e-6f;
    const float gT = inside ? a.w_bg * (log1pf(-pb) - logf(pb)) * invB : 0.0f;
    if (lane == 0) {
        if (a.rgb_out)
            for (int ch = 0; ch < 3; ++ch) a.rgb_out[3 * r + ch] = C[ch];
        a.ray_loss[r] = photo + a.w_pt * pt + a.w_bg * ent;
    }
    // ---- adjoint: walk from the end, suffix sums S of w c (plus T_end bg)
    float S[3] = {Tend * a.bg[0], Tend * a.bg[1], Tend * a.bg[2]};
    const float ptk = 2.0f * a.w_pt * invB;
    for (int64_t it = nsteps - 1; it >= 0; --it) {
        const int64_t s = s0 + it * 64 + lane;
        const bool ok = s < s1;
        CSample cs;
        float sd = 0.0f, alpha = 0.0f, c[3] = {0.0f, 0.0f, 0.0f};
        if (ok) {
            coarse_sample(a, o, d, tn, p, a.sample_k[s], cs);
            sd = softplus_c(cs.raw + a.act_shift) * a.step;
            alpha = -expm1f(-sd);
            for (int ch = 0; ch < 3; ++ch) c[ch] = sigmoid_c(cs.pre[ch]);
        }
        const float logT0 = lane_value(start, static_cast<int>(it));
        const float incl = wave_incl_scan(sd, lane);
        const float excl = dpp_wave<0x138>(incl);
        const float Tafter = expf(logT0 - incl);
        const float w = ok ? expf(logT0 - excl) * alpha : 0.0f;
        float dsig = -Tend * gT;
        float tot[3];
        for (int ch = 0; ch < 3; ++ch) {
            const float sfx = wave_incl_suffix(w * c[ch], lane);
            const float sfx_ex = dpp_wave<0x130>(sfx);
            dsig += gC[ch] * (Tafter * c[ch] - (S[ch] + sfx_ex));
            tot[ch] = lane_value(sfx, 0);
        }
        {
            float draw = 0.0f, dpre[3] = {0.0f, 0.0f, 0.0f};
            if (ok) {
                draw = a.step * dsig * sigmoid_c(cs.raw + a.act_shift);
                for (int ch = 0; ch < 3; ++ch) {
                    const float dc = w * gC[ch] + ptk * w * (c[ch] - tgt[ch]);
                    dpre[ch] = dc * c[ch] * (1.0f - c[ch]);
                }
            }
            // every lane takes part in the shuffles; a lane without a sample
            // has a key of its own and contributes zeros
            const int64_t key = ok ? cs.corner[0] : -1 - static_cast<int64_t>(lane);
            const int64_t prev = __shfl_up(key, 1, 64);
            const bool head = ok && (lane == 0 || prev != key);
            #pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float wk = ok ? cs.w[k] : 0.0f;
                const float gd = run_suffix_sum(wk * draw, key, lane);
                float gr[3];
                for (int ch = 0; ch < 3; ++ch) gr[ch] = run_suffix_sum(wk * dpre[ch], key, lane);
                if (head) {
                    atomicAdd(a.grad_density + cs.corner[k], gd);
                    for (int ch = 0; ch < 3; ++ch) atomicAdd(a.grad_rgb + 3 * cs.corner[k] + ch, gr[ch]);
                }
            }
        }
        for (int ch = 0; ch < 3; ++ch) S[ch] += tot[ch];
    }
}

__global__ __launch_bounds__(256) void ray_loss_reduce_kernel(const float* __restrict__ part, int n, float inv_n,
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

// Prior 2: vertex j at min + idx*((max-min)/(n-1)); visible to a camera
// (row-major camera-to-world R, centre c) when p = R^T (x - c) has p_z < 0
// and its projection (focal p_x/(-p_z) + W/2, -focal p_y/(-p_z) + H/2) lies
// in [0, W) x [0, H).
struct VcArgs {
    float mn[3], stepv[3];
    int n[3];
    const float* cams;   // [ncam][12]: R (9, row-major), centre (3)
    int ncam, H, W;
    float focal;
};

__global__ __launch_bounds__(256) void fill_zero_kernel(int* __restrict__ p) { *p = 0; }

__global__ __launch_bounds__(256) void view_count_kernel(VcArgs a, int* __restrict__ counts, int* __restrict__ nmax) {
    const int64_t nv = static_cast<int64_t>(a.n[0]) * a.n[1] * a.n[2];
    const int64_t v = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (v >= nv) return;
    const int j2 = static_cast<int>(v % a.n[2]), j1 = static_cast<int>((v / a.n[2]) % a.n[1]);
    const int j0 = static_cast<int>(v / (static_cast<int64_t>(a.n[1]) * a.n[2]));
    const float x[3] = {a.mn[0] + j0 * a.stepv[0], a.mn[1] + j1 * a.stepv[1], a.mn[2] + j2 * a.stepv[2]};
    int cnt = 0;
    for (int c = 0; c < a.ncam; ++c) {
        const float* R = a.cams + 12 * c;
        const float dx = x[0] - R[9], dy = x[1] - R[10], dz = x[2] - R[11];
        const float px = R[0] * dx + R[3] * dy + R[6] * dz;
        const float py = R[1] * dx + R[4] * dy + R[7] * dz;
        const float pz = R[2] * dx + R[5] * dy + R[8] * dz;
        const float z = -pz;
        if (!(z > 0.0f)) continue;
        const float u = a.focal * px / z + 0.5f * a.W;
        const float vv = -a.focal * py / z + 0.5f * a.H;
        cnt += (u >= 0.0f && u < static_cast<float>(a.W) && vv >= 0.0f && vv < static_cast<float>(a.H)) ? 1 : 0;
    }
    counts[v] = cnt;
    atomicMax(nmax, cnt);
}

__global__ __launch_bounds__(256) void view_scale_kernel(const int* __restrict__ counts, int64_t nv,
                                                         const int* __restrict__ nmax, float* __restrict__ scale) {
    const int64_t v = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (v >= nv) return;
    const int m = *nmax;
    scale[v] = static_cast<float>(counts[v]) / static_cast<float>(m > 0 ? m : 1);
}

__global__ __launch_bounds__(256) void adam_scaled_kernel(float* __restrict__ p, float* __restrict__ g,
                                                          float* __restrict__ m, float* __restrict__ v,
                                                          const float* __restrict__ scale, int64_t n,
                                                          dvgo::AdamCoef c) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    dvgo::AdamCoef ci = c;
    ci.lr = c.lr * scale[i];
    float pi = p[i], mi = m[i], vi = v[i];
    dvgo::adam_update(ci, pi, g[i], mi, vi);
    p[i] = pi;
    m[i] = mi;
    v[i] = vi;
    g[i] = 0.0f;
}

}  // namespace

extern "C" {

size_t dvgo_coarse_workspace_bytes(int32_t B) {
    if (B < 0) return 0;
    return dvgo::align_up(static_cast<size_t>(B) * 4, 256) + 256;
}

int32_t dvgo_coarse_step(const dvgo_coarse_field* field, const float* rays_o, const float* rays_d,
                         const float* jitter, const float* t_near, const int32_t* perm, const int32_t* ray_offset,
                         const int32_t* sample_k, const int64_t* n_kept, int64_t capacity, int32_t B, int32_t max_samples,
                         float step, const float* bg, const float* target, float w_pt, float w_bg, float* rgb,
                         float* grad_density, float* grad_rgb, float* loss, void* workspace, size_t workspace_bytes,
                         void* stream) {
    if (!field || !field->density || !field->rgb || !dvgo::box_ok(&field->box, 2) || !bg || B < 0 || capacity < 0)
        return DVGO_E_ARG;
    if (!(step > 0.0f) || !(w_pt >= 0.0f) || !(w_bg >= 0.0f) || max_samples < 0) return DVGO_E_ARG;
    if (max_samples > 64 * kMaxSteps) return DVGO_E_UNSUPPORTED;
    if (static_cast<int64_t>(field->box.n[0]) * field->box.n[1] * field->box.n[2] >= (1LL << 31))
        return DVGO_E_UNSUPPORTED;
    if (B > 0 && (!rays_o || !rays_d || !t_near || !perm || !ray_offset || !n_kept || !target || !grad_density ||
                  !grad_rgb || !loss))
        return DVGO_E_ARG;
    if (capacity > 0 && !sample_k) return DVGO_E_ARG;
    if (workspace_bytes < dvgo_coarse_workspace_bytes(B) || (B > 0 && !workspace)) return DVGO_E_CAPACITY;
    if (B == 0) return DVGO_OK;
    CoarseArgs a;
    a.rays_o = rays_o;
    a.rays_d = rays_d;
    a.jitter = jitter;
    a.t_near = t_near;
    a.perm = perm;
    a.ray_offset = ray_offset;
    a.sample_k = sample_k;
    a.n_kept = n_kept;
    a.cap = capacity;
    a.B = B;
    a.step = step;
    a.g = dvgo::make_grid(field->box);
    a.density = field->density;
    a.rgb = field->rgb;
    a.act_shift = field->act_shift;
    for (int i = 0; i < 3; ++i) a.bg[i] = bg[i];
    a.target = target;
    a.w_pt = w_pt;
    a.w_bg = w_bg;
    a.rgb_out = rgb;
    a.ray_loss = static_cast<float*>(workspace);
    a.grad_density = grad_density;
    a.grad_rgb = grad_rgb;
    hipStream_t s = dvgo::as_stream(stream);
    DVGO_LAUNCH(K_COARSE_STEP, coarse_step_kernel, dim3((B + 3) / 4), dim3(256), 0, s, a);
    if (int32_t st = dvgo::launch_status()) return st;
    DVGO_LAUNCH(K_REDUCE, ray_loss_reduce_kernel, dim3(1), dim3(256), 0, s, a.ray_loss, B,
                1.0f / static_cast<float>(B), loss);
    return dvgo::launch_status();
}

size_t dvgo_view_counts_workspace_bytes(void) { return 256; }

int32_t dvgo_view_counts(const dvgo_box* box, const float* cams, int32_t ncam, int32_t H, int32_t W, float focal,
                         int32_t* counts, float* lr_scale, void* workspace, size_t workspace_bytes, void* stream) {
    if (!dvgo::box_ok(box, 2) || ncam < 0 || (ncam > 0 && !cams) || H < 1 || W < 1 || !(focal > 0.0f) || !counts ||
        !lr_scale)
        return DVGO_E_ARG;
    if (!workspace || workspace_bytes < dvgo_view_counts_workspace_bytes()) return DVGO_E_CAPACITY;
    const int64_t nv = static_cast<int64_t>(box->n[0]) * box->n[1] * box->n[2];
    if (nv >= (1LL << 31)) return DVGO_E_UNSUPPORTED;
    VcArgs a;
    for (int i = 0; i < 3; ++i) {
        a.mn[i] = box->xyz_min[i];
        volatile float span = box->xyz_max[i] - box->xyz_min[i];
        volatile float nm1 = static_cast<float>(box->n[i] - 1);
        a.stepv[i] = span / nm1;
        a.n[i] = box->n[i];
    }
    a.cams = cams;
    a.ncam = ncam;
    a.H = H;
    a.W = W;
    a.focal = focal;
    int* nmax = static_cast<int*>(workspace);
    hipStream_t s = dvgo::as_stream(stream);
    const unsigned blocks = static_cast<unsigned>((nv + 255) / 256);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(1), 0, s, nmax);
    if (int32_t st = dvgo::launch_status()) return st;
    DVGO_LAUNCH(K_VIEW_COUNT, view_count_kernel, dim3(blocks), dim3(256), 0, s, a, counts, nmax);
    if (int32_t st = dvgo::launch_status()) return st;
    DVGO_LAUNCH(K_VIEW_COUNT, view_scale_kernel, dim3(blocks), dim3(256), 0, s, counts, nv, nmax, lr_scale);
    return dvgo::launch_status();
}

int32_t dvgo_adam_step_scaled(float* p, float* g, float* m, float* v, const float* lr_scale, int64_t n, float lr,
                              float beta1, float beta2, float eps, int32_t t, void* stream) {
    if (n < 0 || (n > 0 && (!p || !g || !m || !v || !lr_scale)) || !dvgo::adam_hyper_ok(beta1, beta2, eps, t))
        return DVGO_E_ARG;
    if (n == 0) return DVGO_OK;
    const dvgo::AdamCoef c = dvgo::adam_coef(lr, beta1, beta2, eps, t);
    DVGO_LAUNCH(K_ADAM, adam_scaled_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                dvgo::as_stream(stream), p, g, m, v, lr_scale, n, c);
    return dvgo::launch_status();
}

}  // extern "C"
