// Forward volume rendering of the fine stage and its adjoint (paper
// Eq. volume_rendering, Eq. fine_queries, Eq. post_activation,
// Eq. density_activation, Eq. photo_loss).
//
// One render call runs a short pipeline of kernels over the compact sample
// list written by dvgo_sample_rays; per-sample intermediates live in the
// caller's workspace:
//   prep     pack the network weights into matrix-core operand order;
//            per-ray view encoding PE(d) and the first layer's per-ray part
//   gather   trilinear density and feature interpolation per sample
//   mlp      colour network on float32 (or bfloat16) matrix cores
//   compose  per-ray front-to-back compositing with wavefront prefix scans
// and the backward pass adds
//   compose' walk each ray from its end (suffix scans from log_t_end)
//   mlp'     network adjoint, per-block weight-gradient partials
//   scatter  transpose of the trilinear interpolation: samples binned by
//            grid cell, one thread per vertex gathers its gradient (no
//            float atomics), the grids' Adam step fused in
//   reduce   deterministic sum of the per-block weight-gradient partials
#include "adam.hpp"
#include "common.hpp"
#include "mlp_mfma.hpp"
#include "scan.hpp"

using dvgo::GridArgs;
using namespace dvgo_dev;

namespace {

constexpr int kMaxBwdBlocks = 256;

struct WsLayout {
    size_t base, pe, w1p, w2p, w2tp, w1pb, w2pb, w2tpb, w3pb, w3tpb, w1tpb, raw, feat, col, partial, cell_count,
        cell_start, scan_tmp, cell_rank, rec_head, rec, step_rgb, step_grad, step_logt, step_sqerr, total;
};

constexpr int kScanPer = 8192;   // elements per block of the device-wide scan

WsLayout ws_layout(int64_t B, int64_t cap, int64_t ncell) {
    WsLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = dvgo::align_up(off + bytes, 256);
        return o;
    };
    L.base = take(static_cast<size_t>(B) * kH * 4);
    L.pe = take(static_cast<size_t>(B) * 32 * 4);
    L.w1p = take(kW1PackF32Max * 4);
    L.w2p = take(kW2PackF32 * 4);
    L.w2tp = take(kW2PackF32 * 4);
    L.w1pb = take(kW1PackBF16Max * 2);
    L.w2pb = take(kW2PackBF16 * 2);
    L.w2tpb = take(kW2PackBF16 * 2);
    L.w3pb = take(kW3PackBF16 * 2);
    L.w3tpb = take(kW3TPackBF16 * 2);
    L.w1tpb = take(kW1TPackBF16 * 2);
    L.raw = take(static_cast<size_t>(cap) * 4);
    L.feat = take(static_cast<size_t>(cap) * kC * 4);
    L.col = take(static_cast<size_t>(cap) * 4 * 4);
    L.partial = take(static_cast<size_t>(kMaxBwdBlocks) * kPStrideMax * 4);
    L.cell_count = take(static_cast<size_t>(ncell + 1) * 4);
    L.cell_start = take(static_cast<size_t>(ncell + 1) * 4);
    L.scan_tmp = take(static_cast<size_t>((ncell + 1 + kScanPer - 1) / kScanPer + 1) * 8);
    L.cell_rank = take(static_cast<size_t>(cap) * 8);
    L.rec_head = take(static_cast<size_t>(cap) * 16);
    L.rec = take(static_cast<size_t>(cap) * 64);
    L.step_rgb = take(static_cast<size_t>(B) * 3 * 4);    // per-ray state of dvgo_train_step
    L.step_grad = take(static_cast<size_t>(B) * 3 * 4);
    L.step_logt = take(static_cast<size_t>(B) * 4);
    L.step_sqerr = take(static_cast<size_t>(B) * 4);
    L.total = off;
    return L;
}

// ---------------------------------------------------------------------------
// per-sample geometry (float32 recipe for t and x) and trilinear weights
// ---------------------------------------------------------------------------
struct SampleArgs {
    const float* rays_o;
    const float* rays_d;
    const float* jitter;
    const float* t_near;
    const int* sample_ray;
    const int* sample_k;
    float step;
};

__device__ __forceinline__ void sample_point(const SampleArgs& a, int r, int k, float x[3], float* t_out) {
    float o[3], d[3];
    for (int i = 0; i < 3; ++i) {
        o[i] = a.rays_o[3 * r + i];
        d[i] = a.rays_d[3 * r + i];
    }
    const float p = a.jitter ? a.jitter[r] : 0.0f;
    const float t = recipe_tk(a.t_near[r], p, k, a.step);
    recipe_x(o, d, t, x);
    if (t_out) *t_out = t;
}

struct Tri {
    int64_t base;   // linear vertex index of corner (0,0,0)
    int sx, sy;     // vertex strides of x and y (z stride 1)
    float w[8];     // corner c = (c>>2 &1, c>>1 &1, c &1)
};

__device__ __forceinline__ Tri trilinear(const GridArgs& g, const float x[3]) {
    int i0[3];
    float f[3];
    for (int i = 0; i < 3; ++i) {
        const float u = (x[i] - g.mn[i]) * g.scale[i];
        const float fl = fminf(fmaxf(floorf(u), 0.0f), static_cast<float>(g.n[i] - 2));
        i0[i] = static_cast<int>(fl);
        f[i] = fminf(fmaxf(u - fl, 0.0f), 1.0f);
    }
    Tri t;
    t.sy = g.n[2];
    t.sx = g.n[1] * g.n[2];
    t.base = (static_cast<int64_t>(i0[0]) * g.n[1] + i0[1]) * g.n[2] + i0[2];
    const float gx[2] = {1.0f - f[0], f[0]}, gy[2] = {1.0f - f[1], f[1]}, gz[2] = {1.0f - f[2], f[2]};
    for (int c = 0; c < 8; ++c) t.w[c] = gx[(c >> 2) & 1] * gy[(c >> 1) & 1] * gz[c & 1];
    return t;
}

__device__ __forceinline__ int64_t corner(const Tri& t, int c) {
    return t.base + ((c >> 2) & 1) * static_cast<int64_t>(t.sx) + ((c >> 1) & 1) * t.sy + (c & 1);
}

__device__ __forceinline__ float softplus_f(float x) {
    return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x)));
}
__device__ __forceinline__ float sigmoid_f(float x) { return 1.0f / (1.0f + expf(-x)); }

__device__ __forceinline__ int64_t live_count(const int64_t* n_kept, int64_t cap) {
    const int64_t n = *n_kept;
    return n < cap ? n : cap;
}

// ---------------------------------------------------------------------------
// prep: per-ray encodings and first-layer per-ray part
// ---------------------------------------------------------------------------
// base[r][i] = b1[i] + sum_q W1[i][view_col+q] * PE(d_r)[q];  pe[r] = [PE(d_r) (27), 1, 0, 0, 0, 0]
// (view_col: the view part's first column, after the per-sample inputs;
// w1_in: the row stride of W1)
// Per-call preparation, one workgroup role per block: the first
// kPackThreads/256 workgroups pack the network's operands; each following
// workgroup takes kPrepRays rays: 12 threads per ray evaluate its 24 sines
// and cosines once into LDS, then each thread forms one output of the first
// layer's view part for half of the rays; the last zblocks workgroups clear
// the backward's cell counts.
constexpr int kPrepRays = 16;   // rays per workgroup of the preparation
struct PrepArgs {
    PackArgs pk;
    const float* rays_d;
    int B;
    const float* w1;
    const float* b1;
    int w1_in;      // row stride of W1
    int view_col;   // first column of W1's view part
    float* base;
    float* pe;
    int* zero;      // cleared (NULL: none)
    int64_t nzero;
    int zblocks;
    int blocks;     // workgroups of the preparation
};

__device__ __forceinline__ void prep_body(const PrepArgs& P, int blk) {
    constexpr int kPackBlocks = kPackThreads / 256;
    if (blk < kPackBlocks) {
        pack_weights(P.pk, blk * 256 + threadIdx.x);
        return;
    }
    const int B = P.B, w1_in = P.w1_in, view_col = P.view_col, zblocks = P.zblocks;
    const float* __restrict__ rays_d = P.rays_d;
    const float* __restrict__ w1 = P.w1;
    const float* __restrict__ b1 = P.b1;
    float* __restrict__ base = P.base;
    float* __restrict__ pe = P.pe;
    int* __restrict__ zero = P.zero;
    const int64_t nzero = P.nzero;
    const int ray_blocks = (B + kPrepRays - 1) / kPrepRays;
    const int zb = blk - kPackBlocks - ray_blocks;
    if (zb >= 0) {   // the last zblocks workgroups clear `zero` (the backward's cell counts)
        const int64_t stride = static_cast<int64_t>(zblocks) * 256, first = static_cast<int64_t>(zb) * 256 + threadIdx.x;
        int64_t done = 0;
        if ((reinterpret_cast<uintptr_t>(zero) & 15u) == 0) {   // 16-byte stores, then the tail
            int4* z4 = reinterpret_cast<int4*>(zero);
            const int64_t n4 = nzero / 4;
            for (int64_t i = first; i < n4; i += stride) z4[i] = make_int4(0, 0, 0, 0);
            done = 4 * n4;
        }
        for (int64_t i = done + first; i < nzero; i += stride) zero[i] = 0;
        return;
    }
    __shared__ float se[kPrepRays][32];
    const int t = threadIdx.x;
    const int r0 = kPrepRays * (blk - kPackBlocks);
    if (t < 12 * kPrepRays) {
        const int rr = t / 12, q = t % 12, fq = q / 3, c = q % 3;
        const int r = r0 + rr;
        if (r < B) {
            const float dc = rays_d[3 * r + c];
            float sv, cv;
            sincosf(dc * static_cast<float>(1 << fq), &sv, &cv);
            se[rr][3 + 6 * fq + c] = sv;
            se[rr][6 + 6 * fq + c] = cv;
            if (fq == 0) se[rr][c] = dc;
        }
    }
    if (t < 5 * kPrepRays)   // entry 27: the first layer's constant input; 28..31 zero
        se[t / 5][kPE + t % 5] = t % 5 == 0 ? 1.0f : 0.0f;
    __syncthreads();
    // thread (h, i) forms output i for rays h, h + 2, ...; its weights stay in
    // registers across the rays
    const int h = t >> 7, i = t & (kH - 1);
    float wv[kPE];
    const float bi = w1 ? b1[i] : 0.0f;
    if (w1) {
        #pragma unroll
        for (int q = 0; q < kPE; ++q) wv[q] = w1[i * w1_in + view_col + q];
    }
    for (int rr = h; rr < kPrepRays; rr += 2) {
        const int r = r0 + rr;
        if (r >= B) break;
        if (w1) {
            float acc = bi;
            #pragma unroll
            for (int q = 0; q < kPE; ++q) acc += wv[q] * se[rr][q];
            base[static_cast<int64_t>(r) * kH + i] = acc;
        }
        if (i < 32) pe[static_cast<int64_t>(r) * 32 + i] = se[rr][i];
    }
}

__global__ __launch_bounds__(256) void prep_kernel(PrepArgs P) { prep_body(P, blockIdx.x); }

// ---------------------------------------------------------------------------
// gather: raw density and interpolated features per sample
// ---------------------------------------------------------------------------
struct GatherArgs {
    SampleArgs sa;
    GridArgs g;
    const float* density;
    const void* feat;
    int feat_bf16;
    int with_feat;
    const int64_t* n_kept;
    int64_t cap;
    float* raw_out;
    float* feat_out;
};

// kFeat: 0 density only, 1 float32 features, 2 bfloat16 features.  One
// instantiation per case, so that every corner load of a sample (density and
// features) is issued before any of them is consumed.  Workgroup blk of nblk
// takes samples blk*256 + thread, then every nblk*256-th.
template <int kFeat>
__device__ __forceinline__ void gather_body(const GatherArgs& a, int blk, int nblk) {
    const int64_t n = live_count(a.n_kept, a.cap);
    for (int64_t s = static_cast<int64_t>(blk) * blockDim.x + threadIdx.x; s < n;
         s += static_cast<int64_t>(nblk) * blockDim.x) {
        const int r = a.sa.sample_ray[s];
        const int k = a.sa.sample_k[s];
        float x[3];
        sample_point(a.sa, r, k, x, nullptr);
        const Tri t = trilinear(a.g, x);
        float d[8];
        float4 q[8][3];
        #pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t v = corner(t, c);
            d[c] = a.density[v];
            if (kFeat == 1) {
                const float4* F = static_cast<const float4*>(a.feat) + 3 * v;
                q[c][0] = F[0];
                q[c][1] = F[1];
                q[c][2] = F[2];
            } else if (kFeat == 2) {
                const uint2* F = static_cast<const uint2*>(a.feat) + 3 * v;
                #pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const uint2 u = F[e];
                    q[c][e] = make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xFFFF0000u),
                                          __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xFFFF0000u));
                }
            }
        }
        float raw = 0.0f;
        #pragma unroll
        for (int c = 0; c < 8; ++c) raw += t.w[c] * d[c];
        a.raw_out[s] = raw;
        if (kFeat == 0) continue;
        float4 f[3] = {make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0)};
        #pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float w = t.w[c];
            #pragma unroll
            for (int e = 0; e < 3; ++e) {
                f[e].x += w * q[c][e].x;
                f[e].y += w * q[c][e].y;
                f[e].z += w * q[c][e].z;
                f[e].w += w * q[c][e].w;
            }
        }
        float4* out = reinterpret_cast<float4*>(a.feat_out + s * kC);
        out[0] = f[0];
        out[1] = f[1];
        out[2] = f[2];
    }
}

template <int kFeat>
__global__ __launch_bounds__(256) void gather_kernel(GatherArgs a) { gather_body<kFeat>(a, blockIdx.x, gridDim.x); }

// The gather and the per-call preparation in one launch (the two are
// independent: the preparation's workgroups fill the gather's latency-bound
// schedule, 6-9 us per training step at the full configuration): the first
// gather_blocks workgroups gather, the others prepare.
template <int kFeat>
__global__ __launch_bounds__(256) void prep_gather_kernel(PrepArgs P, GatherArgs a, int gather_blocks) {
    const int blk = static_cast<int>(blockIdx.x);
    if (blk < gather_blocks) gather_body<kFeat>(a, blk, gather_blocks);
    else prep_body(P, blk - gather_blocks);
}

// ---------------------------------------------------------------------------
// compose: one wavefront per ray slot, 64 samples per step, prefix scans
// ---------------------------------------------------------------------------
struct ComposeArgs {
    SampleArgs sa;
    const int* perm;
    const int* ray_offset;
    const int* n_uniform;
    const int64_t* n_kept;
    int64_t cap;
    int B;
    float act_shift;
    float bg[3];
    float* raw;        // in: raw density; out (backward): dL/draw
    float* col;        // in: colour [cap][4]; out (backward): dL/dc
    int with_color;
    // forward outputs
    float* rgb;
    float* depth;
    float* acc;
    float* log_t_end;
    float* seg_w;
    float* sample_w;
    // forward, inside dvgo_train_step: the photometric loss's gradient and
    // each ray's loss (summed later in a fixed order); with w_pt or w_bg also
    // the per-point rgb and background entropy terms (the backward reads
    // target for the per-point term)
    const float* target;
    float* grad_rgb_out;
    float* sq_err;
    float w_pt, w_bg;
    // backward inputs
    const float* log_t_end_in;
    const float* grad_rgb;
    const float* grad_depth;
    const float* grad_acc;
    // backward binning by fine cell (cell_count == nullptr: off)
    GridArgs g;
    int* cell_count;       // [ncell + 1], zero on entry
    int2* cell_rank;       // [cap] (cell, rank within cell)
    float4* rec_head;      // [cap] (fx, fy, fz, dL/draw)
    // forward without a network: each sample's raw density interpolated
    // here from this grid (on g) instead of read from raw
    const float* density_in;
};

// Fine cell of a point (its vertex (0,0,0)) and the fractional position f
// inside it, clamped like the trilinear interpolation.
__device__ __forceinline__ int cell_of(const GridArgs& g, const float x[3], float f[3]) {
    int i0[3];
    for (int i = 0; i < 3; ++i) {
        const float u = (x[i] - g.mn[i]) * g.scale[i];
        const float fl = fminf(fmaxf(floorf(u), 0.0f), static_cast<float>(g.n[i] - 2));
        i0[i] = static_cast<int>(fl);
        f[i] = fminf(fmaxf(u - fl, 0.0f), 1.0f);
    }
    return (i0[0] * (g.n[1] - 1) + i0[1]) * (g.n[2] - 1) + i0[2];
}

// Rank of this lane's sample among the samples of its cell.  Lanes hold
// consecutive samples, so equal cells form runs; each run's first lane adds
// the run length to the cell's count with one atomic, and the run shares the
// returned base.  All 64 lanes must call it; lanes with ok == false take part
// in the vote only.
__device__ __forceinline__ int run_rank(int cell, bool ok, int lane, int* __restrict__ counts) {
    const int prev = __shfl_up(cell, 1, 64);
    const bool head = !ok || lane == 0 || prev != cell;
    const uint64_t heads = __ballot(head);
    const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1);
    const uint64_t le = heads & upto;
    const int leader = 63 - __clzll(static_cast<long long>(le));
    const uint64_t gt = heads & ~upto;
    const int next = gt ? __ffsll(static_cast<long long>(gt)) - 1 : 64;
    int rbase = 0;
    if (ok && lane == leader) rbase = atomicAdd(counts + cell, next - lane);
    rbase = __shfl(rbase, leader, 64);
    return rbase + lane - leader;
}

// Forward compositing of ray slot `slot` by one wavefront (segs: its 32
// segment sums in LDS).  With a.target it also forms the photometric
// gradient dL/dC; every lane returns that gradient in g and log T_end in
// *log_t_end (what a fused adjoint needs).
template <bool kInline>   // kInline: the raw densities interpolated here (a.density_in)
__device__ __forceinline__ void compose_fwd_ray(const ComposeArgs& a, int slot, int lane, float* segs, float g[3],
                                                float* log_t_end) {
    const int64_t n = live_count(a.n_kept, a.cap);
    const int r = a.perm[slot];
    int64_t s0 = a.ray_offset[slot], s1 = a.ray_offset[slot + 1];
    s0 = s0 < n ? s0 : n;
    s1 = s1 < n ? s1 : n;
    const int nu = a.n_uniform[r];
    const float tn = a.sa.t_near[r];
    const float p = a.sa.jitter ? a.sa.jitter[r] : 0.0f;
    const float step = a.sa.step;
    float ro[3] = {0.0f, 0.0f, 0.0f}, rd[3] = {0.0f, 0.0f, 0.0f};   // the ray, for the inline density
    if (kInline)
        for (int i = 0; i < 3; ++i) {
            ro[i] = a.sa.rays_o[3 * r + i];
            rd[i] = a.sa.rays_d[3 * r + i];
        }
    if (lane < 32) segs[lane] = 0.0f;
    __builtin_amdgcn_wave_barrier();
    float logT = 0.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, dep = 0.0f, accw = 0.0f, ptl = 0.0f;
    float tg[3] = {0.0f, 0.0f, 0.0f};
    if (a.w_pt > 0.0f)
        for (int c = 0; c < 3; ++c) tg[c] = a.target[3 * r + c];
    for (int64_t base = s0; base < s1; base += 64) {
        const int64_t s = base + lane;
        const bool ok = s < s1;
        float sd = 0.0f, alpha = 0.0f, tk = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
        int k = 0;
        if (ok) {
            k = a.sa.sample_k[s];
            tk = recipe_tk(tn, p, k, step);
            float raw;
            if (kInline) {   // the gather's interpolation, in its order
                float x[3];
                recipe_x(ro, rd, tk, x);
                const Tri t = trilinear(a.g, x);
                float dv[8];
                #pragma unroll
                for (int c = 0; c < 8; ++c) dv[c] = a.density_in[corner(t, c)];
                raw = 0.0f;
                #pragma unroll
                for (int c = 0; c < 8; ++c) raw += t.w[c] * dv[c];
            } else {
                raw = a.raw[s];
            }
            const float sig = softplus_f(raw + a.act_shift);
            sd = sig * step;
            alpha = -expm1f(-sd);
            if (a.with_color) {
                const float4 c = reinterpret_cast<const float4*>(a.col)[s];
                c0 = c.x; c1 = c.y; c2 = c.z;
            }
        }
        const float incl = wave_incl_scan(sd, lane);
        const float excl = dpp_wave<0x138>(incl);   // wave_shr:1, lane 0 reads 0
        const float w = ok ? expf(logT - excl) * alpha : 0.0f;
        cr += w * c0; cg += w * c1; cb += w * c2;
        dep += w * tk;
        accw += w;
        if (a.w_pt > 0.0f) {   // per-point rgb: w_k ||c_k - C*||^2
            const float e0 = c0 - tg[0], e1 = c1 - tg[1], e2 = c2 - tg[2];
            ptl += w * (e0 * e0 + e1 * e1 + e2 * e2);
        }
        if (ok && a.seg_w) atomicAdd(&segs[(32LL * k) / nu], w);
        if (ok && a.sample_w) a.sample_w[s] = w;
        logT -= lane_value(incl, 63);
    }
    cr = wave_sum(cr); cg = wave_sum(cg); cb = wave_sum(cb);
    dep = wave_sum(dep);
    accw = wave_sum(accw);
    if (a.w_pt > 0.0f) ptl = wave_sum(ptl);
    __builtin_amdgcn_wave_barrier();
    // the ray's colour and loss terms, in every lane (the stores from lane 0)
    const float T = expf(logT);
    g[0] = g[1] = g[2] = 0.0f;
    *log_t_end = logT;
    if (a.rgb) {
        const float c3[3] = {cr + T * a.bg[0], cg + T * a.bg[1], cb + T * a.bg[2]};
        if (lane == 0) {
            a.rgb[3 * r + 0] = c3[0];
            a.rgb[3 * r + 1] = c3[1];
            a.rgb[3 * r + 2] = c3[2];
        }
        if (a.target) {   // Eq. photo_loss: gradient 2 (C - C*)/B, as dvgo_photo_loss forms it
            const float invB = 1.0f / static_cast<float>(a.B);
            float e2 = 0.0f;
            for (int c = 0; c < 3; ++c) {
                const float d = c3[c] - a.target[3 * r + c];
                g[c] = 2.0f * d * invB;
                e2 += d * d;
            }
            if (a.w_pt > 0.0f) e2 += a.w_pt * ptl;
            if (a.w_bg > 0.0f) {   // background entropy of T_end, clamped to [1e-6, 1 - 1e-6]
                const float pb = fminf(fmaxf(T, 1e-6f), 1.0f - 1e-6f);
                e2 += a.w_bg * (-pb * logf(pb) - (1.0f - pb) * log1pf(-pb));
            }
            if (lane == 0) {
                for (int c = 0; c < 3; ++c) a.grad_rgb_out[3 * r + c] = g[c];
                a.sq_err[r] = e2;
            }
        }
    }
    if (lane == 0) {
        if (a.depth) a.depth[r] = dep;
        if (a.acc) a.acc[r] = accw;
        a.log_t_end[r] = logT;
    }
    if (a.seg_w && lane < 32) a.seg_w[static_cast<int64_t>(r) * 32 + lane] = segs[lane];
}

// Wavefronts (rays) per workgroup of the compositing kernels: one, so that a
// long ray holds only its own slot (with four, a workgroup's resources stayed
// held until its longest ray was done: the training step's compositing took
// 1 us longer).
constexpr int kComposeWaves = 1;
constexpr int kComposeThreads = 64 * kComposeWaves;
inline dim3 compose_grid(int B) { return dim3((B + kComposeWaves - 1) / kComposeWaves); }

template <bool kInline>
__global__ __launch_bounds__(kComposeThreads) void compose_fwd_kernel(ComposeArgs a) {
    __shared__ float segs[kComposeWaves][32];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = blockIdx.x * kComposeWaves + wave;
    if (slot >= a.B) return;
    float g[3], lt;
    compose_fwd_ray<kInline>(a, slot, lane, segs[wave], g, &lt);
}

// Backward of compose: walk each ray from its end in 64-sample steps,
// carrying the suffix sums S.  The transmittance is recomputed from the
// samples' densities as the forward forms it, by prefix sums from the ray's
// start: log T at the start of each 64-sample step comes from a first pass
// over the ray's steps (lane j keeps the start of step j), so T_k, T_{k+1}
// and w_k are the forward's values bit for bit.  (Forming log T_k as
// log T_end plus the suffix of sigma*delta would cancel: with an optical
// depth D along the ray it loses D*2^-24 of absolute accuracy in log T.)
// Rays of more than 64 steps take the first pass once per group of 64.
__device__ __forceinline__ float sd_of(const ComposeArgs& a, int64_t s, int64_t s1) {
    return s < s1 ? softplus_f(a.raw[s] + a.act_shift) * a.sa.step : 0.0f;
}

// The adjoint of ray slot `slot` by one wavefront.  gin (dL/dC) and
// log_t_end come from the fused forward's registers, or (gin NULL) from
// a.grad_rgb and a.log_t_end_in.
__device__ __forceinline__ void compose_bwd_ray(const ComposeArgs& a, int slot, int lane, const float* gin,
                                                float log_t_end) {
    const int64_t n = live_count(a.n_kept, a.cap);
    const int r = a.perm[slot];
    int64_t s0 = a.ray_offset[slot], s1 = a.ray_offset[slot + 1];
    s0 = s0 < n ? s0 : n;
    s1 = s1 < n ? s1 : n;
    // (r < 0 never holds; testing it keeps the ray's load in flight with
    // the offsets' instead of after this test)
    if (s1 <= s0 || r < 0) return;
    const float tn = a.sa.t_near[r];
    const float p = a.sa.jitter ? a.sa.jitter[r] : 0.0f;
    const float step = a.sa.step;
    float g[5];
    g[0] = gin ? gin[0] : a.grad_rgb ? a.grad_rgb[3 * r + 0] : 0.0f;
    g[1] = gin ? gin[1] : a.grad_rgb ? a.grad_rgb[3 * r + 1] : 0.0f;
    g[2] = gin ? gin[2] : a.grad_rgb ? a.grad_rgb[3 * r + 2] : 0.0f;
    g[3] = a.grad_depth ? a.grad_depth[r] : 0.0f;
    g[4] = a.grad_acc ? a.grad_acc[r] : 0.0f;
    float ro[3] = {0.0f, 0.0f, 0.0f}, rd[3] = {0.0f, 0.0f, 0.0f};   // the ray, for the binning
    if (a.cell_count) {
        for (int i = 0; i < 3; ++i) {
            ro[i] = a.sa.rays_o[3 * r + i];
            rd[i] = a.sa.rays_d[3 * r + i];
        }
    }
    const float Tend = expf(gin ? log_t_end : a.log_t_end_in[r]);
    float S[5] = {Tend * a.bg[0], Tend * a.bg[1], Tend * a.bg[2], 0.0f, 0.0f};
    // auxiliary losses: the background entropy's gradient on T_end reaches
    // every sample through dT_end/dsigma_k = -delta T_end; the per-point rgb
    // loss adds 2 w_pt w_k (c_k - C*)/B to each colour's gradient
    const float invB = 1.0f / static_cast<float>(a.B);
    float dsig_bg = 0.0f;
    if (a.w_bg > 0.0f && Tend > 1e-6f && Tend < 1.0f - 1e-6f)
        dsig_bg = -Tend * a.w_bg * (log1pf(-Tend) - logf(Tend)) * invB;
    float tg[3] = {0.0f, 0.0f, 0.0f};
    if (a.w_pt > 0.0f)
        for (int c = 0; c < 3; ++c) tg[c] = a.target[3 * r + c];
    const float ptk = 2.0f * a.w_pt * invB;
    const int64_t nsteps = (s1 - s0 + 63) / 64;
    const int64_t ngroups = (nsteps + 63) / 64;
    for (int64_t grp = ngroups - 1; grp >= 0; --grp) {
        // log T at the start of steps 64*grp .. 64*grp+63, lane j holding step 64*grp+j
        const int64_t first = 64 * grp, last = first + 63 < nsteps - 1 ? first + 63 : nsteps - 1;
        float start = 0.0f;
        float logT = 0.0f;
        for (int64_t j = 0; j < last; ++j) {
            if (j >= first && lane == static_cast<int>(j - first)) start = logT;
            logT -= wave_sum(sd_of(a, s0 + j * 64 + lane, s1));
        }
        if (lane == static_cast<int>(last - first)) start = logT;
        for (int64_t it = last; it >= first; --it) {
            const int64_t s = s0 + it * 64 + lane;
            const bool ok = s < s1;
            float sd = 0.0f, raw = 0.0f, tk = 0.0f, v[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            if (ok) {
                raw = a.raw[s];
                sd = softplus_f(raw + a.act_shift) * step;
                tk = recipe_tk(tn, p, a.sa.sample_k[s], step);
                if (a.with_color) {
                    const float4 c = reinterpret_cast<const float4*>(a.col)[s];
                    v[0] = c.x; v[1] = c.y; v[2] = c.z;
                }
                v[3] = tk;
                v[4] = 1.0f;
            }
            const float logT0 = lane_value(start, static_cast<int>(it - first));
            const float incl = wave_incl_scan(sd, lane);
            const float excl = dpp_wave<0x138>(incl);   // wave_shr:1, lane 0 reads 0
            const float Tafter = expf(logT0 - incl);     // T_{k+1}
            const float w = ok ? expf(logT0 - excl) * -expm1f(-sd) : 0.0f;   // T_k alpha_k, as the forward
            float dsig = dsig_bg;
            float tot[5];
            for (int ch = 0; ch < 5; ++ch) {
                const float wv = w * v[ch];
                const float sfx = wave_incl_suffix(wv, lane);
                const float sfx_ex = dpp_wave<0x130>(sfx);   // wave_shl:1, lane 63 reads 0
                dsig += g[ch] * (Tafter * v[ch] - (S[ch] + sfx_ex));
                tot[ch] = lane_value(sfx, 0);
            }
            const float draw = step * dsig * sigmoid_f(raw + a.act_shift);
            if (ok) {
                a.raw[s] = draw;
                if (a.with_color) {
                    float4 dc = make_float4(w * g[0], w * g[1], w * g[2], 0.0f);
                    if (a.w_pt > 0.0f) {
                        dc.x += ptk * w * (v[0] - tg[0]);
                        dc.y += ptk * w * (v[1] - tg[1]);
                        dc.z += ptk * w * (v[2] - tg[2]);
                    }
                    reinterpret_cast<float4*>(a.col)[s] = dc;
                }
            }
            if (a.cell_count) {   // bin the sample by fine cell (wave-uniform branch)
                int cell = -1;
                if (ok) {
                    float x[3], f[3];
                    recipe_x(ro, rd, tk, x);   // the sample's point, as sample_point forms it
                    cell = cell_of(a.g, x, f);
                    a.rec_head[s] = make_float4(f[0], f[1], f[2], draw);
                }
                const int rank = run_rank(cell, ok, lane, a.cell_count);
                if (ok) a.cell_rank[s] = make_int2(cell, rank);
            }
            for (int ch = 0; ch < 5; ++ch) S[ch] += tot[ch];
        }
    }
}

__global__ __launch_bounds__(kComposeThreads) void compose_bwd_kernel(ComposeArgs a) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = blockIdx.x * kComposeWaves + wave;
    if (slot >= a.B) return;
    compose_bwd_ray(a, slot, lane, nullptr, 0.0f);
}

// The training step's compositing and its adjoint in one launch: each
// wavefront composites its ray (forward outputs, loss terms, dL/dC), then
// walks it back with dL/dC and log T_end from its registers.  The adjoint
// of a ray depends only on that ray's forward, so no other wavefront waits.
__global__ __launch_bounds__(kComposeThreads) void compose_step_kernel(ComposeArgs fa, ComposeArgs ba) {
    __shared__ float segs[kComposeWaves][32];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = blockIdx.x * kComposeWaves + wave;
    if (slot >= fa.B) return;
    float g[3], lt;
    compose_fwd_ray<false>(fa, slot, lane, segs[wave], g, &lt);
    compose_bwd_ray(ba, slot, lane, g, lt);
}

// ---------------------------------------------------------------------------
// scatter: transpose of the trilinear gathers, without float atomics.
// Samples are counting-sorted by fine cell (one integer atomic per run of
// equal cells in a wavefront), then one thread per grid vertex sums the
// contributions of the samples in its 8 neighbouring cells and adds them to
// the gradient with a plain read-modify-write.
// ---------------------------------------------------------------------------
struct BinArgs {
    SampleArgs sa;
    GridArgs g;
    const int64_t* n_kept;
    int64_t cap;
    int* cell_count;       // [ncell + 1]
    const int* cell_start; // [ncell + 1]
    int2* cell_rank;       // [cap] (cell, rank within cell)
    const float4* rec_head;  // [cap] (fx, fy, fz, draw)
    int with_feat;         // records carry dL/dfeat
    float4* rec;           // [cap][4] in binned order: (fx, fy, fz, draw), df[0..11]
    float* grad_density;
    float* grad_feat;
    int64_t ncell;
};


__global__ __launch_bounds__(256) void fill_int_kernel(int* __restrict__ p, int64_t n, int v) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}


// Records in binned order when no network backward places them (density
// only): the head (fractional position, dL/draw) at cell start + rank.
__global__ __launch_bounds__(256) void bin_place_kernel(BinArgs a) {
    const int64_t n = live_count(a.n_kept, a.cap);
    for (int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; s < n;
         s += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int2 cr = a.cell_rank[s];
        const int64_t pos = static_cast<int64_t>(a.cell_start[cr.x]) + cr.y;
        a.rec[pos * 4] = a.rec_head[s];
    }
}

// Gradient of one vertex (i,j,k): it is corner (dx,dy,dz) of cell
// (i-dx, j-dy, k-dz); the samples binned in those cells are summed with the
// vertex's trilinear weight.  acc[0] density, acc[1..12] features.  Returns
// whether any sample touches the vertex.  For each (dx, dy) the cells k-1
// (dz = 1) and k (dz = 0) are neighbours in the cell order, so their records
// form one run, split at the start of cell k; the run is walked two records
// at a time so that two records' loads are in flight together.
__device__ __forceinline__ void add_record(const float4* r, int dx, int dy, int dz, bool feat, float acc[13]) {
    const float4 h = r[0];
    const float w = (dx ? h.x : 1.0f - h.x) * (dy ? h.y : 1.0f - h.y) * (dz ? h.z : 1.0f - h.z);
    acc[0] += w * h.w;
    if (feat) {
        const float4 q0 = r[1], q1 = r[2], q2 = r[3];
        acc[1] += w * q0.x; acc[2] += w * q0.y; acc[3] += w * q0.z; acc[4] += w * q0.w;
        acc[5] += w * q1.x; acc[6] += w * q1.y; acc[7] += w * q1.z; acc[8] += w * q1.w;
        acc[9] += w * q2.x; acc[10] += w * q2.y; acc[11] += w * q2.z; acc[12] += w * q2.w;
    }
}

__device__ __forceinline__ bool vertex_grad(const BinArgs& a, int i, int j, int k, bool feat, float acc[13]) {
    const int nx = a.g.n[0], cy = a.g.n[1] - 1, cz = a.g.n[2] - 1;
    #pragma unroll
    for (int q = 0; q < 13; ++q) acc[q] = 0.0f;
    // the twelve cell starts first, all in flight together
    int p0[4], pm[4], p1[4];
    #pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int dx = (c >> 1) & 1, dy = c & 1;
        const int ci = i - dx, cj = j - dy;
        p0[c] = pm[c] = p1[c] = 0;
        if (ci < 0 || cj < 0 || ci >= nx - 1 || cj >= cy) continue;
        const int row = (ci * cy + cj) * cz;
        const int klo = k > 0 ? k - 1 : 0, khi = k < cz ? k + 1 : cz;   // cells k-1 and k, where they exist
        p0[c] = a.cell_start[row + klo];
        pm[c] = a.cell_start[row + k];
        p1[c] = a.cell_start[row + khi];
    }
    bool any = false;
    #pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int dx = (c >> 1) & 1, dy = c & 1;
        int p = p0[c];
        for (; p + 1 < p1[c]; p += 2) {
            add_record(a.rec + static_cast<int64_t>(p) * 4, dx, dy, p < pm[c], feat, acc);
            add_record(a.rec + static_cast<int64_t>(p + 1) * 4, dx, dy, p + 1 < pm[c], feat, acc);
        }
        if (p < p1[c]) add_record(a.rec + static_cast<int64_t>(p) * 4, dx, dy, p < pm[c], feat, acc);
        any |= p1[c] > p0[c];
    }
    return any;
}

// One thread per vertex: add its gradient into the gradient grids.
__global__ __launch_bounds__(256) void vertex_gather_kernel(BinArgs a) {
    const int ny = a.g.n[1], nz = a.g.n[2];
    const int64_t nv = static_cast<int64_t>(a.g.n[0]) * ny * nz;
    const bool feat = a.with_feat != 0;
    for (int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; v < nv;
         v += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int k = static_cast<int>(v % nz);
        const int j = static_cast<int>((v / nz) % ny);
        const int i = static_cast<int>(v / (static_cast<int64_t>(nz) * ny));
        float acc[13];
        const bool any = vertex_grad(a, i, j, k, feat, acc);
        if (!any) continue;
        a.grad_density[v] += acc[0];
        if (feat) {
            float4* gf = reinterpret_cast<float4*>(a.grad_feat + v * kC);
            float4 g0 = gf[0], g1 = gf[1], g2 = gf[2];
            g0.x += acc[1]; g0.y += acc[2]; g0.z += acc[3]; g0.w += acc[4];
            g1.x += acc[5]; g1.y += acc[6]; g1.z += acc[7]; g1.w += acc[8];
            g2.x += acc[9]; g2.y += acc[10]; g2.z += acc[11]; g2.w += acc[12];
            gf[0] = g0;
            gf[1] = g1;
            gf[2] = g2;
        }
    }
}

// Grid parameters with their Adam moments, updated in place.
struct GridAdamArgs {
    float* pd;
    float* md;
    float* vd;
    float* pf;
    float* mf;
    float* vf;
    uint16_t* shadow;
    uint32_t* active;   // per-vertex bit: moments may be non-zero (NULL: every vertex steps)
    dvgo::AdamCoef c;
};

// One thread per vertex: its gradient as in vertex_gather_kernel, then the
// Adam step of its density and its 12 features (and their bfloat16 copy);
// a vertex no sample touches takes the step with a zero gradient, as dense
// Adam does.  The gradient never reaches memory.  Feature streams are
// walked in wave-contiguous float4 chunks (the 64 vertices of a wave own
// 768 consecutive values): the wave's gradients go through LDS so that every
// load and store of p, m, v and the copy covers whole cache lines.
//
// With an activity mask, a vertex whose bit is clear (both moments zero)
// and that no sample touches is skipped: its step would compute m = v = 0
// and p - lr * 0 / (0 + eps) = p, so skipping it changes no bit, and its
// parameters and moments are neither read nor written.  A vertex that takes
// a step with any non-zero gradient gets its bit set.
__device__ __forceinline__ void vertex_adam_body(const BinArgs& a, const GridAdamArgs& o, int blk, int nblk) {
    __shared__ float4 sg[4][64 * 3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ny = a.g.n[1], nz = a.g.n[2];
    const int64_t nv = static_cast<int64_t>(a.g.n[0]) * ny * nz;
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    f4* P = reinterpret_cast<f4*>(o.pf);
    f4* M = reinterpret_cast<f4*>(o.mf);
    f4* V = reinterpret_cast<f4*>(o.vf);
    u2* S = reinterpret_cast<u2*>(o.shadow);
    // Workgroups are dealt to the 8 XCDs round robin (block b on XCD b % 8).
    // The vertices are cut into chunks of two x-planes (rounded up to a
    // multiple of 256), dealt to the XCDs round robin as well: a cell's
    // records and start are read by the vertices of two neighbouring
    // x-planes, which then mostly sit in one chunk and so in one XCD's L2,
    // and every XCD gets an even share of the grid's busy middle (its
    // vertices with moments and samples) and of its idle rim.  The blocks of
    // an XCD walk its chunks in 256-vertex steps.  gridDim.x is a multiple of
    // 8; every wave's first vertex is a multiple of 64, so a wave owns two
    // whole words of the activity mask.
    const int64_t kChunk = (2 * static_cast<int64_t>(ny) * nz + 255) / 256 * 256;
    const int xcd = blk & 7, nloc = nblk >> 3, loc = blk >> 3;
    const int64_t nchunk = (nv + kChunk - 1) / kChunk;
    const int64_t mine = nchunk > xcd ? (nchunk - xcd + 7) / 8 : 0;   // chunks of this XCD
    const int64_t hi = nv;
    for (int64_t l = static_cast<int64_t>(loc) * blockDim.x; l < mine * kChunk;
         l += static_cast<int64_t>(nloc) * blockDim.x) {
        const int64_t base = ((l / kChunk) * 8 + xcd) * kChunk + l % kChunk;   // increases with l
        if (base >= hi) break;
        const int64_t v = base + threadIdx.x;
        const int64_t vbase = base + 64 * wave;
        const int64_t nwave = hi - vbase < 64 ? hi - vbase : 64;   // vertices of this wave (may be <= 0)
        const bool in = v < hi;
        const bool was_active = in && (!o.active || ((o.active[v >> 5] >> (v & 31)) & 1u));
        // issue the parameter streams of the active vertices first: they do
        // not depend on the gradient and overlap the latency of the sample
        // gather below
        const uint64_t act_mask = __ballot(was_active);
        float p = 0.0f, m = 0.0f, w = 0.0f;
        if (was_active) {
            p = __builtin_nontemporal_load(o.pd + v);
            m = __builtin_nontemporal_load(o.md + v);
            w = __builtin_nontemporal_load(o.vd + v);
        }
        f4 pq[3], mq[3], vq[3];
        #pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int c = 64 * q + lane;
            if (c < 3 * nwave && ((act_mask >> (c / 3)) & 1u)) {
                const int64_t gi = 3 * vbase + c;
                pq[q] = __builtin_nontemporal_load(P + gi);
                mq[q] = __builtin_nontemporal_load(M + gi);
                vq[q] = __builtin_nontemporal_load(V + gi);
            }
        }
        float acc[13];
        #pragma unroll
        for (int q = 0; q < 13; ++q) acc[q] = 0.0f;
        bool touched = false;
        if (in && a.cell_start) {   // else no samples in the batch
            const int k = static_cast<int>(v % nz);
            const int j = static_cast<int>((v / nz) % ny);
            const int i = static_cast<int>(v / (static_cast<int64_t>(nz) * ny));
            touched = vertex_grad(a, i, j, k, true, acc);
        }
        // vertices newly reached by a sample: their streams now
        const bool need = was_active || touched;
        const uint64_t need_mask = __ballot(need);
        const uint64_t late_mask = need_mask & ~act_mask;
        if (need && !was_active) {
            p = __builtin_nontemporal_load(o.pd + v);
            m = __builtin_nontemporal_load(o.md + v);
            w = __builtin_nontemporal_load(o.vd + v);
        }
        if (late_mask) {
            #pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int c = 64 * q + lane;
                if (c < 3 * nwave && ((late_mask >> (c / 3)) & 1u)) {
                    const int64_t gi = 3 * vbase + c;
                    pq[q] = __builtin_nontemporal_load(P + gi);
                    mq[q] = __builtin_nontemporal_load(M + gi);
                    vq[q] = __builtin_nontemporal_load(V + gi);
                }
            }
        }
        if (need) {
            dvgo::adam_update(o.c, p, acc[0], m, w);
            __builtin_nontemporal_store(p, o.pd + v);
            __builtin_nontemporal_store(m, o.md + v);
            __builtin_nontemporal_store(w, o.vd + v);
        }
        #pragma unroll
        for (int q = 0; q < 3; ++q)
            sg[wave][3 * lane + q] = make_float4(acc[1 + 4 * q], acc[2 + 4 * q], acc[3 + 4 * q], acc[4 + 4 * q]);
        __syncthreads();
        #pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int c = 64 * q + lane;
            if (c < 3 * nwave && ((need_mask >> (c / 3)) & 1u)) {
                const int64_t gi = 3 * vbase + c;
                const float4 g = sg[wave][c];
                const float gg[4] = {g.x, g.y, g.z, g.w};
                #pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float pe = pq[q][e], me = mq[q][e], ve = vq[q][e];
                    dvgo::adam_update(o.c, pe, gg[e], me, ve);
                    pq[q][e] = pe;
                    mq[q][e] = me;
                    vq[q][e] = ve;
                }
                __builtin_nontemporal_store(pq[q], P + gi);
                __builtin_nontemporal_store(mq[q], M + gi);
                __builtin_nontemporal_store(vq[q], V + gi);
                if (S) {
                    const uint2 b = dvgo::bf16x4_bits(make_float4(pq[q].x, pq[q].y, pq[q].z, pq[q].w));
                    u2 bv;
                    bv.x = b.x;
                    bv.y = b.y;
                    __builtin_nontemporal_store(bv, S + gi);
                }
            }
        }
        if (o.active) {
            bool nonzero = false;
            #pragma unroll
            for (int q = 0; q < 13; ++q) nonzero |= acc[q] != 0.0f;
            const uint64_t now = __ballot(was_active || (touched && nonzero));
            if (lane == 0 && nwave > 0) o.active[vbase >> 5] = static_cast<uint32_t>(now);
            if (lane == 1 && nwave > 32) o.active[(vbase >> 5) + 1] = static_cast<uint32_t>(now >> 32);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void vertex_adam_kernel(BinArgs a, GridAdamArgs o) {
    vertex_adam_body(a, o, blockIdx.x, gridDim.x);
}

// Activity mask from given moments: bit v set iff any of vertex v's 26
// moments (density and 12 features, m and v) is non-zero.  Each wave covers
// 64 consecutive vertices, two whole words.
__global__ __launch_bounds__(256) void grid_active_kernel(const float* __restrict__ md, const float* __restrict__ vd,
                                                          const float* __restrict__ mf, const float* __restrict__ vf,
                                                          int64_t nv, uint32_t* __restrict__ active) {
    const int lane = threadIdx.x & 63;
    for (int64_t v0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + (threadIdx.x & ~63); v0 < nv;
         v0 += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t v = v0 + lane;
        bool nz = false;
        if (v < nv) {
            nz = md[v] != 0.0f || vd[v] != 0.0f;
            const float4* a = reinterpret_cast<const float4*>(mf + v * kC);
            const float4* b = reinterpret_cast<const float4*>(vf + v * kC);
            #pragma unroll
            for (int q = 0; q < 3; ++q) {
                const float4 x = a[q], y = b[q];
                nz |= x.x != 0.0f || x.y != 0.0f || x.z != 0.0f || x.w != 0.0f;
                nz |= y.x != 0.0f || y.y != 0.0f || y.z != 0.0f || y.w != 0.0f;
            }
        }
        const uint64_t bits = __ballot(nz);
        if (lane == 0) active[v0 >> 5] = static_cast<uint32_t>(bits);
        if (lane == 1 && v0 + 32 < nv) active[(v0 >> 5) + 1] = static_cast<uint32_t>(bits >> 32);
    }
}

// Device-wide exclusive scan of int32 counts in three passes.
__device__ __forceinline__ int block_excl_scan_1024(int v, int* sh, int* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) sh[wave] = incl;
    __syncthreads();
    int woff = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) woff += sh[w];
        tot += sh[w];
    }
    __syncthreads();
    *total = tot;
    return woff + incl - v;
}

// Eight consecutive counts of one thread (zero past n); 32-byte aligned.
__device__ __forceinline__ void load8(const int* __restrict__ in, int64_t base, int64_t n, int v[8]) {
    if (base + 8 <= n) {
        const int4 a = *reinterpret_cast<const int4*>(in + base);
        const int4 b = *reinterpret_cast<const int4*>(in + base + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
        for (int u = 0; u < 8; ++u) v[u] = base + u < n ? in[base + u] : 0;
    }
}

__global__ __launch_bounds__(1024) void scan_block_sums_kernel(const int* __restrict__ in, int64_t n,
                                                               long long* __restrict__ bsum) {
    __shared__ int sh[16];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanPer + threadIdx.x * 8;
    int v8[8];
    load8(in, base, n, v8);
    int v = 0;
    for (int u = 0; u < 8; ++u) v += v8[u];
    int tot;
    block_excl_scan_1024(v, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of the counts: each workgroup adds the totals of all the
// workgroups before it (read from bsum, summed in the workgroup) to its own
// in-workgroup scan.
__global__ __launch_bounds__(1024) void scan_apply_kernel(const int* __restrict__ in, int64_t n,
                                                          const long long* __restrict__ bsum, int* __restrict__ out) {
    __shared__ int sh[16];
    __shared__ long long sp[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    long long pre = 0;
    for (int b = threadIdx.x; b < static_cast<int>(blockIdx.x); b += 1024) pre += bsum[b];
    for (int off = 32; off > 0; off >>= 1) pre += __shfl_xor(pre, off, 64);
    if (lane == 0) sp[wave] = pre;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanPer + threadIdx.x * 8;
    int v[8];
    load8(in, base, n, v);
    int loc = 0;
    for (int u = 0; u < 8; ++u) loc += v[u];
    int tot;
    const int ex = block_excl_scan_1024(loc, sh, &tot);   // its barriers also publish sp
    long long blk = 0;
    for (int w = 0; w < 16; ++w) blk += sp[w];
    int run = static_cast<int>(blk) + ex;
    int o[8];
    for (int u = 0; u < 8; ++u) {
        o[u] = run;
        run += v[u];
    }
    if (base + 8 <= n) {
        *reinterpret_cast<int4*>(out + base) = make_int4(o[0], o[1], o[2], o[3]);
        *reinterpret_cast<int4*>(out + base + 4) = make_int4(o[4], o[5], o[6], o[7]);
    } else {
        for (int u = 0; u < 8; ++u)
            if (base + u < n) out[base + u] = o[u];
    }
}

// Deterministic sum of the per-block weight-gradient partials (+= into out):
// 64 parameters per workgroup, 16 wavefronts each summing every 16th
// partial row (all its loads issued before the sum, which keeps the row
// order), then a fixed-order sum of the 16 (deterministic).  With
// sq_err, workgroup 0 also forms the photometric loss (1/B) sum of the
// rays' squared errors, in a fixed order.
// With net.param, the summed gradient also takes the network's Adam step
// (the update dvgo_adam_step makes, on the same float32 gradient) and out
// is left zero.
struct NetAdam {
    float* param;
    float* m;
    float* v;
    dvgo::AdamCoef c;
};

struct ReduceArgs {
    const float* partial;   // [nblk][pstride]
    int nblk, nparams, pstride;
    float* out;             // the flat gradient (accumulated), or zeroed after the Adam step
    const float* sq_err;    // per-ray squared errors (NULL: no loss)
    int B;
    float* loss;
    NetAdam net;
};

// Workgroup blk (256 threads) sums the partials of parameters blk*64 ..
// blk*64 + 63 in a fixed order: wavefront w takes rows w, w + 4, ...
// (sixteen loads in flight at a time), then wavefront 0 adds the four sums
// in order; with net.param it then takes the Adam step.  Workgroup 0 also
// sums the squared errors into the loss.
__device__ __forceinline__ void reduce_body(const ReduceArgs& R, int blk) {
    __shared__ float sh[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = blk * 64 + lane;
    const int nblk = R.nblk, nparams = R.nparams, pstride = R.pstride, B = R.B;
    const float* __restrict__ partial = R.partial;
    float* __restrict__ out = R.out;
    const float* __restrict__ sq_err = R.sq_err;
    const NetAdam& net = R.net;
    static_assert(kMaxBwdBlocks <= 4 * 64, "a wavefront sums at most 64 partial rows");
    float s = 0.0f;
    if (p < nparams) {
        #pragma unroll
        for (int u0 = 0; u0 < 64; u0 += 16) {
            float v[16];
            #pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int b = wave + 4 * (u0 + u);
                v[u] = b < nblk ? partial[static_cast<int64_t>(b) * pstride + p] : 0.0f;
            }
            #pragma unroll
            for (int u = 0; u < 16; ++u) s += v[u];
        }
    }
    sh[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && p < nparams) {
        float t = 0.0f;
        for (int w = 0; w < 4; ++w) t += sh[w][lane];
        const float g = out[p] + t;
        if (net.param) {
            float pp = net.param[p], mm = net.m[p], vv = net.v[p];
            dvgo::adam_update(net.c, pp, g, mm, vv);
            net.param[p] = pp;
            net.m[p] = mm;
            net.v[p] = vv;
            out[p] = 0.0f;
        } else {
            out[p] = g;
        }
    }
    if (blk == 0 && sq_err) {
        __syncthreads();
        float e = 0.0f;
        for (int i0 = threadIdx.x; i0 < B; i0 += 256 * 8) {   // eight loads in flight, summed in order
            float v[8];
            #pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = i0 + 256 * u < B ? sq_err[i0 + 256 * u] : 0.0f;
            #pragma unroll
            for (int u = 0; u < 8; ++u) e += v[u];
        }
        for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
        if (lane == 0) sh[0][wave] = e;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.0f;
            for (int w = 0; w < 4; ++w) t += sh[0][w];
            if (R.loss) *R.loss = t * (1.0f / static_cast<float>(B));
        }
    }
}

__global__ __launch_bounds__(256) void reduce_partials_kernel(ReduceArgs R) { reduce_body(R, blockIdx.x); }

// The fused grid Adam and the reduction of the network's gradient partials
// in one launch (independent of each other): the first vblocks workgroups
// step the grids, the rest reduce, filling the grid step's tail.
__global__ __launch_bounds__(256) void vertex_adam_reduce_kernel(BinArgs a, GridAdamArgs o, int vblocks,
                                                                 ReduceArgs R) {
    const int blk = static_cast<int>(blockIdx.x);
    if (blk < vblocks) vertex_adam_body(a, o, blk, vblocks);
    else reduce_body(R, blk - vblocks);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Common {
    SampleArgs sa;
    GridArgs g;
    WsLayout L;
    char* ws;
    int64_t cap;
    int B;
    float box_min[3], box_max[3];
};

int32_t validate(const dvgo_field* field, const dvgo_mlp* mlp, const float* rays_o, const float* rays_d,
                 const float* t_near, const int32_t* n_uniform, const int32_t* perm, const int32_t* ray_offset,
                 const int32_t* sample_ray, const int32_t* sample_k, const int64_t* n_kept, int64_t capacity,
                 int32_t B, float step, const float* bg, void* workspace, size_t workspace_bytes,
                 bool forward_only = false) {
    if (!field || !bg || B < 0 || capacity < 0 || !(step > 0.0f)) return DVGO_E_ARG;
    if (!dvgo::box_ok(&field->box, 2) || !field->density) return DVGO_E_ARG;
    // vertex and cell indices, cell starts and record positions are int32
    if (static_cast<int64_t>(field->box.n[0]) * field->box.n[1] * field->box.n[2] >= (1LL << 31))
        return DVGO_E_UNSUPPORTED;
    if (mlp) {
        if (field->channels != kC) return DVGO_E_SHAPE;
        if (!field->feat) return DVGO_E_ARG;
        if (field->feat_dtype != DVGO_F32 && field->feat_dtype != DVGO_BF16) return DVGO_E_DTYPE;
        if (mlp->hidden != kH) return DVGO_E_SHAPE;
        if (mlp->precision != DVGO_F32 && mlp->precision != DVGO_BF16) return DVGO_E_DTYPE;
        if (mlp->pe_x != 0 && mlp->pe_x != kMaxKX) return DVGO_E_UNSUPPORTED;
        if (!mlp->w1 || !mlp->b1 || !mlp->w2 || !mlp->b2 || !mlp->w3 || !mlp->b3) return DVGO_E_ARG;
    }
    if (B > 0 && (!rays_o || !rays_d || !t_near || !n_uniform || !perm || !ray_offset)) return DVGO_E_ARG;
    if (!n_kept) return DVGO_E_ARG;
    if (capacity > 0 && (!sample_ray || !sample_k)) return DVGO_E_ARG;
    const size_t need = forward_only ? dvgo_render_fwd_workspace_bytes(B, capacity, kC, &field->box)
                                     : dvgo_render_workspace_bytes(B, capacity, kC, &field->box);
    if (workspace_bytes < need || (!workspace && workspace_bytes)) return DVGO_E_CAPACITY;
    return DVGO_OK;
}

int grid_for(int64_t work, int per_block, int max_blocks) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return static_cast<int>(b);
}

// Host-side checks of a dvgo_grid_adam and its kernel arguments.
int32_t grid_adam_args(const dvgo_grid_adam* opt, GridAdamArgs* o) {
    if (!opt->density || !opt->density_m || !opt->density_v || !opt->feat || !opt->feat_m || !opt->feat_v)
        return DVGO_E_ARG;
    if (!dvgo::adam_hyper_ok(opt->beta1, opt->beta2, opt->eps, opt->t)) return DVGO_E_ARG;
    auto al16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    if (!al16(opt->feat) || !al16(opt->feat_m) || !al16(opt->feat_v) ||
        (opt->feat_shadow_bf16 && (reinterpret_cast<uintptr_t>(opt->feat_shadow_bf16) & 7u) != 0) ||
        (opt->active && (reinterpret_cast<uintptr_t>(opt->active) & 3u) != 0))
        return DVGO_E_ARG;
    o->pd = opt->density;
    o->md = opt->density_m;
    o->vd = opt->density_v;
    o->pf = opt->feat;
    o->mf = opt->feat_m;
    o->vf = opt->feat_v;
    o->shadow = opt->feat_shadow_bf16;
    o->active = opt->active;
    o->c = dvgo::adam_coef(opt->lr, opt->beta1, opt->beta2, opt->eps, opt->t);
    return DVGO_OK;
}

// Workgroups of the fused grid Adam: a multiple of 8 (one share per XCD),
// 4 per compute unit (its register use allows 4 wavefronts per SIMD; more
// resident workgroups measured slower), no more than the vertices need.
int grid_adam_blocks(int64_t nv) {
    const int64_t per_xcd = (nv + 8 * 256 - 1) / (8 * 256);
    int64_t b = static_cast<int64_t>(dvgo::device_cu_count()) * 4 / 8;
    if (b > per_xcd) b = per_xcd;
    if (b < 1) b = 1;
    return static_cast<int>(8 * b);
}

// The preparation's arguments (mlp != NULL).
PrepArgs prep_args(const Common& cm, const dvgo_mlp* mlp, int* zero, int64_t nzero) {
    PrepArgs P;
    P.base = reinterpret_cast<float*>(cm.ws + cm.L.base);
    P.pe = reinterpret_cast<float*>(cm.ws + cm.L.pe);
    {
        PackArgs pk;
        pk.w1 = mlp->w1;
        pk.w2 = mlp->w2;
        pk.w1p = reinterpret_cast<float*>(cm.ws + cm.L.w1p);
        pk.w2p = reinterpret_cast<float*>(cm.ws + cm.L.w2p);
        pk.w2tp = reinterpret_cast<float*>(cm.ws + cm.L.w2tp);
        pk.w1pb = reinterpret_cast<uint16_t*>(cm.ws + cm.L.w1pb);
        pk.w2pb = reinterpret_cast<uint16_t*>(cm.ws + cm.L.w2pb);
        pk.w2tpb = reinterpret_cast<uint16_t*>(cm.ws + cm.L.w2tpb);
        pk.w3 = mlp->w3;
        pk.w3pb = reinterpret_cast<uint16_t*>(cm.ws + cm.L.w3pb);
        pk.w3tpb = reinterpret_cast<uint16_t*>(cm.ws + cm.L.w3tpb);
        pk.w1tpb = reinterpret_cast<uint16_t*>(cm.ws + cm.L.w1tpb);
        pk.bf16 = mlp->precision == DVGO_BF16;
        const bool xpe = mlp->pe_x == kMaxKX;
        pk.w1_in = xpe ? NetLayout<kMaxKX>::kIn : kIn;
        pk.w1_ns = xpe ? NetLayout<kMaxKX>::kS : kC;
        pk.w1_q = xpe ? NetLayout<kMaxKX>::kQ1 : NetLayout<0>::kQ1;
        pk.w1_s1 = xpe ? NetLayout<kMaxKX>::kS1 : NetLayout<0>::kS1;
        const int zblocks = zero ? grid_for(nzero, 256, dvgo::device_cu_count() * 4) : 0;
        P.pk = pk;
        P.rays_d = cm.sa.rays_d;
        P.B = cm.B;
        P.w1 = mlp->w1;
        P.b1 = mlp->b1;
        P.w1_in = pk.w1_in;
        P.view_col = pk.w1_ns;
        P.zero = zero;
        P.nzero = nzero;
        P.zblocks = zblocks;
        P.blocks = kPackThreads / 256 + (cm.B + kPrepRays - 1) / kPrepRays + zblocks;
    }
    return P;
}

int32_t run_prep(const Common& cm, const dvgo_mlp* mlp, hipStream_t s, int* zero = nullptr, int64_t nzero = 0) {
    if (mlp) {
        const PrepArgs P = prep_args(cm, mlp, zero, nzero);
        DVGO_LAUNCH(K_RAY_BASE, prep_kernel, dim3(P.blocks), dim3(256), 0, s, P);
        if (int32_t st = dvgo::launch_status()) return st;
    } else if (zero) {
        DVGO_LAUNCH(K_CELL_SCAN, fill_int_kernel, dim3(grid_for(nzero, 256, dvgo::device_cu_count() * 8)), dim3(256),
                    0, s, zero, nzero, 0);
        if (int32_t st = dvgo::launch_status()) return st;
    }
    return DVGO_OK;
}

GatherArgs gather_args(const Common& cm, const dvgo_field* field, bool with_feat, const int64_t* n_kept) {
    GatherArgs ga;
    ga.sa = cm.sa;
    ga.g = cm.g;
    ga.density = field->density;
    ga.feat = field->feat;
    ga.feat_bf16 = field->feat_dtype == DVGO_BF16;
    ga.with_feat = with_feat;
    ga.n_kept = n_kept;
    ga.cap = cm.cap;
    ga.raw_out = reinterpret_cast<float*>(cm.ws + cm.L.raw);
    ga.feat_out = reinterpret_cast<float*>(cm.ws + cm.L.feat);
    return ga;
}

int gather_blocks(const Common& cm) { return grid_for(cm.cap, 256, dvgo::device_cu_count() * 16); }

int32_t run_gather(const Common& cm, const dvgo_field* field, bool with_feat, const int64_t* n_kept,
                   hipStream_t s) {
    if (cm.cap == 0) return DVGO_OK;
    const GatherArgs ga = gather_args(cm, field, with_feat, n_kept);
    const int blocks = gather_blocks(cm);
    if (!with_feat) DVGO_LAUNCH(K_GATHER, gather_kernel<0>, dim3(blocks), dim3(256), 0, s, ga);
    else if (!ga.feat_bf16) DVGO_LAUNCH(K_GATHER, gather_kernel<1>, dim3(blocks), dim3(256), 0, s, ga);
    else DVGO_LAUNCH(K_GATHER, gather_kernel<2>, dim3(blocks), dim3(256), 0, s, ga);
    return dvgo::launch_status();
}

// The preparation and the gather of a render with a network, in one launch
// (the gather's workgroups first); without a network or samples, each alone.
int32_t run_prep_gather(const Common& cm, const dvgo_mlp* mlp, const dvgo_field* field, const int64_t* n_kept,
                        hipStream_t s, int* zero = nullptr, int64_t nzero = 0) {
    if (!mlp || cm.cap == 0) {
        if (int32_t st = run_prep(cm, mlp, s, zero, nzero)) return st;
        return run_gather(cm, field, mlp != nullptr, n_kept, s);
    }
    const PrepArgs P = prep_args(cm, mlp, zero, nzero);
    const GatherArgs ga = gather_args(cm, field, true, n_kept);
    const int gb = gather_blocks(cm);
    const dim3 grid(static_cast<unsigned>(gb + P.blocks));
    if (ga.feat_bf16) DVGO_LAUNCH(K_GATHER, prep_gather_kernel<2>, grid, dim3(256), 0, s, P, ga, gb);
    else DVGO_LAUNCH(K_GATHER, prep_gather_kernel<1>, grid, dim3(256), 0, s, P, ga, gb);
    return dvgo::launch_status();
}

MlpArgs make_mlp_args(const Common& cm, const dvgo_mlp* mlp, const int64_t* n_kept) {
    MlpArgs ma;
    ma.nrays = cm.B;
    ma.sample_ray = cm.sa.sample_ray;
    ma.n_kept = n_kept;
    ma.cap = cm.cap;
    ma.w1 = mlp->w1;
    ma.b2 = mlp->b2;
    ma.w3 = mlp->w3;
    ma.b3 = mlp->b3;
    ma.base = reinterpret_cast<const float*>(cm.ws + cm.L.base);
    ma.pe = reinterpret_cast<const float*>(cm.ws + cm.L.pe);
    ma.w1p = reinterpret_cast<const float*>(cm.ws + cm.L.w1p);
    ma.w2p = reinterpret_cast<const float*>(cm.ws + cm.L.w2p);
    ma.w2tp = reinterpret_cast<const float*>(cm.ws + cm.L.w2tp);
    ma.w1pb = reinterpret_cast<const uint16_t*>(cm.ws + cm.L.w1pb);
    ma.w2pb = reinterpret_cast<const uint16_t*>(cm.ws + cm.L.w2pb);
    ma.w2tpb = reinterpret_cast<const uint16_t*>(cm.ws + cm.L.w2tpb);
    ma.w3pb = reinterpret_cast<const uint16_t*>(cm.ws + cm.L.w3pb);
    ma.w3tpb = reinterpret_cast<const uint16_t*>(cm.ws + cm.L.w3tpb);
    ma.w1tpb = reinterpret_cast<const uint16_t*>(cm.ws + cm.L.w1tpb);
    ma.feat = reinterpret_cast<float*>(cm.ws + cm.L.feat);
    ma.col = reinterpret_cast<float*>(cm.ws + cm.L.col);
    ma.partial = reinterpret_cast<float*>(cm.ws + cm.L.partial);
    ma.bf16 = mlp->precision == DVGO_BF16;
    return ma;
}

PosArgs make_pos_args(const Common& cm) {
    PosArgs pa;
    pa.rays_o = cm.sa.rays_o;
    pa.rays_d = cm.sa.rays_d;
    pa.jitter = cm.sa.jitter;
    pa.t_near = cm.sa.t_near;
    pa.sample_k = cm.sa.sample_k;
    pa.step = cm.sa.step;
    for (int i = 0; i < 3; ++i) {
        // box coordinates: centre and inverse half-extent, rounded once to float32
        pa.pe_c[i] = 0.5f * (cm.box_min[i] + cm.box_max[i]);
        pa.pe_ih[i] = 2.0f / (cm.box_max[i] - cm.box_min[i]);
    }
    return pa;
}

ComposeArgs make_compose(const Common& cm, const int32_t* perm, const int32_t* ray_offset, const int32_t* n_uniform,
                         const int64_t* n_kept, float act_shift, const float* bg, bool with_color) {
    ComposeArgs ca;
    std::memset(&ca, 0, sizeof(ca));
    ca.sa = cm.sa;
    ca.perm = perm;
    ca.ray_offset = ray_offset;
    ca.n_uniform = n_uniform;
    ca.n_kept = n_kept;
    ca.cap = cm.cap;
    ca.B = cm.B;
    ca.act_shift = act_shift;
    for (int i = 0; i < 3; ++i) ca.bg[i] = bg[i];
    ca.raw = reinterpret_cast<float*>(cm.ws + cm.L.raw);
    ca.col = reinterpret_cast<float*>(cm.ws + cm.L.col);
    ca.with_color = with_color;
    return ca;
}

int64_t cell_count_of(const dvgo_box& b) {
    return static_cast<int64_t>(b.n[0] - 1) * (b.n[1] - 1) * (b.n[2] - 1);
}

Common make_common(const dvgo_field* field, const float* rays_o, const float* rays_d, const float* jitter,
                   const float* t_near, const int32_t* sample_ray, const int32_t* sample_k, int64_t capacity,
                   int32_t B, float step, void* workspace) {
    Common cm;
    cm.sa.rays_o = rays_o;
    cm.sa.rays_d = rays_d;
    cm.sa.jitter = jitter;
    cm.sa.t_near = t_near;
    cm.sa.sample_ray = sample_ray;
    cm.sa.sample_k = sample_k;
    cm.sa.step = step;
    cm.g = dvgo::make_grid(field->box);
    for (int i = 0; i < 3; ++i) {
        cm.box_min[i] = field->box.xyz_min[i];
        cm.box_max[i] = field->box.xyz_max[i];
    }
    cm.L = ws_layout(B, capacity, cell_count_of(field->box));
    cm.ws = static_cast<char*>(workspace);
    cm.cap = capacity;
    cm.B = B;
    return cm;
}

// Binning state of a backward call inside the workspace.
struct Bins {
    int64_t ncell;
    int* cell_count;
    int* cell_start;
    int2* cell_rank;
    float4* rec_head;
    float4* rec;
};

Bins bins_of(const Common& cm, const dvgo_field* field) {
    Bins b;
    b.ncell = cell_count_of(field->box);
    b.cell_count = reinterpret_cast<int*>(cm.ws + cm.L.cell_count);
    b.cell_start = reinterpret_cast<int*>(cm.ws + cm.L.cell_start);
    b.cell_rank = reinterpret_cast<int2*>(cm.ws + cm.L.cell_rank);
    b.rec_head = reinterpret_cast<float4*>(cm.ws + cm.L.rec_head);
    b.rec = reinterpret_cast<float4*>(cm.ws + cm.L.rec);
    return b;
}

// Exclusive scan of the per-cell counts into cell starts.
int32_t run_cell_scan(const Common& cm, const Bins& b, hipStream_t s) {
    const int64_t nc1 = b.ncell + 1;
    const int nb = static_cast<int>((nc1 + kScanPer - 1) / kScanPer);
    long long* bsum = reinterpret_cast<long long*>(cm.ws + cm.L.scan_tmp);
    DVGO_LAUNCH(K_CELL_SCAN, scan_block_sums_kernel, dim3(nb), dim3(1024), 0, s, b.cell_count, nc1, bsum);
    DVGO_LAUNCH(K_CELL_SCAN, scan_apply_kernel, dim3(nb), dim3(1024), 0, s, b.cell_count, nc1, bsum, b.cell_start);
    return dvgo::launch_status();
}

// Records placed in binned order (by the network backward, or here when
// there is none), then one thread per vertex: gradient into the grids, or
// the grids' fused Adam step.
int32_t run_vertex(const Common& cm, const dvgo_field* field, const Bins& b, bool with_feat, bool place,
                   const int64_t* n_kept, float* grad_density, float* grad_feat, const GridAdamArgs* opt,
                   hipStream_t s, const ReduceArgs* red = nullptr) {
    BinArgs ba;
    ba.sa = cm.sa;
    ba.g = cm.g;
    ba.n_kept = n_kept;
    ba.cap = cm.cap;
    ba.ncell = b.ncell;
    ba.cell_count = b.cell_count;
    ba.cell_start = b.cell_start;
    ba.cell_rank = b.cell_rank;
    ba.rec_head = b.rec_head;
    ba.with_feat = with_feat;
    ba.rec = b.rec;
    ba.grad_density = grad_density;
    ba.grad_feat = grad_feat;
    const int cus = dvgo::device_cu_count();
    if (place) {
        DVGO_LAUNCH(K_BIN_PLACE, bin_place_kernel, dim3(grid_for(cm.cap, 256, cus * 16)), dim3(256), 0, s, ba);
        if (int32_t st = dvgo::launch_status()) return st;
    }
    const int64_t nv = static_cast<int64_t>(field->box.n[0]) * field->box.n[1] * field->box.n[2];
    if (opt && red) {
        const int vb = grid_adam_blocks(nv);
        DVGO_LAUNCH(K_GRID_ADAM, vertex_adam_reduce_kernel, dim3(vb + (red->nparams + 63) / 64), dim3(256), 0, s, ba,
                    *opt, vb, *red);
    } else if (opt)
        DVGO_LAUNCH(K_GRID_ADAM, vertex_adam_kernel, dim3(grid_adam_blocks(nv)), dim3(256), 0, s, ba, *opt);
    else
        DVGO_LAUNCH(K_SCATTER, vertex_gather_kernel, dim3(grid_for(nv, 256, cus * 16)), dim3(256), 0, s, ba);
    return dvgo::launch_status();
}

int32_t render_bwd_impl(const dvgo_field* field, const dvgo_mlp* mlp, const float* rays_o, const float* rays_d,
                        const float* jitter, const float* t_near, const int32_t* n_uniform, const int32_t* perm,
                        const int32_t* ray_offset, const int32_t* sample_ray, const int32_t* sample_k,
                        const int64_t* n_kept, int64_t capacity, int32_t B, float step, const float* bg,
                        const float* log_t_end, const float* grad_rgb, const float* grad_depth,
                        const float* grad_acc, float* grad_density, float* grad_feat, const GridAdamArgs* opt,
                        float* grad_mlp, void* workspace, size_t workspace_bytes, void* stream,
                        bool forward_done = false, const float* sq_err = nullptr, float* loss = nullptr,
                        const NetAdam* net = nullptr, const float* aux_target = nullptr, float w_pt = 0.0f,
                        float w_bg = 0.0f, const ComposeArgs* fwd_compose = nullptr) {
    if (int32_t st = validate(field, mlp, rays_o, rays_d, t_near, n_uniform, perm, ray_offset, sample_ray, sample_k,
                              n_kept, capacity, B, step, bg, workspace, workspace_bytes))
        return st;
    if (B > 0 && (!log_t_end || (!opt && !grad_density))) return DVGO_E_ARG;
    if (mlp && ((!opt && !grad_feat) || !grad_mlp)) return DVGO_E_ARG;
    if (opt && !mlp) return DVGO_E_ARG;
    if (!mlp && grad_rgb) return DVGO_E_ARG;
    hipStream_t s = dvgo::as_stream(stream);
    if (B == 0 || capacity == 0) {
        if (!opt) return DVGO_OK;
        // no samples: every vertex still takes its zero-gradient Adam step
        BinArgs ba{};
        ba.g = dvgo::make_grid(field->box);
        const int64_t nv = static_cast<int64_t>(field->box.n[0]) * field->box.n[1] * field->box.n[2];
        DVGO_LAUNCH(K_GRID_ADAM, vertex_adam_kernel, dim3(grid_adam_blocks(nv)), dim3(256),
                    0, s, ba, *opt);
        return dvgo::launch_status();
    }
    Common cm = make_common(field, rays_o, rays_d, jitter, t_near, sample_ray, sample_k, capacity, B, step,
                            workspace);
    const Bins bins = bins_of(cm, field);
    MlpArgs ma;
    if (mlp) ma = make_mlp_args(cm, mlp, n_kept);
    if (!forward_done) {
        // prep (packing, per-ray encoding) also clears the cell counts
        if (int32_t st = run_prep_gather(cm, mlp, field, n_kept, s, bins.cell_count, bins.ncell + 1)) return st;
        if (mlp) {
            launch_mlp_fwd(ma, make_pos_args(cm), mlp->pe_x, dvgo::device_cu_count(), s);
            if (int32_t st = dvgo::launch_status()) return st;
        }
    }
    // adjoint of the compositing; bins every sample by fine cell on the way
    ComposeArgs ca = make_compose(cm, perm, ray_offset, n_uniform, n_kept, field->act_shift, bg, mlp != nullptr);
    ca.log_t_end_in = log_t_end;
    ca.target = aux_target;
    ca.w_pt = w_pt;
    ca.w_bg = w_bg;
    ca.grad_rgb = grad_rgb;
    ca.grad_depth = grad_depth;
    ca.grad_acc = grad_acc;
    ca.g = cm.g;
    ca.cell_count = bins.cell_count;
    ca.cell_rank = bins.cell_rank;
    ca.rec_head = bins.rec_head;
    if (fwd_compose)   // the forward compositing not yet run: both in one launch
        DVGO_LAUNCH(K_COMPOSE_BWD, compose_step_kernel, compose_grid(B), dim3(kComposeThreads), 0, s, *fwd_compose, ca);
    else
        DVGO_LAUNCH(K_COMPOSE_BWD, compose_bwd_kernel, compose_grid(B), dim3(kComposeThreads), 0, s, ca);
    if (int32_t st = dvgo::launch_status()) return st;
    if (int32_t st = run_cell_scan(cm, bins, s)) return st;
    int nblk = 0;
    if (mlp) {   // the network adjoint writes each sample's record at its binned position
        ma.cell_rank = bins.cell_rank;
        ma.cell_start = bins.cell_start;
        ma.rec_head = bins.rec_head;
        ma.rec = bins.rec;
        nblk = dvgo::device_cu_count();
        if (nblk > kMaxBwdBlocks) nblk = kMaxBwdBlocks;
        launch_mlp_bwd(ma, make_pos_args(cm), mlp->pe_x, nblk, s);
        if (int32_t st = dvgo::launch_status()) return st;
    }
    ReduceArgs red{};
    if (mlp) {
        red.net = NetAdam{};
        if (net) red.net = *net;
        const bool xpe = mlp->pe_x == kMaxKX;
        red.partial = reinterpret_cast<const float*>(cm.ws + cm.L.partial);
        red.nblk = nblk;
        red.nparams = xpe ? NetLayout<kMaxKX>::kParams : kMlpParams;
        red.pstride = xpe ? NetLayout<kMaxKX>::kPStride : kPStride;
        red.out = grad_mlp;
        red.sq_err = sq_err;
        red.B = B;
        red.loss = loss;
    }
    // with the fused grid Adam, the network's reduction rides in its launch
    const bool merged = mlp && opt;
    if (int32_t st = run_vertex(cm, field, bins, mlp != nullptr, mlp == nullptr, n_kept, grad_density, grad_feat, opt,
                                s, merged ? &red : nullptr))
        return st;
    if (mlp && !merged) {
        DVGO_LAUNCH(K_REDUCE, reduce_partials_kernel, dim3((red.nparams + 63) / 64), dim3(256), 0, s, red);
        if (int32_t st = dvgo::launch_status()) return st;
    }
    return DVGO_OK;
}

}  // namespace

extern "C" {

int64_t dvgo_mlp_param_count(int32_t channels, int32_t hidden, int32_t pe_x) {
    if (channels < 0 || hidden < 0 || pe_x < 0) return 0;
    const int64_t in = channels + (pe_x ? 3 + 6 * pe_x : 0) + kPE;
    return hidden * in + hidden + static_cast<int64_t>(hidden) * hidden + hidden + 3LL * hidden + 3;
}

size_t dvgo_render_workspace_bytes(int32_t B, int64_t capacity, int32_t channels, const dvgo_box* grid) {
    if (B < 0 || capacity < 0 || channels != kC || !dvgo::box_ok(grid, 2)) return 0;
    return ws_layout(B, capacity, cell_count_of(*grid)).total;
}

// The forward uses the front of the layout only: per-ray encodings, packed
// network, per-sample density, features and colour.
size_t dvgo_render_fwd_workspace_bytes(int32_t B, int64_t capacity, int32_t channels, const dvgo_box* grid) {
    if (B < 0 || capacity < 0 || channels != kC || !dvgo::box_ok(grid, 2)) return 0;
    return ws_layout(B, capacity, cell_count_of(*grid)).partial;
}

int32_t dvgo_render_fwd(const dvgo_field* field, const dvgo_mlp* mlp, const float* rays_o, const float* rays_d,
                        const float* jitter, const float* t_near, const int32_t* n_uniform, const int32_t* perm,
                        const int32_t* ray_offset, const int32_t* sample_ray, const int32_t* sample_k,
                        const int64_t* n_kept, int64_t capacity, int32_t B, float step, const float* bg, float* rgb,
                        float* depth, float* acc, float* log_t_end, float* seg_w, float* sample_w, void* workspace,
                        size_t workspace_bytes, void* stream) {
    if (int32_t st = validate(field, mlp, rays_o, rays_d, t_near, n_uniform, perm, ray_offset, sample_ray, sample_k,
                              n_kept, capacity, B, step, bg, workspace, workspace_bytes, true))
        return st;
    if (!log_t_end && B > 0) return DVGO_E_ARG;
    if (!mlp && rgb) return DVGO_E_ARG;
    hipStream_t s = dvgo::as_stream(stream);
    if (B == 0) return DVGO_OK;
    Common cm = make_common(field, rays_o, rays_d, jitter, t_near, sample_ray, sample_k, capacity, B, step,
                            workspace);
    // with a network, the preparation and the gather first; without one
    // the compositing interpolates each sample's density itself
    if (mlp) {
        if (int32_t st = run_prep_gather(cm, mlp, field, n_kept, s)) return st;
    }
    if (mlp && capacity > 0) {
        MlpArgs ma = make_mlp_args(cm, mlp, n_kept);
        launch_mlp_fwd(ma, make_pos_args(cm), mlp->pe_x, dvgo::device_cu_count(), s);
        if (int32_t st = dvgo::launch_status()) return st;
    }
    ComposeArgs ca = make_compose(cm, perm, ray_offset, n_uniform, n_kept, field->act_shift, bg, mlp != nullptr);
    ca.rgb = rgb;
    ca.depth = depth;
    ca.acc = acc;
    ca.log_t_end = log_t_end;
    ca.seg_w = seg_w;
    ca.sample_w = sample_w;
    if (!mlp) {
        ca.density_in = field->density;
        ca.g = cm.g;
        DVGO_LAUNCH(K_COMPOSE_FWD, compose_fwd_kernel<true>, compose_grid(B), dim3(kComposeThreads), 0, s, ca);
    } else {
        DVGO_LAUNCH(K_COMPOSE_FWD, compose_fwd_kernel<false>, compose_grid(B), dim3(kComposeThreads), 0, s, ca);
    }
    return dvgo::launch_status();
}

int32_t dvgo_render_bwd(const dvgo_field* field, const dvgo_mlp* mlp, const float* rays_o, const float* rays_d,
                        const float* jitter, const float* t_near, const int32_t* n_uniform, const int32_t* perm,
                        const int32_t* ray_offset, const int32_t* sample_ray, const int32_t* sample_k,
                        const int64_t* n_kept, int64_t capacity, int32_t B, float step, const float* bg,
                        const float* log_t_end, const float* grad_rgb, const float* grad_depth,
                        const float* grad_acc, float* grad_density, float* grad_feat, float* grad_mlp,
                        void* workspace, size_t workspace_bytes, void* stream) {
    return render_bwd_impl(field, mlp, rays_o, rays_d, jitter, t_near, n_uniform, perm, ray_offset, sample_ray,
                           sample_k, n_kept, capacity, B, step, bg, log_t_end, grad_rgb, grad_depth, grad_acc,
                           grad_density, grad_feat, nullptr, grad_mlp, workspace, workspace_bytes, stream);
}

int32_t dvgo_grid_active_init(const float* density_m, const float* density_v, const float* feat_m,
                              const float* feat_v, int64_t n_vertices, uint32_t* active, void* stream) {
    if (n_vertices < 0) return DVGO_E_ARG;
    if (n_vertices == 0) return DVGO_OK;
    if (!density_m || !density_v || !feat_m || !feat_v || !active) return DVGO_E_ARG;
    if ((reinterpret_cast<uintptr_t>(feat_m) & 15u) || (reinterpret_cast<uintptr_t>(feat_v) & 15u) ||
        (reinterpret_cast<uintptr_t>(active) & 3u))
        return DVGO_E_ARG;
    const int64_t want = (n_vertices + 255) / 256;
    const int64_t cap = static_cast<int64_t>(dvgo::device_cu_count()) * 8;
    const int blocks = static_cast<int>(want < cap ? want : cap);
    DVGO_LAUNCH(K_GRID_ACTIVE, grid_active_kernel, dim3(blocks), dim3(256), 0, dvgo::as_stream(stream), density_m,
                density_v, feat_m, feat_v, n_vertices, active);
    return dvgo::launch_status();
}

int32_t dvgo_render_bwd_adam(const dvgo_field* field, const dvgo_mlp* mlp, const float* rays_o,
                             const float* rays_d, const float* jitter, const float* t_near, const int32_t* n_uniform,
                             const int32_t* perm, const int32_t* ray_offset, const int32_t* sample_ray,
                             const int32_t* sample_k, const int64_t* n_kept, int64_t capacity, int32_t B, float step,
                             const float* bg, const float* log_t_end, const float* grad_rgb, const float* grad_depth,
                             const float* grad_acc, const dvgo_grid_adam* opt, float* grad_mlp, void* workspace,
                             size_t workspace_bytes, void* stream) {
    if (!opt || !field) return DVGO_E_ARG;
    GridAdamArgs o;
    if (int32_t st = grid_adam_args(opt, &o)) return st;
    return render_bwd_impl(field, mlp, rays_o, rays_d, jitter, t_near, n_uniform, perm, ray_offset, sample_ray,
                           sample_k, n_kept, capacity, B, step, bg, log_t_end, grad_rgb, grad_depth, grad_acc, nullptr,
                           nullptr, &o, grad_mlp, workspace, workspace_bytes, stream);
}

int32_t dvgo_train_step(const dvgo_field* field, const dvgo_mlp* mlp, const float* rays_o, const float* rays_d,
                        const float* jitter, const float* t_near, const int32_t* n_uniform, const int32_t* perm,
                        const int32_t* ray_offset, const int32_t* sample_ray, const int32_t* sample_k,
                        const int64_t* n_kept, int64_t capacity, int32_t B, float step, const float* bg,
                        const float* target, float* rgb, float* loss, const dvgo_grid_adam* opt, float* grad_mlp,
                        const dvgo_adam_state* mlp_opt, const dvgo_aux_loss* aux, void* workspace,
                        size_t workspace_bytes, void* stream) {
    if (int32_t st = validate(field, mlp, rays_o, rays_d, t_near, n_uniform, perm, ray_offset, sample_ray, sample_k,
                              n_kept, capacity, B, step, bg, workspace, workspace_bytes))
        return st;
    if (!mlp || !opt || !grad_mlp || (B > 0 && !target)) return DVGO_E_ARG;
    const float w_pt = aux ? aux->w_pt_rgb : 0.0f, w_bg = aux ? aux->w_bg_entropy : 0.0f;
    if (!(w_pt >= 0.0f) || !(w_bg >= 0.0f)) return DVGO_E_ARG;
    NetAdam net{};
    if (mlp_opt) {
        if (!mlp_opt->param || !mlp_opt->m || !mlp_opt->v ||
            !dvgo::adam_hyper_ok(mlp_opt->beta1, mlp_opt->beta2, mlp_opt->eps, mlp_opt->t))
            return DVGO_E_ARG;
        net.param = mlp_opt->param;
        net.m = mlp_opt->m;
        net.v = mlp_opt->v;
        net.c = dvgo::adam_coef(mlp_opt->lr, mlp_opt->beta1, mlp_opt->beta2, mlp_opt->eps, mlp_opt->t);
    }
    char* ws = static_cast<char*>(workspace);
    const WsLayout L = ws_layout(B, capacity, cell_count_of(field->box));
    float* rgb_w = rgb ? rgb : reinterpret_cast<float*>(ws + L.step_rgb);
    float* grad_w = reinterpret_cast<float*>(ws + L.step_grad);
    float* logt_w = reinterpret_cast<float*>(ws + L.step_logt);
    if (B == 0 || capacity == 0) {   // nothing shared to reuse: the separate calls
        if (int32_t st = dvgo_render_fwd(field, mlp, rays_o, rays_d, jitter, t_near, n_uniform, perm, ray_offset,
                                         sample_ray, sample_k, n_kept, capacity, B, step, bg, rgb_w, nullptr,
                                         nullptr, logt_w, nullptr, nullptr, workspace, workspace_bytes, stream))
            return st;
        if (int32_t st = dvgo_photo_loss(rgb_w, target, B, grad_w, loss, stream)) return st;
        if (int32_t st = dvgo_render_bwd_adam(field, mlp, rays_o, rays_d, jitter, t_near, n_uniform, perm,
                                              ray_offset, sample_ray, sample_k, n_kept, capacity, B, step, bg, logt_w,
                                              grad_w, nullptr, nullptr, opt, grad_mlp, workspace, workspace_bytes,
                                              stream))
            return st;
        if (!mlp_opt) return DVGO_OK;
        return dvgo_adam_step(mlp_opt->param, grad_mlp, mlp_opt->m, mlp_opt->v, nullptr,
                              dvgo_mlp_param_count(field->channels, mlp->hidden, mlp->pe_x), mlp_opt->lr, mlp_opt->beta1,
                              mlp_opt->beta2, mlp_opt->eps, mlp_opt->t, stream);
    }
    GridAdamArgs o;
    if (int32_t st = grid_adam_args(opt, &o)) return st;
    hipStream_t s = dvgo::as_stream(stream);
    // forward: prep (also clears the cell counts), gather, network, compositing
    Common cm = make_common(field, rays_o, rays_d, jitter, t_near, sample_ray, sample_k, capacity, B, step,
                            workspace);
    const Bins bins = bins_of(cm, field);
    if (int32_t st = run_prep_gather(cm, mlp, field, n_kept, s, bins.cell_count, bins.ncell + 1)) return st;
    MlpArgs ma = make_mlp_args(cm, mlp, n_kept);
    launch_mlp_fwd(ma, make_pos_args(cm), mlp->pe_x, dvgo::device_cu_count(), s);
    if (int32_t st = dvgo::launch_status()) return st;
    float* sq_w = reinterpret_cast<float*>(ws + L.step_sqerr);
    ComposeArgs ca = make_compose(cm, perm, ray_offset, n_uniform, n_kept, field->act_shift, bg, true);
    ca.rgb = rgb_w;
    ca.log_t_end = logt_w;
    ca.target = target;          // the loss gradient comes out of the compositing
    ca.grad_rgb_out = grad_w;
    ca.sq_err = sq_w;
    ca.w_pt = w_pt;
    ca.w_bg = w_bg;
    // adjoint and Adam, reusing the forward's gathered features, colours and
    // prep; the compositing (ca) runs in the adjoint's first launch
    return render_bwd_impl(field, mlp, rays_o, rays_d, jitter, t_near, n_uniform, perm, ray_offset, sample_ray,
                           sample_k, n_kept, capacity, B, step, bg, logt_w, grad_w, nullptr, nullptr, nullptr,
                           nullptr, &o, grad_mlp, workspace, workspace_bytes, stream, true, sq_w, loss,
                           mlp_opt ? &net : nullptr, target, w_pt, w_bg, &ca);
}

}  // extern "C"
