// Colour network of the fine stage (paper Eq. fine_queries: two ReLU layers
// of 128 and a sigmoid RGB head) on CDNA4 matrix cores.
//
// Layout.  A 32x32 accumulator tile of v_mfma_f32_32x32x{2f32,16bf16} holds,
// in lane l and register r, row 8*(r/4) + 4*(l/32) + (r%4) and column l%32.
// Activations are kept transposed ("feature rows, sample columns"): a wave
// owns 32 samples (one per lane column) and each lane holds 16 features per
// 32-feature tile.  The next layer consumes those registers directly as its
// B operand; the K order this implies is folded into the packed weights
// (phi() below), so a layer chain never leaves registers.  Weight gradients
// need the sample index as the contraction dimension, so the activations of
// a workgroup's 128 samples are staged through LDS once per block and each
// wave accumulates its own slice of dW in registers across the whole
// persistent loop; per-workgroup partials are summed afterwards.
#pragma once

#include "common.hpp"

namespace {

constexpr int kH = 128;                 // hidden width
constexpr int kC = 12;                  // feature channels
constexpr int kPE = 27;                 // PE(d) with 4 frequencies
constexpr int kIn = kC + kPE;           // first-layer input width
// Flat gradient layout of the colour network: w1, b1, w2, b2, w3, b3.
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kIn;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + 3 * kH;
constexpr int kMlpParams = kOffB3 + 3;
constexpr int kPStride = (kMlpParams + 63) / 64 * 64;
constexpr int kW1PackF32 = 4 * 2 * 64 * 4;
constexpr int kW2PackF32 = 4 * 16 * 64 * 4;
constexpr int kW1PackBF16 = 4 * 64 * 8;
constexpr int kW2PackBF16 = 4 * 8 * 64 * 8;
constexpr int kW3PackBF16 = 8 * 64 * 8;    // layer 3 as a 32-row tile (rows >= 3 zero)
constexpr int kW3TPackBF16 = 4 * 64 * 8;   // W3^T, one K step (k >= 3 zero)
constexpr int kW1TPackBF16 = 8 * 64 * 8;   // W1[:, :12]^T as a 32-row tile (rows >= 12 zero)

// Layout of the network whose input also carries the encoded query
// position (Eq. fine_queries with k_x = KX frequencies): input [feat (12),
// PE_KX(u) (3 + 6 KX), PE(d) (27)], u the position in box coordinates.  The
// per-sample part of the first layer is [feat, PE_KX(u)] (kS values); the
// view part is evaluated once per ray as before.  KX = 0 is the 39-input
// network above.  Float32 matrix cores only.
template <int KX>
struct NetLayout {
    static constexpr int kXPE = KX ? 3 + 6 * KX : 0;
    static constexpr int kS = kC + kXPE;              // per-sample first-layer inputs
    static constexpr int kIn = kS + kPE;              // first-layer inputs
    static constexpr int kOffW1 = 0;
    static constexpr int kOffB1 = kOffW1 + kH * kIn;
    static constexpr int kOffW2 = kOffB1 + kH;
    static constexpr int kOffB2 = kOffW2 + kH * kH;
    static constexpr int kOffW3 = kOffB2 + kH;
    static constexpr int kOffB3 = kOffW3 + 3 * kH;
    static constexpr int kParams = kOffB3 + 3;
    static constexpr int kPStride = (kParams + 63) / 64 * 64;
    static constexpr int kQ1 = ((kS + 1) / 2 + 3) / 4;   // float4 groups of K = 2 layer-1 steps
    static constexpr int kS1 = (kS + 15) / 16;            // K = 16 layer-1 steps (bfloat16)
    static constexpr int kXT = (kIn + 1 + 31) / 32;      // 32-column tiles of x' = [input, 1]
};
static_assert(NetLayout<0>::kIn == kIn && NetLayout<0>::kParams == kMlpParams && NetLayout<0>::kQ1 == 2 &&
                  NetLayout<0>::kXT == 2,
              "the 39-input layout");
constexpr int kMaxKX = 5;                                          // the paper's k_x
constexpr int kW1PackF32Max = 4 * NetLayout<kMaxKX>::kQ1 * 64 * 4;   // packed W1 of either layout
constexpr int kW1PackBF16Max = 4 * NetLayout<kMaxKX>::kS1 * 64 * 8;
constexpr int kPStrideMax = NetLayout<kMaxKX>::kPStride;

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x16 mma_f32(float a, float b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Hides a uniform pointer's value from the optimiser.  Used once per
// persistent-loop iteration so weight loads are issued where they are
// consumed instead of being hoisted out of the loop into hundreds of
// registers.
// The pointer is passed through as a global-memory one, so that the loads
// through it stay global loads (a generic pointer would make them flat
// loads, which every LDS wait then has to include).
template <typename T>
__device__ __forceinline__ T* opaque(T* p) {
    typedef __attribute__((address_space(1))) T GT;
    GT* g = (GT*)p;
    asm volatile("" : "+s"(g));
    return (T*)g;
}

// Row within a 32-row accumulator tile of register r in lane half h.
__host__ __device__ __forceinline__ int acc_row(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }
// Feature consumed at float32 chain step st (0..63) by lane half h.
__host__ __device__ __forceinline__ int phi32(int st, int h) { return 32 * (st >> 4) + acc_row(st & 15, h); }
// Feature consumed at bfloat16 chain step st (0..7), element i (0..7), half h.
__host__ __device__ __forceinline__ int phi16(int st, int i, int h) {
    return 32 * (st >> 1) + acc_row(8 * (st & 1) + i, h);
}

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return static_cast<uint16_t>((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

struct PackArgs {
    const float* w1;
    const float* w2;
    const float* w3;
    uint16_t* w3pb;
    uint16_t* w3tpb;
    uint16_t* w1tpb;
    float* w1p;
    float* w2p;
    float* w2tp;
    uint16_t* w1pb;
    uint16_t* w2pb;
    uint16_t* w2tpb;
    int bf16;
    int w1_in;   // first-layer input width (row stride of W1)
    int w1_ns;   // per-sample first-layer inputs (packed into w1p)
    int w1_q;    // float4 groups of w1p per output tile
    int w1_s1;   // K = 16 steps of w1pb per output tile
};

// Pack W1 (feature columns) and W2 / W2^T into matrix-core operand order.
// Operand packing of the network weights, one value per thread `gid` of
// kPackThreads (a device function so that it can share a launch).
constexpr int kPackThreads = kW2PackF32;

__device__ __forceinline__ void pack_weights(const PackArgs& a, int gid) {
    if (gid < kW2PackF32) {
        // float32: index ((mt*16 + q)*64 + lane)*4 + u, step st = 4q + u
        const int u = gid & 3, lane = (gid >> 2) & 63, q = (gid >> 8) & 15, mt = gid >> 12;
        const int st = 4 * q + u, m = lane & 31, h = lane >> 5;
        const int row = 32 * mt + m, kk = phi32(st, h);
        a.w2p[gid] = a.w2[row * kH + kk];
        a.w2tp[gid] = a.w2[kk * kH + row];
        if (a.bf16) {
            // bfloat16: index ((mt*8 + st)*64 + lane)*8 + i
            const int i = gid & 7, lane2 = (gid >> 3) & 63, st2 = (gid >> 9) & 7, mt2 = gid >> 12;
            const int m2 = lane2 & 31, h2 = lane2 >> 5;
            const int row2 = 32 * mt2 + m2, k2 = phi16(st2, i, h2);
            a.w2pb[gid] = f2bf(a.w2[row2 * kH + k2]);
            a.w2tpb[gid] = f2bf(a.w2[k2 * kH + row2]);
        }
    }
    if (gid < 4 * a.w1_q * 64 * 4) {
        // float32 layer 1: index ((mt*Q + q)*64 + lane)*4 + u, st = 4q+u, k = 2st + h (< w1_ns)
        const int u = gid & 3, lane = (gid >> 2) & 63, q = (gid >> 8) % a.w1_q, mt = (gid >> 8) / a.w1_q;
        const int st = 4 * q + u, m = lane & 31, h = lane >> 5;
        const int kk = 2 * st + h;
        a.w1p[gid] = kk < a.w1_ns ? a.w1[(32 * mt + m) * a.w1_in + kk] : 0.0f;
    }
    if (a.bf16 && gid < kW3PackBF16) {
        // index (st*64 + lane)*8 + i; lane (m, h), element i
        const int i = gid & 7, lane = (gid >> 3) & 63, st = gid >> 9;
        const int m = lane & 31, h = lane >> 5;
        const int k = phi16(st, i, h);
        a.w3pb[gid] = m < 3 ? f2bf(a.w3[m * kH + k]) : static_cast<uint16_t>(0);
        a.w1tpb[gid] = m < kC ? f2bf(a.w1[k * a.w1_in + m]) : static_cast<uint16_t>(0);
    }
    if (a.bf16 && gid < kW3TPackBF16) {
        // index (mt*64 + lane)*8 + i, k = 8h + i (< 3)
        const int i = gid & 7, lane = (gid >> 3) & 63, mt = gid >> 9;
        const int m = lane & 31, h = lane >> 5;
        const int k = 8 * h + i;
        a.w3tpb[gid] = k < 3 ? f2bf(a.w3[k * kH + 32 * mt + m]) : static_cast<uint16_t>(0);
    }
    if (a.bf16 && gid < 4 * a.w1_s1 * 64 * 8) {
        // bfloat16 layer 1: index ((mt*S1 + st)*64 + lane)*8 + i, k = 16st + 8h + i (< w1_ns)
        const int i = gid & 7, lane = (gid >> 3) & 63, st = (gid >> 9) % a.w1_s1, mt = (gid >> 9) / a.w1_s1;
        const int m = lane & 31, h = lane >> 5;
        const int kk = 16 * st + 8 * h + i;
        a.w1pb[gid] = kk < a.w1_ns ? f2bf(a.w1[(32 * mt + m) * a.w1_in + kk]) : static_cast<uint16_t>(0);
    }
}


struct MlpArgs {
    const int* sample_ray;
    const int64_t* n_kept;
    int64_t cap;
    const float* w1;      // [128][39] raw, for dL/dfeat
    const float* b2;
    const float* w3;      // [3][128]
    const float* b3;
    const float* base;    // [B][128] per-ray first-layer part incl. b1
    const float* pe;      // [B][32]
    const float* w1p;
    const float* w2p;
    const float* w2tp;
    const uint16_t* w1pb;
    const uint16_t* w2pb;
    const uint16_t* w2tpb;
    const uint16_t* w3pb;
    const uint16_t* w3tpb;
    const uint16_t* w1tpb;
    float* feat;          // [cap][12]: gathered features in
    float* col;           // [cap][4]: colour out (forward) / dL/dc in (backward)
    float* partial;       // [blocks][kPStride] weight-gradient partials
    int bf16;
    // backward: each sample's record (head, dL/dfeat) goes to its binned slot
    const int2* cell_rank;    // [cap] (cell, rank within cell)
    const int* cell_start;    // [ncell + 1]
    const float4* rec_head;   // [cap] (fx, fy, fz, dL/draw)
    float4* rec;              // [cap][4] binned records
    int nrays;                // rows of base and pe
};

// The query position of each sample, for the networks with an encoded
// position (a separate kernel argument, so that the other kernels' argument
// block stays as it is): x = o + t_k d in the sampler's float32 recipe,
// u = (x - pe_c) * pe_ih.
struct PosArgs {
    const float* rays_o;
    const float* rays_d;
    const float* jitter;
    const float* t_near;
    const int* sample_k;
    float step;
    float pe_c[3];
    float pe_ih[3];
};

__device__ __forceinline__ float4* binned_record(const MlpArgs& a, int64_t s) {
    const int2 cr = a.cell_rank[s];
    return a.rec + (static_cast<int64_t>(a.cell_start[cr.x]) + cr.y) * 4;
}

__device__ __forceinline__ MlpArgs refresh(const MlpArgs& a) {
    MlpArgs l = a;
    l.w1 = opaque(a.w1);
    l.b2 = opaque(a.b2);
    l.w3 = opaque(a.w3);
    l.b3 = opaque(a.b3);
    l.w1p = opaque(a.w1p);
    l.w2p = opaque(a.w2p);
    l.w2tp = opaque(a.w2tp);
    l.w1pb = opaque(a.w1pb);
    l.w2pb = opaque(a.w2pb);
    l.w2tpb = opaque(a.w2tpb);
    l.w3pb = opaque(a.w3pb);
    l.w3tpb = opaque(a.w3tpb);
    l.w1tpb = opaque(a.w1tpb);
    return l;
}

// ---------------------------------------------------------------------------
// forward chain for the 32 samples of one wave (float32 matrix cores)
// ---------------------------------------------------------------------------
struct ChainF32 {
    f32x16 h1[4];   // relu(layer-1) per 32-feature tile
    f32x16 z2[4];   // layer-2 pre-activation
};

__device__ __forceinline__ void load_base(const float* base, int r, int h, f32x16 acc[4]) {
    const float* br = base + static_cast<int64_t>(r) * kH;
    #pragma unroll
    for (int mt = 0; mt < 4; ++mt)
        #pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 v = *reinterpret_cast<const float4*>(br + 32 * mt + 8 * q + 4 * h);
            acc[mt][4 * q + 0] = v.x;
            acc[mt][4 * q + 1] = v.y;
            acc[mt][4 * q + 2] = v.z;
            acc[mt][4 * q + 3] = v.w;
        }
}

// One chained 128x128 layer: out[mt] += W * in, one output tile at a time
// (dependent matrix-core ops accumulate back to back).  Packed operands are
// read from `w2op` (LDS or global memory), one float4 per 4 steps.
template <typename P>
__device__ __forceinline__ f32x16 chain_tile_f32(const P* w2op, int lane, int mt, const f32x16 in[4], f32x16 acc) {
    #pragma unroll
    for (int q = 0; q < 16; ++q) {
        const float4 a4 = w2op[(mt * 16 + q) * 64 + lane];
        #pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int st = 4 * q + u;
            acc = mma_f32(a4[u], in[st >> 4][st & 15], acc);
        }
    }
    return acc;
}

// Layer 1 on the per-sample inputs xs (kS values: features, then the
// encoded position), then layer 2.  Lane half h supplies input 2 st + h of
// step st.
template <int KX, typename P>
__device__ __forceinline__ void forward_chain_f32(const MlpArgs& a, const P* w2op, int r,
                                                  const float xs[NetLayout<KX>::kS], int lane, ChainF32& c) {
    using L = NetLayout<KX>;
    const int h = lane >> 5;
    load_base(a.base, r, h, c.h1);
    const float4* w1p = reinterpret_cast<const float4*>(a.w1p);
    #pragma unroll
    for (int q = 0; q < L::kQ1; ++q) {
        float4 a4[4];
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt) a4[mt] = w1p[(mt * L::kQ1 + q) * 64 + lane];
        #pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k0 = 2 * (4 * q + u), k1 = k0 + 1;   // compile-time indices
            const float v0 = k0 < L::kS ? xs[k0 < L::kS ? k0 : 0] : 0.0f;
            const float v1 = k1 < L::kS ? xs[k1 < L::kS ? k1 : 0] : 0.0f;
            const float b = h ? v1 : v0;
            #pragma unroll
            for (int mt = 0; mt < 4; ++mt) c.h1[mt] = mma_f32(a4[mt][u], b, c.h1[mt]);
        }
    }
    #pragma unroll
    for (int mt = 0; mt < 4; ++mt)
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            c.h1[mt][rr] = fmaxf(c.h1[mt][rr], 0.0f);
            c.z2[mt][rr] = a.b2[32 * mt + acc_row(rr, h)];
        }
    #pragma unroll
    for (int mt = 0; mt < 4; ++mt) c.z2[mt] = chain_tile_f32(w2op, lane, mt, c.h1, c.z2[mt]);
}

// Layer 3 and the sigmoid: both lane halves end with the sample's colour.
__device__ __forceinline__ void head(const MlpArgs& a, const f32x16 z2[4], int h, float c[3]) {
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
    #pragma unroll
    for (int mt = 0; mt < 4; ++mt)
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const int j = 32 * mt + acc_row(rr, h);
            const float hv = fmaxf(z2[mt][rr], 0.0f);
            s0 += a.w3[j] * hv;
            s1 += a.w3[kH + j] * hv;
            s2 += a.w3[2 * kH + j] * hv;
        }
    s0 += __shfl_xor(s0, 32, 64);
    s1 += __shfl_xor(s1, 32, 64);
    s2 += __shfl_xor(s2, 32, 64);
    c[0] = 1.0f / (1.0f + expf(-(s0 + a.b3[0])));
    c[1] = 1.0f / (1.0f + expf(-(s1 + a.b3[1])));
    c[2] = 1.0f / (1.0f + expf(-(s2 + a.b3[2])));
}

__device__ __forceinline__ void load_feat(const float* feat, int64_t s, float f[12]) {
    const float4* p = reinterpret_cast<const float4*>(feat + s * 12);
    const float4 q0 = p[0], q1 = p[1], q2 = p[2];
    f[0] = q0.x; f[1] = q0.y; f[2] = q0.z; f[3] = q0.w;
    f[4] = q1.x; f[5] = q1.y; f[6] = q1.z; f[7] = q1.w;
    f[8] = q2.x; f[9] = q2.y; f[10] = q2.z; f[11] = q2.w;
}

// Per-sample first-layer inputs of sample s on ray r: its 12 features,
// then (KX > 0) the encoded position [u, sin(2^j u), cos(2^j u)], j < KX
// (sine and cosine by pe_sincos: |2^j u| <= 16 for a sample in the box).
// (in two parts: the loads, then the arithmetic, so that a caller can place
// other work between them)
struct SampleIn {
    float f[kC];
    float o[3], d[3];
    float p, tn;
    int k;
};

template <int KX>
__device__ __forceinline__ void sample_loads(const PosArgs& a, const float* feat, int64_t s, int r, SampleIn& in) {
    load_feat(feat, s, in.f);
    if constexpr (KX > 0) {
        #pragma unroll
        for (int i = 0; i < 3; ++i) {
            in.o[i] = a.rays_o[3 * r + i];
            in.d[i] = a.rays_d[3 * r + i];
        }
        in.p = a.jitter ? a.jitter[r] : 0.0f;
        in.tn = a.t_near[r];
        in.k = a.sample_k[s];
    }
}

template <int KX>
__device__ __forceinline__ void sample_encode(const PosArgs& a, const SampleIn& in, float xs[NetLayout<KX>::kS]) {
    #pragma unroll
    for (int i = 0; i < kC; ++i) xs[i] = in.f[i];
    if constexpr (KX > 0) {
        float x[3];
        const float t = dvgo_dev::recipe_tk(in.tn, in.p, in.k, a.step);
        dvgo_dev::recipe_x(in.o, in.d, t, x);
        #pragma unroll
        for (int i = 0; i < 3; ++i) xs[kC + i] = (x[i] - a.pe_c[i]) * a.pe_ih[i];
        #pragma unroll
        for (int j = 0; j < KX; ++j)
            #pragma unroll
            for (int i = 0; i < 3; ++i) {
                float sv, cv;
                dvgo_dev::pe_sincos(xs[kC + i] * static_cast<float>(1 << j), &sv, &cv);
                xs[kC + 3 + 6 * j + i] = sv;
                xs[kC + 6 + 6 * j + i] = cv;
            }
    }
}

template <int KX>
__device__ __forceinline__ void sample_inputs(const PosArgs& a, const float* feat, int64_t s, int r,
                                              float xs[NetLayout<KX>::kS]) {
    SampleIn in;
    sample_loads<KX>(a, feat, s, r, in);
    sample_encode<KX>(a, in, xs);
}

// Forward: colour of every listed sample.  LDS holds the packed W2.
template <int KX>
__global__ __launch_bounds__(256, 2) void mlp_fwd_f32_kernel(MlpArgs a0, PosArgs pa) {
    const MlpArgs& a = a0;
    __shared__ float4 sW2[kW2PackF32 / 4];
    for (int i = threadIdx.x; i < kW2PackF32 / 4; i += blockDim.x)
        sW2[i] = reinterpret_cast<const float4*>(a.w2p)[i];
    __syncthreads();
    const int64_t n = *a.n_kept < a.cap ? *a.n_kept : a.cap;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, h = lane >> 5;
    for (int64_t tile = static_cast<int64_t>(blockIdx.x) * 4 + wave; tile * 32 < n;
         tile += static_cast<int64_t>(gridDim.x) * 4) {
        const MlpArgs a = refresh(a0);
        const int64_t s = tile * 32 + m;
        const bool ok = s < n;
        const int64_t sc = ok ? s : n - 1;
        const int r = a.sample_ray[sc];
        float xs[NetLayout<KX>::kS];
        sample_inputs<KX>(pa, a.feat, sc, r, xs);
        ChainF32 c;
        forward_chain_f32<KX>(a, sW2, r, xs, lane, c);
        float col[3];
        head(a, c.z2, h, col);
        if (ok && h == 0) reinterpret_cast<float4*>(a.col)[s] = make_float4(col[0], col[1], col[2], 0.0f);
    }
}

// ---------------------------------------------------------------------------
// backward (float32): recompute, adjoint chain, weight gradients
// ---------------------------------------------------------------------------
constexpr int kSRow = 132;      // LDS row pitch (floats) of a staged sample row

template <int KX>
__global__ __launch_bounds__(256, 1) void mlp_bwd_f32_kernel(MlpArgs a0, PosArgs pa) {
    using L = NetLayout<KX>;
    __shared__ float sA[128 * kSRow];   // h1 rows, then dL/dz1 rows
    __shared__ float sB[128 * kSRow];   // h2 / dL/dz2 rows, then x' = [f, PE, 1, 0..] rows
    const int64_t n = *a0.n_kept < a0.cap ? *a0.n_kept : a0.cap;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, h = lane >> 5;
    f32x16 dW2[4], dW1[L::kXT];
    #pragma unroll
    for (int t = 0; t < 4; ++t)
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) dW2[t][rr] = 0.0f;
    #pragma unroll
    for (int t = 0; t < L::kXT; ++t)
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) dW1[t][rr] = 0.0f;
    float dW3a[3] = {0, 0, 0}, dW3b[3] = {0, 0, 0}, db2a = 0.0f, db2b = 0.0f, db3[3] = {0, 0, 0};
    float* myA = sA + wave * 32 * kSRow;
    float* myB = sB + wave * 32 * kSRow;
    for (int64_t blk = blockIdx.x; blk * 128 < n; blk += gridDim.x) {
        const MlpArgs a = refresh(a0);
        const float4* w2p = reinterpret_cast<const float4*>(a.w2p);
        const float4* w2tp = reinterpret_cast<const float4*>(a.w2tp);
        const int64_t s = blk * 128 + wave * 32 + m;
        const bool ok = s < n;
        const int64_t sc = ok ? s : n - 1;
        const int r = a.sample_ray[sc];
        float xs[L::kS];
        sample_inputs<KX>(pa, a.feat, sc, r, xs);
        ChainF32 c;
        forward_chain_f32<KX>(a, w2p, r, xs, lane, c);
        float col[3];
        head(a, c.z2, h, col);
        float dz3[3] = {0, 0, 0};
        if (ok) {
            const float4 dc = reinterpret_cast<const float4*>(a.col)[s];
            dz3[0] = dc.x * col[0] * (1.0f - col[0]);
            dz3[1] = dc.y * col[1] * (1.0f - col[1]);
            dz3[2] = dc.z * col[2] * (1.0f - col[2]);
        }
        // ---- dW3, db3 from h2 rows and dz3 staged in LDS
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            #pragma unroll
            for (int q = 0; q < 4; ++q)
                *reinterpret_cast<float4*>(myA + m * kSRow + 32 * mt + 8 * q + 4 * h) =
                    make_float4(fmaxf(c.z2[mt][4 * q], 0.0f), fmaxf(c.z2[mt][4 * q + 1], 0.0f),
                                fmaxf(c.z2[mt][4 * q + 2], 0.0f), fmaxf(c.z2[mt][4 * q + 3], 0.0f));
        if (h == 0) {
            myB[m * kSRow + 0] = dz3[0];
            myB[m * kSRow + 1] = dz3[1];
            myB[m * kSRow + 2] = dz3[2];
            db3[0] += dz3[0];
            db3[1] += dz3[1];
            db3[2] += dz3[2];
        }
        __syncthreads();
        #pragma unroll 4
        for (int ss = 0; ss < 32; ++ss) {
            const float ha = myA[ss * kSRow + lane], hb = myA[ss * kSRow + lane + 64];
            const float d0 = myB[ss * kSRow], d1 = myB[ss * kSRow + 1], d2 = myB[ss * kSRow + 2];
            dW3a[0] += d0 * ha; dW3a[1] += d1 * ha; dW3a[2] += d2 * ha;
            dW3b[0] += d0 * hb; dW3b[1] += d1 * hb; dW3b[2] += d2 * hb;
        }
        __syncthreads();
        // ---- dz2 = (W3^T dz3) * relu'(z2), in place of z2
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            #pragma unroll
            for (int rr = 0; rr < 16; ++rr) {
                const int j = 32 * mt + acc_row(rr, h);
                const float dh = a.w3[j] * dz3[0] + a.w3[kH + j] * dz3[1] + a.w3[2 * kH + j] * dz3[2];
                c.z2[mt][rr] = c.z2[mt][rr] > 0.0f ? dh : 0.0f;
            }
        // ---- stage h1 rows (sA) and dz2 rows (sB) of all four waves
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            #pragma unroll
            for (int q = 0; q < 4; ++q) {
                *reinterpret_cast<float4*>(myA + m * kSRow + 32 * mt + 8 * q + 4 * h) =
                    make_float4(c.h1[mt][4 * q], c.h1[mt][4 * q + 1], c.h1[mt][4 * q + 2], c.h1[mt][4 * q + 3]);
                *reinterpret_cast<float4*>(myB + m * kSRow + 32 * mt + 8 * q + 4 * h) =
                    make_float4(c.z2[mt][4 * q], c.z2[mt][4 * q + 1], c.z2[mt][4 * q + 2], c.z2[mt][4 * q + 3]);
            }
        __syncthreads();
        #pragma unroll 4
        for (int ss = 0; ss < 32; ++ss) {
            db2a += myB[ss * kSRow + lane];
            db2b += myB[ss * kSRow + lane + 64];
        }
        // dW2[j in tile `wave`][i] += sum over the 128 staged samples
        #pragma unroll 1
        for (int src = 0; src < 4; ++src)
            #pragma unroll 4
            for (int st = 0; st < 16; ++st) {
                const int row = src * 32 + 2 * st + h;
                const float av = sB[row * kSRow + 32 * wave + m];
                #pragma unroll
                for (int nt = 0; nt < 4; ++nt) dW2[nt] = mma_f32(av, sA[row * kSRow + 32 * nt + m], dW2[nt]);
            }
        // ---- dh1 = W2^T dz2 (chained), dz1 = dh1 * relu'(h1), in place of h1
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x16 dh1;
            #pragma unroll
            for (int rr = 0; rr < 16; ++rr) dh1[rr] = 0.0f;
            dh1 = chain_tile_f32(w2tp, lane, mt, c.z2, dh1);
            #pragma unroll
            for (int rr = 0; rr < 16; ++rr) c.h1[mt][rr] = c.h1[mt][rr] > 0.0f ? dh1[rr] : 0.0f;
        }
        // ---- dL/dfeat = W1[:, :12]^T dz1
        float df[12];
        #pragma unroll
        for (int cc = 0; cc < 12; ++cc) df[cc] = 0.0f;
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            #pragma unroll
            for (int rr = 0; rr < 16; ++rr) {
                const int i = 32 * mt + acc_row(rr, h);
                const float d = c.h1[mt][rr];
                #pragma unroll
                for (int cc = 0; cc < 12; ++cc) df[cc] += a.w1[i * L::kIn + cc] * d;
            }
        #pragma unroll
        for (int cc = 0; cc < 12; ++cc) df[cc] += __shfl_xor(df[cc], 32, 64);
        __syncthreads();
        // ---- stage dz1 rows (sA) and x' rows (sB)
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            #pragma unroll
            for (int q = 0; q < 4; ++q)
                *reinterpret_cast<float4*>(myA + m * kSRow + 32 * mt + 8 * q + 4 * h) =
                    make_float4(c.h1[mt][4 * q], c.h1[mt][4 * q + 1], c.h1[mt][4 * q + 2], c.h1[mt][4 * q + 3]);
        {
            // x' = [per-sample inputs, PE(d), 1, 0...]: lane half h stages
            // columns kHalf h .. kHalf h + kHalf - 1 (both candidates of a
            // column are compile-time indices)
            constexpr int kHalf = 16 * L::kXT;
            const float* per = a.pe + static_cast<int64_t>(r) * 32;
            float* row = myB + m * kSRow + kHalf * h;
            auto xval = [&](int j) -> float {
                if (j < L::kS) return xs[j < L::kS ? j : 0];
                if (j < L::kIn) return per[j - L::kS];
                return j == L::kIn ? 1.0f : 0.0f;
            };
            #pragma unroll
            for (int cc = 0; cc < kHalf; ++cc) row[cc] = h ? xval(kHalf + cc) : xval(cc);
        }
        if (ok && h == 0) {
            float4* rec = binned_record(a, s);
            rec[0] = a.rec_head[s];
            rec[1] = make_float4(df[0], df[1], df[2], df[3]);
            rec[2] = make_float4(df[4], df[5], df[6], df[7]);
            rec[3] = make_float4(df[8], df[9], df[10], df[11]);
        }
        __syncthreads();
        // dW1[i in tile `wave`][col] (col 39 = bias) over the 128 staged samples
        #pragma unroll 1
        for (int src = 0; src < 4; ++src)
            #pragma unroll 4
            for (int st = 0; st < 16; ++st) {
                const int row = src * 32 + 2 * st + h;
                const float av = sA[row * kSRow + 32 * wave + m];
                #pragma unroll
                for (int nt = 0; nt < L::kXT; ++nt) dW1[nt] = mma_f32(av, sB[row * kSRow + 32 * nt + m], dW1[nt]);
            }
        __syncthreads();
    }
    // ---- epilogue: this workgroup's partial of the flat gradient
    float* out = a0.partial + static_cast<int64_t>(blockIdx.x) * L::kPStride;
    #pragma unroll
    for (int nt = 0; nt < 4; ++nt)
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const int j = 32 * wave + acc_row(rr, h);
            out[L::kOffW2 + j * kH + 32 * nt + m] = dW2[nt][rr];
        }
    #pragma unroll
    for (int nt = 0; nt < L::kXT; ++nt)
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const int i = 32 * wave + acc_row(rr, h);
            const int col = 32 * nt + m;
            if (col < L::kIn) out[L::kOffW1 + i * L::kIn + col] = dW1[nt][rr];
            else if (col == L::kIn) out[L::kOffB1 + i] = dW1[nt][rr];
        }
    #pragma unroll
    for (int t = 0; t < 3; ++t) {
        db3[t] += __shfl_xor(db3[t], 32, 64);
        #pragma unroll
        for (int off = 16; off > 0; off >>= 1) db3[t] += __shfl_xor(db3[t], off, 64);
    }
    float* red = sA;   // [4 waves][512]
    #pragma unroll
    for (int t = 0; t < 3; ++t) {
        red[wave * 512 + t * kH + lane] = dW3a[t];
        red[wave * 512 + t * kH + lane + 64] = dW3b[t];
    }
    red[wave * 512 + 384 + lane] = db2a;
    red[wave * 512 + 384 + lane + 64] = db2b;
    if (lane == 0)
        #pragma unroll
        for (int t = 0; t < 3; ++t) sB[wave * 4 + t] = db3[t];
    __syncthreads();
    for (int i = threadIdx.x; i < 512; i += blockDim.x) {
        const float v = red[i] + red[512 + i] + red[1024 + i] + red[1536 + i];
        if (i < 384) out[L::kOffW3 + i] = v;
        else out[L::kOffB2 + (i - 384)] = v;
    }
    if (threadIdx.x < 3) out[L::kOffB3 + threadIdx.x] = sB[threadIdx.x] + sB[4 + threadIdx.x] + sB[8 + threadIdx.x] +
                                                   sB[12 + threadIdx.x];
}

// ---------------------------------------------------------------------------
// bfloat16 matrix cores (v_mfma_f32_32x32x16_bf16): same dataflow, K = 16
// per step, 8 consecutive K values per lane half; float32 accumulation.
// Weight-gradient operands are staged as [feature][sample] bfloat16 so that
// a lane's 8 consecutive samples are one 16-byte LDS read.
// ---------------------------------------------------------------------------
constexpr int kBP = 136;   // LDS pitch (bf16 elements) of a staged feature row
constexpr int kTP = 128;   // LDS pitch (bf16) of a staged sample row [sample][feature]

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;

// A staged row is 32 chunks of 8 bytes (4 features); chunk j of sample row r
// sits at chunk j ^ swz(r).  swz swaps the two low 2-bit fields of the row
// index, so that both the 16 rows one staging store covers per 16 lanes and
// the 4 rows x 4 chunks one transpose read covers per 16 lanes land on 16
// distinct chunk positions modulo 16 (all 32 LDS banks).
__device__ __forceinline__ int swz(int r) { return ((r & 3) << 2) | ((r >> 2) & 3); }
__device__ __forceinline__ __bf16* chunk_at(__bf16* T, int r, int j) { return T + r * kTP + 4 * (j ^ swz(r)); }
__device__ __forceinline__ const __bf16* chunk_at(const __bf16* T, int r, int j) {
    return T + r * kTP + 4 * (j ^ swz(r));
}

// This lane's packed operand fragment of step st (features phi16(st, 0..7, h),
// two runs of four) into its sample's row: two 8-byte stores.
__device__ __forceinline__ void stage_row(__bf16* T, int col_s, int st, int h, const bf16x8& v) {
    const int j = 8 * (st >> 1) + 4 * (st & 1) + h;   // chunk of features 32(st/2) + 16(st%2) + 4h ..
    bf16x4 lo, hi;
    #pragma unroll
    for (int e = 0; e < 4; ++e) {
        lo[e] = v[e];
        hi[e] = v[4 + e];
    }
    *reinterpret_cast<bf16x4*>(chunk_at(T, col_s, j)) = lo;
    *reinterpret_cast<bf16x4*>(chunk_at(T, col_s, j + 2)) = hi;
}

// K-major operand from [sample][feature] rows with two LDS transpose reads:
// lane (m, h) receives feature col0 + m of samples row0 + 8h .. row0 + 8h + 7.
// Each read transposes a 16x4 block within a 16-lane group: source lane t of
// group G addresses sample row0 + 8(G/2) + t/4, features col0 + 16(G%2) + 4(t%4)
// .. +3, and output lane i of the group receives feature col0 + 16(G%2) + i of
// those four samples.
__device__ __forceinline__ bf16x8 tr_operand(const __bf16* T, int row0, int col0, int lane) {
    const int G = lane >> 4, t = lane & 15;
    const int r = row0 + 8 * (G >> 1) + (t >> 2), j = (col0 + 16 * (G & 1)) / 4 + (t & 3);
    const s16x4 a = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)chunk_at(T, r, j));
    const s16x4 b = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)chunk_at(T, r + 4, j));
    typedef short s16x8 __attribute__((ext_vector_type(8)));
    const s16x8 ab = __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_bit_cast(bf16x8, ab);
}

// Round-to-nearest-even bfloat16 pairs of accumulator values, as the packed
// 32-bit words of an 8-element operand (one v_cvt_pk_bf16_f32 per pair).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 cvt_pair(const f32x16& v, int i) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const f32x2 x = {v[i], v[i + 1]};
    return __builtin_bit_cast(u16x2, __builtin_convertvector(x, bf16x2));
}

__device__ __forceinline__ bf16x8 pack8(const f32x16& v, int g) {
    u32x4 w;
    #pragma unroll
    for (int p = 0; p < 4; ++p) w[p] = __builtin_bit_cast(unsigned int, cvt_pair(v, 8 * g + 2 * p));
    return __builtin_bit_cast(bf16x8, w);
}

// bf16(relu(x)) for 8 accumulator values: round first, then clamp the signed
// 16-bit patterns at 0 (two values per packed integer max).  Rounding is
// monotone and maps no positive float32 to a negative bfloat16, so this
// equals rounding relu(x) (a negative input gives +0 either way).
__device__ __forceinline__ bf16x8 relu_pack8(const f32x16& v, int g) {
    const s16x2 zero = {0, 0};
    u32x4 w;
    #pragma unroll
    for (int p = 0; p < 4; ++p) {
        const s16x2 q = __builtin_elementwise_max(__builtin_bit_cast(s16x2, cvt_pair(v, 8 * g + 2 * p)), zero);
        w[p] = __builtin_bit_cast(unsigned int, q);
    }
    return __builtin_bit_cast(bf16x8, w);
}

// bf16(d) where the activation (a bf16 relu output, so a non-negative
// pattern) is non-zero, else +0: the relu derivative applied after
// rounding, with packed 16-bit min(act, 1) as the 0/1 factor (written as
// the two packed instructions; the optimiser would otherwise split each
// pair into compares and selects).  The constant 1 goes in a register
// holding it in both halves: an inline constant of a packed instruction
// would give the high half 0.
__device__ __forceinline__ bf16x8 relu_grad_pack8(const f32x16& d, int g, const bf16x8& act) {
    const u32x4 aw = __builtin_bit_cast(u32x4, act);
    const unsigned int ones = 0x00010001u;
    u32x4 w;
    #pragma unroll
    for (int p = 0; p < 4; ++p) {
        unsigned int m, r;
        asm("v_pk_min_u16 %0, %1, %2" : "=v"(m) : "v"(aw[p]), "v"(ones));
        asm("v_pk_mul_lo_u16 %0, %1, %2" : "=v"(r) : "v"(__builtin_bit_cast(unsigned int, cvt_pair(d, 8 * g + 2 * p))),
            "v"(m));
        w[p] = r;
    }
    return __builtin_bit_cast(bf16x8, w);
}

__device__ __forceinline__ float bf16r(float x) { return static_cast<float>(static_cast<__bf16>(x)); }

// NT output tiles mt0 .. mt0+NT-1 of a chained 128-wide layer, K step
// outermost: the NT weight fragments of step st+1 are read from LDS while
// the NT matrix-core ops of step st run (the order is pinned with
// scheduling-group barriers: the register allocator would otherwise
// serialise every read with its consumer).
template <int NT>
__device__ __forceinline__ void chain_tiles_bf16(const bf16x8* w, int lane, int mt0, const bf16x8 in[8],
                                                 f32x16 acc[NT]) {
    __builtin_amdgcn_sched_barrier(0);
    bf16x8 cur[NT];
    #pragma unroll
    for (int t = 0; t < NT; ++t) cur[t] = w[((mt0 + t) * 8) * 64 + lane];
    #pragma unroll
    for (int st = 0; st < 8; ++st) {
        bf16x8 nxt[NT];
        if (st < 7) {
            #pragma unroll
            for (int t = 0; t < NT; ++t) nxt[t] = w[((mt0 + t) * 8 + st + 1) * 64 + lane];
        }
        #pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mma_bf16(cur[t], in[st], acc[t]);
        if (st < 7) {
            #pragma unroll
            for (int t = 0; t < NT; ++t) cur[t] = nxt[t];
        }
    }
    __builtin_amdgcn_sched_group_barrier(0x100, NT, 0);       // LDS reads of step 0
    #pragma unroll
    for (int st = 0; st < 7; ++st) {
        __builtin_amdgcn_sched_group_barrier(0x100, NT, 0);   // LDS reads of step st+1
        __builtin_amdgcn_sched_group_barrier(0x008, NT, 0);   // matrix-core ops of step st
    }
    __builtin_amdgcn_sched_group_barrier(0x008, NT, 0);
    __builtin_amdgcn_sched_barrier(0);
}

struct ChainBF16 {
    f32x16 z2[4];   // layer-2 pre-activation
    bf16x8 hb[8];   // bf16(relu(layer 1)) in chained operand order
};

// Operand of layer-1 K step st for lane half h: per-sample inputs
// 16st + 8h .. 16st + 8h + 7 (zero beyond kS), selected with constant
// indices.
template <int KX>
__device__ __forceinline__ bf16x8 layer1_operand(const float xs[NetLayout<KX>::kS], int st, int h) {
    constexpr int kS = NetLayout<KX>::kS;
    bf16x8 fb;
    #pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k0 = 16 * st + e, k1 = k0 + 8;
        const float v0 = k0 < kS ? xs[k0 < kS ? k0 : 0] : 0.0f;
        const float v1 = k1 < kS ? xs[k1 < kS ? k1 : 0] : 0.0f;
        fb[e] = static_cast<__bf16>(h ? v1 : v0);
    }
    return fb;
}

template <int KX>
__device__ __forceinline__ void forward_chain_bf16(const MlpArgs& a, const bf16x8* sW1, const bf16x8* sW2,
                                                   const float* sB2, int r, const float xs[NetLayout<KX>::kS],
                                                   int lane, ChainBF16& c) {
    constexpr int kS1 = NetLayout<KX>::kS1;
    const int h = lane >> 5;
    f32x16 h1[4];
    load_base(a.base, r, h, h1);
    #pragma unroll
    for (int st = 0; st < kS1; ++st) {
        const bf16x8 fb = layer1_operand<KX>(xs, st, h);
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt) h1[mt] = mma_bf16(sW1[(mt * kS1 + st) * 64 + lane], fb, h1[mt]);
    }
    #pragma unroll
    for (int mt = 0; mt < 4; ++mt)
        #pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 b = *reinterpret_cast<const float4*>(sB2 + 32 * mt + 8 * q + 4 * h);
            c.z2[mt][4 * q] = b.x;
            c.z2[mt][4 * q + 1] = b.y;
            c.z2[mt][4 * q + 2] = b.z;
            c.z2[mt][4 * q + 3] = b.w;
        }
    #pragma unroll
    for (int st = 0; st < 8; ++st) c.hb[st] = relu_pack8(h1[st >> 1], st & 1);
    chain_tiles_bf16<4>(sW2, lane, 0, c.hb, c.z2);
}

// Layer 3 on matrix cores: logits of sample m land in lane m (half 0),
// registers 0..2; bfloat16 relu(z2) and W3, float32 accumulation.
__device__ __forceinline__ f32x16 head_bf16(const MlpArgs& a, const f32x16 z2[4], int lane, float c[3],
                                            bf16x8 h2b[8]) {
    const int h = lane >> 5;
    f32x16 z3;
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) z3[rr] = (h == 0 && rr < 3) ? a.b3[rr] : 0.0f;
    const bf16x8* w3 = reinterpret_cast<const bf16x8*>(a.w3pb);
    #pragma unroll
    for (int st = 0; st < 8; ++st) {
        const bf16x8 hv = relu_pack8(z2[st >> 1], st & 1);
        h2b[st] = hv;
        z3 = mma_bf16(w3[st * 64 + lane], hv, z3);
    }
    c[0] = 1.0f / (1.0f + expf(-z3[0]));
    c[1] = 1.0f / (1.0f + expf(-z3[1]));
    c[2] = 1.0f / (1.0f + expf(-z3[2]));
    return z3;
}

// kN 16-byte operand fragments copied from global memory to LDS by a
// workgroup of kThreads, in two steps: load() issues a thread's loads into
// registers, store() writes them to LDS.  Trip counts are compile-time
// constants, so loads of several copies can all be issued before the first
// store (a runtime-bounded copy loop waits on each load in turn).
template <int kThreads, int kN>
struct Frags {
    static constexpr int kPer = (kN + kThreads - 1) / kThreads;
    bf16x8 t[kPer];
    __device__ __forceinline__ void load(const bf16x8* src) {
        #pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int i = static_cast<int>(threadIdx.x) + u * kThreads;
            if (kN % kThreads == 0 || i < kN) t[u] = src[i];
        }
    }
    __device__ __forceinline__ void store(bf16x8* dst) const {
        #pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int i = static_cast<int>(threadIdx.x) + u * kThreads;
            if (kN % kThreads == 0 || i < kN) dst[i] = t[u];
        }
    }
};

// The forward's operands: packed W1 (kW1 fragments), W2 and b2 (float32).
template <int kThreads, int kW1>
__device__ __forceinline__ void load_packed_bf16(const MlpArgs& a, bf16x8* sW1, bf16x8* sW2, float* sB2) {
    Frags<kThreads, kW2PackBF16 / 8> f2;
    Frags<kThreads, kW1> f1;
    f2.load(reinterpret_cast<const bf16x8*>(a.w2pb));
    f1.load(reinterpret_cast<const bf16x8*>(a.w1pb));
    const float b2 = threadIdx.x < kH ? a.b2[threadIdx.x] : 0.0f;
    f2.store(sW2);
    f1.store(sW1);
    if (threadIdx.x < kH) sB2[threadIdx.x] = b2;
}

template <int KX>
__global__ __launch_bounds__(256, 3) void mlp_fwd_bf16_kernel(MlpArgs a0, PosArgs pa) {
    constexpr int kW1 = 4 * NetLayout<KX>::kS1 * 64;   // layer-1 operand fragments
    __shared__ bf16x8 sW2[kW2PackBF16 / 8];
    __shared__ bf16x8 sW1[kW1];
    __shared__ __attribute__((aligned(16))) float sB2[kH];
    load_packed_bf16<256, kW1>(a0, sW1, sW2, sB2);
    __syncthreads();
    const int64_t n = *a0.n_kept < a0.cap ? *a0.n_kept : a0.cap;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, h = lane >> 5;
    for (int64_t tile = static_cast<int64_t>(blockIdx.x) * 4 + wave; tile * 32 < n;
         tile += static_cast<int64_t>(gridDim.x) * 4) {
        const MlpArgs a = refresh(a0);
        const int64_t s = tile * 32 + m;
        const bool ok = s < n;
        const int64_t sc = ok ? s : n - 1;
        const int r = a.sample_ray[sc];
        float xs[NetLayout<KX>::kS];
        sample_inputs<KX>(pa, a.feat, sc, r, xs);
        ChainBF16 c;
        forward_chain_bf16<KX>(a, sW1, sW2, sB2, r, xs, lane, c);
        float col[3];
        bf16x8 h2b[8];
        head_bf16(a, c.z2, lane, col, h2b);
        if (ok && h == 0) reinterpret_cast<float4*>(a.col)[s] = make_float4(col[0], col[1], col[2], 0.0f);
    }
}

// NT output tiles of a chained 128-wide layer without the explicit read
// pipelining (for kernels with two wavefronts per SIMD, where the other
// wavefront covers the LDS latency).
template <int NT>
__device__ __forceinline__ void chain_tiles_plain_bf16(const bf16x8* w, int lane, int mt0, const bf16x8 in[8],
                                                       f32x16 acc[NT]) {
    #pragma unroll
    for (int st = 0; st < 8; ++st)
        #pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mma_bf16(w[((mt0 + t) * 8 + st) * 64 + lane], in[st], acc[t]);
}

// Inverse of stage_row: this lane's operand fragment of step st read back
// from its sample's row.
__device__ __forceinline__ bf16x8 read_row(const __bf16* T, int col_s, int st, int h) {
    const int j = 8 * (st >> 1) + 4 * (st & 1) + h;
    const s16x4 lo = *reinterpret_cast<const s16x4*>(chunk_at(T, col_s, j));
    const s16x4 hi = *reinterpret_cast<const s16x4*>(chunk_at(T, col_s, j + 2));
    typedef short s16x8 __attribute__((ext_vector_type(8)));
    const s16x8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_bit_cast(bf16x8, v);
}

// The per-ray first-layer part of two output tiles mt0, mt0 + 1.
__device__ __forceinline__ void load_base2(const float* base, int r, int h, int mt0, f32x16 acc[2]) {
    const float* br = base + static_cast<int64_t>(r) * kH;
    #pragma unroll
    for (int t = 0; t < 2; ++t)
        #pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 v = *reinterpret_cast<const float4*>(br + 32 * (mt0 + t) + 8 * q + 4 * h);
            acc[t][4 * q + 0] = v.x;
            acc[t][4 * q + 1] = v.y;
            acc[t][4 * q + 2] = v.z;
            acc[t][4 * q + 3] = v.w;
        }
}

// bfloat16 network adjoint with eight wavefronts per workgroup (two per
// SIMD, so that one wavefront's LDS and matrix-core latency hides behind the
// other's work).  The 128 samples of a block form four groups of 32
// (g = wave % 4); the two wavefronts of a group split every layer's output
// features in halves (q = wave / 4: tiles 2q, 2q + 1 of 32), exchanging the
// other half through the sample-row staging that the weight gradients read
// anyway.  Weight-gradient accumulators per wavefront: dW2 rows 32g, columns
// of tiles 2q, 2q + 1; dW1 rows 32g, x' columns of tile q; dW3 (q = 0) or
// db2 (q = 1) rows 32g.  The two halves of the head's logits and of
// dL/dfeat are summed through LDS.
//
// With the encoded position (KX > 0) the first layer takes kS1 K steps, the
// x' rows hold [f, PE_KX(u), PE(d), 1] (three tiles: the q = 0 wavefronts
// also accumulate tile 2, whose nine non-zero columns share dX with dW3,
// moved to columns 29..31), and the next block's inputs are not prefetched
// (its LDS goes to the wider first-layer operand).
template <int KX>
__global__ __launch_bounds__(512, 2) void mlp_bwd_bf16_kernel(MlpArgs a0, PosArgs pa) {
    using L = NetLayout<KX>;
    constexpr int kS1 = L::kS1;
    constexpr bool kPre = KX == 0;   // the next block's layer-1 inputs prefetched into LDS
    // dX columns of dW3 (q = 0): 0..2, or 29..31 when x' tile 2 takes
    // columns 0..8 (x' columns 64..72; its columns 73..95 are zero)
    constexpr int kW3Col = KX > 0 ? 29 : 0;
    static_assert(KX == 0 || NetLayout<KX>::kIn + 1 - 64 <= kW3Col, "x' tile 2 and dW3 share dX");
    __shared__ bf16x8 sW2[kW2PackBF16 / 8];
    __shared__ bf16x8 sW2T[kW2PackBF16 / 8];
    __shared__ bf16x8 sW1[4 * kS1 * 64];
    __shared__ __attribute__((aligned(16))) __bf16 tA[128 * kTP];   // h1 then dL/dz1, [sample][feature]
    __shared__ __attribute__((aligned(16))) __bf16 tB[128 * kTP];   // h2, then dL/dz2, then x'
    // dL/dz3 [channel][sample]: rows 0..2, row 3 zero (the B operand rows of
    // lanes m >= 3)
    __shared__ __attribute__((aligned(16))) __bf16 sC[4 * kBP];
    __shared__ __attribute__((aligned(16))) float sB2[kH];
    __shared__ float sB3[4];
    // The halves' logit partials (until B3) and the second half's dL/dfeat
    // partial (B6 .. B7) share one buffer.
    __shared__ __attribute__((aligned(16))) float sX[128 * kC];
    float4 (*sZ)[128] = reinterpret_cast<float4 (*)[128]>(sX);
    float (*sD)[kC] = reinterpret_cast<float (*)[kC]>(sX);
    // Packed operands of the head (W3, W3^T) and of dL/dfeat (W1[:, :12]^T),
    // only the lanes whose fragments are not zero: W3 rows 0..2 and W1^T
    // rows 0..11 (both lane halves), W3^T's lane half 0 (its K is the three
    // colour channels).  Other lanes use a zero fragment.
    __shared__ bf16x8 sW3c[8 * 2 * 3];
    __shared__ bf16x8 sW3Tc[4 * 32];
    __shared__ bf16x8 sW1Tc[8 * 2 * kC];
    // The next block's layer-1 inputs, copied straight from global memory to
    // LDS during the current block (no registers): the first-layer rows of
    // the rays r0 .. r0 + kPreRays - 1 (r0: the ray of the block's first
    // sample) and the features of the block's 128 samples.
    constexpr int kPreRays = 8;
    __shared__ __attribute__((aligned(16))) float sPB[kPre ? kPreRays * kH : 4];
    __shared__ __attribute__((aligned(16))) float sPF[kPre ? 128 * kC : 4];
    __shared__ float sRed[4 * 4];
    {   // every operand this kernel keeps in LDS: all loads first, then the stores
        Frags<512, kW2PackBF16 / 8> f2, f2t;
        Frags<512, 4 * kS1 * 64> f1;
        f2.load(reinterpret_cast<const bf16x8*>(a0.w2pb));
        f2t.load(reinterpret_cast<const bf16x8*>(a0.w2tpb));
        f1.load(reinterpret_cast<const bf16x8*>(a0.w1pb));
        // the compact operands, at most one fragment per thread each;
        // fragment (st, lane) of a packed operand is at st * 64 + lane
        const int ti = static_cast<int>(threadIdx.x);
        const bf16x8* g3 = reinterpret_cast<const bf16x8*>(a0.w3pb);
        const bf16x8* g3t = reinterpret_cast<const bf16x8*>(a0.w3tpb);
        const bf16x8* g1t = reinterpret_cast<const bf16x8*>(a0.w1tpb);
        bf16x8 c3, c3t, c1t;
        if (ti < 8 * 2 * 3) c3 = g3[(ti / 6) * 64 + 32 * ((ti / 3) & 1) + ti % 3];
        if (ti < 4 * 32) c3t = g3t[(ti / 32) * 64 + ti % 32];
        if (ti < 8 * 2 * kC) c1t = g1t[(ti / (2 * kC)) * 64 + 32 * ((ti / kC) & 1) + ti % kC];
        const float b2 = threadIdx.x < kH ? a0.b2[threadIdx.x] : 0.0f;
        const float b3 = threadIdx.x < 3 ? a0.b3[threadIdx.x] : 0.0f;
        f2.store(sW2);
        f2t.store(sW2T);
        f1.store(sW1);
        if (ti < 8 * 2 * 3) sW3c[ti] = c3;
        if (ti < 4 * 32) sW3Tc[ti] = c3t;
        if (ti < 8 * 2 * kC) sW1Tc[ti] = c1t;
        if (threadIdx.x < kH) sB2[threadIdx.x] = b2;
        if (threadIdx.x < 3) sB3[threadIdx.x] = b3;
    }
    for (int i = threadIdx.x; i < 4 * kBP; i += blockDim.x) sC[i] = static_cast<__bf16>(0.0f);
    __syncthreads();
    const int64_t n = *a0.n_kept < a0.cap ? *a0.n_kept : a0.cap;
    // The wavefront index in a scalar register: the role branches below are
    // then scalar branches.  Under a vector-masked branch a matrix
    // instruction still updates its accumulator in a wavefront whose mask is
    // empty.
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = wave & 3, q = wave >> 2;
    const int m = lane & 31, h = lane >> 5;
    const int col_s = g * 32 + m;     // this lane's sample column in the staged block
    f32x16 dW2[2], dW1, dX;           // dX: dW3 and (KX > 0) x' tile 2 (q = 0), or db2 (q = 1)
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
        dW2[0][rr] = 0.0f;
        dW2[1][rr] = 0.0f;
        dW1[rr] = 0.0f;
        dX[rr] = 0.0f;
    }
    float db3[3] = {0, 0, 0};
    bf16x8 ones, zero8;
    #pragma unroll
    for (int e = 0; e < 8; ++e) {
        ones[e] = static_cast<__bf16>(m == 0 ? 1.0f : 0.0f);
        zero8[e] = static_cast<__bf16>(0.0f);
    }
    // Block b's layer-1 inputs into sPB / sPF, by every wavefront: waves
    // 0..3 copy a 1 KB piece of sPB each (two 512-byte rows; rows past the
    // last ray read the last), waves 4..7 and 0..1 the six 1 KB pieces of
    // sPF (addresses past the capacity read the last feature quad).  The
    // copies land asynchronously; a wait on all memory operations precedes
    // the barrier before their use.
    typedef __attribute__((address_space(3))) void lds_void;
    auto prefetch = [&](const MlpArgs& a, int64_t b, int r0) {
        if constexpr (!kPre) return;
        if (wave < 4) {
            const int row = 2 * wave + (lane >> 5);
            const int rr = r0 + row < a.nrays ? r0 + row : a.nrays - 1;
            __builtin_amdgcn_global_load_lds(a.base + static_cast<int64_t>(rr) * kH + 4 * (lane & 31),
                                             (lds_void*)(sPB + 256 * wave), 16, 0, 0);
        }
        if (wave >= 4 || wave < 2) {
            const int piece = wave >= 4 ? wave - 4 : wave + 4;
            const int64_t fmax = a.cap * kC - 4;
            int64_t fo = b * 128 * kC + 256 * piece + 4 * lane;
            fo = fo < fmax ? fo : fmax;
            __builtin_amdgcn_global_load_lds(a.feat + fo, (lds_void*)(sPF + 256 * piece), 16, 0, 0);
        }
    };
    int r_next = 0, r0 = 0;   // r0: the ray of the current block's first sample (scalar)
    if (static_cast<int64_t>(blockIdx.x) * 128 < n) {
        const int64_t s0 = static_cast<int64_t>(blockIdx.x) * 128 + col_s;
        r_next = a0.sample_ray[s0 < n ? s0 : n - 1];
        r0 = __builtin_amdgcn_readfirstlane(a0.sample_ray[static_cast<int64_t>(blockIdx.x) * 128]);
        prefetch(a0, blockIdx.x, r0);
    }
    __builtin_amdgcn_s_waitcnt(0);   // the first block's copies (and r_next)
    __syncthreads();
    for (int64_t blk = blockIdx.x; blk * 128 < n; blk += gridDim.x) {
        const MlpArgs a = refresh(a0);
        const int64_t s = blk * 128 + col_s;
        const bool ok = s < n;
        const int64_t sc = ok ? s : n - 1;
        const int r = r_next;
        const bool more = (blk + gridDim.x) * 128 < n;
        int r0_next = r0;
        if (more) {
            const int64_t s1 = (blk + gridDim.x) * 128 + col_s;
            r_next = a.sample_ray[s1 < n ? s1 : n - 1];
            r0_next = a.sample_ray[(blk + gridDim.x) * 128];
        }
        // per-sample inputs of the head and of the record, issued here so
        // that their latency hides behind layers 1 and 2.  Every lane loads
        // (at a clamped, valid index): a load under a lane-dependent branch
        // is waited on inside that branch.
        const float4 dc = reinterpret_cast<const float4*>(a.col)[sc];
        const int2 cr = a.cell_rank[sc];
        const float4 rh = a.rec_head[sc];
        // ---- layer 1, this half's two tiles, staged as h1 rows
        {
            // features and the ray's first-layer row from the copies in LDS
            // (a ray outside the copied rows reads global memory); a sample
            // past the end takes zero inputs, its copy may be stale.  With
            // the encoded position: features and row from global memory, the
            // encoding evaluated here.
            float xs[L::kS];
            f32x16 h1[2];
            if constexpr (kPre) {
                load_feat(sPF, col_s, xs);
                const unsigned d = static_cast<unsigned>(r - r0);
                if (d < static_cast<unsigned>(kPreRays)) load_base2(sPB, static_cast<int>(d), h, 2 * q, h1);
                else load_base2(a.base, r, h, 2 * q, h1);
            } else {
                sample_inputs<KX>(pa, a.feat, sc, r, xs);
                load_base2(a.base, r, h, 2 * q, h1);
            }
            #pragma unroll
            for (int st = 0; st < kS1; ++st) {
                const bf16x8 fb = ok ? layer1_operand<KX>(xs, st, h) : zero8;
                #pragma unroll
                for (int t = 0; t < 2; ++t) h1[t] = mma_bf16(sW1[((2 * q + t) * kS1 + st) * 64 + lane], fb, h1[t]);
            }
            #pragma unroll
            for (int t = 0; t < 2; ++t)
                #pragma unroll
                for (int gg = 0; gg < 2; ++gg) stage_row(tA, col_s, 4 * q + 2 * t + gg, h, relu_pack8(h1[t], gg));
        }
        __syncthreads();   // B1: h1 rows complete; sPB, sPF read
        // ---- layer 2 and the head on this half
        f32x16 z2[2];
        #pragma unroll
        for (int t = 0; t < 2; ++t)
            #pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const float4 b = *reinterpret_cast<const float4*>(sB2 + 32 * (2 * q + t) + 8 * qq + 4 * h);
                z2[t][4 * qq] = b.x;
                z2[t][4 * qq + 1] = b.y;
                z2[t][4 * qq + 2] = b.z;
                z2[t][4 * qq + 3] = b.w;
            }
        {
            bf16x8 hb[8];
            #pragma unroll
            for (int st = 0; st < 8; ++st) hb[st] = read_row(tA, col_s, st, h);
            chain_tiles_plain_bf16<2>(sW2, lane, 2 * q, hb, z2);
        }
        bf16x8 h2h[4];   // bf16(relu(z2)) of this half, steps 4q .. 4q + 3
        f32x16 z3;
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) z3[rr] = (q == 0 && h == 0 && rr < 3) ? sB3[rr < 3 ? rr : 0] : 0.0f;
        {
            #pragma unroll
            for (int t = 0; t < 2; ++t)
                #pragma unroll
                for (int gg = 0; gg < 2; ++gg) {
                    const int st = 4 * q + 2 * t + gg;
                    h2h[2 * t + gg] = relu_pack8(z2[t], gg);
                    stage_row(tB, col_s, st, h, h2h[2 * t + gg]);
                    z3 = mma_bf16(m < 3 ? sW3c[(st * 2 + h) * 3 + (m < 3 ? m : 0)] : zero8, h2h[2 * t + gg], z3);
                }
        }
        if (h == 0) sZ[q][col_s] = make_float4(z3[0], z3[1], z3[2], 0.0f);
        __syncthreads();   // B2: h2 rows and both logit halves complete
        // The next block's copies, issued after layers 1 and 2 (the wait on
        // its first ray, loaded with this block's first loads, then costs
        // little) and before this block's record-slot load (which that wait
        // would otherwise include).
        if (more) prefetch(a, blk + gridDim.x, __builtin_amdgcn_readfirstlane(r0_next));
        const int slot0 = a.cell_start[cr.x];   // every lane, as above
        float dz3[3] = {0, 0, 0};
        if (h == 0) {
            const float4 z0 = sZ[0][col_s], z1 = sZ[1][col_s];
            const float zz[3] = {z0.x + z1.x, z0.y + z1.y, z0.z + z1.z};
            if (ok) {
                const float dcc[3] = {dc.x, dc.y, dc.z};
                #pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const float cv = 1.0f / (1.0f + expf(-zz[t]));
                    dz3[t] = dcc[t] * cv * (1.0f - cv);
                }
            }
            if (q == 0) {
                #pragma unroll
                for (int t = 0; t < 3; ++t) {
                    sC[t * kBP + col_s] = static_cast<__bf16>(dz3[t]);
                    db3[t] += dz3[t];
                }
            }
        }
        // dz2 of this half = (W3^T bf16(dz3)) * relu'(z2)
        bf16x8 zh[4];
        {
            bf16x8 dzb;
            #pragma unroll
            for (int e = 0; e < 8; ++e) dzb[e] = static_cast<__bf16>(e < 3 ? dz3[e < 3 ? e : 0] : 0.0f);
            #pragma unroll
            for (int t = 0; t < 2; ++t) {
                f32x16 dh;
                #pragma unroll
                for (int rr = 0; rr < 16; ++rr) dh[rr] = 0.0f;
                dh = mma_bf16(h == 0 ? sW3Tc[(2 * q + t) * 32 + m] : zero8, dzb, dh);
                #pragma unroll
                for (int gg = 0; gg < 2; ++gg) zh[2 * t + gg] = relu_grad_pack8(dh, gg, h2h[2 * t + gg]);
            }
        }
        __syncthreads();   // B3: dz3 rows complete
        if (q == 0) {      // dW3^T rows 32g over the 128 staged samples
            #pragma unroll
            for (int st = 0; st < 8; ++st) {
                const bf16x8 av = tr_operand(tB, 16 * st, 32 * g, lane);
                const int cm = m - kW3Col;   // dz3 channel of this lane's column (row 3 of sC is zero)
                const bf16x8 bv = *reinterpret_cast<const bf16x8*>(sC + (cm >= 0 && cm < 3 ? cm : 3) * kBP + 16 * st + 8 * h);
                dX = mma_bf16(av, bv, dX);
            }
        }
        __syncthreads();   // B4: h2 rows read
        #pragma unroll
        for (int u = 0; u < 4; ++u) stage_row(tB, col_s, 4 * q + u, h, zh[u]);
        __syncthreads();   // B5: dz2 rows complete
        // dW2 rows 32g, columns of tiles 2q, 2q + 1 (and db2 through a ones column)
        #pragma unroll 2
        for (int st = 0; st < 8; ++st) {
            const bf16x8 av = tr_operand(tB, 16 * st, 32 * g, lane);
            #pragma unroll
            for (int t = 0; t < 2; ++t) dW2[t] = mma_bf16(av, tr_operand(tA, 16 * st, 32 * (2 * q + t), lane), dW2[t]);
            if (q == 1) dX = mma_bf16(av, ones, dX);
        }
        // dh1 = W2^T dz2 on this half's tiles, dz1 = dh1 * relu'(z1), and this
        // half's share of dL/dfeat = W1[:, :12]^T dz1
        bf16x8 d1[4];
        f32x16 dft;
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) dft[rr] = 0.0f;
        {
            bf16x8 zb[8];
            #pragma unroll
            for (int st = 0; st < 8; ++st) zb[st] = read_row(tB, col_s, st, h);
            f32x16 dh1[2];
            #pragma unroll
            for (int t = 0; t < 2; ++t)
                #pragma unroll
                for (int rr = 0; rr < 16; ++rr) dh1[t][rr] = 0.0f;
            chain_tiles_plain_bf16<2>(sW2T, lane, 2 * q, zb, dh1);
            #pragma unroll
            for (int t = 0; t < 2; ++t)
                #pragma unroll
                for (int gg = 0; gg < 2; ++gg) {
                    const int st = 4 * q + 2 * t + gg;
                    d1[2 * t + gg] = relu_grad_pack8(dh1[t], gg, read_row(tA, col_s, st, h));
                    dft = mma_bf16(m < kC ? sW1Tc[(st * 2 + h) * kC + (m < kC ? m : 0)] : zero8, d1[2 * t + gg], dft);
                }
        }
        if (q == 1) {
            if (h == 0) {
                *reinterpret_cast<float4*>(&sD[col_s][0]) = make_float4(dft[0], dft[1], dft[2], dft[3]);
                *reinterpret_cast<float4*>(&sD[col_s][8]) = make_float4(dft[4], dft[5], dft[6], dft[7]);
            } else {
                *reinterpret_cast<float4*>(&sD[col_s][4]) = make_float4(dft[0], dft[1], dft[2], dft[3]);
            }
        }
        __syncthreads();   // B6: h1 and dz2 rows read; the second half's dL/dfeat in sD
        // Take delivery of the next block's ray index here, long after its
        // load: the memory counter that a later wait on it would use also
        // counts the record stores below, so consuming it at the top of the
        // next block would wait for those stores to complete.
        asm volatile("" ::"v"(r_next));
        #pragma unroll
        for (int u = 0; u < 4; ++u) stage_row(tA, col_s, 4 * q + u, h, d1[u]);
        // The sample's record: dft[0..3] hold channels 4h .. 4h + 3 of this
        // half, dft[4..7] (half 0) channels 8..11: half h writes record word
        // 1 + h, half 0 also words 0 and 3.  Written with fixed register
        // indices and one float4 store per word (the two halves' stores
        // merged into one with a lane-dependent register index had become
        // 16-way selects and four dword stores).
        auto write_record = [&]() {
            if (!ok) return;
            float4* rec = a.rec + (static_cast<int64_t>(slot0) + cr.y) * 4;
            const float4 oa = *reinterpret_cast<const float4*>(&sD[col_s][4 * h]);
            rec[1 + h] = make_float4(dft[0] + oa.x, dft[1] + oa.y, dft[2] + oa.z, dft[3] + oa.w);
            if (h == 0) {
                const float4 o8 = *reinterpret_cast<const float4*>(&sD[col_s][8]);
                rec[0] = rh;
                rec[3] = make_float4(dft[4] + o8.x, dft[5] + o8.y, dft[6] + o8.z, dft[7] + o8.w);
            }
        };
        if (q == 0) {
            if constexpr (KX > 0) {
                // x' = [f, PE_KX(u), PE(d), 1, 0...] -> tB (96 columns, this
                // lane's half of 24 four-column chunks), the per-sample
                // inputs evaluated again (every lane, at its clamped
                // sample).  Their loads go first, then the record (whose
                // operands then die before the encoding), then the
                // arithmetic: a wait on those loads does not include the
                // record stores.
                SampleIn in;
                sample_loads<KX>(pa, a.feat, sc, r, in);
                write_record();
                float xs[L::kS];
                sample_encode<KX>(pa, in, xs);
                const float* per = a.pe + static_cast<int64_t>(r) * 32;
                auto xval = [&](int j) -> float {
                    if (j < L::kS) return xs[j < L::kS ? j : 0];
                    if (j < L::kIn) return per[j - L::kS];
                    return j == L::kIn ? 1.0f : 0.0f;
                };
                constexpr int kChunks = 4 * L::kXT;   // per lane half
                #pragma unroll
                for (int kk = 0; kk < kChunks; ++kk) {
                    bf16x4 bv;
                    #pragma unroll
                    for (int e = 0; e < 4; ++e)
                        bv[e] = static_cast<__bf16>(h ? xval(4 * (kChunks + kk) + e) : xval(4 * kk + e));
                    *reinterpret_cast<uint2*>(chunk_at(tB, col_s, kChunks * h + kk)) = __builtin_bit_cast(uint2, bv);
                }
            } else {
                // x' = [f, PE, 1, 0...] -> tB (64 columns, this lane's half of
                // 8 float4 chunks): half 0 takes f[0..11] and PE[0..19], half 1
                // PE[20..26] and the constant 1 (stored after the PE) and zeros.
                // Every lane issues the same unconditional loads; half 1 then
                // zeroes chunks 2..7.
                const float4* f4 = reinterpret_cast<const float4*>(a.feat + sc * kC);
                const float4* p4 = reinterpret_cast<const float4*>(a.pe + static_cast<int64_t>(r) * 32);
                const float4* c01 = h ? p4 + 5 : f4;
                float4 v[8] = {c01[0], c01[1], f4[2], p4[0], p4[1], p4[2], p4[3], p4[4]};
                const uint32_t keep = static_cast<uint32_t>(h) - 1u;   // all ones in half 0, zero in half 1
                #pragma unroll
                for (int k = 0; k < 8; ++k) {
                    bf16x4 b;
                    b[0] = static_cast<__bf16>(v[k].x);
                    b[1] = static_cast<__bf16>(v[k].y);
                    b[2] = static_cast<__bf16>(v[k].z);
                    b[3] = static_cast<__bf16>(v[k].w);
                    uint2 bits = __builtin_bit_cast(uint2, b);
                    if (k >= 2) {   // a mask, not a branch: both halves run the same code
                        bits.x &= keep;
                        bits.y &= keep;
                    }
                    *reinterpret_cast<uint2*>(chunk_at(tB, col_s, 8 * h + k)) = bits;
                }
                write_record();
            }
        }
        __syncthreads();   // B7: dz1 and x' rows complete
        #pragma unroll
        for (int st = 0; st < 8; ++st) {
            const bf16x8 av = tr_operand(tA, 16 * st, 32 * g, lane);
            dW1 = mma_bf16(av, tr_operand(tB, 16 * st, 32 * q, lane), dW1);
            if (KX > 0 && q == 0) dX = mma_bf16(av, tr_operand(tB, 16 * st, 64, lane), dX);
        }
        __builtin_amdgcn_s_waitcnt(0);   // the next block's copies to sPB, sPF have landed
        __syncthreads();   // B8: rows read before the next block's staging
        r0 = __builtin_amdgcn_readfirstlane(r0_next);
    }
    // ---- epilogue: this workgroup's partial of the flat gradient
    float* out = a0.partial + static_cast<int64_t>(blockIdx.x) * L::kPStride;
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
        const int row = 32 * g + acc_row(rr, h);
        #pragma unroll
        for (int t = 0; t < 2; ++t) out[L::kOffW2 + row * kH + 32 * (2 * q + t) + m] = dW2[t][rr];
        const int cidx = 32 * q + m;
        if (cidx < L::kIn) out[L::kOffW1 + row * L::kIn + cidx] = dW1[rr];
        else if (cidx == L::kIn) out[L::kOffB1 + row] = dW1[rr];
        if (KX > 0 && q == 0) {
            const int c2 = 64 + m;
            if (c2 < L::kIn) out[L::kOffW1 + row * L::kIn + c2] = dX[rr];
            else if (c2 == L::kIn) out[L::kOffB1 + row] = dX[rr];
        }
        if (q == 0 && m >= kW3Col && m < kW3Col + 3) out[L::kOffW3 + (m - kW3Col) * kH + row] = dX[rr];
        if (q == 1 && m == 0) out[L::kOffB2 + row] = dX[rr];
    }
    if (q == 0) {
        #pragma unroll
        for (int t = 0; t < 3; ++t) {
            db3[t] += __shfl_xor(db3[t], 32, 64);
            for (int off = 16; off > 0; off >>= 1) db3[t] += __shfl_xor(db3[t], off, 64);
        }
        if (lane == 0)
            for (int t = 0; t < 3; ++t) sRed[g * 4 + t] = db3[t];
    }
    __syncthreads();
    if (threadIdx.x < 3)
        out[L::kOffB3 + threadIdx.x] = sRed[threadIdx.x] + sRed[4 + threadIdx.x] + sRed[8 + threadIdx.x] +
                                    sRed[12 + threadIdx.x];
}

// kx: frequencies of the encoded position in the input (0 or kMaxKX).
// The bfloat16 forward (under 168 registers) fits three wavefronts per SIMD:
// three workgroups per compute unit (2 -> 3: 25.7 -> 23.9 us per step at the
// full configuration); the float32 one, two.
inline void launch_mlp_fwd(const MlpArgs& a, const PosArgs& pa, int kx, int cus, hipStream_t s) {
    if (a.bf16 && kx == kMaxKX)
        DVGO_LAUNCH(K_MLP_FWD, mlp_fwd_bf16_kernel<kMaxKX>, dim3(cus * 3), dim3(256), 0, s, a, pa);
    else if (a.bf16) DVGO_LAUNCH(K_MLP_FWD, mlp_fwd_bf16_kernel<0>, dim3(cus * 3), dim3(256), 0, s, a, pa);
    else if (kx == kMaxKX)
        DVGO_LAUNCH(K_MLP_FWD, mlp_fwd_f32_kernel<kMaxKX>, dim3(cus * 2), dim3(256), 0, s, a, pa);
    else DVGO_LAUNCH(K_MLP_FWD, mlp_fwd_f32_kernel<0>, dim3(cus * 2), dim3(256), 0, s, a, pa);
}
inline void launch_mlp_bwd(const MlpArgs& a, const PosArgs& pa, int kx, int blocks, hipStream_t s) {
    if (a.bf16 && kx == kMaxKX)
        DVGO_LAUNCH(K_MLP_BWD, mlp_bwd_bf16_kernel<kMaxKX>, dim3(blocks), dim3(512), 0, s, a, pa);
    else if (a.bf16) DVGO_LAUNCH(K_MLP_BWD, mlp_bwd_bf16_kernel<0>, dim3(blocks), dim3(512), 0, s, a, pa);
    else if (kx == kMaxKX)
        DVGO_LAUNCH(K_MLP_BWD, mlp_bwd_f32_kernel<kMaxKX>, dim3(blocks), dim3(256), 0, s, a, pa);
    else DVGO_LAUNCH(K_MLP_BWD, mlp_bwd_f32_kernel<0>, dim3(blocks), dim3(256), 0, s, a, pa);
}

}  // namespace
