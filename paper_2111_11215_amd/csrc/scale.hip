// Progressive scaling of the fine stage (paper Sec. 4.2, "Progressive
// scaling"): a vertex grid resized by trilinear interpolation.  One thread
// per destination vertex; its position is min + j*((max-min)/(n-1)) per
// axis on the destination box, interpolated on the source grid (clamped at
// its faces like every gather of the library), all channels of the vertex.
#include "common.hpp"

namespace {

struct DstArgs {
    float mn[3];
    float step[3];   // (max-min)/(n-1), float32
    int n[3];
};

__global__ __launch_bounds__(256) void grid_resample_kernel(const float* __restrict__ src, dvgo::GridArgs gs, int C,
                                                            DstArgs d, float* __restrict__ dst) {
    const int64_t nv = static_cast<int64_t>(d.n[0]) * d.n[1] * d.n[2];
    const int64_t v = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (v >= nv) return;
    const int j2 = static_cast<int>(v % d.n[2]);
    const int j1 = static_cast<int>((v / d.n[2]) % d.n[1]);
    const int j0 = static_cast<int>(v / (static_cast<int64_t>(d.n[1]) * d.n[2]));
    const float x[3] = {d.mn[0] + static_cast<float>(j0) * d.step[0], d.mn[1] + static_cast<float>(j1) * d.step[1],
                        d.mn[2] + static_cast<float>(j2) * d.step[2]};
    int i0[3];
    float f[3];
    for (int i = 0; i < 3; ++i) {
        const float u = (x[i] - gs.mn[i]) * gs.scale[i];
        const float fl = fminf(fmaxf(floorf(u), 0.0f), static_cast<float>(gs.n[i] - 2));
        i0[i] = static_cast<int>(fl);
        f[i] = fminf(fmaxf(u - fl, 0.0f), 1.0f);
    }
    const int64_t sx = static_cast<int64_t>(gs.n[1]) * gs.n[2], sy = gs.n[2];
    const int64_t base = i0[0] * sx + i0[1] * sy + i0[2];
    float w[8];
    int64_t off[8];
    for (int c = 0; c < 8; ++c) {
        const int bx = (c >> 2) & 1, by = (c >> 1) & 1, bz = c & 1;
        w[c] = (bx ? f[0] : 1.0f - f[0]) * (by ? f[1] : 1.0f - f[1]) * (bz ? f[2] : 1.0f - f[2]);
        off[c] = (base + bx * sx + by * sy + bz) * C;
    }
    for (int ch = 0; ch < C; ++ch) {
        float acc = 0.0f;
        for (int c = 0; c < 8; ++c) acc += w[c] * src[off[c] + ch];
        dst[v * C + ch] = acc;
    }
}

}  // namespace

extern "C" {

int32_t dvgo_grid_resample(const float* src, const dvgo_box* src_box, int32_t channels, float* dst,
                           const dvgo_box* dst_box, void* stream) {
    if (!src || !dst || channels < 1 || !dvgo::box_ok(src_box, 2) || !dvgo::box_ok(dst_box, 2)) return DVGO_E_ARG;
    const int64_t ns = static_cast<int64_t>(src_box->n[0]) * src_box->n[1] * src_box->n[2];
    const int64_t nd = static_cast<int64_t>(dst_box->n[0]) * dst_box->n[1] * dst_box->n[2];
    if (ns * channels >= (1LL << 40) || nd >= (1LL << 31)) return DVGO_E_UNSUPPORTED;
    DstArgs d;
    for (int i = 0; i < 3; ++i) {
        d.mn[i] = dst_box->xyz_min[i];
        volatile float span = dst_box->xyz_max[i] - dst_box->xyz_min[i];
        volatile float nm1 = static_cast<float>(dst_box->n[i] - 1);
        d.step[i] = span / nm1;
        d.n[i] = dst_box->n[i];
    }
    DVGO_LAUNCH(K_GRID_RESAMPLE, grid_resample_kernel, dim3(static_cast<unsigned>((nd + 255) / 256)), dim3(256), 0,
                dvgo::as_stream(stream), src, dvgo::make_grid(*src_box), static_cast<int>(channels), d, dst);
    return dvgo::launch_status();
}

}  // extern "C"
