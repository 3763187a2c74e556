// Standalone hash-grid encoding (Sec. 3.1 Fig. "overview" step 1).
// One thread per (point, level): consecutive threads cover the levels of one
// point, so the F-wide outputs of a point form one contiguous, coalesced row.
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace nvc {

GridDev grid_to_dev(const GridHost& g) {
    GridDev d{};
    d.n_levels = g.n_levels;
    d.n_feat = g.n_feat;
    d.T = 1u << g.log2_T;
    d.dense_mask = g.dense_mask;
    for (int l = 0; l < kMaxLevels; ++l) d.res[l] = g.res[l];
    return d;
}

template <int F, typename OUT>
__global__ __launch_bounds__(256) void encode_kernel(GridDev g, const float* __restrict__ table,
                                                    const float* __restrict__ pos, int64_t n,
                                                    OUT* __restrict__ enc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int L = g.n_levels;
    if (t >= n * L) return;
    const int64_t p = t / L;
    const int l = (int)(t - p * L);
    const float x = clamp_unit(pos[p * 3 + 0]);
    const float y = clamp_unit(pos[p * 3 + 1]);
    const float z = clamp_unit(pos[p * 3 + 2]);
    float v[F];
    encode_level<F>(table, g, l, x, y, z, v);
    OUT* o = enc + p * (int64_t)(L * F) + l * F;
#pragma unroll
    for (int j = 0; j < F; ++j) o[j] = (OUT)v[j];
}

template <int F>
static void run_encode(const GridDev& g, const float* table, const float* pos, int64_t n, void* enc, int dt,
                       hipStream_t st) {
    const int64_t total = n * g.n_levels;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (dt == DT_F32)
        encode_kernel<F, float><<<blocks, 256, 0, st>>>(g, table, pos, n, (float*)enc);
    else if (dt == DT_F16)
        encode_kernel<F, _Float16><<<blocks, 256, 0, st>>>(g, table, pos, n, (_Float16*)enc);
    else
        encode_kernel<F, __bf16><<<blocks, 256, 0, st>>>(g, table, pos, n, (__bf16*)enc);
}

hipError_t launch_encode(const GridHost& gh, const float* table, const float* pos, int64_t n, void* enc,
                         int enc_dtype, hipStream_t st) {
    const GridDev g = grid_to_dev(gh);
    if (g.n_feat == 1)
        run_encode<1>(g, table, pos, n, enc, enc_dtype, st);
    else if (g.n_feat == 2)
        run_encode<2>(g, table, pos, n, enc, enc_dtype, st);
    else
        run_encode<4>(g, table, pos, n, enc, enc_dtype, st);
    return hipGetLastError();
}

}  // namespace nvc
