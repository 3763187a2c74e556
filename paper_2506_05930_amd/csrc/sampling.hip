// Light selection by weighted reservoir sampling with neural DI (Sec. 1,
// Sec. 3.1, Sec. 3.2).
//
// The picked light is an integer decided by FP32 arithmetic, so every product
// and sum is a separately rounded
// FP32 operation in the order documented in nvc.h: the library is built with
// FP contraction off, division is the compiler's correctly rounded sequence and
// the square root is refined to the correctly rounded one (sqrt_rn).
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace nvc {

// ------------------------------------------------------------------ WRS
// One thread per pixel; the lights sit in LDS and every lane reads the same
// light at the same time (broadcast).  The weights are kept in registers
// (MAXM >= m) and scanned sequentially in light order.
template <int MAXM, typename VT>
__global__ __launch_bounds__(256) void wrs_kernel(const VT* __restrict__ vis, int64_t n, int m,
                                                 const float* __restrict__ pos, const float* __restrict__ nrm,
                                                 const float* __restrict__ lights, float vis_floor, uint32_t k0,
                                                 uint32_t k1, uint32_t frame, const uint32_t* __restrict__ frame_dev,
                                                 int32_t* __restrict__ idx_out,
                                                 float* __restrict__ pmf_out, float* __restrict__ wsum_out,
                                                 float* __restrict__ di_out) {
    __shared__ float4 L[MAXM];
    for (int i = threadIdx.x; i < m; i += blockDim.x)
        L[i] = make_float4(lights[4 * i + 0], lights[4 * i + 1], lights[4 * i + 2], lights[4 * i + 3]);
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float px = pos[p * 3 + 0], py = pos[p * 3 + 1], pz = pos[p * 3 + 2];
    float nx = 0.f, ny = 0.f, nz = 0.f;
    const bool has_n = nrm != nullptr;
    if (has_n) {
        nx = nrm[p * 3 + 0];
        ny = nrm[p * 3 + 1];
        nz = nrm[p * 3 + 2];
    }
    const VT* vrow = vis + p * (int64_t)m;
    float w[MAXM];
    float W = 0.0f, di = 0.0f;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        w[i] = 0.0f;
        if (i < m) {
            const float4 l = L[i];
            const float dx = l.x - px, dy = l.y - py, dz = l.z - pz;
            const float d2 = fmaxf((dx * dx + dy * dy) + dz * dz, 1e-6f);
            float f;
            if (has_n) {
                const float nd = (nx * dx + ny * dy) + nz * dz;
                f = __fdiv_rn(l.w * fmaxf(nd, 0.0f), d2 * sqrt_rn(d2));
            } else {
                f = __fdiv_rn(l.w, d2);
            }
            const float v = (float)vrow[i];
            w[i] = f * fmaxf(v, vis_floor);
            W = W + w[i];
            di = fmaf(v, f, di);
        }
    }
    const uint32_t fr = frame_dev ? *frame_dev : frame;
    const uint32_t r0 = philox_first_word((uint32_t)p, (uint32_t)((uint64_t)p >> 32), fr, 0u, k0, k1);
    const float u = (float)(r0 >> 8) * 0x1.0p-24f;
    const float t = u * W;
    int pick = -1, last_pos = -1;
    float C = 0.0f, wsel = 0.0f;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        if (i < m) {
            C = C + w[i];
            if (w[i] > 0.0f) last_pos = i;
            if (pick < 0 && C > t) {
                pick = i;
                wsel = w[i];
            }
        }
    }
    if (pick < 0 && last_pos >= 0) {          // only through rounding
        pick = last_pos;
#pragma unroll
        for (int i = 0; i < MAXM; ++i)
            if (i == last_pos) wsel = w[i];
    }
    if (!(W > 0.0f)) pick = -1;
    idx_out[p] = pick;
    pmf_out[p] = pick >= 0 ? __fdiv_rn(wsel, W) : 0.0f;
    wsum_out[p] = W;
    if (di_out) di_out[p] = di * 0.318309886183790672f;    // 1/pi
}

template <typename VT>
static void run_wrs(const VT* vis, int64_t n, int m, const float* pos, const float* nrm, const float* lights,
                    float vis_floor, uint32_t k0, uint32_t k1, uint32_t frame, const uint32_t* frame_dev,
                    int32_t* idx, float* pmf, float* wsum, float* di, hipStream_t st) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    auto go = [&](auto kernel) {
        kernel<<<blocks, 256, 0, st>>>(vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, frame_dev, idx, pmf,
                                       wsum, di);
    };
    if (m <= 8)
        go(wrs_kernel<8, VT>);
    else if (m <= 32)
        go(wrs_kernel<32, VT>);
    else if (m <= 64)
        go(wrs_kernel<64, VT>);
    else
        go(wrs_kernel<128, VT>);
}

hipError_t launch_wrs(const void* vis, int vis_dtype, int64_t n, int m, const float* pos, const float* nrm,
                      const float* lights, float vis_floor, uint64_t seed, uint32_t frame,
                      const uint32_t* frame_dev, int32_t* idx, float* pmf, float* wsum, float* di,
                      hipStream_t st) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (vis_dtype == DT_F32)
        run_wrs((const float*)vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, frame_dev, idx, pmf, wsum, di, st);
    else if (vis_dtype == DT_F16)
        run_wrs((const _Float16*)vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, frame_dev, idx, pmf, wsum, di, st);
    else
        run_wrs((const __bf16*)vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, frame_dev, idx, pmf, wsum, di, st);
    return hipGetLastError();
}

}  // namespace nvc
