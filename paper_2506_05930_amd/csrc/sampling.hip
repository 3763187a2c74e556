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
// light at the same time (broadcast).  Lights are taken in groups of eight
// (one vector load of the visibilities when the rows allow it).  Pass 1 runs
// the sequential FP32 sum W = C_{m-1} and keeps the running sum at the end of
// every group in LDS; pass 2 finds the first group whose end exceeds u * W
// (the sum never decreases, so the pick lies in it) and recomputes that
// group's eight weights with the same operations from the sum before it,
// which reproduces C_i exactly.
constexpr int kWrsThreads = 256;

// The eight visibilities of group g of a row (missing lights read as 0).
template <typename VT>
__device__ inline void wrs_load8(const VT* __restrict__ row, int g, int m, bool vec, float (&v)[8]) {
    const int i0 = 8 * g;
    if (vec && i0 + 8 <= m) {
        if constexpr (sizeof(VT) == 4) {
            const float4 a = reinterpret_cast<const float4*>(row + i0)[0];
            const float4 b = reinterpret_cast<const float4*>(row + i0)[1];
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
            v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        } else {
            typedef VT v8 __attribute__((ext_vector_type(8)));
            const v8 a = *reinterpret_cast<const v8*>(row + i0);
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (float)a[j];
        }
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = i0 + j < m ? (float)row[i0 + j] : 0.0f;
    }
}

template <typename VT>
__global__ __launch_bounds__(kWrsThreads) void wrs_kernel(const VT* __restrict__ vis, int64_t n, int m,
                                                         const float* __restrict__ pos,
                                                         const float* __restrict__ nrm,
                                                         const float* __restrict__ lights, float vis_floor,
                                                         uint32_t k0, uint32_t k1, uint32_t frame,
                                                         const uint32_t* __restrict__ frame_dev, int vec,
                                                         int32_t* __restrict__ idx_out, float* __restrict__ pmf_out,
                                                         float* __restrict__ wsum_out, float* __restrict__ di_out,
                                                         const uint8_t* __restrict__ mask,
                                                         nvc_reservoir* __restrict__ res) {
    __shared__ float4 L[128];
    __shared__ float cend[16][kWrsThreads];       // running sum at the end of each group of 8 lights
    for (int i = threadIdx.x; i < m; i += blockDim.x)
        L[i] = make_float4(lights[4 * i + 0], lights[4 * i + 1], lights[4 * i + 2], lights[4 * i + 3]);
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (mask && mask[p] == 0) {                 // not needed at this pixel: an empty result
        idx_out[p] = -1;
        pmf_out[p] = 0.0f;
        wsum_out[p] = 0.0f;
        if (di_out) di_out[p] = 0.0f;
        if (res) res[p] = nvc_reservoir{-1, 0, 0.0f, 0.0f};
        return;
    }
    const int tid = threadIdx.x;
    const float px = pos[p * 3 + 0], py = pos[p * 3 + 1], pz = pos[p * 3 + 2];
    float nx = 0.f, ny = 0.f, nz = 0.f;
    const bool has_n = nrm != nullptr;
    if (has_n) {
        nx = nrm[p * 3 + 0];
        ny = nrm[p * 3 + 1];
        nz = nrm[p * 3 + 2];
    }
    const VT* row = vis + p * (int64_t)m;
    const int ng = (m + 7) / 8;
    float W = 0.0f, di = 0.0f, wlast = 0.0f, flast = 0.0f;
    int last_pos = -1;
    for (int g = 0; g < ng; ++g) {
        float v[8];
        wrs_load8(row, g, m, vec != 0, v);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int i = 8 * g + j;
            if (i < m) {
                float f, w;
                wrs_weight(L[i], px, py, pz, nx, ny, nz, has_n, v[j], vis_floor, f, w);
                W = W + w;
                di = fmaf(v[j], f, di);
                if (w > 0.0f) {
                    last_pos = i;
                    wlast = w;
                    flast = f;
                }
            }
        }
        cend[g][tid] = W;
    }
    const uint32_t fr = frame_dev ? *frame_dev : frame;
    const uint32_t r0 = philox_first_word((uint32_t)p, (uint32_t)((uint64_t)p >> 32), fr, 0u, k0, k1);
    const float u = (float)(r0 >> 8) * 0x1.0p-24f;
    const float t = u * W;
    int pick = -1;
    float wsel = 0.0f, fsel = 0.0f;
    int gs = -1;
    float c0 = 0.0f;
    for (int g = 0; g < ng; ++g) {
        const float ce = cend[g][tid];
        if (ce > t) {
            gs = g;
            break;
        }
        c0 = ce;
    }
    if (gs >= 0) {
        float v[8];
        wrs_load8(row, gs, m, vec != 0, v);
        float C = c0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int i = 8 * gs + j;
            if (i < m) {
                float f, w;
                wrs_weight(L[i], px, py, pz, nx, ny, nz, has_n, v[j], vis_floor, f, w);
                C = C + w;
                if (pick < 0 && C > t) {
                    pick = i;
                    wsel = w;
                    fsel = f;
                }
            }
        }
    }
    if (pick < 0 && last_pos >= 0) {          // only through rounding
        pick = last_pos;
        wsel = wlast;
        fsel = flast;
    }
    if (!(W > 0.0f)) pick = -1;
    idx_out[p] = pick;
    pmf_out[p] = pick >= 0 ? __fdiv_rn(wsel, W) : 0.0f;
    wsum_out[p] = W;
    if (di_out) di_out[p] = di * 0.318309886183790672f;    // 1/pi
    if (res) {
        // One candidate drawn with probability pmf, for a target f: M = 1, W = 1/pmf, w_sum = f W.
        const float Wr = pick >= 0 ? __fdiv_rn(W, wsel) : 0.0f;
        res[p] = nvc_reservoir{pick, pick >= 0 ? 1 : 0, fsel * Wr, Wr};
    }
}

template <typename VT>
static void run_wrs(const VT* vis, int64_t n, int m, const float* pos, const float* nrm, const float* lights,
                    float vis_floor, uint32_t k0, uint32_t k1, uint32_t frame, const uint32_t* frame_dev,
                    int32_t* idx, float* pmf, float* wsum, float* di, const uint8_t* mask, nvc_reservoir* res,
                    hipStream_t st) {
    const unsigned blocks = (unsigned)((n + kWrsThreads - 1) / kWrsThreads);
    const int vec = m % 8 == 0 && ((uintptr_t)vis & 15u) == 0;
    wrs_kernel<VT><<<blocks, kWrsThreads, 0, st>>>(vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, frame_dev,
                                                    vec, idx, pmf, wsum, di, mask, res);
}

hipError_t launch_wrs(const void* vis, int vis_dtype, int64_t n, int m, const float* pos, const float* nrm,
                      const float* lights, float vis_floor, uint64_t seed, uint32_t frame,
                      const uint32_t* frame_dev, int32_t* idx, float* pmf, float* wsum, float* di,
                      const uint8_t* mask, nvc_reservoir* res, hipStream_t st) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (vis_dtype == DT_F32)
        run_wrs((const float*)vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, frame_dev, idx, pmf, wsum, di, mask,
                res, st);
    else if (vis_dtype == DT_F16)
        run_wrs((const _Float16*)vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, frame_dev, idx, pmf, wsum, di, mask,
                res, st);
    else
        run_wrs((const __bf16*)vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, frame_dev, idx, pmf, wsum, di, mask,
                res, st);
    return hipGetLastError();
}

}  // namespace nvc
