// Light selection by weighted reservoir sampling with neural DI (Sec. 1,
// Sec. 3.1, Sec. 3.2), training-pixel selection and shadow-ray labels
// against sphere occluders (Sec. 3.4).
//
// These kernels take integer decisions from FP32 arithmetic (the picked
// light, the binary label), so every product and sum is a separately rounded
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
                                                 uint32_t k1, uint32_t frame, int32_t* __restrict__ idx_out,
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
    const uint32_t r0 = philox_first_word((uint32_t)p, (uint32_t)((uint64_t)p >> 32), frame, 0u, k0, k1);
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
                    float vis_floor, uint32_t k0, uint32_t k1, uint32_t frame, int32_t* idx, float* pmf,
                    float* wsum, float* di, hipStream_t st) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (m <= 8)
        wrs_kernel<8, VT><<<blocks, 256, 0, st>>>(vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, idx, pmf,
                                                  wsum, di);
    else if (m <= 32)
        wrs_kernel<32, VT><<<blocks, 256, 0, st>>>(vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, idx, pmf,
                                                   wsum, di);
    else if (m <= 64)
        wrs_kernel<64, VT><<<blocks, 256, 0, st>>>(vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, idx, pmf,
                                                   wsum, di);
    else
        wrs_kernel<128, VT><<<blocks, 256, 0, st>>>(vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, idx,
                                                    pmf, wsum, di);
}

hipError_t launch_wrs(const void* vis, int vis_dtype, int64_t n, int m, const float* pos, const float* nrm,
                      const float* lights, float vis_floor, uint64_t seed, uint32_t frame, int32_t* idx,
                      float* pmf, float* wsum, float* di, hipStream_t st) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (vis_dtype == DT_F32)
        run_wrs((const float*)vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, idx, pmf, wsum, di, st);
    else if (vis_dtype == DT_F16)
        run_wrs((const _Float16*)vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, idx, pmf, wsum, di, st);
    else
        run_wrs((const __bf16*)vis, n, m, pos, nrm, lights, vis_floor, k0, k1, frame, idx, pmf, wsum, di, st);
    return hipGetLastError();
}

// ------------------------------------------------------------------ training pixels
__global__ __launch_bounds__(256) void select_pixels_kernel(uint32_t k0, uint32_t k1, uint32_t frame,
                                                            uint32_t n_pix, int64_t batch, int32_t* __restrict__ pix) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const uint32_t r0 = philox_first_word((uint32_t)b, (uint32_t)((uint64_t)b >> 32), frame, 1u, k0, k1);
    pix[b] = (int32_t)__umulhi(r0, n_pix);
}

hipError_t launch_select_pixels(uint64_t seed, uint32_t frame, int64_t n_pix, int64_t batch, int32_t* pix,
                                hipStream_t st) {
    const unsigned blocks = (unsigned)((batch + 255) / 256);
    select_pixels_kernel<<<blocks, 256, 0, st>>>((uint32_t)seed, (uint32_t)(seed >> 32), frame, (uint32_t)n_pix,
                                                 batch, pix);
    return hipGetLastError();
}

// ------------------------------------------------------------------ shadow labels
// A thread owns one sample and LPT lights.  Per sphere, the terms that depend
// only on (sample, sphere) are computed once and shared by the thread's
// lights; spheres, and the per-(light, sphere) "light inside" bits, sit in LDS.
constexpr int kLabelLPT = 8;
constexpr int kMaxSpheresLds = 4096;

__global__ __launch_bounds__(256) void labels_kernel(const float* __restrict__ pos, const int32_t* __restrict__ pix,
                                                     int64_t n, const float* __restrict__ lights, int m,
                                                     const float* __restrict__ spheres, int n_spheres,
                                                     uint8_t* __restrict__ labels) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    float4* S = reinterpret_cast<float4*>(smem_raw);                       // (cx, cy, cz, r*r)
    uint32_t* inside = reinterpret_cast<uint32_t*>(S + n_spheres);         // [n_spheres][groups]
    const int groups = (m + kLabelLPT - 1) / kLabelLPT;
    for (int s = threadIdx.x; s < n_spheres; s += blockDim.x) {
        const float cx = spheres[4 * s + 0], cy = spheres[4 * s + 1], cz = spheres[4 * s + 2], r = spheres[4 * s + 3];
        const float rr = r * r;
        S[s] = make_float4(cx, cy, cz, rr);
        for (int gi = 0; gi < groups; ++gi) {
            uint32_t bits = 0;
            for (int j = 0; j < kLabelLPT; ++j) {
                const int li = gi * kLabelLPT + j;
                if (li >= m) break;
                const float ex = cx - lights[4 * li + 0], ey = cy - lights[4 * li + 1], ez = cz - lights[4 * li + 2];
                if (((ex * ex + ey * ey) + ez * ez) < rr) bits |= 1u << j;
            }
            inside[s * groups + gi] = bits;
        }
    }
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * groups) return;
    const int64_t b = t / groups;
    const int gi = (int)(t - b * groups);
    const int64_t src = pix ? (int64_t)pix[b] : b;
    const float px = pos[src * 3 + 0], py = pos[src * 3 + 1], pz = pos[src * 3 + 2];
    float dx[kLabelLPT], dy[kLabelLPT], dz[kLabelLPT], dd[kLabelLPT];
    uint32_t vis = 0;
#pragma unroll
    for (int j = 0; j < kLabelLPT; ++j) {
        const int li = min(gi * kLabelLPT + j, m - 1);
        dx[j] = lights[4 * li + 0] - px;
        dy[j] = lights[4 * li + 1] - py;
        dz[j] = lights[4 * li + 2] - pz;
        dd[j] = (dx[j] * dx[j] + dy[j] * dy[j]) + dz[j] * dz[j];
        vis |= 1u << j;
    }
    for (int s = 0; s < n_spheres; ++s) {
        const float4 c = S[s];
        const uint32_t in_bits = inside[s * groups + gi];
        const float ox = c.x - px, oy = c.y - py, oz = c.z - pz;
        const float cc = ((ox * ox + oy * oy) + oz * oz) - c.w;
#pragma unroll
        for (int j = 0; j < kLabelLPT; ++j) {
            const float bb = (ox * dx[j] + oy * dy[j]) + oz * dz[j];
            bool occ;
            if (bb <= 0.0f)
                occ = cc < 0.0f;
            else if (bb >= dd[j])
                occ = (in_bits >> j) & 1u;
            else
                occ = cc * dd[j] < bb * bb;
            if (occ) vis &= ~(1u << j);
        }
    }
    uint8_t* out = labels + b * (int64_t)m + gi * kLabelLPT;
#pragma unroll
    for (int j = 0; j < kLabelLPT; ++j)
        if (gi * kLabelLPT + j < m) out[j] = (uint8_t)((vis >> j) & 1u);
}

hipError_t launch_labels(const float* pos, const int32_t* pix, int64_t n, const float* lights, int m,
                         const float* spheres, int n_spheres, uint8_t* labels, hipStream_t st) {
    const int groups = (m + kLabelLPT - 1) / kLabelLPT;
    const size_t smem = (size_t)n_spheres * 16 + (size_t)n_spheres * groups * 4;
    const int64_t total = n * groups;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(labels_kernel, dim3(blocks), dim3(256), smem, st, pos, pix, n, lights, m, spheres, n_spheres,
                       labels);
    return hipGetLastError();
}

}  // namespace nvc
