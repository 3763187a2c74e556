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
// light at the same time (broadcast).
//
// Up to 32 lights (wrs_reg_kernel): the row's visibilities and the m light
// weights stay in registers.  Pass 1 computes every weight, the sequential
// FP32 sum W = C_{m-1} and the DI sum; pass 2 repeats the running sum from
// the registers and counts the C_i <= u * W (C never decreases, so the count
// is the first i with C_i > u * W); the picked light's weight and unshadowed
// term are then recomputed once with the same operations, bit for bit.
//
// More lights (wrs_group_kernel): lights are taken in groups of eight (one
// vector load of the visibilities when the rows allow it).  Pass 1 runs the
// sequential sum and keeps the running sum at the end of every group in LDS;
// pass 2 finds the first group whose end exceeds u * W and recomputes that
// group's eight weights from the sum before it, which reproduces C_i exactly.
//
// If no running sum exceeds u * W (only when u * W rounds to W) the pick is
// the last light with a positive weight; both kernels find it only then.
constexpr int kWrsThreads = 256;

struct WrsArgs {
    const void* vis;
    int64_t n;
    int m;
    const float* pos;
    const float* nrm;
    const float* lights;
    float vis_floor;
    uint32_t k0, k1, frame;
    const uint32_t* frame_dev;
    int32_t* idx_out;
    float* pmf_out;
    float* wsum_out;
    float* di_out;
    const uint8_t* mask;
    nvc_reservoir* res;
};

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

struct WrsPixel {
    float px, py, pz, nx, ny, nz;
    bool has_n;
};

__device__ inline bool wrs_begin(const WrsArgs& a, int64_t p, WrsPixel& q) {
    if (a.mask && a.mask[p] == 0) {             // not needed at this pixel: an empty result
        a.idx_out[p] = -1;
        a.pmf_out[p] = 0.0f;
        a.wsum_out[p] = 0.0f;
        if (a.di_out) a.di_out[p] = 0.0f;
        if (a.res) a.res[p] = nvc_reservoir{-1, 0, 0.0f, 0.0f};
        return false;
    }
    q.px = a.pos[p * 3 + 0];
    q.py = a.pos[p * 3 + 1];
    q.pz = a.pos[p * 3 + 2];
    q.nx = q.ny = q.nz = 0.0f;
    q.has_n = a.nrm != nullptr;
    if (q.has_n) {
        q.nx = a.nrm[p * 3 + 0];
        q.ny = a.nrm[p * 3 + 1];
        q.nz = a.nrm[p * 3 + 2];
    }
    return true;
}

__device__ inline float wrs_uniform(const WrsArgs& a, int64_t p) {
    const uint32_t fr = a.frame_dev ? *a.frame_dev : a.frame;
    const uint32_t r0 = philox_first_word((uint32_t)p, (uint32_t)((uint64_t)p >> 32), fr, 0u, a.k0, a.k1);
    return (float)(r0 >> 8) * 0x1.0p-24f;
}

__device__ inline void wrs_finish(const WrsArgs& a, int64_t p, int pick, float W, float wsel, float fsel, float di) {
    a.idx_out[p] = pick;
    a.pmf_out[p] = pick >= 0 ? __fdiv_rn(wsel, W) : 0.0f;
    a.wsum_out[p] = W;
    if (a.di_out) a.di_out[p] = di * 0.318309886183790672f;    // 1/pi
    if (a.res) {
        // One candidate drawn with probability pmf, for a target f: M = 1, W = 1/pmf, w_sum = f W.
        const float Wr = pick >= 0 ? __fdiv_rn(W, wsel) : 0.0f;
        a.res[p] = nvc_reservoir{pick, pick >= 0 ? 1 : 0, fsel * Wr, Wr};
    }
}

// FULL: m == MAXM and 16-byte aligned rows (vector loads, no light-count tests).
template <typename VT, int MAXM, bool HAS_N, bool FULL>
__global__ __launch_bounds__(kWrsThreads) void wrs_reg_kernel(WrsArgs a, const float4* __restrict__ LG,
                                                             const VT* __restrict__ vis) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    WrsPixel q;
    if (!wrs_begin(a, p, q)) return;
    const int m = FULL ? MAXM : a.m;
    const VT* row = vis + p * (int64_t)m;
    float v[MAXM];
    if constexpr (FULL) {
        constexpr int E = 16 / (int)sizeof(VT);
        typedef VT vecE __attribute__((ext_vector_type(E)));
#pragma unroll
        for (int g = 0; g < MAXM / E; ++g) {
            const vecE x = reinterpret_cast<const vecE*>(row)[g];
#pragma unroll
            for (int j = 0; j < E; ++j) v[g * E + j] = (float)x[j];
        }
    } else {
#pragma unroll
        for (int i = 0; i < MAXM; ++i) v[i] = i < m ? (float)row[i] : 0.0f;
    }
    // Every lane reads the same light (LG[i], i uniform): scalar loads.
    float w[MAXM];
    float W = 0.0f, di = 0.0f;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        w[i] = 0.0f;
        if (i < m) {
            float f;
            wrs_weight(LG[i], q.px, q.py, q.pz, q.nx, q.ny, q.nz, HAS_N, v[i], a.vis_floor, f, w[i]);
            W = W + w[i];
            di = fmaf(v[i], f, di);
        }
    }
    const float t = wrs_uniform(a, p) * W;
    int cnt = 0;
    float C = 0.0f;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        if (i < m) {
            C = C + w[i];
            cnt += C <= t ? 1 : 0;
        }
    }
    int pick = cnt < m ? cnt : -1;
    if (pick < 0 && W > 0.0f) {                    // only through rounding
#pragma unroll
        for (int i = 0; i < MAXM; ++i)
            if (i < m && w[i] > 0.0f) pick = i;
    }
    if (!(W > 0.0f)) pick = -1;
    float wsel = 0.0f, fsel = 0.0f;
    if (pick >= 0)
        wrs_weight(LG[pick], q.px, q.py, q.pz, q.nx, q.ny, q.nz, HAS_N, (float)row[pick], a.vis_floor, fsel, wsel);
    wrs_finish(a, p, pick, W, wsel, fsel, di);
}

// FULL8: m a multiple of SLAB and 16-byte aligned rows (vector loads, no light-count tests).
// SLAB lights are loaded at once (SLAB / 8 back-to-back 16-byte loads of one row), so that the
// cache lines of a row are used whole while they are resident, then weighed from registers.
template <typename VT, bool HAS_N, bool FULL8, int SLAB>
__global__ __launch_bounds__(kWrsThreads) void wrs_group_kernel(WrsArgs a, const float4* __restrict__ LG,
                                                               const VT* __restrict__ vis) {
    static_assert(SLAB % 8 == 0 && (FULL8 || SLAB == 8), "slabs of whole groups");
    constexpr int GPS = SLAB / 8;                 // groups of eight per slab
    __shared__ float cend[16][kWrsThreads];       // running sum at the end of each group of 8 lights
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    WrsPixel q;
    if (!wrs_begin(a, p, q)) return;
    const int tid = threadIdx.x;
    const int m = a.m;
    const VT* row = vis + p * (int64_t)m;
    const int ng = (m + 7) / 8;
    float W = 0.0f, di = 0.0f;
    for (int g0 = 0; g0 < ng; g0 += GPS) {
        float v[GPS][8];
#pragma unroll
        for (int k = 0; k < GPS; ++k) wrs_load8(row, g0 + k, m, FULL8, v[k]);
#pragma unroll
        for (int k = 0; k < GPS; ++k) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = 8 * (g0 + k) + j;
                if (FULL8 || i < m) {
                    float f, w;
                    wrs_weight(LG[i], q.px, q.py, q.pz, q.nx, q.ny, q.nz, HAS_N, v[k][j], a.vis_floor, f, w);
                    W = W + w;
                    di = fmaf(v[k][j], f, di);
                }
            }
            cend[g0 + k][tid] = W;
        }
    }
    const float t = wrs_uniform(a, p) * W;
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
        wrs_load8(row, gs, m, FULL8, v);
        float C = c0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int i = 8 * gs + j;
            if (FULL8 || i < m) {
                float f, w;
                wrs_weight(LG[i], q.px, q.py, q.pz, q.nx, q.ny, q.nz, HAS_N, v[j], a.vis_floor, f, w);
                C = C + w;
                if (pick < 0 && C > t) {
                    pick = i;
                    wsel = w;
                    fsel = f;
                }
            }
        }
    }
    if (pick < 0 && W > 0.0f) {                 // only through rounding: the last light with a positive weight
        for (int i = m - 1; i >= 0 && pick < 0; --i) {
            float f, w;
            wrs_weight(LG[i], q.px, q.py, q.pz, q.nx, q.ny, q.nz, HAS_N, (float)row[i], a.vis_floor, f, w);
            if (w > 0.0f) {
                pick = i;
                wsel = w;
                fsel = f;
            }
        }
    }
    if (!(W > 0.0f)) pick = -1;
    wrs_finish(a, p, pick, W, wsel, fsel, di);
}

template <typename VT>
static void run_wrs(WrsArgs a, hipStream_t st) {
    const unsigned blocks = (unsigned)((a.n + kWrsThreads - 1) / kWrsThreads);
    const bool aligned = ((uintptr_t)a.vis & 15u) == 0;
    const int m = a.m;
    auto reg = [&]<int MAXM>() {
        const bool full = m == MAXM && aligned && (MAXM * sizeof(VT)) % 16 == 0;
        const float4* lg = reinterpret_cast<const float4*>(a.lights);
        const VT* vis = reinterpret_cast<const VT*>(a.vis);
        if (a.nrm && full)
            wrs_reg_kernel<VT, MAXM, true, true><<<blocks, kWrsThreads, 0, st>>>(a, lg, vis);
        else if (a.nrm)
            wrs_reg_kernel<VT, MAXM, true, false><<<blocks, kWrsThreads, 0, st>>>(a, lg, vis);
        else if (full)
            wrs_reg_kernel<VT, MAXM, false, true><<<blocks, kWrsThreads, 0, st>>>(a, lg, vis);
        else
            wrs_reg_kernel<VT, MAXM, false, false><<<blocks, kWrsThreads, 0, st>>>(a, lg, vis);
    };
    if (m <= 8)
        reg.template operator()<8>();
    else if (m <= 32)
        reg.template operator()<32>();
    else {
        const bool full32 = m % 32 == 0 && aligned;
        const float4* lg = reinterpret_cast<const float4*>(a.lights);
        const VT* vis = reinterpret_cast<const VT*>(a.vis);
        if (a.nrm && full32)
            wrs_group_kernel<VT, true, true, 32><<<blocks, kWrsThreads, 0, st>>>(a, lg, vis);
        else if (a.nrm)
            wrs_group_kernel<VT, true, false, 8><<<blocks, kWrsThreads, 0, st>>>(a, lg, vis);
        else if (full32)
            wrs_group_kernel<VT, false, true, 32><<<blocks, kWrsThreads, 0, st>>>(a, lg, vis);
        else
            wrs_group_kernel<VT, false, false, 8><<<blocks, kWrsThreads, 0, st>>>(a, lg, vis);
    }
}

hipError_t launch_wrs(const void* vis, int vis_dtype, int64_t n, int m, const float* pos, const float* nrm,
                      const float* lights, float vis_floor, uint64_t seed, uint32_t frame,
                      const uint32_t* frame_dev, int32_t* idx, float* pmf, float* wsum, float* di,
                      const uint8_t* mask, nvc_reservoir* res, hipStream_t st) {
    WrsArgs a{vis, n, m, pos, nrm, lights, vis_floor, (uint32_t)seed, (uint32_t)(seed >> 32), frame, frame_dev,
              idx, pmf, wsum, di, mask, res};
    if (vis_dtype == DT_F32)
        run_wrs<float>(a, st);
    else if (vis_dtype == DT_F16)
        run_wrs<_Float16>(a, st);
    else
        run_wrs<__bf16>(a, st);
    return hipGetLastError();
}

}  // namespace nvc
