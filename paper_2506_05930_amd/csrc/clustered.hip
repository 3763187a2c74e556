// Clustered neural visibility cache (Sec. 3.6): k-means clusters of the
// lights (host), one shadow ray per cluster per training sample, and the
// two-step light pick (WRS over clusters, then RIS inside the cluster).
//
// Random words: Philox4x32-10, counter (index lo, index hi, frame, tag), key =
// seed; tag 0 word 0: cluster-pick uniform; tag 2 word 0: RIS selection
// uniform; tag 4 + k/4, word k%4: RIS candidate k; tag 32 + c/4, word c%4:
// the training light of cluster c.  An index in [0, m) is (word * m) >> 32.
//
// Picks are integers decided by FP32 arithmetic: every product and sum is a
// separately rounded FP32 operation in the order documented in nvc.h (FP
// contraction is off, divisions are correctly rounded, sqrt is sqrt_rn).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "device_common.hpp"

namespace nvc {

constexpr uint32_t kTagRisSelect = 2;
constexpr uint32_t kTagRisCand = 4;
constexpr uint32_t kTagClusterLight = 32;

__device__ inline uint32_t index_in(uint32_t word, uint32_t m) {
    return (uint32_t)(((uint64_t)word * (uint64_t)m) >> 32);
}

// Cluster c's lights [o0, o1) of `members`, or an empty range if the offsets
// are not an ordered range inside [0, n_lights].
__device__ inline void cluster_range(const int32_t* __restrict__ offsets, int c, int n_lights, int& o0, int& m) {
    const int a = offsets[c], b = offsets[c + 1];
    const bool ok = a >= 0 && b >= a && b <= n_lights;
    o0 = ok ? a : 0;
    m = ok ? b - a : 0;
}

// ------------------------------------------------------------------ labels
// One thread per (sample, cluster): the cluster's training light for the
// sample, then the segment test against every sphere (staged in LDS), in the
// FP32 order of the plain labels.
constexpr int kClLabelThreads = 256;

__global__ __launch_bounds__(kClLabelThreads) void clustered_labels_kernel(
    const float* __restrict__ pos, const int32_t* __restrict__ pix, int64_t n, const float* __restrict__ lights,
    int n_lights, const int32_t* __restrict__ offsets, const int32_t* __restrict__ members, int k,
    const float* __restrict__ spheres, int n_spheres, uint32_t k0, uint32_t k1, uint32_t frame,
    const uint32_t* __restrict__ frame_dev, uint8_t* __restrict__ labels) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    float4* S = reinterpret_cast<float4*>(smem_raw);                 // (cx, cy, cz, r*r)
    for (int s = threadIdx.x; s < n_spheres; s += blockDim.x) {
        const float r = spheres[4 * s + 3];
        S[s] = make_float4(spheres[4 * s + 0], spheres[4 * s + 1], spheres[4 * s + 2], r * r);
    }
    __syncthreads();
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * (int64_t)k) return;
    const int64_t b = e / k;
    const int c = (int)(e - b * k);
    int o0, m;
    cluster_range(offsets, c, n_lights, o0, m);
    uint8_t vis = 0;
    if (m > 0) {
        const uint32_t fr = frame_dev ? *frame_dev : frame;
        uint32_t w[4];
        philox_words((uint32_t)b, (uint32_t)((uint64_t)b >> 32), fr, kTagClusterLight + (uint32_t)(c / 4), k0, k1, w);
        const int l = members[o0 + (int)index_in(w[c % 4], (uint32_t)m)];
        if (l >= 0 && l < n_lights) {
            const int64_t src = pix ? (int64_t)pix[b] : b;
            const float px = pos[src * 3 + 0], py = pos[src * 3 + 1], pz = pos[src * 3 + 2];
            const float lx = lights[4 * l + 0], ly = lights[4 * l + 1], lz = lights[4 * l + 2];
            const float dx = lx - px, dy = ly - py, dz = lz - pz;
            const float dd = (dx * dx + dy * dy) + dz * dz;
            bool occ = false;
            for (int s = 0; s < n_spheres; ++s) {
                const float4 q = S[s];
                const float ox = q.x - px, oy = q.y - py, oz = q.z - pz;
                const float cc = ((ox * ox + oy * oy) + oz * oz) - q.w;
                const float bb = (ox * dx + oy * dy) + oz * dz;
                const float ex = q.x - lx, ey = q.y - ly, ez = q.z - lz;
                const bool near_p = bb <= 0.0f;
                const bool near_l = !near_p && bb >= dd;
                const bool o = near_p ? cc < 0.0f : (near_l ? ((ex * ex + ey * ey) + ez * ez) < q.w : cc * dd < bb * bb);
                occ = occ || o;                    // no early exit: lanes stay converged
            }
            vis = occ ? 0 : 1;
        }
    }
    labels[b * k + c] = vis;
}

// ------------------------------------------------------------------ sampling
constexpr int kClSampleThreads = 256;

// Candidate kk's light (or -1) and its unshadowed weight f at the pixel.
__device__ inline void ris_candidate(const uint32_t (&w)[4], int kk, const int32_t* __restrict__ members, int o0,
                                     int m, int n_lights, const float* __restrict__ lights, float px, float py,
                                     float pz, float nx, float ny, float nz, bool has_n, int& l, float& f) {
    l = members[o0 + (int)index_in(w[kk % 4], (uint32_t)m)];
    f = 0.0f;
    if (l < 0 || l >= n_lights) {
        l = -1;
        return;
    }
    const float4 L = make_float4(lights[4 * l + 0], lights[4 * l + 1], lights[4 * l + 2], lights[4 * l + 3]);
    float wdummy;
    wrs_weight(L, px, py, pz, nx, ny, nz, has_n, 1.0f, 0.0f, f, wdummy);
}

// NC > 0: the candidate count is NC (compile time) and the candidates stay in
// registers between the two passes; NC = 0: n_cand at run time, pass 2
// recomputes them.
template <typename VT, int NC>
__global__ __launch_bounds__(kClSampleThreads) void clustered_sample_kernel(
    const VT* __restrict__ vis, int64_t n, int k, const float* __restrict__ pos, const float* __restrict__ nrm,
    const float* __restrict__ lights, int n_lights, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ members, float vis_floor, int n_cand, uint32_t k0, uint32_t k1, uint32_t frame,
    const uint32_t* __restrict__ frame_dev, int32_t* __restrict__ idx_out, float* __restrict__ weight_out,
    int32_t* __restrict__ cluster_out, const uint8_t* __restrict__ mask, nvc_reservoir* __restrict__ res) {
    __shared__ int off0[128];
    __shared__ int msize[128];
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
        int o, m;
        cluster_range(offsets, c, n_lights, o, m);
        off0[c] = o;
        msize[c] = m;
    }
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (mask && mask[p] == 0) {                 // not needed at this pixel: an empty result
        idx_out[p] = -1;
        weight_out[p] = 0.0f;
        if (cluster_out) cluster_out[p] = -1;
        if (res) res[p] = nvc_reservoir{-1, 0, 0.0f, 0.0f};
        return;
    }
    const uint32_t fr = frame_dev ? *frame_dev : frame;
    const uint32_t plo = (uint32_t)p, phi = (uint32_t)((uint64_t)p >> 32);
    const VT* row = vis + p * (int64_t)k;

    // Step 1: WRS over the clusters, w_j = m_j * max(v_j, floor).
    float W = 0.0f, wlast = 0.0f;
    int last_pos = -1;
    for (int j = 0; j < k; ++j) {
        const float w = (float)msize[j] * fmaxf((float)row[j], vis_floor);
        W = W + w;
        if (w > 0.0f) {
            last_pos = j;
            wlast = w;
        }
    }
    int y = -1;
    float wy = 0.0f;
    if (W > 0.0f) {
        const uint32_t r0 = philox_first_word(plo, phi, fr, 0u, k0, k1);
        const float t = ((float)(r0 >> 8) * 0x1.0p-24f) * W;
        float C = 0.0f;
        for (int j = 0; j < k; ++j) {
            const float w = (float)msize[j] * fmaxf((float)row[j], vis_floor);
            C = C + w;
            if (C > t) {
                y = j;
                wy = w;
                break;
            }
        }
        if (y < 0) {                               // only through rounding
            y = last_pos;
            wy = wlast;
        }
    }
    int pick = -1, cl = -1;
    float Wx = 0.0f, wsum_r = 0.0f;
    if (y >= 0) {
        const float P = __fdiv_rn(wy, W);
        const int o0 = off0[y], m = msize[y];
        const float px = pos[p * 3 + 0], py = pos[p * 3 + 1], pz = pos[p * 3 + 2];
        float nx = 0.f, ny = 0.f, nz = 0.f;
        const bool has_n = nrm != nullptr;
        if (has_n) {
            nx = nrm[p * 3 + 0];
            ny = nrm[p * 3 + 1];
            nz = nrm[p * 3 + 2];
        }
        // Step 2: streaming RIS over n_cand uniform candidates of cluster y, target f.
        // Pass 1: S = sum of f (sequential).  Pass 2: the running sum again, up to the pick.
        if constexpr (NC > 0) n_cand = NC;
        constexpr int NR = NC > 0 ? NC : 1;
        int cl_l[NR];
        float cl_f[NR];
        float Ssum = 0.0f, flast = 0.0f;
        int llast = -1;
        uint32_t w4[4];
#pragma unroll
        for (int kk = 0; kk < (NC > 0 ? NC : n_cand); ++kk) {
            if (kk % 4 == 0) philox_words(plo, phi, fr, kTagRisCand + (uint32_t)(kk / 4), k0, k1, w4);
            int l;
            float f;
            ris_candidate(w4, kk, members, o0, m, n_lights, lights, px, py, pz, nx, ny, nz, has_n, l, f);
            if constexpr (NC > 0) {
                cl_l[kk] = l;
                cl_f[kk] = f;
            }
            Ssum = Ssum + f;
            if (f > 0.0f) {
                llast = l;
                flast = f;
            }
        }
        if (Ssum > 0.0f) {
            const uint32_t r2 = philox_first_word(plo, phi, fr, kTagRisSelect, k0, k1);
            const float t2 = ((float)(r2 >> 8) * 0x1.0p-24f) * Ssum;
            float C = 0.0f, fx = 0.0f;
            if constexpr (NC > 0) {
#pragma unroll
                for (int kk = 0; kk < NC; ++kk) {
                    C = C + cl_f[kk];
                    if (pick < 0 && C > t2) {
                        pick = cl_l[kk];
                        fx = cl_f[kk];
                    }
                }
            } else {
                for (int kk = 0; kk < n_cand && pick < 0; ++kk) {
                    if (kk % 4 == 0) philox_words(plo, phi, fr, kTagRisCand + (uint32_t)(kk / 4), k0, k1, w4);
                    int l;
                    float f;
                    ris_candidate(w4, kk, members, o0, m, n_lights, lights, px, py, pz, nx, ny, nz, has_n, l, f);
                    C = C + f;
                    if (C > t2) {
                        pick = l;
                        fx = f;
                    }
                }
            }
            if (pick < 0) {                        // only through rounding
                pick = llast;
                fx = flast;
            }
            cl = y;
            Wx = __fdiv_rn(Ssum * (float)m, ((float)n_cand * P) * fx);
            wsum_r = __fdiv_rn(Ssum * (float)m, P);
        }
    }
    idx_out[p] = pick;
    weight_out[p] = Wx;
    if (cluster_out) cluster_out[p] = cl;
    if (res) res[p] = nvc_reservoir{pick, pick >= 0 ? n_cand : 0, pick >= 0 ? wsum_r : 0.0f, Wx};
}

// ------------------------------------------------------------------ host
// The visibility pointer type of a clustered_sample_kernel instance (its first parameter).
template <typename VT, typename... R>
const VT* kern_vis_type(void (*)(const VT*, R...));

hipError_t launch_clustered_labels(const float* pos, const int32_t* pix, int64_t n, const float* lights, int n_lights,
                                   const int32_t* offsets, const int32_t* members, int k, const float* spheres,
                                   int n_spheres, uint64_t seed, uint32_t frame, const uint32_t* frame_dev,
                                   uint8_t* labels, hipStream_t st) {
    const int64_t total = n * (int64_t)k;
    const int64_t blocks = (total + kClLabelThreads - 1) / kClLabelThreads;
    const size_t smem = (size_t)n_spheres * 16;
    hipLaunchKernelGGL(clustered_labels_kernel, dim3((unsigned)blocks), dim3(kClLabelThreads), smem, st, pos, pix, n,
                       lights, n_lights, offsets, members, k, spheres, n_spheres, (uint32_t)seed,
                       (uint32_t)(seed >> 32), frame, frame_dev, labels);
    return hipGetLastError();
}

hipError_t launch_clustered_sample(const void* vis, int vis_dtype, int64_t n, int k, const float* pos, const float* nrm,
                                   const float* lights, int n_lights, const int32_t* offsets, const int32_t* members,
                                   float vis_floor, int n_cand, uint64_t seed, uint32_t frame,
                                   const uint32_t* frame_dev, int32_t* idx, float* weight, int32_t* cluster,
                                   const uint8_t* mask, nvc_reservoir* res, hipStream_t st) {
    const unsigned blocks = (unsigned)((n + kClSampleThreads - 1) / kClSampleThreads);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    auto go = [&](auto kern, const void* v) {
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(kClSampleThreads), 0, st,
                           reinterpret_cast<decltype(kern_vis_type(kern))>(v), n, k, pos, nrm, lights, n_lights, offsets,
                           members, vis_floor, n_cand, k0, k1, frame, frame_dev, idx, weight, cluster, mask, res);
    };
    const bool c8 = n_cand == 8;
    if (vis_dtype == DT_F32)
        c8 ? go(clustered_sample_kernel<float, 8>, vis) : go(clustered_sample_kernel<float, 0>, vis);
    else if (vis_dtype == DT_F16)
        c8 ? go(clustered_sample_kernel<_Float16, 8>, vis) : go(clustered_sample_kernel<_Float16, 0>, vis);
    else
        c8 ? go(clustered_sample_kernel<__bf16, 8>, vis) : go(clustered_sample_kernel<__bf16, 0>, vis);
    return hipGetLastError();
}

// k-means of the light positions on the host (FP64): farthest-point initial
// centroids, then Lloyd iterations (nearest centroid, ties to the lower
// cluster; non-empty clusters move to the mean of their lights, coordinates
// summed in light order) until no assignment changes or `iters` ran.
void cluster_lights_host(const float* lights, int n, int k, int iters, int32_t* offsets, int32_t* members) {
    std::vector<double> P(3 * (size_t)n);
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) P[3 * (size_t)i + d] = (double)lights[4 * (size_t)i + d];
    auto d2 = [&](int i, const double* c) {
        const double dx = P[3 * (size_t)i] - c[0], dy = P[3 * (size_t)i + 1] - c[1], dz = P[3 * (size_t)i + 2] - c[2];
        return (dx * dx + dy * dy) + dz * dz;
    };
    std::vector<double> cent(3 * (size_t)k);
    std::vector<double> dmin(n);
    for (int d = 0; d < 3; ++d) cent[d] = P[d];
    for (int i = 0; i < n; ++i) dmin[i] = d2(i, &cent[0]);
    for (int j = 1; j < k; ++j) {
        int best = 0;
        for (int i = 1; i < n; ++i)
            if (dmin[i] > dmin[best]) best = i;
        for (int d = 0; d < 3; ++d) cent[3 * (size_t)j + d] = P[3 * (size_t)best + d];
        for (int i = 0; i < n; ++i) dmin[i] = std::min(dmin[i], d2(i, &cent[3 * (size_t)j]));
    }
    std::vector<int> assign(n, -1);
    for (int it = 0; it < iters; ++it) {
        bool changed = false;
        for (int i = 0; i < n; ++i) {
            int best = 0;
            double bd = d2(i, &cent[0]);
            for (int j = 1; j < k; ++j) {
                const double dj = d2(i, &cent[3 * (size_t)j]);
                if (dj < bd) {
                    bd = dj;
                    best = j;
                }
            }
            if (assign[i] != best) changed = true;
            assign[i] = best;
        }
        std::vector<double> sum(3 * (size_t)k, 0.0);
        std::vector<int> cnt(k, 0);
        for (int i = 0; i < n; ++i) {
            for (int d = 0; d < 3; ++d) sum[3 * (size_t)assign[i] + d] += P[3 * (size_t)i + d];
            ++cnt[assign[i]];
        }
        for (int j = 0; j < k; ++j)
            if (cnt[j] > 0)
                for (int d = 0; d < 3; ++d) cent[3 * (size_t)j + d] = sum[3 * (size_t)j + d] / (double)cnt[j];
        if (!changed) break;
    }
    std::vector<int> cnt(k, 0);
    for (int i = 0; i < n; ++i) ++cnt[assign[i]];
    offsets[0] = 0;
    for (int j = 0; j < k; ++j) offsets[j + 1] = offsets[j] + cnt[j];
    std::vector<int> fill(offsets, offsets + k);
    for (int i = 0; i < n; ++i) members[fill[assign[i]]++] = i;
}

}  // namespace nvc
