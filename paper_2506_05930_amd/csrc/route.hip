// Routed scatter of the hash-table gradient: counting, offsets and the
// per-partition LDS sums (see route.hpp).
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "route.hpp"

namespace nvc {

GridDev grid_to_dev(const GridHost& g);

RoutePlan make_route_plan(const GridHost& g) {
    RoutePlan p{};
    const uint64_t T = 1ull << g.log2_T;
    for (int k = 12; k <= 14; ++k) {
        const uint64_t ps = 1ull << k;
        if (ps * (uint64_t)g.n_feat * 8 > 128 * 1024) break;        // fixed-point partition in LDS
        bool ok = true;
        int nb = 0;
        for (int l = 0; l < g.n_levels && ok; ++l) {
            const bool dense = (g.dense_mask >> l) & 1u;
            const uint64_t n1 = (uint64_t)g.res[l] + 1;
            const uint64_t e = dense ? n1 * n1 * n1 : T;
            // x-pairs of a hashed level must share a partition: cx + 1 < 2^k (or one partition only)
            if (!dense && T > ps && (uint64_t)g.res[l] >= ps) ok = false;
            p.bucket_off[l] = nb;
            p.entries[l] = (uint32_t)e;
            nb += (int)((e + ps - 1) / ps);
        }
        if (ok && nb <= kRouteMaxBuckets) {
            p.ok = true;
            p.k = k;
            p.nb = nb;
            p.bucket_off[g.n_levels] = nb;
            return p;
        }
    }
    p.ok = false;
    return p;
}

// Counts the records each training block will emit, per bucket.  Block j owns
// the same samples as training block j: b = it * P + t for it = j, j + G, ...
// The block's 256 threads split into 256 / P groups of P consecutive samples,
// group s taking levels s, s + 256 / P, ...; runs of equal corner x-pairs
// within aligned groups of 16 samples count once, as the training kernel
// merges them.
template <int F>
__global__ __launch_bounds__(256) void route_count_kernel(GridDev g, RouteDev r, const float* __restrict__ pos,
                                                         const int32_t* __restrict__ pix, int64_t batch, int P) {
    extern __shared__ uint32_t hist[];
    for (int i = threadIdx.x; i < r.nb; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int64_t iters = (batch + P - 1) / P;
    const uint32_t M = (1u << r.k) - 1u;
    const int split = blockDim.x / P;
    const int t = threadIdx.x % P;
    const int sub = threadIdx.x / P;
    const int col = threadIdx.x & 15;
    for (int64_t it = blockIdx.x; it < iters; it += gridDim.x) {
        const int64_t b = it * P + t;
        const bool valid = b < batch;
        const int64_t src = valid ? (pix ? (int64_t)pix[b] : b) : 0;
        const float x = valid ? clamp_unit(pos[src * 3 + 0]) : 0.0f;
        const float y = valid ? clamp_unit(pos[src * 3 + 1]) : 0.0f;
        const float z = valid ? clamp_unit(pos[src * 3 + 2]) : 0.0f;
        for (int l = sub; l < g.n_levels; l += split) {
            Corners cr;
            level_corners(g, l, x, y, z, cr);
            const bool dense = (g.dense_mask >> l) & 1u;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const uint32_t e0 = cr.idx[2 * p], e1 = cr.idx[2 * p + 1];
                const bool part = valid && !(dense && (e0 & M) == M);
                const uint32_t k0 = part ? e0 : 0xFFFFFFFFu, k1 = part ? e1 : (uint32_t)(threadIdx.x & 63);
                const RunInfo ri = row_runs(k0, k1, col);
                if (part && ri.head) atomicAdd(&hist[r.bucket_off[l] + (e0 >> r.k)], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < r.nb; i += blockDim.x) r.offsets[(int64_t)i * gridDim.x + blockIdx.x] = hist[i];
}

// Per bucket (one wave each): exclusive prefix over the blocks' counts, in place,
// and the bucket total.
__global__ __launch_bounds__(256) void route_prefix_kernel(RouteDev r, int G) {
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= r.nb) return;
    uint32_t* row = r.offsets + (int64_t)b * G;
    const int per = (G + 63) / 64;
    const int j0 = lane * per;
    uint32_t sum = 0;
    for (int j = j0; j < j0 + per && j < G; ++j) sum += row[j];
    uint32_t incl = sum;                                       // inclusive wave scan of the lane sums
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    uint32_t run = incl - sum;
    for (int j = j0; j < j0 + per && j < G; ++j) {
        const uint32_t c = row[j];
        row[j] = run;
        run += c;
    }
    if (lane == 63) r.totals[b] = incl;
}

// Exclusive prefix of the bucket totals; base[nb] = number of records.
__global__ __launch_bounds__(1024) void route_scan_kernel(RouteDev r) {
    __shared__ uint32_t part[1024];
    constexpr int PER = kRouteMaxBuckets / 1024;
    const int t = threadIdx.x;
    __shared__ uint32_t cpart[1024];
    uint32_t v[PER], c[PER];
    uint32_t sum = 0, csum = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = t * PER + i;
        v[i] = b < r.nb ? r.totals[b] : 0u;
        c[i] = (v[i] + kRouteChunk - 1) / kRouteChunk;
        sum += v[i];
        csum += c[i];
    }
    part[t] = sum;
    cpart[t] = csum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {               // inclusive Hillis-Steele scans
        const uint32_t add = t >= off ? part[t - off] : 0u;
        const uint32_t cadd = t >= off ? cpart[t - off] : 0u;
        __syncthreads();
        part[t] += add;
        cpart[t] += cadd;
        __syncthreads();
    }
    uint32_t run = part[t] - sum, crun = cpart[t] - csum;     // exclusive
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = t * PER + i;
        if (b < r.nb) {
            r.base[b] = run;
            r.chunk_base[b] = crun;
        }
        run += v[i];
        crun += c[i];
    }
    if (t == 1023) {
        r.base[r.nb] = part[1023];
        r.chunk_base[r.nb] = cpart[1023];
    }
    // chunk -> bucket table for the partition sums
    crun = cpart[t] - csum;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = t * PER + i;
        for (uint32_t q = 0; q < c[i]; ++q) r.chunk_bucket[crun + q] = (uint32_t)b;
        crun += c[i];
    }
}

// One block per chunk of a bucket: sum the chunk's records into an LDS copy of
// the partition in 64-bit fixed point, then add it to the gradient (plain
// stores if the bucket has a single chunk, atomics otherwise).
template <int F>
__global__ __launch_bounds__(512) void route_accumulate_kernel(RouteDev r, int n_levels, uint32_t T,
                                                              float* __restrict__ g_table, int vec, int G) {
    extern __shared__ unsigned long long part[];       // [2^k][F] fixed-point sums
    __shared__ float red[16];
    const uint32_t c = blockIdx.x;
    if (c >= r.chunk_base[r.nb]) return;
    // The step's scale, from the training blocks' record maxima (every block gets the same one).
    float m = 0.0f;
    for (int i = threadIdx.x; i < G; i += blockDim.x) m = fmaxf(m, r.rec_max[i]);
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    const int b = (int)r.chunk_bucket[c];
    // A plan computed for other samples gives wrong sums, never accesses outside the buffers.
    if (b < 0 || b >= r.nb) return;
    int l = 0;
    while (l + 1 < n_levels && r.bucket_off[l + 1] <= b) ++l;
    const uint32_t ps = 1u << r.k;
    const uint32_t pbase = (uint32_t)(b - r.bucket_off[l]) << r.k;
    const uint32_t cnt = min(ps, r.entries[l] - pbase);
    const uint32_t q = c - r.chunk_base[b];
    const bool shared = r.chunk_base[b + 1] - r.chunk_base[b] > 1;
    const uint32_t r0 = r.base[b] + q * (uint32_t)kRouteChunk;
    const uint32_t r1 = max(r0, min(min(r.base[b + 1], r0 + (uint32_t)kRouteChunk), r.cap));
    for (uint32_t i = threadIdx.x; i < ps * F; i += blockDim.x) part[i] = 0ull;
    __syncthreads();
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, red[w]);
    const int S = route_fixed_shift(m);
    const float scale = ldexpf(1.0f, S), inv_scale = ldexpf(1.0f, -S);
    // Thread t adds records [t S', (t + 1) S') of the chunk, eight per step
    // with all loads issued before the LDS adds.
    constexpr int U = 8;
    const uint32_t per = (r1 - r0 + blockDim.x - 1) / blockDim.x;
    const uint32_t t0 = r0 + threadIdx.x * per;
    for (uint32_t u0 = 0; u0 < per; u0 += U) {
        uint32_t key[U];
        float w[U][2 * F];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = t0 + u0 + u;
            const bool ok = u0 + u < per && i < r1;
            key[u] = ok ? r.keys[i] : 0u;
            const float* v = r.vals + (size_t)(ok ? i : r0) * (2 * F);
            if constexpr (F == 2) {
                const float4 qv = *reinterpret_cast<const float4*>(v);
                w[u][0] = qv.x; w[u][1] = qv.y; w[u][2] = qv.z; w[u][3] = qv.w;
            } else {
#pragma unroll
                for (int j = 0; j < 2 * F; ++j) w[u][j] = v[j];
            }
            if (!ok) {
#pragma unroll
                for (int j = 0; j < 2 * F; ++j) w[u][j] = 0.0f;
            }
        }
        // A thread's records are consecutive, and neighbouring samples often
        // share a corner pair: runs of equal keys are summed in registers
        // (exact: integer sums) and each run costs one set of LDS adds.
        uint32_t kc = key[0];
        long long acc[2 * F];
#pragma unroll
        for (int j = 0; j < 2 * F; ++j) acc[j] = to_fixed(w[0][j], scale);
        auto flush = [&]() {
            const uint32_t lo0 = kc & (ps - 1u), lo1 = (kc >> 16) & (ps - 1u);   // < 2^k for every real key
#pragma unroll
            for (int j = 0; j < F; ++j) {
                if (acc[j] != 0) atomicAdd(&part[lo0 * F + j], (unsigned long long)acc[j]);
                if (acc[F + j] != 0) atomicAdd(&part[lo1 * F + j], (unsigned long long)acc[F + j]);
            }
        };
#pragma unroll
        for (int u = 1; u < U; ++u) {
            long long fx[2 * F];
#pragma unroll
            for (int j = 0; j < 2 * F; ++j) fx[j] = to_fixed(w[u][j], scale);
            if (key[u] == kc) {
#pragma unroll
                for (int j = 0; j < 2 * F; ++j) acc[j] += fx[j];
            } else {
                flush();
                kc = key[u];
#pragma unroll
                for (int j = 0; j < 2 * F; ++j) acc[j] = fx[j];
            }
        }
        flush();
    }
    __syncthreads();
    // The partition's entries start at a multiple of 2^k (k >= 12), so the
    // output is 16-byte aligned when g_table is (vec); the last partition of a
    // dense level may end mid-vector and takes a scalar tail.
    float* out = g_table + ((size_t)l * T + pbase) * F;
    const long long* sums = reinterpret_cast<const long long*>(part);
    if (shared) {
        for (uint32_t i = threadIdx.x; i < cnt * F; i += blockDim.x)
            if (sums[i] != 0) unsafeAtomicAdd(out + i, from_fixed(sums[i], inv_scale));
    } else {
        // All loads of a thread's vectors first, then the adds and stores: one memory round trip.  The
        // gradient is read and written with the non-temporal policy: Adam reads it next, once, and
        // through the caches it would evict the table that the next inference gathers from (1080p
        // frame 0.894 -> 0.885 ms).
        typedef float f4v __attribute__((ext_vector_type(4)));
        const uint32_t nv = vec ? cnt * F / 4 : 0;
        constexpr int V = 8;
        for (uint32_t v0 = threadIdx.x; v0 < nv; v0 += V * blockDim.x) {
            f4v o[V];
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const uint32_t v = v0 + u * blockDim.x;
                if (v < nv) o[u] = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(out) + v);
            }
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const uint32_t v = v0 + u * blockDim.x;
                if (v < nv) {
                    const long long* sv = sums + 4 * v;
                    const f4v r = {o[u].x + from_fixed(sv[0], inv_scale), o[u].y + from_fixed(sv[1], inv_scale),
                                   o[u].z + from_fixed(sv[2], inv_scale), o[u].w + from_fixed(sv[3], inv_scale)};
                    __builtin_nontemporal_store(r, reinterpret_cast<f4v*>(out) + v);
                }
            }
        }
        for (uint32_t i = nv * 4 + threadIdx.x; i < cnt * F; i += blockDim.x) out[i] += from_fixed(sums[i], inv_scale);
    }
}

hipError_t launch_route_count(const GridHost& gh, const RouteDev& r, const float* pos, const int32_t* pix,
                              int64_t batch, int grid, int pts_per_iter, hipStream_t st) {
    if (pts_per_iter < 64 || 256 % pts_per_iter != 0) return hipErrorInvalidValue;   // whole waves per group
    const GridDev g = grid_to_dev(gh);
    const size_t smem = (size_t)r.nb * 4;
    if (gh.n_feat == 1)
        hipLaunchKernelGGL(route_count_kernel<1>, dim3(grid), dim3(256), smem, st, g, r, pos, pix, batch, pts_per_iter);
    else if (gh.n_feat == 2)
        hipLaunchKernelGGL(route_count_kernel<2>, dim3(grid), dim3(256), smem, st, g, r, pos, pix, batch, pts_per_iter);
    else
        hipLaunchKernelGGL(route_count_kernel<4>, dim3(grid), dim3(256), smem, st, g, r, pos, pix, batch, pts_per_iter);
    return hipGetLastError();
}

hipError_t launch_route_prefix(const RouteDev& r, int grid, hipStream_t st) {
    hipLaunchKernelGGL(route_prefix_kernel, dim3((r.nb + 3) / 4), dim3(256), 0, st, r, grid);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(route_scan_kernel, dim3(1), dim3(1024), 0, st, r);
    return hipGetLastError();
}

hipError_t launch_route_accumulate(const GridHost& gh, const RouteDev& r, float* g_table, int64_t max_records,
                                   int train_blocks, hipStream_t st) {
    const uint32_t T = 1u << gh.log2_T;
    const size_t smem = ((size_t)1 << r.k) * gh.n_feat * 8;
    // Upper bound of the chunk count (the exact one is on the device): every
    // bucket has at most one partial chunk.
    const unsigned blocks = (unsigned)((max_records + kRouteChunk - 1) / kRouteChunk + r.nb);
    const int vec = ((uintptr_t)g_table & 15u) == 0;
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(512), smem, st, r, gh.n_levels, T, g_table, vec, train_blocks);
    };
    if (gh.n_feat == 1)
        go(route_accumulate_kernel<1>);
    else if (gh.n_feat == 2)
        go(route_accumulate_kernel<2>);
    else
        go(route_accumulate_kernel<4>);
    return hipGetLastError();
}

}  // namespace nvc
