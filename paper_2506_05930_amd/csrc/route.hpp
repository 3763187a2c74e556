// Routed scatter of the hash-table gradient.
//
// Global FP32 atomics on gfx950 are limited by the number of distinct cache
// lines per instruction, and the table gradient receives ~64 random updates
// per training sample (2^18 samples x 16 levels x 8 corners x 2 features), so
// scattering it with per-lane atomics is slow.  Instead every update is routed
// to the 4096-entry (2^k) partition of the table it falls in and summed there
// in LDS by the block that owns the partition:
//
//   count     for the samples each training block will own, count the records
//             per partition ("bucket")                        route_count_kernel
//   prefix    per bucket, an exclusive prefix over the blocks' counts gives
//             every block a private write range              route_prefix_kernel
//   scan      exclusive prefix of the bucket totals           route_scan_kernel
//   emit      the training kernel writes one record per corner x-pair
//             (the corners at dx = 0 and dx = 1 of one (dy, dz)) into its range
//   sum       one block per chunk of up to kRouteChunk records of a bucket sums
//             them in an LDS copy of the partition and adds it to the gradient:
//             plain coalesced stores when the bucket has one chunk, line-coalesced
//             atomics when several blocks share it      route_accumulate_kernel
//
// The LDS sums are exact 64-bit fixed point: FP32 atomic adds on LDS cost
// about 40 times as much as 64-bit integer ones on gfx950 (measured ~190 vs
// ~9 cycles per wave instruction).  The training blocks report the largest
// record magnitude; with it one power-of-two scale per step is chosen so that
// no partition sum of a chunk can overflow (a chunk adds at most 2 * 16384
// values to an entry) while a record is resolved to 2^-45 of the largest one.
// The sums are then independent of the order of the additions.
//
// A record carries both entries of an x-pair.  On a hashed level the low 12
// (k) bits of the hash are the only ones the x coordinate reaches when
// N < 2^k, so both entries always share a partition.  On a dense level the
// pair (e, e+1) straddles a partition boundary when e is the partition's last
// entry; those pairs (1 in 2^k) are added with direct atomics by the training
// kernel, which runs before the partition sums.
#pragma once

#include <stdint.h>

#include "nvc_internal.hpp"

namespace nvc {

constexpr int kRouteMaxBuckets = 8192;
constexpr int kRouteChunk = 16384;        // records summed by one block

struct RouteDev {
    int32_t enabled;
    int32_t k;                                // partition = 2^k entries
    int32_t nb;                               // buckets over all levels
    int32_t bucket_off[kMaxLevels + 1];       // first bucket of each level
    uint32_t entries[kMaxLevels];             // entries a level uses: (N+1)^3 dense, T hashed
    uint32_t* offsets;                        // [nb][G]: counts, then each block's offset within the bucket
    uint32_t* totals;                         // [nb]
    uint32_t* base;                           // [nb + 1]: first record of each bucket
    uint32_t* chunk_base;                     // [nb + 1]: first chunk (of kRouteChunk records) of each bucket
    uint32_t* chunk_bucket;                   // [max chunks]: bucket of every chunk
    float* vals;                              // [R][2F]: values of entry e0, then of e1
    uint32_t* keys;                           // [R]: (e0 & M) | (e1 & M) << 16, M = 2^k - 1
    float* rec_max;                           // [G]: largest |value| each training block wrote
    uint32_t cap;                             // records the buffers hold (batch * n_levels * 4)
};

// Fixed-point scale 2^S for the partition sums, from the largest record
// magnitude m: S = 45 - E with m < 2^(E + 1), so that 2 * kRouteChunk * m * 2^S
// < 2^62; clamped to the FP32 exponent range.  m = 0 (or not finite) gives 1.
__host__ __device__ inline int route_fixed_shift(float m) {
    const uint32_t bits = __builtin_bit_cast(uint32_t, m);
    const int biased = (int)((bits >> 23) & 0xFFu);
    if (!(m > 0.0f) || biased == 0xFF) return 0;
    const int E = biased == 0 ? -127 : biased - 127;
    int S = 45 - E;
    if (S > 126) S = 126;
    if (S < -126) S = -126;
    return S;
}

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)
// x = v * 2^S (exact: a power-of-two scaling) rounded to the nearest integer,
// for |x| < 2^54: the part above 2^24 is taken exactly by truncation, the
// rest (|r| < 2^24) is rounded to an integer.  With the scale above every
// record has |x| < 2^46.
__device__ inline long long to_fixed(float v, float scale) {
    const float x = v * scale;
    const float hi = truncf(x * 0x1.0p-24f);
    const float r = x - hi * 0x1.0p24f;               // exact
    return (long long)(int)hi * (1ll << 24) + (long long)(int)rintf(r);
}

// a * 2^-S as FP32 (two roundings: within one ulp).
__device__ inline float from_fixed(long long a, float inv_scale) {
    const int hi = (int)(a >> 32);
    const uint32_t lo = (uint32_t)a;
    return ((float)hi * 0x1.0p32f + (float)lo) * inv_scale;
}

// Row shifts within the 16-lane rows of a wave (DPP): lane i reads lane i + D
// (row_shl) or lane i - D (row_shr) of its own row; reads past the row's ends
// return 0 and are masked by the callers.
template <int D> __device__ inline uint32_t row_from_next(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x100 + D, 0xF, 0xF, true);
}
template <int D> __device__ inline float row_from_next(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x100 + D, 0xF, 0xF, true));
}
__device__ inline uint32_t row_from_prev1(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x110 + 1, 0xF, 0xF, true);
}

// Runs of equal keys among the 16 lanes of a row (lanes 16r .. 16r+15 hold 16
// consecutive samples): `head` marks the first lane of a run, `last` the last.
struct RunInfo {
    bool head;
    bool last;
};

__device__ inline RunInfo row_runs(uint32_t k0, uint32_t k1, int col) {
    const uint32_t p0 = row_from_prev1(k0), p1 = row_from_prev1(k1);
    const uint32_t n0 = row_from_next<1>(k0), n1 = row_from_next<1>(k1);
    RunInfo r;
    r.head = col == 0 || p0 != k0 || p1 != k1;
    r.last = col == 15 || n0 != k0 || n1 != k1;
    return r;
}

// Reverse segmented sum within the row: afterwards each lane holds the sum of
// its own value and those of the later lanes of its run (the head: the run).
template <int D, int NV>
__device__ inline void row_run_step(float (&v)[NV], uint32_t& e, int col) {
    float o[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) o[j] = row_from_next<D>(v[j]);
    const uint32_t eo = col + D < 16 ? row_from_next<D>(e) : 1u;
    if (!e) {                                  // e == 0 implies col + D < 16 for the lanes that add
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] += o[j];
    }
    e |= eo;
}

template <int NV>
__device__ inline void row_run_sums(float (&v)[NV], bool last, int col) {
    uint32_t e = last ? 1u : 0u;
    row_run_step<1>(v, e, col);
    row_run_step<2>(v, e, col);
    row_run_step<4>(v, e, col);
    row_run_step<8>(v, e, col);
}
#endif

// Host-side plan: partition size, bucket numbering, whether routing applies.
struct RoutePlan {
    bool ok;
    int k;
    int nb;
    int bucket_off[kMaxLevels + 1];
    uint32_t entries[kMaxLevels];
};

RoutePlan make_route_plan(const GridHost& g);

hipError_t launch_route_count(const GridHost& g, const RouteDev& r, const float* pos, const int32_t* pix,
                              int64_t batch, int grid, int pts_per_iter, hipStream_t st);
hipError_t launch_route_prefix(const RouteDev& r, int grid, hipStream_t st);
hipError_t launch_route_accumulate(const GridHost& g, const RouteDev& r, float* g_table, int64_t max_records,
                                   int train_blocks, hipStream_t st);

}  // namespace nvc
