// Device-side building blocks shared by the cache's kernels (gfx950 / CDNA4).
//
// Matrix-core tiling.  Every MLP layer is computed transposed, as
//     D[neuron][point] = sum_k W[neuron][k] * H[k][point]
// on 16x16 output tiles (16 neurons x 16 points) with
//   v_mfma_f32_16x16x32_{f16,bf16}  (K = 32 per instruction, 8 K-values per lane)
//   v_mfma_f32_16x16x4_f32          (K = 4, 1 K-value per lane)
// Lane l of a wave64 holds, for operand A, row l%16 and K-slots 8*(l/16)..+7
// (f32: K-slot l/16); for operand B, column l%16 and the same K-slots; for the
// accumulator, column l%16 and rows 4*(l/16)+i, i < 4.
//
// The accumulator of one layer therefore leaves lane l with point l%16 and
// neurons 16*b + 4*g + i (g = l/16) of every 16-neuron block b.  The next
// layer consumes exactly those values as its B operand without any data
// movement, by numbering the K dimension to match:
//   f16/bf16: K-chunk c, lane group g, slot s  ->  neuron 32c + 4g + s        (s < 4)
//                                                  neuron 32c + 16 + 4g + s-4 (s >= 4)
//   f32:      K-chunk c = 4b + i, lane group g  ->  neuron 16b + 4g + i
// The weight fragments (operand A) are packed on the host side with the same
// numbering, so activations stay in registers from the encoding to the
// sigmoid.  The same holds for the backward pass with the transposed weights.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nvc_internal.hpp"

namespace nvc {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// --------------------------------------------------------------- dtypes
template <int DT> struct Mma;

template <> struct Mma<DT_F16> {
    using elem = _Float16;
    using frag = half8_t;
    static constexpr int EPL = 8;      // K values per lane per instruction
    static constexpr int KSTEP = 32;   // K per instruction
    static constexpr int PADK = 32;    // K padding granule (two 16-neuron blocks)
    __device__ static inline float4_t mma(frag a, frag b, float4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    __device__ static inline elem cvt(float x) { return (elem)x; }
};

template <> struct Mma<DT_BF16> {
    using elem = __bf16;
    using frag = bf16x8_t;
    static constexpr int EPL = 8;
    static constexpr int KSTEP = 32;
    static constexpr int PADK = 32;
    __device__ static inline float4_t mma(frag a, frag b, float4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static inline elem cvt(float x) { return (elem)x; }
};

template <> struct Mma<DT_F32> {
    using elem = float;
    using frag = float;
    static constexpr int EPL = 1;
    static constexpr int KSTEP = 4;
    static constexpr int PADK = 16;
    __device__ static inline float4_t mma(frag a, frag b, float4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline elem cvt(float x) { return x; }
};

template <int DT> __device__ inline float to_f32(typename Mma<DT>::elem x) { return (float)x; }

// Number of K-chunks covering NB 16-neuron blocks (NB already padded to PADK/16).
template <int DT> __host__ __device__ constexpr int kchunks(int nb) {
    return DT == DT_F32 ? nb * 4 : nb / 2;
}

// Neuron number of (chunk kc, lane group g, slot s), see the file comment.
template <int DT> __host__ __device__ constexpr int kperm(int kc, int g, int s) {
    return DT == DT_F32 ? 16 * (kc / 4) + 4 * g + (kc % 4)
                        : 32 * kc + (s < 4 ? 4 * g + s : 16 + 4 * g + (s - 4));
}

// B operand for chunk kc from a lane's register activations act[block][i].
template <int DT, int NB>
__device__ inline typename Mma<DT>::frag make_frag(const float (&act)[NB][4], int kc) {
    typename Mma<DT>::frag f;
    if constexpr (DT == DT_F32) {
        f = act[kc / 4][kc % 4];
    } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) f[s] = Mma<DT>::cvt(act[2 * kc + s / 4][s % 4]);
    }
    return f;
}

// A operand fragment (ob, kc) of a packed matrix with KC chunks per row block.
template <int DT>
__device__ inline typename Mma<DT>::frag load_frag(const typename Mma<DT>::elem* base, int ob, int kc, int KC,
                                                   int lane) {
    using M = Mma<DT>;
    const typename M::elem* p = base + ((size_t)(ob * KC + kc) * 64 + lane) * M::EPL;
    return *reinterpret_cast<const typename M::frag*>(p);
}

// --------------------------------------------------------------- Philox4x32-10
// Salmon et al. 2011: ten rounds of two 32x32->64 multiplies; high halves are
// mixed with the other counter words and the round key; Weyl key schedule.
__device__ inline uint32_t philox_first_word(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return c0;
}

// All four output words of the same generator.
__device__ inline void philox_words(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                    uint32_t (&out)[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// --------------------------------------------------------------- hash grid
struct GridDev {
    int32_t n_levels;
    int32_t n_feat;
    uint32_t T;
    uint32_t dense_mask;          // bit l: level l stored densely
    int32_t res[kMaxLevels];      // N_l
};

__device__ inline float clamp_unit(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// Cell, fraction and table indices of the 8 corners of a position at level l.
// Corner k = (k&1, (k>>1)&1, (k>>2)&1).  Decided in FP32: s = fl32(x * N).
struct Corners {
    uint32_t idx[8];
    float w[8];
};

__device__ inline void level_corners(const GridDev& g, int l, float x, float y, float z, Corners& c) {
    const int N = g.res[l];
    const float Nf = (float)N;                          // exact, N < 2^24
    const float sx = x * Nf, sy = y * Nf, sz = z * Nf;
    const int cx = min((int)floorf(sx), N - 1);
    const int cy = min((int)floorf(sy), N - 1);
    const int cz = min((int)floorf(sz), N - 1);
    const float fx = sx - (float)cx, fy = sy - (float)cy, fz = sz - (float)cz;   // exact
    if ((g.dense_mask >> l) & 1u) {
        const uint32_t n1 = (uint32_t)N + 1u;
        const uint32_t b = (uint32_t)cx + n1 * ((uint32_t)cy + n1 * (uint32_t)cz);
        const uint32_t sy1 = n1, sz1 = n1 * n1;
#pragma unroll
        for (int k = 0; k < 8; ++k) c.idx[k] = b + ((k & 1) ? 1u : 0u) + ((k & 2) ? sy1 : 0u) + ((k & 4) ? sz1 : 0u);
    } else {
        const uint32_t mask = g.T - 1u;
        const uint32_t hx0 = (uint32_t)cx, hx1 = (uint32_t)cx + 1u;
        const uint32_t hy0 = (uint32_t)cy * 2654435761u, hy1 = ((uint32_t)cy + 1u) * 2654435761u;
        const uint32_t hz0 = (uint32_t)cz * 805459861u, hz1 = ((uint32_t)cz + 1u) * 805459861u;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            c.idx[k] = (((k & 1) ? hx1 : hx0) ^ ((k & 2) ? hy1 : hy0) ^ ((k & 4) ? hz1 : hz0)) & mask;
    }
    const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
#pragma unroll
    for (int k = 0; k < 8; ++k) c.w[k] = (wx[k & 1] * wy[(k >> 1) & 1]) * wz[(k >> 2) & 1];
}

// F features of level l at a (clamped) position: sum over corners of w * table[l][idx][j].
template <int F>
__device__ inline void encode_level(const float* __restrict__ table, const GridDev& g, int l, float x, float y,
                                    float z, float (&out)[F]) {
    Corners c;
    level_corners(g, l, x, y, z, c);
    const float* base = table + (size_t)l * g.T * F;
#pragma unroll
    for (int j = 0; j < F; ++j) out[j] = 0.0f;
    if constexpr (F == 2) {
        float2 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = *reinterpret_cast<const float2*>(base + (size_t)c.idx[k] * 2);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            out[0] = fmaf(c.w[k], v[k].x, out[0]);
            out[1] = fmaf(c.w[k], v[k].y, out[1]);
        }
    } else if constexpr (F == 4) {
        float4 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = *reinterpret_cast<const float4*>(base + (size_t)c.idx[k] * 4);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            out[0] = fmaf(c.w[k], v[k].x, out[0]);
            out[1] = fmaf(c.w[k], v[k].y, out[1]);
            out[2] = fmaf(c.w[k], v[k].z, out[2]);
            out[3] = fmaf(c.w[k], v[k].w, out[3]);
        }
    } else {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = base[c.idx[k]];
#pragma unroll
        for (int k = 0; k < 8; ++k) out[0] = fmaf(c.w[k], v[k], out[0]);
    }
}

// The encoding features a lane owns in the MLP operand layout: for each input
// 16-block b, features 16b + 4g + i (i < 4) where g = lane/16.  Features past
// n_levels*F are zero.  Result is act[b][i].
template <int F, int NINB>
__device__ inline void encode_lane(const float* __restrict__ table, const GridDev& g, int grp, float x, float y,
                                   float z, float (&act)[NINB][4]) {
    static_assert(F == 1 || F == 2 || F == 4, "features per level");
#pragma unroll
    for (int b = 0; b < NINB; ++b) {
#pragma unroll
        for (int q = 0; q < 4; q += F) {
            const int feat = 16 * b + 4 * grp + q;
            const int l = feat / F;
            float v[F];
            if (l < g.n_levels) {
                encode_level<F>(table, g, l, x, y, z, v);
            } else {
#pragma unroll
                for (int j = 0; j < F; ++j) v[j] = 0.0f;
            }
#pragma unroll
            for (int j = 0; j < F; ++j) {
                asm volatile("" : "+v"(v[j]));      // an FP32 value (see encode_lane_lv)
                act[b][q + j] = v[j];
            }
        }
    }
}

// ------------------------------------------------------------ per-lane levels
// A level as one lane sees it, computed once per kernel (a lane always feeds
// the same levels to the MLP).  The dense and hashed indices share one form:
// with hx = cx + dx, hy = (cy + dy) * my, hz = (cz + dz) * mz,
//   dense:  hx + hy + hz            (my = N + 1, mz = (N + 1)^2)
//   hashed: (hx ^ hy ^ hz) & (T-1)  (my = 2654435761, mz = 805459861)
// so a wave whose lanes mix dense and hashed levels does not branch.
struct LevelLane {
    float Nf;           // N_l
    int nmax;           // N_l - 1
    uint32_t my, mz;
    uint32_t mask;      // T - 1 (hashed)
    uint32_t base;      // first entry of the level: l * T
    bool dense;
    bool valid;         // l < n_levels (else the features are 0)
};

__device__ inline LevelLane level_lane(const GridDev& g, int l) {
    LevelLane v;
    v.valid = l < g.n_levels;
    const int lc = v.valid ? l : 0;
    const int N = g.res[lc];
    v.Nf = (float)N;
    v.nmax = N - 1;
    v.dense = (g.dense_mask >> lc) & 1u;
    const uint32_t n1 = (uint32_t)N + 1u;
    v.my = v.dense ? n1 : 2654435761u;
    v.mz = v.dense ? n1 * n1 : 805459861u;
    v.mask = g.T - 1u;
    v.base = (uint32_t)lc * g.T;
    return v;
}

// Entry indices (level-relative) and fractions of the 8 corners at a level.
__device__ inline void lane_corners(const LevelLane& v, float x, float y, float z, uint32_t (&idx)[8],
                                    float (&f)[3]) {
    const float sx = x * v.Nf, sy = y * v.Nf, sz = z * v.Nf;
    const int cx = min((int)floorf(sx), v.nmax);
    const int cy = min((int)floorf(sy), v.nmax);
    const int cz = min((int)floorf(sz), v.nmax);
    f[0] = sx - (float)cx;
    f[1] = sy - (float)cy;
    f[2] = sz - (float)cz;
    const uint32_t hx[2] = {(uint32_t)cx, (uint32_t)cx + 1u};
    const uint32_t y0 = (uint32_t)cy * v.my, z0 = (uint32_t)cz * v.mz;
    const uint32_t hy[2] = {y0, y0 + v.my}, hz[2] = {z0, z0 + v.mz};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t a = hx[k & 1], b = hy[(k >> 1) & 1], c = hz[k >> 2];
        idx[k] = v.dense ? a + b + c : (a ^ b ^ c) & v.mask;
    }
}

// Trilinear weight of corner k, in the order of level_corners.
__device__ inline float corner_weight(const float (&f)[3], int k) {
    const float wx = (k & 1) ? f[0] : 1.0f - f[0];
    const float wy = (k & 2) ? f[1] : 1.0f - f[1];
    const float wz = (k & 4) ? f[2] : 1.0f - f[2];
    return (wx * wy) * wz;
}

// The lane's encoding features (as encode_lane) from its precomputed levels:
// all corner indices first, then every gather of every level, then the sums,
// so the loads of all levels are in flight together.
template <int F, int NINB>
__device__ inline void encode_lane_lv(const float* __restrict__ table, const LevelLane (&lv)[NINB][4 / F], float x,
                                      float y, float z, float (&act)[NINB][4]) {
    constexpr int NQ = 4 / F;
    uint32_t idx[NINB][NQ][8];
    float fr[NINB][NQ][3];
#pragma unroll
    for (int b = 0; b < NINB; ++b)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            lane_corners(lv[b][q], x, y, z, idx[b][q], fr[b][q]);
#pragma unroll
            for (int k = 0; k < 8; ++k) idx[b][q][k] = lv[b][q].valid ? lv[b][q].base + idx[b][q][k] : 0u;
        }
    float val[NINB][NQ][8][F];
#pragma unroll
    for (int b = 0; b < NINB; ++b)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float* p = table + (size_t)idx[b][q][k] * F;
                if constexpr (F == 2) {
                    const float2 t = *reinterpret_cast<const float2*>(p);
                    val[b][q][k][0] = t.x;
                    val[b][q][k][1] = t.y;
                } else if constexpr (F == 4) {
                    const float4 t = *reinterpret_cast<const float4*>(p);
                    val[b][q][k][0] = t.x;
                    val[b][q][k][1] = t.y;
                    val[b][q][k][2] = t.z;
                    val[b][q][k][3] = t.w;
                } else {
                    val[b][q][k][0] = p[0];
                }
            }
#pragma unroll
    for (int b = 0; b < NINB; ++b)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            float o[F];
#pragma unroll
            for (int j = 0; j < F; ++j) o[j] = 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float w = corner_weight(fr[b][q], k);
#pragma unroll
                for (int j = 0; j < F; ++j) o[j] = fmaf(w, val[b][q][k][j], o[j]);
            }
#pragma unroll
            for (int j = 0; j < F; ++j) {
                // The feature is an FP32 value: the empty asm keeps the compiler from
                // folding the last FMA into the conversion to the matrix-core dtype
                // (v_fma_mix rounds once, straight to FP16).
                asm volatile("" : "+v"(o[j]));
                act[b][q * F + j] = lv[b][q].valid ? o[j] : 0.0f;
            }
        }
}

// The lane's levels: feature 16b + 4*grp + q*F .. belongs to level (16b + 4*grp + q*F) / F.
template <int F, int NINB>
__device__ inline void lane_levels(const GridDev& g, int grp, LevelLane (&lv)[NINB][4 / F]) {
#pragma unroll
    for (int b = 0; b < NINB; ++b)
#pragma unroll
        for (int q = 0; q < 4 / F; ++q) lv[b][q] = level_lane(g, (16 * b + 4 * grp + q * F) / F);
}

// Correctly rounded FP32 square root of a positive normal x.  The hardware
// square root is accurate to 1 ulp but not correctly rounded; with s its
// result and s-, s+ the neighbouring floats, the exact root lies below the
// midpoint of (s-, s) iff x <= s- * s, and above the midpoint of (s, s+) iff
// x > s * s+ (no float lies between those products and the squared
// midpoints), and one fused multiply-add gives each sign exactly.
__device__ inline float sqrt_rn(float x) {
    float s = __builtin_amdgcn_sqrtf(x);
    const float s_dn = __int_as_float(__float_as_int(s) - 1);
    const float s_up = __int_as_float(__float_as_int(s) + 1);
    const bool down = fmaf(-s_dn, s, x) <= 0.0f;
    const bool up = fmaf(-s_up, s, x) > 0.0f;
    return down ? s_dn : (up ? s_up : s);            // selects, no branches
}

// exp(-|z|) with the hardware base-2 exponential (within 1 ulp of exp2 of
// the rounded product; 0 once it underflows).
__device__ inline float exp_neg_abs(float z) { return __builtin_amdgcn_exp2f(-fabsf(z) * 1.44269504088896341f); }

// Logistic function of the FP32 accumulator in the stable form, given
// e = exp(-|z|): 1 / (1 + e) for z >= 0, e / (1 + e) otherwise, with the
// hardware reciprocal (relative error a few 1e-7 for |z| < 16).
__device__ inline float sigmoid_from(float z, float e) {
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    return z >= 0.0f ? r : e * r;
}

__device__ inline float sigmoidf_(float z) { return sigmoid_from(z, exp_neg_abs(z)); }

// 1 / (1 + exp(-z)) from the hardware exp2 and reciprocal without the stable
// split: exp2 overflows to +inf for very negative z and the reciprocal gives
// 0; relative error a few 1e-7 (as sigmoidf_ for |z| < 16).
__device__ inline float sigmoid_fast(float z) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z * -1.44269504088896341f));
}

// --------------------------------------------------------------- lights
// Unshadowed weight f and light weight w = f * max(v, floor) of light l at p (order as in nvc.h).
__device__ inline void wrs_weight(const float4& l, float px, float py, float pz, float nx, float ny, float nz,
                                  bool has_n, float v, float vis_floor, float& f, float& w) {
    const float dx = l.x - px, dy = l.y - py, dz = l.z - pz;
    const float d2 = fmaxf((dx * dx + dy * dy) + dz * dz, 1e-6f);
    if (has_n) {
        const float nd = (nx * dx + ny * dy) + nz * dz;
        // max(nd, 0) = 0 (nd <= 0, or NaN): the denominator is positive (d2 >= 1e-6), so the quotient is
        // the numerator l.w * 0 itself (a zero, or NaN for a non-finite intensity), and the division and
        // the root are skipped; a wave skips them whenever none of its pixels faces the light.  (The sign
        // of such a zero never reaches an output: the sums start at +0 and a picked light has w > 0.)
        if (nd > 0.0f)
            f = __fdiv_rn(l.w * nd, d2 * sqrt_rn(d2));
        else
            f = l.w * 0.0f;
    } else {
        f = __fdiv_rn(l.w, d2);
    }
    w = f * (v >= vis_floor ? v : vis_floor);           // max(v, floor), a NaN v taken as the floor
}

}  // namespace nvc
