// One training pass of the cache (Sec. 3.3-3.4): recompute the encoding and the
// forward pass per tile (nothing is stored to memory), take the loss gradient
// at the sigmoid output, backpropagate on the matrix cores, accumulate the
// weight gradient across the block, and scatter the encoding gradient into
// the hash table with FP32 atomics.
//
// Block = 4 waves, one 16-sample tile per wave and iteration (64 samples).
// The forward pass keeps only the current layer in registers and writes every
// layer input h_k (in the matrix-core dtype) to LDS as [neuron][sample].  For
// each layer k, from the output down:
//   1. every wave writes its delta_k to the LDS delta buffer;
//   2. every wave computes delta_{k-1} = W_k^T delta_k * act'(h_k) in registers
//      (the transposed weight fragments make it a plain matrix-core product;
//      the mask reads the wave's own columns of h_k);
//   3. after a barrier, each wave adds its share of the 16x16 tiles of
//      dW_k = delta_k h_k^T over the block's samples into accumulators that
//      live for the whole kernel;
//   4. barrier.
// At the end each block writes its partial dW to the workspace and a second
// kernel reduces the partials (deterministic; no weight atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device_common.hpp"
#include "kernel_config.hpp"
#include "route.hpp"

namespace nvc {

GridDev grid_to_dev(const GridHost& g);

template <int B, int E, class F>
__device__ inline void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr int kTrainWaves = 4;
constexpr int kTrainPts = 16 * kTrainWaves;   // samples per block iteration: one 16-point tile per wave

struct TrainArgs {
    GridDev g;
    const float* table;
    const void* packed;
    int64_t off_f[kMaxLayers];
    int64_t off_b[kMaxLayers];
    int64_t w_off[kMaxLayers];
    int lin[kMaxLayers];
    int lout[kMaxLayers];
    const float* pos;
    const int32_t* pix;
    int64_t batch;
    int n_out;
    const uint8_t* labels;
    const float* dvis;
    int loss;             // 0 bce, 1 l2
    float out_mul;        // multiplies the output gradient before the low-precision backward
    float final_mul;      // multiplies every gradient written out
    float* g_table;
    float* ws_w;          // [gridDim.x][n_w]
    float* ws_loss;       // [gridDim.x]
    int64_t n_w;
    int act;
    float slope;
    RouteDev route;       // routed table scatter (route.enabled == 0: direct atomics)
    // shadow labels computed in the kernel (SHADOW instantiations): scene-space positions (indexed like
    // pos), lights [n_lights][4] (one network output per light), spheres [n_spheres][4] (c, r);
    // labels_out [batch][n_out] receives them if not NULL
    const float* pos_scene;
    const float* lights;
    int n_lights;
    const float* spheres;
    int n_spheres;
    uint8_t* labels_out;
};

// Largest sphere count and light count of the in-kernel shadow labels (LDS: 24 B per sphere, 16 B per light).
constexpr int kShadowMaxSpheres = NVC_TRAIN_SHADOW_MAX_SPHERES;
constexpr int kShadowMaxLights = NVC_TRAIN_SHADOW_MAX_LIGHTS;

__host__ __device__ constexpr size_t shadow_smem_bytes(int n_spheres) {
    return (size_t)n_spheres * 24 + (size_t)kShadowMaxLights * 16 + 16;
}

// LDS of one block, in the matrix-core dtype, [neuron][sample] with row stride
// SD: the inputs h_0 .. h_{NL-1} of every layer (written by the forward pass,
// read by the backward pass for the activation masks and the weight
// gradients), then one delta buffer.
template <class C>
struct TrainShape {
    static constexpr int DT = C::DT;
    static constexpr int NL = C::NHID + 1;
    static constexpr int PADB = DT == DT_F32 ? 1 : 2;      // K granule in 16-blocks
    static constexpr int NOUTB_K = (C::NOUTB + PADB - 1) / PADB * PADB;
    __host__ __device__ static constexpr int nbi(int k) { return k == 0 ? C::NINB : C::WB; }
    __host__ __device__ static constexpr int nbo(int k) { return k == NL - 1 ? C::NOUTB : C::WB; }
    __host__ __device__ static constexpr int tiles(int k) { return nbi(k) * nbo(k); }
    __host__ __device__ static constexpr int owned(int k) { return (tiles(k) + kTrainWaves - 1) / kTrainWaves; }
    __host__ __device__ static constexpr int acc_off(int k) {
        int o = 0;
        for (int j = 0; j < k; ++j) o += owned(j);
        return o;
    }
    __host__ __device__ static constexpr int hrow(int k) { return k == 0 ? 0 : 16 * C::NINB + 16 * C::WB * (k - 1); }
    static constexpr int ACC = acc_off(NL);
    static constexpr int RH = hrow(NL);
    static constexpr int RD = 16 * (C::WB > NOUTB_K ? C::WB : NOUTB_K);
    static constexpr int PAD = DT == DT_F32 ? 4 : 8;
    static constexpr int SD = kTrainPts + PAD;              // row stride (elements)
    static constexpr int ELEM = DT == DT_F32 ? 4 : 2;
    static constexpr size_t SMEM = (size_t)(RH + RD) * SD * ELEM;
};

// Shapes whose weight-gradient accumulators fit the register file (at most 56
// owned 16x16 tiles per wave: the 128-wide network, one wave per SIMD) and
// whose activations fit the LDS get a training kernel.  The routed scatter's
// cursors take 4 bytes per bucket on top; when they do not fit in the 160 KiB
// of LDS the table gradient goes through direct atomics.
template <class C> constexpr bool train_built() {
    return TrainShape<C>::ACC <= 56 && TrainShape<C>::SMEM <= 150 * 1024;
}

// delta_{k-1} (or d_enc) = W^T delta, with W^T fragments (rows = input neurons, K = output neurons).
template <int DT, int NBK, int NBI>
__device__ inline void back_layer(const typename Mma<DT>::elem* WT, int lane, const float (&d)[NBK][4],
                                  float (&out)[NBI][4]) {
    using M = Mma<DT>;
    constexpr int KC = kchunks<DT>(NBK);
#pragma unroll
    for (int ib = 0; ib < NBI; ++ib) {
        float4_t acc = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) acc = M::mma(load_frag<DT>(WT, ib, kc, KC, lane), make_frag<DT, NBK>(d, kc), acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) out[ib][i] = acc[i];
    }
}

template <int DT, int NBI, int NBO>
__device__ inline void fwd_layer(const typename Mma<DT>::elem* W, int lane, const float (&in)[NBI][4],
                                 float (&out)[NBO][4]) {
    using M = Mma<DT>;
    constexpr int KC = kchunks<DT>(NBI);
#pragma unroll
    for (int ob = 0; ob < NBO; ++ob) {
        float4_t acc = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) acc = M::mma(load_frag<DT>(W, ob, kc, KC, lane), make_frag<DT, NBI>(in, kc), acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) out[ob][i] = acc[i];
    }
}

// Round a register tile to the matrix-core dtype (what the MFMA consumed), so
// staging and masks see the same values as the products.
template <int DT, int NB>
__device__ inline void round_to_dtype(float (&a)[NB][4]) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) a[b][i] = (float)Mma<DT>::cvt(a[b][i]);
}

// The wave's 16 columns of a [neuron][sample] LDS region.
template <int DT, int NB, int SD>
__device__ inline void stage(typename Mma<DT>::elem* buf, int wave, int lane, const float (&a)[NB][4]) {
    const int grp = lane >> 4, col = lane & 15;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) buf[(16 * b + 4 * grp + i) * SD + wave * 16 + col] = Mma<DT>::cvt(a[b][i]);
}

// acc[j] += tile (ob, ib) of delta h^T over the block's samples, for the wave's owned tiles.
template <int DT, int NBI, int NBO, int OWN, int OFF, int ACC, int SD>
__device__ inline void accumulate_dw(const typename Mma<DT>::elem* D, const typename Mma<DT>::elem* H, int wave,
                                     int lane, float4_t (&acc)[ACC]) {
    using M = Mma<DT>;
    using E = typename M::elem;
    const int grp = lane >> 4, col = lane & 15;
#pragma unroll
    for (int j = 0; j < OWN; ++j) {
        const int t = j * kTrainWaves + wave;
        if (t >= NBI * NBO) break;
        const int ob = t / NBI, ib = t % NBI;
        const E* arow = D + (16 * ob + col) * SD;
        const E* brow = H + (16 * ib + col) * SD;
        float4_t c = acc[OFF + j];
        if constexpr (DT == DT_F32) {
#pragma unroll
            for (int kc = 0; kc < kTrainPts / 4; ++kc) c = M::mma(arow[4 * kc + grp], brow[4 * kc + grp], c);
        } else {
#pragma unroll
            for (int kc = 0; kc < kTrainPts / 32; ++kc) {
                const typename M::frag a = *reinterpret_cast<const typename M::frag*>(arow + 32 * kc + 8 * grp);
                const typename M::frag b = *reinterpret_cast<const typename M::frag*>(brow + 32 * kc + 8 * grp);
                c = M::mma(a, b, c);
            }
        }
        acc[OFF + j] = c;
    }
}

// Shadow labels of the wave's 16 samples for the lane's lights 16 ob + 4 grp + i (ob < NOB, i < 4),
// decided in FP32 exactly as by the separate label kernel (the operation order of nvc.h):
// returns bit 4 ob + i set iff that light is visible from the lane's sample.  The spheres are
// culled against the bundle of the 16 segments to each light (a conservative capsule test, margin
// 1e-3 (1 + scene scale)); a sphere that survives for some light of some lane is tested exactly by
// every lane for each of its lights that it may reach.
template <int NOB>
__device__ inline uint32_t shadow_bits(const TrainArgs& a, const float4* __restrict__ SL, const float4* __restrict__ SS,
                                       const float* __restrict__ SR, const uint32_t* __restrict__ SIN, float scene_scale,
                                       int lane, int grp, float px, float py, float pz) {
    const int m = a.n_lights, ns = a.n_spheres;
    // bundle of the wave's 16 samples (every 16-lane row holds the same ones)
    float mn[3] = {px, py, pz}, mx[3] = {px, py, pz};
#pragma unroll
    for (int off = 1; off < 16; off <<= 1)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            mn[k] = fminf(mn[k], __shfl_xor(mn[k], off));
            mx[k] = fmaxf(mx[k], __shfl_xor(mx[k], off));
        }
    const float cx = 0.5f * (mn[0] + mx[0]), cy = 0.5f * (mn[1] + mx[1]), cz = 0.5f * (mn[2] + mx[2]);
    const float hx = 0.5f * (mx[0] - mn[0]), hy = 0.5f * (mx[1] - mn[1]), hz = 0.5f * (mx[2] - mn[2]);
    const float rho = sqrtf(hx * hx + hy * hy + hz * hz) * 1.0001f;
    const float scale = fmaxf(scene_scale, fmaxf(fabsf(cx), fmaxf(fabsf(cy), fabsf(cz))) + rho);
    const float margin = 1e-3f * (1.0f + scale);
    const bool cull_ok = isfinite(rho) && isfinite(cx) && isfinite(cy) && isfinite(cz) && isfinite(margin);
    // the lane's segments: light li = 16 ob + 4 grp + i
    float dx[NOB][4], dy[NOB][4], dz[NOB][4], dd[NOB][4];
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int li = min(16 * ob + 4 * grp + i, m - 1);
            const float4 l = SL[li];
            dx[ob][i] = l.x - px;
            dy[ob][i] = l.y - py;
            dz[ob][i] = l.z - pz;
            dd[ob][i] = (dx[ob][i] * dx[ob][i] + dy[ob][i] * dy[ob][i]) + dz[ob][i] * dz[ob][i];
        }
    uint32_t occ = 0;
    for (int c0 = 0; c0 < ns; c0 += 64) {
        // cull: lane j takes sphere c0 + j against every light's bundle capsule
        const int s = c0 + lane;
        const bool in_range = s < ns;
        const float4 sc = in_range ? SS[s] : make_float4(0.f, 0.f, 0.f, 0.f);
        const uint32_t s_in = in_range ? SIN[s] : 0u;
        uint32_t lmask = 0;
        if (in_range) {
            if (!cull_ok) {
                lmask = m >= 32 ? 0xFFFFFFFFu : ((1u << m) - 1u);
            } else {
                const float ox = sc.x - cx, oy = sc.y - cy, oz = sc.z - cz;
                const float lim = SR[s] + rho + margin;
                const float lim2 = lim * lim;
                for (int l = 0; l < m; ++l) {
                    const float4 L = SL[l];
                    const float gx = L.x - cx, gy = L.y - cy, gz = L.z - cz;
                    const float gg = gx * gx + gy * gy + gz * gz;
                    const float ginv = gg > 0.0f ? 1.0f / gg : 0.0f;
                    const float t = fminf(fmaxf((ox * gx + oy * gy + oz * gz) * ginv, 0.0f), 1.0f);
                    const float qx = ox - t * gx, qy = oy - t * gy, qz = oz - t * gz;
                    if (qx * qx + qy * qy + qz * qz <= lim2) lmask |= 1u << l;
                }
            }
        }
        uint64_t surv = __ballot(lmask != 0u);
        while (surv) {
            const int j = __builtin_ctzll(surv);
            surv &= surv - 1;
            const uint32_t ls = (uint32_t)__builtin_amdgcn_readlane((int)lmask, j);
            const float sx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sc.x), j));
            const float sy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sc.y), j));
            const float sz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sc.z), j));
            const float sw = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sc.w), j));
            const uint32_t ib = (uint32_t)__builtin_amdgcn_readlane((int)s_in, j);
            const float ox = sx - px, oy = sy - py, oz = sz - pz;
            const float cc = ((ox * ox + oy * oy) + oz * oz) - sw;
#pragma unroll
            for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // lights 16 ob + 4 g + i of the four lane groups g
                    const uint32_t slot_lights = (0x1111u << (16 * ob + i)) & 0xFFFFFFFFu;
                    if (!(ls & slot_lights)) continue;
                    const float bb = (ox * dx[ob][i] + oy * dy[ob][i]) + oz * dz[ob][i];
                    const uint32_t near_p = bb <= 0.0f;
                    const uint32_t near_l = (bb >= dd[ob][i]) & ~near_p;
                    const uint32_t mid = ~(near_p | near_l) & 1u;
                    const int li = 16 * ob + 4 * grp + i;
                    const uint32_t o = (near_p & (uint32_t)(cc < 0.0f)) | (near_l & (ib >> (li & 31))) |
                                       (mid & (uint32_t)(cc * dd[ob][i] < bb * bb));
                    occ |= (o & 1u) << (4 * ob + i);
                }
        }
    }
    return ~occ & ((1u << (4 * NOB)) - 1u);
}

// The in-kernel labels hold the lane's light segments across the sphere loop; the register budget of two
// waves per SIMD keeps the occupancy of the plain kernel.
template <class C, bool SHADOW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SHADOW ? 2 : 1))) void train_kernel(TrainArgs a) {
    constexpr int DT = C::DT;
    using M = Mma<DT>;
    using E = typename M::elem;
    using TS = TrainShape<C>;
    constexpr int NL = TS::NL;
    constexpr int SD = TS::SD;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    E* stH = reinterpret_cast<E*>(smem_raw);
    E* stD = stH + TS::RH * SD;
    __shared__ float red[kTrainWaves];
    __shared__ float red_max[kTrainWaves];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int grp = lane >> 4;
    const int col = lane & 15;
    const E* packed0 = reinterpret_cast<const E*>(a.packed);

    // Write cursors of the routed scatter: the next free record of this block in every bucket.
    uint32_t* cursor = reinterpret_cast<uint32_t*>(smem_raw + TS::SMEM);
    if (a.route.enabled) {
        for (int i = threadIdx.x; i < a.route.nb; i += blockDim.x)
            cursor[i] = a.route.base[i] + a.route.offsets[(int64_t)i * gridDim.x + blockIdx.x];
        __syncthreads();
    }
    // In-kernel shadow labels: lights, spheres (c, r^2), radii and light-inside bits in LDS after the cursors.
    float4* SL = nullptr;
    float4* SS = nullptr;
    float* SR = nullptr;
    uint32_t* SIN = nullptr;
    float scene_scale = 0.0f;
    if constexpr (SHADOW) {
        const size_t off = (TS::SMEM + (a.route.enabled ? (size_t)a.route.nb * 4 : 0) + 15) / 16 * 16;
        SL = reinterpret_cast<float4*>(smem_raw + off);
        SS = SL + kShadowMaxLights;
        SR = reinterpret_cast<float*>(SS + a.n_spheres);
        SIN = reinterpret_cast<uint32_t*>(SR + a.n_spheres);
        uint32_t* scale_bits = SIN + a.n_spheres;
        if (threadIdx.x == 0) *scale_bits = 0u;
        __syncthreads();
        uint32_t my_scale = 0;
        for (int j = threadIdx.x; j < a.n_lights; j += blockDim.x) {
            const float lx = a.lights[4 * j + 0], ly = a.lights[4 * j + 1], lz = a.lights[4 * j + 2];
            SL[j] = make_float4(lx, ly, lz, 0.0f);
            my_scale = max(my_scale, __float_as_uint(fmaxf(fabsf(lx), fmaxf(fabsf(ly), fabsf(lz)))));
        }
        for (int q = threadIdx.x; q < a.n_spheres; q += blockDim.x) {
            const float cx = a.spheres[4 * q + 0], cy = a.spheres[4 * q + 1], cz = a.spheres[4 * q + 2];
            const float r = a.spheres[4 * q + 3];
            const float rr = r * r;
            SS[q] = make_float4(cx, cy, cz, rr);
            SR[q] = r;
            my_scale = max(my_scale, __float_as_uint(fmaxf(fabsf(cx), fmaxf(fabsf(cy), fabsf(cz))) + fabsf(r)));
            uint32_t bits = 0;
            for (int j = 0; j < a.n_lights; ++j) {
                const float ex = cx - a.lights[4 * j + 0], ey = cy - a.lights[4 * j + 1], ez = cz - a.lights[4 * j + 2];
                if (((ex * ex + ey * ey) + ez * ez) < rr) bits |= 1u << j;
            }
            SIN[q] = bits;
        }
        atomicMax(scale_bits, my_scale);
        __syncthreads();
        scene_scale = __uint_as_float(*scale_bits);
    }

    float4_t acc[TS::ACC];
#pragma unroll
    for (int j = 0; j < TS::ACC; ++j) acc[j] = float4_t{0.f, 0.f, 0.f, 0.f};
    float loss_acc = 0.0f;
    float rec_max = 0.0f;          // largest |value| this thread wrote into a record

    const int64_t iters = (a.batch + kTrainPts - 1) / kTrainPts;
    for (int64_t it = blockIdx.x; it < iters; it += gridDim.x) {
        // ---------------- forward (recomputed); layer inputs go to LDS ----------------
        // The weight fragments are loaded where they are used (from L1/L2) in
        // every iteration: the empty asm stops the compiler from hoisting them
        // out of the loop into registers, which would cost occupancy.
        const E* packed = packed0;
        asm volatile("" : "+s"(packed));
        const int64_t b = it * kTrainPts + wave * 16 + col;
        const bool valid = b < a.batch;
        const int64_t bc = valid ? b : a.batch - 1;
        const int64_t src = a.pix ? (int64_t)a.pix[bc] : bc;
        const float x0 = clamp_unit(a.pos[src * 3 + 0]);
        const float x1 = clamp_unit(a.pos[src * 3 + 1]);
        const float x2 = clamp_unit(a.pos[src * 3 + 2]);
        uint32_t shadow = 0;            // bit 4 ob + i: light 16 ob + 4 grp + i is visible (SHADOW)
        if constexpr (SHADOW) {
            shadow = shadow_bits<C::NOUTB>(a, SL, SS, SR, SIN, scene_scale, lane, grp, a.pos_scene[src * 3 + 0],
                                           a.pos_scene[src * 3 + 1], a.pos_scene[src * 3 + 2]);
            if (a.labels_out && valid) {
                // lights 16 ob + 4 grp .. + 3 of this lane: one 4-byte store when the row keeps them aligned
#pragma unroll
                for (int ob = 0; ob < C::NOUTB; ++ob) {
                    const int l0 = 16 * ob + 4 * grp;
                    uint8_t* out = a.labels_out + b * a.n_out + l0;
                    const uint32_t nib = (shadow >> (4 * ob)) & 0xFu;
                    if ((a.n_out & 3) == 0 && ((uintptr_t)a.labels_out & 3u) == 0 && l0 < a.n_out) {
                        const uint32_t word = (nib & 1u) | ((nib >> 1) & 1u) << 8 | ((nib >> 2) & 1u) << 16 |
                                              ((nib >> 3) & 1u) << 24;
                        *reinterpret_cast<uint32_t*>(out) = word;
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (l0 + i < a.n_out) out[i] = (uint8_t)((nib >> i) & 1u);
                    }
                }
            }
        }
        float z[TS::NOUTB_K][4];
        {
            float h0[C::NINB][4];
            encode_lane<C::F, C::NINB>(a.table, a.g, grp, x0, x1, x2, h0);
            round_to_dtype<DT, C::NINB>(h0);
            stage<DT, C::NINB, SD>(stH, wave, lane, h0);
            float h[C::WB][4];
            fwd_layer<DT, C::NINB, C::WB>(packed + a.off_f[0], lane, h0, h);
            static_for<1, NL>([&](auto kc_) {
                constexpr int k = decltype(kc_)::value;      // h = pre-activation input of layer k
#pragma unroll
                for (int ob = 0; ob < C::WB; ++ob)
#pragma unroll
                    for (int i = 0; i < 4; ++i) h[ob][i] = fmaxf(h[ob][i], a.slope * h[ob][i]);   // 0 <= slope <= 1
                round_to_dtype<DT, C::WB>(h);
                stage<DT, C::WB, SD>(stH + TS::hrow(k) * SD, wave, lane, h);
                if constexpr (k < NL - 1) {
                    float hn[C::WB][4];
                    fwd_layer<DT, C::WB, C::WB>(packed + a.off_f[k], lane, h, hn);
#pragma unroll
                    for (int ob = 0; ob < C::WB; ++ob)
#pragma unroll
                        for (int i = 0; i < 4; ++i) h[ob][i] = hn[ob][i];
                } else {
                    float zz[C::NOUTB][4];
                    fwd_layer<DT, C::WB, C::NOUTB>(packed + a.off_f[k], lane, h, zz);
#pragma unroll
                    for (int ob = 0; ob < TS::NOUTB_K; ++ob)
#pragma unroll
                        for (int i = 0; i < 4; ++i) z[ob][i] = ob < C::NOUTB ? zz[ob][i] : 0.0f;
                }
            });
        }

        // ---------------- output gradient and loss ----------------
        float d[TS::NOUTB_K][4];
#pragma unroll
        for (int ob = 0; ob < TS::NOUTB_K; ++ob)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int li = 16 * ob + 4 * grp + i;
                float g = 0.0f;
                if (valid && li < a.n_out) {
                    const float zv = z[ob][i];
                    const float e = exp_neg_abs(zv);
                    const float v = sigmoid_from(zv, e);
                    if (SHADOW || a.labels) {
                        float y;
                        if constexpr (SHADOW)
                            y = (float)((shadow >> (4 * ob + i)) & 1u);
                        else
                            y = (float)a.labels[b * a.n_out + li];
                        if (a.loss == 0) {
                            g = v - y;
                            loss_acc += fmaxf(zv, 0.0f) + log1pf(e) - y * zv;
                        } else {
                            g = 2.0f * (v - y) * v * (1.0f - v);
                            loss_acc += (v - y) * (v - y);
                        }
                    } else {
                        g = a.dvis[b * a.n_out + li] * v * (1.0f - v);
                    }
                    g *= a.out_mul;
                }
                d[ob][i] = g;
            }

        // ---------------- backward, output layer first ----------------
        float dh[C::WB][4];      // delta of the current hidden layer
        float denc[C::NINB][4];
        static_for<0, NL>([&](auto kk_) {
            constexpr int k = NL - 1 - decltype(kk_)::value;
            // 1. stage delta_k
            if constexpr (k == NL - 1) {
                round_to_dtype<DT, TS::NOUTB_K>(d);
                stage<DT, TS::NOUTB_K, SD>(stD, wave, lane, d);
            } else {
                round_to_dtype<DT, C::WB>(dh);
                stage<DT, C::WB, SD>(stD, wave, lane, dh);
            }
            // 2. propagate; the activation mask comes from the wave's own columns of h_k
            if constexpr (k > 0) {
                float nd[C::WB][4];
                if constexpr (k == NL - 1)
                    back_layer<DT, TS::NOUTB_K, C::WB>(packed + a.off_b[k], lane, d, nd);
                else
                    back_layer<DT, C::WB, C::WB>(packed + a.off_b[k], lane, dh, nd);
                const E* hk = stH + TS::hrow(k) * SD + wave * 16 + col;
#pragma unroll
                for (int ob = 0; ob < C::WB; ++ob)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float h = (float)hk[(16 * ob + 4 * grp + i) * SD];
                        dh[ob][i] = h > 0.0f ? nd[ob][i] : a.slope * nd[ob][i];
                    }
            } else {
                back_layer<DT, C::WB, C::NINB>(packed + a.off_b[0], lane, dh, denc);
            }
            __syncthreads();
            // 3. weight-gradient tiles over the block's samples
            accumulate_dw<DT, TS::nbi(k), TS::nbo(k), TS::owned(k), TS::acc_off(k), TS::ACC, SD>(
                stD, stH + TS::hrow(k) * SD, wave, lane, acc);
            __syncthreads();
        });

        // ---------------- hash-table gradient ----------------
        // Lane (grp, col) holds sample col of the wave's tile for the levels of
        // group grp, so each 16-lane row covers 16 consecutive samples of one
        // level.  With the routed scatter, equal corner x-pairs of consecutive
        // samples (frequent on coarse levels) are summed across the row first
        // and only the first lane of each run writes a record.
#pragma unroll
        for (int bb = 0; bb < C::NINB; ++bb) {
#pragma unroll
            for (int q = 0; q < 4; q += C::F) {
                const int feat = 16 * bb + 4 * grp + q;
                const int l = feat / C::F;
                const bool lvl_ok = l < a.g.n_levels;
                if (!a.route.enabled && (!valid || !lvl_ok)) continue;
                Corners cr;
                level_corners(a.g, lvl_ok ? l : 0, x0, x1, x2, cr);
                float* gl = a.g_table + (size_t)(lvl_ok ? l : 0) * a.g.T * C::F;
                float dj[C::F];
#pragma unroll
                for (int j = 0; j < C::F; ++j) dj[j] = denc[bb][q + j] * a.final_mul;
                if (a.route.enabled) {
                    const uint32_t Mk = (1u << a.route.k) - 1u;
                    const bool dense = lvl_ok && ((a.g.dense_mask >> l) & 1u);
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        const uint32_t e0 = cr.idx[2 * p], e1 = cr.idx[2 * p + 1];
                        float v[2 * C::F];
#pragma unroll
                        for (int j = 0; j < C::F; ++j) {
                            v[j] = cr.w[2 * p] * dj[j];
                            v[C::F + j] = cr.w[2 * p + 1] * dj[j];
                        }
                        const bool straddle = dense && (e0 & Mk) == Mk;   // pair spans two partitions
                        if (valid && lvl_ok && straddle) {
#pragma unroll
                            for (int j = 0; j < C::F; ++j) {
                                unsafeAtomicAdd(gl + (size_t)e0 * C::F + j, v[j]);
                                unsafeAtomicAdd(gl + (size_t)e1 * C::F + j, v[C::F + j]);
                            }
                        }
                        const bool part = valid && lvl_ok && !straddle;
                        // Keys of lanes that do not take part differ from every real key.
                        const uint32_t k0 = part ? e0 : 0xFFFFFFFFu, k1 = part ? e1 : (uint32_t)lane;
                        if (!part) {
#pragma unroll
                            for (int j = 0; j < 2 * C::F; ++j) v[j] = 0.0f;
                        }
                        const RunInfo ri = row_runs(k0, k1, col);
                        row_run_sums<2 * C::F>(v, ri.last, col);
                        if (part && ri.head) {
                            const int bkt = a.route.bucket_off[l] + (int)(e0 >> a.route.k);
                            const uint32_t end = a.route.base[bkt + 1];
                            const uint32_t slot = atomicAdd(&cursor[bkt], 1u);
                            if (slot < end && slot < a.route.cap) {
                                float* dst = a.route.vals + (size_t)slot * (2 * C::F);
#pragma unroll
                                for (int j = 0; j < 2 * C::F; ++j) rec_max = fmaxf(rec_max, fabsf(v[j]));
                                if constexpr (C::F == 2) {
                                    *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
                                } else {
#pragma unroll
                                    for (int j = 0; j < 2 * C::F; ++j) dst[j] = v[j];
                                }
                                a.route.keys[slot] = (e0 & Mk) | ((e1 & Mk) << 16);
                            } else {                    // cannot happen when the counts match
#pragma unroll
                                for (int j = 0; j < C::F; ++j) {
                                    unsafeAtomicAdd(gl + (size_t)e0 * C::F + j, v[j]);
                                    unsafeAtomicAdd(gl + (size_t)e1 * C::F + j, v[C::F + j]);
                                }
                            }
                        }
                    }
                } else {
#pragma unroll
                    for (int kk = 0; kk < 8; ++kk)
#pragma unroll
                        for (int j = 0; j < C::F; ++j)
                            unsafeAtomicAdd(gl + (size_t)cr.idx[kk] * C::F + j, cr.w[kk] * dj[j]);
                }
            }
        }
    }

    // ---------------- write the block's partial weight gradient and loss ----------------
    float* part = a.ws_w + (int64_t)blockIdx.x * a.n_w;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int nbi = TS::nbi(k), nbo = TS::nbo(k);
        const int in = a.lin[k], out = a.lout[k];
        float* wk = part + a.w_off[k];
#pragma unroll
        for (int j = 0; j < TS::owned(k); ++j) {
            const int t = j * kTrainWaves + wave;
            if (t >= nbi * nbo) break;
            const int ob = t / nbi, ib = t % nbi;
            const float4_t c = acc[TS::acc_off(k) + j];
            const int ci = 16 * ib + col;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ro = 16 * ob + 4 * grp + i;
                if (ro < out && ci < in) wk[(int64_t)ro * in + ci] = c[i] * a.final_mul;
            }
        }
    }
    // Tiles no wave owns do not exist, but entries of partially covered tiles
    // outside (out, in) are skipped above; every (ro, ci) inside is written
    // exactly once because each tile has one owner.
    for (int off = 32; off > 0; off >>= 1) {
        loss_acc += __shfl_xor(loss_acc, off);
        rec_max = fmaxf(rec_max, __shfl_xor(rec_max, off));
    }
    if (lane == 0) {
        red[wave] = loss_acc;
        red_max[wave] = rec_max;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float sacc = 0.0f, m = 0.0f;
        for (int w = 0; w < kTrainWaves; ++w) {
            sacc += red[w];
            m = fmaxf(m, red_max[w]);
        }
        a.ws_loss[blockIdx.x] = sacc;
        if (a.route.enabled) a.route.rec_max[blockIdx.x] = m;
    }
}

// Sum of the blocks' partial weight gradients: slice y of the grid sums
// blocks [y*G/S, (y+1)*G/S) and adds its sum to g_w (the weight gradient's
// summation order across slices is not fixed).  The last block column sums
// the loss once (slice 0 only): a strided pass per thread, then a fixed-order
// tree in LDS.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const float* __restrict__ ws_w,
                                                             const float* __restrict__ ws_loss, int nblocks,
                                                             int64_t n_w, float* __restrict__ g_w,
                                                             float* __restrict__ loss_out, float loss_norm) {
    const int S = gridDim.y, y = blockIdx.y;
    if (blockIdx.x == gridDim.x - 1) {
        if (y != 0 || !loss_out) return;
        __shared__ float red[256];
        float s = 0.0f;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += ws_loss[b];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) *loss_out = red[0] * loss_norm;
        return;
    }
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int b0 = (int)((int64_t)nblocks * y / S), b1 = (int)((int64_t)nblocks * (y + 1) / S);
    if (j < n_w) {
        float s = 0.0f;
        for (int b = b0; b < b1; ++b) s += ws_w[(int64_t)b * n_w + j];
        unsafeAtomicAdd(g_w + j, s);
    }
}

// Shapes that get the in-kernel shadow labels: one 16-output block or two (at most 32 lights).
template <class C> constexpr bool shadow_built() { return train_built<C>() && C::NOUTB <= 2; }

// Persistent grid: one block per CU (every shape fits at least one), at most one per iteration.
// Alone, two per CU (all the resident slots) is faster, but a frame runs this kernel beside
// inference and the next frame's labels: with one block per CU the 1080p frame took 0.921 ms against
// 0.945-0.951 with two (1.5 per CU: 0.931; 0.75: 0.98; 0.5: 1.17), and the per-block weight partials
// and routing offsets halve.  The in-kernel-label variant runs on the same grid (its blocks take the
// same iterations, so given the same labels its gradients are the plain kernel's bit for bit).
static int train_grid(const GridHost& gh, const NetShape& s, int64_t batch, size_t cursor_bytes) {
    (void)gh;
    (void)s;
    (void)cursor_bytes;
    const int64_t iters = (batch + kTrainPts - 1) / kTrainPts;
    int64_t g = (int64_t)cu_count();
    if (g > iters) g = iters;
    if (g < 1) g = 1;
    return (int)g;
}

static size_t route_cursor_bytes(const RoutePlan& rp) { return rp.ok ? (size_t)rp.nb * 4 : 0; }

// The routed scatter for this shape and batch, if its cursors fit the LDS
// beside the activations and its record numbers fit the 32-bit offsets,
// bucket bases and cursors (batch * n_levels * 4 records < 2^32).  Otherwise
// every corner goes through direct FP32 atomics.
static RoutePlan train_route_plan(const GridHost& g, const NetShape& s, int64_t batch) {
    RoutePlan rp = make_route_plan(g);
    size_t smem = 0;
    dispatch_config(g.n_feat, s, [&]<class C>() { smem = TrainShape<C>::SMEM; });
    if (rp.ok && smem + route_cursor_bytes(rp) > 160 * 1024) rp.ok = false;
    if (rp.ok && batch * (int64_t)g.n_levels * 4 >= ((int64_t)1 << 32)) rp.ok = false;
    return rp;
}

bool train_supported(const GridHost& g, const NetShape& s) {
    bool ok = false;
    dispatch_config(g.n_feat, s, [&]<class C>() { ok = train_built<C>(); });
    return ok;
}

// Workspace layout (each part 256-byte aligned):
//   [G][n_w] partial weight gradients | [G] partial losses |
//   routed scatter: [nb][G] offsets | [nb] totals | [nb+1] bases | [nb+1] chunk bases |
//                   [R / chunk + nb] chunk buckets | [R][2F] values | [R] keys | [G] record maxima
// with R = batch * n_levels * 4 records (one per corner x-pair).
struct WsLayout {
    int64_t w, loss, offsets, totals, base, chunk_base, chunk_bucket, vals, keys, rec_max, total;
};

static int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

static WsLayout ws_layout(const GridHost& g, int64_t n_w, int64_t batch, int G, const RoutePlan& rp) {
    WsLayout L{};
    int64_t o = 0;
    L.w = o;
    o = align256(o + (int64_t)G * n_w * 4);
    L.loss = o;
    o = align256(o + (int64_t)G * 4);
    if (rp.ok) {
        const int64_t R = batch * g.n_levels * 4;
        L.offsets = o;
        o = align256(o + (int64_t)G * rp.nb * 4);
        L.totals = o;
        o = align256(o + (int64_t)rp.nb * 4);
        L.base = o;
        o = align256(o + (int64_t)(rp.nb + 1) * 4);
        L.chunk_base = o;
        o = align256(o + (int64_t)(rp.nb + 1) * 4);
        L.chunk_bucket = o;
        o = align256(o + ((R + kRouteChunk - 1) / kRouteChunk + rp.nb) * 4);
        L.vals = o;
        o = align256(o + R * 2 * g.n_feat * 4);
        L.keys = o;
        o = align256(o + R * 4);
        L.rec_max = o;
        o = align256(o + (int64_t)G * 4);
    }
    L.total = o;
    return L;
}

// Routing plan (nvc_train_plan): the plan arrays of the workspace layout, in a buffer of their own
// (each part 256-byte aligned): [nb][G] offsets | [nb] totals | [nb+1] bases | [nb+1] chunk bases |
// [R / chunk + nb] chunk buckets.
struct PlanLayout {
    int64_t offsets, totals, base, chunk_base, chunk_bucket, total;
};

static PlanLayout plan_layout(const GridHost& g, int64_t batch, int G, const RoutePlan& rp) {
    PlanLayout L{};
    if (!rp.ok) return L;
    const int64_t R = batch * g.n_levels * 4;
    int64_t o = 0;
    L.offsets = o;
    o = align256(o + (int64_t)G * rp.nb * 4);
    L.totals = o;
    o = align256(o + (int64_t)rp.nb * 4);
    L.base = o;
    o = align256(o + (int64_t)(rp.nb + 1) * 4);
    L.chunk_base = o;
    o = align256(o + (int64_t)(rp.nb + 1) * 4);
    L.chunk_bucket = o;
    o = align256(o + ((R + kRouteChunk - 1) / kRouteChunk + rp.nb) * 4);
    L.total = o;
    return L;
}

static int64_t n_weights(const NetShape& s) {
    return (int64_t)s.n_in * s.width + (int64_t)(s.n_hidden - 1) * s.width * s.width + (int64_t)s.width * s.n_out;
}

int64_t train_workspace_bytes(const GridHost& g, const NetShape& s, int64_t batch) {
    const RoutePlan rp = train_route_plan(g, s, batch);
    return ws_layout(g, n_weights(s), batch, train_grid(g, s, batch, route_cursor_bytes(rp)), rp).total;
}

// A shape gets the in-kernel labels if such a kernel is built and its LDS (activations, scatter cursors,
// lights and spheres) fits the 160 KiB of a CU.
bool train_shadow_supported(const GridHost& g, const NetShape& s, int64_t batch, int n_spheres) {
    bool ok = false;
    const size_t cb = route_cursor_bytes(train_route_plan(g, s, batch));
    dispatch_config(g.n_feat, s, [&]<class C>() {
        if constexpr (shadow_built<C>())
            ok = (TrainShape<C>::SMEM + cb + 15) / 16 * 16 + shadow_smem_bytes(n_spheres) <= 160 * 1024;
    });
    return ok;
}


static hipError_t launch_train_impl(const GridHost& gh, const NetShape& s, const PackPlan& plan, const float* table,
                                    const void* packed, const float* pos, const int32_t* pix, int64_t batch,
                                    const uint8_t* labels, const float* dvis, int loss, float grad_scale,
                                    float* g_table, float* g_w, float* loss_out, void* workspace,
                                    const ShadowArgs* sh, const void* plan_buf, hipStream_t st) {
    TrainArgs a{};
    a.g = grid_to_dev(gh);
    a.table = table;
    a.packed = packed;
    a.n_w = 0;
    for (int k = 0; k < plan.n_layers; ++k) {
        a.off_f[k] = plan.layer[k].off_f;
        a.off_b[k] = plan.layer[k].off_b;
        a.w_off[k] = plan.layer[k].w_off;
        a.lin[k] = plan.layer[k].in;
        a.lout[k] = plan.layer[k].out;
        a.n_w += (int64_t)plan.layer[k].in * plan.layer[k].out;
    }
    a.pos = pos;
    a.pix = pix;
    a.batch = batch;
    a.n_out = s.n_out;
    a.labels = labels;
    a.dvis = dvis;
    a.loss = loss;
    if (sh) {
        a.pos_scene = sh->pos_scene;
        a.lights = sh->lights;
        a.n_lights = sh->n_lights;
        a.spheres = sh->spheres;
        a.n_spheres = sh->n_spheres;
        a.labels_out = sh->labels_out;
    }
    const double count = (double)batch * s.n_out;
    if (labels || sh) {
        const double gs = grad_scale > 0.0f ? grad_scale : count;
        a.out_mul = (float)(gs / count);
        a.final_mul = (float)(1.0 / gs);
    } else {
        const double gs = grad_scale > 0.0f ? grad_scale : 1.0;
        a.out_mul = (float)gs;
        a.final_mul = (float)(1.0 / gs);
    }
    a.g_table = g_table;
    const RoutePlan rp = train_route_plan(gh, s, batch);
    const size_t cursor_bytes = route_cursor_bytes(rp);
    const int G = train_grid(gh, s, batch, cursor_bytes);
    const WsLayout wl = ws_layout(gh, a.n_w, batch, G, rp);
    unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
    a.ws_w = reinterpret_cast<float*>(ws + wl.w);
    a.ws_loss = reinterpret_cast<float*>(ws + wl.loss);
    a.act = s.act;
    a.slope = s.slope;
    a.route = RouteDev{};
    hipError_t err = hipSuccess;
    if (rp.ok) {
        RouteDev& r = a.route;
        r.enabled = 1;
        r.k = rp.k;
        r.nb = rp.nb;
        for (int l = 0; l <= kMaxLevels; ++l) r.bucket_off[l] = l <= gh.n_levels ? rp.bucket_off[l] : rp.nb;
        for (int l = 0; l < kMaxLevels; ++l) r.entries[l] = rp.entries[l];
        if (plan_buf) {
            // the plan was computed beforehand (nvc_train_plan) from the same samples
            const PlanLayout pl = plan_layout(gh, batch, G, rp);
            unsigned char* pb = reinterpret_cast<unsigned char*>(const_cast<void*>(plan_buf));
            r.offsets = reinterpret_cast<uint32_t*>(pb + pl.offsets);
            r.totals = reinterpret_cast<uint32_t*>(pb + pl.totals);
            r.base = reinterpret_cast<uint32_t*>(pb + pl.base);
            r.chunk_base = reinterpret_cast<uint32_t*>(pb + pl.chunk_base);
            r.chunk_bucket = reinterpret_cast<uint32_t*>(pb + pl.chunk_bucket);
        } else {
            r.offsets = reinterpret_cast<uint32_t*>(ws + wl.offsets);
            r.totals = reinterpret_cast<uint32_t*>(ws + wl.totals);
            r.base = reinterpret_cast<uint32_t*>(ws + wl.base);
            r.chunk_base = reinterpret_cast<uint32_t*>(ws + wl.chunk_base);
            r.chunk_bucket = reinterpret_cast<uint32_t*>(ws + wl.chunk_bucket);
        }
        r.vals = reinterpret_cast<float*>(ws + wl.vals);
        r.keys = reinterpret_cast<uint32_t*>(ws + wl.keys);
        r.rec_max = reinterpret_cast<float*>(ws + wl.rec_max);
        r.cap = (uint32_t)(batch * gh.n_levels * 4);
        if (!plan_buf) {
            err = launch_route_count(gh, r, pos, pix, batch, G, kTrainPts, st);
            if (err == hipSuccess) err = launch_route_prefix(r, G, st);
            if (err != hipSuccess) return err;
        }
    }
    err = hipErrorNotSupported;
    dispatch_config(gh.n_feat, s, [&]<class C>() {
        if (sh) {
            if constexpr (shadow_built<C>()) {
                const size_t smem = (TrainShape<C>::SMEM + cursor_bytes + 15) / 16 * 16 + shadow_smem_bytes(sh->n_spheres);
                hipLaunchKernelGGL((train_kernel<C, true>), dim3(G), dim3(256), smem, st, a);
                err = hipGetLastError();
            }
        } else if constexpr (train_built<C>()) {
            hipLaunchKernelGGL((train_kernel<C, false>), dim3(G), dim3(256), TrainShape<C>::SMEM + cursor_bytes, st, a);
            err = hipGetLastError();
        }
    });
    if (err != hipSuccess) return err;
    if (a.route.enabled) {
        err = launch_route_accumulate(gh, a.route, g_table, batch * gh.n_levels * 4, G, st);
        if (err != hipSuccess) return err;
    }
    const int slices = std::min(G, 64);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((a.n_w + 255) / 256 + 1), slices), dim3(256), 0, st,
                       a.ws_w, a.ws_loss, G, a.n_w, g_w, (labels || sh) ? loss_out : nullptr, (float)(1.0 / count));
    return hipGetLastError();
}

hipError_t launch_train(const GridHost& gh, const NetShape& s, const PackPlan& plan, const float* table,
                        const void* packed, const float* pos, const int32_t* pix, int64_t batch,
                        const uint8_t* labels, const float* dvis, int loss, float grad_scale, float* g_table,
                        float* g_w, float* loss_out, void* workspace, hipStream_t st) {
    return launch_train_impl(gh, s, plan, table, packed, pos, pix, batch, labels, dvis, loss, grad_scale, g_table, g_w,
                             loss_out, workspace, nullptr, nullptr, st);
}

hipError_t launch_train_planned(const GridHost& gh, const NetShape& s, const PackPlan& plan, const float* table,
                                const void* packed, const float* pos, const int32_t* pix, int64_t batch,
                                const uint8_t* labels, const float* dvis, int loss, float grad_scale, float* g_table,
                                float* g_w, float* loss_out, const void* route_plan, void* workspace, hipStream_t st) {
    return launch_train_impl(gh, s, plan, table, packed, pos, pix, batch, labels, dvis, loss, grad_scale, g_table, g_w,
                             loss_out, workspace, nullptr, route_plan, st);
}

int64_t train_plan_bytes(const GridHost& g, const NetShape& s, int64_t batch) {
    const RoutePlan rp = train_route_plan(g, s, batch);
    return plan_layout(g, batch, train_grid(g, s, batch, route_cursor_bytes(rp)), rp).total;
}

hipError_t launch_train_plan(const GridHost& gh, const NetShape& s, const float* pos, const int32_t* pix,
                             int64_t batch, void* plan_buf, hipStream_t st) {
    const RoutePlan rp = train_route_plan(gh, s, batch);
    if (!rp.ok) return hipSuccess;                         // direct atomics: nothing to plan
    const int G = train_grid(gh, s, batch, route_cursor_bytes(rp));
    const PlanLayout pl = plan_layout(gh, batch, G, rp);
    unsigned char* pb = reinterpret_cast<unsigned char*>(plan_buf);
    RouteDev r{};
    r.enabled = 1;
    r.k = rp.k;
    r.nb = rp.nb;
    for (int l = 0; l <= kMaxLevels; ++l) r.bucket_off[l] = l <= gh.n_levels ? rp.bucket_off[l] : rp.nb;
    for (int l = 0; l < kMaxLevels; ++l) r.entries[l] = rp.entries[l];
    r.offsets = reinterpret_cast<uint32_t*>(pb + pl.offsets);
    r.totals = reinterpret_cast<uint32_t*>(pb + pl.totals);
    r.base = reinterpret_cast<uint32_t*>(pb + pl.base);
    r.chunk_base = reinterpret_cast<uint32_t*>(pb + pl.chunk_base);
    r.chunk_bucket = reinterpret_cast<uint32_t*>(pb + pl.chunk_bucket);
    r.cap = (uint32_t)(batch * gh.n_levels * 4);
    hipError_t err = launch_route_count(gh, r, pos, pix, batch, G, kTrainPts, st);
    if (err == hipSuccess) err = launch_route_prefix(r, G, st);
    return err;
}

hipError_t launch_train_shadow(const GridHost& gh, const NetShape& s, const PackPlan& plan, const float* table,
                               const void* packed, const float* pos, const int32_t* pix, int64_t batch,
                               const ShadowArgs& sh, int loss, float grad_scale, float* g_table, float* g_w,
                               float* loss_out, void* workspace, hipStream_t st) {
    return launch_train_impl(gh, s, plan, table, packed, pos, pix, batch, nullptr, nullptr, loss, grad_scale, g_table,
                             g_w, loss_out, workspace, &sh, nullptr, st);
}

}  // namespace nvc
