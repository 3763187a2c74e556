// Fused cache inference (Sec. 3.1 steps 1-2, Sec. 3.3): hash-grid encoding and
// the visibility MLP in one kernel, plus packing of the weights into
// matrix-core operand fragments.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "kernel_config.hpp"

namespace nvc {

size_t dtype_size(int dt) { return dt == DT_F32 ? 4 : 2; }

static int padk(int dt) { return dt == DT_F32 ? 16 : 32; }
static int ceil_to(int x, int m) { return (x + m - 1) / m * m; }
static int chunks(int dt, int nb) { return dt == DT_F32 ? nb * 4 : nb / 2; }
static int epl(int dt) { return dt == DT_F32 ? 1 : 8; }

PackPlan make_pack_plan(const NetShape& s) {
    PackPlan p{};
    p.n_layers = s.n_hidden + 1;
    int64_t off = 0, woff = 0;
    for (int k = 0; k < p.n_layers; ++k) {
        LayerPack& L = p.layer[k];
        L.in = k == 0 ? s.n_in : s.width;
        L.out = k == p.n_layers - 1 ? s.n_out : s.width;
        L.nb_out_f = ceil_to(L.out, 16) / 16;
        L.kc_in_f = chunks(s.dtype, ceil_to(L.in, padk(s.dtype)) / 16);
        L.nb_in_b = ceil_to(L.in, padk(s.dtype)) / 16;   // rows of W^T, padded like the kernels' input blocks
        L.kc_out_b = chunks(s.dtype, ceil_to(L.out, padk(s.dtype)) / 16);
        L.w_off = woff;
        woff += (int64_t)L.in * L.out;
        L.off_f = off;
        off += (int64_t)L.nb_out_f * L.kc_in_f * 64 * epl(s.dtype);
        L.off_b = off;
        off += (int64_t)L.nb_in_b * L.kc_out_b * 64 * epl(s.dtype);
    }
    p.total_elems = off;
    return p;
}

// ------------------------------------------------------------------ packing
template <int DT>
__global__ void pack_kernel(PackPlan plan, const float* __restrict__ w, typename Mma<DT>::elem* __restrict__ out) {
    using M = Mma<DT>;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= plan.total_elems) return;
    int k = 0;
    while (k + 1 < plan.n_layers && e >= plan.layer[k + 1].off_f) ++k;
    const LayerPack& L = plan.layer[k];
    const float* W = w + L.w_off;
    float v = 0.0f;
    if (e < L.off_b) {                       // forward: A[row = out neuron][K = in neuron]
        const int64_t r = e - L.off_f;
        const int s = (int)(r % M::EPL);
        const int lane = (int)((r / M::EPL) % 64);
        const int64_t fr = r / (M::EPL * 64);
        const int kc = (int)(fr % L.kc_in_f);
        const int ob = (int)(fr / L.kc_in_f);
        const int row = 16 * ob + lane % 16;
        const int col = kperm<DT>(kc, lane / 16, s);
        if (row < L.out && col < L.in) v = W[(int64_t)row * L.in + col];
    } else {                                 // backward: A[row = in neuron][K = out neuron] = W^T
        const int64_t r = e - L.off_b;
        const int s = (int)(r % M::EPL);
        const int lane = (int)((r / M::EPL) % 64);
        const int64_t fr = r / (M::EPL * 64);
        const int kc = (int)(fr % L.kc_out_b);
        const int ib = (int)(fr / L.kc_out_b);
        const int row = 16 * ib + lane % 16;
        const int col = kperm<DT>(kc, lane / 16, s);
        if (row < L.in && col < L.out) v = W[(int64_t)col * L.in + row];
    }
    out[e] = M::cvt(v);
}

hipError_t launch_pack(const NetShape& s, const PackPlan& plan, const float* w, void* packed, hipStream_t st) {
    const int threads = 256;
    const int blocks = (int)((plan.total_elems + threads - 1) / threads);
    if (s.dtype == DT_F16)
        pack_kernel<DT_F16><<<blocks, threads, 0, st>>>(plan, w, (_Float16*)packed);
    else if (s.dtype == DT_BF16)
        pack_kernel<DT_BF16><<<blocks, threads, 0, st>>>(plan, w, (__bf16*)packed);
    else
        pack_kernel<DT_F32><<<blocks, threads, 0, st>>>(plan, w, (float*)packed);
    return hipGetLastError();
}

// ------------------------------------------------------------------ inference
// One wave computes NSUB sub-tiles of 16 points at a time.  Lane l encodes, for
// point l%16 of each sub-tile, the levels whose features it feeds to the first
// layer (see encode_lane); the layers then run on the matrix cores with the
// activations in registers and the forward weight fragments in LDS.
template <int DT, int NSUB, int NBI, int NBO>
__device__ inline void mlp_layer(const typename Mma<DT>::elem* W, int lane, const float (&in)[NSUB][NBI][4],
                                 float (&out)[NSUB][NBO][4]) {
    using M = Mma<DT>;
    constexpr int KC = kchunks<DT>(NBI);
#pragma unroll
    for (int ob = 0; ob < NBO; ++ob) {
        float4_t acc[NSUB];
#pragma unroll
        for (int s = 0; s < NSUB; ++s) acc[s] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const typename M::frag a = load_frag<DT>(W, ob, kc, KC, lane);
#pragma unroll
            for (int s = 0; s < NSUB; ++s) acc[s] = M::mma(a, make_frag<DT, NBI>(in[s], kc), acc[s]);
        }
#pragma unroll
        for (int s = 0; s < NSUB; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) out[s][ob][i] = acc[s][i];
    }
}

template <int NSUB, int NB>
__device__ inline void activate(float (&a)[NSUB][NB][4], float slope) {
    if (slope == 0.0f) {       // ReLU: a float with the sign bit set is a negative int32, so max(bits, 0) is one op
#pragma unroll
        for (int s = 0; s < NSUB; ++s)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int i = 0; i < 4; ++i) a[s][b][i] = __int_as_float(max(__float_as_int(a[s][b][i]), 0));
    } else {                   // leaky, 0 < slope <= 1
#pragma unroll
        for (int s = 0; s < NSUB; ++s)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int i = 0; i < 4; ++i) a[s][b][i] = fmaxf(a[s][b][i], slope * a[s][b][i]);
    }
}

// Fragments of the forward matrices, compact in LDS: layer 0, hidden layers, output layer.
template <class C>
struct FwdLayout {
    static constexpr int EPL = Mma<C::DT>::EPL;
    static constexpr int frag_elems = 64 * EPL;
    static constexpr int L0 = C::WB * kchunks<C::DT>(C::NINB) * frag_elems;
    static constexpr int LH = C::WB * kchunks<C::DT>(C::WB) * frag_elems;
    static constexpr int LO = C::NOUTB * kchunks<C::DT>(C::WB) * frag_elems;
    static constexpr int total = L0 + (C::NHID - 1) * LH + LO;
    __host__ __device__ static constexpr int off(int k) { return k == 0 ? 0 : L0 + (k - 1) * LH; }
};

constexpr int kInferLdsMax = 112 * 1024;

struct InferArgs {
    GridDev g;
    const float* table;
    const void* packed;
    int64_t layer_off[kMaxLayers];    // element offsets of the forward fragments in `packed`
    const float* pos;
    int64_t n;
    int n_out;
    void* vis;
    int vis_dtype;
    int act;
    float slope;
    int vec_ok;           // rows start 4-element aligned and vis is 16-byte aligned: vector stores
    const void* enc;      // pre-computed encoding [n][n_in] (nvc_mlp_forward), else nullptr
    int enc_dtype;
    int n_in;
    int enc_vec;          // n_in % 4 == 0 and enc 16-byte aligned
};

// Encoding features of point p a lane owns (layout of encode_lane), read from
// a pre-computed [n][n_in] buffer and rounded to FP32.  vec: n_in is a
// multiple of 4 and the buffer 16-byte aligned, so a lane's four features of
// a block are one aligned load.
template <int NINB>
__device__ inline void load_lane_encoding(const void* enc, int enc_dtype, int n_in, bool vec, int64_t p, int grp,
                                          float (&act)[NINB][4]) {
#pragma unroll
    for (int b = 0; b < NINB; ++b) {
        const int f0 = 16 * b + 4 * grp;
        const int64_t o = p * n_in + f0;
        if (vec && f0 + 4 <= n_in) {
            if (enc_dtype == DT_F32) {
                const float4 v = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(enc) + o);
                act[b][0] = v.x; act[b][1] = v.y; act[b][2] = v.z; act[b][3] = v.w;
            } else if (enc_dtype == DT_F16) {
                typedef _Float16 h4 __attribute__((ext_vector_type(4)));
                const h4 v = *reinterpret_cast<const h4*>(reinterpret_cast<const _Float16*>(enc) + o);
#pragma unroll
                for (int i = 0; i < 4; ++i) act[b][i] = (float)v[i];
            } else {
                typedef __bf16 b4 __attribute__((ext_vector_type(4)));
                const b4 v = *reinterpret_cast<const b4*>(reinterpret_cast<const __bf16*>(enc) + o);
#pragma unroll
                for (int i = 0; i < 4; ++i) act[b][i] = (float)v[i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = 0.0f;
                if (f0 + i < n_in) {
                    if (enc_dtype == DT_F32)
                        v = reinterpret_cast<const float*>(enc)[o + i];
                    else if (enc_dtype == DT_F16)
                        v = (float)reinterpret_cast<const _Float16*>(enc)[o + i];
                    else
                        v = (float)reinterpret_cast<const __bf16*>(enc)[o + i];
                }
                act[b][i] = v;
            }
        }
    }
}

// Waves per block: eight for the 128-wide network (twelve when the encoding
// is read from memory: fewer registers), whose weights fill most of the LDS
// (one block per CU); four otherwise.
template <class C, bool PRE> constexpr int infer_waves() { return C::WB >= 8 ? (PRE ? 12 : 8) : 4; }

// PRE: the encoding comes from a.enc (nvc_mlp_forward) instead of the table.
template <class C, bool PRE>
__global__ __launch_bounds__((64 * infer_waves<C, PRE>())) void infer_kernel(InferArgs a) {
    constexpr int DT = C::DT;
    using M = Mma<DT>;
    using E = typename M::elem;
    using LY = FwdLayout<C>;
    constexpr int NSUB = C::NSUB_INFER;
    constexpr int NL = C::NHID + 1;
    constexpr bool WLDS = LY::total * (int)sizeof(E) <= kInferLdsMax;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    E* wl = reinterpret_cast<E*>(smem_raw);
    const E* wk[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k)
        wk[k] = WLDS ? wl + LY::off(k) : reinterpret_cast<const E*>(a.packed) + a.layer_off[k];

    // Stage the forward fragments once per (persistent) block.
    if constexpr (WLDS) {
        const E* src = reinterpret_cast<const E*>(a.packed);
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int len = k == 0 ? LY::L0 : (k == NL - 1 ? LY::LO : LY::LH);
            const E* s = src + a.layer_off[k];
            E* d = wl + LY::off(k);
            for (int i = threadIdx.x * 8; i < len; i += blockDim.x * 8) {
                if (i + 8 <= len) {
                    *reinterpret_cast<uint4*>(d + i) = *reinterpret_cast<const uint4*>(s + i);
                    if constexpr (sizeof(E) == 4) *reinterpret_cast<uint4*>(d + i + 4) = *reinterpret_cast<const uint4*>(s + i + 4);
                } else {
                    for (int j = i; j < len; ++j) d[j] = s[j];
                }
            }
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int grp = lane >> 4;
    const int col = lane & 15;
    constexpr int PTS = 16 * NSUB;
    const int64_t ntiles = (a.n + PTS - 1) / PTS;
    // XCD-aware: blocks are dealt round-robin to the 8 XCDs, so give each XCD a
    // contiguous range of tiles (screen-space locality per L2).
    const int G = gridDim.x;
    const int lb = (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8;
    const int64_t per_block = (ntiles + G - 1) / G;
    const int64_t t0 = (int64_t)lb * per_block;
    const int64_t t1 = min(ntiles, t0 + per_block);

    LevelLane lv[C::NINB][4 / C::F];
    if constexpr (!PRE) lane_levels<C::F, C::NINB>(a.g, grp, lv);
    for (int64_t t = t0 + wave; t < t1; t += infer_waves<C, PRE>()) {
        // Weight fragments are read from LDS (or L1) in every iteration: the
        // opaque zero offset stops the compiler from hoisting all of them into
        // registers, which would cost occupancy.
        int opq = 0;
        asm volatile("" : "+s"(opq));
        const E* w_it[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) w_it[k] = wk[k] + opq;
        float h0[NSUB][C::NINB][4];
#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
            const int64_t p = t * PTS + s * 16 + col;
            const int64_t pc = p < a.n ? p : a.n - 1;
            if constexpr (PRE) {
                load_lane_encoding<C::NINB>(a.enc, a.enc_dtype, a.n_in, a.enc_vec != 0, pc, grp, h0[s]);
            } else {
                const float x = clamp_unit(a.pos[pc * 3 + 0]);
                const float y = clamp_unit(a.pos[pc * 3 + 1]);
                const float z = clamp_unit(a.pos[pc * 3 + 2]);
                encode_lane_lv<C::F, C::NINB>(a.table, lv, x, y, z, h0[s]);
            }
        }
        float ha[NSUB][C::WB][4], hb[NSUB][C::WB][4];
        mlp_layer<DT, NSUB, C::NINB, C::WB>(w_it[0], lane, h0, ha);
        activate<NSUB, C::WB>(ha, a.slope);
#pragma unroll
        for (int k = 1; k < C::NHID; ++k) {
            if (k % 2 == 1) {
                mlp_layer<DT, NSUB, C::WB, C::WB>(w_it[k], lane, ha, hb);
                activate<NSUB, C::WB>(hb, a.slope);
            } else {
                mlp_layer<DT, NSUB, C::WB, C::WB>(w_it[k], lane, hb, ha);
                activate<NSUB, C::WB>(ha, a.slope);
            }
        }
        float z[NSUB][C::NOUTB][4];
        if (C::NHID % 2 == 1)
            mlp_layer<DT, NSUB, C::WB, C::NOUTB>(w_it[NL - 1], lane, ha, z);
        else
            mlp_layer<DT, NSUB, C::WB, C::NOUTB>(w_it[NL - 1], lane, hb, z);

#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
            const int64_t p = t * PTS + s * 16 + col;
            if (p >= a.n) continue;
#pragma unroll
            for (int ob = 0; ob < C::NOUTB; ++ob) {
                const int l0 = 16 * ob + 4 * grp;
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = sigmoid_fast(z[s][ob][i]);
                const int64_t base = p * a.n_out + l0;
                if (a.vec_ok && l0 + 4 <= a.n_out) {
                    if (a.vis_dtype == DT_F32) {
                        *reinterpret_cast<float4*>((float*)a.vis + base) = make_float4(v[0], v[1], v[2], v[3]);
                    } else if (a.vis_dtype == DT_F16) {
                        typedef _Float16 h4 __attribute__((ext_vector_type(4)));
                        h4 o = {(_Float16)v[0], (_Float16)v[1], (_Float16)v[2], (_Float16)v[3]};
                        *reinterpret_cast<h4*>((_Float16*)a.vis + base) = o;
                    } else {
                        typedef __bf16 b4 __attribute__((ext_vector_type(4)));
                        b4 o = {(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
                        *reinterpret_cast<b4*>((__bf16*)a.vis + base) = o;
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (l0 + i >= a.n_out) break;
                        if (a.vis_dtype == DT_F32)
                            ((float*)a.vis)[base + i] = v[i];
                        else if (a.vis_dtype == DT_F16)
                            ((_Float16*)a.vis)[base + i] = (_Float16)v[i];
                        else
                            ((__bf16*)a.vis)[base + i] = (__bf16)v[i];
                    }
                }
            }
        }
    }
}

static int device_cu_count_impl() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
        cached[dev] = cu;
    }
    return cached[dev];
}
int cu_count() { return device_cu_count_impl(); }

template <class C>
static hipError_t run_infer(const GridDev& g, const PackPlan& plan, const float* table, const void* packed,
                            const float* pos, int64_t n, int n_out, void* vis, int vis_dtype, int act, float slope,
                            const void* enc, int enc_dtype, int n_in, hipStream_t st) {
    InferArgs a{};
    a.enc = enc;
    a.enc_dtype = enc_dtype;
    a.n_in = n_in;
    a.enc_vec = n_in % 4 == 0 && ((uintptr_t)enc % 16) == 0;
    a.g = g;
    a.table = table;
    a.packed = packed;
    for (int k = 0; k < plan.n_layers; ++k) a.layer_off[k] = plan.layer[k].off_f;
    a.pos = pos;
    a.n = n;
    a.n_out = n_out;
    a.vis = vis;
    a.vis_dtype = vis_dtype;
    a.act = act;
    a.slope = slope;
    a.vec_ok = (n_out % 4) == 0 && ((uintptr_t)vis % 16) == 0;
    using LY = FwdLayout<C>;
    const size_t wbytes = (size_t)LY::total * sizeof(typename Mma<C::DT>::elem);
    const size_t smem = wbytes <= (size_t)kInferLdsMax ? wbytes : 0;
    const int64_t pts = 16 * C::NSUB_INFER;
    const int64_t ntiles = (n + pts - 1) / pts;
    const int per_cu = smem > 80 * 1024 ? 1 : (smem > 40 * 1024 ? 2 : 4);
    const int IW = enc ? infer_waves<C, true>() : infer_waves<C, false>();
    int64_t want = (ntiles + IW - 1) / IW;                  // at least one tile per wave
    int64_t G = std::min<int64_t>(want, (int64_t)cu_count() * per_cu);
    G = std::max<int64_t>(8, (G + 7) / 8 * 8);
    if (enc)
        hipLaunchKernelGGL((infer_kernel<C, true>), dim3((unsigned)G), dim3(64 * IW), smem, st, a);
    else
        hipLaunchKernelGGL((infer_kernel<C, false>), dim3((unsigned)G), dim3(64 * IW), smem, st, a);
    return hipGetLastError();
}

static GridDev to_dev(const GridHost& g) {
    GridDev d{};
    d.n_levels = g.n_levels;
    d.n_feat = g.n_feat;
    d.T = 1u << g.log2_T;
    d.dense_mask = g.dense_mask;
    for (int l = 0; l < kMaxLevels; ++l) d.res[l] = g.res[l];
    return d;
}

bool infer_supported(const GridHost& g, const NetShape& s) {
    return dispatch_config(g.n_feat, s, [&]<class C>() {});
}

hipError_t launch_infer(const GridHost& g, const NetShape& s, const PackPlan& plan, const float* table,
                        const void* packed, const float* pos, int64_t n, void* vis, int vis_dtype, hipStream_t st) {
    hipError_t err = hipErrorNotSupported;
    const GridDev gd = to_dev(g);
    dispatch_config(g.n_feat, s, [&]<class C>() {
        err = run_infer<C>(gd, plan, table, packed, pos, n, s.n_out, vis, vis_dtype, s.act, s.slope, nullptr, 0,
                           s.n_in, st);
    });
    return err;
}

// The MLP alone on a given encoding: the configurations differ in features
// per level only through the encoding, so any matching one serves.
static int mlp_feat(const NetShape& s) {
    for (int F : {2, 4, 1})
        if (dispatch_config(F, s, [&]<class C>() {})) return F;
    return 0;
}

bool mlp_supported(const NetShape& s) { return mlp_feat(s) != 0; }

hipError_t launch_mlp_forward(const NetShape& s, const PackPlan& plan, const void* packed, const void* enc,
                              int enc_dtype, int64_t n, void* vis, int vis_dtype, hipStream_t st) {
    hipError_t err = hipErrorNotSupported;
    const GridDev gd{};
    dispatch_config(mlp_feat(s), s, [&]<class C>() {
        err = run_infer<C>(gd, plan, nullptr, packed, nullptr, n, s.n_out, vis, vis_dtype, s.act, s.slope, enc,
                           enc_dtype, s.n_in, st);
    });
    return err;
}

}  // namespace nvc
