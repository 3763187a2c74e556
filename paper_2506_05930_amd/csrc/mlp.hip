// Fused cache inference (Sec. 3.1 steps 1-2, Sec. 3.3): hash-grid encoding and
// the visibility MLP in one kernel, plus packing of the weights into
// matrix-core operand fragments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

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
        L.off_o = L.off_f;
        L.gb_o = 1;
    }
    // 16-bit inference stores pairs of output blocks (out_neuron order).
    LayerPack& O = p.layer[p.n_layers - 1];
    if (s.dtype != DT_F32 && O.nb_out_f % 2 == 0) {
        O.gb_o = 2;
        O.off_o = off;
        off += (int64_t)O.nb_out_f * O.kc_in_f * 64 * epl(s.dtype);
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
    const bool inf_copy = L.off_o != L.off_f && e >= L.off_o;
    if (e < L.off_b || inf_copy) {           // forward: A[row = out neuron][K = in neuron]
        const int64_t r = e - (inf_copy ? L.off_o : L.off_f);
        const int s = (int)(r % M::EPL);
        const int lane = (int)((r / M::EPL) % 64);
        const int64_t fr = r / (M::EPL * 64);
        const int kc = (int)(fr % L.kc_in_f);
        const int ob = (int)(fr / L.kc_in_f);
        const int row = inf_copy ? out_neuron(ob, lane % 16, L.gb_o) : 16 * ob + lane % 16;
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

// Hidden activation in FP32: ReLU (a float with the sign bit set is a
// negative int32, so max(bits, 0) is one instruction) or leaky ReLU with
// 0 < slope <= 1.
template <bool LEAKY, int NSUB, int NB>
__device__ inline void activate(float (&a)[NSUB][NB][4], float slope) {
#pragma unroll
    for (int s = 0; s < NSUB; ++s)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a[s][b][i] = LEAKY ? fmaxf(a[s][b][i], slope * a[s][b][i])
                                   : __int_as_float(max(__float_as_int(a[s][b][i]), 0));
}

// Next layer's B fragment from the accumulators of output blocks 2c (lo) and
// 2c+1 (hi), in kperm order, after the hidden activation.  The ReLU is taken
// on the rounded 16-bit values as a packed integer max with zero: a negative
// value (-0 included) has the sign bit set, so this equals rounding the FP32
// ReLU, in one instruction per two neurons.
template <int DT>
__device__ inline typename Mma<DT>::frag frag_of(float4_t lo, float4_t hi) {
    // Pairwise vector conversions: one packed convert per two neurons.
    using E = typename Mma<DT>::elem;
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef E e2 __attribute__((ext_vector_type(2)));
    const e2 p0 = __builtin_convertvector((f2){lo[0], lo[1]}, e2);
    const e2 p1 = __builtin_convertvector((f2){lo[2], lo[3]}, e2);
    const e2 p2 = __builtin_convertvector((f2){hi[0], hi[1]}, e2);
    const e2 p3 = __builtin_convertvector((f2){hi[2], hi[3]}, e2);
    return typename Mma<DT>::frag{p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
}

template <bool LEAKY, int DT>
__device__ inline typename Mma<DT>::frag act_frag(float4_t lo, float4_t hi, float slope) {
    if constexpr (!LEAKY) {
        typedef short short8_t __attribute__((ext_vector_type(8)));
        const short8_t b = __builtin_elementwise_max(__builtin_bit_cast(short8_t, frag_of<DT>(lo, hi)), (short8_t)0);
        return __builtin_bit_cast(typename Mma<DT>::frag, b);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        lo[i] = fmaxf(lo[i], slope * lo[i]);
        hi[i] = fmaxf(hi[i], slope * hi[i]);
    }
    return frag_of<DT>(lo, hi);
}

// 16-bit layers are software-pipelined over 16-neuron output blocks: the
// weight fragments of block u+1 are read from LDS while the matrix cores work
// on block u (a scheduling barrier keeps the reads ahead), and the finished
// blocks are activated (or passed through the sigmoid and stored) under the
// next block's matrix work.
template <int DT, int KCI>
__device__ inline void load_block(const typename Mma<DT>::elem* W, int ob, int lane,
                                  typename Mma<DT>::frag (&w)[KCI]) {
#pragma unroll
    for (int kc = 0; kc < KCI; ++kc) w[kc] = load_frag<DT>(W, ob, kc, KCI, lane);
}

template <int DT, int NSUB, int KCI>
__device__ inline void mma_block(const typename Mma<DT>::frag (&w)[KCI],
                                 const typename Mma<DT>::frag (&in)[NSUB][KCI], float4_t (&acc)[NSUB]) {
#pragma unroll
    for (int s = 0; s < NSUB; ++s) acc[s] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KCI; ++kc)
#pragma unroll
        for (int s = 0; s < NSUB; ++s) acc[s] = Mma<DT>::mma(w[kc], in[s][kc], acc[s]);
}

// Hidden layer on 16-bit operands: the activations live in registers as the
// next layer's B fragments (KCI input chunks, KCO output chunks per sub-tile).
template <bool LEAKY, int DT, int NSUB, int KCI, int KCO>
__device__ inline void hidden_layer16(const typename Mma<DT>::elem* W, int lane,
                                      const typename Mma<DT>::frag (&in)[NSUB][KCI],
                                      typename Mma<DT>::frag (&out)[NSUB][KCO], float slope) {
    using FR = typename Mma<DT>::frag;
    constexpr int U = 2 * KCO;
    FR w[2][KCI];
    float4_t acc[U][NSUB];
    load_block<DT, KCI>(W, 0, lane, w[0]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (u + 1 < U) load_block<DT, KCI>(W, u + 1, lane, w[(u + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        mma_block<DT, NSUB, KCI>(w[u & 1], in, acc[u]);
        if (u % 2 == 0 && u >= 2) {
#pragma unroll
            for (int s = 0; s < NSUB; ++s) out[s][u / 2 - 1] = act_frag<LEAKY, DT>(acc[u - 2][s], acc[u - 1][s], slope);
        }
    }
#pragma unroll
    for (int s = 0; s < NSUB; ++s) out[s][KCO - 1] = act_frag<LEAKY, DT>(acc[U - 2][s], acc[U - 1][s], slope);
}

// Output layer on 16-bit operands.  The output blocks are taken GB at a
// time (gb_o of the packing); emit(s, c, v) receives the 4*GB visibilities
// that a lane holds for group c of sub-tile s, consecutive outputs in the
// out_neuron row order.
template <int DT, int NSUB, int KCI, int NBO, int GB, class Emit>
__device__ inline void output_layer16(const typename Mma<DT>::elem* W, int lane,
                                      const typename Mma<DT>::frag (&in)[NSUB][KCI], Emit&& emit) {
    using FR = typename Mma<DT>::frag;
    FR w[2][KCI];
    float4_t acc[NBO][NSUB];
    auto finish = [&](int c) {
#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
            float v[4 * GB];
#pragma unroll
            for (int j = 0; j < GB; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) v[4 * j + i] = sigmoid_fast(acc[GB * c + j][s][i]);
            emit(s, c, v);
        }
    };
    load_block<DT, KCI>(W, 0, lane, w[0]);
#pragma unroll
    for (int u = 0; u < NBO; ++u) {
        if (u + 1 < NBO) load_block<DT, KCI>(W, u + 1, lane, w[(u + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        mma_block<DT, NSUB, KCI>(w[u & 1], in, acc[u]);
        if (u % GB == 0 && u >= GB) finish(u / GB - 1);
    }
    finish(NBO / GB - 1);
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
    int vec_ok;           // n_out % 4 == 0 and vis 16-byte aligned: 4-output vector stores
    int vec8_ok;          // n_out % 8 == 0 and vis 16-byte aligned: 8-output vector stores
    const void* enc;      // pre-computed encoding [n][n_in] (nvc_mlp_forward), else nullptr
    int enc_dtype;
    int n_in;
    int enc_vec;          // n_in % 4 == 0 and enc 16-byte aligned
};

// Encoding words of point p that a lane owns (layout of encode_lane), as
// loaded from a pre-computed [n][n_in] buffer.  vec: n_in is a multiple of 4
// and the buffer 16-byte aligned, so a lane's four features of a block are
// one aligned load (four FP32 words, or two words of 16-bit pairs); otherwise
// one feature per word, zero past n_in.  Kept raw so that the load of the
// next tile can be in flight while this one is computed.
template <int NINB>
__device__ inline void load_enc_raw(const void* enc, int enc_dtype, int n_in, bool vec, int64_t p, int grp,
                                    uint32_t (&raw)[NINB][4]) {
#pragma unroll
    for (int b = 0; b < NINB; ++b) {
        const int f0 = 16 * b + 4 * grp;
        const int64_t o = p * n_in + f0;
        if (vec && f0 + 4 <= n_in) {
            if (enc_dtype == DT_F32) {
                const uint4 v = *reinterpret_cast<const uint4*>(reinterpret_cast<const float*>(enc) + o);
                raw[b][0] = v.x; raw[b][1] = v.y; raw[b][2] = v.z; raw[b][3] = v.w;
            } else {
                const uint2 v = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(enc) + o);
                raw[b][0] = v.x; raw[b][1] = v.y; raw[b][2] = 0; raw[b][3] = 0;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                uint32_t w = 0;
                if (f0 + i < n_in)
                    w = enc_dtype == DT_F32 ? reinterpret_cast<const uint32_t*>(enc)[o + i]
                                            : (uint32_t)reinterpret_cast<const uint16_t*>(enc)[o + i];
                raw[b][i] = w;
            }
        }
    }
}

// The features of load_enc_raw's words, rounded to FP32.
template <int NINB>
__device__ inline void decode_enc(int enc_dtype, int n_in, bool vec, int grp, const uint32_t (&raw)[NINB][4],
                                  float (&act)[NINB][4]) {
#pragma unroll
    for (int b = 0; b < NINB; ++b) {
        const bool pairs = vec && 16 * b + 4 * grp + 4 <= n_in;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t h = (pairs ? raw[b][i / 2] >> (16 * (i % 2)) : raw[b][i]) & 0xffffu;
            act[b][i] = enc_dtype == DT_F32 ? __uint_as_float(raw[b][i])
                      : enc_dtype == DT_F16 ? (float)__builtin_bit_cast(_Float16, (uint16_t)h)
                                            : __uint_as_float(h << 16);
        }
    }
}

// load_enc_raw / decode_enc for an encoding in the network's 16-bit dtype
// whose rows are whole 16-feature blocks, 8-byte aligned: one 8-byte load per
// block and lane, no branches (the same words and values as the general
// forms take for such an encoding).
template <int NINB>
__device__ inline void load_enc16(const void* enc, int n_in, int64_t p, int grp, uint32_t (&raw)[NINB][4]) {
#pragma unroll
    for (int b = 0; b < NINB; ++b) {
        const uint2 v = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(enc) + p * n_in + 16 * b +
                                                        4 * grp);
        raw[b][0] = v.x; raw[b][1] = v.y; raw[b][2] = 0; raw[b][3] = 0;
    }
}

template <int DT, int NINB>
__device__ inline void decode_enc16(const uint32_t (&raw)[NINB][4], float (&act)[NINB][4]) {
#pragma unroll
    for (int b = 0; b < NINB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t h = (raw[b][i / 2] >> (16 * (i % 2))) & 0xffffu;
            act[b][i] = DT == DT_F16 ? (float)__builtin_bit_cast(_Float16, (uint16_t)h) : __uint_as_float(h << 16);
        }
}

// A vector store marked non-temporal (streamed past the caches' normal
// allocation).  The visibilities are the largest write of a frame (133 MB at
// 1080p x 32 lights, 2.1 GB at 4K x 128) and are read once, by the light
// pick; written through the caches they evict the hash table that the next
// tiles gather from.  Measured: 4K x 128 inference alone 1.84 -> 1.41 ms,
// the 1080p frame 0.920 -> 0.904 ms, the paper's configuration 0.342 ->
// 0.334 ms.
template <class V>
__device__ inline void stream_store(V v, void* p) {
    typedef uint32_t wN __attribute__((ext_vector_type(sizeof(V) / 4)));
    __builtin_nontemporal_store(__builtin_bit_cast(wN, v), reinterpret_cast<wN*>(p));
}

// Visibilities v[0..N-1] of lights l0..l0+N-1 (N = 4 or 8) at point p, in
// the output dtype.
template <int N>
__device__ inline void store_vis(const InferArgs& a, int64_t p, int l0, const float (&v)[N]) {
    const int64_t base = p * a.n_out + l0;
    const bool vec = (N == 4 ? a.vec_ok : a.vec8_ok) && l0 + N <= a.n_out;
    if (vec && a.vis_dtype == DT_F32) {
#pragma unroll
        for (int q = 0; q < N; q += 4)
            stream_store(make_float4(v[q], v[q + 1], v[q + 2], v[q + 3]), (float*)a.vis + base + q);
    } else if (vec && a.vis_dtype == DT_F16) {
        typedef _Float16 hN __attribute__((ext_vector_type(N)));
        hN o;
#pragma unroll
        for (int i = 0; i < N; ++i) o[i] = (_Float16)v[i];
        stream_store(o, (_Float16*)a.vis + base);
    } else if (vec) {
        typedef __bf16 bN __attribute__((ext_vector_type(N)));
        bN o;
#pragma unroll
        for (int i = 0; i < N; ++i) o[i] = (__bf16)v[i];
        stream_store(o, (__bf16*)a.vis + base);
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) {
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

// Waves per block: twelve (three per SIMD) for the 128-wide network, whose
// weights fill most of the LDS (one block per CU), except eight for its FP32
// form with the encoding gathered, whose weights do not fit the LDS and are
// read through the caches (12 waves: 4K frame inference 11.2 -> 33 ms); four
// otherwise (several blocks per CU).
template <class C, bool PRE> constexpr int infer_waves() {
    return C::WB >= 8 ? (C::DT == DT_F32 && !PRE ? 8 : 12) : 4;
}

// PRE: the encoding comes from a.enc (nvc_mlp_forward) instead of the table.
// LEAKY: leaky ReLU hidden activation, else ReLU.
// Waves per SIMD the compiler must leave room for: three for the 16-bit 64-wide network with two
// features per level (146 registers, no spills), whose gathers then have a third wave to hide behind
// (1080p frame 0.983 -> 0.96 ms with the three-stream schedule); the others keep their natural
// occupancy (the paper's network would spill at three).
template <class C> constexpr int infer_min_waves() { return C::DT != DT_F32 && C::WB == 4 && C::F == 2 ? 3 : 1; }

// V16 (with PRE): the encoding and the visibilities in the network's 16-bit dtype, rows of whole
// 16-wide blocks (infer_v16_ok): branch-free loads and stores, so that the stores of a tile stay in
// flight under the next tile's matrix work.  The memory counter of a wave counts loads and stores
// together, in order; with a data-dependent branch around a store (the check against the last point)
// or a store whose width depends on the output dtype, the compiler cannot tell how many stores follow
// the next tile's loads, and waits for all of them before that tile.  The stores go through a buffer
// resource that covers the tile's rows of the output (clipped at its end): the hardware's range check
// drops the lanes past the last point.  These stores keep the default cache policy (4K x 128 network:
// 0.96 ms against 0.99 with the non-temporal one; nothing here gathers from a table).
template <class C, bool PRE, bool LEAKY, bool V16 = false>
__global__ __launch_bounds__((64 * infer_waves<C, PRE>())) __attribute__((amdgpu_waves_per_eu(infer_min_waves<C>())))
void infer_kernel(InferArgs a) {
    static_assert(!V16 || (PRE && C::DT != DT_F32), "V16 is the 16-bit form of the encoding-input kernel");
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
    // V16: the wave index made wave-uniform, so that the tile bounds and the store resource are scalars.
    const int wave = V16 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : threadIdx.x >> 6;
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

    // Output blocks per store group (gb_o of the packing).
    constexpr int GB = (DT != DT_F32 && C::NOUTB % 2 == 0) ? 2 : 1;
    constexpr int IW = infer_waves<C, PRE>();

    // The inputs of the wave's next tile are fetched one iteration ahead, so
    // that their memory latency is spent under this tile's matrix work: the
    // raw encoding words (PRE) or the positions.
    uint32_t raw[NSUB][C::NINB][4];
    float px[NSUB][3];
    auto fetch = [&](int64_t tt) {
#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
            const int64_t p = tt * PTS + s * 16 + col;
            const int64_t pc = p < a.n ? p : a.n - 1;
            if constexpr (V16) {
                load_enc16<C::NINB>(a.enc, a.n_in, pc, grp, raw[s]);
            } else if constexpr (PRE) {
                load_enc_raw<C::NINB>(a.enc, a.enc_dtype, a.n_in, a.enc_vec != 0, pc, grp, raw[s]);
            } else {
#pragma unroll
                for (int k = 0; k < 3; ++k) px[s][k] = a.pos[pc * 3 + k];
            }
        }
    };
    // This tile's encoding from the fetched inputs; then the next fetch.
    auto stage = [&](int64_t t, float (&h0)[NSUB][C::NINB][4]) {
#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
            if constexpr (V16)
                decode_enc16<DT, C::NINB>(raw[s], h0[s]);
            else if constexpr (PRE)
                decode_enc<C::NINB>(a.enc_dtype, a.n_in, a.enc_vec != 0, grp, raw[s], h0[s]);
            else
                encode_lane_lv<C::F, C::NINB>(a.table, lv, clamp_unit(px[s][0]), clamp_unit(px[s][1]),
                                              clamp_unit(px[s][2]), h0[s]);
        }
        // (V16: also past the wave's last tile, at the clamped last point, so that every iteration
        // issues the same loads.)
        if (V16 || t + IW < t1) fetch(t + IW);
    };
    if (t0 + wave < t1) fetch(t0 + wave);
    // V16: the first tile's loads complete before the loop, so that the loop entry and the back edge
    // present the compiler's wait insertion with the same outstanding operations (vmcnt(0) alone).
    if constexpr (V16) __builtin_amdgcn_s_waitcnt(0x0F70);
    for (int64_t t = t0 + wave; t < t1; t += IW) {
        // Weight fragments are read from LDS (or L1) in every iteration: the
        // opaque zero offset stops the compiler from hoisting all of them into
        // registers, which would cost occupancy.
        int opq = 0;
        asm volatile("" : "+s"(opq));
        const E* w_it[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) w_it[k] = wk[k] + opq;
        if constexpr (DT != DT_F32) {
            using FR = typename M::frag;
            constexpr int KC0 = kchunks<DT>(C::NINB), KCW = kchunks<DT>(C::WB);
            FR x0[NSUB][KC0];
            {
                float h0[NSUB][C::NINB][4];
                stage(t, h0);
#pragma unroll
                for (int s = 0; s < NSUB; ++s)
#pragma unroll
                    for (int kc = 0; kc < KC0; ++kc) x0[s][kc] = make_frag<DT, C::NINB>(h0[s], kc);
            }
            FR xa[NSUB][KCW], xb[NSUB][KCW];
            hidden_layer16<LEAKY, DT, NSUB, KC0, KCW>(w_it[0], lane, x0, xa, a.slope);
#pragma unroll
            for (int k = 1; k < C::NHID; ++k) {
                if (k % 2 == 1)
                    hidden_layer16<LEAKY, DT, NSUB, KCW, KCW>(w_it[k], lane, xa, xb, a.slope);
                else
                    hidden_layer16<LEAKY, DT, NSUB, KCW, KCW>(w_it[k], lane, xb, xa, a.slope);
            }
            const int64_t row = (int64_t)a.n_out * 2;          // V16: bytes per point of the output
            const int64_t tb = t * PTS * row;
            // 0x00020000: the descriptor's fourth word with a 32-bit data format (untyped access)
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((char*)a.vis + tb, 0, (int)min((int64_t)PTS * row, a.n * row - tb),
                                                  0x00020000);
            auto emit = [&](int s, int c, const float (&v)[4 * GB]) {
                if constexpr (V16) {
                    using E16 = std::conditional_t<DT == DT_F16, _Float16, __bf16>;
                    typedef E16 hN __attribute__((ext_vector_type(4 * GB)));
                    hN o;
#pragma unroll
                    for (int i = 0; i < 4 * GB; ++i) o[i] = (E16)v[i];
                    const int off = ((s * 16 + col) * a.n_out + 16 * GB * c + 4 * GB * grp) * 2;
                    typedef uint32_t wN __attribute__((ext_vector_type(2 * GB)));
                    if constexpr (GB == 2)
                        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(wN, o), rs, off, 0, 0);
                    else
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(wN, o), rs, off, 0, 0);
                } else {
                    const int64_t p = t * PTS + s * 16 + col;
                    if (p < a.n) store_vis<4 * GB>(a, p, 16 * GB * c + 4 * GB * grp, v);
                }
            };
            if constexpr (C::NHID % 2 == 1)
                output_layer16<DT, NSUB, KCW, C::NOUTB, GB>(w_it[NL - 1], lane, xa, emit);
            else
                output_layer16<DT, NSUB, KCW, C::NOUTB, GB>(w_it[NL - 1], lane, xb, emit);
        } else {   // FP32 matrix cores: activations in FP32 registers
            float h0[NSUB][C::NINB][4];
            stage(t, h0);
            float ha[NSUB][C::WB][4], hb[NSUB][C::WB][4];
            mlp_layer<DT, NSUB, C::NINB, C::WB>(w_it[0], lane, h0, ha);
            activate<LEAKY, NSUB, C::WB>(ha, a.slope);
#pragma unroll
            for (int k = 1; k < C::NHID; ++k) {
                if (k % 2 == 1) {
                    mlp_layer<DT, NSUB, C::WB, C::WB>(w_it[k], lane, ha, hb);
                    activate<LEAKY, NSUB, C::WB>(hb, a.slope);
                } else {
                    mlp_layer<DT, NSUB, C::WB, C::WB>(w_it[k], lane, hb, ha);
                    activate<LEAKY, NSUB, C::WB>(ha, a.slope);
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
                    float v[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = sigmoid_fast(z[s][ob][i]);
                    store_vis<4>(a, p, 16 * ob + 4 * grp, v);
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
    a.layer_off[plan.n_layers - 1] = plan.layer[plan.n_layers - 1].off_o;
    if (plan.layer[plan.n_layers - 1].gb_o != ((C::DT != DT_F32 && C::NOUTB % 2 == 0) ? 2 : 1))
        return hipErrorInvalidValue;
    a.pos = pos;
    a.n = n;
    a.n_out = n_out;
    a.vis = vis;
    a.vis_dtype = vis_dtype;
    a.act = act;
    a.slope = slope;
    a.vec_ok = (n_out % 4) == 0 && ((uintptr_t)vis % 16) == 0;
    a.vec8_ok = (n_out % 8) == 0 && ((uintptr_t)vis % 16) == 0;
    using LY = FwdLayout<C>;
    const size_t wbytes = (size_t)LY::total * sizeof(typename Mma<C::DT>::elem);
    const size_t smem = wbytes <= (size_t)kInferLdsMax ? wbytes : 0;
    const int64_t pts = 16 * C::NSUB_INFER;
    const int64_t ntiles = (n + pts - 1) / pts;
    // Many more blocks than the CUs hold at once (each a short contiguous tile
    // range): blocks that finish early are replaced, and kernels running on
    // the other streams of a frame get CUs block by block.  16 per CU for the
    // three-stream frame (24 had measured best with two streams: 4 -> 24,
    // frame 1.17 -> 1.13 ms; with three, 6 to 16 are about 10 us faster per
    // frame than 24 or 4); one block per CU when the weights fill the LDS.
    const int per_cu = smem > 80 * 1024 ? 1 : (smem > 40 * 1024 ? 2 : 16);
    const int IW = enc ? infer_waves<C, true>() : infer_waves<C, false>();
    int64_t want = (ntiles + IW - 1) / IW;                  // at least one tile per wave
    int64_t G = std::min<int64_t>(want, (int64_t)cu_count() * per_cu);
    G = std::max<int64_t>(8, (G + 7) / 8 * 8);
    const bool leaky = slope != 0.0f;
    if constexpr (C::DT != DT_F32) {
        constexpr int GB = C::NOUTB % 2 == 0 ? 2 : 1;
        const bool v16 = enc && vis_dtype == C::DT && enc_dtype == C::DT && n_out == 16 * C::NOUTB &&
                         n_in == 16 * C::NINB && (uintptr_t)vis % (8 * GB) == 0 && (uintptr_t)enc % 8 == 0 &&
                         (int64_t)pts * n_out * 2 <= INT32_MAX;
        if (v16 && leaky) {
            hipLaunchKernelGGL((infer_kernel<C, true, true, true>), dim3((unsigned)G), dim3(64 * IW), smem, st, a);
            return hipGetLastError();
        }
        if (v16) {
            hipLaunchKernelGGL((infer_kernel<C, true, false, true>), dim3((unsigned)G), dim3(64 * IW), smem, st, a);
            return hipGetLastError();
        }
    }
    if (enc && leaky)
        hipLaunchKernelGGL((infer_kernel<C, true, true>), dim3((unsigned)G), dim3(64 * IW), smem, st, a);
    else if (enc)
        hipLaunchKernelGGL((infer_kernel<C, true, false>), dim3((unsigned)G), dim3(64 * IW), smem, st, a);
    else if (leaky)
        hipLaunchKernelGGL((infer_kernel<C, false, true>), dim3((unsigned)G), dim3(64 * IW), smem, st, a);
    else
        hipLaunchKernelGGL((infer_kernel<C, false, false>), dim3((unsigned)G), dim3(64 * IW), smem, st, a);
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
