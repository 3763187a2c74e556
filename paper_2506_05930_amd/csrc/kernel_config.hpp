// Network shapes the kernels are built for.  Each configuration fixes the
// register layout of the MLP at compile time; the host dispatches on
// (dtype, features per level, padded input blocks, width, hidden layers,
// output blocks).  Shapes outside this list return NVC_ERR_UNSUPPORTED.
#pragma once

#include "nvc_internal.hpp"

namespace nvc {

// DT: matrix-core dtype.  NINB: 16-neuron blocks of the input after padding
// to the K granule (f32: 16, f16/bf16: 32).  WB: width / 16.  NOUTB: output
// blocks (n_out padded to 16).  NHID: hidden layers.  F: features per level.
// NSUB: 16-point sub-tiles per wave in the inference kernel (weight-fragment
// reuse vs. registers).
template <int DT_, int NINB_, int WB_, int NOUTB_, int NHID_, int F_, int NSUB_>
struct Cfg {
    static constexpr int DT = DT_, NINB = NINB_, WB = WB_, NOUTB = NOUTB_, NHID = NHID_, F = F_,
                         NSUB_INFER = NSUB_;
};

template <class T> struct Tag { using type = T; };

template <class Fn> inline void for_each_config(Fn&& f) {
    // 16 -> 32 -> 32 -> 8 (small unit-cube workload)
    f(Tag<Cfg<DT_F32, 1, 2, 1, 2, 2, 2>>{});
    f(Tag<Cfg<DT_F16, 2, 2, 1, 2, 2, 2>>{});
    f(Tag<Cfg<DT_BF16, 2, 2, 1, 2, 2, 2>>{});
    // 32 -> 64 -> 64 -> 64 -> 32 (1080p workload)
    f(Tag<Cfg<DT_F16, 2, 4, 2, 3, 2, 2>>{});
    f(Tag<Cfg<DT_BF16, 2, 4, 2, 3, 2, 2>>{});
    f(Tag<Cfg<DT_F32, 2, 4, 2, 3, 2, 2>>{});
    // 32 -> 128 -> 128 -> 128 -> 128 (4K, 128-light workload)
    f(Tag<Cfg<DT_F16, 2, 8, 8, 3, 2, 2>>{});
    f(Tag<Cfg<DT_BF16, 2, 8, 8, 3, 2, 2>>{});
    f(Tag<Cfg<DT_F32, 2, 8, 8, 3, 2, 1>>{});
    // 32 -> 32 -> 32 -> 32 (clustered cache: eight levels of four features, 32 clusters, Sec. 3.6)
    f(Tag<Cfg<DT_F16, 2, 2, 2, 2, 4, 2>>{});
    f(Tag<Cfg<DT_BF16, 2, 2, 2, 2, 4, 2>>{});
    f(Tag<Cfg<DT_F32, 2, 2, 2, 2, 4, 2>>{});
    // 40 -> 32 -> 32 -> 32 (the paper's network: ten levels of four features, Sec. 3.3)
    f(Tag<Cfg<DT_F16, 4, 2, 2, 2, 4, 2>>{});
    f(Tag<Cfg<DT_BF16, 4, 2, 2, 2, 4, 2>>{});
    f(Tag<Cfg<DT_F32, 3, 2, 2, 2, 4, 2>>{});
}

// Padded input blocks for n_in features.
inline int padded_in_blocks(int dtype, int n_in) {
    return dtype == DT_F32 ? (n_in + 15) / 16 : (n_in + 31) / 32 * 2;
}

template <class C> inline bool cfg_matches(int n_feat, const NetShape& s) {
    return s.dtype == C::DT && n_feat == C::F && padded_in_blocks(s.dtype, s.n_in) == C::NINB &&
           s.width == C::WB * 16 && s.n_hidden == C::NHID && (s.n_out + 15) / 16 == C::NOUTB;
}

// Calls f.template operator()<C>() for the first built configuration matching the shape.
template <class Fn> inline bool dispatch_config(int n_feat, const NetShape& s, Fn&& f) {
    bool done = false;
    for_each_config([&](auto tag) {
        using C = typename decltype(tag)::type;
        if (!done && cfg_matches<C>(n_feat, s)) {
            f.template operator()<C>();
            done = true;
        }
    });
    return done;
}

int cu_count();

}  // namespace nvc
