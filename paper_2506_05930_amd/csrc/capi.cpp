// C ABI of the cache (declared in include/nvc.h): argument validation on the
// host, translation to the internal shapes, kernel launches.  Nothing here
// allocates, synchronises or keeps state.
#include <math.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "nvc.h"
#include "nvc_internal.hpp"

using namespace nvc;

namespace {

bool valid_dtype(int32_t dt) { return dt == NVC_F32 || dt == NVC_F16 || dt == NVC_BF16; }

int check_grid(const nvc_grid* g, GridHost* out) {
    if (!g) return NVC_ERR_NULL;
    if (g->n_levels < 1 || g->n_levels > kMaxLevels) return NVC_ERR_SHAPE;
    if (g->n_feat != 1 && g->n_feat != 2 && g->n_feat != 4) return NVC_ERR_UNSUPPORTED;
    if (g->n_levels * g->n_feat > 64) return NVC_ERR_UNSUPPORTED;
    if (g->log2_T < 10 || g->log2_T > 24) return NVC_ERR_SHAPE;
    if (g->base_res < 1 || !(g->growth >= 1.0) || !isfinite(g->growth)) return NVC_ERR_SHAPE;
    GridHost h{};
    h.n_levels = g->n_levels;
    h.n_feat = g->n_feat;
    h.log2_T = g->log2_T;
    const double T = (double)(1u << g->log2_T);
    for (int l = 0; l < g->n_levels; ++l) {
        // N_l = floor(base * growth^l) in FP64 (Mueller et al. 2022, eq. 2).
        const double r = floor((double)g->base_res * pow(g->growth, (double)l));
        if (!(r >= 1.0) || r > 16777215.0) return NVC_ERR_SHAPE;     // N + 1 must stay exact in FP32
        h.res[l] = (int32_t)r;
        const double v = (r + 1.0) * (r + 1.0) * (r + 1.0);
        if (v <= T) h.dense_mask |= 1u << l;
    }
    if (out) *out = h;
    return NVC_OK;
}

int check_mlp(const nvc_mlp* m, NetShape* out) {
    if (!m) return NVC_ERR_NULL;
    if (!valid_dtype(m->dtype)) return NVC_ERR_DTYPE;
    if (m->n_in < 1 || m->width < 1 || m->n_hidden < 1 || m->n_out < 1) return NVC_ERR_SHAPE;
    if (m->n_hidden + 1 > kMaxLayers) return NVC_ERR_UNSUPPORTED;
    if (m->n_out > 128 || m->n_in > 64 || m->width > 128) return NVC_ERR_UNSUPPORTED;
    if (m->act != NVC_ACT_RELU && m->act != NVC_ACT_LEAKY) return NVC_ERR_SHAPE;
    if (m->act == NVC_ACT_LEAKY && !(m->leaky_slope >= 0.0f && m->leaky_slope <= 1.0f)) return NVC_ERR_SHAPE;
    NetShape s{};
    s.dtype = m->dtype;
    s.n_in = m->n_in;
    s.width = m->width;
    s.n_hidden = m->n_hidden;
    s.n_out = m->n_out;
    s.act = m->act;
    s.slope = m->act == NVC_ACT_LEAKY ? m->leaky_slope : 0.0f;
    if (out) *out = s;
    return NVC_OK;
}

int check_net(const nvc_grid* g, const nvc_mlp* m, GridHost* gh, NetShape* s) {
    int st = check_grid(g, gh);
    if (st) return st;
    st = check_mlp(m, s);
    if (st) return st;
    if (m->n_in != g->n_levels * g->n_feat) return NVC_ERR_SHAPE;
    return NVC_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? NVC_OK : NVC_ERR_HIP; }

}  // namespace

extern "C" {

int nvc_version(void) { return NVC_VERSION; }

const char* nvc_status_string(int status) {
    switch (status) {
        case NVC_OK: return "ok";
        case NVC_ERR_NULL: return "a required pointer is NULL";
        case NVC_ERR_SHAPE: return "a size is negative, inconsistent or out of range";
        case NVC_ERR_DTYPE: return "unknown dtype code";
        case NVC_ERR_UNSUPPORTED: return "shape or option not built into this library";
        case NVC_ERR_HIP: return "a HIP launch failed";
        case NVC_ERR_WORKSPACE: return "workspace missing or too small";
        default: return "unknown status";
    }
}

int nvc_grid_levels(const nvc_grid* grid, int32_t* res, int32_t* dense) {
    GridHost h{};
    const int st = check_grid(grid, &h);
    if (st) return st;
    for (int l = 0; l < h.n_levels; ++l) {
        if (res) res[l] = h.res[l];
        if (dense) dense[l] = (h.dense_mask >> l) & 1u;
    }
    return NVC_OK;
}

int64_t nvc_mlp_param_count(const nvc_mlp* mlp) {
    NetShape s{};
    const int st = check_mlp(mlp, &s);
    if (st) return st;
    return (int64_t)s.n_in * s.width + (int64_t)(s.n_hidden - 1) * s.width * s.width + (int64_t)s.width * s.n_out;
}

int64_t nvc_mlp_packed_bytes(const nvc_mlp* mlp) {
    NetShape s{};
    const int st = check_mlp(mlp, &s);
    if (st) return st;
    const PackPlan p = make_pack_plan(s);
    return p.total_elems * (int64_t)dtype_size(s.dtype);
}

int nvc_pack_mlp(const nvc_mlp* mlp, const float* w, void* packed, void* stream) {
    NetShape s{};
    const int st = check_mlp(mlp, &s);
    if (st) return st;
    if (!w || !packed) return NVC_ERR_NULL;
    const PackPlan p = make_pack_plan(s);
    return hip_status(launch_pack(s, p, w, packed, (hipStream_t)stream));
}

int nvc_encode(const nvc_grid* grid, const float* table, const float* pos, int64_t n, void* enc, int32_t enc_dtype,
               void* stream) {
    GridHost g{};
    const int st = check_grid(grid, &g);
    if (st) return st;
    if (!valid_dtype(enc_dtype)) return NVC_ERR_DTYPE;
    if (n < 0) return NVC_ERR_SHAPE;
    if (n == 0) return NVC_OK;
    if (!table || !pos || !enc) return NVC_ERR_NULL;
    if (n > ((int64_t)1 << 40) / g.n_levels) return NVC_ERR_SHAPE;
    return hip_status(launch_encode(g, table, pos, n, enc, enc_dtype, (hipStream_t)stream));
}

int nvc_infer(const nvc_grid* grid, const nvc_mlp* mlp, const float* table, const void* packed, const float* pos,
              int64_t n, void* vis, int32_t vis_dtype, void* stream) {
    GridHost g{};
    NetShape s{};
    const int st = check_net(grid, mlp, &g, &s);
    if (st) return st;
    if (!valid_dtype(vis_dtype)) return NVC_ERR_DTYPE;
    if (n < 0) return NVC_ERR_SHAPE;
    if (!infer_supported(g, s)) return NVC_ERR_UNSUPPORTED;
    if (n == 0) return NVC_OK;
    if (!table || !packed || !pos || !vis) return NVC_ERR_NULL;
    const PackPlan p = make_pack_plan(s);
    return hip_status(launch_infer(g, s, p, table, packed, pos, n, vis, vis_dtype, (hipStream_t)stream));
}

int nvc_mlp_forward(const nvc_mlp* mlp, const void* packed, const void* enc, int32_t enc_dtype, int64_t n, void* vis,
                    int32_t vis_dtype, void* stream) {
    NetShape s{};
    const int st = check_mlp(mlp, &s);
    if (st) return st;
    if (!valid_dtype(enc_dtype) || !valid_dtype(vis_dtype)) return NVC_ERR_DTYPE;
    if (n < 0) return NVC_ERR_SHAPE;
    if (!mlp_supported(s)) return NVC_ERR_UNSUPPORTED;
    if (n == 0) return NVC_OK;
    if (!packed || !enc || !vis) return NVC_ERR_NULL;
    const PackPlan p = make_pack_plan(s);
    return hip_status(launch_mlp_forward(s, p, packed, enc, enc_dtype, n, vis, vis_dtype, (hipStream_t)stream));
}

int nvc_sample_wrs(const void* vis, int32_t vis_dtype, int64_t n, int32_t m, const float* pos, const float* nrm,
                   const float* lights, float vis_floor, uint64_t seed, uint32_t frame, const nvc_counters* ctr,
                   int32_t* idx, float* pmf, float* wsum, float* di, const uint8_t* mask, nvc_reservoir* res,
                   void* stream) {
    if (!valid_dtype(vis_dtype)) return NVC_ERR_DTYPE;
    if (n < 0 || m < 1 || m > 128) return NVC_ERR_SHAPE;
    if (!(vis_floor >= 0.0f) || !isfinite(vis_floor)) return NVC_ERR_SHAPE;
    if (n == 0) return NVC_OK;
    if (!vis || !pos || !lights || !idx || !pmf || !wsum) return NVC_ERR_NULL;
    return hip_status(launch_wrs(vis, vis_dtype, n, m, pos, nrm, lights, vis_floor, seed, frame,
                                 ctr ? &ctr->frame : nullptr, idx, pmf, wsum, di, mask, res, (hipStream_t)stream));
}

int64_t nvc_select_pixels_workspace_bytes(int64_t n_pix) {
    if (n_pix < 1 || n_pix >= ((int64_t)1 << 31)) return NVC_ERR_SHAPE;
    return select_pixels_workspace_bytes(n_pix);
}

int nvc_select_pixels(uint64_t seed, uint32_t frame, const nvc_counters* ctr, int64_t n_pix, int64_t batch,
                      int32_t* pix, void* workspace, int64_t workspace_bytes, void* stream) {
    if (n_pix < 1 || n_pix >= ((int64_t)1 << 31) || batch < 0 || batch >= ((int64_t)1 << 31)) return NVC_ERR_SHAPE;
    if (batch == 0) return NVC_OK;
    if (!pix) return NVC_ERR_NULL;
    if (!workspace || workspace_bytes < select_pixels_workspace_bytes(n_pix)) return NVC_ERR_WORKSPACE;
    return hip_status(launch_select_pixels(seed, frame, ctr ? &ctr->frame : nullptr, n_pix, batch, pix, workspace,
                                           (hipStream_t)stream));
}

int nvc_select_pixels_noalloc(uint64_t seed, uint32_t frame, const nvc_counters* ctr, int64_t n_pix, int64_t batch,
                              int32_t* pix, void* stream) {
    if (n_pix < 1 || n_pix > select_pixels_noalloc_max_pixels() || batch < 0 || batch >= ((int64_t)1 << 31))
        return NVC_ERR_SHAPE;
    if (batch == 0) return NVC_OK;
    if (!pix) return NVC_ERR_NULL;
    return hip_status(launch_select_pixels_noalloc(seed, frame, ctr ? &ctr->frame : nullptr, n_pix, batch, pix,
                                                   (hipStream_t)stream));
}

int nvc_shadow_labels(const float* pos, const int32_t* pix, int64_t n, const float* lights, int32_t m,
                      const float* spheres, int32_t n_spheres, uint8_t* labels, void* stream) {
    if (n < 0 || m < 1 || m > 128 || n_spheres < 0 || n_spheres > 4096) return NVC_ERR_SHAPE;
    if (labels_smem_bytes(m, n_spheres) > 150 * 1024) return NVC_ERR_UNSUPPORTED;   // unreachable within the limits
    if (n == 0) return NVC_OK;
    if (!pos || !lights || !labels || (n_spheres > 0 && !spheres)) return NVC_ERR_NULL;
    return hip_status(launch_labels(pos, pix, n, lights, m, spheres, n_spheres, labels, (hipStream_t)stream));
}

int nvc_world_samples(uint64_t seed, uint32_t frame, const nvc_counters* ctr, int64_t n, const float* box,
                      float extent, float* pos_scene, float* pos_unit, void* stream) {
    if (n < 0 || !(extent > 0.0f) || !isfinite(extent)) return NVC_ERR_SHAPE;
    if (!box) return NVC_ERR_NULL;
    for (int k = 0; k < 3; ++k)
        if (!isfinite(box[k]) || !isfinite(box[k + 3]) || !(box[k] <= box[k + 3])) return NVC_ERR_SHAPE;
    if (n == 0) return NVC_OK;
    if (!pos_scene || !pos_unit) return NVC_ERR_NULL;
    return hip_status(launch_world_samples(seed, frame, ctr ? &ctr->frame : nullptr, n, box, extent, pos_scene,
                                           pos_unit, (hipStream_t)stream));
}

int nvc_cluster_lights(const float* lights, int32_t n_lights, int32_t k, int32_t iters, int32_t* offsets,
                       int32_t* members) {
    if (n_lights < 1 || k < 1 || k > 128 || k > n_lights || iters < 1) return NVC_ERR_SHAPE;
    if (!lights || !offsets || !members) return NVC_ERR_NULL;
    for (int64_t i = 0; i < 4 * (int64_t)n_lights; ++i)
        if (!isfinite(lights[i])) return NVC_ERR_SHAPE;
    cluster_lights_host(lights, n_lights, k, iters, offsets, members);
    return NVC_OK;
}

int nvc_shadow_labels_clustered(const float* pos, const int32_t* pix, int64_t n, const float* lights,
                                int32_t n_lights, const int32_t* offsets, const int32_t* members, int32_t k,
                                const float* spheres, int32_t n_spheres, uint64_t seed, uint32_t frame,
                                const nvc_counters* ctr, uint8_t* labels, void* stream) {
    if (n < 0 || k < 1 || k > 128 || n_lights < 0 || n_spheres < 0 || n_spheres > 4096) return NVC_ERR_SHAPE;
    if (n > ((int64_t)1 << 40) / k) return NVC_ERR_SHAPE;
    if (n == 0) return NVC_OK;
    if (!pos || !offsets || !labels || (n_lights > 0 && (!lights || !members)) || (n_spheres > 0 && !spheres))
        return NVC_ERR_NULL;
    return hip_status(launch_clustered_labels(pos, pix, n, lights, n_lights, offsets, members, k, spheres, n_spheres,
                                              seed, frame, ctr ? &ctr->frame : nullptr, labels, (hipStream_t)stream));
}

int nvc_sample_clustered(const void* vis, int32_t vis_dtype, int64_t n, int32_t k, const float* pos,
                         const float* nrm, const float* lights, int32_t n_lights, const int32_t* offsets,
                         const int32_t* members, float vis_floor, int32_t n_cand, uint64_t seed, uint32_t frame,
                         const nvc_counters* ctr, int32_t* idx, float* weight, int32_t* cluster,
                         const uint8_t* mask, nvc_reservoir* res, void* stream) {
    if (n < 0 || k < 1 || k > 128 || n_lights < 0 || n_cand < 1 || n_cand > 64) return NVC_ERR_SHAPE;
    if (vis_dtype != NVC_F32 && vis_dtype != NVC_F16 && vis_dtype != NVC_BF16) return NVC_ERR_DTYPE;
    if (!(vis_floor >= 0.0f) || !isfinite(vis_floor)) return NVC_ERR_SHAPE;
    if (n == 0) return NVC_OK;
    if (!vis || !pos || !offsets || !idx || !weight || (n_lights > 0 && (!lights || !members))) return NVC_ERR_NULL;
    return hip_status(launch_clustered_sample(vis, vis_dtype, n, k, pos, nrm, lights, n_lights, offsets, members,
                                              vis_floor, n_cand, seed, frame, ctr ? &ctr->frame : nullptr, idx,
                                              weight, cluster, mask, res, (hipStream_t)stream));
}

int64_t nvc_train_workspace_bytes(const nvc_grid* grid, const nvc_mlp* mlp, int64_t batch) {
    GridHost g{};
    NetShape s{};
    const int st = check_net(grid, mlp, &g, &s);
    if (st) return st;
    if (batch < 0) return NVC_ERR_SHAPE;
    if (!train_supported(g, s)) return NVC_ERR_UNSUPPORTED;
    if (batch == 0) return 0;
    return train_workspace_bytes(g, s, batch);
}

int nvc_train_step(const nvc_grid* grid, const nvc_mlp* mlp, const float* table, const void* packed, const float* pos,
                   const int32_t* pix, int64_t batch, const uint8_t* labels, const float* dvis, int32_t loss,
                   float grad_scale, float* g_table, float* g_w, float* loss_out, void* workspace,
                   int64_t workspace_bytes, void* stream) {
    GridHost g{};
    NetShape s{};
    const int st = check_net(grid, mlp, &g, &s);
    if (st) return st;
    if (batch < 0 || batch >= ((int64_t)1 << 31)) return NVC_ERR_SHAPE;
    if (loss != NVC_LOSS_BCE && loss != NVC_LOSS_L2) return NVC_ERR_SHAPE;
    if (!(grad_scale >= 0.0f) || !isfinite(grad_scale)) return NVC_ERR_SHAPE;
    if ((labels == nullptr) == (dvis == nullptr)) return labels ? NVC_ERR_SHAPE : NVC_ERR_NULL;
    if (!train_supported(g, s)) return NVC_ERR_UNSUPPORTED;
    if (batch == 0) return NVC_OK;
    if (!table || !packed || !pos || !g_table || !g_w) return NVC_ERR_NULL;
    const int64_t need = train_workspace_bytes(g, s, batch);
    if (!workspace || workspace_bytes < need) return NVC_ERR_WORKSPACE;
    const PackPlan p = make_pack_plan(s);
    return hip_status(launch_train(g, s, p, table, packed, pos, pix, batch, labels, dvis, loss, grad_scale, g_table,
                                   g_w, loss_out, workspace, (hipStream_t)stream));
}

int64_t nvc_train_plan_bytes(const nvc_grid* grid, const nvc_mlp* mlp, int64_t batch) {
    GridHost g{};
    NetShape s{};
    const int st = check_net(grid, mlp, &g, &s);
    if (st) return st;
    if (batch < 0 || batch >= ((int64_t)1 << 31)) return NVC_ERR_SHAPE;
    if (!train_supported(g, s)) return NVC_ERR_UNSUPPORTED;
    if (batch == 0) return 0;
    return train_plan_bytes(g, s, batch);
}

int nvc_train_plan(const nvc_grid* grid, const nvc_mlp* mlp, const float* pos, const int32_t* pix, int64_t batch,
                   void* plan, int64_t plan_bytes, void* stream) {
    GridHost g{};
    NetShape s{};
    const int st = check_net(grid, mlp, &g, &s);
    if (st) return st;
    if (batch < 0 || batch >= ((int64_t)1 << 31)) return NVC_ERR_SHAPE;
    if (!train_supported(g, s)) return NVC_ERR_UNSUPPORTED;
    if (batch == 0) return NVC_OK;
    const int64_t need = train_plan_bytes(g, s, batch);
    if (need == 0) return NVC_OK;
    if (!pos) return NVC_ERR_NULL;
    if (!plan || plan_bytes < need) return NVC_ERR_WORKSPACE;
    return hip_status(launch_train_plan(g, s, pos, pix, batch, plan, (hipStream_t)stream));
}

int nvc_train_step_planned(const nvc_grid* grid, const nvc_mlp* mlp, const float* table, const void* packed,
                           const float* pos, const int32_t* pix, int64_t batch, const uint8_t* labels,
                           const float* dvis, int32_t loss, float grad_scale, float* g_table, float* g_w,
                           float* loss_out, const void* plan, int64_t plan_bytes, void* workspace,
                           int64_t workspace_bytes, void* stream) {
    GridHost g{};
    NetShape s{};
    const int st = check_net(grid, mlp, &g, &s);
    if (st) return st;
    if (batch < 0 || batch >= ((int64_t)1 << 31)) return NVC_ERR_SHAPE;
    if (loss != NVC_LOSS_BCE && loss != NVC_LOSS_L2) return NVC_ERR_SHAPE;
    if (!(grad_scale >= 0.0f) || !isfinite(grad_scale)) return NVC_ERR_SHAPE;
    if ((labels == nullptr) == (dvis == nullptr)) return labels ? NVC_ERR_SHAPE : NVC_ERR_NULL;
    if (!train_supported(g, s)) return NVC_ERR_UNSUPPORTED;
    if (batch == 0) return NVC_OK;
    if (!table || !packed || !pos || !g_table || !g_w) return NVC_ERR_NULL;
    const int64_t need = train_workspace_bytes(g, s, batch);
    if (!workspace || workspace_bytes < need) return NVC_ERR_WORKSPACE;
    const int64_t pneed = train_plan_bytes(g, s, batch);
    if (pneed > 0 && (!plan || plan_bytes < pneed)) return NVC_ERR_WORKSPACE;
    const PackPlan p = make_pack_plan(s);
    return hip_status(launch_train_planned(g, s, p, table, packed, pos, pix, batch, labels, dvis, loss, grad_scale,
                                           g_table, g_w, loss_out, pneed > 0 ? plan : nullptr, workspace,
                                           (hipStream_t)stream));
}

int nvc_train_step_shadow(const nvc_grid* grid, const nvc_mlp* mlp, const float* table, const void* packed,
                          const float* pos, const float* pos_scene, const int32_t* pix, int64_t batch,
                          const float* lights, int32_t m, const float* spheres, int32_t n_spheres, int32_t loss,
                          float grad_scale, float* g_table, float* g_w, float* loss_out, uint8_t* labels_out,
                          void* workspace, int64_t workspace_bytes, void* stream) {
    GridHost g{};
    NetShape s{};
    const int st = check_net(grid, mlp, &g, &s);
    if (st) return st;
    if (batch < 0 || batch >= ((int64_t)1 << 31)) return NVC_ERR_SHAPE;
    if (loss != NVC_LOSS_BCE && loss != NVC_LOSS_L2) return NVC_ERR_SHAPE;
    if (!(grad_scale >= 0.0f) || !isfinite(grad_scale)) return NVC_ERR_SHAPE;
    if (m != s.n_out || m < 1 || m > NVC_TRAIN_SHADOW_MAX_LIGHTS) return NVC_ERR_SHAPE;
    if (n_spheres < 0 || n_spheres > NVC_TRAIN_SHADOW_MAX_SPHERES) return NVC_ERR_SHAPE;
    if (!train_shadow_supported(g, s, batch, n_spheres)) return NVC_ERR_UNSUPPORTED;
    if (batch == 0) return NVC_OK;
    if (!table || !packed || !pos || !pos_scene || !lights || !g_table || !g_w) return NVC_ERR_NULL;
    if (n_spheres > 0 && !spheres) return NVC_ERR_NULL;
    const int64_t need = train_workspace_bytes(g, s, batch);
    if (!workspace || workspace_bytes < need) return NVC_ERR_WORKSPACE;
    const PackPlan p = make_pack_plan(s);
    const ShadowArgs sh{pos_scene, lights, m, spheres, n_spheres, labels_out};
    return hip_status(launch_train_shadow(g, s, p, table, packed, pos, pix, batch, sh, loss, grad_scale, g_table, g_w,
                                          loss_out, workspace, (hipStream_t)stream));
}

int nvc_adam(float* p, float* g, float* m, float* v, int64_t count, int32_t step, const nvc_counters* ctr, float lr,
             float lr_end, int32_t lr_decay_steps, float beta1, float beta2, float eps, int32_t zero_grad,
             void* stream) {
    if (count < 0 || (!ctr && step < 1) || lr_decay_steps < 0) return NVC_ERR_SHAPE;
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f)) return NVC_ERR_SHAPE;
    if (!(lr >= 0.0f) || !isfinite(lr) || !(eps >= 0.0f) || !isfinite(eps)) return NVC_ERR_SHAPE;
    if (!(lr_end >= 0.0f) || !isfinite(lr_end)) return NVC_ERR_SHAPE;
    if (count == 0) return NVC_OK;
    if (!p || !g || !m || !v) return NVC_ERR_NULL;
    return hip_status(launch_adam(p, g, m, v, count, step, ctr ? &ctr->step : nullptr, lr, lr_end, lr_decay_steps,
                                  beta1, beta2, eps, zero_grad, (hipStream_t)stream));
}

int nvc_counters_advance(nvc_counters* ctr, void* stream) {
    if (!ctr) return NVC_ERR_NULL;
    return hip_status(launch_counters_advance(&ctr->frame, &ctr->step, (hipStream_t)stream));
}

int nvc_forward_f64(const nvc_grid* grid, const nvc_mlp* mlp, const double* table, const double* w,
                    const float* pos, int64_t n, const uint8_t* labels, int32_t loss, double* z, uint8_t* masks,
                    double* loss_out, void* stream) {
    GridHost g{};
    NetShape s{};
    const int st = check_net(grid, mlp, &g, &s);
    if (st) return st;
    if (n < 0 || n > ((int64_t)1 << 20)) return NVC_ERR_SHAPE;
    if (labels && loss != NVC_LOSS_BCE && loss != NVC_LOSS_L2) return NVC_ERR_SHAPE;
    if (n == 0) return NVC_OK;
    if (!table || !w || !pos) return NVC_ERR_NULL;
    if (labels && !loss_out) return NVC_ERR_NULL;
    return hip_status(launch_forward_f64(g, s, table, w, pos, n, labels, loss, z, masks, labels ? loss_out : nullptr,
                                         (hipStream_t)stream));
}

int nvc_graph_begin(void* stream) {
    if (!stream) return NVC_ERR_NULL;       // the legacy default stream cannot be captured
    return hip_status(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
}

int nvc_graph_end(void* stream, void** exec) {
    if (!stream || !exec) return NVC_ERR_NULL;
    *exec = nullptr;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture((hipStream_t)stream, &graph);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return NVC_ERR_HIP;
    }
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);           // the executable keeps what it needs
    if (e != hipSuccess) return NVC_ERR_HIP;
    *exec = (void*)ge;
    return NVC_OK;
}

int nvc_graph_launch(void* exec, void* stream) {
    if (!exec || !stream) return NVC_ERR_NULL;
    return hip_status(hipGraphLaunch((hipGraphExec_t)exec, (hipStream_t)stream));
}

int nvc_graph_destroy(void* exec) {
    if (!exec) return NVC_ERR_NULL;
    return hip_status(hipGraphExecDestroy((hipGraphExec_t)exec));
}

}  // extern "C"
