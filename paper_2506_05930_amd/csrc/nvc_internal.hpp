// Internal declarations shared by the C-ABI layer and the kernel translation units.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "nvc.h"

namespace nvc {

constexpr int DT_F32 = 0;
constexpr int DT_F16 = 1;
constexpr int DT_BF16 = 2;
constexpr int kMaxLevels = 32;

// Host copy of the level table, passed to kernels by value.
struct GridHost {
    int32_t n_levels;
    int32_t n_feat;
    int32_t log2_T;
    uint32_t dense_mask;
    int32_t res[kMaxLevels];
};

// Network shape after padding to matrix-core granules.
struct NetShape {
    int dtype;
    int n_in, width, n_hidden, n_out;
    int act;              // 0 relu, 1 leaky
    float slope;
};

// Packed-weight layout: per layer, the forward fragments then the transposed
// ones; after the output layer's, a copy of its forward fragments with the
// rows in the inference kernel's store order (out_neuron, gb_o = 2), or
// off_o = off_f when that order is the natural one (gb_o = 1).
struct LayerPack {
    int in, out;              // logical sizes
    int nb_out_f, kc_in_f;    // forward: 16-row blocks of `out`, K-chunks over `in`
    int nb_in_b, kc_out_b;    // backward: 16-row blocks of `in`, K-chunks over `out`
    int64_t off_f, off_b;     // element offsets into the packed buffer
    int64_t off_o;            // forward fragments in inference row order
    int gb_o;                 // output blocks per store group of the inference kernel
    int64_t w_off;            // float offset of this layer in the master weights
};

// Output neuron held in row r (0..15) of forward block ob for store groups of
// gb blocks.  gb = 2: a 16x16 matrix-core result gives lane group g = r/4 the
// rows 4g..4g+3 of a block, so group g of the block pair (2c, 2c+1) holds the
// eight consecutive neurons 32c + 8g + [0, 8).
__host__ __device__ constexpr int out_neuron(int ob, int r, int gb) {
    return gb == 2 ? 32 * (ob / 2) + 8 * (r / 4) + 4 * (ob % 2) + (r % 4) : 16 * ob + r;
}

constexpr int kMaxLayers = 8;

struct PackPlan {
    int n_layers;
    LayerPack layer[kMaxLayers];
    int64_t total_elems;
};

PackPlan make_pack_plan(const NetShape& s);
size_t dtype_size(int dt);

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_pack(const NetShape& s, const PackPlan& plan, const float* w, void* packed, hipStream_t st);
hipError_t launch_encode(const GridHost& g, const float* table, const float* pos, int64_t n, void* enc,
                         int enc_dtype, hipStream_t st);
// Returns hipErrorNotSupported (without launching) if no kernel is built for this shape.
hipError_t launch_infer(const GridHost& g, const NetShape& s, const PackPlan& plan, const float* table,
                        const void* packed, const float* pos, int64_t n, void* vis, int vis_dtype, hipStream_t st);
bool infer_supported(const GridHost& g, const NetShape& s);
bool mlp_supported(const NetShape& s);
hipError_t launch_mlp_forward(const NetShape& s, const PackPlan& plan, const void* packed, const void* enc,
                              int enc_dtype, int64_t n, void* vis, int vis_dtype, hipStream_t st);
hipError_t launch_wrs(const void* vis, int vis_dtype, int64_t n, int m, const float* pos, const float* nrm,
                      const float* lights, float vis_floor, uint64_t seed, uint32_t frame,
                      const uint32_t* frame_dev, int32_t* idx, float* pmf, float* wsum, float* di,
                      const uint8_t* mask, nvc_reservoir* res, hipStream_t st);
int64_t select_pixels_workspace_bytes(int64_t n_pix);
hipError_t launch_select_pixels(uint64_t seed, uint32_t frame, const uint32_t* frame_dev, int64_t n_pix,
                                int64_t batch, int32_t* pix, void* workspace, hipStream_t st);
int64_t select_pixels_noalloc_max_pixels();
hipError_t launch_select_pixels_noalloc(uint64_t seed, uint32_t frame, const uint32_t* frame_dev, int64_t n_pix,
                                        int64_t batch, int32_t* pix, hipStream_t st);
size_t labels_smem_bytes(int m, int n_spheres);
hipError_t launch_world_samples(uint64_t seed, uint32_t frame, const uint32_t* frame_dev, int64_t n, const float* box,
                                float extent, float* pos_scene, float* pos_unit, hipStream_t st);
hipError_t launch_labels(const float* pos, const int32_t* pix, int64_t n, const float* lights, int m,
                         const float* spheres, int n_spheres, uint8_t* labels, hipStream_t st);
bool train_supported(const GridHost& g, const NetShape& s);
int64_t train_workspace_bytes(const GridHost& g, const NetShape& s, int64_t batch);
hipError_t launch_train(const GridHost& g, const NetShape& s, const PackPlan& plan, const float* table,
                        const void* packed, const float* pos, const int32_t* pix, int64_t batch,
                        const uint8_t* labels, const float* dvis, int loss, float grad_scale, float* g_table,
                        float* g_w, float* loss_out, void* workspace, hipStream_t st);
// The routing plan of the table scatter computed ahead (for the same samples and batch), and the
// training pass that uses it instead of computing its own.
int64_t train_plan_bytes(const GridHost& g, const NetShape& s, int64_t batch);
hipError_t launch_train_plan(const GridHost& g, const NetShape& s, const float* pos, const int32_t* pix,
                             int64_t batch, void* plan, hipStream_t st);
hipError_t launch_train_planned(const GridHost& g, const NetShape& s, const PackPlan& plan, const float* table,
                                const void* packed, const float* pos, const int32_t* pix, int64_t batch,
                                const uint8_t* labels, const float* dvis, int loss, float grad_scale, float* g_table,
                                float* g_w, float* loss_out, const void* route_plan, void* workspace, hipStream_t st);
// Shadow-label inputs of the training pass that computes its labels in the kernel.
struct ShadowArgs {
    const float* pos_scene;   // [*][3] scene units, indexed like the unit-cube positions
    const float* lights;      // [n_lights][4]
    int n_lights;
    const float* spheres;     // [n_spheres][4]
    int n_spheres;
    uint8_t* labels_out;      // [batch][n_lights] or NULL
};
bool train_shadow_supported(const GridHost& g, const NetShape& s, int64_t batch, int n_spheres);
hipError_t launch_train_shadow(const GridHost& g, const NetShape& s, const PackPlan& plan, const float* table,
                               const void* packed, const float* pos, const int32_t* pix, int64_t batch,
                               const ShadowArgs& sh, int loss, float grad_scale, float* g_table, float* g_w,
                               float* loss_out, void* workspace, hipStream_t st);
hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t count, int step, const int32_t* step_dev,
                       float lr, float lr_end, int lr_decay_steps, float beta1, float beta2, float eps, int zero_grad,
                       hipStream_t st);
hipError_t launch_clustered_labels(const float* pos, const int32_t* pix, int64_t n, const float* lights, int n_lights,
                                   const int32_t* offsets, const int32_t* members, int k, const float* spheres,
                                   int n_spheres, uint64_t seed, uint32_t frame, const uint32_t* frame_dev,
                                   uint8_t* labels, hipStream_t st);
hipError_t launch_clustered_sample(const void* vis, int vis_dtype, int64_t n, int k, const float* pos, const float* nrm,
                                   const float* lights, int n_lights, const int32_t* offsets, const int32_t* members,
                                   float vis_floor, int n_cand, uint64_t seed, uint32_t frame,
                                   const uint32_t* frame_dev, int32_t* idx, float* weight, int32_t* cluster,
                                   const uint8_t* mask, nvc_reservoir* res, hipStream_t st);
void cluster_lights_host(const float* lights, int n, int k, int iters, int32_t* offsets, int32_t* members);
hipError_t launch_forward_f64(const GridHost& g, const NetShape& s, const double* table, const double* w,
                              const float* pos, int64_t n, const uint8_t* labels, int loss, double* z,
                              uint8_t* masks, double* loss_out, hipStream_t st);
// frame += 1, step += 1 of the device counters {uint32 frame; int32 step}.
hipError_t launch_counters_advance(uint32_t* frame_dev, int32_t* step_dev, hipStream_t st);

}  // namespace nvc
