/*
 * nvc.h -- C ABI of the neural visibility cache hot path on MI355X (gfx950).
 *
 * The cache (Boksansky & Meister, "Neural Visibility Cache for Real-Time
 * Light Sampling", JCGT 14(2), 2025) answers: given a 3D position, how
 * visible is each light?  A multi-resolution hash-grid encoding feeds a small
 * MLP with one sigmoid output per light (Sec. 3.1, Fig. "overview"; Sec. 3.3);
 * a light is then picked by weighted reservoir sampling with weights equal to
 * the unshadowed contribution times the clamped predicted visibility
 * (Sec. 1, Sec. 3.1); the network is fitted online to shadow-ray labels with
 * one Adam step per frame (Sec. 3.4).
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (hipMalloc'd, coarse-grained) unless
 *    marked "host".  The caller owns all memory; the library allocates
 *    nothing and keeps no state between calls.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *    enqueues work on that stream: it never synchronises, so the results are
 *    ready when the stream is.  Calls are safe to capture into a HIP graph
 *    (no allocation, no memset, no host synchronisation inside).
 *  - Arguments are validated on the host before anything is launched; a
 *    negative nvc_status is returned and nothing is enqueued.  A failed
 *    launch returns NVC_ERR_HIP.  There is no device-side error reporting.
 *  - n == 0 (or batch == 0) is a valid no-op returning NVC_OK.
 *  - NaN or Inf inputs are not checked; they propagate into the outputs.
 *  - Layouts are row-major and dense (no strides).
 */
#ifndef NVC_H
#define NVC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NVC_VERSION 1

typedef enum nvc_status {
    NVC_OK = 0,
    NVC_ERR_NULL = -1,        /* a required pointer is NULL                        */
    NVC_ERR_SHAPE = -2,       /* a size is negative, inconsistent or out of range  */
    NVC_ERR_DTYPE = -3,       /* unknown dtype code                                */
    NVC_ERR_UNSUPPORTED = -4, /* valid but not built: network shape, F, L*F, ...   */
    NVC_ERR_HIP = -5,         /* a HIP launch failed                               */
    NVC_ERR_WORKSPACE = -6    /* workspace missing or smaller than required        */
} nvc_status;

typedef enum nvc_dtype { NVC_F32 = 0, NVC_F16 = 1, NVC_BF16 = 2 } nvc_dtype;
typedef enum nvc_act { NVC_ACT_RELU = 0, NVC_ACT_LEAKY = 1 } nvc_act;
typedef enum nvc_loss { NVC_LOSS_BCE = 0, NVC_LOSS_L2 = 1 } nvc_loss;

/* Multi-resolution hash grid (Sec. 3.3; Mueller et al. 2022 eq. 2-4), host struct.
 * Level l has resolution N_l = floor(base_res * growth^l) (FP64 on the host);
 * it is stored densely (vertex x + (N+1)y + (N+1)^2 z) when (N_l+1)^3 <= T,
 * otherwise through the spatial hash (x*1 ^ y*2654435761 ^ z*805459861) mod T.
 * Table layout: float32 [n_levels][T = 2^log2_T][n_feat], level-major.
 * Supported: n_feat in {1, 2, 4}; 1 <= n_levels <= 32; n_levels*n_feat <= 64;
 * 10 <= log2_T <= 24; 1 <= base_res; growth >= 1. */
typedef struct nvc_grid {
    int32_t n_levels;
    int32_t n_feat;
    int32_t log2_T;
    int32_t base_res;
    double growth;
} nvc_grid;

/* Visibility MLP (Sec. 3.3), host struct: n_in -> width (x n_hidden) -> n_out,
 * no biases, hidden activation `act` (NVC_ACT_LEAKY uses leaky_slope, which
 * must lie in [0, 1]), sigmoid output, evaluated from the FP32 accumulator as
 * 1 / (1 + e) or e / (1 + e) with e = exp(-|z|) from the hardware exp2 and
 * reciprocal (relative error a few 1e-7).  `dtype` is the precision of weights and activations fed to the
 * matrix cores (NVC_F32 uses FP32 matrix cores); accumulation is FP32.
 * n_in must equal n_levels * n_feat of the grid it is used with.
 * Master weights: float32, the layers' row-major [out][in] matrices
 * concatenated, input layer first (nvc_mlp_param_count floats). */
typedef struct nvc_mlp {
    int32_t n_in;
    int32_t width;
    int32_t n_hidden;
    int32_t n_out;
    int32_t act;
    float leaky_slope;
    int32_t dtype;
} nvc_mlp;

int nvc_version(void);

/* Short English description of a status code (static storage). */
const char* nvc_status_string(int status);

/* Host only.  Level resolutions N_l and dense flags (1 dense, 0 hashed) of a
 * grid, each written to host arrays of n_levels entries (either may be NULL). */
int nvc_grid_levels(const nvc_grid* grid, int32_t* res, int32_t* dense);

/* Host only.  Number of FP32 master weights of the network, or a negative status. */
int64_t nvc_mlp_param_count(const nvc_mlp* mlp);

/* Host only.  Bytes of the packed low-precision copy of the weights that
 * nvc_infer and nvc_train_step read, or a negative status.  The packed copy
 * holds, per layer, the matrix and its transpose cut into matrix-core
 * operand fragments, in mlp->dtype; for 16-bit networks whose output count
 * spans an even number of 16-neuron blocks, also a copy of the output
 * layer with its rows in the order the inference kernel stores them. */
int64_t nvc_mlp_packed_bytes(const nvc_mlp* mlp);

/* Cast and reorder FP32 master weights `w` (nvc_mlp_param_count floats) into
 * the packed buffer `packed` (nvc_mlp_packed_bytes bytes).  Call after every
 * change of the master weights (e.g. after nvc_adam). */
int nvc_pack_mlp(const nvc_mlp* mlp, const float* w, void* packed, void* stream);

/* Hash-grid encoding (Sec. 3.1 Fig. "overview" step 1).
 * table: float32 [L][T][F]; pos: float32 [n][3], unit cube (values are
 * clamped to [0,1], NaN -> 0); enc: [n][L*F] in enc_dtype, feature j of level
 * l at column l*F + j.  The cell of a position is decided in FP32:
 * s = fl32(x * N_l), c = min(floor(s), N_l - 1); weights are trilinear in s - c. */
int nvc_encode(const nvc_grid* grid, const float* table, const float* pos, int64_t n,
               void* enc, int32_t enc_dtype, void* stream);

/* Cache inference (Sec. 3.1 steps 1-2; Sec. 3.3): encoding followed by the
 * MLP, fused in one kernel.  vis: [n][n_out] in vis_dtype, the raw sigmoid
 * output in (0,1) (the clamp of Sec. 3.1 is applied by nvc_sample_wrs).
 * packed: the output of nvc_pack_mlp for the same mlp.
 * Built network shapes: n_in in {16, 32, 40}, width in {32, 64, 128},
 * 1 <= n_hidden <= 4, 1 <= n_out <= 128 (others: NVC_ERR_UNSUPPORTED). */
int nvc_infer(const nvc_grid* grid, const nvc_mlp* mlp, const float* table, const void* packed,
              const float* pos, int64_t n, void* vis, int32_t vis_dtype, void* stream);

/* The MLP of nvc_infer alone (Sec. 3.3), on a given encoding: enc [n][n_in]
 * in enc_dtype (e.g. the output of nvc_encode), vis [n][n_out] in vis_dtype.
 * The encoding is rounded to mlp->dtype for the matrix cores, as inside
 * nvc_infer, so nvc_mlp_forward(nvc_encode(x)) with enc_dtype = mlp->dtype
 * (or FP32) equals nvc_infer(x).  Same network shapes as nvc_infer. */
int nvc_mlp_forward(const nvc_mlp* mlp, const void* packed, const void* enc, int32_t enc_dtype, int64_t n,
                    void* vis, int32_t vis_dtype, void* stream);

/* A pick as a reservoir of resampled importance sampling for the target
 * function f (the unshadowed weight), the form in which ReSTIR takes its
 * initial candidates (Sec. 4.2: the clustered cache generates a reservoir):
 * y the light (-1: none), M the number of candidates it was resampled from,
 * w_sum the sum of their resampling weights, W = w_sum / (M f_y) the
 * unbiased contribution weight (f_y V_y W estimates sum_i f_i V_i). */
typedef struct nvc_reservoir {
    int32_t y;
    int32_t M;
    float w_sum;
    float W;
} nvc_reservoir;

/* Per-frame counters in DEVICE memory, for frames recorded once into a HIP
 * graph and replayed: nvc_sample_wrs and nvc_select_pixels given a non-NULL
 * `ctr` take the frame number from ctr->frame, and nvc_adam takes its step
 * from ctr->step, when they run on the stream (the value arguments are then
 * ignored).  nvc_counters_advance increments both on the stream. */
typedef struct nvc_counters {
    uint32_t frame;
    int32_t step;             /* Adam step, >= 1 */
} nvc_counters;

/* ctr->frame += 1 and ctr->step += 1, enqueued on `stream`. */
int nvc_counters_advance(nvc_counters* ctr, void* stream);

/* Recording a frame once and replaying it (Sec. 4: the cache runs every
 * frame; a frame's launches are the same each time, and the device counters
 * above make each replay the next frame).  These wrap HIP stream capture.
 * nvc_graph_begin starts capturing `stream` (a created stream, not NULL:
 * the legacy default stream cannot be captured), in thread-local mode: this
 * thread may then make no call that would allocate or synchronise.  Every
 * entry point of this library may be captured.  Work may fork to other
 * streams through events recorded on the capturing stream, and every such
 * stream must be joined back (its last work recorded in an event the
 * capturing stream waits on) before nvc_graph_end, or capture fails.
 * nvc_graph_end ends the capture and instantiates it: *exec receives an
 * executable graph owned by the caller (NULL and NVC_ERR_HIP if capture or
 * instantiation failed; the stream is no longer capturing either way).
 * nvc_graph_launch enqueues one replay on `stream` (not NULL); replays on
 * one stream run in order.  nvc_graph_destroy releases the executable (not
 * while a replay may still run: synchronise first).  The buffers the
 * recorded calls received must stay allocated while the graph is used. */
int nvc_graph_begin(void* stream);
int nvc_graph_end(void* stream, void** exec);
int nvc_graph_launch(void* exec, void* stream);
int nvc_graph_destroy(void* exec);

/* Light selection by weighted reservoir sampling (Sec. 1, Sec. 3.1) and
 * neural direct illumination (Sec. 3.2).
 * vis: [n][m] in vis_dtype; pos: float32 [n][3] in scene units; nrm:
 * float32 [n][3] unit normals or NULL (then the cosine term is dropped);
 * lights: float32 [m][4] = (x, y, z, intensity); 1 <= m <= 128.
 * Light weight w_i = f_i * max(v_i, vis_floor) (vis_floor = 0.001 keeps the
 * sampler unbiased; 0 gives the biased variant), with the Lambertian
 * unshadowed contribution, evaluated in FP32 in this order:
 *   d = l - p; d2 = max((dx*dx + dy*dy) + dz*dz, 1e-6);
 *   with normals: nd = (nx*dx + ny*dy) + nz*dz, f = (I * max(nd, 0)) / (d2 * sqrt(d2));
 *   without:      f = I / d2.
 * One uniform per pixel u = (r0 >> 8) * 2^-24 where r0 is the first word of
 * Philox4x32-10 with counter (pixel lo32, pixel hi32, frame, 0) and key
 * (seed lo32, seed hi32).  With C_i the sequential FP32 running sum of w in
 * light order and W = C_{m-1}: idx = the first i with C_i > u * W.
 * Outputs (float32 / int32 [n]): idx (-1 when W = 0), pmf = w_idx / W (0 when
 * W = 0), wsum = W, and, if di != NULL, di = sum_i v_i f_i / pi (raw v).
 * ctr (device, or NULL): if given, frame = ctr->frame at run time.
 * mask (uint8 [n], or NULL): pixels with mask 0 are skipped (the cache is
 * run only where needed, e.g. where a screen-space reuse lost its history):
 * idx = -1, pmf = wsum = di = 0, an empty reservoir.
 * res (nvc_reservoir [n], or NULL): the pick as a one-candidate reservoir
 * for target f: y = idx, M = 1, W = W / w_idx (= 1 / pmf, FP32 division),
 * w_sum = f_idx * W; {-1, 0, 0, 0} without a pick. */
int nvc_sample_wrs(const void* vis, int32_t vis_dtype, int64_t n, int32_t m,
                   const float* pos, const float* nrm, const float* lights, float vis_floor,
                   uint64_t seed, uint32_t frame, const nvc_counters* ctr,
                   int32_t* idx, float* pmf, float* wsum, float* di, const uint8_t* mask, nvc_reservoir* res,
                   void* stream);

/* Host only.  Workspace bytes nvc_select_pixels needs for an image of n_pix pixels. */
int64_t nvc_select_pixels_workspace_bytes(int64_t n_pix);

/* Training-pixel selection (Sec. 3.4: random screen-space positions).
 * Sample b draws pixel (r0 * n_pix) >> 32, r0 the first word of
 * Philox4x32-10 with counter (b lo32, b hi32, frame, 1) and key (seed lo32,
 * seed hi32): uniform with replacement over [0, n_pix).  The batch is a
 * multiset and pix (int32 [batch]) receives it in ascending order, so that
 * consecutive samples lie on nearby surfaces (nvc_shadow_labels and
 * nvc_train_step run faster on such batches; the training step sums over
 * the batch, so the order does not change it).  Deterministic.
 * workspace: nvc_select_pixels_workspace_bytes(n_pix) bytes of device memory.
 * ctr (device, or NULL): if given, frame = ctr->frame at run time.
 * 1 <= n_pix < 2^31, 0 <= batch < 2^31. */
int nvc_select_pixels(uint64_t seed, uint32_t frame, const nvc_counters* ctr, int64_t n_pix, int64_t batch,
                      int32_t* pix, void* workspace, int64_t workspace_bytes, void* stream);

/* nvc_select_pixels without allocation or workspace, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same result as
 * nvc_select_pixels; the workspace is a static device buffer inside the
 * library, sized for n_pix <= NVC_SELECT_PIXELS_NOALLOC_MAX_PIX (2^23 pixels:
 * 64 MiB + 8.5 KiB), which each GPU the library runs on holds until the
 * process ends.  Larger images: NVC_ERR_SHAPE, nothing enqueued.  The first
 * call on a device (the current device) looks up the buffer's address there
 * (no allocation, but it may load the library's code on that device: make it
 * outside stream capture).  Every call on a GPU shares that GPU's buffer and
 * keeps nothing from the previous call: calls that overlap on one GPU (e.g.
 * on two streams without an ordering between them) race and must be
 * serialised by the caller.  ctr as in nvc_select_pixels. */
#define NVC_SELECT_PIXELS_NOALLOC_MAX_PIX (1 << 23)
int nvc_select_pixels_noalloc(uint64_t seed, uint32_t frame, const nvc_counters* ctr, int64_t n_pix, int64_t batch,
                              int32_t* pix, void* stream);

/* World-space training points (Sec. 3.4: training examples at random scene
 * positions, which prepare the cache for views it has not seen yet; the
 * paper mixes them with the screen-space ones).  Point i is, per axis,
 * lo + u * (hi - lo) (FP32: the difference, then the product, then the sum)
 * with u = (r >> 8) * 2^-24 from words 0, 1, 2 of Philox4x32-10 with counter
 * (i lo32, i hi32, frame, 6) and key (seed lo32, seed hi32); pos_unit =
 * p / extent (correctly rounded), the unit-cube position the encoding takes.
 * box: HOST float [6] = lo xyz, hi xyz (lo <= hi, finite); extent > 0.
 * pos_scene, pos_unit: float32 [n][3] device.  ctr as in nvc_select_pixels. */
int nvc_world_samples(uint64_t seed, uint32_t frame, const nvc_counters* ctr, int64_t n, const float* box,
                      float extent, float* pos_scene, float* pos_unit, void* stream);

/* Shadow-ray labels (Sec. 3.4: one shadow ray from each training point to
 * each light) against sphere occluders.  Sample b uses position
 * pos[pix[b]] (pix may be NULL: pos[b]); every pix[b] must index a row of
 * pos (device data is not validated); pos: float32 scene units [*][3];
 * lights: float32 [m][4]; spheres: float32 [n_spheres][4] = (cx, cy, cz, r).
 * labels: uint8 [n][m], 1 = visible, 0 = occluded.  A ray p -> l is occluded
 * when a sphere comes closer than r to the segment, decided in FP32 as
 *   o = c - p, cc = ((ox*ox + oy*oy) + oz*oz) - r*r, d = l - p,
 *   dd = (dx*dx + dy*dy) + dz*dz, b = (ox*dx + oy*dy) + oz*dz;
 *   b <= 0: cc < 0;  b >= dd: |c - l|^2 < r*r;  otherwise cc*dd < b*b.
 * The kernel skips spheres that provably lie farther than r from all the
 * segments of a group of 64 samples; the labels equal the brute-force ones.
 * Groups of nearby samples (as nvc_select_pixels returns them) run fastest.
 * 1 <= m <= 128; 0 <= n_spheres <= 4096 (spheres, lights and their bit
 * masks are held in at most 146 KiB of LDS). */
int nvc_shadow_labels(const float* pos, const int32_t* pix, int64_t n,
                      const float* lights, int32_t m, const float* spheres, int32_t n_spheres,
                      uint8_t* labels, void* stream);

/* ---------------------------------------------------------------------------
 * Clustered cache (Sec. 3.6): the output neurons predict the average
 * visibility of clusters of lights, so the light count is not bounded by the
 * output layer.  A clustering is CSR: offsets int32 [k+1] (offsets[0] = 0,
 * non-decreasing, offsets[k] = n_lights) and members int32 [n_lights], the
 * light indices of cluster c in members[offsets[c] .. offsets[c+1]).  On the
 * device, an ill-formed range or a member outside [0, n_lights) is treated as
 * an empty cluster or a missing light, never read out of bounds.
 * ------------------------------------------------------------------------- */

/* Host only.  k-means clustering of the lights by position (Sec. 3.6).
 * lights: HOST float32 [n_lights][4]; 1 <= k <= min(n_lights, 128); iters >= 1.
 * Initial centroids by farthest points (light 0, then repeatedly the light
 * farthest from the chosen ones, ties to the lower index); then Lloyd
 * iterations in FP64: each light to its nearest centroid (squared distance
 * (dx*dx + dy*dy) + dz*dz, ties to the lower cluster), each non-empty cluster's
 * centroid to the mean of its lights (coordinates summed in light order),
 * until no assignment changes or `iters` iterations ran.  Writes HOST offsets
 * [k+1] and members [n_lights] (ascending light index within a cluster). */
int nvc_cluster_lights(const float* lights, int32_t n_lights, int32_t k, int32_t iters, int32_t* offsets,
                       int32_t* members);

/* Clustered training labels (Sec. 3.6): for sample b (position pos[pix[b]],
 * or pos[b] if pix is NULL) and cluster c, one light of the cluster is drawn
 * uniformly, members[offsets[c] + ((r * m_c) >> 32)] with m_c the cluster's
 * size and r word c%4 of Philox4x32-10 with counter (b lo32, b hi32, frame,
 * 32 + c/4) and key (seed lo32, seed hi32), and labels[b][c] (uint8 [n][k])
 * is 1 if the segment to it misses every sphere (the FP32 test of
 * nvc_shadow_labels), else 0; 0 for an empty cluster.  Device pointers.
 * 1 <= k <= 128, 0 <= n_spheres <= 4096; ctr as in nvc_sample_wrs. */
int nvc_shadow_labels_clustered(const float* pos, const int32_t* pix, int64_t n, const float* lights,
                                int32_t n_lights, const int32_t* offsets, const int32_t* members, int32_t k,
                                const float* spheres, int32_t n_spheres, uint64_t seed, uint32_t frame,
                                const nvc_counters* ctr, uint8_t* labels, void* stream);

/* Two-step light pick of the clustered cache (Sec. 3.6), one per pixel.
 * vis: [n][k] cluster visibilities in vis_dtype; pos, nrm, lights as in
 * nvc_sample_wrs (lights [n_lights][4]).
 * Step 1, WRS over the clusters: w_j = fl(m_j) * max(v_j, vis_floor) (m_j the
 * cluster's size), the pick uniform and the inverse-CDF rule of
 * nvc_sample_wrs give cluster y, P = w_y / W (W the sequential FP32 sum).
 * Step 2, streaming RIS over n_cand candidates drawn uniformly from cluster
 * y: candidate kk is members[offsets[y] + ((r * m_y) >> 32)], r word kk%4 of
 * Philox with counter (pixel lo32, pixel hi32, frame, 4 + kk/4); its target
 * is its unshadowed weight f (the order of nvc_sample_wrs) and its source
 * pdf P / m_y.  With S the sequential FP32 sum of the candidates' f and u2
 * from word 0 of counter (pixel, frame, 2), the kept candidate x is the first
 * whose running sum exceeds u2 * S, and its contribution weight is
 *   weight = (S * fl(m_y)) / ((fl(n_cand) * P) * f_x),
 * so that f_x V_x weight is an unbiased estimate of sum_i f_i V_i.
 * Outputs [n]: idx (int32, the light, -1 if W = 0 or S = 0), weight (float32,
 * 0 then), cluster (int32 y or -1; may be NULL).  1 <= k <= 128,
 * 1 <= n_cand <= 64; ctr and mask as in nvc_sample_wrs.
 * res (or NULL): the RIS reservoir, y = idx, M = n_cand, W = weight,
 * w_sum = (S * fl(m_y)) / P, the sum of the candidates' resampling weights
 * f_k / (P / m_y); {-1, 0, 0, 0} without a pick. */
int nvc_sample_clustered(const void* vis, int32_t vis_dtype, int64_t n, int32_t k, const float* pos,
                         const float* nrm, const float* lights, int32_t n_lights, const int32_t* offsets,
                         const int32_t* members, float vis_floor, int32_t n_cand, uint64_t seed, uint32_t frame,
                         const nvc_counters* ctr, int32_t* idx, float* weight, int32_t* cluster,
                         const uint8_t* mask, nvc_reservoir* res, void* stream);

/* Host only.  Workspace bytes nvc_train_step needs for this network and batch. */
int64_t nvc_train_workspace_bytes(const nvc_grid* grid, const nvc_mlp* mlp, int64_t batch);

/* One training pass (Sec. 3.3-3.4): re-encode and re-run the network on the
 * batch (activations are recomputed, never stored to memory), take the loss
 * gradient at the output, backpropagate through the MLP on the matrix cores,
 * and scatter the encoding gradient into the hash table: routed to 2^k-entry
 * partitions of the table and summed there exactly (64-bit fixed point in
 * LDS), with FP32 atomics only for corner pairs that straddle a partition
 * boundary, partitions summed by several blocks, and grids whose hashed
 * levels are too fine to partition (then every corner).
 * Sample b uses unit-cube position pos[pix[b]] (pix may be NULL: pos[b]).
 * Mode A (labels != NULL, dvis == NULL): loss over the batch of
 *   NVC_LOSS_BCE: mean over batch*n_out of softplus(z) - y z,
 *   NVC_LOSS_L2:  mean of (sigmoid(z) - y)^2;
 *   labels: uint8 [batch][n_out] (0/1); *loss_out (if not NULL) = the loss.
 * Mode B (labels == NULL, dvis != NULL): dvis float32 [batch][n_out] is an
 *   upstream gradient dL/dv; loss_out is left untouched.
 * grad_scale > 0 multiplies the output gradient before the low-precision
 * backward and divides the results afterwards (loss scaling; exact in
 * real arithmetic).  0 selects the default (batch*n_out in mode A, 1 in B).
 * Gradients are ADDED to g_table (float32 [L][T][F]) and g_w (float32,
 * master-weight layout); the caller zeroes them (nvc_adam can).  Those FP32
 * atomics, and the weight gradient's sum over slices of the training blocks,
 * make the last bits of g_table and g_w vary from run to run.
 * workspace: nvc_train_workspace_bytes bytes of device memory. */
int nvc_train_step(const nvc_grid* grid, const nvc_mlp* mlp, const float* table,
                   const void* packed, const float* pos, const int32_t* pix, int64_t batch,
                   const uint8_t* labels, const float* dvis, int32_t loss, float grad_scale,
                   float* g_table, float* g_w, float* loss_out,
                   void* workspace, int64_t workspace_bytes, void* stream);

/* The routing plan of nvc_train_step's table scatter, computed on its own
 * (Sec. 3.3: the gradient of every corner of every sample's cell goes to the
 * table).  For each training block and each partition of the table (2^k
 * consecutive entries of a level) the plan holds how many records the block's
 * samples write there and where, and the chunk table of the partition sums.
 * It depends only on the positions pos[pix[b]] (as for nvc_train_step), the
 * batch and the grid, not on the parameters, so it can be computed ahead of
 * the gradient pass, beside other work, into a buffer of
 * nvc_train_plan_bytes bytes (0: this batch trains through direct atomics
 * and needs no plan; nvc_train_plan then does nothing).  Errors as
 * nvc_train_step; NVC_ERR_WORKSPACE if plan is NULL or too small.  Device
 * pointers; the plan is owned by the caller. */
int64_t nvc_train_plan_bytes(const nvc_grid* grid, const nvc_mlp* mlp, int64_t batch);
int nvc_train_plan(const nvc_grid* grid, const nvc_mlp* mlp, const float* pos, const int32_t* pix, int64_t batch,
                   void* plan, int64_t plan_bytes, void* stream);

/* nvc_train_step with the routing plan from nvc_train_plan instead of its own
 * (the same pos, pix and batch; the plan must be complete when this pass runs,
 * e.g. computed earlier on the same stream or behind an event).  Given the
 * plan of the same samples the gradients are those of nvc_train_step.  A plan
 * of other samples gives wrong gradients but no access outside the buffers:
 * the kernels bound every record index by the batch's record count.  plan and
 * plan_bytes as for nvc_train_plan (ignored when that size is 0); everything
 * else as nvc_train_step. */
int nvc_train_step_planned(const nvc_grid* grid, const nvc_mlp* mlp, const float* table, const void* packed,
                           const float* pos, const int32_t* pix, int64_t batch, const uint8_t* labels,
                           const float* dvis, int32_t loss, float grad_scale, float* g_table, float* g_w,
                           float* loss_out, const void* plan, int64_t plan_bytes, void* workspace,
                           int64_t workspace_bytes, void* stream);

/* nvc_train_step in labelled mode with the shadow labels computed inside the
 * training kernel instead of read from memory (Sec. 3.4: each training example
 * pairs a position with the visibility of every light, from one shadow ray per
 * light; Sec. 4.4 and Table "perf_breakdown" fuse data generation into the
 * training pass).  The label of sample b and light j is the one
 * nvc_shadow_labels gives for scene-space position pos_scene[pix[b]] (pos_scene
 * indexed like pos; pix may be NULL), lights [m][4] and spheres [n_spheres][4]
 * (the same FP32 decision), and the network has one output per light
 * (m == mlp->n_out).  Each wave culls the spheres against the bundle of its 16
 * samples' segments to every light before the exact tests.  labels_out
 * (uint8 [batch][m], or NULL) receives the labels.  Limits: 1 <= m <=
 * NVC_TRAIN_SHADOW_MAX_LIGHTS, 0 <= n_spheres <= NVC_TRAIN_SHADOW_MAX_SPHERES
 * (else NVC_ERR_SHAPE); networks with more than 32 outputs have no such kernel,
 * nor shapes whose activations, scatter cursors, lights and spheres overflow the
 * 160 KiB of LDS of a compute unit (NVC_ERR_UNSUPPORTED).  The pass runs on the
 * grid of nvc_train_step, so its gradients and loss equal those of
 * nvc_train_step given the same labels, bit for bit; the workspace is
 * nvc_train_workspace_bytes for the same network and batch.  Everything else as
 * nvc_train_step. */
#define NVC_TRAIN_SHADOW_MAX_LIGHTS 32
#define NVC_TRAIN_SHADOW_MAX_SPHERES 512
int nvc_train_step_shadow(const nvc_grid* grid, const nvc_mlp* mlp, const float* table, const void* packed,
                          const float* pos, const float* pos_scene, const int32_t* pix, int64_t batch,
                          const float* lights, int32_t m, const float* spheres, int32_t n_spheres, int32_t loss,
                          float grad_scale, float* g_table, float* g_w, float* loss_out, uint8_t* labels_out,
                          void* workspace, int64_t workspace_bytes, void* stream);

/* One Adam step (Sec. 3.4; Kingma & Ba) over `count` FP32 parameters, dense:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= (lr_t / (1 - b1^step)) * m / (sqrt(v) / sqrt(1 - b2^step) + eps)
 * step >= 1 counts from 1 (with ctr: ctr->step at run time, values below 1
 * taken as 1).  The learning rate lr_t is lr, or with lr_decay_steps = D > 0
 * the schedule of Sec. 3.4 (a rate lowered linearly over the first training
 * steps): with f = min(step - 1, D) / D, lr_t = (1 - f) lr + f lr_end, from lr
 * at step 1 to lr_end at step D + 1 and after.  The rate and the bias corrections are
 * computed on the device in FP32: b^step by repeated squaring, then correctly
 * rounded divisions and square root.  If zero_grad != 0, g is set to 0
 * afterwards (the next nvc_train_step then accumulates into a clean buffer).
 * lr, lr_end and eps must be finite and >= 0, lr_decay_steps >= 0, betas in
 * [0, 1) (else NVC_ERR_SHAPE). */
int nvc_adam(float* p, float* g, float* m, float* v, int64_t count, int32_t step, const nvc_counters* ctr,
             float lr, float lr_end, int32_t lr_decay_steps, float beta1, float beta2, float eps,
             int32_t zero_grad, void* stream);

/* FP64 forward pass and training loss, for checking gradients by central
 * finite differences (Sec. 3.3: the cache is trained by backpropagation; a
 * difference quotient with a step of 1e-3 needs the loss to many more digits
 * than the FP16 / FP32 paths give).  Not a hot-path call: plain FP64
 * arithmetic on the vector units, one block per point.
 * table: double [L][T][F]; w: double, the master-weight layout (per layer
 * [out][in], input layer first); pos: float32 [n][3] unit cube, clamped as in
 * nvc_encode.  The cell and fraction of a position are decided in FP32 as in
 * every other kernel (s = fl32(x N)); trilinear weights, features, network,
 * sigmoid and loss are FP64; dot products run over their inputs in index
 * order.  mlp->dtype is ignored.
 * z: double [n][n_out] logits, or NULL.
 * masks: uint8 [n][n_hidden][ceil(width/8)], or NULL: bit j%8 of byte j/8 of
 *   layer k is set iff hidden pre-activation j of layer k is > 0 (the ReLU /
 *   leaky-ReLU branch taken), so that a caller can tell whether a
 *   perturbation changed any branch.
 * labels: uint8 [n][n_out] (0/1), or NULL.  With labels, loss_out (double,
 *   n + 1 entries) receives each point's loss summed over its outputs in order
 *   (NVC_LOSS_BCE: softplus(z) - y z; NVC_LOSS_L2: (sigmoid(z) - y)^2) and,
 *   at [n], their mean over n * n_out, summed over the points in index order.
 * n in [0, 2^20] (else NVC_ERR_SHAPE); n = 0 is a no-op. */
int nvc_forward_f64(const nvc_grid* grid, const nvc_mlp* mlp, const double* table, const double* w,
                    const float* pos, int64_t n, const uint8_t* labels, int32_t loss, double* z,
                    uint8_t* masks, double* loss_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NVC_H */
