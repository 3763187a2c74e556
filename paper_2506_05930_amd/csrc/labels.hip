// Training data (Sec. 3.4): the batch of training pixels and their shadow-ray
// labels against sphere occluders.
//
// Pixels.  The batch is a multiset of pixels drawn uniformly with replacement
// by Philox; it is returned in ascending pixel order (a counting sort over the
// image), so neighbouring samples lie on nearby surfaces.  Training sums over
// the batch, so its order does not change the step.
//
// Labels.  One wave labels 64 consecutive samples.  For each light the wave
// first tests every sphere against the bundle of its 64 segments at once: all
// segments p -> l lie within rho of the segment pbar -> l (pbar the centre of
// the samples' bounding box, rho its radius), so a sphere whose distance to
// that segment exceeds r + rho + m cannot come within r + m of any of them.
// The margin m = 1e-3 (1 + scene scale) is far above the FP32 error of the
// exact test, so culled spheres are exactly those the exact FP32 test would
// also reject.  Survivors get the exact test (operation order in nvc.h), and
// the label equals the brute-force FP32 label.
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace nvc {

// ------------------------------------------------------------------ training pixels
__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void pixel_count_kernel(uint32_t k0, uint32_t k1, uint32_t frame,
                                                          const uint32_t* __restrict__ frame_dev, uint32_t n_pix,
                                                          int64_t batch, uint32_t* __restrict__ counts) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const uint32_t fr = frame_dev ? *frame_dev : frame;
    const uint32_t r0 = philox_first_word((uint32_t)b, (uint32_t)((uint64_t)b >> 32), fr, 1u, k0, k1);
    atomicAdd(&counts[__umulhi(r0, n_pix)], 1u);
}

constexpr int kScanBlock = 4096;    // entries per block of the pixel scan (1024 threads x 4)

// Exclusive scan of counts within blocks of kScanBlock entries; block totals to sums[].
__global__ __launch_bounds__(1024) void pixel_scan_local_kernel(const uint32_t* __restrict__ counts, int64_t n,
                                                                uint32_t* __restrict__ offs,
                                                                uint32_t* __restrict__ sums) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + t * 4;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = base + i < n ? counts[base + i] : 0u;
        s += v[i];
    }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (base + i < n) offs[base + i] = run;
        run += v[i];
    }
    if (t == 1023) sums[blockIdx.x] = part[1023];
}

// Exclusive scan of the block totals (one block, any count).
__global__ __launch_bounds__(1024) void pixel_scan_sums_kernel(uint32_t* __restrict__ sums, int nsums) {
    __shared__ uint32_t part[1024];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nsums; base += 1024) {
        const int i = base + threadIdx.x;
        const uint32_t v = i < nsums ? sums[i] : 0u;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nsums) sums[i] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void pixel_emit_kernel(const uint32_t* __restrict__ counts,
                                                         const uint32_t* __restrict__ offs,
                                                         const uint32_t* __restrict__ sums, int64_t n,
                                                         int32_t* __restrict__ pix) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t c = counts[p];
    if (c == 0) return;
    const uint32_t o = offs[p] + sums[p / kScanBlock];
    for (uint32_t i = 0; i < c; ++i) pix[o + i] = (int32_t)p;
}

int64_t select_pixels_workspace_bytes(int64_t n_pix) {
    const int64_t nsums = (n_pix + kScanBlock - 1) / kScanBlock;
    return (2 * n_pix + nsums) * 4 + 512;
}

hipError_t launch_select_pixels(uint64_t seed, uint32_t frame, const uint32_t* frame_dev, int64_t n_pix,
                                int64_t batch, int32_t* pix, void* workspace, hipStream_t st) {
    uint32_t* counts = reinterpret_cast<uint32_t*>(workspace);
    uint32_t* offs = counts + n_pix;
    uint32_t* sums = offs + n_pix;
    const int64_t nsums = (n_pix + kScanBlock - 1) / kScanBlock;
    const unsigned pb = (unsigned)((n_pix + 255) / 256);
    fill_u32_kernel<<<pb, 256, 0, st>>>(counts, n_pix, 0u);
    pixel_count_kernel<<<(unsigned)((batch + 255) / 256), 256, 0, st>>>((uint32_t)seed, (uint32_t)(seed >> 32), frame,
                                                                       frame_dev, (uint32_t)n_pix, batch, counts);
    pixel_scan_local_kernel<<<(unsigned)nsums, 1024, 0, st>>>(counts, n_pix, offs, sums);
    pixel_scan_sums_kernel<<<1, 1024, 0, st>>>(sums, (int)nsums);
    pixel_emit_kernel<<<pb, 256, 0, st>>>(counts, offs, sums, n_pix, pix);
    return hipGetLastError();
}

// ------------------------------------------------------------------ world-space samples
// Training points at random scene positions (not only on the visible
// surfaces): p = lo + u * (hi - lo) per axis, u from words 0..2 of Philox
// counter (i, frame, 6); unit-cube position p / extent.
__global__ void world_samples_kernel(uint32_t k0, uint32_t k1, uint32_t frame, const uint32_t* __restrict__ frame_dev,
                                     int64_t n, float lx, float ly, float lz, float hx, float hy, float hz,
                                     float extent, float* __restrict__ pos_scene, float* __restrict__ pos_unit) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t fr = frame_dev ? *frame_dev : frame;
    uint32_t w[4];
    philox_words((uint32_t)i, (uint32_t)((uint64_t)i >> 32), fr, 6u, k0, k1, w);
    const float lo[3] = {lx, ly, lz}, hi[3] = {hx, hy, hz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float u = (float)(w[k] >> 8) * 0x1.0p-24f;
        const float p = u * (hi[k] - lo[k]) + lo[k];
        pos_scene[i * 3 + k] = p;
        pos_unit[i * 3 + k] = __fdiv_rn(p, extent);
    }
}

hipError_t launch_world_samples(uint64_t seed, uint32_t frame, const uint32_t* frame_dev, int64_t n, const float* box,
                                float extent, float* pos_scene, float* pos_unit, hipStream_t st) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(world_samples_kernel, dim3(blocks), dim3(256), 0, st, (uint32_t)seed, (uint32_t)(seed >> 32),
                       frame, frame_dev, n, box[0], box[1], box[2], box[3], box[4], box[5], extent, pos_scene,
                       pos_unit);
    return hipGetLastError();
}

// ------------------------------------------------------------------ shadow labels
__device__ inline uint32_t float_key(float v) { return __float_as_uint(v); }   // order-preserving for v >= 0

__device__ inline uint32_t spread10(uint32_t v) {        // 10 bits -> every third bit of 30
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

int cu_count();

constexpr int kLabelBlock = 1024;   // samples per block (waves of 64; a power of two up to 1024)
constexpr int kLabelLights = 8;     // most lights per block (grid.y covers all lights)

// Block (x, y): samples [x*kLabelBlock, (x+1)*kLabelBlock) and lights [lpb*y, lpb*y + lpb),
// lpb <= 8 lights per block (fewer when the batch is small, so that the grid
// still covers the chip).  The
// block sorts its samples by the 3D Morton code of their position inside the
// block's bounding box, so each wave of 64 consecutive sorted samples is
// compact in space (samples on both sides of a depth edge go to different
// waves); labels are written at the samples' own rows.
__global__ __launch_bounds__(kLabelBlock) void labels_kernel(const float* __restrict__ pos, const int32_t* __restrict__ pix,
                                                      int64_t n, const float* __restrict__ lights, int m,
                                                      const float* __restrict__ spheres, int n_spheres,
                                                      uint8_t* __restrict__ labels, int lpb) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    float4* S = reinterpret_cast<float4*>(smem_raw);                          // (cx, cy, cz, r*r)
    float* R = reinterpret_cast<float*>(S + n_spheres);                       // r
    float4* Lg = reinterpret_cast<float4*>(R + ((n_spheres + 3) & ~3));       // this block's lights
    uint32_t* inside = reinterpret_cast<uint32_t*>(Lg + kLabelLights);        // [n_spheres]: bit i = light l0+i
    __shared__ uint64_t keys[kLabelBlock];
    __shared__ uint32_t scale_bits;
    const int l0 = blockIdx.y * lpb;
    const int nl = min(lpb, m - l0);
    if (threadIdx.x == 0) scale_bits = 0;
    __syncthreads();
    uint32_t my_scale = 0;
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        const float lx = lights[4 * j + 0], ly = lights[4 * j + 1], lz = lights[4 * j + 2];
        if (j >= l0 && j < l0 + nl) Lg[j - l0] = make_float4(lx, ly, lz, 0.0f);
        my_scale = max(my_scale, float_key(fmaxf(fabsf(lx), fmaxf(fabsf(ly), fabsf(lz)))));
    }
    for (int s = threadIdx.x; s < n_spheres; s += blockDim.x) {
        const float cx = spheres[4 * s + 0], cy = spheres[4 * s + 1], cz = spheres[4 * s + 2], r = spheres[4 * s + 3];
        const float rr = r * r;
        S[s] = make_float4(cx, cy, cz, rr);
        R[s] = r;
        my_scale = max(my_scale, float_key(fmaxf(fabsf(cx), fmaxf(fabsf(cy), fabsf(cz))) + fabsf(r)));
        uint32_t bits = 0;
        for (int i = 0; i < nl; ++i) {
            const int li = l0 + i;
            const float ex = cx - lights[4 * li + 0], ey = cy - lights[4 * li + 1], ez = cz - lights[4 * li + 2];
            if (((ex * ex + ey * ey) + ez * ez) < rr) bits |= 1u << i;
        }
        inside[s] = bits;
    }

    // This thread's sample (unsorted) and the block's bounding box.
    const int64_t b_own = (int64_t)blockIdx.x * kLabelBlock + threadIdx.x;
    const bool own_valid = b_own < n;
    float ox0 = 0.f, oy0 = 0.f, oz0 = 0.f;
    if (own_valid) {
        const int64_t src = pix ? (int64_t)pix[b_own] : b_own;
        ox0 = pos[src * 3 + 0];
        oy0 = pos[src * 3 + 1];
        oz0 = pos[src * 3 + 2];
    }
    atomicMax(&scale_bits, my_scale);
    // Block bounding box of the finite samples (NaN / Inf samples sort last).
    __shared__ float bmin[3], bmax[3];
    if (threadIdx.x < 3) { bmin[threadIdx.x] = INFINITY; bmax[threadIdx.x] = -INFINITY; }
    __syncthreads();
    const bool fin = own_valid && isfinite(ox0) && isfinite(oy0) && isfinite(oz0);
    {
        float mn[3] = {fin ? ox0 : INFINITY, fin ? oy0 : INFINITY, fin ? oz0 : INFINITY};
        float mx[3] = {fin ? ox0 : -INFINITY, fin ? oy0 : -INFINITY, fin ? oz0 : -INFINITY};
#pragma unroll
        for (int k = 0; k < 3; ++k)
            for (int off = 32; off > 0; off >>= 1) {
                mn[k] = fminf(mn[k], __shfl_xor(mn[k], off));
                mx[k] = fmaxf(mx[k], __shfl_xor(mx[k], off));
            }
        __shared__ float wmn[kLabelBlock / 64][3], wmx[kLabelBlock / 64][3];
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0)
            for (int k = 0; k < 3; ++k) { wmn[w][k] = mn[k]; wmx[w][k] = mx[k]; }
        __syncthreads();
        if (threadIdx.x < 3) {
            float a = INFINITY, c = -INFINITY;
            for (int i = 0; i < (int)(blockDim.x >> 6); ++i) { a = fminf(a, wmn[i][threadIdx.x]); c = fmaxf(c, wmx[i][threadIdx.x]); }
            bmin[threadIdx.x] = a;
            bmax[threadIdx.x] = c;
        }
        __syncthreads();
    }
    // Morton key inside the box; invalid or non-finite samples get the largest keys.
    {
        uint64_t key;
        if (fin) {
            uint32_t q[3];
            const float v[3] = {ox0, oy0, oz0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float ext = bmax[k] - bmin[k];
                const float t = ext > 0.0f ? (v[k] - bmin[k]) / ext : 0.0f;
                q[k] = (uint32_t)fminf(fmaxf(t * 1023.0f, 0.0f), 1023.0f);
            }
            key = (uint64_t)(spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2)) << 11;
        } else {
            key = (own_valid ? (1ull << 41) : (1ull << 42));
        }
        keys[threadIdx.x] = key | (uint64_t)threadIdx.x;
    }
    __syncthreads();
    // Bitonic sort of the block's keys in LDS.
    for (int k = 2; k <= kLabelBlock; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            const int i = threadIdx.x, ixj = i ^ jj;
            if (ixj > i) {
                const uint64_t a = keys[i], c = keys[ixj];
                const bool up = (i & k) == 0;
                if ((a > c) == up) {
                    keys[i] = c;
                    keys[ixj] = a;
                }
            }
            __syncthreads();
        }
    }

    const int lane = threadIdx.x & 63;
    const int local = (int)(keys[threadIdx.x] & (uint64_t)(kLabelBlock - 1));
    const int64_t b = (int64_t)blockIdx.x * kLabelBlock + local;
    const bool valid = b < n;
    const int64_t src = valid ? (pix ? (int64_t)pix[b] : b) : 0;
    const float px = valid ? pos[src * 3 + 0] : 0.0f;
    const float py = valid ? pos[src * 3 + 1] : 0.0f;
    const float pz = valid ? pos[src * 3 + 2] : 0.0f;
    if (__ballot(valid) == 0) return;

    // Bounding sphere of the wave's points (valid lanes only).
    float mnx = valid ? px : INFINITY, mny = valid ? py : INFINITY, mnz = valid ? pz : INFINITY;
    float mxx = valid ? px : -INFINITY, mxy = valid ? py : -INFINITY, mxz = valid ? pz : -INFINITY;
    for (int off = 32; off > 0; off >>= 1) {
        mnx = fminf(mnx, __shfl_xor(mnx, off));
        mny = fminf(mny, __shfl_xor(mny, off));
        mnz = fminf(mnz, __shfl_xor(mnz, off));
        mxx = fmaxf(mxx, __shfl_xor(mxx, off));
        mxy = fmaxf(mxy, __shfl_xor(mxy, off));
        mxz = fmaxf(mxz, __shfl_xor(mxz, off));
    }
    const float cx = 0.5f * (mnx + mxx), cy = 0.5f * (mny + mxy), cz = 0.5f * (mnz + mxz);
    const float hx = 0.5f * (mxx - mnx), hy = 0.5f * (mxy - mny), hz = 0.5f * (mxz - mnz);
    const float rho = sqrtf(hx * hx + hy * hy + hz * hz) * 1.0001f;
    const float scale = fmaxf(__uint_as_float(scale_bits), fmaxf(fabsf(cx), fmaxf(fabsf(cy), fabsf(cz))) + rho);
    const float margin = 1e-3f * (1.0f + scale);
    // With a non-finite bounding box, nothing is culled (the exact test alone decides).
    const bool cull_ok = isfinite(rho) && isfinite(cx) && isfinite(cy) && isfinite(cz) && isfinite(margin);

    uint32_t word = 0;                                   // bit i: light l0 + i is visible
    for (int i = 0; i < nl; ++i) {
        const float4 l = Lg[i];
        const float dx = l.x - px, dy = l.y - py, dz = l.z - pz;
        const float dd = (dx * dx + dy * dy) + dz * dz;
        const float gx = l.x - cx, gy = l.y - cy, gz = l.z - cz;                // bundle axis pbar -> l
        const float gg = gx * gx + gy * gy + gz * gz;
        const float ginv = gg > 0.0f ? 1.0f / gg : 0.0f;
        uint32_t occ_bits = 0;
        for (int c0 = 0; c0 < n_spheres; c0 += 64) {
            const int s = c0 + lane;
            bool keep = false;
            if (s < n_spheres) {
                const float4 sc = S[s];
                const float ox = sc.x - cx, oy = sc.y - cy, oz = sc.z - cz;
                const float t = fminf(fmaxf((ox * gx + oy * gy + oz * gz) * ginv, 0.0f), 1.0f);
                const float qx = ox - t * gx, qy = oy - t * gy, qz = oz - t * gz;
                const float lim = R[s] + rho + margin;
                keep = !cull_ok || qx * qx + qy * qy + qz * qz <= lim * lim;
            }
            uint64_t mask = __ballot(keep);
            // Survivors in groups of four (a short group repeats its last sphere; a
            // repeated test leaves the OR unchanged): all LDS reads are issued before
            // the tests, and the test is branch-free.
            while (mask) {
                int sq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    sq[q] = mask ? c0 + __builtin_ctzll(mask) : sq[q > 0 ? q - 1 : 0];
                    mask &= mask - 1;
                }
                float4 sc[4];
                uint32_t ib[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    sc[q] = S[sq[q]];
                    ib[q] = inside[sq[q]];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float ox = sc[q].x - px, oy = sc[q].y - py, oz = sc[q].z - pz;
                    const float cc = ((ox * ox + oy * oy) + oz * oz) - sc[q].w;
                    const float bb = (ox * dx + oy * dy) + oz * dz;
                    // closest point p (bb <= 0): p inside; the light (bb >= dd): light inside;
                    // otherwise the interior test, as bit arithmetic (no divergent branches)
                    const uint32_t near_p = bb <= 0.0f;
                    const uint32_t near_l = (bb >= dd) & ~near_p;
                    const uint32_t mid = ~(near_p | near_l) & 1u;
                    const uint32_t o = (near_p & (uint32_t)(cc < 0.0f)) | (near_l & (ib[q] >> i)) |
                                       (mid & (uint32_t)(cc * dd < bb * bb));
                    occ_bits |= o;
                }
            }
        }
        if (!(occ_bits & 1u)) word |= 1u << i;
    }
    if (!valid) return;
    uint8_t* out = labels + b * (int64_t)m + l0;
    if (nl == 8 && ((uintptr_t)out & 7u) == 0) {
        uint32_t w0 = 0, w1 = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            w0 |= ((word >> i) & 1u) << (8 * i);
            w1 |= ((word >> (4 + i)) & 1u) << (8 * i);
        }
        *reinterpret_cast<uint2*>(out) = make_uint2(w0, w1);
    } else {
        for (int i = 0; i < nl; ++i) out[i] = (uint8_t)((word >> i) & 1u);
    }
}

size_t labels_smem_bytes(int m, int n_spheres) {
    (void)m;
    return (size_t)n_spheres * 16 + (size_t)((n_spheres + 3) & ~3) * 4 + (size_t)kLabelLights * 16 +
           (size_t)n_spheres * 4;
}

hipError_t launch_labels(const float* pos, const int32_t* pix, int64_t n, const float* lights, int m,
                         const float* spheres, int n_spheres, uint8_t* labels, hipStream_t st) {
    const size_t smem = labels_smem_bytes(m, n_spheres);
    const int64_t bx = (n + kLabelBlock - 1) / kLabelBlock;
    // Eight lights per block unless that leaves fewer than two blocks per CU.
    int lpb = kLabelLights;
    while (lpb > 1 && bx * ((m + lpb - 1) / lpb) < 2 * (int64_t)cu_count()) lpb >>= 1;
    const dim3 grid((unsigned)bx, (unsigned)((m + lpb - 1) / lpb));
    hipLaunchKernelGGL(labels_kernel, grid, dim3(kLabelBlock), smem, st, pos, pix, n, lights, m, spheres, n_spheres,
                       labels, lpb);
    return hipGetLastError();
}

}  // namespace nvc
