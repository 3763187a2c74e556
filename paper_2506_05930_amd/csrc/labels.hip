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

__global__ __launch_bounds__(256) void pixel_count_kernel(uint32_t k0, uint32_t k1, uint32_t frame, uint32_t n_pix,
                                                          int64_t batch, uint32_t* __restrict__ counts) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const uint32_t r0 = philox_first_word((uint32_t)b, (uint32_t)((uint64_t)b >> 32), frame, 1u, k0, k1);
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

hipError_t launch_select_pixels(uint64_t seed, uint32_t frame, int64_t n_pix, int64_t batch, int32_t* pix,
                                void* workspace, hipStream_t st) {
    uint32_t* counts = reinterpret_cast<uint32_t*>(workspace);
    uint32_t* offs = counts + n_pix;
    uint32_t* sums = offs + n_pix;
    const int64_t nsums = (n_pix + kScanBlock - 1) / kScanBlock;
    const unsigned pb = (unsigned)((n_pix + 255) / 256);
    fill_u32_kernel<<<pb, 256, 0, st>>>(counts, n_pix, 0u);
    pixel_count_kernel<<<(unsigned)((batch + 255) / 256), 256, 0, st>>>((uint32_t)seed, (uint32_t)(seed >> 32), frame,
                                                                       (uint32_t)n_pix, batch, counts);
    pixel_scan_local_kernel<<<(unsigned)nsums, 1024, 0, st>>>(counts, n_pix, offs, sums);
    pixel_scan_sums_kernel<<<1, 1024, 0, st>>>(sums, (int)nsums);
    pixel_emit_kernel<<<pb, 256, 0, st>>>(counts, offs, sums, n_pix, pix);
    return hipGetLastError();
}

// ------------------------------------------------------------------ shadow labels
__device__ inline uint32_t float_key(float v) { return __float_as_uint(v); }   // order-preserving for v >= 0

__global__ __launch_bounds__(256) void labels_kernel(const float* __restrict__ pos, const int32_t* __restrict__ pix,
                                                     int64_t n, const float* __restrict__ lights, int m,
                                                     const float* __restrict__ spheres, int n_spheres,
                                                     uint8_t* __restrict__ labels) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    float4* S = reinterpret_cast<float4*>(smem_raw);                          // (cx, cy, cz, r*r)
    float* R = reinterpret_cast<float*>(S + n_spheres);                       // r
    float4* Lg = reinterpret_cast<float4*>(R + ((n_spheres + 3) & ~3));       // (lx, ly, lz, 0)
    const int lw = (m + 31) / 32;                                             // words of light bits
    uint32_t* inside = reinterpret_cast<uint32_t*>(Lg + m);                   // [n_spheres][lw]
    __shared__ uint32_t scale_bits;
    if (threadIdx.x == 0) scale_bits = 0;
    __syncthreads();
    uint32_t my_scale = 0;
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        const float lx = lights[4 * j + 0], ly = lights[4 * j + 1], lz = lights[4 * j + 2];
        Lg[j] = make_float4(lx, ly, lz, 0.0f);
        my_scale = max(my_scale, float_key(fmaxf(fabsf(lx), fmaxf(fabsf(ly), fabsf(lz)))));
    }
    for (int s = threadIdx.x; s < n_spheres; s += blockDim.x) {
        const float cx = spheres[4 * s + 0], cy = spheres[4 * s + 1], cz = spheres[4 * s + 2], r = spheres[4 * s + 3];
        const float rr = r * r;
        S[s] = make_float4(cx, cy, cz, rr);
        R[s] = r;
        my_scale = max(my_scale, float_key(fmaxf(fabsf(cx), fmaxf(fabsf(cy), fabsf(cz))) + fabsf(r)));
        for (int w = 0; w < lw; ++w) {
            uint32_t bits = 0;
            for (int j = 0; j < 32 && 32 * w + j < m; ++j) {
                const int li = 32 * w + j;
                const float ex = cx - lights[4 * li + 0], ey = cy - lights[4 * li + 1], ez = cz - lights[4 * li + 2];
                if (((ex * ex + ey * ey) + ez * ez) < rr) bits |= 1u << j;
            }
            inside[s * lw + w] = bits;
        }
    }
    atomicMax(&scale_bits, my_scale);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int64_t b = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64 + lane;
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
    uint8_t* out = labels + (valid ? b : 0) * (int64_t)m;
    for (int j0 = 0; j0 < m; j0 += 32) {
        uint32_t word = 0;                       // bit i: light j0 + i is visible
        const int jn = min(32, m - j0);
        for (int i = 0; i < jn; ++i) {
            const int j = j0 + i;
            const float4 l = Lg[j];
            const float dx = l.x - px, dy = l.y - py, dz = l.z - pz;
            const float dd = (dx * dx + dy * dy) + dz * dz;
            const float gx = l.x - cx, gy = l.y - cy, gz = l.z - cz;            // bundle axis pbar -> l
            const float gg = gx * gx + gy * gy + gz * gz;
            const float ginv = gg > 0.0f ? 1.0f / gg : 0.0f;
            bool occ = false;
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
                while (mask) {
                    const int s2 = c0 + __builtin_ctzll(mask);
                    mask &= mask - 1;
                    const float4 sc = S[s2];
                    const float ox = sc.x - px, oy = sc.y - py, oz = sc.z - pz;
                    const float cc = ((ox * ox + oy * oy) + oz * oz) - sc.w;
                    const float bb = (ox * dx + oy * dy) + oz * dz;
                    bool o;
                    if (bb <= 0.0f)
                        o = cc < 0.0f;
                    else if (bb >= dd)
                        o = (inside[s2 * lw + (j >> 5)] >> (j & 31)) & 1u;
                    else
                        o = cc * dd < bb * bb;
                    occ = occ || o;
                }
            }
            if (!occ) word |= 1u << i;
        }
        if (!valid) continue;
        if (jn == 32 && ((uintptr_t)(out + j0) & 15u) == 0) {   // 32 labels as two 16-byte stores
            uint32_t w8[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                uint32_t v = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) v |= ((word >> (4 * q + i)) & 1u) << (8 * i);
                w8[q] = v;
            }
            *reinterpret_cast<uint4*>(out + j0) = make_uint4(w8[0], w8[1], w8[2], w8[3]);
            *reinterpret_cast<uint4*>(out + j0 + 16) = make_uint4(w8[4], w8[5], w8[6], w8[7]);
        } else {
            for (int i = 0; i < jn; ++i) out[j0 + i] = (uint8_t)((word >> i) & 1u);
        }
    }
}

size_t labels_smem_bytes(int m, int n_spheres) {
    const int lw = (m + 31) / 32;
    return (size_t)n_spheres * 16 + (size_t)((n_spheres + 3) & ~3) * 4 + (size_t)m * 16 + (size_t)n_spheres * lw * 4;
}

hipError_t launch_labels(const float* pos, const int32_t* pix, int64_t n, const float* lights, int m,
                         const float* spheres, int n_spheres, uint8_t* labels, hipStream_t st) {
    const size_t smem = labels_smem_bytes(m, n_spheres);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(labels_kernel, dim3(blocks), dim3(256), smem, st, pos, pix, n, lights, m, spheres, n_spheres,
                       labels);
    return hipGetLastError();
}

}  // namespace nvc
