// FP64 forward pass of the cache and its training loss, for gradient checks by
// central finite differences (Sec. 3.3: the network and the grid are trained by
// backpropagation; a difference quotient with h = 1e-3 needs the loss to far
// more digits than the FP32 / FP16 paths give).  Not part of the hot path:
// plain FP64 arithmetic on the vector units, no matrix cores.
//
// One block per point.  The cell and fraction of a position are decided in
// FP32 exactly as in the other kernels (s = fl32(x N), the fraction s - c is
// exact); trilinear weights, features, network, sigmoid and loss are FP64.
// Every dot product runs over its inputs in index order; a point's loss sums
// its lights in order; the mean sums the points in index order (a second,
// one-block kernel), so the result does not depend on the launch.
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace nvc {

GridDev grid_to_dev(const GridHost& g);

namespace {

constexpr int kThreads = 128;          // >= width, n_out (<= 128) and n_levels (<= 32)

struct F64Args {
    GridDev g;
    NetShape s;
    const double* table;
    const double* w;
    const float* pos;
    int64_t n;
    const uint8_t* labels;
    int loss;
    double* z;
    uint8_t* masks;
    double* loss_pt;                   // [n] per-point loss sums, or NULL
};

__device__ inline double sigmoid_f64(double z) {
    if (z >= 0.0) return 1.0 / (1.0 + exp(-z));
    const double e = exp(z);
    return e / (1.0 + e);
}

__global__ __launch_bounds__(kThreads) void forward_f64_kernel(F64Args a) {
    __shared__ double hbuf[2][kThreads];
    __shared__ double lterm[kThreads];
    const int64_t p = blockIdx.x;
    const int t = threadIdx.x;
    const GridDev& g = a.g;
    const int L = g.n_levels, F = g.n_feat;
    const int64_t T = (int64_t)g.T;

    // encoding: thread l gathers level l
    if (t < L) {
        const float x = clamp_unit(a.pos[p * 3 + 0]);
        const float y = clamp_unit(a.pos[p * 3 + 1]);
        const float zz = clamp_unit(a.pos[p * 3 + 2]);
        Corners c;
        level_corners(g, t, x, y, zz, c);                 // corner indices (the cell decided in FP32)
        const int N = g.res[t];
        const float Nf = (float)N;
        const float sx = x * Nf, sy = y * Nf, sz = zz * Nf;
        const double fx = (double)(sx - (float)min((int)floorf(sx), N - 1));
        const double fy = (double)(sy - (float)min((int)floorf(sy), N - 1));
        const double fz = (double)(sz - (float)min((int)floorf(sz), N - 1));
        const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
        for (int j = 0; j < F; ++j) {
            double e = 0.0;
            for (int k = 0; k < 8; ++k) {
                const double wk = (wx[k & 1] * wy[(k >> 1) & 1]) * wz[(k >> 2) & 1];
                e += wk * a.table[((int64_t)t * T + c.idx[k]) * F + j];
            }
            hbuf[0][t * F + j] = e;
        }
    }
    __syncthreads();

    const NetShape& s = a.s;
    const int n_layers = s.n_hidden + 1;
    const int mbytes = (s.width + 7) / 8;
    int64_t woff = 0;
    int cur = 0;
    for (int k = 0; k < n_layers; ++k) {
        const int in = k == 0 ? s.n_in : s.width;
        const int out = k == n_layers - 1 ? s.n_out : s.width;
        double pre = 0.0;
        if (t < out) {
            const double* wr = a.w + woff + (int64_t)t * in;
            for (int i = 0; i < in; ++i) pre += wr[i] * hbuf[cur][i];
        }
        if (k < n_layers - 1) {
            const bool pos_pre = t < out && pre > 0.0;
            const uint64_t bits = __ballot(pos_pre);
            if (a.masks && (t & 63) == 0) {
                const int b0 = (t >> 6) * 8;
                uint8_t* mrow = a.masks + p * (int64_t)(s.n_hidden * mbytes) + k * mbytes;
                for (int b = b0; b < min(b0 + 8, mbytes); ++b) mrow[b] = (uint8_t)(bits >> (8 * (b - b0)));
            }
            const double slope = s.act == 1 ? (double)s.slope : 0.0;
            if (t < out) hbuf[cur ^ 1][t] = pos_pre ? pre : slope * pre;
        } else if (t < out) {
            if (a.z) a.z[p * s.n_out + t] = pre;
            if (a.labels) {
                const double y = (double)a.labels[p * s.n_out + t];
                double term;
                if (a.loss == NVC_LOSS_BCE) {
                    term = fmax(pre, 0.0) - y * pre + log1p(exp(-fabs(pre)));
                } else {
                    const double d = sigmoid_f64(pre) - y;
                    term = d * d;
                }
                lterm[t] = term;
            }
        }
        __syncthreads();
        woff += (int64_t)in * out;
        cur ^= 1;
    }
    if (a.labels && a.loss_pt && t == 0) {
        double sum = 0.0;
        for (int j = 0; j < s.n_out; ++j) sum += lterm[j];
        a.loss_pt[p] = sum;
    }
}

// mean = (sum over points in index order) / (n * n_out): 256 threads sum
// consecutive ranges, thread 0 adds the 256 partial sums in order.
__global__ __launch_bounds__(256) void mean_f64_kernel(const double* __restrict__ loss_pt, int64_t n, int n_out,
                                                       double* __restrict__ out) {
    __shared__ double part[256];
    const int t = threadIdx.x;
    const int64_t per = (n + 255) / 256;
    const int64_t lo = min(n, (int64_t)t * per), hi = min(n, lo + per);
    double s = 0.0;
    for (int64_t i = lo; i < hi; ++i) s += loss_pt[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
        for (int i = 0; i < 256; ++i) tot += part[i];
        *out = tot / ((double)n * (double)n_out);
    }
}

}  // namespace

hipError_t launch_forward_f64(const GridHost& gh, const NetShape& s, const double* table, const double* w,
                              const float* pos, int64_t n, const uint8_t* labels, int loss, double* z,
                              uint8_t* masks, double* loss_out, hipStream_t st) {
    F64Args a{};
    a.g = grid_to_dev(gh);
    a.s = s;
    a.table = table;
    a.w = w;
    a.pos = pos;
    a.n = n;
    a.labels = labels;
    a.loss = loss;
    a.z = z;
    a.masks = masks;
    a.loss_pt = labels ? loss_out : nullptr;
    forward_f64_kernel<<<(unsigned)n, kThreads, 0, st>>>(a);
    if (labels) mean_f64_kernel<<<1, 256, 0, st>>>(loss_out, n, s.n_out, loss_out + n);
    return hipGetLastError();
}

}  // namespace nvc
