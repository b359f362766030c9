// Warm-start network kernels for gfx950: per-node features, a small MLP
// (16 -> 128 -> 128 -> 1, ReLU) trained and evaluated with BF16 MFMA
// operands and FP32 accumulation, AdamW, and the rounding of its prediction
// to an initial Lam.  Not part of the paper's method: the GDP started from
// the prediction reaches the same certified optimum as from zero; only the
// iteration count changes.
//
// Layout: activations are node-major (row v, column j); bf16 values are
// stored as uint16 (the upper half of the float32 pattern, rounded to
// nearest even).  Parameter vector (FP32 master copy, f2m_mlp.h order):
//   W1 [128][16], b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1].
#include "f2m_mlp.h"

#include <hipcub/hipcub.hpp>

namespace f2m {

namespace {

constexpr int kB = 256;
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return (uint16_t)((b >> 16) | 0x40u);   // NaN
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C[m][n] (+)= sum_k A(m, k) * B(k, n) over k in one K chunk, bf16 operands
// with arbitrary strides, FP32 accumulate on v_mfma_f32_16x16x16_bf16.
// One wave per 16x16 output tile: lane l holds A(i = l%16, k = 4(l/16)+q),
// B(k = 4(l/16)+q, j = l%16) and returns C(4(l/16)+q, l%16), q = 0..3.
// Out-of-range rows/columns/k read as zero; out is [chunk][M][N].
__global__ __launch_bounds__(64) void k_gemm_bf16(GemmArgs g)
{
    const int l = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * 16, n0 = (int64_t)blockIdx.y * 16;
    const int64_t chunk = blockIdx.z;
    const int64_t k0 = chunk * g.kchunk, k1 = min(g.K, k0 + g.kchunk);
    const int64_t i = m0 + (l & 15), j = n0 + (l & 15);
    const int kq = 4 * (l >> 4);
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t k = k0; k < k1; k += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t kk = k + kq + q;
            const bool ok = kk < k1;
            a[q] = (ok && i < g.M) ? (short)g.A[i * g.sam + kk * g.sak] : (short)0;
            b[q] = (ok && j < g.N) ? (short)g.B[kk * g.sbk + j * g.sbn] : (short)0;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t r = m0 + kq + q;
        if (r < g.M && j < g.N) g.out[(chunk * g.M + r) * g.N + j] = acc[q];
    }
}

// out[m][n] = sum over chunks (fixed order: deterministic)
__global__ __launch_bounds__(kB) void k_sum_chunks(const float *part, int64_t nchunks, int64_t mn, float *out)
{
    const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (e >= mn) return;
    float s = 0.0f;
    for (int64_t c = 0; c < nchunks; ++c) s += part[c * mn + e];
    out[e] = s;
}

__global__ __launch_bounds__(kB) void k_to_bf16(const float *src, int64_t count, uint16_t *dst)
{
    const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (e < count) dst[e] = to_bf16(src[e]);
}

// h = relu(z + bias[col]) as bf16 (and fp32 if hf is set)
__global__ __launch_bounds__(kB) void k_bias_relu(const float *z, const float *bias, int64_t rows, int64_t cols,
                                                  uint16_t *hb, float *hf)
{
    const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (e >= rows * cols) return;
    const float h = fmaxf(z[e] + bias[e % cols], 0.0f);
    hb[e] = to_bf16(h);
    if (hf) hf[e] = h;
}

// y[v] = sum_j relu(z2[v][j] + b2[j]) * w3[j] + b3 (layer 3 in FP32)
__global__ __launch_bounds__(kB) void k_out(const float *z2, const float *theta, int64_t rows, float *y, float *h2)
{
    const int64_t v = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (v >= rows) return;
    const float *b2 = theta + kMlpB2, *w3 = theta + kMlpW3;
    float s = theta[kMlpB3];
    for (int j = 0; j < kMlpH; ++j) {
        const float h = fmaxf(z2[v * kMlpH + j] + b2[j], 0.0f);
        if (h2) h2[v * kMlpH + j] = h;
        s = fmaf(h, w3[j], s);
    }
    y[v] = s;
}

// dy = 2 (y - t) / N; g2 = dy * w3 * [h2 > 0] as bf16; per-row sums for
// the loss
__global__ __launch_bounds__(kB) void k_out_grad(const float *y, const float *t, const float *h2, const float *theta,
                                                 int64_t rows, float inv_n, float *dy, uint16_t *g2b, float *g2f,
                                                 float *sq)
{
    const int64_t v = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (v >= rows) return;
    const float r = y[v] - t[v];
    const float d = 2.0f * r * inv_n;
    dy[v] = d;
    sq[v] = r * r;
    const float *w3 = theta + kMlpW3;
    for (int j = 0; j < kMlpH; ++j) {
        const float g = h2[v * kMlpH + j] > 0.0f ? d * w3[j] : 0.0f;
        g2f[v * kMlpH + j] = g;
        g2b[v * kMlpH + j] = to_bf16(g);
    }
}

// g1 = pre * [h1 > 0] (h1 as bf16 from the forward pass)
__global__ __launch_bounds__(kB) void k_mask_bf16(const float *pre, const uint16_t *h1b, int64_t count, uint16_t *gb,
                                                  float *gf)
{
    const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (e >= count) return;
    const float g = from_bf16(h1b[e]) > 0.0f ? pre[e] : 0.0f;
    gb[e] = to_bf16(g);
    gf[e] = g;
}

// column sums of a [rows][cols] matrix, weighted by w[row] if given: block
// partials [block][cols] (rows in fixed blocks, deterministic)
__global__ __launch_bounds__(kB) void k_col_partials(const float *a, const float *w, int64_t rows, int64_t cols,
                                                     int64_t rows_per_block, float *part)
{
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block, r1 = min(rows, r0 + rows_per_block);
    for (int64_t c = threadIdx.x; c < cols; c += kB) {
        float s = 0.0f;
        for (int64_t r = r0; r < r1; ++r) s += w ? a[r * cols + c] * w[r] : a[r * cols + c];
        part[blockIdx.x * cols + c] = s;
    }
}

__global__ __launch_bounds__(kB) void k_adamw(float *theta, const float *grad, float *m, float *v, int64_t count,
                                              float lr, float b1, float b2, float eps, float wd, float c1, float c2)
{
    const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (e >= count) return;
    const float g = grad[e];
    const float mm = b1 * m[e] + (1.0f - b1) * g;
    const float vv = b2 * v[e] + (1.0f - b2) * g * g;
    m[e] = mm;
    v[e] = vv;
    const float mh = mm / c1, vh = vv / c2;
    theta[e] -= lr * (mh / (sqrtf(vh) + eps) + wd * theta[e]);
}

// features of position p (sorted order) written at its label: 16 sorted
// neighbour distances / scale, bf16
__global__ __launch_bounds__(kB) void k_features(const int64_t *nbr_d, const int32_t *orig, int64_t n,
                                                 const float *scale, uint16_t *feat)
{
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= n) return;
    const int64_t v = orig[p];
    const float inv = 1.0f / scale[0];
    for (int j = 0; j < kMlpIn; ++j) feat[v * kMlpIn + j] = to_bf16(sqrtf((float)nbr_d[p * kMlpIn + j]) * inv);
}

__global__ void k_median_scale(const uint64_t *sorted_d, int64_t count, float *scale)
{
    if (threadIdx.x != 0) return;
    const float s = sqrtf((float)sorted_d[(count - 1) / 2]);
    scale[0] = s > 1.0f ? s : 1.0f;
}

// Lam0[v] = round_half_even(2 * scale * y[v]), clamped to |Lam0| <= limit
__global__ __launch_bounds__(kB) void k_lam_from_pred(const float *y, const float *scale, int64_t n, int64_t limit,
                                                      int64_t *lam)
{
    const int64_t v = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (v >= n) return;
    double x = rint(2.0 * (double)scale[0] * (double)y[v]);
    if (!(x == x)) x = 0.0;
    x = x > (double)limit ? (double)limit : (x < -(double)limit ? -(double)limit : x);
    lam[v] = (int64_t)x;
}

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_gemm_bf16(const GemmArgs &g, hipStream_t st)
{
    const int64_t chunks = (g.K + g.kchunk - 1) / g.kchunk;
    hipLaunchKernelGGL(k_gemm_bf16, dim3(nblk(g.M, 16), nblk(g.N, 16), (unsigned)std::max<int64_t>(chunks, 1)),
                       dim3(64), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_sum_chunks(const float *part, int64_t nchunks, int64_t mn, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_chunks, dim3(nblk(mn, kB)), dim3(kB), 0, st, part, nchunks, mn, out);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *src, int64_t count, uint16_t *dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(count, kB)), dim3(kB), 0, st, src, count, dst);
    return hipGetLastError();
}

hipError_t launch_bias_relu(const float *z, const float *bias, int64_t rows, int64_t cols, uint16_t *hb, float *hf,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_bias_relu, dim3(nblk(rows * cols, kB)), dim3(kB), 0, st, z, bias, rows, cols, hb, hf);
    return hipGetLastError();
}

hipError_t launch_out(const float *z2, const float *theta, int64_t rows, float *y, float *h2, hipStream_t st)
{
    hipLaunchKernelGGL(k_out, dim3(nblk(rows, kB)), dim3(kB), 0, st, z2, theta, rows, y, h2);
    return hipGetLastError();
}

hipError_t launch_out_grad(const float *y, const float *t, const float *h2, const float *theta, int64_t rows,
                           float inv_n, float *dy, uint16_t *g2b, float *g2f, float *sq, hipStream_t st)
{
    hipLaunchKernelGGL(k_out_grad, dim3(nblk(rows, kB)), dim3(kB), 0, st, y, t, h2, theta, rows, inv_n, dy, g2b, g2f,
                       sq);
    return hipGetLastError();
}

hipError_t launch_mask_bf16(const float *pre, const uint16_t *h1b, int64_t count, uint16_t *gb, float *gf,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_mask_bf16, dim3(nblk(count, kB)), dim3(kB), 0, st, pre, h1b, count, gb, gf);
    return hipGetLastError();
}

hipError_t launch_col_sums(const float *a, const float *w, int64_t rows, int64_t cols, float *part, float *out,
                           int64_t nparts, hipStream_t st)
{
    const int64_t rpb = (rows + nparts - 1) / nparts;
    hipLaunchKernelGGL(k_col_partials, dim3((unsigned)nparts), dim3(kB), 0, st, a, w, rows, cols, rpb, part);
    return launch_sum_chunks(part, nparts, cols, out, st);
}

hipError_t launch_adamw(float *theta, const float *grad, float *m, float *v, int64_t count, float lr, float b1,
                        float b2, float eps, float wd, int64_t step, hipStream_t st)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adamw, dim3(nblk(count, kB)), dim3(kB), 0, st, theta, grad, m, v, count, lr, b1, b2, eps, wd,
                       c1, c2);
    return hipGetLastError();
}

size_t median_temp_bytes(int64_t count)
{
    size_t b = 0;
    (void)hipcub::DeviceRadixSort::SortKeys(nullptr, b, (const uint64_t *)nullptr, (uint64_t *)nullptr, (int)count, 0,
                                            64);
    return b;
}

hipError_t launch_features(const int64_t *nbr_d, const int32_t *orig, int64_t n, uint64_t *sorted_tmp, void *temp,
                           size_t temp_bytes, float *scale, uint16_t *feat, hipStream_t st)
{
    const int64_t count = n * kMlpIn;
    size_t tb = temp_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortKeys(temp, tb, (const uint64_t *)nbr_d, sorted_tmp, (int)count, 0, 64,
                                                     st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_median_scale, dim3(1), dim3(64), 0, st, sorted_tmp, count, scale);
    hipLaunchKernelGGL(k_features, dim3(nblk(n, kB)), dim3(kB), 0, st, nbr_d, orig, n, scale, feat);
    return hipGetLastError();
}

hipError_t launch_lam_from_pred(const float *y, const float *scale, int64_t n, int64_t limit, int64_t *lam,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_lam_from_pred, dim3(nblk(n, kB)), dim3(kB), 0, st, y, scale, n, limit, lam);
    return hipGetLastError();
}

}  // namespace f2m
