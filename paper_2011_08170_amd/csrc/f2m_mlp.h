// Interface of the warm-start network kernels (f2m_mlp.hip) for the host
// runtime.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace f2m {

constexpr int kMlpIn = 16;    // features per node: sorted neighbour distances
constexpr int kMlpH = 128;    // hidden width
// offsets in the FP32 parameter vector
constexpr int64_t kMlpW1 = 0;
constexpr int64_t kMlpB1 = kMlpW1 + kMlpH * kMlpIn;
constexpr int64_t kMlpW2 = kMlpB1 + kMlpH;
constexpr int64_t kMlpB2 = kMlpW2 + kMlpH * kMlpH;
constexpr int64_t kMlpW3 = kMlpB2 + kMlpH;
constexpr int64_t kMlpB3 = kMlpW3 + kMlpH;
constexpr int64_t kMlpParams = kMlpB3 + 1;

// C (M x N) = sum over k of A(m, k) B(k, n); element (m, k) of A at
// A[m*sam + k*sak], (k, n) of B at B[k*sbk + n*sbn]; bf16 as uint16.
// The K range is cut in chunks of kchunk (a multiple of 16); out holds
// one [M][N] FP32 block per chunk.
struct GemmArgs {
    const uint16_t *A;
    const uint16_t *B;
    float *out;
    int64_t M, N, K, kchunk;
    int64_t sam, sak, sbk, sbn;
};

hipError_t launch_gemm_bf16(const GemmArgs &g, hipStream_t st);
hipError_t launch_sum_chunks(const float *part, int64_t nchunks, int64_t mn, float *out, hipStream_t st);
hipError_t launch_to_bf16(const float *src, int64_t count, uint16_t *dst, hipStream_t st);
hipError_t launch_bias_relu(const float *z, const float *bias, int64_t rows, int64_t cols, uint16_t *hb, float *hf,
                            hipStream_t st);
hipError_t launch_out(const float *z2, const float *theta, int64_t rows, float *y, float *h2, hipStream_t st);
hipError_t launch_out_grad(const float *y, const float *t, const float *h2, const float *theta, int64_t rows,
                           float inv_n, float *dy, uint16_t *g2b, float *g2f, float *sq, hipStream_t st);
hipError_t launch_mask_bf16(const float *pre, const uint16_t *h1b, int64_t count, uint16_t *gb, float *gf,
                            hipStream_t st);
// column sums (optionally weighted by w[row]) with nparts fixed row blocks
hipError_t launch_col_sums(const float *a, const float *w, int64_t rows, int64_t cols, float *part, float *out,
                           int64_t nparts, hipStream_t st);
hipError_t launch_adamw(float *theta, const float *grad, float *m, float *v, int64_t count, float lr, float b1,
                        float b2, float eps, float wd, int64_t step, hipStream_t st);
size_t median_temp_bytes(int64_t count);
// nbr_d: [n][16] squared distances by position; features by label
hipError_t launch_features(const int64_t *nbr_d, const int32_t *orig, int64_t n, uint64_t *sorted_tmp, void *temp,
                           size_t temp_bytes, float *scale, uint16_t *feat, hipStream_t st);
hipError_t launch_lam_from_pred(const float *y, const float *scale, int64_t n, int64_t limit, int64_t *lam,
                                hipStream_t st);

}  // namespace f2m
