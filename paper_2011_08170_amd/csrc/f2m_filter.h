// The complete-graph scan's float filter and culling test, written once for
// the device kernels and for host-side checks of their conservativeness.
//
// For a row v with threshold theta_v >= 0 (an upper bound of the row's 4th
// smallest Z; a pair with Z > theta_v cannot change any statistic the GDP
// needs) plus a slack slk >= 0, a pair (v, u) is needed only if
//     Z_vu = 2c_vu - Lam_v - Lam_u <= theta_v + slk.
// With c = nint(sqrt D) >= sqrt(D) - 1/2 that requires sqrt(D) < h = hv + hu,
// hv = (theta_v + slk + Lam_v + 1)/2, hu = Lam_u/2, i.e. E = D - h^2 < 0.  In
// centred coordinates
//     E = K_v + q_u + (-2x_v) x_u + (-2y_v) y_u + (-2hv) hu,
//     K_v = x_v^2 + y_v^2 - hv^2,  q_u = x_u^2 + y_u^2 - hu^2,
// three FMAs per pair in float.  Every rounding of that chain is bounded by
// 2^-24 M_v, M_v = 2(x_v^2 + y_v^2 + hv^2 + max_u(x_u^2 + y_u^2) + max_u hu^2),
// so the pair is skipped only when the float value exceeds -K_v by more than
// 2^-18 M_v (four times the bound and more): the filter never drops a pair
// with Z <= theta_v + slk.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace f2m {

struct Row {
    float a, b, c, thr;   // filter: skip when a*xu + b*yu + c*hu + qu > thr
    float xv, yv;
    int64_t lamv, theta;
    int64_t v;
    int64_t slk = 0;      // the filter passes Z <= theta + slk
};

// Column record of a city: centred coordinates (exact integers in float),
// h = Lam/2 and q = x^2 + y^2 - h^2.
__host__ __device__ __forceinline__ float4 col_record(float x, float y, int64_t lam)
{
    const float h = (float)(0.5 * (double)lam);
    return make_float4(x, y, h, fmaf(x, x, fmaf(y, y, -h * h)));
}

// An upper bound of x^2 + y^2 (rounded up by a relative 2^-22, plus one).
__host__ __device__ __forceinline__ float xy2_bound(float x, float y)
{
    return fmaf(x, x, y * y) * (1.0f + 0x1p-22f) + 1.0f;
}

// Recomputes the filter of a row from theta and slk.
__host__ __device__ __forceinline__ void set_filter(Row &r, float colmax)
{
    const float hv = (float)(0.5 * (double)(r.theta + r.slk + r.lamv + 1));
    r.a = -2.0f * r.xv;
    r.b = -2.0f * r.yv;
    r.c = -2.0f * hv;
    const float K = fmaf(r.xv, r.xv, fmaf(r.yv, r.yv, -hv * hv));
    const float M = 2.0f * (r.xv * r.xv + r.yv * r.yv + hv * hv + colmax);
    r.thr = M * 0x1p-18f - K;
}

__host__ __device__ __forceinline__ float filter_value(const Row &r, float4 cd)
{
    return fmaf(r.c, cd.z, fmaf(r.b, cd.y, fmaf(r.a, cd.x, cd.w)));
}

// max over columns of x^2 + y^2 plus the square of an upper bound on |hu|
__host__ __device__ __forceinline__ float col_bound(float xy2max, long long maxabs_lam)
{
    const float hu = (float)(maxabs_lam / 2 + 1);
    return xy2max + hu * hu;
}

// Culling test of a column box against a box of rows.  A pair (v, u) can
// pass the filter only if sqrt(D) <= hv + hu with hv = (theta_v + slk +
// Lam_v + 1)/2 (the largest over the rows) and hu = Lam_u/2 (the largest
// over the columns).  Every pair of the two boxes has D >= dx^2 + dy^2 (the
// squared distance between the boxes); false means no pair can pass.  Box
// corners are integers below 2^20 in magnitude, so dx and dy are exact;
// hv and hu are float roundings of exact values, hence the widening of
// hv + hu, and the 2^-16 relative margin covers the roundings of the two
// squares.  Empty boxes (min +inf, max -inf) and hv = -inf never pass.
__host__ __device__ __forceinline__ bool may_pass(float4 b, float4 rbox, float hv, float hu)
{
    const float dx = fmaxf(0.0f, fmaxf(b.x - rbox.y, rbox.x - b.y));
    const float dy = fmaxf(0.0f, fmaxf(b.z - rbox.w, rbox.z - b.w));
    float hs = hv + hu;
    hs += 1e-6f * (fabsf(hv) + fabsf(hu)) + 1.0f;
    if (!(hs > 0.0f)) return false;
    return fmaf(dx, dx, dy * dy) <= hs * hs * (1.0f + 0x1p-16f);
}

}  // namespace f2m
