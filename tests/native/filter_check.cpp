// Host check of the scan's float filter and culling test (f2m_filter.h): no
// pair whose exact Z is at most theta + slk may be skipped.  Adversarial
// inputs: coordinates at the full 2^20 span, multipliers up to 2^37 in
// magnitude, thresholds placed exactly at, one below and one above each
// pair's Z, distances at the EUC_2D rounding boundaries D = k^2 + k and
// k^2 + k + 1.  Prints "checked tight violations" for the pair filter and
// for the box test; the test suite requires zero violations.
#include "f2m_filter.h"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

using namespace f2m;

// floor(sqrt(x)) exactly, then the EUC_2D length nint(sqrt(D))
static int64_t isqrt_exact(int64_t x)
{
    int64_t r = (int64_t)sqrt((double)x);
    while (r > 0 && r * r > x) --r;
    while ((r + 1) * (r + 1) <= x) ++r;
    return r;
}
static int64_t nint_exact(int64_t D) { return (isqrt_exact(4 * D) + 1) / 2; }

struct City {
    int32_t x, y;   // centred, |.| <= 2^19
    int64_t lam;
};

struct Tally {
    long long checked = 0, tight = 0, bad = 0;
};

// One row against one column with threshold theta and slack slk; the
// instance's column bound comes from xy2max and maxabs.
static void check_pair(const City &v, const City &u, int64_t theta, int64_t slk, float xy2max, long long maxabs,
                       Tally &pf, Tally &pb)
{
    const int64_t dx = (int64_t)v.x - u.x, dy = (int64_t)v.y - u.y;
    const int64_t Z = 2 * nint_exact(dx * dx + dy * dy) - v.lam - u.lam;
    const bool needed = Z <= theta + slk;
    Row r;
    r.xv = (float)v.x;
    r.yv = (float)v.y;
    r.lamv = v.lam;
    r.theta = theta;
    r.slk = slk;
    set_filter(r, col_bound(xy2max, maxabs));
    const float4 cu = col_record((float)u.x, (float)u.y, u.lam);
    const bool pass = filter_value(r, cu) <= r.thr;
    ++pf.checked;
    if (Z == theta + slk) ++pf.tight;
    if (needed && !pass) {
        ++pf.bad;
        if (pf.bad <= 5)
            std::printf("filter drops Z=%lld theta=%lld slk=%lld v=(%d,%d,%lld) u=(%d,%d,%lld)\n", (long long)Z,
                        (long long)theta, (long long)slk, v.x, v.y, (long long)v.lam, u.x, u.y, (long long)u.lam);
    }
    // the same pair as two one-point boxes, with the kernel's hv and hu
    const float4 rb = make_float4((float)v.x, (float)v.x, (float)v.y, (float)v.y);
    const float4 cb = make_float4((float)u.x, (float)u.x, (float)u.y, (float)u.y);
    const bool bp = may_pass(cb, rb, -0.5f * r.c, cu.z);
    ++pb.checked;
    if (Z == theta + slk) ++pb.tight;
    if (needed && !bp) {
        ++pb.bad;
        if (pb.bad <= 5)
            std::printf("box test drops Z=%lld theta=%lld slk=%lld\n", (long long)Z, (long long)theta,
                        (long long)slk);
    }
}

int main(int argc, char **argv)
{
    const long long rounds = argc > 1 ? std::atoll(argv[1]) : 200000;
    std::mt19937_64 rng(20111708);
    Tally pf, pb;
    const int32_t H = 1 << 19;   // centred coordinates in [-2^19, 2^19)
    std::uniform_int_distribution<int32_t> coord(-H, H - 1);
    for (long long it = 0; it < rounds; ++it) {
        // a small instance: the row, its column and a few others that set
        // the column bounds (the largest |Lam| and x^2 + y^2 of the columns)
        const int scale_case = (int)(it % 4);
        const int64_t lam_mag = scale_case == 0 ? (int64_t(1) << 37) : scale_case == 1 ? (int64_t(1) << 24)
                                                                 : scale_case == 2 ? 4000000 : 3000;
        std::uniform_int_distribution<int64_t> lamd(-lam_mag, lam_mag);
        City v{coord(rng), coord(rng), lamd(rng)};
        City u;
        const int geo = (int)((it / 4) % 3);
        if (geo == 0) {
            u = City{coord(rng), coord(rng), lamd(rng)};
        } else {
            // a short or a rounding-boundary distance from v
            std::uniform_int_distribution<int32_t> off(-3000, 3000);
            u = City{v.x + off(rng), v.y + off(rng), lamd(rng)};
            if (geo == 2) {
                // D = k^2 + k or k^2 + k + 1 along x
                std::uniform_int_distribution<int64_t> kd(1, 700);
                const int64_t k = kd(rng);
                const int64_t D = k * k + k + (int64_t)(rng() & 1);
                int64_t dx = isqrt_exact(D), dy2 = D - dx * dx;
                int64_t dy = isqrt_exact(dy2);
                if (dy * dy != dy2) { dx = 0; dy = isqrt_exact(D); }   // not a sum of these squares: keep near
                u.x = v.x + (int32_t)dx;
                u.y = v.y + (int32_t)dy;
            }
            if (u.x >= H) u.x -= 2 * 3001;
            if (u.y >= H) u.y -= 2 * 3001;
            if (u.x < -H) u.x += 2 * 3001;
            if (u.y < -H) u.y += 2 * 3001;
        }
        float xy2max = fmaxf(xy2_bound((float)v.x, (float)v.y), xy2_bound((float)u.x, (float)u.y));
        long long maxabs = std::max(std::llabs(v.lam), std::llabs(u.lam));
        // other columns of the instance raise the bounds
        if (rng() & 1) {
            xy2max = fmaxf(xy2max, xy2_bound((float)(-H), (float)(-H)));
            maxabs = std::max<long long>(maxabs, lam_mag);
        }
        const int64_t dx = (int64_t)v.x - u.x, dy = (int64_t)v.y - u.y;
        const int64_t Z = 2 * nint_exact(dx * dx + dy * dy) - v.lam - u.lam;
        for (int64_t slk : {int64_t(0), int64_t(2), int64_t(96)}) {
            // thresholds at Z - slk (tight), one above and one below; and a
            // random one; theta >= 0 always
            for (int64_t d : {int64_t(0), int64_t(1), int64_t(-1)}) {
                const int64_t th = Z - slk + d;
                if (th >= 0) check_pair(v, u, th, slk, xy2max, maxabs, pf, pb);
            }
            std::uniform_int_distribution<int64_t> thd(0, 1 << 20);
            check_pair(v, u, thd(rng), slk, xy2max, maxabs, pf, pb);
        }
    }
    std::printf("filter %lld %lld %lld\n", pf.checked, pf.tight, pf.bad);
    std::printf("box %lld %lld %lld\n", pb.checked, pb.tight, pb.bad);
    return 0;
}
