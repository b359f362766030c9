// Host run of the exact finish (f2m_finish.cpp) through the CPU harness,
// built with AddressSanitizer and UndefinedBehaviorSanitizer: random,
// tie-heavy and lattice instances, cold and perturbed starts, b-matching
// degrees, pairs as a list or as keys, and every workspace mode of the harness (fresh, reused, four
// threads with the chunked tail, one thread).  Exit status 0 when every call
// returns a solution; the sanitizers abort on the first error they find.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" int64_t finish_cpu(int64_t n, const int32_t *xy, const int64_t *lam0, int64_t *lam_out, int64_t cap,
                              int32_t *eu, int32_t *ev, uint8_t *ex2, int64_t *stats, int32_t bulk, int32_t reuse,
                              const int32_t *b);

int main()
{
    std::mt19937_64 rng(20111708);
    int failures = 0, calls = 0;
    for (int n : {5, 9, 40, 300, 1500}) {
        for (int mode = 0; mode < 4; ++mode) {
            std::vector<int32_t> xy(2 * n);
            const int span = mode == 1 ? 40 : 100000;   // mode 1: many equal lengths
            for (int v = 0; v < n; ++v) {
                if (mode == 3) {                          // a lattice: ties everywhere
                    const int side = 1 + (int)std::sqrt((double)n);
                    xy[2 * v] = 10 * (v % side);
                    xy[2 * v + 1] = 10 * (v / side);
                } else {
                    xy[2 * v] = (int32_t)(rng() % span);
                    xy[2 * v + 1] = (int32_t)(rng() % span);
                }
            }
            std::vector<int64_t> lam0(n, 0), lam(n);
            if (mode == 2)
                for (int v = 0; v < n; ++v) lam0[v] = (int64_t)(rng() % 2000) - 500;
            std::vector<int32_t> b;
            if (mode == 2 && n >= 9) {
                b.resize(n);
                for (int v = 0; v < n; ++v) b[v] = 1 + (int32_t)(rng() % 3);
            }
            const int64_t cap = 6 * (int64_t)n;
            std::vector<int32_t> eu(cap), ev(cap);
            std::vector<uint8_t> ex(cap);
            int64_t st[4];
            for (int reuse = 0; reuse < 4; ++reuse) {
                for (int bulk = 0; bulk < 3; ++bulk) {
                    const int64_t m = finish_cpu(n, xy.data(), lam0.data(), lam.data(), cap, eu.data(), ev.data(),
                                                 ex.data(), st, bulk, reuse, b.empty() ? nullptr : b.data());
                    ++calls;
                    if (m < 0) {
                        ++failures;
                        std::fprintf(stderr, "finish failed: n=%d mode=%d reuse=%d bulk=%d\n", n, mode, reuse, bulk);
                    }
                }
            }
        }
    }
    std::printf("finish calls %d failures %d\n", calls, failures);
    return failures ? 1 : 0;
}
