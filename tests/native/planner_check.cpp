// Host-side check of the product planner, built with address and undefined-behaviour
// sanitizers by tests/test_sanitizers.py.  Runs the optimiser, the integer counts, both step
// orders and the scheme checks for a spread of (P, kappa_min), and checks their basic
// invariants; any sanitizer report or failed invariant makes the program exit non-zero.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "planner.h"

int main()
{
    using namespace srj;
    const int64_t n2[3] = {4096, 4096, 1};
    const int64_t n3[3] = {512, 512, 512};
    const double cases[][2] = {{1, 1e-3}, {2, 1e-3}, {3, 2.5e-4}, {5, 1e-5}, {8, grid_kappa_min(3, n3)},
                               {10, grid_kappa_min(2, n2)}};
    int bad = 0;
    for (const auto& c : cases) {
        const int P = (int)c[0];
        const double km = c[1];
        Optimum o;
        std::string err;
        if (!optimal_schedule(P, km, 2.0, &o, &err)) {
            std::printf("P=%d km=%g: optimiser failed: %s\n", P, km, err.c_str());
            ++bad;
            continue;
        }
        double sb = 0;
        for (double b : o.beta) sb += b;
        if (std::fabs(sb - 1.0) > 1e-9) ++bad;
        std::vector<int64_t> q = floor_counts(o.beta);
        int64_t M = 0;
        for (int64_t x : q) M += x;
        for (int ord = 0; ord < 2; ++ord) {
            std::vector<int32_t> seq = order_steps(P, o.w.data(), q.data(), km, 2.0, ord);
            std::vector<int64_t> cnt(P, 0);
            for (int32_t i : seq) {
                if (i < 0 || i >= P) { ++bad; continue; }
                cnt[i]++;
            }
            for (int i = 0; i < P; ++i) bad += cnt[i] != q[i];
            double pre = 0, suf = 0;
            partial_peaks(P, o.w.data(), seq, km, 2.0, &pre, &suf);
            if (!std::isfinite(pre) || !std::isfinite(suf)) ++bad;
        }
        const double g = gamma_q_max(P, o.w.data(), q.data(), km, 2.0);
        if (!(g < 1.0)) ++bad;
        std::printf("P=%d km=%.6g M=%lld gamma_q=%.9f\n", P, km, (long long)M, g);
    }
    std::printf("%s\n", bad ? "FAILED" : "ok");
    return bad ? 1 : 0;
}
