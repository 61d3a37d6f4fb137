// plan_driver.cpp -- host-only driver of the library's planner for the CPU
// tests: built with g++ and the address / undefined-behaviour sanitizers, it
// reads one product per line on stdin,
//     m l n L algo cutoff policy leaf tcl
// builds its plan (contiguous operands), runs the planner's own bounds
// validation, and prints
//     depth n_mul n_addsub ws_words n_launches n_leaf_tasks valid
// A line "batch k" followed by k product lines plans them as one batch and
// prints the same fields for the batch plan.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "plan.hpp"

using namespace mpg;

static void report(const Plan& P)
{
    const char* why = nullptr;
    const bool ok = validate_plan(P, &why);
    std::printf("%d %.0f %.0f %lld %zu %zu %d\n", P.depth, P.n_mul, P.n_addsub, (long long)P.ws_words,
                P.steps.size(), P.gemm.size(), ok ? 1 : 0);
    if (!ok) std::fprintf(stderr, "invalid plan: %s\n", why ? why : "?");
}

int main()
{
    char word[16];
    while (std::scanf("%15s", word) == 1) {
        if (word[0] == 'b') {                           // batch k
            int k = 0, L = 8, algo = 3, cutoff = 1, policy = 0, leaf = 0;
            if (std::scanf("%d", &k) != 1 || k < 1) return 2;
            std::vector<BatchItem> items;
            for (int r = 0; r < k; r++) {
                long long m, l, n;
                int tcl;
                if (std::scanf("%lld %lld %lld %d %d %d %d %d %d", &m, &l, &n, &L, &algo, &cutoff, &policy, &leaf,
                               &tcl) != 9)
                    return 2;
                items.push_back(BatchItem{m, l, n, l, m * l, n, l * n, n, m * n});
            }
            PlanKey key{0, 0, 0, L, algo, cutoff, policy, leaf, 0, 0, 0, 0, 0, 0};
            Plan P;
            build_plan_batched(P, key, items);
            report(P);
            continue;
        }
        long long m = std::atoll(word), l, n;
        int L, algo, cutoff, policy, leaf, tcl;
        if (std::scanf("%lld %lld %d %d %d %d %d %d", &l, &n, &L, &algo, &cutoff, &policy, &leaf, &tcl) != 8) return 2;
        PlanKey key{m, l, n, L, algo, cutoff, policy, leaf, l, m * l, n, l * n, n, m * n};
        key.tcl = tcl;
        Plan P;
        build_plan(P, key);
        report(P);
    }
    return 0;
}
