// Host-only check of the graph replay plan the step loops follow: for every
// pair (graph_steps, diag_every) up to 40, the plan is refused exactly when
// the rounded graph length and diag_every do not divide one another; and for
// the accepted ones, random sequences of step calls up to t = 600 run the
// diagnostics at exactly the steps t with (t + 1) % diag_every == 0, start
// every graph replay at a multiple of its length, and run every step once.
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2009_12584_amd/csrc/lbm_plan.hpp"

using namespace mclbm;

int main() {
    std::mt19937 rng(7);
    long runs = 0;
    for (int gs = 0; gs <= 40; ++gs)
        for (int de = 0; de <= 40; ++de) {
            GraphPlan g;
            const bool ok = graph_plan(gs, de, g);
            const int glen = gs > 0 ? (gs + 1) / 2 * 2 : 0;
            const bool expect = gs <= 0 || de <= 0 || glen % de == 0 || de % glen == 0;
            if (ok != expect) {
                std::printf("graph_steps %d diag_every %d: accepted %d, expected %d\n", gs, de, ok, expect);
                return 1;
            }
            if (!ok) continue;
            for (int rep = 0; rep < 20; ++rep) {
                const int64_t T = 600;
                std::vector<int> diag(T, 0), ran(T, 0);
                int64_t t = 0;
                while (t < T) {
                    int64_t n = 1 + (int64_t)(rng() % 90);
                    if (t + n > T) n = T - t;
                    while (n > 0) {
                        const int v = next_launch(g, t, n);
                        if (v >= 0) {
                            if (t % g.glen != 0 || (t & 1)) {
                                std::printf("graph replay at t=%lld\n", (long long)t);
                                return 1;
                            }
                            for (int s = 0; s < g.glen; ++s) {
                                ran[t + s] += 1;
                                diag[t + s] += graph_diag(g, v, s);
                            }
                            t += g.glen;
                            n -= g.glen;
                        } else {
                            ran[t] += 1;
                            diag[t] += plain_diag(g.diag_every > 0 ? g.diag_every : de, t);
                            t += 1;
                            n -= 1;
                        }
                    }
                }
                for (int64_t k = 0; k < T; ++k) {
                    const int want = de > 0 && (k + 1) % de == 0;
                    if (ran[k] != 1 || diag[k] != want) {
                        std::printf("graph_steps %d diag_every %d: step %lld ran %d times, diagnostics %d (want %d)\n",
                                    gs, de, (long long)k, ran[k], diag[k], want);
                        return 1;
                    }
                }
                ++runs;
            }
        }
    std::printf("ok %ld runs\n", runs);
    return 0;
}
