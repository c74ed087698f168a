// Replay plan of captured step graphs, shared by the single and batched
// forms; host logic free of HIP types (a host-only test compiles it with a
// plain C++ compiler).
//
// A graph of glen steps (graph_steps rounded up to even, so the buffer read
// at its start is always buffer 0) replays only from a time that is a
// multiple of glen; other steps are plain launches.  The fused diagnostics
// then run at exactly the steps t with (t + 1) % diag_every == 0, graph or
// not: either diag_every divides glen (one graph, diagnostics at those of its
// steps) or glen divides diag_every (a graph without diagnostics and one with
// them at its last step, chosen per replay).  Other pairs are refused.
#pragma once

#include <cstdint>

namespace mclbm {

struct GraphPlan {
    int glen = 0;  // 0: no graphs
    int diag_every = 0;
    bool two = false;
};

// Fills g; returns false when graph_steps and diag_every do not divide one
// another (after rounding graph_steps up to even).
inline bool graph_plan(int graph_steps, int diag_every, GraphPlan &g) {
    g = GraphPlan{};
    if (graph_steps <= 0) return true;
    g.glen = (graph_steps + 1) / 2 * 2;
    g.diag_every = diag_every > 0 ? diag_every : 0;
    if (g.diag_every > 0 && g.glen % g.diag_every != 0) {
        if (g.diag_every % g.glen != 0) return false;
        g.two = true;
    }
    return true;
}
inline int graph_variants(const GraphPlan &g) { return g.glen ? (g.two ? 2 : 1) : 0; }
// does step s (0-based) of graph variant v run the diagnostics?
inline bool graph_diag(const GraphPlan &g, int v, int s) {
    if (g.diag_every <= 0) return false;
    if (!g.two) return (s + 1) % g.diag_every == 0;
    return v == 1 && s == g.glen - 1;
}
// the variant that replays from time t (a multiple of glen)
inline int graph_variant(const GraphPlan &g, int64_t t) {
    return g.two && (t + g.glen) % g.diag_every == 0 ? 1 : 0;
}
// plain launch at time t: does it run the diagnostics?
inline bool plain_diag(int diag_every, int64_t t) { return diag_every > 0 && (t + 1) % diag_every == 0; }
// What a step loop launches at time t with n steps left: a graph variant
// (>= 0, glen steps) or -1 for one plain step.
inline int next_launch(const GraphPlan &g, int64_t t, int64_t n) {
    return g.glen > 0 && t % g.glen == 0 && n >= g.glen ? graph_variant(g, t) : -1;
}

}  // namespace mclbm
