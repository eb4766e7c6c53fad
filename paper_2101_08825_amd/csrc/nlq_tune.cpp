// Autotuner of the integration launch: register-budget variant, persistent
// workgroups per CU and pair-list part per work item, timed on a sample of the
// system's own outer elements and kept per (dim, precision, kernel, L_max,
// pair-list size class) in the context.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "nlq_internal.hpp"

namespace nlq {

TuneKey tune_key(const System &s)
{
    int lg = 0;
    while ((int64_t(1) << lg) < std::max<int64_t>(s.max_pairs, 1)) ++lg;
    // element type: 1 P1, 2 P2, 3 Q1, 4 serendipity
    return TuneKey(s.mesh->dim, s.mesh->order + 2 * s.mesh->shape, s.p.precision, s.p.kernel, s.p.lmax, lg);
}

namespace {

// the untuned configuration: 3D pair lists are cut into parts of 256 pairs (the
// autotuner's choice on every 3D case measured; finer work items balance the
// longer per-pair work of tetrahedra), 2D ones into parts of 512
TuneConfig default_config(const System &s)
{
    TuneConfig c{};
    if (s.mesh->dim == 3) c.pairs_per_item = 256;
    return c;
}

}  // namespace

TuneConfig tuned_config(Ctx &ctx, const System &s)
{
    std::lock_guard<std::mutex> g(ctx.tune_mu);
    auto it = ctx.tuned.find(tune_key(s));
    return it != ctx.tuned.end() ? it->second : default_config(s);
}

namespace {

// milliseconds of one launch over outer elements [lo, hi) with configuration c
double time_range(System &s, const TuneConfig &c, int64_t lo, int64_t hi, hipStream_t st, LaunchBlock &lb,
                  hipEvent_t e0, hipEvent_t e1)
{
    s.cfg = c;
    launch_integrate_jobs(s.ctx, lb, {IntegrateJob{&s, lo, hi}}, st, e0, e1);
    NLQ_HIP(hipStreamSynchronize(st));
    float ms = 0.0f;
    NLQ_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms;
}

}  // namespace

int autotune(System &s, hipStream_t st, double budget_s, double *best_ms, double *default_ms)
{
    Ctx &ctx = *s.ctx;
    const int64_t ne = s.mesh->n_elems;
    const TuneConfig base = default_config(s);
    *best_ms = *default_ms = 0.0;
    if (s.p.deterministic) return 0;   // sample ranges are not integrated on their own in this mode
    // stage 1 candidates: the default first, then the register variant (P1
    // simplices only: the other element types have one), one workgroup less per
    // CU, and other work-item sizes where the pair lists get cut
    std::vector<TuneConfig> cand{base};
    for (int occ = 0; occ < (s.mesh->order == 1 && s.mesh->shape == 0 ? 2 : 1); ++occ)
        for (int less = 0; less < 2; ++less)
            for (int ppi : {512, 256, 1024}) {
                if (ppi != 512 && s.max_pairs <= 256) continue;
                TuneConfig c;
                c.occ = occ;
                c.pairs_per_item = ppi;
                if (less) {
                    s.cfg = c;
                    const int64_t per_cu = integrate_slots(&ctx, s) / std::max(ctx.n_cu, 1);
                    if (per_cu < 2) continue;
                    c.wg_per_cu = static_cast<int>(per_cu - 1);
                }
                if (occ == 0 && !less && ppi == base.pairs_per_item) continue;   // the default
                cand.push_back(c);
            }
    // a sample in the middle of the mesh (away from the first and last element,
    // whose ranges would clear or finish the values) with about four work items
    // per resident workgroup
    s.cfg = base;
    const int64_t slots = integrate_slots(&ctx, s);
    const int64_t per_elem = std::max(1, integrate_split(s));
    int64_t len = std::max<int64_t>(1, 4 * slots / per_elem);
    len = std::min(len, ne / 2);
    const int64_t lo = ne / 4, hi = lo + len;
    *best_ms = *default_ms = 0.0;
    if (len < 1 || lo < 1 || hi >= ne) {
        s.cfg = base;
        return 0;
    }
    LaunchBlock lb;
    hipEvent_t e0, e1;
    NLQ_HIP(hipEventCreate(&e0));
    NLQ_HIP(hipEventCreate(&e1));
    const double t_start = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
    TuneConfig best = base;
    double best_t = 1e300;
    int timed = 0;
    bool out_of_time = false;
    // times c and keeps it if it beats the fastest so far by the factor `margin`;
    // its time (huge once the budget is spent and nothing more is timed)
    auto try_config = [&](const TuneConfig &c, double margin) {
        if (out_of_time) return 1e300;
        (void)time_range(s, c, lo, hi, st, lb, e0, e1);   // warm (code object, caches)
        const double t = std::min(time_range(s, c, lo, hi, st, lb, e0, e1), time_range(s, c, lo, hi, st, lb, e0, e1));
        ++timed;
        if (timed == 1) *default_ms = t;
        if (t < best_t * margin) {
            best_t = t;
            best = c;
        }
        const double now = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
        if (now - t_start > budget_s) out_of_time = true;
        return t;
    };
    for (const TuneConfig &c : cand) try_config(c, 1.0);
    // stage 2, from the best launch shape: the traversal stack's logical capacity
    // (how many sub-elements one pass may pop and expand) and the leaf buffer's
    // (how many leaves are integrated per flush), one at a time, then together if
    // both helped.  A capacity is kept only when it beats the shape by more than
    // 2%: on the 24^3 x 6 problem the sample launches ranked capacities by a few
    // percent that the whole launch did not show (0.5% slower with stack 256 or
    // 512 than with the untuned 128).
    const TuneConfig shape = best;
    TuneConfig best_stack = shape, best_leaf = shape;
    double t_stack = best_t, t_leaf = best_t;
    for (int sc : {64, 256, 512}) {
        TuneConfig c = shape;
        c.stack_cap = sc;
        const double t = try_config(c, 0.98);
        if (t < t_stack * 0.98) {
            t_stack = t;
            best_stack = c;
        }
    }
    for (int lc : {64, 256}) {
        TuneConfig c = shape;
        c.leaf_cap = lc;
        const double t = try_config(c, 0.98);
        if (t < t_leaf * 0.98) {
            t_leaf = t;
            best_leaf = c;
        }
    }
    if (best_stack.stack_cap != shape.stack_cap && best_leaf.leaf_cap != shape.leaf_cap) {
        TuneConfig c = shape;
        c.stack_cap = best_stack.stack_cap;
        c.leaf_cap = best_leaf.leaf_cap;
        try_config(c, 0.98);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *best_ms = best_t;
    s.cfg = best;
    {
        std::lock_guard<std::mutex> g(ctx.tune_mu);
        ctx.tuned[tune_key(s)] = best;
    }
    // the sample launches added partial sums: recompute an integrated system
    // whole; a prepared one (never integrated) gets its zero values back
    if (s.integrated) {
        run_integrate(s, st);
    } else {
        NLQ_HIP(hipMemsetAsync(s.val.as<void>(), 0, sizeof(double) * std::max<int64_t>(s.nnz, 1), st));
        NLQ_HIP(hipStreamSynchronize(st));
    }
    return timed;
}

}  // namespace nlq
