// Serving loop: continuous batching of assemble + solve requests on one GPU.
//
//   submit -> pending --(admission by HBM footprint)--> setup (mesh from the
//   resident cache, element tables, pair list, pattern) -> ready -> shared
//   integration launches (several requests per launch, chunked by outer-element
//   ranges) -> solve (load vector, lifting, CG, copy of u) -> done.
//
// One device thread owns the GPU and time-slices it: every pass first finishes
// the requests whose integration is complete (their CG), then sets up newly
// admitted requests (for at most about two launch targets), then runs one
// shared integration launch of about the target duration.  Kernels are never
// issued from several streams at once: the persistent integration launch holds
// every CU's registers, so a small kernel on another stream could only start
// between two launches, which would stretch a CG of hundreds of kernels over
// hundreds of launches.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <list>
#include <tuple>
#include <unordered_map>

#include "nlq_internal.hpp"

namespace nlq {

namespace {

double serve_now()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

using MeshKey = std::tuple<int, int, int>;
// mesh key + every parameter that changes the matrix
using SysKey = std::tuple<int, int, int, int, double, double, double, int, int, int, int, int, int>;

SysKey sys_key(const nlq_request &r)
{
    const nlq_params &p = r.params;
    return SysKey(r.dim, r.n, r.k_gamma, p.kernel, p.delta, p.eps, p.scale, p.lmin, p.lmax, p.form, p.precision,
                  p.deterministic, p.min_dist_l2);
}

// Integration group: one launch takes systems of one (dim, precision, kernel);
// the rate model is kept per (group, lmax).
using GroupKey = std::tuple<int, int, int>;
using RateKey = std::tuple<int, int, int, int>;

// Upper estimate of the device memory of one box request (pair list, pattern,
// CSR values, element and diagonal-block tables, vectors, setup temporaries).
uint64_t estimate_bytes(const nlq_request &r)
{
    const int dim = r.dim;
    const double n = r.n;
    const double reach = (r.params.delta + r.params.eps) * r.n;   // in cells
    const double K = std::floor(reach) + 1.0;
    const double types = dim == 2 ? 2.0 : 6.0;
    const double ne = types * std::pow(n, dim), nn = std::pow(n + 1.0, dim);
    const double pairs = ne * types * std::pow(std::min(n, 2.0 * K + 1.0), dim);
    const double nnz = nn * std::pow(std::min(n + 1.0, 2.0 * K + 3.0), dim);
    const int nv = dim + 1, nr = nv * (nv + 1) / 2;
    const double b = 4.0 * pairs * 2.0 + 8.0 * (ne + 1.0) * 3.0 + nnz * (4.0 + 4.0 + 8.0) + 8.0 * (nn + 1.0) +
                     ne * nv * nv * 4.0 + ne * nr * 8.0 + ne * (nv * dim + 2.0 * dim + 1.0) * 8.0 + 12.0 * 8.0 * nn;
    return static_cast<uint64_t>(1.2 * b) + (uint64_t(1) << 20);
}

struct CacheEntry {
    SysKey key;
    std::unique_ptr<nlq_system> sys;
    bool busy = false;
};

struct Request {
    uint64_t ticket = 0;
    nlq_request req{};
    std::vector<double> f, g;
    double t_submit = 0.0, t_admit = 0.0, t_setup = 0.0, t_ready = 0.0, t_done = 0.0;
    double t_turn = 0.0;              // waiting for a launch since (set up, or its last launch)
    nlq_status status = NLQ_ENOTREADY;
    std::atomic<bool> cancelled{false};
    bool done = false;
    std::vector<double> u;
    int64_t n_nodes = 0, n_pairs = 0, n_free = 0;
    int cg_iterations = 0;
    double rel_residual = 0.0;
    std::string error;
    uint64_t est = 0;                 // admission estimate, held until setup ends
    // in flight
    nlq_mesh *mesh = nullptr;
    std::unique_ptr<nlq_system> own;  // system assembled for this request
    CacheEntry *cached = nullptr;     // or a resident one it borrows
    int64_t cursor = 0;               // next outer element to integrate
    std::vector<int64_t> pair_off;    // host copy, for chunking by pairs
    int launches = 0;
    int split = 1;                    // work items per outer element
    int64_t slots = 1;                // resident workgroups of its launches
    bool cache_hit = false;
    System &sys() { return cached ? cached->sys->impl : own->impl; }
};

using ReqPtr = std::shared_ptr<Request>;

}  // namespace

struct Server {
    Ctx *ctx = nullptr;
    nlq_serve_config cfg{};
    std::mutex mu;
    std::condition_variable cv_dev, cv_done;
    std::deque<ReqPtr> pending;          // submitted, not admitted
    std::deque<ReqPtr> setup_q;          // admitted, waiting for setup
    std::deque<ReqPtr> solve_q;          // matrix ready, waiting for CG
    std::vector<ReqPtr> ready;           // set up, integrating (admission order)
    std::unordered_map<uint64_t, ReqPtr> all;
    int admitted = 0;                   // admitted, not done
    uint64_t reserved = 0;              // estimates of admitted requests not yet set up
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread dev;                    // the device thread
    hipStream_t stream = nullptr;
    std::mutex mesh_mu;
    std::map<MeshKey, std::unique_ptr<nlq_mesh>> meshes;
    std::list<CacheEntry> cache;        // most recently used at the front (under mu)
    // systems to free: moved here under mu, destroyed outside it (hipFree may
    // wait for the device, which must not happen while mu is held)
    std::vector<std::unique_ptr<nlq_system>> graveyard;
    std::map<RateKey, double> rate;     // integrated pairs per second
    nlq_serve_stats stats{};
};

namespace {

// ---- helpers under S.mu -----------------------------------------------------

void finish_locked(Server &S, const ReqPtr &r, nlq_status st, const std::string &err)
{
    r->status = st;
    r->error = err;
    r->done = true;
    r->t_done = serve_now();
    if (st == NLQ_OK) ++S.stats.completed;
    else if (st == NLQ_ECANCELLED) ++S.stats.cancelled;
    else ++S.stats.failed;
    S.cv_done.notify_all();
}

// drop resident matrices (LRU, not in use) until `need` more bytes fit
void evict_locked(Server &S, uint64_t need)
{
    while (S.ctx->used.load() + S.reserved + need > S.ctx->budget) {
        auto it = S.cache.end();
        for (auto q = S.cache.begin(); q != S.cache.end(); ++q)
            if (!q->busy) it = q;   // last = least recently used
        if (it == S.cache.end()) return;
        S.graveyard.push_back(std::move(it->sys));
        S.cache.erase(it);
    }
}

void admit_locked(Server &S)
{
    while (!S.pending.empty() && S.admitted < S.cfg.max_active) {
        ReqPtr r = S.pending.front();
        if (r->cancelled) {
            S.pending.pop_front();
            finish_locked(S, r, NLQ_ECANCELLED, "cancelled");
            continue;
        }
        r->est = estimate_bytes(r->req);
        evict_locked(S, r->est);
        const bool fits = S.ctx->used.load() + S.reserved + r->est <= S.ctx->budget;
        if (!fits && S.admitted > 0) return;   // wait for memory (FIFO)
        S.pending.pop_front();
        S.reserved += r->est;
        ++S.admitted;
        S.stats.max_admitted = std::max(S.stats.max_admitted, S.admitted);
        r->t_admit = serve_now();
        S.setup_q.push_back(r);
        S.cv_dev.notify_all();
    }
}

// release what an ended request holds (under S.mu)
void release_locked(Server &S, const ReqPtr &r, bool keep)
{
    if (r->est) {
        S.reserved -= r->est;
        r->est = 0;
    }
    if (r->cached) {
        r->cached->busy = false;
        r->cached = nullptr;
    } else if (r->own) {
        const SysKey k = sys_key(r->req);
        bool have = false;
        for (auto &c : S.cache) have = have || (c.key == k);
        if (keep && S.cfg.cache_systems && !have) S.cache.push_front(CacheEntry{k, std::move(r->own), false});
        else S.graveyard.push_back(std::move(r->own));
    }
    --S.admitted;
    admit_locked(S);
    S.cv_dev.notify_all();
}

// free buried systems outside the lock, then admit what now fits
void drain(Server &S)
{
    std::vector<std::unique_ptr<nlq_system>> dead;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        dead.swap(S.graveyard);
    }
    if (dead.empty()) return;
    dead.clear();
    std::lock_guard<std::mutex> lk(S.mu);
    admit_locked(S);
}

nlq_mesh *get_mesh(Server &S, const nlq_request &q, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(S.mesh_mu);
    const MeshKey k(q.dim, q.n, q.k_gamma);
    auto it = S.meshes.find(k);
    if (it != S.meshes.end()) return it->second.get();
    auto m = make_box_mesh(*S.ctx, q.dim, q.n, q.k_gamma, st);
    nlq_mesh *raw = m.get();
    S.meshes[k] = std::move(m);
    return raw;
}

// ---- worker: setup and solve ---------------------------------------------

void do_setup(Server &S, const ReqPtr &r, hipStream_t st)
{
    if (r->cancelled) throw Error{NLQ_ECANCELLED, "cancelled"};
    r->mesh = get_mesh(S, r->req, st);
    const Mesh &M = r->mesh->impl;
    r->n_nodes = M.n_nodes;
    r->n_free = M.n_free;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        if (S.cfg.cache_systems) {
            const SysKey k = sys_key(r->req);
            for (auto it = S.cache.begin(); it != S.cache.end(); ++it) {
                if (it->key == k && !it->busy) {
                    it->busy = true;
                    S.cache.splice(S.cache.begin(), S.cache, it);
                    r->cached = &S.cache.front();
                    r->cache_hit = true;
                    ++S.stats.cache_hits;
                    break;
                }
            }
        }
    }
    if (r->cached) {
        r->n_pairs = r->cached->sys->impl.n_pairs;
        std::lock_guard<std::mutex> lk(S.mu);
        S.reserved -= r->est;
        r->est = 0;
        r->t_ready = r->t_setup = serve_now();
        S.solve_q.push_back(r);
        return;
    }
    r->own = prepare_system(*S.ctx, M, r->req.params, st);
    System &s = r->own->impl;
    // a deterministic request is integrated by itself, here
    const bool det = r->req.params.deterministic != 0;
    if (det && M.n_elems > 0) run_integrate(s, st);
    r->n_pairs = s.n_pairs;
    r->split = integrate_split(s);
    r->slots = integrate_slots(S.ctx, s);
    r->pair_off.resize(M.n_elems + 1);
    NLQ_HIP(hipMemcpyAsync(r->pair_off.data(), s.pair_off.as<void>(), sizeof(int64_t) * (M.n_elems + 1),
                           hipMemcpyDeviceToHost, st));
    NLQ_HIP(hipStreamSynchronize(st));
    std::lock_guard<std::mutex> lk(S.mu);
    S.reserved -= r->est;
    r->est = 0;
    if (r->cancelled) throw Error{NLQ_ECANCELLED, "cancelled"};
    r->t_setup = r->t_turn = serve_now();
    if (M.n_elems == 0 || det) {
        r->t_ready = r->t_setup;
        r->launches = det && M.n_elems > 0 ? 1 : 0;
        S.solve_q.push_back(r);
        return;
    }
    S.ready.push_back(r);
}

void do_solve(Server &S, const ReqPtr &r, hipStream_t st)
{
    if (r->cancelled) throw Error{NLQ_ECANCELLED, "cancelled"};
    System &s = r->sys();
    load_data(s, r->f.data(), r->g.data(), st);
    r->u.assign(s.mesh->n_nodes, 0.0);
    nlq_solve_info info{};
    const double rtol = r->req.rtol > 0 ? r->req.rtol : 1e-10;
    const int maxit = r->req.maxit > 0 ? r->req.maxit : 10000;
    const bool conv = solve_system(s, rtol, maxit, r->u.data(), &info, st);
    r->cg_iterations = info.iterations;
    r->rel_residual = info.rel_residual;
    if (!conv) throw Error{NLQ_ENOCONV, "CG did not reach the tolerance"};
}

// ---- scheduler: shared integration launches -------------------------------

GroupKey group_of(const Request &r)
{
    return GroupKey(r.req.dim, r.req.params.precision, r.req.params.kernel);
}

RateKey rate_key(const Request &r)
{
    return RateKey(r.req.dim, r.req.params.precision, r.req.params.kernel, r.req.params.lmax);
}

double initial_rate(const Request &r)
{
    // pairs/s of a first launch before any measurement (deliberately low)
    const double base = r.req.dim == 2 ? 2e8 : 2e7;
    return base / std::pow(r.req.dim == 2 ? 4.0 : 8.0, std::max(0, r.req.params.lmax - 3));
}

struct Chunk {
    ReqPtr r;
    int64_t lo, hi, pairs, items;
};

// Scheduling score (lower goes first): the estimated integration time left
// (remaining pairs / the group's measured rate) minus a quarter of the time the
// request has waited for a launch -- shortest remaining work first, so small
// requests pass large ones, with aging: a request waits at most about four
// times its own remaining time before it outranks new arrivals.
double urgency(const Server &S, const Request &r, double now)
{
    auto it = S.rate.find(rate_key(r));
    const double rate = it != S.rate.end() ? it->second : initial_rate(r);
    const double left = static_cast<double>(r.pair_off.back() - r.pair_off[r.cursor]) / rate;
    return left - 0.25 * (now - r.t_turn);
}

// Greedy filling of a pair budget, most urgent request first: each takes all it
// has left while the budget lasts, so the smallest requests finish in this
// launch and the rest of the budget goes to the next ones; requests the budget
// does not reach are left out.  Returns outer-element ranges (at least one
// element each).
std::vector<Chunk> greedy_fill(const std::vector<ReqPtr> &rs, double budget)
{
    std::vector<Chunk> out;
    double rest = budget;
    for (const ReqPtr &rp : rs) {
        if (rest < 0.5) break;
        Request &r = *rp;
        const int64_t ne = static_cast<int64_t>(r.pair_off.size()) - 1;
        const int64_t base = r.pair_off[r.cursor];
        const double share = std::min(static_cast<double>(r.pair_off.back() - base), rest);
        rest -= share;
        const int64_t target = base + static_cast<int64_t>(std::ceil(share));
        // first hi with pair_off[hi] >= target, at least cursor + 1
        int64_t hi = std::lower_bound(r.pair_off.begin() + r.cursor + 1, r.pair_off.end(), target) -
                     r.pair_off.begin();
        hi = std::min(std::max(hi, r.cursor + 1), ne);
        out.push_back(Chunk{rp, r.cursor, hi, r.pair_off[hi] - base, (hi - r.cursor) * r.split});
    }
    return out;
}

// The launch of one group: a pair budget from the measured rate and the target
// duration -- or, when finish_pairs > 0, only the most urgent request's remaining
// pairs -- raised until the launch holds at least two work items per resident
// workgroup (or everything that is left), so that the persistent grid is busy.
std::vector<Chunk> plan_launch(Server &S, const GroupKey &g, int64_t finish_pairs, double now)
{
    // up to 32 requests of the group, most urgent first
    std::vector<ReqPtr> rs;
    for (auto &r : S.ready)
        if (group_of(*r) == g) rs.push_back(r);
    std::stable_sort(rs.begin(), rs.end(),
                     [&](const ReqPtr &a, const ReqPtr &b) { return urgency(S, *a, now) < urgency(S, *b, now); });
    if (rs.size() > 32) rs.resize(32);
    double budget = 0.0;
    int64_t slots = 1, left_items = 0;
    for (auto &r : rs) {
        auto it = S.rate.find(rate_key(*r));
        const double rate = it != S.rate.end() ? it->second : initial_rate(*r);
        budget = std::max(budget, rate * S.cfg.target_launch_ms * 1e-3);
        slots = std::max(slots, r->slots);
        left_items += (static_cast<int64_t>(r->pair_off.size()) - 1 - r->cursor) * r->split;
    }
    if (finish_pairs > 0)
        budget = std::min(budget, static_cast<double>(finish_pairs) + 1.0);
    const int64_t want = std::min<int64_t>(2 * slots, left_items);
    std::vector<Chunk> plan;
    for (int round = 0; round < 40; ++round) {
        plan = greedy_fill(rs, budget);
        int64_t items = 0;
        for (auto &c : plan) items += c.items;
        if (items >= want) break;
        budget *= std::max(1.5, 1.2 * static_cast<double>(want) / std::max<int64_t>(items, 1));
    }
    return plan;
}

// one shared integration launch for the ready requests of the next group
void run_launch(Server *S, LaunchBlock &lb, hipEvent_t e0, hipEvent_t e1)
{
    std::vector<Chunk> plan;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        // drop cancelled requests before they take launch time
        for (size_t i = 0; i < S->ready.size();) {
            if (S->ready[i]->cancelled) {
                ReqPtr r = S->ready[i];
                S->ready.erase(S->ready.begin() + i);
                finish_locked(*S, r, NLQ_ECANCELLED, "cancelled");
                release_locked(*S, r, false);
            } else {
                ++i;
            }
        }
        if (S->ready.empty()) return;
        // the group of the most urgent request, in a launch just long enough
        // for that request to finish (at most the target duration), so that a
        // small request goes through at once
        const double now = serve_now();
        const Request *pick = S->ready.front().get();
        double best = urgency(*S, *pick, now);
        for (auto &r : S->ready) {
            const double u = urgency(*S, *r, now);
            if (u < best) {
                best = u;
                pick = r.get();
            }
        }
        plan = plan_launch(*S, group_of(*pick), pick->pair_off.back() - pick->pair_off[pick->cursor], now);
    }
    std::vector<IntegrateJob> jobs;
    for (auto &c : plan) jobs.push_back(IntegrateJob{&c.r->sys(), c.lo, c.hi});
    nlq_status code = NLQ_OK;
    std::string err;
    float ms = 0.0f;
    try {
        launch_integrate_jobs(S->ctx, lb, jobs, S->stream, e0, e1);
        NLQ_HIP(hipStreamSynchronize(S->stream));
        NLQ_HIP(hipEventElapsedTime(&ms, e0, e1));
        for (auto &c : plan)
            if (c.hi == static_cast<int64_t>(c.r->pair_off.size()) - 1) collect_counters(c.r->sys(), S->stream);
    } catch (const Error &e) {
        code = e.status;
        err = e.msg;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    ++S->stats.launches;
    S->stats.launch_segments += static_cast<int64_t>(plan.size());
    S->stats.max_per_launch = std::max(S->stats.max_per_launch, static_cast<int32_t>(plan.size()));
    S->stats.launch_s += 1e-3 * ms;
    S->stats.peak_bytes = std::max<uint64_t>(S->stats.peak_bytes, S->ctx->used.load());
    int64_t pairs = 0, items = 0, slots = 1;
    for (auto &c : plan) {
        pairs += c.pairs;
        items += c.items;
        slots = std::max(slots, c.r->slots);
    }
    if (code == NLQ_OK && ms > 0.5f && !plan.empty() && items >= slots) {
        // rate model: measured pairs per second of this launch, smoothed
        const RateKey k = rate_key(*plan[0].r);
        const double meas = pairs / (1e-3 * ms);
        auto it = S->rate.find(k);
        S->rate[k] = it == S->rate.end() ? meas : 0.5 * it->second + 0.5 * meas;
    }
    for (auto &c : plan) {
        Request &r = *c.r;
        r.launches += 1;
        auto pos = std::find(S->ready.begin(), S->ready.end(), c.r);
        if (code != NLQ_OK) {
            if (pos != S->ready.end()) S->ready.erase(pos);
            finish_locked(*S, c.r, code, err);
            release_locked(*S, c.r, false);
            continue;
        }
        r.cursor = c.hi;
        r.t_turn = serve_now();
        if (r.cursor == static_cast<int64_t>(r.pair_off.size()) - 1) {
            if (pos != S->ready.end()) S->ready.erase(pos);
            r.t_ready = serve_now();
            S->solve_q.push_back(c.r);
        }
    }
}

// setup or solve of one request on the device thread; failures end the request
void run_phase(Server *S, const ReqPtr &r, bool solve)
{
    nlq_status code = NLQ_OK;
    std::string err;
    try {
        if (solve) do_solve(*S, r, S->stream);
        else do_setup(*S, r, S->stream);
    } catch (const Error &e) {
        code = e.status;
        err = e.msg;
    } catch (const std::exception &e) {
        code = NLQ_EDEVICE;
        err = e.what();
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (code != NLQ_OK) {
        // a failed CG still leaves a valid matrix; other failures drop it
        finish_locked(*S, r, code, err);
        release_locked(*S, r, code == NLQ_ENOCONV);
    } else if (solve) {
        finish_locked(*S, r, NLQ_OK, "");
        release_locked(*S, r, true);
    }
}

// The device thread: each pass finishes every request whose matrix is ready
// (CG), sets up admitted requests, then runs one shared integration launch.
void device_main(Server *S)
{
    (void)hipSetDevice(S->ctx->device);
    LaunchBlock lb;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_dev.wait(lk, [&] {
                return !S->solve_q.empty() || !S->setup_q.empty() || !S->ready.empty() ||
                       (S->stop && S->admitted == 0 && S->pending.empty());
            });
            if (S->solve_q.empty() && S->setup_q.empty() && S->ready.empty()) break;
        }
        for (;;) {
            ReqPtr r;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                if (S->solve_q.empty()) break;
                r = S->solve_q.front();
                S->solve_q.pop_front();
            }
            run_phase(S, r, true);
            drain(*S);
        }
        // set up admitted requests (for up to one launch target, at least one),
        // so that the next launch shares as many as possible: the smallest
        // first (by the admission estimate), unless the longest-waiting one has
        // waited for more than a second
        const double t_pass = serve_now();
        const double setup_budget = std::max(1e-3 * S->cfg.target_launch_ms, 0.005);
        for (;;) {
            ReqPtr r;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                if (S->setup_q.empty()) break;
                auto at = S->setup_q.begin();
                if (serve_now() - (*at)->t_admit <= 1.0)
                    for (auto it = S->setup_q.begin(); it != S->setup_q.end(); ++it)
                        if ((*it)->est < (*at)->est) at = it;
                r = *at;
                S->setup_q.erase(at);
            }
            run_phase(S, r, false);
            drain(*S);
            if (serve_now() - t_pass > setup_budget) break;
        }
        run_launch(S, lb, e0, e1);
        drain(*S);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

}  // namespace

}  // namespace nlq

using namespace nlq;

nlq::Ctx::Ctx() = default;
nlq::Ctx::~Ctx() = default;

extern "C" {

nlq_status nlq_serve_start(nlq_ctx *ctx, const nlq_serve_config *cfg)
{
    if (!ctx) {
        set_last_error("ctx is NULL");
        return NLQ_EINVAL;
    }
    if (ctx->impl.server) {
        set_last_error("server already running");
        return NLQ_EBUSY;
    }
    auto S = std::make_unique<Server>();
    S->ctx = &ctx->impl;
    nlq_serve_config c{};
    if (cfg) c = *cfg;
    if (c.max_active <= 0) c.max_active = 256;
    if (!(c.target_launch_ms > 0.0)) c.target_launch_ms = 25.0;
    c.cache_systems = c.cache_systems ? 1 : 0;
    S->cfg = c;
    if (hipSetDevice(ctx->impl.device) != hipSuccess) {
        set_last_error("hipSetDevice failed");
        return NLQ_EDEVICE;
    }
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
        set_last_error("hipStreamCreate failed");
        return NLQ_EDEVICE;
    }
    Server *raw = S.get();
    ctx->impl.server = std::move(S);
    raw->dev = std::thread(device_main, raw);
    return NLQ_OK;
}

nlq_status nlq_submit(nlq_ctx *ctx, const nlq_request *req, uint64_t *ticket)
{
    if (!ctx || !req || !ticket) {
        set_last_error("NULL argument");
        return NLQ_EINVAL;
    }
    Server *S = ctx->impl.server.get();
    if (!S) {
        set_last_error("nlq_serve_start has not been called");
        return NLQ_EINVAL;
    }
    if ((req->dim != 2 && req->dim != 3) || req->n < 1 || req->k_gamma < 0 || !req->f_nodal || !req->g_nodal ||
        req->params.dim != req->dim) {
        set_last_error("bad request (dim, n, k_gamma, data pointers or params.dim)");
        return NLQ_EINVAL;
    }
    auto r = std::make_shared<Request>();
    r->req = *req;
    r->req.f_nodal = r->req.g_nodal = nullptr;
    int64_t nn = 1;
    for (int k = 0; k < req->dim; ++k) nn *= (req->n + 1);
    r->f.assign(req->f_nodal, req->f_nodal + nn);
    r->g.assign(req->g_nodal, req->g_nodal + nn);
    r->t_submit = serve_now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            set_last_error("server is stopping");
            return NLQ_EBUSY;
        }
        r->ticket = S->next_ticket++;
        S->all[r->ticket] = r;
        S->pending.push_back(r);
        ++S->stats.submitted;
        admit_locked(*S);
    }
    drain(*S);
    *ticket = r->ticket;
    return NLQ_OK;
}

nlq_status nlq_wait(nlq_ctx *ctx, uint64_t ticket, int32_t timeout_ms, nlq_result *out)
{
    if (!ctx || !out) {
        set_last_error("NULL argument");
        return NLQ_EINVAL;
    }
    Server *S = ctx->impl.server.get();
    if (!S) {
        set_last_error("server not running");
        return NLQ_EINVAL;
    }
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) {
        set_last_error("unknown ticket");
        return NLQ_EINVAL;
    }
    auto r = it->second;
    auto ready = [&] { return r->done; };
    if (timeout_ms < 0) S->cv_done.wait(lk, ready);
    else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) return NLQ_ENOTREADY;
    out->status = r->status;
    out->n_nodes = r->n_nodes;
    out->n_pairs = r->n_pairs;
    out->n_free = r->n_free;
    out->u = r->u.empty() ? nullptr : r->u.data();
    out->cg_iterations = r->cg_iterations;
    out->rel_residual = r->rel_residual;
    out->latency_s = r->t_done - r->t_submit;
    out->queue_s = (r->t_admit > 0 ? r->t_admit : r->t_done) - r->t_submit;
    out->assemble_s = (r->t_ready > 0 && r->t_admit > 0 && !r->cache_hit) ? r->t_ready - r->t_admit : 0.0;
    out->solve_s = r->t_ready > 0 ? r->t_done - r->t_ready : 0.0;
    out->launches = r->launches;
    out->cache_hit = r->cache_hit ? 1 : 0;
    out->setup_s = (r->t_setup > 0 && r->t_admit > 0) ? r->t_setup - r->t_admit : 0.0;
    if (r->status != NLQ_OK) set_last_error(r->error);
    return NLQ_OK;
}

nlq_status nlq_cancel(nlq_ctx *ctx, uint64_t ticket)
{
    if (!ctx || !ctx->impl.server) {
        set_last_error("server not running");
        return NLQ_EINVAL;
    }
    Server *S = ctx->impl.server.get();
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) {
        set_last_error("unknown ticket");
        return NLQ_EINVAL;
    }
    ReqPtr r = it->second;
    if (r->done) return NLQ_OK;
    r->cancelled = true;
    auto pos = std::find(S->pending.begin(), S->pending.end(), r);
    if (pos != S->pending.end()) {
        S->pending.erase(pos);
        finish_locked(*S, r, NLQ_ECANCELLED, "cancelled");
    }
    S->cv_dev.notify_all();
    return NLQ_OK;
}

nlq_status nlq_result_release(nlq_ctx *ctx, uint64_t ticket)
{
    if (!ctx || !ctx->impl.server) {
        set_last_error("server not running");
        return NLQ_EINVAL;
    }
    Server *S = ctx->impl.server.get();
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end() || !it->second->done) {
        set_last_error("unknown or unfinished ticket");
        return NLQ_EINVAL;
    }
    S->all.erase(it);
    return NLQ_OK;
}

nlq_status nlq_serve_stats_get(nlq_ctx *ctx, nlq_serve_stats *out)
{
    if (!ctx || !out || !ctx->impl.server) {
        set_last_error("server not running or NULL argument");
        return NLQ_EINVAL;
    }
    Server *S = ctx->impl.server.get();
    std::lock_guard<std::mutex> lk(S->mu);
    S->stats.peak_bytes = std::max<uint64_t>(S->stats.peak_bytes, S->ctx->used.load());
    *out = S->stats;
    return NLQ_OK;
}

nlq_status nlq_serve_stop(nlq_ctx *ctx)
{
    if (!ctx) return NLQ_EINVAL;
    Server *S = ctx->impl.server.get();
    if (!S) return NLQ_OK;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->stop = true;
        // every submitted request finishes first
        S->cv_done.wait(lk, [&] {
            if (!S->pending.empty() || S->admitted > 0) return false;
            for (auto &kv : S->all)
                if (!kv.second->done) return false;
            return true;
        });
        S->cv_dev.notify_all();
    }
    if (S->dev.joinable()) S->dev.join();
    (void)hipSetDevice(ctx->impl.device);
    S->cache.clear();
    S->graveyard.clear();
    S->all.clear();
    S->meshes.clear();
    if (S->stream) (void)hipStreamDestroy(S->stream);
    ctx->impl.server.reset();
    return NLQ_OK;
}

}  // extern "C"
