// Serving loop: requests are queued by nlq_submit and executed by a scheduler
// thread that owns the context's device work; results are fetched with
// nlq_wait.  Meshes stay resident in a cache keyed by (dim, n, k_gamma).
#include <chrono>
#include <unordered_map>

#include "nlq_internal.hpp"

namespace nlq {

struct Request {
    uint64_t ticket = 0;
    nlq_request req{};
    std::vector<double> f, g;
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
    nlq_status status = NLQ_ENOTREADY;
    bool cancelled = false, done = false;
    std::vector<double> u;
    int64_t n_nodes = 0, n_pairs = 0, n_free = 0;
    int cg_iterations = 0;
    double rel_residual = 0.0;
    std::string error;
};

struct Server {
    Ctx *ctx = nullptr;
    int max_active = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    std::map<std::tuple<int, int, int>, nlq_mesh *> meshes;
};

double serve_now()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace nlq

using namespace nlq;

extern "C" {
nlq_status nlq_mesh_box(nlq_ctx *ctx, int32_t dim, int32_t n, int32_t k_gamma, nlq_mesh **out);
nlq_status nlq_mesh_destroy(nlq_mesh *mesh);
}

nlq::Ctx::Ctx() = default;
nlq::Ctx::~Ctx() = default;

namespace {

void run_request(Server &S, nlq_ctx *ctx, Request &r)
{
    const auto key = std::make_tuple(r.req.dim, r.req.n, r.req.k_gamma);
    nlq_mesh *mesh = nullptr;
    auto it = S.meshes.find(key);
    if (it != S.meshes.end()) {
        mesh = it->second;
    } else {
        nlq_status st = nlq_mesh_box(ctx, r.req.dim, r.req.n, r.req.k_gamma, &mesh);
        if (st != NLQ_OK) {
            r.status = st;
            r.error = nlq_last_error();
            return;
        }
        S.meshes[key] = mesh;
    }
    nlq_system *sys = nullptr;
    nlq_status st = nlq_assemble(ctx, mesh, &r.req.params, &sys);
    if (st != NLQ_OK) {
        r.status = st;
        r.error = nlq_last_error();
        return;
    }
    int64_t nn = 0, nnz = 0, np = 0, nf = 0;
    nlq_info(sys, &nn, &nnz, &np, &nf);
    r.n_nodes = nn;
    r.n_pairs = np;
    r.n_free = nf;
    st = nlq_set_data(sys, r.f.data(), r.g.data());
    if (st == NLQ_OK) {
        r.u.assign(nn, 0.0);
        nlq_solve_info info{};
        st = nlq_solve(sys, r.req.rtol > 0 ? r.req.rtol : 1e-10, r.req.maxit > 0 ? r.req.maxit : 10000,
                       r.u.data(), &info);
        r.cg_iterations = info.iterations;
        r.rel_residual = info.rel_residual;
    }
    r.status = st;
    if (st != NLQ_OK) r.error = nlq_last_error();
    nlq_system_destroy(sys);
}

void worker_main(Server *S, nlq_ctx *ctx)
{
    (void)hipSetDevice(ctx->impl.device);
    for (;;) {
        std::shared_ptr<Request> r;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            if (S->stop && S->queue.empty()) return;
            r = S->queue.front();
            S->queue.pop_front();
            if (r->cancelled) {
                r->status = NLQ_ECANCELLED;
                r->done = true;
                r->t_done = serve_now();
                S->cv_done.notify_all();
                continue;
            }
            r->t_admit = serve_now();
        }
        run_request(*S, ctx, *r);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            r->t_done = serve_now();
            r->done = true;
        }
        S->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

nlq_status nlq_serve_start(nlq_ctx *ctx, int32_t max_active)
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
    S->max_active = max_active > 0 ? max_active : 1;
    Server *raw = S.get();
    ctx->impl.server = std::move(S);
    raw->worker = std::thread(worker_main, raw, ctx);
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
    if ((req->dim != 2 && req->dim != 3) || req->n < 1 || !req->f_nodal || !req->g_nodal) {
        set_last_error("bad request");
        return NLQ_EINVAL;
    }
    auto r = std::make_shared<Request>();
    r->req = *req;
    int64_t nn = 1;
    for (int k = 0; k < req->dim; ++k) nn *= (req->n + 1);
    r->f.assign(req->f_nodal, req->f_nodal + nn);
    r->g.assign(req->g_nodal, req->g_nodal + nn);
    r->t_submit = serve_now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r->ticket = S->next_ticket++;
        S->all[r->ticket] = r;
        S->queue.push_back(r);
    }
    S->cv_work.notify_one();
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
    it->second->cancelled = true;
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

nlq_status nlq_serve_stop(nlq_ctx *ctx)
{
    if (!ctx) return NLQ_EINVAL;
    Server *S = ctx->impl.server.get();
    if (!S) return NLQ_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (auto &kv : S->meshes) nlq_mesh_destroy(kv.second);
    ctx->impl.server.reset();
    return NLQ_OK;
}

}  // extern "C"
