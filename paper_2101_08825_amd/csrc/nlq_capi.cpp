// C-ABI of libnlq: argument checking, ownership, device memory accounting and
// the sequencing of the assembly / solve stages.  Every entry point catches
// errors and returns an nlq_status; nothing aborts.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>

#include "nlq_internal.hpp"

namespace nlq {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string &msg) { g_last_error = msg; }

[[noreturn]] void fail(nlq_status st, const std::string &msg) { throw Error{st, msg}; }

namespace {

// size class of a cached block: powers of two up to 1 MiB, then whole MiB
size_t size_class(size_t b)
{
    constexpr size_t kMiB = size_t(1) << 20;
    if (b > kMiB) return (b + kMiB - 1) / kMiB * kMiB;
    size_t c = 256;
    while (c < b) c <<= 1;
    return c;
}

}  // namespace

void *Ctx::cache_take(size_t cls)
{
    std::lock_guard<std::mutex> lk(cache_mu);
    auto it = cache.find(cls);
    if (it == cache.end()) return nullptr;
    void *p = it->second;
    cache.erase(it);
    cached -= cls;
    return p;
}

void Ctx::cache_put(void *p, size_t cls)
{
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        if (cached + cls <= kCacheMax && used.load() + cached + cls <= budget) {
            cache.emplace(cls, p);
            cached += cls;
            return;
        }
    }
    (void)hipFree(p);
}

void Ctx::cache_trim(uint64_t need)
{
    std::vector<void *> drop;
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        while (!cache.empty() && (need == UINT64_MAX || used.load() + cached + need > budget)) {
            auto it = std::prev(cache.end());   // largest first
            drop.push_back(it->second);
            cached -= it->first;
            cache.erase(it);
        }
    }
    for (void *p : drop) (void)hipFree(p);
    if (need == UINT64_MAX || !drop.empty()) {
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) (void)hipMemPoolTrimTo(pool, 0);
    }
}

void DevBuf::alloc(Ctx *ctx, size_t bytes, hipStream_t st)
{
    release();
    if (bytes == 0) bytes = 8;
    if (ctx->allocs.fetch_add(1) == ctx->alloc_fail_at)
        fail(NLQ_ENOMEM, "injected allocation failure (NLQ_FAIL_ALLOC_AT)");
    const size_t charge = st ? bytes : size_class(bytes);
    const uint64_t now = ctx->used.fetch_add(charge) + charge;
    if (now > ctx->budget) {
        ctx->used.fetch_sub(charge);
        fail(NLQ_ENOMEM, "device memory budget exceeded (" + std::to_string(now) + " > " +
                             std::to_string(ctx->budget) + " bytes)");
    }
    void *p = nullptr;
    hipError_t e = hipSuccess;
    if (st) {
        e = hipMallocAsync(&p, bytes, st);
    } else if (!(p = ctx->cache_take(charge))) {
        ctx->cache_trim(0);
        e = hipMalloc(&p, charge);
        if (e != hipSuccess) {
            // the device may be short of memory the cache still holds
            ctx->cache_trim(UINT64_MAX);
            e = hipMalloc(&p, charge);
        }
    }
    if (e != hipSuccess) {
        ctx->used.fetch_sub(charge);
        fail(NLQ_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    p_ = p;
    bytes_ = bytes;
    cls_ = st ? 0 : charge;
    ctx_ = ctx;
    st_ = st;
}

void DevBuf::release()
{
    if (p_) {
        if (st_) {
            (void)hipFreeAsync(p_, st_);
            ctx_->used.fetch_sub(bytes_);
        } else {
            // no kernel may still use the block when it is handed out again
            (void)hipDeviceSynchronize();
            ctx_->used.fetch_sub(cls_);
            ctx_->cache_put(p_, cls_);
        }
    }
    p_ = nullptr;
    bytes_ = 0;
    cls_ = 0;
}

namespace {

template <class F> nlq_status guard(F &&f)
{
    try {
        f();
        g_last_error.clear();
        return NLQ_OK;
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return NLQ_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return NLQ_EINVAL;
    }
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void check_params(const Mesh &m, const nlq_params &p)
{
    if (p.dim != m.dim) fail(NLQ_EINVAL, "params.dim does not match the mesh");
    if (!(p.delta > 0.0) || !(p.eps > 0.0) || !(p.eps < p.delta))
        fail(NLQ_EINVAL, "need 0 < eps < delta");
    if (p.lmin < 1 || p.lmax < p.lmin) fail(NLQ_EINVAL, "need 1 <= lmin <= lmax");
    if (p.lmax > (m.dim == 2 ? 8 : 6)) fail(NLQ_EINVAL, "lmax too large (max 8 in 2D, 6 in 3D)");
    if (p.kernel != NLQ_ETA_CONST && p.kernel != NLQ_ETA_GAUSS) fail(NLQ_EINVAL, "unknown kernel");
    if (p.form != NLQ_FORM_SYM4 && p.form != NLQ_FORM_PAPER2 && p.form != NLQ_FORM_PAPER2_INNER)
        fail(NLQ_EINVAL, "unknown form");
    if (p.form == NLQ_FORM_PAPER2_INNER && p.deterministic)
        fail(NLQ_EINVAL, "the adaptive-inner two-term form has no deterministic mode");
    if ((m.order == 2 || m.shape == 1) && p.deterministic)
        fail(NLQ_EINVAL, "P2, quadrilateral and hexahedral elements have no deterministic mode");
    if ((m.order == 2 || m.shape == 1) && p.precision != NLQ_FP64_PLAIN)
        fail(NLQ_EINVAL, "P2, quadrilateral and hexahedral elements are integrated in FP64 (NLQ_FP64_PLAIN)");
    if (p.precision != NLQ_FP64_PLAIN && p.precision != NLQ_FP32_MIXED)
        fail(NLQ_EINVAL, "unknown precision");
    if (p.deterministic != 0 && p.deterministic != 1) fail(NLQ_EINVAL, "deterministic must be 0 or 1");
    if (p.min_dist_l2 < 0 || p.min_dist_l2 > 2) fail(NLQ_EINVAL, "min_dist_l2 must be 0, 1 or 2");
    if (p.scale < 0.0) fail(NLQ_EINVAL, "scale must be >= 0");
}

void mesh_stats(Mesh &m)
{
    const int dim = m.dim, nv = m.ngeo, nb = m.nb;
    for (int k = 0; k < 3; ++k) {
        m.gmin[k] = 0.0;
        m.gmax[k] = 0.0;
        m.ext_max[k] = 0.0;
    }
    for (int k = 0; k < dim; ++k) {
        m.gmin[k] = INFINITY;
        m.gmax[k] = -INFINITY;
    }
    for (int64_t n = 0; n < m.n_nodes; ++n)
        for (int k = 0; k < dim; ++k) {
            const double x = m.h_coords[n * dim + k];
            if (!std::isfinite(x)) fail(NLQ_EINVAL, "non-finite coordinate");
            m.gmin[k] = std::min(m.gmin[k], x);
            m.gmax[k] = std::max(m.gmax[k], x);
        }
    for (int64_t e = 0; e < m.n_elems; ++e) {
        double V[8][3];
        for (int v = 0; v < nv; ++v) {
            const int32_t id = m.h_conn[e * nb + v];
            if (id < 0 || id >= m.n_nodes) fail(NLQ_EINVAL, "node id out of range in element " + std::to_string(e));
            for (int k = 0; k < dim; ++k) V[v][k] = m.h_coords[static_cast<int64_t>(id) * dim + k];
        }
        for (int k = 0; k < dim; ++k) {
            double a = V[0][k], b = V[0][k];
            for (int v = 1; v < nv; ++v) {
                a = std::min(a, V[v][k]);
                b = std::max(b, V[v][k]);
            }
            m.ext_max[k] = std::max(m.ext_max[k], b - a);
        }
        // the simplex's edges from vertex 0; a box's edges from corner 0 (corners
        // 1, 2 and 4 in tensor order)
        const int i1 = 1, i2 = 2, i3 = m.shape ? 4 : 3;
        double det;
        if (dim == 2) {
            det = (V[i1][0] - V[0][0]) * (V[i2][1] - V[0][1]) - (V[i1][1] - V[0][1]) * (V[i2][0] - V[0][0]);
        } else {
            double a[3], b[3], c[3];
            for (int k = 0; k < 3; ++k) {
                a[k] = V[i1][k] - V[0][k];
                b[k] = V[i2][k] - V[0][k];
                c[k] = V[i3][k] - V[0][k];
            }
            det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                  a[2] * (b[0] * c[1] - b[1] * c[0]);
        }
        if (!(std::fabs(det) > 0.0)) fail(NLQ_EINVAL, "element " + std::to_string(e) + " has zero measure");
        for (int v = nv; v < nb; ++v) {
            const int32_t id = m.h_conn[e * nb + v];
            if (id < 0 || id >= m.n_nodes) fail(NLQ_EINVAL, "node id out of range in element " + std::to_string(e));
        }
    }
    m.n_free = 0;
    for (int64_t n = 0; n < m.n_nodes; ++n) m.n_free += m.h_constrained[n] ? 0 : 1;
}

void upload_mesh(Mesh &m, hipStream_t st)
{
    const int nv = m.nb;
    m.coords.alloc(m.ctx, sizeof(double) * m.n_nodes * m.dim);
    m.conn.alloc(m.ctx, sizeof(int32_t) * m.n_elems * nv);
    m.constrained.alloc(m.ctx, m.n_nodes);
    NLQ_HIP(hipMemcpyAsync(m.coords.as<void>(), m.h_coords.data(), sizeof(double) * m.n_nodes * m.dim,
                           hipMemcpyHostToDevice, st));
    NLQ_HIP(hipMemcpyAsync(m.conn.as<void>(), m.h_conn.data(), sizeof(int32_t) * m.n_elems * nv,
                           hipMemcpyHostToDevice, st));
    NLQ_HIP(hipMemcpyAsync(m.constrained.as<void>(), m.h_constrained.data(), m.n_nodes,
                           hipMemcpyHostToDevice, st));
    NLQ_HIP(hipStreamSynchronize(st));
}

}  // namespace

// Everything up to the integration: element tables, pair list, pattern, value
// arrays (on stream st; returns with st synchronised).
std::unique_ptr<nlq_system> prepare_system(Ctx &ctx, const Mesh &mesh, const nlq_params &params, hipStream_t st)
{
    check_params(mesh, params);
    auto sys = std::make_unique<nlq_system>();
    System &s = sys->impl;
    s.ctx = &ctx;
    s.mesh = &mesh;
    s.p = params;
    s.C = params.scale > 0.0 ? params.scale : kernel_constant(params.dim, params.kernel, params.delta, params.eps);
    (void)ctx.get_tables(mesh.dim, s.p.lmax);
    s.counters.alloc(s.ctx, sizeof(AsmCounters));
    NLQ_HIP(hipStreamSynchronize(st));
    const double t0 = now_s();
    launch_elem_tables(s, st);
    NLQ_HIP(hipStreamSynchronize(st));
    const double t1 = now_s();
    build_pairs(s, st);
    const double t2 = now_s();
    build_pattern(s, st);
    s.cfg = tuned_config(ctx, s);
    s.val.alloc(s.ctx, sizeof(double) * std::max<int64_t>(s.nnz, 1));
    const int nr = mesh.nb * (mesh.nb + 1) / 2;   // upper-triangle slots of a diagonal block
    s.dmm.alloc(s.ctx, sizeof(double) * std::max<int64_t>(mesh.n_elems * nr, 1));
    NLQ_HIP(hipStreamSynchronize(st));
    const double t3 = now_s();
    s.info.n_pairs = s.n_pairs;
    s.info.nnz = s.nnz;
    s.info.t_tables = t1 - t0;
    s.info.t_pairs = t2 - t1;
    s.info.t_pattern = t3 - t2;
    return sys;
}

void check_counter_error(int error)
{
    if (!error) return;
    std::string msg;
    if (error & kErrStack) msg += "refinement traversal exceeded its stack";
    if (error & kErrPattern) msg += std::string(msg.empty() ? "" : "; ") + "a block entry fell outside the CSR pattern";
    if (error & ~(kErrStack | kErrPattern)) msg += std::string(msg.empty() ? "" : "; ") + "unknown integration error";
    fail(NLQ_EDEVICE, msg);
}

// counters of a finished integration -> info (synchronises st)
void collect_counters(System &s, hipStream_t st)
{
    AsmCounters c{};
    NLQ_HIP(hipMemcpyAsync(&c, s.counters.as<void>(), sizeof(AsmCounters), hipMemcpyDeviceToHost, st));
    NLQ_HIP(hipStreamSynchronize(st));
    // rule points per element: 7 / 15 on simplices, 9 / 27 on boxes
    const int nq = s.mesh->shape == 1 ? (s.mesh->dim == 2 ? 9 : 27) : (s.mesh->dim == 2 ? 7 : 15);
    int64_t leaves = 0;
    for (int q = 0; q < 9; ++q) {
        s.info.n_leaf[q] = (q >= 1 && q <= 8) ? static_cast<int64_t>(c.leaf[q]) : 0;
        leaves += s.info.n_leaf[q];
    }
    s.info.n_evals = leaves * nq * nq;
    s.info.n_leaf_zero = static_cast<int64_t>(c.zero_leaves);
    check_counter_error(c.error);
    if (static_cast<int64_t>(c.pairs_done) != s.n_pairs)
        fail(NLQ_EDEVICE, "integration did not visit every pair");
}

void run_integrate(System &s, hipStream_t st)
{
    const double t0 = now_s();
    hipEvent_t e0, e1;
    NLQ_HIP(hipEventCreate(&e0));
    NLQ_HIP(hipEventCreate(&e1));
    launch_integrate(s, st, e0, e1);
    collect_counters(s, st);
    s.info.t_integrate = now_s() - t0;
    float ms = 0.0f;
    NLQ_HIP(hipEventElapsedTime(&ms, e0, e1));
    s.info.t_kernel = 1e-3 * ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    s.integrated = true;
}

std::unique_ptr<nlq_mesh> make_box_mesh(Ctx &ctx, int dim, int n, int k_gamma, hipStream_t st)
{
    if (dim != 2 && dim != 3) fail(NLQ_EINVAL, "dim must be 2 or 3");
    if (n < 1 || k_gamma < 0) fail(NLQ_EINVAL, "bad box size");
    int64_t nn = 1, ne = 1;
    for (int k = 0; k < dim; ++k) {
        nn *= (n + 1);
        ne *= n;
    }
    ne *= (dim == 2 ? 2 : 6);
    if (nn > INT32_MAX || ne > INT32_MAX) fail(NLQ_EINVAL, "mesh too large for int32 ids");
    auto m = std::make_unique<nlq_mesh>();
    Mesh &M = m->impl;
    M.ctx = &ctx;
    M.dim = dim;
    M.order = 1;
    M.nb = dim + 1;
    M.ngeo = dim + 1;
    M.n_nodes = nn;
    M.n_elems = ne;
    M.coords.alloc(M.ctx, sizeof(double) * nn * dim);
    M.conn.alloc(M.ctx, sizeof(int32_t) * ne * (dim + 1));
    M.constrained.alloc(M.ctx, nn);
    launch_box_mesh(dim, n, k_gamma, M.coords.as<double>(), M.conn.as<int32_t>(), M.constrained.as<uint8_t>(), st);
    M.h_coords.resize(nn * dim);
    M.h_conn.resize(ne * (dim + 1));
    M.h_constrained.resize(nn);
    NLQ_HIP(hipMemcpyAsync(M.h_coords.data(), M.coords.as<void>(), sizeof(double) * nn * dim,
                           hipMemcpyDeviceToHost, st));
    NLQ_HIP(hipMemcpyAsync(M.h_conn.data(), M.conn.as<void>(), sizeof(int32_t) * ne * (dim + 1),
                           hipMemcpyDeviceToHost, st));
    NLQ_HIP(hipMemcpyAsync(M.h_constrained.data(), M.constrained.as<void>(), nn, hipMemcpyDeviceToHost, st));
    NLQ_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < 3; ++k) {
        M.gmin[k] = 0.0;
        M.gmax[k] = k < dim ? 1.0 : 0.0;
        M.ext_max[k] = k < dim ? 1.0 / n : 0.0;
    }
    M.n_free = 0;
    for (int64_t q = 0; q < nn; ++q) M.n_free += M.h_constrained[q] ? 0 : 1;
    return m;
}

void load_data(System &s, const double *f_nodal, const double *g_nodal, hipStream_t st)
{
    const int64_t n = s.mesh->n_nodes;
    DevBuf f(s.ctx, sizeof(double) * n, st);
    if (s.g.empty()) s.g.alloc(s.ctx, sizeof(double) * n);
    NLQ_HIP(hipMemcpyAsync(f.as<void>(), f_nodal, sizeof(double) * n, hipMemcpyHostToDevice, st));
    NLQ_HIP(hipMemcpyAsync(s.g.as<void>(), g_nodal, sizeof(double) * n, hipMemcpyHostToDevice, st));
    launch_load_lift(s, st, f.as<double>(), s.g.as<double>());
    NLQ_HIP(hipStreamSynchronize(st));
    s.has_rhs = true;
}

bool solve_system(System &s, double rtol, int maxit, double *u_out, nlq_solve_info *info, hipStream_t st)
{
    if (!s.has_rhs) fail(NLQ_EINVAL, "nlq_set_data must be called before nlq_solve");
    if (!(rtol > 0.0) || maxit < 1) fail(NLQ_EINVAL, "need rtol > 0 and maxit >= 1");
    const double t0 = now_s();
    double relres = 0.0;
    int converged = 0;
    // the two-term forms are not symmetric: BiCGSTAB instead of CG
    const int it = s.p.form == NLQ_FORM_SYM4 ? cg_solve(s, st, rtol, maxit, &relres, &converged)
                                             : bicgstab_solve(s, st, rtol, maxit, &relres, &converged);
    if (u_out) {
        NLQ_HIP(hipMemcpyAsync(u_out, s.u.as<void>(), sizeof(double) * s.mesh->n_nodes, hipMemcpyDeviceToHost, st));
        NLQ_HIP(hipStreamSynchronize(st));
    }
    if (info) {
        info->iterations = it;
        info->converged = converged;
        info->rel_residual = relres;
        info->seconds = now_s() - t0;
    }
    return converged != 0;
}

}  // namespace nlq

using namespace nlq;

extern "C" {

const char *nlq_last_error(void) { return g_last_error.c_str(); }

nlq_status nlq_ctx_create(int32_t device, uint64_t hbm_budget_bytes, nlq_ctx **out)
{
    return guard([&] {
        if (!out) fail(NLQ_EINVAL, "out is NULL");
        int ndev = 0;
        NLQ_HIP(hipGetDeviceCount(&ndev));
        if (device < 0 || device >= ndev) fail(NLQ_EINVAL, "no such device");
        NLQ_HIP(hipSetDevice(device));
        // the device address of the allocation-free solve's scratch, once per device
        noalloc_scratch_init(device);
        auto c = std::make_unique<nlq_ctx>();
        c->impl.device = device;
        hipDeviceProp_t prop;
        NLQ_HIP(hipGetDeviceProperties(&prop, device));
        c->impl.n_cu = prop.multiProcessorCount;
        c->impl.arch = prop.gcnArchName;
        c->impl.arch = c->impl.arch.substr(0, c->impl.arch.find(':'));
        size_t fr = 0, tot = 0;
        NLQ_HIP(hipMemGetInfo(&fr, &tot));
        c->impl.budget = hbm_budget_bytes ? hbm_budget_bytes : static_cast<uint64_t>(0.9 * fr);
        NLQ_HIP(hipStreamCreateWithFlags(&c->impl.own_stream, hipStreamNonBlocking));
        c->impl.stream = c->impl.own_stream;
        if (const char *env = std::getenv("NLQ_FAIL_ALLOC_AT")) c->impl.alloc_fail_at = std::atoll(env);
        // stream-ordered temporaries come from the device's default pool; keep
        // what they free there instead of unmapping it at every synchronisation
        // (the pool is trimmed with the block cache when memory runs short)
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
        *out = c.release();
    });
}

nlq_status nlq_ctx_set_stream(nlq_ctx *ctx, void *hip_stream)
{
    return guard([&] {
        if (!ctx) fail(NLQ_EINVAL, "ctx is NULL");
        ctx->impl.stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : ctx->impl.own_stream;
    });
}

nlq_status nlq_ctx_memory(const nlq_ctx *ctx, uint64_t *used, uint64_t *budget)
{
    return guard([&] {
        if (!ctx) fail(NLQ_EINVAL, "ctx is NULL");
        if (used) *used = ctx->impl.used.load();
        if (budget) *budget = ctx->impl.budget;
    });
}

nlq_status nlq_serve_stop(nlq_ctx *ctx);

nlq_status nlq_ctx_destroy(nlq_ctx *ctx)
{
    return guard([&] {
        if (!ctx) return;
        nlq_serve_stop(ctx);
        (void)hipSetDevice(ctx->impl.device);
        (void)hipStreamSynchronize(ctx->impl.stream);
        ctx->impl.tables.clear();
        ctx->impl.cache_trim(UINT64_MAX);
        (void)hipStreamDestroy(ctx->impl.own_stream);
        delete ctx;
    });
}

nlq_status nlq_mesh_create_shape(nlq_ctx *ctx, int32_t dim, int32_t shape, int32_t order, int64_t n_nodes,
                                 const double *coords, int64_t n_elems, const int32_t *conn,
                                 const uint8_t *constrained, nlq_mesh **out)
{
    return guard([&] {
        if (!ctx || !out || !coords || !conn || !constrained) fail(NLQ_EINVAL, "NULL argument");
        if (dim != 2 && dim != 3) fail(NLQ_EINVAL, "dim must be 2 or 3");
        if (shape != NLQ_SHAPE_SIMPLEX && shape != NLQ_SHAPE_BOX) fail(NLQ_EINVAL, "unknown element shape");
        if (order != 1 && order != 2) fail(NLQ_EINVAL, "order must be 1 or 2");
        const int ngeo = shape == NLQ_SHAPE_BOX ? 1 << dim : dim + 1;
        if (n_nodes < ngeo || n_elems < 1) fail(NLQ_EINVAL, "empty mesh");
        if (n_nodes > INT32_MAX || n_elems > INT32_MAX) fail(NLQ_EINVAL, "mesh too large for int32 ids");
        NLQ_HIP(hipSetDevice(ctx->impl.device));
        auto m = std::make_unique<nlq_mesh>();
        Mesh &M = m->impl;
        M.ctx = &ctx->impl;
        M.dim = dim;
        M.shape = shape;
        M.order = order;
        M.ngeo = ngeo;
        M.nb = shape == NLQ_SHAPE_BOX ? (order == 2 ? (dim == 2 ? 8 : 20) : 1 << dim)
                                      : (order == 2 ? (dim + 1) * (dim + 2) / 2 : dim + 1);
        M.n_nodes = n_nodes;
        M.n_elems = n_elems;
        M.h_coords.assign(coords, coords + n_nodes * dim);
        M.h_conn.assign(conn, conn + n_elems * M.nb);
        M.h_constrained.assign(constrained, constrained + n_nodes);
        for (auto &c : M.h_constrained) c = c ? 1 : 0;
        mesh_stats(M);
        upload_mesh(M, ctx->impl.stream);
        *out = m.release();
    });
}

nlq_status nlq_mesh_create_order(nlq_ctx *ctx, int32_t dim, int32_t order, int64_t n_nodes, const double *coords,
                                 int64_t n_elems, const int32_t *conn, const uint8_t *constrained, nlq_mesh **out)
{
    return nlq_mesh_create_shape(ctx, dim, NLQ_SHAPE_SIMPLEX, order, n_nodes, coords, n_elems, conn, constrained,
                                 out);
}

nlq_status nlq_mesh_create(nlq_ctx *ctx, int32_t dim, int64_t n_nodes, const double *coords,
                           int64_t n_elems, const int32_t *conn, const uint8_t *constrained,
                           nlq_mesh **out)
{
    return nlq_mesh_create_order(ctx, dim, 1, n_nodes, coords, n_elems, conn, constrained, out);
}

nlq_status nlq_mesh_box(nlq_ctx *ctx, int32_t dim, int32_t n, int32_t k_gamma, nlq_mesh **out)
{
    return guard([&] {
        if (!ctx || !out) fail(NLQ_EINVAL, "NULL argument");
        NLQ_HIP(hipSetDevice(ctx->impl.device));
        *out = make_box_mesh(ctx->impl, dim, n, k_gamma, ctx->impl.stream).release();
    });
}

nlq_status nlq_mesh_info(const nlq_mesh *mesh, int32_t *dim, int64_t *n_nodes, int64_t *n_elems,
                         int64_t *n_free)
{
    return guard([&] {
        if (!mesh) fail(NLQ_EINVAL, "mesh is NULL");
        if (dim) *dim = mesh->impl.dim;
        if (n_nodes) *n_nodes = mesh->impl.n_nodes;
        if (n_elems) *n_elems = mesh->impl.n_elems;
        if (n_free) *n_free = mesh->impl.n_free;
    });
}

nlq_status nlq_mesh_copy(const nlq_mesh *mesh, double *coords, int32_t *conn, uint8_t *constrained)
{
    return guard([&] {
        if (!mesh) fail(NLQ_EINVAL, "mesh is NULL");
        const Mesh &M = mesh->impl;
        if (coords) std::copy(M.h_coords.begin(), M.h_coords.end(), coords);
        if (conn) std::copy(M.h_conn.begin(), M.h_conn.end(), conn);
        if (constrained) std::copy(M.h_constrained.begin(), M.h_constrained.end(), constrained);
    });
}

nlq_status nlq_mesh_destroy(nlq_mesh *mesh)
{
    return guard([&] {
        if (!mesh) return;
        (void)hipSetDevice(mesh->impl.ctx->device);
        delete mesh;
    });
}

nlq_status nlq_assemble(nlq_ctx *ctx, const nlq_mesh *mesh, const nlq_params *params,
                        nlq_system **out)
{
    return guard([&] {
        if (!ctx || !mesh || !params || !out) fail(NLQ_EINVAL, "NULL argument");
        if (mesh->impl.ctx != &ctx->impl) fail(NLQ_EINVAL, "mesh belongs to another context");
        NLQ_HIP(hipSetDevice(ctx->impl.device));
        hipStream_t st = ctx->impl.stream;
        auto sys = prepare_system(ctx->impl, mesh->impl, *params, st);
        System &s = sys->impl;
        const double t3 = now_s();
        run_integrate(s, st);
        s.info.t_total = (now_s() - t3) + s.info.t_tables + s.info.t_pairs + s.info.t_pattern;
        *out = sys.release();
    });
}

nlq_status nlq_prepare(nlq_ctx *ctx, const nlq_mesh *mesh, const nlq_params *params, nlq_system **out)
{
    return guard([&] {
        if (!ctx || !mesh || !params || !out) fail(NLQ_EINVAL, "NULL argument");
        if (mesh->impl.ctx != &ctx->impl) fail(NLQ_EINVAL, "mesh belongs to another context");
        NLQ_HIP(hipSetDevice(ctx->impl.device));
        hipStream_t st = ctx->impl.stream;
        auto sys = prepare_system(ctx->impl, mesh->impl, *params, st);
        System &s = sys->impl;
        NLQ_HIP(hipMemsetAsync(s.val.as<void>(), 0, sizeof(double) * std::max<int64_t>(s.nnz, 1), st));
        NLQ_HIP(hipStreamSynchronize(st));
        s.info.t_total = s.info.t_tables + s.info.t_pairs + s.info.t_pattern;
        *out = sys.release();
    });
}

nlq_status nlq_integrate_ranges(nlq_system *sys, int32_t n_ranges, const int64_t *lo, const int64_t *hi,
                                double *kernel_s, int64_t *n_leaf, int64_t *n_leaf_zero)
{
    return guard([&] {
        if (!sys) fail(NLQ_EINVAL, "sys is NULL");
        if (n_ranges < 1 || n_ranges > 32 || !lo || !hi) fail(NLQ_EINVAL, "need 1..32 ranges and both bound arrays");
        System &s = sys->impl;
        const int64_t ne = s.mesh->n_elems;
        std::vector<std::pair<int64_t, int64_t>> r;
        for (int k = 0; k < n_ranges; ++k) {
            if (lo[k] < 1 || hi[k] >= ne || lo[k] >= hi[k])
                fail(NLQ_EINVAL, "need 0 < lo < hi < n_elems (a range that neither clears nor finishes the values)");
            r.emplace_back(lo[k], hi[k]);
        }
        std::sort(r.begin(), r.end());
        for (size_t k = 1; k < r.size(); ++k)
            if (r[k].first < r[k - 1].second) fail(NLQ_EINVAL, "ranges overlap");
        if (s.p.deterministic) fail(NLQ_EINVAL, "a deterministic system is integrated whole");
        NLQ_HIP(hipSetDevice(s.ctx->device));
        hipStream_t st = s.ctx->stream;
        hipEvent_t e0, e1;
        NLQ_HIP(hipEventCreate(&e0));
        NLQ_HIP(hipEventCreate(&e1));
        std::vector<IntegrateJob> jobs;
        for (const auto &q : r) jobs.push_back(IntegrateJob{&s, q.first, q.second});
        NLQ_HIP(hipMemsetAsync(s.counters.as<void>(), 0, sizeof(AsmCounters), st));
        launch_integrate_jobs(s.ctx, s.launch, jobs, st, e0, e1);
        AsmCounters c{};
        NLQ_HIP(hipMemcpyAsync(&c, s.counters.as<void>(), sizeof(AsmCounters), hipMemcpyDeviceToHost, st));
        NLQ_HIP(hipStreamSynchronize(st));
        float ms = 0.0f;
        NLQ_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        check_counter_error(c.error);
        if (kernel_s) *kernel_s = 1e-3 * ms;
        if (n_leaf)
            for (int q = 0; q < 9; ++q) n_leaf[q] = (q >= 1 && q <= 8) ? static_cast<int64_t>(c.leaf[q]) : 0;
        if (n_leaf_zero) *n_leaf_zero = static_cast<int64_t>(c.zero_leaves);
        s.has_rhs = false;
    });
}

nlq_status nlq_integrate_range(nlq_system *sys, int64_t lo, int64_t hi, double *kernel_s, int64_t *n_leaf)
{
    return nlq_integrate_ranges(sys, 1, &lo, &hi, kernel_s, n_leaf, nullptr);
}

nlq_status nlq_assemble_batch(nlq_ctx *ctx, int32_t n, const nlq_mesh *const *meshes, const nlq_params *params,
                              nlq_system **out)
{
    std::vector<std::unique_ptr<nlq_system>> made;
    return guard([&] {
        if (!ctx || n < 0 || (n > 0 && (!meshes || !params || !out))) fail(NLQ_EINVAL, "NULL argument");
        for (int32_t i = 0; i < n; ++i) {
            if (!meshes[i]) fail(NLQ_EINVAL, "NULL mesh");
            if (meshes[i]->impl.ctx != &ctx->impl) fail(NLQ_EINVAL, "mesh belongs to another context");
        }
        NLQ_HIP(hipSetDevice(ctx->impl.device));
        hipStream_t st = ctx->impl.stream;
        for (int32_t i = 0; i < n; ++i) made.push_back(prepare_system(ctx->impl, meshes[i]->impl, params[i], st));
        // one group per (dim, precision, kernel); up to 32 systems per launch
        std::vector<int> order(n);
        for (int i = 0; i < n; ++i) order[i] = i;
        // (a deterministic system is a group of its own)
        auto key = [&](int i) {
            const System &s = made[i]->impl;
            return std::make_tuple(s.mesh->dim, s.p.precision, s.p.kernel, s.p.deterministic ? i + 1 : 0);
        };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key(x) < key(y); });
        LaunchBlock lb;
        hipEvent_t e0, e1;
        NLQ_HIP(hipEventCreate(&e0));
        NLQ_HIP(hipEventCreate(&e1));
        for (size_t g0 = 0; g0 < order.size();) {
            size_t g1 = g0;
            std::vector<IntegrateJob> jobs;
            while (g1 < order.size() && key(order[g1]) == key(order[g0]) && jobs.size() < 32) {
                System &s = made[order[g1]]->impl;
                jobs.push_back(IntegrateJob{&s, 0, s.mesh->n_elems});
                ++g1;
            }
            const double t0 = now_s();
            if (jobs.size() == 1 && jobs[0].s->p.deterministic) launch_integrate(*jobs[0].s, st, e0, e1);
            else launch_integrate_jobs(&ctx->impl, lb, jobs, st, e0, e1);
            NLQ_HIP(hipStreamSynchronize(st));
            const double t1 = now_s();
            float ms = 0.0f;
            NLQ_HIP(hipEventElapsedTime(&ms, e0, e1));
            for (auto &j : jobs) {
                collect_counters(*j.s, st);
                j.s->info.t_integrate = t1 - t0;
                j.s->info.t_kernel = 1e-3 * ms;
                j.s->info.t_total = j.s->info.t_tables + j.s->info.t_pairs + j.s->info.t_pattern + (t1 - t0);
            }
            g0 = g1;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        for (int32_t i = 0; i < n; ++i) out[i] = made[i].release();
    });
}

nlq_status nlq_autotune(nlq_system *sys, double budget_s, nlq_tune_info *info)
{
    return guard([&] {
        if (!sys) fail(NLQ_EINVAL, "sys is NULL");
        System &s = sys->impl;
        NLQ_HIP(hipSetDevice(s.ctx->device));
        double best = 0.0, def = 0.0;
        const int n = autotune(s, s.ctx->stream, budget_s > 0.0 ? budget_s : 2.0, &best, &def);
        s.has_rhs = false;
        if (info) {
            info->occupancy_variant = s.cfg.occ;
            info->workgroups_per_cu = static_cast<int32_t>(integrate_slots(s.ctx, s) / std::max(s.ctx->n_cu, 1));
            info->pairs_per_item = s.cfg.pairs_per_item;
            info->work_items_per_element = integrate_split(s);
            info->stack_capacity = s.cfg.stack_cap;
            info->leaf_capacity = s.cfg.leaf_cap;
            info->candidates = n;
            info->best_ms = best;
            info->default_ms = def;
        }
    });
}

nlq_status nlq_tune_save(const nlq_ctx *ctx, const char *path)
{
    return guard([&] {
        if (!ctx || !path) fail(NLQ_EINVAL, "NULL argument");
        const Ctx &c = ctx->impl;
        std::string text =
            "# nlq tuning cache v2: arch dim element precision kernel lmax size_class occ wg_per_cu pairs_per_item "
            "stack_cap leaf_cap\n";
        {
            std::lock_guard<std::mutex> g(const_cast<Ctx &>(c).tune_mu);
            for (const auto &kv : c.tuned) {
                const TuneKey &k = kv.first;
                const TuneConfig &t = kv.second;
                const int fields[] = {std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                                      std::get<4>(k), std::get<5>(k), t.occ, t.wg_per_cu, t.pairs_per_item,
                                      t.stack_cap, t.leaf_cap};
                text += c.arch;
                for (int v : fields) text += " " + std::to_string(v);
                text += "\n";
            }
        }
        FILE *f = std::fopen(path, "w");
        if (!f) fail(NLQ_EINVAL, std::string("cannot open ") + path);
        const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
        if (std::fclose(f) != 0 || !ok) fail(NLQ_EINVAL, std::string("cannot write ") + path);
    });
}

nlq_status nlq_tune_load(nlq_ctx *ctx, const char *path, int32_t *n_loaded)
{
    return guard([&] {
        if (!ctx || !path) fail(NLQ_EINVAL, "NULL argument");
        FILE *f = std::fopen(path, "r");
        if (!f) fail(NLQ_EINVAL, std::string("cannot open ") + path);
        std::vector<std::pair<TuneKey, TuneConfig>> got;
        char line[512];
        int lineno = 0;
        bool bad = false;
        while (std::fgets(line, sizeof line, f)) {
            ++lineno;
            if (line[0] == '#' || line[0] == '\n' || line[0] == '\0') continue;
            // v2 lines: arch and 11 fields; v1 lines (P1 only, default capacities):
            // arch dim precision kernel lmax size_class occ wg_per_cu pairs_per_item
            char arch[64];
            int v[11];
            const int got_n = std::sscanf(line, "%63s %d %d %d %d %d %d %d %d %d %d %d", arch, &v[0], &v[1], &v[2],
                                          &v[3], &v[4], &v[5], &v[6], &v[7], &v[8], &v[9], &v[10]);
            int dim, order = 1, prec, kernel, lmax, lg;
            TuneConfig t;
            if (got_n == 12) {
                dim = v[0], order = v[1], prec = v[2], kernel = v[3], lmax = v[4], lg = v[5];
                t.occ = v[6], t.wg_per_cu = v[7], t.pairs_per_item = v[8], t.stack_cap = v[9], t.leaf_cap = v[10];
            } else if (got_n == 9) {
                dim = v[0], prec = v[1], kernel = v[2], lmax = v[3], lg = v[4];
                t.occ = v[5], t.wg_per_cu = v[6], t.pairs_per_item = v[7];
            } else {
                bad = true;
                break;
            }
            if ((dim != 2 && dim != 3) || order < 1 || order > 4 || (prec != 0 && prec != 1) ||
                (t.occ != 0 && t.occ != 1) || t.wg_per_cu < 0 || t.pairs_per_item < 1 || lmax < 1 || lg < 0 ||
                t.stack_cap < 64 || t.stack_cap > 1024 || t.leaf_cap < 64 || t.leaf_cap > 512) {
                bad = true;
                break;
            }
            if (ctx->impl.arch != arch) continue;
            got.emplace_back(TuneKey(dim, order, prec, kernel, lmax, lg), t);
        }
        std::fclose(f);
        if (bad) fail(NLQ_EINVAL, std::string(path) + ": line " + std::to_string(lineno) + " does not parse");
        {
            std::lock_guard<std::mutex> g(ctx->impl.tune_mu);
            for (const auto &kv : got) ctx->impl.tuned[kv.first] = kv.second;
        }
        if (n_loaded) *n_loaded = static_cast<int32_t>(got.size());
    });
}

nlq_status nlq_assemble_info_get(const nlq_system *sys, nlq_assemble_info *info)
{
    return guard([&] {
        if (!sys || !info) fail(NLQ_EINVAL, "NULL argument");
        *info = sys->impl.info;
    });
}

nlq_status nlq_reassemble(nlq_system *sys)
{
    return guard([&] {
        if (!sys) fail(NLQ_EINVAL, "sys is NULL");
        NLQ_HIP(hipSetDevice(sys->impl.ctx->device));
        run_integrate(sys->impl, sys->impl.ctx->stream);
        sys->impl.has_rhs = false;
    });
}

nlq_status nlq_set_data(nlq_system *sys, const double *f_nodal, const double *g_nodal)
{
    return guard([&] {
        if (!sys || !f_nodal || !g_nodal) fail(NLQ_EINVAL, "NULL argument");
        NLQ_HIP(hipSetDevice(sys->impl.ctx->device));
        load_data(sys->impl, f_nodal, g_nodal, sys->impl.ctx->stream);
    });
}

nlq_status nlq_set_data_device(nlq_system *sys, const double *f_dev, const double *g_dev)
{
    return guard([&] {
        if (!sys || !f_dev || !g_dev) fail(NLQ_EINVAL, "NULL argument");
        System &s = sys->impl;
        NLQ_HIP(hipSetDevice(s.ctx->device));
        const int64_t n = s.mesh->n_nodes;
        hipStream_t st = s.ctx->stream;
        if (s.g.empty()) s.g.alloc(s.ctx, sizeof(double) * n);
        NLQ_HIP(hipMemcpyAsync(s.g.as<void>(), g_dev, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        launch_load_lift(s, st, f_dev, s.g.as<double>());
        NLQ_HIP(hipStreamSynchronize(st));
        s.has_rhs = true;
    });
}

nlq_status nlq_solution_device(const nlq_system *sys, const double **u_dev)
{
    return guard([&] {
        if (!sys || !u_dev) fail(NLQ_EINVAL, "NULL argument");
        *u_dev = sys->impl.u.empty() ? nullptr : sys->impl.u.as<double>();
    });
}

nlq_status nlq_solve(nlq_system *sys, double rtol, int32_t maxit, double *u_out, nlq_solve_info *info)
{
    bool converged = true;
    nlq_status st = guard([&] {
        if (!sys) fail(NLQ_EINVAL, "sys is NULL");
        NLQ_HIP(hipSetDevice(sys->impl.ctx->device));
        converged = solve_system(sys->impl, rtol, maxit, u_out, info, sys->impl.ctx->stream);
    });
    if (st == NLQ_OK && !converged) {
        set_last_error("CG did not reach the tolerance");
        return NLQ_ENOCONV;
    }
    return st;
}

nlq_status nlq_solve_noalloc(nlq_system *sys, double rtol, int32_t maxit, double *u_dev, nlq_solve_info *info)
{
    bool converged = true;
    nlq_status st = guard([&] {
        if (!sys || !u_dev) fail(NLQ_EINVAL, "NULL argument");
        System &s = sys->impl;
        if (!s.has_rhs) fail(NLQ_EINVAL, "nlq_set_data must be called before nlq_solve_noalloc");
        if (s.p.form != NLQ_FORM_SYM4)
            fail(NLQ_EINVAL, "nlq_solve_noalloc runs CG: four-term form only (the two-term forms need nlq_solve)");
        if (!(rtol > 0.0) || maxit < 1) fail(NLQ_EINVAL, "need rtol > 0 and maxit >= 1");
        NLQ_HIP(hipSetDevice(s.ctx->device));
        const double t0 = now_s();
        double relres = 0.0;
        int conv = 0;
        const int it = cg_solve_noalloc(s, s.ctx->stream, rtol, maxit, &relres, &conv, u_dev);
        if (info) {
            info->iterations = it;
            info->converged = conv;
            info->rel_residual = relres;
            info->seconds = now_s() - t0;
        }
        converged = conv != 0;
    });
    if (st == NLQ_OK && !converged) {
        set_last_error("CG did not reach the tolerance");
        return NLQ_ENOCONV;
    }
    return st;
}

nlq_status nlq_info(const nlq_system *sys, int64_t *n_rows, int64_t *nnz, int64_t *n_pairs,
                    int64_t *n_free)
{
    return guard([&] {
        if (!sys) fail(NLQ_EINVAL, "sys is NULL");
        if (n_rows) *n_rows = sys->impl.mesh->n_nodes;
        if (nnz) *nnz = sys->impl.nnz;
        if (n_pairs) *n_pairs = sys->impl.n_pairs;
        if (n_free) *n_free = sys->impl.mesh->n_free;
    });
}

nlq_status nlq_csr_copy(const nlq_system *sys, int64_t *row_ptr, int32_t *col, double *val)
{
    return guard([&] {
        if (!sys) fail(NLQ_EINVAL, "sys is NULL");
        const System &s = sys->impl;
        NLQ_HIP(hipSetDevice(s.ctx->device));
        NLQ_HIP(hipStreamSynchronize(s.ctx->stream));
        const int64_t n = s.mesh->n_nodes;
        if (row_ptr)
            NLQ_HIP(hipMemcpy(row_ptr, s.row_ptr.as<void>(), sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
        if (col) NLQ_HIP(hipMemcpy(col, s.col.as<void>(), sizeof(int32_t) * s.nnz, hipMemcpyDeviceToHost));
        if (val) NLQ_HIP(hipMemcpy(val, s.val.as<void>(), sizeof(double) * s.nnz, hipMemcpyDeviceToHost));
    });
}

nlq_status nlq_csr_device(const nlq_system *sys, const int64_t **row_ptr, const int32_t **col,
                          const double **val)
{
    return guard([&] {
        if (!sys) fail(NLQ_EINVAL, "sys is NULL");
        if (row_ptr) *row_ptr = sys->impl.row_ptr.as<int64_t>();
        if (col) *col = sys->impl.col.as<int32_t>();
        if (val) *val = sys->impl.val.as<double>();
    });
}

nlq_status nlq_pairs_copy(const nlq_system *sys, int64_t *offsets, int32_t *m)
{
    return guard([&] {
        if (!sys) fail(NLQ_EINVAL, "sys is NULL");
        const System &s = sys->impl;
        NLQ_HIP(hipSetDevice(s.ctx->device));
        NLQ_HIP(hipStreamSynchronize(s.ctx->stream));
        if (offsets)
            NLQ_HIP(hipMemcpy(offsets, s.pair_off.as<void>(), sizeof(int64_t) * (s.mesh->n_elems + 1),
                              hipMemcpyDeviceToHost));
        if (m) NLQ_HIP(hipMemcpy(m, s.pair_m.as<void>(), sizeof(int32_t) * s.n_pairs, hipMemcpyDeviceToHost));
    });
}

nlq_status nlq_rhs_copy(const nlq_system *sys, double *f_tilde)
{
    return guard([&] {
        if (!sys || !f_tilde) fail(NLQ_EINVAL, "NULL argument");
        const System &s = sys->impl;
        if (!s.has_rhs) fail(NLQ_EINVAL, "nlq_set_data has not been called");
        NLQ_HIP(hipSetDevice(s.ctx->device));
        NLQ_HIP(hipStreamSynchronize(s.ctx->stream));
        NLQ_HIP(hipMemcpy(f_tilde, s.Ft.as<void>(), sizeof(double) * s.mesh->n_nodes, hipMemcpyDeviceToHost));
    });
}

nlq_status nlq_pair_blocks(nlq_system *sys, int64_t n, const int32_t *l, const int32_t *m, double *out)
{
    return guard([&] {
        if (!sys || (n > 0 && (!l || !m || !out))) fail(NLQ_EINVAL, "NULL argument");
        if (n <= 0) return;
        System &s = sys->impl;
        const int64_t ne = s.mesh->n_elems;
        for (int64_t k = 0; k < n; ++k)
            if (l[k] < 0 || l[k] >= ne || m[k] < 0 || m[k] >= ne) fail(NLQ_EINVAL, "element id out of range");
        if (n > (1ll << 30)) fail(NLQ_EINVAL, "too many pairs");
        NLQ_HIP(hipSetDevice(s.ctx->device));
        hipStream_t st = s.ctx->stream;
        const int nv = s.mesh->nb;
        const size_t blk = static_cast<size_t>(4 * nv * nv);
        DevBuf dl(s.ctx, sizeof(int32_t) * n), dm(s.ctx, sizeof(int32_t) * n),
            dout(s.ctx, sizeof(double) * n * blk);
        NLQ_HIP(hipMemcpyAsync(dl.as<void>(), l, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
        NLQ_HIP(hipMemcpyAsync(dm.as<void>(), m, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
        NLQ_HIP(hipMemsetAsync(s.counters.as<void>(), 0, sizeof(AsmCounters), st));
        launch_pair_blocks(s, st, n, dl.as<int32_t>(), dm.as<int32_t>(), dout.as<double>());
        AsmCounters c{};
        NLQ_HIP(hipMemcpyAsync(out, dout.as<void>(), sizeof(double) * n * blk, hipMemcpyDeviceToHost, st));
        NLQ_HIP(hipMemcpyAsync(&c, s.counters.as<void>(), sizeof(AsmCounters), hipMemcpyDeviceToHost, st));
        NLQ_HIP(hipStreamSynchronize(st));
        check_counter_error(c.error);
    });
}

nlq_status nlq_system_destroy(nlq_system *sys)
{
    return guard([&] {
        if (!sys) return;
        (void)hipSetDevice(sys->impl.ctx->device);
        (void)hipStreamSynchronize(sys->impl.ctx->stream);
        delete sys;
    });
}

}  // extern "C"
