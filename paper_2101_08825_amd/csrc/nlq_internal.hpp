// Internal runtime structures of libnlq (host side).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "nlq.h"

struct nlq_system;
struct nlq_mesh;

namespace nlq {

struct Error {
    nlq_status status;
    std::string msg;
};

[[noreturn]] void fail(nlq_status st, const std::string &msg);
void set_last_error(const std::string &msg);

#define NLQ_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            ::nlq::fail(NLQ_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define NLQ_CHECK_LAUNCH() NLQ_HIP(hipGetLastError())

struct Ctx;

// Device allocation charged against the context budget.  With a stream the
// allocation is stream ordered (hipMallocAsync / hipFreeAsync on that stream),
// so that freeing a temporary does not wait for the whole device; the stream
// must outlive the buffer.  Without one the block comes from the context's
// cache of released blocks of its size class when there is one (hipMalloc
// otherwise), and goes back there on release, after the device has finished
// all work (what hipFree would wait for).
class DevBuf {
  public:
    DevBuf() = default;
    DevBuf(Ctx *ctx, size_t bytes, hipStream_t st = nullptr) { alloc(ctx, bytes, st); }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p_ = o.p_;
            bytes_ = o.bytes_;
            ctx_ = o.ctx_;
            st_ = o.st_;
            cls_ = o.cls_;
            o.p_ = nullptr;
            o.bytes_ = 0;
            o.cls_ = 0;
        }
        return *this;
    }
    void alloc(Ctx *ctx, size_t bytes, hipStream_t st = nullptr);
    void release();
    template <class T> T *as() const { return reinterpret_cast<T *>(p_); }
    size_t bytes() const { return bytes_; }
    bool empty() const { return p_ == nullptr; }

  private:
    void *p_ = nullptr;
    size_t bytes_ = 0;
    size_t cls_ = 0;   // size class charged and cached (no stream)
    Ctx *ctx_ = nullptr;
    hipStream_t st_ = nullptr;
};

// Quadrature rule and refinement tables for one (dim, lmax): the degree-5 rule
// on the reference simplex and, for every sub-element of Algorithm 1's
// midpoint refinement up to lmax, the barycentric coordinates (w.r.t. the root
// element) of its quadrature points.
struct Tables {
    int dim = 0, lmax = 0, nq = 0, nv = 0;
    std::vector<double> bary;   // [nq][nv]
    std::vector<double> w;      // [nq], sum 1
    std::vector<int64_t> lvl_off;  // [lmax+2] first sub index of each level (level 1 at 0)
    int64_t n_sub = 0;
    DevBuf rule;                // [nq][nv] points, then [nq] weights (double)
    DevBuf lam64;               // [n_sub][nq][nv] double
    // per quadrature point of every sub-element, the FP32 rows of the
    // contraction (w lambda_i, then w lambda_i lambda_j, i < j; w the rule weight
    // scaled by the level's volume ratio) and lambda_1..lambda_dim:
    // [n_sub*nq + 1][8 (2D) or 16 (3D)], the last row zero (lanes without a point)
    DevBuf pt32;
    // P2 elements: the monomial rows -> epilogue rows map of make_p2_map (double)
    DevBuf p2map;
    // quadrilaterals / hexahedra (make_box_tables), per element order o = 1, 2:
    // the 3^N rule ([nq][dim] points, then [nq] weights), and per order the basis
    // at the rule points [nb][qs] (qs = 16 in 2D, 32 in 3D; padding zero), the
    // basis functions and their products over the product monomials
    // [nb][nr] and [nu][nr] (double)
    DevBuf boxrule;
    DevBuf boxpsi[2], boxphi[2], boxprod[2];
};

struct Server;

// Launch configuration of the integration kernel (chosen by nlq_autotune).
struct TuneConfig {
    int occ = 0;               // register budget: 0 = default, 1 = one wave more (2D FP32) / fewer (others)
    int wg_per_cu = 0;         // persistent workgroups per CU (0 = as many as fit)
    int pairs_per_item = 512;  // largest part of one J_l handled as one work item
    int stack_cap = 128;       // logical traversal stack entries per wave (64 .. 1024)
    int leaf_cap = 128;        // leaf buffer entries per wave (64 .. 512)
};
// dim, element order, precision, kernel, lmax, ceil(log2(max |J_l|))
using TuneKey = std::tuple<int, int, int, int, int, int>;

struct Ctx {
    int device = 0;
    int n_cu = 0;
    std::string arch;                  // e.g. gfx950 (keys the saved tuning cache)
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};
    // failure injection for tests: the device allocation with this ordinal
    // (counted per context from 0) fails with NLQ_ENOMEM; -1: none
    std::atomic<int64_t> allocs{0};
    int64_t alloc_fail_at = -1;
    // released device blocks by size class, kept for reuse (a step that builds
    // and frees the same systems again then maps no memory); live + cached
    // bytes stay within the budget, cached bytes within kCacheMax
    static constexpr uint64_t kCacheMax = 8ull << 30;
    std::mutex cache_mu;
    std::multimap<size_t, void *> cache;
    uint64_t cached = 0;
    void *cache_take(size_t cls);
    void cache_put(void *p, size_t cls);
    void cache_trim(uint64_t need);   // free cached blocks until used + cached + need <= budget
    std::mutex tables_mu;
    std::map<std::pair<int, int>, std::unique_ptr<Tables>> tables;
    std::unique_ptr<Server> server;
    std::mutex tune_mu;
    std::map<TuneKey, TuneConfig> tuned;
    const Tables &get_tables(int dim, int lmax);
    Ctx();
    ~Ctx();
};

struct Mesh {
    Ctx *ctx = nullptr;
    int dim = 0;
    int64_t n_nodes = 0, n_elems = 0, n_free = 0;
    double gmin[3] = {0, 0, 0}, gmax[3] = {0, 0, 0};
    double ext_max[3] = {0, 0, 0};   // largest element bbox extent per axis
    DevBuf coords;                   // [n_nodes][dim] double
    int shape = 0;                   // 0: simplices; 1: quadrilaterals / hexahedra (tensor order)
    int order = 1;                   // 1: P1 / Q1; 2: P2 / serendipity (then the edge midpoints)
    int nb = 0;                      // nodes per element: dim + 1 (P1), (dim+1)(dim+2)/2 (P2),
                                     // 2^dim (Q1), 8 / 20 (serendipity)
    int ngeo = 0;                    // geometric vertices: dim + 1, or the 2^dim corners
    DevBuf conn;                     // [n_elems][nb] int32
    DevBuf constrained;              // [n_nodes] uint8
    std::vector<double> h_coords;
    std::vector<int32_t> h_conn;
    std::vector<uint8_t> h_constrained;
};

struct AsmCounters {
    unsigned long long leaf[9];
    unsigned long long zero_leaves;   // leaves at L_max counted but not integrated (all-zero integrals)
    unsigned long long pairs_done;
    int error;   // kErr* bits
    int pad;
};
// error bits of an integration launch
constexpr int kErrStack = 1;     // a refinement traversal would have passed its stack
constexpr int kErrPattern = 2;   // a block entry fell outside the CSR pattern

// throws NLQ_EDEVICE naming every bit set in `error` (no-op for 0)
void check_counter_error(int error);

// Pinned host + device staging of a launch's argument block.  The host side is
// rewritten by the next launch, so a caller synchronises the stream in between.
struct LaunchBlock {
    DevBuf dev;
    void *host = nullptr;
    size_t cap = 0;
    void ensure(Ctx *ctx, size_t bytes);
    LaunchBlock() = default;
    LaunchBlock(const LaunchBlock &) = delete;
    LaunchBlock &operator=(const LaunchBlock &) = delete;
    ~LaunchBlock();
};

struct System {
    Ctx *ctx = nullptr;
    const Mesh *mesh = nullptr;
    nlq_params p{};
    double C = 0.0;              // kernel constant
    int64_t n_pairs = 0, nnz = 0, max_row = 0;
    int64_t max_pairs = 0;       // largest |J_l|
    // element tables
    DevBuf vert;                 // [nv*dim][ne] SoA double
    DevBuf lo, hi;               // [dim][ne]
    DevBuf qlo, qhi;             // [dim][ne] box of the element's quadrature points
    DevBuf meas;                 // [ne]
    // pair list
    DevBuf pair_off;             // [ne+1] int64
    DevBuf pair_m;               // [n_pairs] int32
    // pattern
    DevBuf row_ptr;              // [n+1] int64
    DevBuf col;                  // [nnz] int32
    DevBuf tmap;                 // [nnz] int32: position of the transposed entry
    DevBuf elpos;                // [ne][nv*nv] int32: positions of the element's own block
    DevBuf val;                  // [nnz] double
    DevBuf dmm;                  // [ne][NR] double: upper-triangle diagonal-block sums per element
    // rhs / solution
    DevBuf F, Ft, u, g;          // [n] double
    DevBuf counters;             // AsmCounters
    // deterministic mode: node -> elements (ascending), element row offsets, and
    // the per-pair output buffer of the slab being integrated
    DevBuf n2e_off, n2e, eoff;
    double *det_pb = nullptr;
    int64_t det_pb_base = 0;
    LaunchBlock launch;          // argument block of this system's own launches
    TuneConfig cfg;              // integration launch configuration
    nlq_assemble_info info{};
    bool has_rhs = false;
    bool integrated = false;     // the values hold a whole integration (not a prepared system)
    std::vector<double> h_g;
};

// kernels launched from the runtime (defined in the .hip files)
// Assembly steps of the runtime (nlq_capi.cpp): everything up to the
// integration (returns with st synchronised), the counters of a finished
// integration into info, and both plus the system's own integration launch.
std::unique_ptr<nlq_system> prepare_system(Ctx &ctx, const Mesh &mesh, const nlq_params &params, hipStream_t st);
void collect_counters(System &s, hipStream_t st);
void run_integrate(System &s, hipStream_t st);
// Kuhn box mesh built on the device (st synchronised on return).
std::unique_ptr<nlq_mesh> make_box_mesh(Ctx &ctx, int dim, int n, int k_gamma, hipStream_t st);
// Nodal f, g (host) -> F~ of the system (st synchronised on return).
void load_data(System &s, const double *f_nodal, const double *g_nodal, hipStream_t st);
// CG on the free rows; u copied to u_out (host) when given.  Returns convergence.
bool solve_system(System &s, double rtol, int maxit, double *u_out, nlq_solve_info *info, hipStream_t st);

void launch_elem_tables(System &s, hipStream_t st);
void build_pairs(System &s, hipStream_t st);
void build_pattern(System &s, hipStream_t st);
// Outer elements [lo, hi) of system s (each cut into integrate_split(s) work
// items of at most 512 pairs).  One launch takes up to 32 ranges of
// systems of one dimension, precision and kernel; a range starting at 0 clears
// the system's values first, a range ending at n_elems finishes its matrix.
struct IntegrateJob {
    System *s;
    int64_t lo, hi;
};
void launch_integrate_jobs(Ctx *ctx, LaunchBlock &lb, const std::vector<IntegrateJob> &jobs, hipStream_t st,
                           hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
void launch_integrate(System &s, hipStream_t st, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// deterministic mode (nlq_params.deterministic): the whole integration with
// fixed-order sums (nlq_det.hip); launch_integrate calls it for such systems
void integrate_deterministic(System &s, hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop);
// A = R + R^T in place (four-term form)
void launch_symmetrize(const System &s, hipStream_t st);
// resident workgroups of one integration launch of s, and work items per outer element
int64_t integrate_slots(Ctx *ctx, const System &s);
int integrate_split(const System &s);
// key of the tuned configuration of a system, and the configuration to use
TuneKey tune_key(const System &s);
TuneConfig tuned_config(Ctx &ctx, const System &s);
// time candidate configurations on a sample of s's outer elements (about
// budget_s in total), keep the fastest in ctx and in s; s's values are
// recomputed with it.  Returns the configurations timed and the two times.
int autotune(System &s, hipStream_t st, double budget_s, double *best_ms, double *default_ms);
void launch_pair_blocks(System &s, hipStream_t st, int64_t n, const int32_t *ex_l, const int32_t *ex_m,
                        double *ex_out);
void launch_load_lift(System &s, hipStream_t st, const double *f_dev, const double *g_dev);
int cg_solve(System &s, hipStream_t st, double rtol, int maxit, double *relres, int *converged);
int bicgstab_solve(System &s, hipStream_t st, double rtol, int maxit, double *relres, int *converged);
// the allocation-free solve: CG vectors in the library's static device scratch
// (address taken per device by noalloc_scratch_init), plain launches, u into u_dev
void noalloc_scratch_init(int device);
size_t noalloc_scratch_limit();
int cg_solve_noalloc(System &s, hipStream_t st, double rtol, int maxit, double *relres, int *converged,
                     double *u_dev);
void launch_box_mesh(int dim, int n, int k_gamma, double *coords, int32_t *conn,
                     uint8_t *constrained, hipStream_t st);

void exclusive_scan_i64(Ctx *ctx, const int64_t *in, int64_t *out, int64_t n, hipStream_t st);

double kernel_constant(int dim, int kernel, double delta, double eps);
std::unique_ptr<Tables> make_tables(Ctx *ctx, int dim, int lmax);
std::vector<double> make_p2_map(int dim);
struct BoxTablesHost {
    std::vector<double> rule, psi, phi, prod;
};
BoxTablesHost make_box_tables(int dim, int order);

}  // namespace nlq

struct nlq_ctx {
    nlq::Ctx impl;
};
struct nlq_mesh {
    nlq::Mesh impl;
};
struct nlq_system {
    nlq::System impl;
};
