/*
 * nlq -- mollified nonlocal finite-element assembly and solve on one AMD MI355X
 * (gfx950), after Aulisa, Capodaglio, Chierici, D'Elia, "Efficient quadrature
 * rules for finite element discretizations of nonlocal equations"
 * (arXiv 2101.08825).
 *
 * Problem (Section 2, eqs. (poisson), (A-F); Section 3, eqs. (approx-kernel),
 * (mollifier), (Aeps)): find u with u = g on the interaction layer Gamma and
 *     A_eps(u, phi) = int_Omega f phi   for every P1 test function phi
 * vanishing on Gamma, where
 *     A_eps(u, phi) = iint (u(y)-u(x)) (phi(y)-phi(x)) gamma_eps(x, y) dy dx,
 *     gamma_eps = C eta(|x-y|) mu_{delta,eps}(|x-y|),
 * and mu is the C^4 mollifier that replaces the indicator of the ball B_delta
 * (band of width 2 eps around |x-y| = delta).  The stiffness entries
 * (Section 4, eq. (Aij-support2)) are summed over ordered element pairs (l, m)
 * within the horizon (Section 5, eq. (k_l) with the bbox distance of eq.
 * (mindist)); each pair is integrated with the adaptive outer quadrature of
 * Algorithm 1 (Section 5) and a fixed Gauss rule on the inner element.
 *
 * Conventions
 *  - Every call returns nlq_status: 0 = OK, < 0 = error; nothing aborts.  The
 *    message of the last error of the calling thread is nlq_last_error().
 *  - Arrays are 0-based and row-major.  Ids are int32, counts int64, physical
 *    data double.  "host" pointers are CPU memory; "device" pointers are HBM.
 *  - The library copies every input it keeps.  Outputs are either copied into
 *    caller-owned buffers (nlq_*_copy) or borrowed device pointers valid until
 *    the owning handle is destroyed (nlq_csr_device).
 *  - Handles are not thread-safe, except nlq_submit / nlq_wait / nlq_cancel /
 *    nlq_result_release, which may be called from any thread.
 *  - All device work of a context runs on the context's HIP stream (a stream
 *    of its own unless nlq_ctx_set_stream was called); calls that return host
 *    data synchronise that stream.
 */
#ifndef NLQ_H
#define NLQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NLQ_OK = 0,
    NLQ_EINVAL = -1,      /* bad argument (message in nlq_last_error) */
    NLQ_ENOMEM = -2,      /* would exceed the context's HBM budget, or allocation failed */
    NLQ_EDEVICE = -3,     /* HIP runtime error */
    NLQ_ENOTREADY = -4,   /* nlq_wait timed out */
    NLQ_ECANCELLED = -5,  /* request was cancelled */
    NLQ_EBUSY = -6,       /* queue full */
    NLQ_ENOCONV = -7      /* CG did not reach the tolerance; u holds the last iterate */
} nlq_status;

enum { NLQ_ETA_CONST = 0, NLQ_ETA_GAUSS = 1 };
enum { NLQ_FORM_SYM4 = 0, NLQ_FORM_PAPER2 = 1, NLQ_FORM_PAPER2_INNER = 2 };
enum { NLQ_FP64_PLAIN = 0, NLQ_FP32_MIXED = 1 };

typedef struct nlq_ctx nlq_ctx;
typedef struct nlq_mesh nlq_mesh;
typedef struct nlq_system nlq_system;

/* Method parameters.
 *  dim        2 (P1 triangles) or 3 (P1 tetrahedra); must match the mesh.
 *  kernel     NLQ_ETA_CONST: eta = 1.  NLQ_ETA_GAUSS: eta = exp(-|x-y|^2/delta^2).
 *  delta, eps horizon and mollifier half-width, 0 < eps < delta (Section 3).
 *  scale      > 0: use as the kernel constant C.  0: C_{delta,eps} of Section 6
 *             (eta = 1; kappa = 1), or for the Gaussian the constant c with
 *             c omega_N int rho^{N+1} eta mu = N, i.e. L_eps u = Laplacian u for
 *             quadratic u (the same normalisation).
 *  lmin, lmax Algorithm 1 levels, 1 <= lmin <= lmax <= 8 (2D) / 6 (3D).
 *  form       NLQ_FORM_SYM4: four-term integrand of eq. (Aij-support2) per
 *             ordered pair (exactly symmetric, zero row sums).  NLQ_FORM_PAPER2:
 *             2 A21 + 2 A22 of the Corollary in Section 5 (rows of the inner
 *             test function; zero row sums, symmetric only in the limit).
 *             NLQ_FORM_PAPER2_INNER: the same two-term form with the adaptive
 *             rule on the inner integral instead of the outer one (Section 5
 *             calls the choice empirical): every element is refined against
 *             its J_l and carries the rows, 2 B_ll and 2 B_lm, which summed over
 *             the symmetric pair list is the adaptive-inner assembly.  Not
 *             available with deterministic = 1.
 *  precision  NLQ_FP64_PLAIN: FP64 kernel evaluation and contraction.
 *             NLQ_FP32_MIXED: FP32 evaluation at anchor-relative coordinates,
 *             FP32 matrix-core contraction per 64-point batch, FP64 per-pair
 *             blocks and FP64 global accumulation.
 *  deterministic  0: the per-pair blocks are added to the matrix with FP64
 *             atomics (the order of additions, and so the last bits of the
 *             values, vary from run to run).  1: fixed-order sums (each pair's
 *             block is stored, then every entry sums its contributions in
 *             element and pair-list order), so the matrix is the same bit for
 *             bit from run to run and however launches are shared; slower, and
 *             it needs about (N+1)^2 + (N+1)(N+2) doubles per pair of a slab of
 *             up to 8M pairs plus one double per entry and element of its
 *             node.  Such a system is integrated by itself: nlq_integrate_range
 *             rejects it, nlq_assemble_batch and the serving loop integrate it
 *             alone, nlq_autotune leaves it untuned.
 *  min_dist_l2  0: Algorithm 1's refine test uses the L_inf box gap of Section
 *             5.1, eq. (mindist) (the paper).  1: the Euclidean box gap
 *             (an ablation): a sub-element whose box is at least delta + eps
 *             from the inner element's box holds no point pair within the
 *             kernel's support, so dropping it removes only zero contributions
 *             -- the same matrix to round-off from fewer leaves.  2: the
 *             Euclidean gap to the box of the inner element's quadrature
 *             points instead (a tighter test of our own, same argument: every
 *             inner point lies in that box), fewer leaves still.  The J^int
 *             test and the pair list J_l keep the paper's form either way.
 */
typedef struct {
    int32_t dim;
    int32_t kernel;
    double delta, eps;
    double scale;
    int32_t lmin, lmax;
    int32_t form;
    int32_t precision;
    int32_t deterministic;
    int32_t min_dist_l2;
} nlq_params;

/* Counts and stage timings of one assembly (seconds from HIP events). */
typedef struct {
    int64_t n_pairs;          /* ordered element pairs (l, m), m in J_l */
    int64_t n_leaf[9];        /* Integration(s, m) calls per level 1..8 (index = level) */
    int64_t n_evals;          /* kernel evaluations gamma_eps(x_a, y_b) of those calls */
    int64_t nnz;
    double t_tables, t_pairs, t_pattern, t_integrate, t_total;  /* host wall clock */
    double t_kernel;          /* integration kernel alone, HIP events on its stream */
    int64_t n_leaf_zero;      /* of the calls at L_max, those not evaluated: the box of the
                                 sub-element lies at Euclidean distance >= delta + eps from
                                 the box of m's quadrature points, so every term is zero */
} nlq_assemble_info;

typedef struct {
    int32_t iterations;
    int32_t converged;
    double rel_residual;      /* ||r||_2 / ||F~||_2 at exit */
    double seconds;
} nlq_solve_info;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the context may hold (0 = 90% of the device's free memory).
 * For failure-path tests, the environment variable NLQ_FAIL_ALLOC_AT=k (read
 * here) makes the k-th device allocation of this context (counted from 0)
 * fail once with NLQ_ENOMEM. */
nlq_status nlq_ctx_create(int32_t device, uint64_t hbm_budget_bytes, nlq_ctx **out);
/* Run all later device work of this context on `hip_stream` (a hipStream_t,
 * e.g. torch's current stream); NULL restores the context's own stream. */
nlq_status nlq_ctx_set_stream(nlq_ctx *ctx, void *hip_stream);
/* Bytes of device memory currently held by the context. */
nlq_status nlq_ctx_memory(const nlq_ctx *ctx, uint64_t *used, uint64_t *budget);
nlq_status nlq_ctx_destroy(nlq_ctx *ctx);

/* ---- mesh --------------------------------------------------------------- */

/* Copy a P1 simplicial mesh of Omega u Gamma to the device (Section 4: a
 * triangulation of Omega u Gamma into N_L elements).
 *  coords       host [n_nodes][dim] double
 *  conn         host [n_elems][dim+1] int32, node ids in [0, n_nodes)
 *  constrained  host [n_nodes] uint8, 1 = node in Gamma (value fixed by g)
 * Errors: EINVAL for dim not in {2,3}, ids out of range, zero-measure elements. */
nlq_status nlq_mesh_create(nlq_ctx *ctx, int32_t dim, int64_t n_nodes, const double *coords,
                           int64_t n_elems, const int32_t *conn, const uint8_t *constrained,
                           nlq_mesh **out);
/* As nlq_mesh_create with element order `order`: 1 (P1, conn [e][dim+1]) or 2
 * (quadratic Lagrange elements with straight sides, conn [e][(dim+1)(dim+2)/2]:
 * the dim+1 vertices, then the edge midpoints in the order (0,1), (0,2), (1,2)
 * in 2D and (0,1), (0,2), (0,3), (1,2), (1,3), (2,3) in 3D).  The geometry (boxes,
 * pair list, refinement) uses the vertices; the pattern, blocks, load vector and
 * solution all the nodes (Section 4: Lagrange bases; Section 6.1 uses linear and
 * quadratic ones).  P2 systems are assembled in FP64 (NLQ_FP64_PLAIN), without
 * deterministic mode. */
nlq_status nlq_mesh_create_order(nlq_ctx *ctx, int32_t dim, int32_t order, int64_t n_nodes, const double *coords,
                                 int64_t n_elems, const int32_t *conn, const uint8_t *constrained, nlq_mesh **out);
/* Element shapes (Section 4: the triangulation may consist of triangles or
 * quadrilaterals in 2D, tetrahedra or hexahedra in 3D). */
#define NLQ_SHAPE_SIMPLEX 0
#define NLQ_SHAPE_BOX 1
/* As nlq_mesh_create_order with an element shape.  NLQ_SHAPE_SIMPLEX: as above.
 * NLQ_SHAPE_BOX: quadrilaterals / hexahedra on the reference box [0,1]^dim with
 * the multilinear map of their 2^dim corners; the corners come first in tensor
 * order (corner c = c0 + 2 c1 + 4 c2 at the reference point (c0, c1, c2), i.e.
 * (0,0), (1,0), (0,1), (1,1) in 2D), then, for order 2 (serendipity: 8 nodes in
 * 2D, 20 in 3D, the quadratic elements of Section 6's quadrilateral and
 * hexahedral meshes), the edge midpoints in increasing t0 + 3 t1 + 9 t2 of
 * their position t in half units (exactly one t_k = 1).  Both sides of every
 * pair are integrated with the 3 x 3 (x 3) Gauss-Legendre product rule
 * (Section 6); Algorithm 1 splits a box into its 2^dim half boxes.  Box
 * systems are assembled in FP64 (NLQ_FP64_PLAIN), without deterministic mode.
 * Errors: EINVAL for an unknown shape or order, ids out of range, degenerate
 * elements (zero edge determinant at corner 0). */
nlq_status nlq_mesh_create_shape(nlq_ctx *ctx, int32_t dim, int32_t shape, int32_t order, int64_t n_nodes,
                                 const double *coords, int64_t n_elems, const int32_t *conn,
                                 const uint8_t *constrained, nlq_mesh **out);
/* Kuhn mesh of [0,1]^dim with n cells per direction built on the device:
 * x = i/n, node id = i0 + (n+1)(i1 + (n+1) i2), element id = dim!*cell + p with
 * p the lexicographic index of the permutation of the Kuhn path; Gamma = nodes
 * with some index <= k_gamma or >= n - k_gamma. */
nlq_status nlq_mesh_box(nlq_ctx *ctx, int32_t dim, int32_t n, int32_t k_gamma, nlq_mesh **out);
nlq_status nlq_mesh_info(const nlq_mesh *mesh, int32_t *dim, int64_t *n_nodes, int64_t *n_elems,
                         int64_t *n_free);
/* Host copies of a mesh (coords [n][dim], conn [e][nodes per element], constrained [n]). */
nlq_status nlq_mesh_copy(const nlq_mesh *mesh, double *coords, int32_t *conn, uint8_t *constrained);
nlq_status nlq_mesh_destroy(nlq_mesh *mesh);

/* ---- assembly ----------------------------------------------------------- */

/* Assemble the stiffness matrix of all nodes (constrained rows included, needed
 * for the lifting): element tables, pair list J_l, structural CSR pattern,
 * Algorithm 1 per pair, per-pair blocks, FP64 accumulation.  The system keeps a
 * reference to the mesh, which must outlive it.
 * Errors: EINVAL for inconsistent params, ENOMEM when the estimated footprint
 * exceeds the budget. */
nlq_status nlq_assemble(nlq_ctx *ctx, const nlq_mesh *mesh, const nlq_params *params,
                        nlq_system **out);
/* Set a system up without integrating it: element tables, pair list J_l and CSR
 * pattern are built, the values are zero (nlq_info and the copies work; the
 * leaf counts are zero).  For sampled work at sizes too large to integrate
 * whole: nlq_pair_blocks of chosen pairs, nlq_integrate_range of a slab. */
nlq_status nlq_prepare(nlq_ctx *ctx, const nlq_mesh *mesh, const nlq_params *params,
                       nlq_system **out);
/* Integrate the outer elements lo <= l < hi (0 < lo < hi < n_elems) of a
 * prepared or assembled system with the assembly kernels, adding their pairs'
 * contributions to the values (which then hold partial sums; a range touching
 * the first or last element is refused because those clear and finish the
 * matrix).  kernel_s: host [1] launch time from HIP events; n_leaf: host [9]
 * leaf integrations per level of this range (either may be NULL). */
nlq_status nlq_integrate_range(nlq_system *sys, int64_t lo, int64_t hi, double *kernel_s, int64_t *n_leaf);
/* As nlq_integrate_range for n_ranges (1..32) disjoint ranges lo[k] <= l < hi[k]
 * (host arrays, each 0 < lo[k] < hi[k] < n_elems) in ONE launch: a sample of outer
 * elements spread over the mesh, timed and counted together.  kernel_s: host [1]
 * launch time; n_leaf: host [9] leaf integrations per level summed over the
 * ranges; n_leaf_zero: host [1] those of them not evaluated (as in
 * nlq_assemble_info).  Any output may be NULL.  EINVAL for a bad or overlapping
 * range or a deterministic system. */
nlq_status nlq_integrate_ranges(nlq_system *sys, int32_t n_ranges, const int64_t *lo, const int64_t *hi,
                                double *kernel_s, int64_t *n_leaf, int64_t *n_leaf_zero);
/* Assemble n systems (meshes[i], params[i]) as n calls of nlq_assemble would,
 * but with shared integration launches: the outer elements of every system of
 * one (dim, precision, kernel) group, up to 32 systems per launch, are
 * interleaved in one persistent work queue (Algorithm 1 runs per pair, so the
 * order of pairs does not change any block).  out: host [n] handles.  The
 * systems' t_kernel is the time of the launch they shared.  On error no
 * system is returned. */
nlq_status nlq_assemble_batch(nlq_ctx *ctx, int32_t n, const nlq_mesh *const *meshes,
                              const nlq_params *params, nlq_system **out);
nlq_status nlq_assemble_info_get(const nlq_system *sys, nlq_assemble_info *info);

/* Autotuner of the integration launch.  Candidate configurations are timed on a
 * sample of the system's own outer elements (about four work items per resident
 * workgroup, middle of the mesh) for about budget_s seconds (<= 0: 2): first the
 * launch shape (register budget variant of the kernel, persistent workgroups
 * per CU, largest part of one pair list J_l per work item), then, from the best
 * shape, the capacity of each wave's traversal stack (64..512 entries: how many
 * sub-elements of Algorithm 1 one pass may pop and refine) and of its leaf
 * buffer (64..256: how many leaves are integrated per flush).  The fastest is
 * kept in the context for every later assembly with the same (dim, element
 * type, precision, kernel, L_max, size class of max |J_l|), including the
 * serving loop's.  An assembled
 * system's values are recomputed with it (nlq_set_data must be called again); a
 * prepared one's (nlq_prepare) are set back to zero. */
typedef struct {
    int32_t occupancy_variant;      /* 0: default waves per SIMD (2D 5, 3D FP32 4, 3D FP64 3); 1: one more (2D FP32) or one fewer (others) */
    int32_t workgroups_per_cu;      /* persistent workgroups per CU */
    int32_t pairs_per_item;         /* largest part of one J_l per work item (untuned: 512 in 2D, 256 in 3D) */
    int32_t work_items_per_element; /* parts each outer element is cut into */
    int32_t candidates;             /* configurations timed */
    double best_ms, default_ms;     /* sample launch time: chosen and default configuration */
    int32_t stack_capacity;         /* traversal stack entries per wave (untuned: 128) */
    int32_t leaf_capacity;          /* leaf buffer entries per wave (untuned: 128) */
} nlq_tune_info;
nlq_status nlq_autotune(nlq_system *sys, double budget_s, nlq_tune_info *info);
/* The context's tuned configurations as a text file, so that a later process
 * can start tuned: a comment line, then one line per class key
 * "arch dim element precision kernel lmax size_class occ wg_per_cu
 * pairs_per_item stack_cap leaf_cap" (arch of the device, e.g. gfx950; element
 * 1 = P1, 2 = P2, 3 = Q1, 4 = serendipity; lines of the earlier format without
 * element and capacities load as P1 with the untuned capacities).  nlq_tune_save writes (overwrites) path;
 * nlq_tune_load reads such a file and keeps the lines of this context's
 * architecture (others are skipped), setting *n_loaded (may be NULL) to their
 * number.  A file that cannot be opened, or a line that does not parse, gives
 * NLQ_EINVAL and loads nothing. */
nlq_status nlq_tune_save(const nlq_ctx *ctx, const char *path);
nlq_status nlq_tune_load(nlq_ctx *ctx, const char *path, int32_t *n_loaded);
/* Re-run only the integration step (pair list and pattern kept) -- the hot loop;
 * values are recomputed from zero. */
nlq_status nlq_reassemble(nlq_system *sys);

/* Load vector and lifting (Section 2, eqs. (A-F), (weak-homo)):
 * F_i = int_Omega f_h phi_i with f_h the P1 interpolant of f_nodal, and
 * F~ = F - A g~ on free rows, with g~ = g on Gamma and 0 elsewhere (the lifting
 * enters with a minus sign).  f_nodal, g_nodal: host [n_nodes]. */
nlq_status nlq_set_data(nlq_system *sys, const double *f_nodal, const double *g_nodal);
/* As nlq_set_data with device pointers [n_nodes] (e.g. torch tensors already in
 * HBM); read on the context's stream, not retained after the call. */
nlq_status nlq_set_data_device(nlq_system *sys, const double *f_dev, const double *g_dev);
/* Jacobi-preconditioned CG on A_{Omega,Omega} w = F~_Omega (FP64 SpMV, dots and
 * residuals); u = w on free nodes, g on Gamma.  u_out: host [n_nodes] or NULL.
 * Returns ENOCONV (u = last iterate) when maxit is reached. */
nlq_status nlq_solve(nlq_system *sys, double rtol, int32_t maxit, double *u_out,
                     nlq_solve_info *info);
/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the solve of nlq_solve
 * with no allocation at all.  The CG vectors, block partials and scalars live in
 * a static device scratch array of the library (16 MiB per GPU, held until the
 * process ends; enough for about 290,000 nodes), whose device address the
 * context's creation takes once per device.  u_dev: caller-owned DEVICE buffer
 * [n_nodes] receiving u (w on free nodes, g on Gamma).  Iterations run as plain
 * launches (no graph), in the same order as nlq_solve's, with the same result.
 * Calls on one GPU share its scratch: calls that overlap in time on one GPU (two
 * host threads, two contexts) race and must be serialised by the caller.
 * Errors: EINVAL when nlq_set_data has not run, for bad rtol/maxit or NULL u_dev,
 * and when the system needs more scratch than the limit (the message names both
 * sizes); ENOCONV as nlq_solve. */
nlq_status nlq_solve_noalloc(nlq_system *sys, double rtol, int32_t maxit, double *u_dev, nlq_solve_info *info);
/* Borrowed device pointer to the last solution u [n_nodes], valid until
 * nlq_system_destroy (NULL before the first nlq_solve). */
nlq_status nlq_solution_device(const nlq_system *sys, const double **u_dev);

nlq_status nlq_info(const nlq_system *sys, int64_t *n_rows, int64_t *nnz, int64_t *n_pairs,
                    int64_t *n_free);
/* Host copies (caller-allocated): row_ptr [n_rows+1], col [nnz], val [nnz]. */
nlq_status nlq_csr_copy(const nlq_system *sys, int64_t *row_ptr, int32_t *col, double *val);
/* Borrowed device pointers, valid until nlq_system_destroy. */
nlq_status nlq_csr_device(const nlq_system *sys, const int64_t **row_ptr, const int32_t **col,
                          const double **val);
/* Host copies of the pair list: offsets [n_elems+1], inner ids [n_pairs]. */
nlq_status nlq_pairs_copy(const nlq_system *sys, int64_t *offsets, int32_t *m);
/* Host copy of F~ [n_rows] (0 on Gamma rows). */
nlq_status nlq_rhs_copy(const nlq_system *sys, double *f_tilde);
/* Per-pair blocks of selected ordered pairs (l[k], m[k]), recomputed with the
 * assembly kernels: out [n][2 nb][2 nb] (nb nodes per element: N+1 for P1,
 * (N+1)(N+2)/2 for P2) in the extended index space [local nodes of l, local
 * nodes of m] (the four-term form fills all four blocks, the two-term form the
 * rows of m, its adaptive-inner variant the rows of l). */
nlq_status nlq_pair_blocks(nlq_system *sys, int64_t n, const int32_t *l, const int32_t *m,
                           double *out);
nlq_status nlq_system_destroy(nlq_system *sys);

/* ---- serving: continuous batching of assemble + solve requests ------------
 * The problem of Section 2 posed on a Kuhn box mesh, as a request: mesh size,
 * horizon, kernel and data in; nodal solution out (Section 4, eq. (AW=F)).
 *  - Admission: a scheduler thread admits queued requests (FIFO) while the
 *    context's HBM in use plus the estimated footprint of the admitted but not
 *    yet assembled requests fits the budget; resident matrices of earlier
 *    requests are evicted (least recently used first) to make room.
 *  - One device thread owns the GPU and time-slices it; each pass: the CG of
 *    every request whose matrix is ready, the setup (element tables, pair list,
 *    pattern) of the admitted requests, smallest first (for about one launch
 *    target), then one shared integration launch of one group: that of the
 *    most urgent request -- least estimated integration time left, minus a
 *    quarter of its wait for a launch -- in a launch just long enough for it
 *    to finish (at most the target duration), holding up to 32 requests of
 *    the group, most urgent first.
 *  - Integration: outer elements of all assembled-but-not-integrated requests of
 *    one (dim, precision, kernel) group share persistent launches (at most 32
 *    requests per launch, see nlq_assemble_batch); a launch is sized from the
 *    measured integration rate to about target_launch_ms (raised until it
 *    fills the grid) and filled in urgency order, each request taking all it
 *    has left while the budget lasts: shortest remaining work first, so small
 *    requests finish in one launch.  Requests that arrive while a launch runs
 *    join the next one.
 *  - Residency: meshes stay on the device for the server's lifetime (keyed by
 *    dim, n, k_gamma); with cache_systems = 1 assembled matrices stay too and a
 *    request with the same mesh and parameters only reloads f, g and solves.
 * Latency = completion - submission. */
typedef struct {
    int32_t dim, n, k_gamma;     /* box mesh (nlq_mesh_box) */
    nlq_params params;
    const double *f_nodal;       /* host [n_nodes], copied at submit */
    const double *g_nodal;       /* host [n_nodes], copied at submit */
    double rtol;                 /* CG tolerance (<= 0: 1e-10) */
    int32_t maxit;               /* CG iteration cap (<= 0: 10000) */
} nlq_request;

typedef struct {
    nlq_status status;
    int64_t n_nodes, n_pairs, n_free;
    const double *u;             /* host [n_nodes], library-owned until release */
    int32_t cg_iterations;
    double rel_residual;
    double latency_s;            /* submit -> result ready */
    double queue_s;              /* submit -> admitted */
    double assemble_s;           /* admitted -> matrix ready (setup + integration; 0 on a cache hit) */
    double solve_s;              /* matrix ready -> result ready (load vector, lifting, CG, copy) */
    int32_t launches;            /* shared integration launches the request took part in */
    int32_t cache_hit;           /* 1: its matrix was resident from an earlier request */
    double setup_s;              /* admitted -> set up (mesh, pair list, pattern; the first part of assemble_s) */
} nlq_result;

typedef struct {
    int32_t max_active;          /* admitted requests at once (<= 0: 256) */
    double target_launch_ms;     /* duration aimed at per shared launch (<= 0: 25) */
    int32_t cache_systems;       /* 1: keep assembled matrices resident for reuse */
} nlq_serve_config;

typedef struct {
    int64_t submitted, completed, failed, cancelled;
    int64_t launches;            /* shared integration launches */
    int64_t launch_segments;     /* sum over launches of the requests in each */
    int32_t max_per_launch;      /* most requests in one launch */
    int32_t max_admitted;        /* most requests admitted at once */
    int64_t cache_hits;
    uint64_t peak_bytes;         /* peak of the context's HBM accounting */
    double launch_s;             /* sum of launch durations (HIP events) */
} nlq_serve_stats;

/* cfg may be NULL (defaults). EBUSY if a server is already running. */
nlq_status nlq_serve_start(nlq_ctx *ctx, const nlq_serve_config *cfg);
/* Copies the request (f, g included).  EINVAL for a malformed request (checked
 * again at setup: parameter errors end the request with EINVAL). */
nlq_status nlq_submit(nlq_ctx *ctx, const nlq_request *req, uint64_t *ticket);
/* timeout_ms < 0: wait forever; 0: poll.  ENOTREADY when not finished. */
nlq_status nlq_wait(nlq_ctx *ctx, uint64_t ticket, int32_t timeout_ms, nlq_result *out);
/* A queued request ends with ECANCELLED at once; an admitted one at its next
 * phase boundary (after setup, after integration, before CG). */
nlq_status nlq_cancel(nlq_ctx *ctx, uint64_t ticket);
nlq_status nlq_result_release(nlq_ctx *ctx, uint64_t ticket);
nlq_status nlq_serve_stats_get(nlq_ctx *ctx, nlq_serve_stats *out);
/* Finishes every submitted request, then stops the threads and frees the
 * resident meshes and matrices. */
nlq_status nlq_serve_stop(nlq_ctx *ctx);

/* Thread-local message of the last failed call ("" if none). */
const char *nlq_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
