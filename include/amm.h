/*
 * amm.h -- C ABI of the MI355X (gfx950) library for robust non-rigid
 * registration by accelerated majorization-minimization (Yao, Deng, Xu,
 * Zhang, "Fast and Robust Non-Rigid Registration Using Accelerated
 * Majorization-Minimization", arXiv 2206.03410).
 *
 * Problem (Sec. 3 of the paper): source points V = {v_i} (i < n_src),
 * target points U = {u_l} (l < n_tgt), an embedded deformation graph whose
 * nodes p_j are a subset of V, per-point influence sets I(v_i) of k nodes
 * with weights w_ij (Eq. 3), and undirected node edges E_G.  Unknowns are
 * one affine transform X_j = [A_j, t_j] per node.  The library minimizes
 *     E(X) = E_align + alpha E_reg + beta E_rot                     (Eq. 4)
 * with Welsch's function on alignment and regularization residuals
 * (Eqs. 5-10), by MM iterations whose quadratic surrogate is minimized
 * through the normal equations K X = B (Eq. 21), accelerated by Anderson
 * acceleration with an energy-decrease fallback, inside the nu
 * continuation of Alg. 2.
 *
 * Conventions (every call):
 *  - Floating-point arrays have the element type named by the call
 *    (amm_dtype); integer arrays are int32.  Layouts are row-major and
 *    contiguous.  Points are [count][3].
 *  - Transforms X are [n_nodes][4][3]: rows 0..2 hold A_j^T, row 3 holds
 *    t_j^T; this is the block X_j of the paper's stacked X in R^{4n x 3}.
 *  - Unless a parameter says "host", pointers are device pointers on the
 *    handle's device.  Work is ordered on the handle's stream; calls that
 *    return host values synchronize that stream before returning.
 *  - The library never keeps a caller pointer: what it needs is copied.
 *  - A handle is not thread-safe: one call at a time per handle.
 *  - Every call returns an amm_status; on failure amm_last_error() gives a
 *    message.  No call aborts the process.
 */
#ifndef AMM_H
#define AMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMM_OK = 0,
    AMM_ERR_INVALID_ARG = 1, /* null pointer, bad size, index out of range */
    AMM_ERR_STATE = 2,       /* call order (e.g. solve before set_problem) */
    AMM_ERR_OOM = 3,         /* device allocation failed / workspace too small */
    AMM_ERR_HIP = 4,         /* a HIP runtime call failed (no device, ...) */
    AMM_ERR_NONFINITE = 5,   /* NaN or Inf in an input, or the iteration blew up */
    AMM_ERR_GRAPH = 6,       /* weights do not sum to 1, node graph disconnected, ... */
    AMM_ERR_NOT_SPD = 7      /* K not positive definite (CG breakdown) */
} amm_status;

typedef enum { AMM_F32 = 0, AMM_F64 = 1 } amm_dtype;

/* Arithmetic of the solve.
 * AMM_FP64_PLAIN : every step in float64; the linear solve is float64
 *                  preconditioned CG to the requested relative residual.
 * AMM_FP32_REFINE: closest points, warp, weights, energies and assembly in
 *                  float32; the solve is float32 preconditioned CG inside
 *                  float64 iterative refinement (float64 residual B - K X and
 *                  float64 solution accumulator); the Anderson Gram matrix
 *                  and its solve are float64. */
typedef enum { AMM_FP64_PLAIN = 0, AMM_FP32_REFINE = 1 } amm_precision;

/* Preconditioner of the CG solve of Eq. (21).  Block Jacobi inverts the 4x4
 * diagonal blocks of K (one per node and column).  Two-level adds a coarse
 * correction P A_c^{-1} P^T, A_c = P^T K P, over one affine field per
 * aggregate of spatially consecutive graph nodes (at most 32 aggregates per
 * pair): the same solution, several times fewer CG iterations. */
typedef enum { AMM_PRECOND_TWO_LEVEL = 0, AMM_PRECOND_BLOCK_JACOBI = 1 } amm_precond;

/* Robust terms.  WELSCH is the method (Eqs. 5, 9 with the surrogate weights
 * of Eqs. 13-16).  The other two are the squared-norm variants of Sec. 4.1:
 * L2 uses unit weights on every alignment residual and a plain squared norm
 * on the regularization residuals; L2_TRUNC keeps weight 1 only for points
 * whose closest-point distance is below 3 nu_a (0 otherwise), which is MM on
 * the truncated quadratic min(|e|^2, 9 nu_a^2), with the same squared-norm
 * regularization.  Both squared-norm variants weight the terms by
 * alpha = k_alpha |V|/|E_G| and beta = k_beta |V|/|V_G| (the small-residual
 * scale of Eq. 26's Welsch weighting). */
typedef enum { AMM_ROBUST_WELSCH = 0, AMM_ROBUST_L2 = 1, AMM_ROBUST_L2_TRUNC = 2 } amm_robust;

/* nu schedule.  DYNAMIC is the continuation of Sec. 3.3.3.  The fixed modes
 * are Sec. 4.1's Welsch-fmax / -fmin / -fmed: (nu_a, nu_r) held for one
 * stage at the largest, the smallest, or the mean of the two, of the values
 * the dynamic update would reach from the same start (nu_a halves down to
 * its bound, nu_r halves with it).  With AMM_ROBUST_L2 there is no parameter
 * and the solve runs one stage. */
typedef enum {
    AMM_NU_DYNAMIC = 0,
    AMM_NU_FIXED_MAX = 1,
    AMM_NU_FIXED_MIN = 2,
    AMM_NU_FIXED_MED = 3
} amm_nu_mode;

typedef struct amm_handle amm_handle;

/* One registration problem.  `on_device` = 1: the pointers are device
 * pointers; 0: host pointers.  Normals are optional (NULL) and unused by the
 * energy of Eq. (5), which is point-to-point; they are validated when given. */
typedef struct {
    amm_dtype dtype;              /* type of src_xyz, src_nrm, tgt_xyz, tgt_nrm, infl_w */
    int32_t on_device;
    int64_t n_src;
    const void* src_xyz;          /* [n_src][3] */
    const void* src_nrm;          /* [n_src][3] or NULL */
    int64_t n_tgt;
    const void* tgt_xyz;          /* [n_tgt][3] */
    const void* tgt_nrm;          /* [n_tgt][3] or NULL */
    int64_t n_nodes;
    const int32_t* node_src_idx;  /* [n_nodes] distinct indices into V (nodes lie on V) */
    int32_t k;                    /* influences per point, 1 <= k <= 8, k <= n_nodes */
    const int32_t* infl_idx;      /* [n_src][k] node ids (0 <= id < n_nodes, distinct per row);
                                   * -1 marks an unused slot (a point with fewer than k
                                   * influencing nodes); every point needs one used slot */
    const void* infl_w;           /* [n_src][k] weights of Eq. (3), 0 in unused slots; each row sums to 1 */
    int64_t n_edges;
    const int32_t* edges;         /* [n_edges][2] undirected node edges, i != j, no duplicates */
    double mean_edge_len;         /* average source edge length l (Sec. 3.3.3), > 0 */
} amm_problem;

typedef struct {
    /* nu continuation (Sec. 3.3.3).  Each value <= 0 selects the paper's
     * rule: nu_a0 = median closest-point distance at the initial X,
     * nu_a_min = mean_edge_len / sqrt(3), nu_r0 = 3 mean_edge_len. */
    double nu_a0, nu_a_min, nu_r0;
    /* term weights of Eq. (26): alpha = k_alpha |V|/|E_G| nu_r^2/nu_a^2,
     * beta = k_beta |V|/|V_G| / (2 nu_a^2), recomputed at every stage. */
    double k_alpha, k_beta;
    double eps;                   /* stage ends when max_i |v_hat_i^{k+1} - v_hat_i^k| < eps */
    int32_t imax;                 /* surrogate solves per stage at most */
    int32_t max_total_iters;      /* surrogate solves overall at most; 0 = no cap */
    int32_t aa_m;                 /* Anderson depth m, 0 <= m <= AMM_MAX_AA_M (0 = plain MM) */
    int32_t precision;            /* amm_precision */
    double cg_rtol;               /* relative residual |B - K X| / |B| per column, e.g. 1e-10 */
    int32_t cg_maxit;             /* CG iterations per solve at most (0 = 20000) */
    int32_t init_identity;        /* 1: start from X = I (ignore X_inout's contents) */
    /* Replay of decisions (host arrays, may be NULL): entry t applies to the
     * t-th surrogate solve.  force_accept: -1 decide, 0 reject the Anderson
     * candidate, 1 accept it.  force_stage_end: -1 decide, 0 continue the
     * stage, 1 end it.  With force_per_pair = 0 every pair reads the same
     * force_len entries; with 1 the arrays hold one row of force_len
     * entries per pair (row p for pair p). */
    const int8_t* force_accept;
    const int8_t* force_stage_end;
    int32_t force_len;
    int32_t cg_precond;           /* amm_precond (0 = two-level, the default) */
    int32_t robust;               /* amm_robust (0 = Welsch, the method) */
    int32_t nu_mode;              /* amm_nu_mode (0 = dynamic, the method) */
    int32_t force_per_pair;
} amm_params;

#define AMM_MAX_AA_M 10

/* Fills p with the paper's defaults: eps = 1e-5, imax = 100 (Sec. 4.1),
 * k_alpha = 100, k_beta = 1, aa_m = 5, nu rules, FP32 refinement,
 * cg_rtol = 1e-10, start from identity. */
void amm_params_default(amm_params* p);

typedef struct {
    int32_t iters;               /* surrogate solves performed */
    int32_t stages;              /* nu stages entered */
    int32_t converged;           /* 1 if the last stage (nu_a at its bound) met eps */
    int32_t aa_accepted, aa_rejected;
    int64_t cg_iters;            /* total CG iterations (all refinement steps) */
    int32_t refine_steps;        /* total iterative-refinement steps (FP32_REFINE) */
    double energy, e_align, e_reg, e_rot; /* at the returned X, final nu */
    double nu_a, nu_r, alpha, beta;       /* final stage values */
    double max_disp;             /* last max displacement */
    double max_rel_residual;     /* worst final relative residual over all solves */
    double time_ms;              /* wall time of the solve for this pair */
    /* surrogate solves whose final relative residual stayed above cg_rtol
     * (float32 refinement stopped improving, or the CG step budget ran out);
     * 0 when every solve of Eq. (21) met its tolerance */
    int32_t solves_above_rtol;
} amm_stats;

/* One MM iteration (one surrogate solve) of one pair, as decided by Alg. 2. */
typedef struct {
    int32_t pair, iter, stage, m_k;
    int32_t aa_used;             /* the Anderson candidate differs from G(X^k) */
    int32_t accepted;            /* 1 accepted, 0 rejected (G(X^k) taken), -1 not tested */
    int32_t cg_iters, refine_steps;
    double energy_before;        /* E(X^k) */
    double energy_candidate;     /* E of the candidate that was evaluated first */
    double energy_after;         /* E(X^{k+1}) */
    double max_disp;             /* max_i |v_hat^{k+1} - v_hat^k| */
    double nu_a, nu_r, alpha, beta;
    double rel_residual;         /* |B - K X'| / |B| of the solve (worst column) */
} amm_iter_record;

/* ---------------------------------------------------------------- handle */

/* Creates a handle on `device` that orders its work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Fails with AMM_ERR_HIP when no
 * such device exists. */
amm_status amm_create(amm_handle** h, int device, void* hip_stream);
void amm_destroy(amm_handle* h);
amm_status amm_set_stream(amm_handle* h, void* hip_stream);

/* ---------------------------------------------------------------- problem */

/* Host-only validation of a problem given by HOST pointers (on_device = 0);
 * needs no GPU.  Checks sizes and index ranges, and that unused influence
 * slots (-1) carry weight 0 (AMM_ERR_INVALID_ARG), finiteness
 * (AMM_ERR_NONFINITE), and the structure (AMM_ERR_GRAPH): distinct node
 * indices, at least one and distinct influences per point with non-negative
 * weights that sum to 1 within 1e-5, and a connected node graph without
 * duplicate or self edges. */
amm_status amm_check_problem(const amm_problem* p);

/* Replaces the target points of pair `pair` (0-based within the last
 * amm_set_problems batch) by n_tgt new ones of the same count, keeping the
 * source side (graph, pattern of K, point lists, coarse aggregates) as it
 * is; only the pair's closest-point structure (the targets in Morton order
 * and the octree's run-start tables, at the pair's octree depth) is rebuilt,
 * on the device (the coordinates of host inputs are copied there first).
 * For registering one template to a sequence of frames (Sec. 4's sequences)
 * without a new upload.  The result equals a new amm_set_problems with the
 * new targets.  Pointers are device pointers when on_device = 1; the call
 * synchronizes the device before reading them and returns once the new
 * structure is in place.  Errors: AMM_ERR_STATE before a
 * problem is set, AMM_ERR_INVALID_ARG (pair, count, dtype, null),
 * AMM_ERR_NONFINITE. */
amm_status amm_set_targets(amm_handle* h, int32_t pair, amm_dtype dtype, const void* tgt_xyz, int64_t n_tgt,
                           int32_t on_device);

/* Device bytes that amm_set_problems needs for these problems (a static
 * analysis of the inputs; the result is exact). */
amm_status amm_workspace_size(amm_handle* h, const amm_problem* probs, int32_t n_pairs,
                              size_t* bytes);

/* Hands the library a caller-owned device buffer (256-byte aligned) that
 * amm_set_problems carves all its device memory from; it must outlive the
 * handle's use of the problems.  ptr = NULL reverts to library-owned memory
 * (allocated once, in amm_set_problems). */
amm_status amm_set_workspace(amm_handle* h, void* ptr, size_t bytes);

/* Validates and uploads a batch of independent registration problems
 * (n_pairs >= 1, all with the same k).  Computes the edge weights r_ij of
 * Eq. (8), a spatial ordering of points and nodes, the block pattern of K,
 * and the nearest-neighbour structures over each target set (a bounding-box
 * tree over Morton-ordered targets, and a uniform grid over the same order
 * for warm-started searches).  Replaces any previous problems. */
amm_status amm_set_problems(amm_handle* h, const amm_problem* probs, int32_t n_pairs);
amm_status amm_set_problem(amm_handle* h, const amm_problem* p);

/* Sizes of the batch set on the handle (host outputs, each nullable): the
 * pair count (the length of the stats array amm_solve fills), and the totals
 * over pairs of source points (rows of v_out and of gV), graph nodes (rows
 * of X_inout, of X and of gX) and target points, and k.  For pair 0 alone
 * (amm_step, amm_energy, amm_energy_grad) use n_pairs = 1 batches.
 * AMM_ERR_STATE before a problem is set. */
amm_status amm_get_sizes(const amm_handle* h, int32_t* n_pairs, int64_t* n_src_total, int64_t* n_nodes_total,
                         int64_t* n_tgt_total, int32_t* k);

/* Cell size of the closest-point search structure, as the mean number of
 * targets per occupied leaf cell (1..256, default 8), used by the next
 * amm_workspace_size / amm_set_problems.  Each pair's targets are sorted
 * along a Morton curve and covered by an implicit octree of cells
 * (Morton prefixes); the pair's depth is the smallest in 2..8 whose
 * occupied leaf cells hold at most this many targets on average.  Smaller
 * values make the octree deeper (more cells read per search), larger ones
 * scan more targets per leaf. */
amm_status amm_set_leaf_size(amm_handle* h, int32_t leaf);

/* Step budget of one point's closest-point search (the rho(i) of Eq. 5,
 * Sec. 3.2) inside an evaluation, in search steps (cell expansions and cell
 * visits; 0..1000000, default 64; 0 = unlimited).  Searches that exceed it
 * stop with their best target so far and are finished afterwards by an
 * exact search that spreads each point over a whole wavefront, so that a
 * few far points (outliers, uncovered regions) do not hold up the waves of
 * near ones.  Results do not depend on the budget (the search is exact,
 * ties to the lowest target index), only the time does.  Takes effect at
 * the next evaluation.  Errors: AMM_ERR_INVALID_ARG outside the range. */
amm_status amm_set_search_budget(amm_handle* h, int32_t steps);

/* The step budget in use (set, or picked by amm_autotune). */
amm_status amm_get_search_budget(const amm_handle* h, int32_t* steps);

/* Autotuner: uploads the problems once per candidate leaf size (candidates
 * NULL: 2, 4, 8, 16) and, for each, times a warm-started float32 evaluation
 * (warp, closest points, Welsch terms, the per-iteration search of Alg. 2)
 * of every pair at X = I with HIP events under search step budgets of 32,
 * 48, 64, 96, 128 and unlimited (amm_set_search_budget); leaves the handle
 * set up with the fastest leaf size and budget.  best_leaf and best_ms
 * (host, nullable) receive the leaf size and the time; the budget is read
 * with amm_get_search_budget.  With a caller workspace, candidates that do not fit it are
 * skipped.  Replaces any previous problems, like amm_set_problems. */
amm_status amm_autotune(amm_handle* h, const amm_problem* probs, int32_t n_pairs, const int32_t* candidates,
                        int32_t n_candidates, int32_t* best_leaf, double* best_ms);

/* ---------------------------------------------------------------- solve */

/* Alg. 2 for every pair set on the handle, all pairs advancing together.
 * X_inout: concatenation over pairs of [n_nodes][4][3] in the precision's
 * type (float32 for AMM_FP32_REFINE, float64 for AMM_FP64_PLAIN); read as
 * the start unless params->init_identity, overwritten with the result.
 * v_out: concatenation of [n_src][3] deformed source points (Eq. 2 at the
 * result), same type; may be NULL.  stats: host array of n_pairs entries,
 * may be NULL.  Non-convergence within imax / max_total_iters is not an
 * error (stats.converged = 0). */
amm_status amm_solve(amm_handle* h, const amm_params* params, void* X_inout, void* v_out,
                     amm_stats* stats);

/* Per-iteration record of the last amm_solve, all pairs in the order the
 * iterations completed: out[i] for i < min(*count, capacity) (out may be
 * NULL to query the count). */
amm_status amm_iter_log(amm_handle* h, amm_iter_record* out, int32_t capacity, int32_t* count);

/* Work counters of the closest-point search (Sec. 3.2's correspondence
 * step), for reporting how much target data an exact search examines.
 * amm_count_nn_work(h, 1) zeroes the counters and switches every later
 * evaluation (solve, step, energy) to a counting variant of its kernel,
 * which is slower; 0 switches back and frees them.  amm_set_problems also
 * switches counting off.  amm_nn_work returns, since counting was switched
 * on: the queries searched, the cell lower-bound tests (computed from the
 * cell's coordinates, no memory read), the target distance evaluations
 * (each reads one target) and, if cell_lookups is not null, the cell
 * expansions that read their children's nine run starts from memory (the
 * upper levels, kept in LDS, are not counted).  Errors:
 * AMM_ERR_STATE before a problem is set, or when counting is off. */
amm_status amm_count_nn_work(amm_handle* h, int32_t enable);
amm_status amm_nn_work(amm_handle* h, int64_t* queries, int64_t* box_tests, int64_t* distance_evals,
                       int64_t* cell_lookups);

/* ---------------------------------------------------------------- graph construction */

/* Deformation graph of Sec. 3.1 (Alg. 1) built on the device, with
 * Euclidean distance or with the geodesic distance D of Eq. (1) (field
 * `geodesic`): the source points are
 * ordered along their principal axis (largest eigenvalue of the covariance;
 * the axis component of largest magnitude taken positive, equal projections
 * in index order); in that order a point becomes a node when no earlier node
 * lies strictly within R of it; each point is influenced by the nodes
 * strictly within R, weighted by Eq. (3); nodes that influence a common
 * point are joined by an edge.  Node ids follow the order of insertion.
 * Each point keeps its k nearest influencing nodes (ties to the lower node
 * id) with the weights renormalized over them, so that the result feeds
 * amm_problem directly; unused slots are -1 with weight 0, and edges come
 * from kept slots.  The mean edge length l (Sec. 3.3.3) is that of the
 * symmetrized, deduplicated 6-nearest-neighbour graph of the source points.
 * Geodesic distance on a point cloud (whose edge set Sec. 3 builds from each
 * point's nearest neighbours): the shortest path over that same 6-NN graph
 * (ties to the lower index), each edge as long as its Euclidean length; the
 * search from a point stays inside its Euclidean ball of radius R (which a
 * path shorter than R never leaves), at most 1024 points (larger balls are
 * refused with AMM_ERR_INVALID_ARG); Eq. (3) takes D^2 = D * D. */
typedef struct {
    amm_dtype dtype;          /* type of src_xyz and of the weights amm_graph_copy writes */
    const void* src_xyz;      /* DEVICE pointer, [n_src][3] */
    int64_t n_src;            /* >= 2 */
    double radius;            /* R; <= 0 selects radius_factor * l */
    double radius_factor;     /* used when radius <= 0; <= 0 selects 5 (Sec. 4.1) */
    int32_t k;                /* influence slots per point, 1 <= k <= 8 */
    int32_t geodesic;         /* 0: Euclidean distance; 1: geodesic distance (Eq. 1); equal over sets */
} amm_graph_in;

typedef struct {
    int64_t n_nodes, n_edges;
    double radius;            /* R used */
    double mean_edge_len;     /* l */
    int64_t n_capped;         /* points with more than k nodes within R */
    int32_t max_influences;   /* most nodes within R of one point */
    int32_t rounds;           /* parallel rounds the node selection took */
} amm_graph_info;

/* Builds the graph of the given points on the handle's device and stream
 * and keeps it in the handle (replacing an earlier one) until
 * amm_graph_copy fetches it.  The node selection equals the sequential
 * greedy pass exactly: a point is decided as soon as every earlier point
 * within R is, in rounds that run until none is left.  Needs no problem set.
 * Errors: AMM_ERR_INVALID_ARG (sizes, k, a non-positive R),
 * AMM_ERR_NONFINITE, AMM_ERR_OOM, AMM_ERR_HIP. */
amm_status amm_build_graph(amm_handle* h, const amm_graph_in* in, amm_graph_info* info);

/* The same for n_sets independent point sets (the pairs of a batch) in one
 * pass: every round of the node selection, every sort and scan covers all
 * sets; each set's result equals its own amm_build_graph.  k and dtype must
 * agree over the sets; info receives n_sets records. */
amm_status amm_build_graphs(amm_handle* h, const amm_graph_in* in, int32_t n_sets, amm_graph_info* info);

/* Copies set `set` (0 for amm_build_graph) of the last build into
 * caller-owned DEVICE buffers (any may be NULL): node_src_idx [n_nodes]
 * (indices into the set's points), infl_idx [n_src][k] (the set's node ids),
 * infl_w [n_src][k] in the build's dtype, edges [n_edges][2] (i < j,
 * sorted).  AMM_ERR_STATE if no graph was built, AMM_ERR_INVALID_ARG for a
 * set out of range. */
amm_status amm_graph_copy_set(amm_handle* h, int32_t set, int32_t* node_src_idx, int32_t* infl_idx, void* infl_w,
                              int32_t* edges);
amm_status amm_graph_copy(amm_handle* h, int32_t* node_src_idx, int32_t* infl_idx, void* infl_w,
                          int32_t* edges);

/* ---------------------------------------------------------------- single step */

typedef struct {
    const void* X;           /* [n_nodes][4][3] current iterate X^k (pair 0) */
    double nu_a, nu_r, alpha, beta;
    int32_t precision;       /* amm_precision */
    double cg_rtol;
    int32_t cg_maxit;
    int32_t cg_precond;      /* amm_precond */
    int32_t robust;          /* amm_robust; nu_a, alpha, beta are taken as given */
} amm_step_in;

typedef struct {
    double energy[4];        /* host: E, E_align, E_reg, E_rot at X^k */
    int32_t* rho;            /* [n_src] closest target index per point, or NULL */
    void* d2;                /* [n_src] squared closest distance, or NULL */
    void* v_hat;             /* [n_src][3] warped points at X^k, or NULL */
    void* X_next;            /* [n_nodes][4][3] minimizer of the surrogate, or NULL */
    /* Normal equations of Eq. (21) at X^k in node order of the caller, or NULL:
     * K_blocks [nnzb][4][4], K_row/K_col [nnzb] node ids, B [n_nodes][4][3].
     * Query nnzb with amm_k_nnzb. */
    void* K_blocks;
    int32_t* K_row;
    int32_t* K_col;
    void* B;
    int32_t cg_iters;        /* host */
    double rel_residual;     /* host */
} amm_step_out;

/* One surrogate solve at explicit (nu_a, nu_r, alpha, beta) for pair 0,
 * teacher-forced from X^k: closest points and energy at X^k, assembly of
 * K, B and their solve.  For checking each step against a reference. */
amm_status amm_step(amm_handle* h, const amm_step_in* in, amm_step_out* out);
amm_status amm_k_nnzb(amm_handle* h, int64_t* nnzb);

/* ---------------------------------------------------------------- energy and gradient */

/* E(X) of Eq. (4) for pair 0 at transforms X and source positions src
 * (NULL = the stored source), both of type `dtype` (which also selects the
 * arithmetic).  energy: host double[4] = {E, E_align, E_reg, E_rot}.
 * rho (int32 [n_src]) and d2 ([n_src], dtype) may be NULL.  The graph
 * (p_j, w_ij, r_ij) is the one given to amm_set_problem. */
amm_status amm_energy(amm_handle* h, amm_dtype dtype, const void* X, const void* src,
                      double nu_a, double nu_r, double alpha, double beta, double* energy,
                      int32_t* rho, void* d2);

/* Gradient of E with respect to X (gX [n_nodes][4][3]) and the source
 * positions (gV [n_src][3]), both of type `dtype`, with the closest points
 * of the evaluation held fixed and the graph frozen: only the v_i appearing
 * explicitly in Eq. (2) move with the source.  gV may be NULL.  energy as in
 * amm_energy (may be NULL). */
amm_status amm_energy_grad(amm_handle* h, amm_dtype dtype, const void* X, const void* src,
                           double nu_a, double nu_r, double alpha, double beta, void* gX,
                           void* gV, double* energy);

/* The energy of amm_energy for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the same evaluation kernels, the same results (bitwise), but
 * every per-call buffer (imported transforms and source positions, the
 * warped points, closest points, residuals and weights, the deferred
 * searches' list, per-point terms, tile partial sums, the pair's parameters
 * and outputs) lives in a file-scope device array of
 * 64 MiB that each GPU the library runs on holds until the process ends;
 * the handle's workspace still holds the problem set up by
 * amm_set_problem.  Nothing is allocated: no hipMalloc, no host or pinned
 * allocation.  The search starts cold (no warm start from earlier calls).
 * Problems whose per-call buffers exceed 64 MiB (about 4.9e5 source points
 * in float64, 8.8e5 in float32) are refused with AMM_ERR_INVALID_ARG.  Every call
 * on one GPU uses that GPU's single array: calls that overlap in time on one
 * GPU (two host threads, or two streams) race and must be serialized by the
 * caller.  Arguments and errors as amm_energy. */
amm_status amm_energy_noalloc(amm_handle* h, amm_dtype dtype, const void* X, const void* src,
                              double nu_a, double nu_r, double alpha, double beta, double* energy,
                              int32_t* rho, void* d2);

/* ---------------------------------------------------------------- misc */

const char* amm_status_string(amm_status s);
const char* amm_last_error(const amm_handle* h);   /* h may be NULL: last global error */

/* Kernel timing with HIP events recorded on the handle's stream around each
 * launch group (names: "eval_points", "eval_edges", "eval_nodes",
 * "energy_final", "assemble", "coarse_matrix", "coarse_invert", "cg_init", "cg_step",
 * "residual64", "anderson").  amm_enable_timing(h, 1, NULL) times every
 * group, (h, 1, name) only that group, (h, 0, NULL) stops; enabling clears
 * the totals.  amm_kernel_times returns, per group seen since, the summed
 * milliseconds and the launch count: names[i], ms[i], launches[i] for
 * i < min(*count, capacity). */
amm_status amm_enable_timing(amm_handle* h, int32_t on, const char* only);
amm_status amm_kernel_times(amm_handle* h, const char** names, double* ms, int32_t* launches,
                            int32_t capacity, int32_t* count);

/* Version string of the library build. */
const char* amm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* AMM_H */
