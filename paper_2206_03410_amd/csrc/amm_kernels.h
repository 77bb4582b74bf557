// Kernel argument blocks and launchers (internal).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "amm_internal.h"

namespace amm {

template <typename T> struct V4Of;
template <> struct V4Of<float> { using type = float4; };
template <> struct V4Of<double> { using type = double4; };

constexpr int kAaParts = 72;   // >= m(m+1)/2 + m for m = AMM_MAX_AA_M

// Records HIP events around launches on a stream and sums their durations
// per kernel name (host side; enabled on demand).
struct KernelTimer {
    virtual void begin(const char* name, hipStream_t s) = 0;
    virtual void end(hipStream_t s) = 0;
    // Events to attach to the next single-kernel dispatch of group `name`
    // (false: the group is not timed).
    virtual bool dispatch(const char* name, hipEvent_t* start, hipEvent_t* stop) = 0;
    virtual ~KernelTimer() {}
};

// Launches one kernel.  When the timer times `name`, the start and stop
// events ride on the dispatch packet itself (hipExtLaunchKernel), so the
// measured time is the kernel's own execution, without the host's launch
// latency that events recorded around the launch would include.
template <typename F, typename... Args>
void launch_one(KernelTimer* tm, const char* name, F kernel, dim3 grid, dim3 block, hipStream_t s,
                Args... args) {
    hipEvent_t e0, e1;
    if (tm && tm->dispatch(name, &e0, &e1))
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

template <typename T>
struct EvalArgs {
    using V = typename V4Of<T>::type;
    const int4* pt_tiles;
    const int4* eg_tiles;
    const int4* nd_tiles;
    const PairInfo* info;
    const PairDyn* dyn;
    const V* src;
    const V* src_override;   // internal-order source positions replacing src, or null
    const int* iidx;
    const T* iw;
    int k;
    int64_t Ntot;
    const V* nodes;
    const V* tgt;
    const int* grid;         // per pair, the target octree's run-start tables (PairInfo.grid_off)
    const int* adj_row;
    const int* adj_nbr;
    const T* adj_r;
    T* X[3];                 // transform sets 0, 1 and the MM update G(X^k)
    V* vhat[2];
    int* rho[2];             // global index into the sorted targets
    T* d2[2];
    V* qw[2];                // (e_i = v_hat_i - u_rho(i), w_a,i)
    T* wr[2];                // w_r per directed entry
    V* Dres[2];              // (D, |D|^2) per directed entry
    T* R[2];                 // proj(A_j) - A_j, row-major 3x3
    double* pt_part;
    double* pt_max;
    double* eg_part;
    double* nd_part;
    long long* nn_work;      // per point tile: queries, cell bound tests, distance evaluations,
                             // cell expansions read from memory (or null)
    int nn_budget;           // search steps before a point is deferred (0: never)
    int2* far_list;          // [Ntot] deferred points (point, pair)
    int* far_seed;           // [Ntot] a deferred point's best target so far (sorted position, or -1)
    int* far_count;          // zero between evaluations
    T* pt_psi;               // [Ntot] each point's alignment term
    T* pt_disp;              // [Ntot] each point's displacement
};

struct FinalArgs {
    const PairInfo* info;
    const PairDyn* dyn;
    PairOut* out;
    const double* pt_part;
    const double* pt_max;
    const double* eg_part;
    const double* nd_part;
};

template <typename T>
struct AsmArgs {
    using V = typename V4Of<T>::type;
    const PairDyn* dyn;
    const int* node_pair;
    const V* src;
    const int* iidx;
    const T* iw;
    int k;
    int64_t Ntot;
    const V* nodes;
    const int* K_ptr;
    const int* K_col;
    const int* K_adj;
    const int* pj_ptr;
    const int* pj_ent;
    const uint64_t* pj_pos;  // per entry: byte b = column position of influence b
    const T* iw_pt;          // [Ntot][kMaxK] influence weights, point-major
    const int* adj_ptr;
    const int* adj_nbr;
    const int* adj_rev;
    const T* adj_r;
    const V* qw[2];          // (e_i = v_hat_i - u_rho(i), w_a,i)
    const T* wr[2];
    const V* Dres[2];
    const T* R[2];
    const T* X[2];
    T* Kval;
    T* B;
    T* rvec;                 // r = B - K X^k
    T* Dinv;
};

// Per solver tile, per step parity: (r,u), (w,u), (r,r) per column, then the
// tile's part of P^T w (12 values, [4][3]) for the coarse level.
constexpr int kCgPart = 21;

template <typename T>
struct CgArgs {
    using V = typename V4Of<T>::type;
    const int4* nd_tiles;
    const PairInfo* info;
    const PairDyn* dyn;
    const int* K_ptr;
    const int* K_col;
    const T* Kval;
    const T* Dinv;
    const T* b;
    const T* bnorm;          // vector whose norm scales the stopping test (null: b)
    T* x;
    T* pv;
    T* r[2];                 // r, u, w, s double-buffered by step parity
    T* u[2];
    T* w[2];
    T* s[2];
    double* part[2];         // [tile][kCgPart] partials of the vectors of each parity
    double* part_bb;         // [tile][3] (n,n) of the stopping-test scale
    CgState* state;          // [P][2]
    double rtol2;
    double floor2;           // also stop once (r,r) <= floor2 (r0,r0) (0: off)
    // two-level preconditioner (coarse = 1): M^{-1} = D^{-1} + P A_c^{-1} P^T
    // with an affine field per aggregate of nodes
    int coarse;
    const T* Ainv;           // per pair, dense inverse of A_c = P^T K P (row-major)
    const V* node_rel;       // node position minus its aggregate's centroid
    const int* tile_agg_ptr; // aggregates (pair-local) each tile's rows of K touch
    const int* tile_agg;
    const int* tile_cols;    // [tiles][kTileColCap] distinct column nodes of each tile
    const int* tile_ncols;   // [tiles] their count (> kTileColCap: no list)
    const int* tile_rowl;    // [tiles][kNodeTile] local index of each row's node
    const uint16_t* K_lcol;  // [nnzb] local index of each block's column
    T* gr[2];                // [nagg][12] P^T r per aggregate
    T* gs[2];                // [nagg][12] P^T s per aggregate
    // host-visible [P][2]: last step reported; at convergence one 64-bit word
    // (iterations << 32) | (breakdown << 60) | step of convergence
    long long* prog;
};

template <typename T>
struct CoarseArgs {
    using V = typename V4Of<T>::type;
    const int4* aggs;        // [nagg] pair, first node, end node, pair-local id
    const int4* nd_tiles;
    const int* tile_agg_ptr;
    const int* tile_agg;
    const PairInfo* info;
    const PairDyn* dyn;
    const int* K_ptr;
    const int* K_col;
    const T* Kval;
    const V* node_rel;
    double* Ac_tile;         // [nd_tiles][kCoarseMaxAgg][16] per-tile partial coarse rows
    double* Ac;              // float64 coarse matrices
    T* Ainv;
};

template <typename T>
struct NodeVecArgs {
    const int4* nd_tiles;
    const PairDyn* dyn;
    int flag;
    int op;
    double* x64;
    const T* src_t;
    T* dst_t;
    T* X[3];
};

template <typename T>
struct AaArgs {
    const int4* nd_tiles;
    const PairDyn* dyn;
    const PairOut* out;
    int64_t ntot;
    T* G;                    // ring [(m+1)][ntot*12]
    double* F;               // residual history in float64: its differences cancel
    T* X[3];
    const double* dx;        // increment X' - X^k (float64)
    double* part;            // [nd_tiles][kAaParts]
};

struct AaSolveArgs {
    const PairInfo* info;
    const PairDyn* dyn;
    PairOut* out;
    const double* part;
    int P;
};

template <typename T>
struct GradArgs {
    using V = typename V4Of<T>::type;
    const int4* pt_tiles;
    const PairInfo* info;
    const PairDyn* dyn;
    const int* node_pair;
    const V* src;
    const V* src_override;
    const int* src_user;
    const int* node_user;
    const int* iidx;
    const T* iw;
    int k;
    int64_t Ntot;
    const V* nodes;
    const V* tgt;
    const int* pj_ptr;
    const int* pj_ent;
    const int* adj_ptr;
    const int* adj_nbr;
    const int* adj_rev;
    const T* adj_r;
    const T* X;
    const V* vhat[2];
    const int* rho[2];
    const T* d2[2];
    const V* qw[2];
    const V* Dres[2];
    const T* R[2];
    V* gpt;
    T* gX;                   // user node order
    T* gV;                   // user point order, may be null
};

// Per-pair parameters carried to the device in the kernel arguments of a
// small copy kernel (no host-memory access by the GPU, no blit), in packs of
// 1, 8 or 32 so that the arguments are no larger than the pairs sent.
constexpr int kDynPerLaunch = 32;
template <int N>
struct DynPack {
    PairDyn d[N];
    PairDyn* dst;
    int n;
};
void launch_dyn_set(const PairDyn* src, int n, PairDyn* dst, hipStream_t s);

template <typename T>
void launch_eval(const EvalArgs<T>& a, int n_pt_tiles, int n_eg_tiles, int n_nd_tiles, const FinalArgs& f,
                 int P, hipStream_t s, KernelTimer* tm);
template <typename T>
void launch_assemble(const AsmArgs<T>& a, int64_t ntot, hipStream_t s, KernelTimer* tm);
// CG on K x = b from x = 0 for the pairs flagged PF_SOLVE: the start
// (r = b, u = M^{-1} r, w = K u), then one fused update + product per step.
template <typename T>
void launch_cg_init(const CgArgs<T>& a, int n_nd_tiles, hipStream_t s, KernelTimer* tm);
template <typename T>
void launch_cg_iter(const CgArgs<T>& a, int n_nd_tiles, int it, hipStream_t s, KernelTimer* tm);
// Coarse matrices A_c = P^T K P and their inverses for the pairs flagged PF_SOLVE.
template <typename T>
void launch_coarse(const CoarseArgs<T>& a, int n_nd_tiles, int64_t nagg, int P, hipStream_t s, KernelTimer* tm);
template <typename T>
void launch_residual64(const CgArgs<T>& a, int n_nd_tiles, const T* B, const T* Bn, const double* x64,
                       T* rhs_out, double* part_rr, double* part_bb, hipStream_t s, KernelTimer* tm);
template <typename T>
void launch_node_vec_op(const NodeVecArgs<T>& a, int n_nd_tiles, hipStream_t s);
template <typename T>
void launch_aa(const AaArgs<T>& a, const AaSolveArgs& sa, int n_nd_tiles, hipStream_t s, KernelTimer* tm);
template <typename T>
void launch_grad(const GradArgs<T>& a, int n_pt_tiles, int64_t ntot, hipStream_t s);
template <typename T, typename U>
void launch_x_import(const U* xu, T* xi, const int* node_user, int64_t ntot, hipStream_t s);
template <typename T, typename U>
void launch_x_export(const T* xi, U* xu, const int* node_user, int64_t ntot, hipStream_t s);
template <typename T, typename U>
void launch_src_import(const U* su, void* si, const int* src_user, int64_t Ntot, hipStream_t s);
template <typename T, typename U>
void launch_points_export(const void* vi, U* vu, const int* src_user, int64_t Ntot, hipStream_t s);
template <typename T, typename U>
void launch_nn_export(const int* rho, const T* d2, const int* src_user, const int* tgt_user, int32_t* rho_u,
                      U* d2_u, int64_t Ntot, hipStream_t s);
template <typename T>
void launch_cast_static(const double* in, T* out, int64_t n, hipStream_t s);
// out[2 p + r] = the (N_p / 2 - 1 + r)-th smallest of pair p's d2 values
// (exact); work: device memory of select_mid_work_bytes(P)
template <typename T>
void launch_select_mid(const T* d2, const PairInfo* info, const int4* pt_tiles, int n_pt_tiles, int P, T* out,
                       void* work, hipStream_t s);
size_t select_mid_work_bytes(int P);
// out[i][a] = iw[a][i] for a < k, 0 for k <= a < kMaxK (the influence
// weights point-major, for the assembly)
template <typename T>
void launch_weights_point_major(const T* iw, int k, int64_t N, T* out, hipStream_t s);

}  // namespace amm
