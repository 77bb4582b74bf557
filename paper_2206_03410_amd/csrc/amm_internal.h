// Internal declarations shared by the host setup, the kernels and the C ABI
// layer.  Not part of the public interface.
#pragma once

#include <cstdint>
#include <memory>
#include <utility>
#include <string>
#include <vector>

#include "amm.h"

namespace amm {

// Static description of one pair inside a batch (all offsets are into the
// concatenated arrays; counts are this pair's).
struct PairInfo {
    int64_t src_off, N;      // source points (internal, Morton order)
    int64_t tgt_off, M;      // target points (sorted by Morton code)
    int64_t node_off, n;     // graph nodes (internal, Morton order)
    int64_t adj_off, nadj;   // directed adjacency entries (2 |E_G|)
    int32_t pt_tile0, pt_ntile;   // point tiles
    int32_t nd_tile0, nd_ntile;   // node tiles (solver rows)
    int32_t eg_tile0, eg_ntile;   // edge tiles
    int32_t n_undirected;
    // coarse level of the CG preconditioner: aggregates of 2^agg_shift
    // consecutive (Morton-ordered) nodes, agg0 = first global aggregate,
    // nagg <= kCoarseMaxAgg; the dense inverse of the coarse matrix (order
    // 4 nagg) starts at ainv_off
    int32_t agg0, nagg, agg_shift;
    int64_t ainv_off;
    // closest-point octree over the targets: a cell of level l holds the
    // targets whose 10-bit quantized coordinates floor((x - glo) gscale)
    // share their top l bits on every axis, i.e. a Morton prefix of the
    // targets' sort order.  Level l's 8^l + 1 run starts begin at grid_off +
    // oct_level_off(l), for l = 0..grid_bits (the leaf level).  cs: the root
    // cell's size per axis, 1024 / gscale (0 on a flat axis); gpad: a
    // distance margin covering the rounding of cell bounds and of the
    // targets' stored coordinates
    int64_t grid_off;
    int32_t grid_bits, pad_g;
    double glo[3], gscale[3], cs[3], gpad;
};

// Dynamic per-pair state the host writes before launches.
enum : int32_t {
    PF_ACTIVE = 1,       // pair takes part in this MM iteration
    PF_EVAL = 2,         // evaluate energy at the candidate transforms
    PF_SOLVE = 4,        // assemble and solve
};

struct PairDyn {
    double nu_a, nu_r, alpha, beta;
    int32_t flags;
    int32_t cur;             // which eval/transform set holds the accepted iterate
    int32_t eval_dst;        // set written by the next evaluation
    int32_t eval_x;          // which transform buffer the next evaluation reads (0,1 = X sets, 2 = Xp)
    int32_t aa_mk;           // Anderson window m_k for this iteration
    int32_t aa_slot[11];     // ring slots: [0] = newest (k), [1] = k-1, ...
    int32_t has_prev;        // closest-point warm start available in set `cur`
    int32_t robust;          // amm_robust
    int32_t pad_c, pad_d;
    double cg_rtol;          // CG stopping tolerance of this pair (0: the launch's)
};

// Per-pair outputs read back by the host after an evaluation.
struct PairOut {
    double E, Ea, Er, Eo;    // energy and terms of the last evaluation
    double maxdisp;          // max |v_hat(eval) - v_hat(cur)|
    double aa_used;          // 1 if the Anderson candidate differs from G(X^k)
    double theta[10];
};

// CG state per pair, per column (double-buffered by iteration parity).
struct CgState {
    double alpha[3], gamma[3];
    double rr[3], bb[3];
    double rr0[3];           // (r, r) at the start of the solve
    int32_t conv[3];
    int32_t iters;
    int32_t breakdown;
    int32_t pad;
};

// Host copy of one validated problem (float64).
struct HostPair {
    int64_t N = 0, M = 0, n = 0, E = 0;
    int k = 0;
    std::vector<double> src, tgt, src_nrm, tgt_nrm, infl_w;
    std::vector<int32_t> node_idx, infl_idx, edges;
    double lbar = 0.0;
};

// std::vector whose resize leaves new elements uninitialised: large host
// arrays that the set-up writes in full, from parallel threads (which then
// also take the pages' first-touch cost, instead of one zero-filling thread)
template <typename T>
struct UninitAlloc : std::allocator<T> {
    template <typename U>
    struct rebind {
        using other = UninitAlloc<U>;
    };
    UninitAlloc() = default;
    template <typename U>
    UninitAlloc(const UninitAlloc<U>&) {}
    template <typename U, typename... A>
    void construct(U* p, A&&... a) {
        if constexpr (sizeof...(A) == 0)
            ::new ((void*)p) U;
        else
            ::new ((void*)p) U(std::forward<A>(a)...);
    }
};
template <typename T>
using hvec = std::vector<T, UninitAlloc<T>>;

// Everything set_problems uploads (built on the host).
struct Layout {
    int P = 0, k = 0;
    int64_t Ntot = 0, Mtot = 0, ntot = 0, nadj = 0, nnzb = 0, pj_entries = 0;
    int n_pt_tiles = 0, n_nd_tiles = 0, n_eg_tiles = 0;
    std::vector<PairInfo> info;
    hvec<double> src4;        // [Ntot][4] internal order
    hvec<int32_t> src_user;   // internal point -> user index (concatenated)
    hvec<int32_t> src_internal;  // user index -> internal point
    hvec<int32_t> iidx;       // [k][Ntot] internal node ids
    hvec<double> iw;          // [k][Ntot]
    hvec<uint8_t> ipad;       // [k][Ntot] 1 = unused slot (host only)
    std::vector<double> nodes4;      // [ntot][4]
    std::vector<int32_t> node_user;  // internal node -> user node (concatenated)
    std::vector<int32_t> node_internal;
    std::vector<int32_t> node_pair;  // internal node -> pair
    std::vector<int32_t> adj_ptr, adj_nbr, adj_row, adj_rev;   // directed CSR
    std::vector<double> adj_r;       // r_ij of Eq. (8)
    std::vector<int32_t> K_ptr, K_diag;
    hvec<int32_t> K_col, K_adj;           // written in full by the merge of the pairs' parts
    std::vector<int32_t> pj_ptr;
    hvec<int32_t> pj_ent;   // points influenced by each node: (pt << 3) | slot (written by the pairs' threads)
    // per point-list entry of row j: byte b = position, within row j's column
    // list, of the point's influence b
    hvec<uint64_t> pj_pos;
    hvec<double> tgt4;        // [Mtot][4] sorted; w = user index within the pair
    hvec<int32_t> tgt_user;   // sorted position -> user index within the pair
    std::vector<int32_t> pt_tiles, nd_tiles, eg_tiles;   // [tiles][4] = pair, start, end, 0
    int max_row_cols = 0;
    // coarse level: per aggregate (pair, first node, end node, pair-local id),
    // node position minus its aggregate's centroid, and per node tile the
    // sorted pair-local aggregates that its rows of K touch
    int64_t nagg = 0, ainv_size = 0;
    std::vector<int32_t> aggs;       // [nagg][4]
    std::vector<double> node_rel;    // [ntot][4]
    std::vector<int32_t> tile_agg_ptr, tile_agg;
    hvec<int32_t> grid_cells;   // per pair, the target octree's run-start tables
    // per node tile, the distinct column nodes of its rows of K (sorted;
    // [tiles][kTileColCap], padded with the first), their count (a tile with
    // more than kTileColCap has no list), the local index of every K block's
    // column in its tile's list, and of every row's own node
    std::vector<int32_t> tile_cols, tile_ncols, tile_rowl;
    std::vector<uint16_t> K_lcol;
};

constexpr int kPointTile = 256;
constexpr int kNodeTile = 16;        // solver rows per tile (4 threads per row: one wave)
constexpr int kEdgeTile = 256;
constexpr int kMaxCols = 192;        // K blocks per row supported by the assembly
static_assert(kMaxCols < 255, "column positions are stored in one byte");
constexpr unsigned kPosUnused = 255;  // column byte of an unused influence slot

// Offset of level l's run-start table within a pair's concatenated octree
// tables: the sum over j < l of (8^j + 1).
constexpr int64_t oct_level_off(int l) { return ((int64_t(1) << (3 * l)) - 1) / 7 + l; }
// Levels whose tables a block of the evaluation kernel copies to LDS
// (levels 0..4: 4,686 starts, 18.7 KB); deeper tables are read from memory.
constexpr int kOctLdsLevels = 4;
constexpr int kOctLdsInts = (int)oct_level_off(kOctLdsLevels + 1);
constexpr int kOctMaxDepth = 8;

// One pair's targets in search order: [M][4] (w = user index), the user
// index per position, and the octree's run-start tables of levels
// 0..grid_bits, concatenated.  The depth is the smallest in 2..8 whose
// occupied leaf cells hold at most `leaf` targets on average (8 if none),
// unless `depth` (2..8) fixes it.
struct TargetLayout {
    std::vector<double> tgt4;
    std::vector<int32_t> tgt_user;
    int32_t grid_bits = 0;
    double glo[3] = {0, 0, 0}, gscale[3] = {0, 0, 0}, cs[3] = {0, 0, 0}, gpad = 0;
    std::vector<int32_t> cells;      // sum over l <= grid_bits of (8^l + 1)
};
void target_layout(const double* tgt, int64_t M, int leaf, TargetLayout& out, int depth = 0);
// glo, gscale, cs and gpad of a target set with bounding box [lo, hi]
void target_frame(const double lo[3], const double hi[3], TargetLayout& out);

// The same layout built on the device for a target set whose octree depth is
// already fixed (a pair's targets replaced): tgt (float32 or float64 by
// dtype_f64, M points, device memory) -> sorted targets in both precisions,
// their user indices, the run-start tables (levels 0..depth) and the frame
// fields of `frame`.  The work buffer grows as needed (freed by the caller).
struct DeviceTargetWork {
    void* buf = nullptr;
    size_t bytes = 0;
};
amm_status device_target_layout(void* stream, DeviceTargetWork& w, bool dtype_f64, const void* tgt, int64_t M,
                                int depth, void* tgt_f4, void* tgt_d4, int32_t* tgt_user, int32_t* cells,
                                TargetLayout& frame, std::string& err);

// Device-built deformation graph (Alg. 1), kept by a handle between
// amm_build_graph and amm_graph_copy.  stream is a hipStream_t.
struct GraphBuild;
void graph_release(GraphBuild* g);
amm_status graph_build(void* stream, const amm_graph_in* in, int n_sets, amm_graph_info* info, GraphBuild** out,
                       std::string& err);
amm_status graph_copy(const GraphBuild* g, void* stream, int set, int32_t* node_src_idx, int32_t* infl_idx,
                      void* infl_w, int32_t* edges, std::string& err);
constexpr int kMaxK = 8;
constexpr int kCoarseMaxAgg = 32;    // aggregates per pair (coarse order <= 128)
constexpr int kTileColCap = 160;     // distinct column nodes of a solver tile shared in LDS
constexpr int kAggMinShift = 6;      // at least 64 nodes (4 node tiles) per aggregate

amm_status validate_pair(const HostPair& hp, std::string& err);
// validate_pair for every pair on host threads; the first failing pair's
// error, prefixed with its index
amm_status validate_pairs(const std::vector<HostPair>& pairs, std::string& err);
// The device layout of a batch; pairs are laid out on host threads and
// merged in order (the result does not depend on the thread count).
amm_status build_layout(const std::vector<HostPair>& pairs, int leaf_size, Layout& L,
                        std::string& err);

}  // namespace amm
