// C ABI of the registration library and the host driver of Alg. 2
// (nu continuation around Anderson-accelerated MM iterations).
//
// The driver keeps per-pair scalar state on the host and launches batched
// kernels over every pair that is still running; per-pair decisions (accept
// the Anderson candidate, end a stage, finish) are taken after one small
// device-to-host copy of the pair energies per MM iteration.
#include <hip/hip_runtime.h>

#include <mutex>

#include <algorithm>
#include <array>
#include <atomic>
#include <thread>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "amm.h"
#include "amm_internal.h"
#include "amm_kernels.h"

using namespace amm;

namespace {

thread_local std::string g_last_error;

const char* kVersion = "amm-gfx950 0.1";
constexpr int kDynRing = 16;
// CG steps in flight ahead of the last one reported.  Steps report every
// 4th step (3, 7, ...) and the host starts from "step -2 reported", so the
// first report (step 3) is launched only if the lookahead is at least 5;
// each step queued past convergence costs an early-exit launch.
constexpr int kCgLookahead = 6;
constexpr int kNnBudgetDefault = 64;
static_assert(kCgLookahead >= 5, "the first progress report (step 3) must be launchable");

struct EventTimer final : KernelTimer {
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Rec> pending;
    const char* cur_name = nullptr;
    hipEvent_t cur_a = nullptr;
    std::string only;        // time only launches of this kernel group (empty: all)
    bool skip = false;
    struct Acc {
        const char* name;
        double ms;
        int n;
    };
    std::vector<Acc> acc;

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        (void)hipEventCreate(&e);
        return e;
    }
    void begin(const char* name, hipStream_t s) override {
        skip = !only.empty() && only != name;
        if (skip) return;
        cur_name = name;
        cur_a = get();
        (void)hipEventRecord(cur_a, s);
    }
    void end(hipStream_t s) override {
        if (skip) return;
        hipEvent_t b = get();
        (void)hipEventRecord(b, s);
        pending.push_back({cur_name, cur_a, b});
    }
    bool dispatch(const char* name, hipEvent_t* start, hipEvent_t* stop) override {
        if (!only.empty() && only != name) return false;
        *start = get();
        *stop = get();
        pending.push_back({name, *start, *stop});
        return true;
    }
    void collect() {
        for (auto& r : pending) {
            (void)hipEventSynchronize(r.b);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, r.a, r.b);
            bool found = false;
            for (auto& x : acc)
                if (std::strcmp(x.name, r.name) == 0) {
                    x.ms += ms;
                    x.n += 1;
                    found = true;
                }
            if (!found) acc.push_back({r.name, (double)ms, 1});
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }
    ~EventTimer() override {
        for (auto& r : pending) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// Carves one device buffer into aligned arrays (or just sums their sizes).
struct Carver {
    char* base = nullptr;
    size_t off = 0;
    template <typename P>
    void take(P*& ptr, size_t count) {
        off = (off + 255) & ~size_t(255);
        ptr = base ? reinterpret_cast<P*>(base + off) : nullptr;
        off += std::max<size_t>(count, 1) * sizeof(P);
    }
};

template <typename T>
struct StaticT {
    typename V4Of<T>::type* src = nullptr;
    T* iw = nullptr;
    T* iw_pt = nullptr;
    typename V4Of<T>::type* nodes = nullptr;
    typename V4Of<T>::type* tgt = nullptr;
    T* adj_r = nullptr;
    typename V4Of<T>::type* node_rel = nullptr;
};

// Dynamic arrays are sized for 8-byte elements and reinterpreted for float.
struct Dyn {
    double* X[3];
    double* x64;
    double* vhat[2];   // 4 per point
    int* rho[2];
    double* d2[2];
    double* qw[2];     // 4 per point
    double* wr[2];
    double* Dres[2];   // 4 per entry
    double* R[2];      // 9 per node
    double* pt_part;
    double* pt_max;
    double* eg_part;
    double* nd_part;
    double* Kval;
    double* B;
    double* rvec;
    double* Dinv;
    double* cg[11];    // x p r0 r1 u0 u1 w0 w1 s0 s1 rhs
    double* part[2];   // [nd_tiles][kCgPart]
    double* part_bb;
    double* gr[2];     // [nagg][12]
    double* gs[2];
    double* Ac_tile;   // [nd_tiles][kCoarseMaxAgg][16]
    double* Ac;        // float64 coarse matrices
    double* Ainv;
    double* part_rr64;
    double* part_bb64;
    double* G;
    double* F;
    double* aa_part;
    double* gpt;       // 4 per point
    double* src_ovr;   // 4 per point
    double* pts_out;   // 4 per point
    double* sel;       // work of the median selection
    int* far_count;    // deferred closest-point searches (zero between evaluations)
    int2* far_list;
    int* far_seed;
    double* pt_psi;    // per point: alignment term and displacement (T)
    double* pt_disp;
};

struct Dev {
    int* iidx;
    int* src_user;
    int* node_user;
    int* node_pair;
    int* adj_ptr;
    int* adj_nbr;
    int* adj_row;
    int* adj_rev;
    int* K_ptr;
    int* K_col;
    int* K_adj;
    int* pj_ptr;
    int* pj_ent;
    uint64_t* pj_pos;
    int* tgt_user;
    int4* pt_tiles;
    int4* nd_tiles;
    int4* eg_tiles;
    int4* aggs;
    int* tile_agg_ptr;
    int* tile_agg;
    int* grid_cells;
    int* tile_cols;
    int* tile_ncols;
    int* tile_rowl;
    uint16_t* K_lcol;
    PairInfo* info;
    PairDyn* dyn;        // slot of dyn_ring used by the next launches
    PairDyn* dyn_ring;   // [kDynRing][P]
    PairOut* out;
    CgState* state;
    double* staging;   // float64 staging for static arrays during upload
    StaticT<float> sf;
    StaticT<double> sd;
    Dyn d;
};

void plan(const Layout& L, Carver& c, Dev& v) {
    const size_t N = L.Ntot, M = L.Mtot, n = L.ntot, na = L.nadj, nb = L.nnzb;
    const size_t npt = L.n_pt_tiles, nnd = L.n_nd_tiles, neg = L.n_eg_tiles;
    const size_t k = L.k;
    c.take(v.iidx, k * N);
    c.take(v.src_user, N);
    c.take(v.node_user, n);
    c.take(v.node_pair, n);
    c.take(v.adj_ptr, n + 1);
    c.take(v.adj_nbr, na);
    c.take(v.adj_row, na);
    c.take(v.adj_rev, na);
    c.take(v.K_ptr, n + 1);
    c.take(v.K_col, nb);
    c.take(v.K_adj, nb);
    c.take(v.pj_ptr, n + 1);
    c.take(v.pj_ent, L.pj_entries);
    c.take(v.pj_pos, L.pj_entries);
    c.take(v.tgt_user, M);
    c.take(v.pt_tiles, npt);
    c.take(v.nd_tiles, nnd);
    c.take(v.eg_tiles, neg);
    c.take(v.aggs, (size_t)L.nagg);
    c.take(v.tile_agg_ptr, nnd + 1);
    c.take(v.tile_agg, L.tile_agg.size());
    c.take(v.grid_cells, L.grid_cells.size());
    c.take(v.tile_cols, L.tile_cols.size());
    c.take(v.tile_ncols, L.tile_ncols.size());
    c.take(v.tile_rowl, L.tile_rowl.size());
    c.take(v.K_lcol, L.K_lcol.size());
    c.take(v.info, L.P);
    c.take(v.dyn_ring, (size_t)kDynRing * L.P);
    v.dyn = v.dyn_ring;
    c.take(v.out, L.P);
    c.take(v.state, 2 * (size_t)L.P);
    size_t stage = std::max({4 * N, 4 * M, (size_t)kMaxK * N, 4 * n, na});
    c.take(v.staging, stage);
    auto statics = [&](auto& s) {
        c.take(s.src, N);
        c.take(s.iw, k * N);
        c.take(s.iw_pt, (size_t)kMaxK * N);
        c.take(s.nodes, n);
        c.take(s.tgt, M);
        c.take(s.adj_r, na);
        c.take(s.node_rel, n);
    };
    statics(v.sf);
    statics(v.sd);
    Dyn& d = v.d;
    for (int q = 0; q < 3; ++q) c.take(d.X[q], 12 * n);
    c.take(d.x64, 12 * n);
    for (int q = 0; q < 2; ++q) {
        c.take(d.vhat[q], 4 * N);
        c.take(d.rho[q], N);
        c.take(d.d2[q], N);
        c.take(d.qw[q], 4 * N);
        c.take(d.wr[q], na);
        c.take(d.Dres[q], 4 * na);
        c.take(d.R[q], 9 * n);
    }
    c.take(d.pt_part, npt);
    c.take(d.pt_max, npt);
    c.take(d.eg_part, neg);
    c.take(d.nd_part, nnd);
    c.take(d.Kval, 16 * nb);
    c.take(d.B, 12 * n);
    c.take(d.rvec, 12 * n);
    c.take(d.Dinv, 16 * n);
    for (int q = 0; q < 11; ++q) c.take(d.cg[q], 12 * n);
    for (int q = 0; q < 2; ++q) {
        c.take(d.part[q], (size_t)kCgPart * nnd);
        c.take(d.gr[q], 12 * (size_t)L.nagg);
        c.take(d.gs[q], 12 * (size_t)L.nagg);
    }
    c.take(d.part_bb, 3 * nnd);
    c.take(d.Ac_tile, nnd * kCoarseMaxAgg * 16);
    c.take(d.Ac, (size_t)L.ainv_size);
    c.take(d.Ainv, (size_t)L.ainv_size);
    c.take(d.part_rr64, 6 * nnd);   // (r,r) then (n,n): read back in one copy
    d.part_bb64 = d.part_rr64 ? d.part_rr64 + 3 * nnd : nullptr;
    c.take(d.G, (AMM_MAX_AA_M + 1) * 12 * n);
    c.take(d.F, (AMM_MAX_AA_M + 1) * 12 * n);
    c.take(d.aa_part, (size_t)kAaParts * nnd);
    c.take(d.gpt, 4 * N);
    c.take(d.src_ovr, 4 * N);
    c.take(d.pts_out, 4 * N);
    c.take(d.sel, (select_mid_work_bytes(L.P) + 7) / 8);
    c.take(d.far_count, 1);
    c.take(d.far_list, N);
    c.take(d.far_seed, N);
    c.take(d.pt_psi, N);
    c.take(d.pt_disp, N);
}

}  // namespace


struct amm_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    void* ws_user = nullptr;
    size_t ws_user_bytes = 0;
    void* ws_own = nullptr;
    size_t ws_own_bytes = 0;
    bool has_problem = false;
    // closest points of evaluation set 0 of pair 0 hold valid target
    // positions (an evaluation wrote them since the last upload): energy and
    // step evaluations then seed their searches with them
    bool rho_set0 = false;
    Layout L;
    Dev v{};
    std::vector<double> lbar;
    std::vector<PairDyn> dyn;        // host working copy of the per-pair parameters
    int dyn_slot = 0;
    PairOut* h_out = nullptr;        // pinned
    CgState* h_state = nullptr;      // pinned
    // CG progress written by the step kernels straight into coherent pinned
    // host memory: [2p] = last step completed, [2p+1] = step at which all
    // three columns had converged (-1 while not)
    long long* prog = nullptr;
    long long* prog_dev = nullptr;
    double* h_scratch = nullptr;     // pinned, grown on demand (small read-backs)
    char* rb_pin = nullptr;          // pinned staging of the problem arrays read back at set-up
    size_t rb_cap = 0;
    hipEvent_t sync_ev = nullptr;    // recorded to wait for the stream by polling
    std::thread freer;               // frees the previous layout after a new set-up
    size_t h_scratch_cap = 0;
    size_t h_cap = 0;
    bool timing = false;
    bool cg_coarse = true;           // two-level CG preconditioner
    int leaf = 8;                    // mean targets per occupied octree leaf cell (next upload)
    int nn_budget = kNnBudgetDefault;   // closest-point search steps before a point goes to the wave search
    long long* nn_work = nullptr;    // [n_pt_tiles][4] search counters while counting is on
    int nn_work_tiles = 0;
    GraphBuild* graph = nullptr;     // last amm_build_graph result
    DeviceTargetWork tw;             // work buffer of the device target layout (amm_set_targets)
    EventTimer timer;
    std::vector<amm_iter_record> iter_log;
};

namespace {

amm_status fail(amm_handle* h, amm_status s, const std::string& msg) {
    if (h) h->err = msg;
    g_last_error = msg;
    return s;
}

#define HIPC(expr)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return fail(h, AMM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
    } while (0)

#define TRY(expr)                          \
    do {                                   \
        amm_status s_ = (expr);            \
        if (s_ != AMM_OK) return s_;       \
    } while (0)

KernelTimer* tmr(amm_handle* h) { return h->timing ? &h->timer : nullptr; }

amm_status read_pair(amm_handle* h, const amm_problem& p, HostPair& hp) {
    if (p.n_src < 1 || p.n_tgt < 1 || p.n_nodes < 1 || p.k < 1 || p.k > kMaxK || p.n_edges < 0)
        return fail(h, AMM_ERR_INVALID_ARG, "bad sizes in amm_problem");
    if (!p.src_xyz || !p.tgt_xyz || !p.node_src_idx || !p.infl_idx || !p.infl_w || (p.n_edges > 0 && !p.edges))
        return fail(h, AMM_ERR_INVALID_ARG, "null array in amm_problem");
    if (p.dtype != AMM_F32 && p.dtype != AMM_F64) return fail(h, AMM_ERR_INVALID_ARG, "bad dtype");
    hp.N = p.n_src;
    hp.M = p.n_tgt;
    hp.n = p.n_nodes;
    hp.E = p.n_edges;
    hp.k = p.k;
    hp.lbar = p.mean_edge_len;
    const size_t es = p.dtype == AMM_F32 ? 4 : 8;
    auto fetch = [&](const void* src, size_t bytes, void* dst) -> bool {
        if (!bytes) return true;
        if (p.on_device) return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost) == hipSuccess;
        std::memcpy(dst, src, bytes);
        return true;
    };
    auto fetch_real = [&](const void* src, size_t count, std::vector<double>& out) -> bool {
        if (!src || !count) {
            out.clear();
            return true;
        }
        out.resize(count);
        if (es == 8) return fetch(src, count * 8, out.data());
        std::vector<float> tmp(count);
        if (!fetch(src, count * 4, tmp.data())) return false;
        for (size_t i = 0; i < count; ++i) out[i] = tmp[i];
        return true;
    };
    if (p.on_device && hipDeviceSynchronize() != hipSuccess)
        return fail(h, AMM_ERR_HIP, "device synchronization failed before reading the problem");
    bool ok = fetch_real(p.src_xyz, 3 * hp.N, hp.src) && fetch_real(p.tgt_xyz, 3 * hp.M, hp.tgt) &&
              fetch_real(p.src_nrm, 3 * hp.N, hp.src_nrm) && fetch_real(p.tgt_nrm, 3 * hp.M, hp.tgt_nrm) &&
              fetch_real(p.infl_w, (size_t)hp.k * hp.N, hp.infl_w);
    hp.node_idx.resize(hp.n);
    hp.infl_idx.resize((size_t)hp.k * hp.N);
    hp.edges.resize(2 * hp.E);
    ok = ok && fetch(p.node_src_idx, 4 * hp.n, hp.node_idx.data()) &&
         fetch(p.infl_idx, 4 * (size_t)hp.k * hp.N, hp.infl_idx.data()) &&
         fetch(p.edges, 8 * (size_t)hp.E, hp.edges.data());
    if (!ok) return fail(h, AMM_ERR_HIP, "could not read the problem arrays");
    return AMM_OK;
}

// The arrays of one problem in reading order: real arrays in the problem's
// element type (optional ones may be null), index arrays as int32.
struct ProblemArray {
    const void* ptr;
    size_t count;         // elements
    bool real;
    size_t off;           // byte offset in the pinned staging buffer (device arrays)
};

// Reads the problems into host pairs.  Arrays on the device are copied
// asynchronously into one pinned staging buffer (kept by the handle) and
// waited for once; each pair's arrays are then converted or copied into its
// host vectors on parallel threads.
amm_status read_pairs(amm_handle* h, const amm_problem* probs, int n_pairs, std::vector<HostPair>& hps) {
    std::vector<std::array<ProblemArray, 8>> arrs(n_pairs);
    size_t staged = 0;
    bool any_device = false;
    for (int q = 0; q < n_pairs; ++q) {
        const amm_problem& p = probs[q];
        HostPair& hp = hps[q];
        if (p.n_src < 1 || p.n_tgt < 1 || p.n_nodes < 1 || p.k < 1 || p.k > kMaxK || p.n_edges < 0)
            return fail(h, AMM_ERR_INVALID_ARG, "bad sizes in amm_problem");
        if (!p.src_xyz || !p.tgt_xyz || !p.node_src_idx || !p.infl_idx || !p.infl_w || (p.n_edges > 0 && !p.edges))
            return fail(h, AMM_ERR_INVALID_ARG, "null array in amm_problem");
        if (p.dtype != AMM_F32 && p.dtype != AMM_F64) return fail(h, AMM_ERR_INVALID_ARG, "bad dtype");
        hp.N = p.n_src;
        hp.M = p.n_tgt;
        hp.n = p.n_nodes;
        hp.E = p.n_edges;
        hp.k = p.k;
        hp.lbar = p.mean_edge_len;
        std::array<ProblemArray, 8>& arr = arrs[q];
        arr[0] = {p.src_xyz, 3 * (size_t)hp.N, true, 0};
        arr[1] = {p.tgt_xyz, 3 * (size_t)hp.M, true, 0};
        arr[2] = {p.src_nrm, p.src_nrm ? 3 * (size_t)hp.N : 0, true, 0};
        arr[3] = {p.tgt_nrm, p.tgt_nrm ? 3 * (size_t)hp.M : 0, true, 0};
        arr[4] = {p.infl_w, (size_t)hp.k * hp.N, true, 0};
        arr[5] = {p.node_src_idx, (size_t)hp.n, false, 0};
        arr[6] = {p.infl_idx, (size_t)hp.k * hp.N, false, 0};
        arr[7] = {p.edges, 2 * (size_t)hp.E, false, 0};
        if (!p.on_device) continue;
        const size_t es = p.dtype == AMM_F32 ? 4 : 8;
        for (ProblemArray& a : arr) {
            if (!a.ptr || !a.count) continue;
            any_device = true;
            a.off = staged;
            staged += (a.count * (a.real ? es : 4) + 255) & ~size_t(255);
        }
    }
    if (any_device) {
        if (h->rb_cap < staged) {
            if (h->rb_pin) (void)hipHostFree(h->rb_pin);
            h->rb_pin = nullptr;
            h->rb_cap = 0;
            HIPC(hipHostMalloc((void**)&h->rb_pin, staged));
            h->rb_cap = staged;
        }
        // the arrays may have been written on other streams
        if (hipDeviceSynchronize() != hipSuccess)
            return fail(h, AMM_ERR_HIP, "device synchronization failed before reading the problems");
        for (int q = 0; q < n_pairs; ++q) {
            if (!probs[q].on_device) continue;
            const size_t es = probs[q].dtype == AMM_F32 ? 4 : 8;
            for (const ProblemArray& a : arrs[q]) {
                if (!a.ptr || !a.count) continue;
                if (hipMemcpyAsync(h->rb_pin + a.off, a.ptr, a.count * (a.real ? es : 4), hipMemcpyDeviceToHost,
                                   h->stream) != hipSuccess)
                    return fail(h, AMM_ERR_HIP, "could not read the problem arrays");
            }
        }
        if (hipStreamSynchronize(h->stream) != hipSuccess)
            return fail(h, AMM_ERR_HIP, "could not read the problem arrays");
    }
    const unsigned hc = std::thread::hardware_concurrency();
    const int threads = (int)std::min<int64_t>(n_pairs, std::min(16u, std::max(1u, hc)));
    std::atomic<int> next{0};
    auto work = [&]() {
        for (int q = next.fetch_add(1); q < n_pairs; q = next.fetch_add(1)) {
            const amm_problem& p = probs[q];
            HostPair& hp = hps[q];
            const bool f32 = p.dtype == AMM_F32;
            std::vector<double>* reals[5] = {&hp.src, &hp.tgt, &hp.src_nrm, &hp.tgt_nrm, &hp.infl_w};
            std::vector<int32_t>* ints[3] = {&hp.node_idx, &hp.infl_idx, &hp.edges};
            for (int a = 0; a < 8; ++a) {
                const ProblemArray& pa = arrs[q][a];
                const void* from = p.on_device ? (const void*)(h->rb_pin + pa.off) : pa.ptr;
                if (pa.real) {
                    std::vector<double>& out = *reals[a];
                    if (!pa.ptr || !pa.count) {
                        out.clear();
                        continue;
                    }
                    out.resize(pa.count);
                    if (f32) {
                        const float* f = static_cast<const float*>(from);
                        for (size_t i = 0; i < pa.count; ++i) out[i] = f[i];
                    } else {
                        std::memcpy(out.data(), from, pa.count * 8);
                    }
                } else {
                    std::vector<int32_t>& out = *ints[a - 5];
                    out.resize(pa.count);
                    if (pa.count) std::memcpy(out.data(), from, pa.count * 4);
                }
            }
        }
    };
    if (threads <= 1) {
        work();
    } else {
        std::vector<std::thread> pool;
        for (int t = 0; t < threads; ++t) pool.emplace_back(work);
        for (auto& th : pool) th.join();
    }
    return AMM_OK;
}

// Uploads of the layout: stream-ordered, with no wait of their own (the
// layout's host arrays outlive them: amm_set_problems waits for the stream
// before it returns, and the uploads through the device staging buffer
// follow one another on the stream).
template <typename P, typename A>
amm_status up(amm_handle* h, P* dst, const std::vector<P, A>& src) {
    if (src.empty()) return AMM_OK;
    HIPC(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(P), hipMemcpyHostToDevice, h->stream));
    return AMM_OK;
}

// uploads a float64 host array and writes its float32 and float64 copies
template <typename PF, typename PD, typename A>
amm_status up_real(amm_handle* h, PF* dst_f, PD* dst_d, const std::vector<double, A>& src) {
    if (src.empty()) return AMM_OK;
    HIPC(hipMemcpyAsync(h->v.staging, src.data(), src.size() * 8, hipMemcpyHostToDevice, h->stream));
    launch_cast_static<float>(h->v.staging, reinterpret_cast<float*>(dst_f), (int64_t)src.size(), h->stream);
    launch_cast_static<double>(h->v.staging, reinterpret_cast<double*>(dst_d), (int64_t)src.size(), h->stream);
    HIPC(hipGetLastError());
    return AMM_OK;
}

amm_status ensure_host(amm_handle* h, size_t P) {
    h->dyn.assign(P, PairDyn{});
    if (P <= h->h_cap) return AMM_OK;
    if (h->h_out) (void)hipHostFree(h->h_out);
    if (h->h_state) (void)hipHostFree(h->h_state);
    if (h->prog) (void)hipHostFree(h->prog);
    h->h_out = nullptr;
    h->h_state = nullptr;
    h->prog = nullptr;
    HIPC(hipHostMalloc((void**)&h->prog, sizeof(long long) * 2 * P, hipHostMallocMapped | hipHostMallocCoherent));
    HIPC(hipHostGetDevicePointer((void**)&h->prog_dev, h->prog, 0));
    HIPC(hipHostMalloc((void**)&h->h_out, sizeof(PairOut) * P));
    HIPC(hipHostMalloc((void**)&h->h_state, sizeof(CgState) * 2 * P));
    h->h_cap = P;
    return AMM_OK;
}

// Uploads the host copy of the per-pair parameters into the next ring slot,
// stream-ordered, through the arguments of a copy kernel (captured at
// launch, so the host copy may change right after); launches built
// afterwards read that slot.
amm_status push_dyn(amm_handle* h) {
    const int P = h->L.P;
    const int slot = (h->dyn_slot + 1) % kDynRing;
    PairDyn* ds = h->v.dyn_ring + (size_t)slot * P;
    for (int b = 0; b < P; b += kDynPerLaunch)
        launch_dyn_set(h->dyn.data() + b, std::min(kDynPerLaunch, P - b), ds + b, h->stream);
    HIPC(hipGetLastError());
    h->dyn_slot = slot;
    h->v.dyn = ds;
    return AMM_OK;
}

// Waits for the handle's stream.  The host is usually waiting for a short
// tail of work: polling an event for up to 2 ms wakes it far sooner than a
// blocking wait; longer waits fall back to blocking.
amm_status sync_spin(amm_handle* h) {
    if (!h->sync_ev) HIPC(hipEventCreateWithFlags(&h->sync_ev, hipEventDisableTiming));
    HIPC(hipEventRecord(h->sync_ev, h->stream));
    const auto t0 = std::chrono::steady_clock::now();
    while (true) {
        const hipError_t q = hipEventQuery(h->sync_ev);
        if (q == hipSuccess) return AMM_OK;
        if (q != hipErrorNotReady) return fail(h, AMM_ERR_HIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) break;
    }
    HIPC(hipEventSynchronize(h->sync_ev));
    return AMM_OK;
}

amm_status pull_out(amm_handle* h) {
    HIPC(hipMemcpyAsync(h->h_out, h->v.out, sizeof(PairOut) * h->L.P, hipMemcpyDeviceToHost, h->stream));
    TRY(sync_spin(h));
    HIPC(hipGetLastError());
    if (h->timing) h->timer.collect();
    return AMM_OK;
}

template <typename T>
const StaticT<T>& statics(const amm_handle* h);
template <>
const StaticT<float>& statics<float>(const amm_handle* h) { return h->v.sf; }
template <>
const StaticT<double>& statics<double>(const amm_handle* h) { return h->v.sd; }

template <typename T>
EvalArgs<T> eval_args(amm_handle* h, bool use_override = false) {
    using V = typename V4Of<T>::type;
    const StaticT<T>& s = statics<T>(h);
    const Dyn& d = h->v.d;
    EvalArgs<T> a{};
    a.pt_tiles = h->v.pt_tiles;
    a.eg_tiles = h->v.eg_tiles;
    a.nd_tiles = h->v.nd_tiles;
    a.info = h->v.info;
    a.dyn = h->v.dyn;
    a.src = s.src;
    a.src_override = use_override ? reinterpret_cast<const V*>(d.src_ovr) : nullptr;
    a.iidx = h->v.iidx;
    a.iw = s.iw;
    a.k = h->L.k;
    a.Ntot = h->L.Ntot;
    a.nodes = s.nodes;
    a.tgt = s.tgt;
    a.grid = h->v.grid_cells;
    a.adj_row = h->v.adj_row;
    a.adj_nbr = h->v.adj_nbr;
    a.adj_r = s.adj_r;
    for (int q = 0; q < 3; ++q) a.X[q] = reinterpret_cast<T*>(d.X[q]);
    for (int q = 0; q < 2; ++q) {
        a.vhat[q] = reinterpret_cast<V*>(d.vhat[q]);
        a.rho[q] = d.rho[q];
        a.d2[q] = reinterpret_cast<T*>(d.d2[q]);
        a.qw[q] = reinterpret_cast<V*>(d.qw[q]);
        a.wr[q] = reinterpret_cast<T*>(d.wr[q]);
        a.Dres[q] = reinterpret_cast<V*>(d.Dres[q]);
        a.R[q] = reinterpret_cast<T*>(d.R[q]);
    }
    a.pt_part = d.pt_part;
    a.pt_max = d.pt_max;
    a.eg_part = d.eg_part;
    a.nd_part = d.nd_part;
    a.nn_work = h->nn_work;
    a.nn_budget = h->nn_budget;
    a.far_count = d.far_count;
    a.far_list = d.far_list;
    a.far_seed = d.far_seed;
    a.pt_psi = reinterpret_cast<T*>(d.pt_psi);
    a.pt_disp = reinterpret_cast<T*>(d.pt_disp);
    return a;
}

FinalArgs final_args(amm_handle* h) {
    FinalArgs f{};
    f.info = h->v.info;
    f.dyn = h->v.dyn;
    f.out = h->v.out;
    f.pt_part = h->v.d.pt_part;
    f.pt_max = h->v.d.pt_max;
    f.eg_part = h->v.d.eg_part;
    f.nd_part = h->v.d.nd_part;
    return f;
}

template <typename T>
AsmArgs<T> asm_args(amm_handle* h) {
    using V = typename V4Of<T>::type;
    const StaticT<T>& s = statics<T>(h);
    const Dyn& d = h->v.d;
    AsmArgs<T> a{};
    a.dyn = h->v.dyn;
    a.node_pair = h->v.node_pair;
    a.src = s.src;
    a.iidx = h->v.iidx;
    a.iw = s.iw;
    a.k = h->L.k;
    a.Ntot = h->L.Ntot;
    a.nodes = s.nodes;
    a.K_ptr = h->v.K_ptr;
    a.K_col = h->v.K_col;
    a.K_adj = h->v.K_adj;
    a.pj_ptr = h->v.pj_ptr;
    a.pj_ent = h->v.pj_ent;
    a.pj_pos = h->v.pj_pos;
    a.iw_pt = s.iw_pt;
    a.adj_ptr = h->v.adj_ptr;
    a.adj_nbr = h->v.adj_nbr;
    a.adj_rev = h->v.adj_rev;
    a.adj_r = s.adj_r;
    for (int q = 0; q < 2; ++q) {
        a.qw[q] = reinterpret_cast<const V*>(d.qw[q]);
        a.wr[q] = reinterpret_cast<const T*>(d.wr[q]);
        a.Dres[q] = reinterpret_cast<const V*>(d.Dres[q]);
        a.R[q] = reinterpret_cast<const T*>(d.R[q]);
        a.X[q] = reinterpret_cast<const T*>(d.X[q]);
    }
    a.Kval = reinterpret_cast<T*>(d.Kval);
    a.B = reinterpret_cast<T*>(d.B);
    a.rvec = reinterpret_cast<T*>(d.rvec);
    a.Dinv = reinterpret_cast<T*>(d.Dinv);
    return a;
}

template <typename T>
CgArgs<T> cg_args(amm_handle* h, const T* b, const T* bnorm, double rtol) {
    const Dyn& d = h->v.d;
    CgArgs<T> a{};
    a.nd_tiles = h->v.nd_tiles;
    a.info = h->v.info;
    a.dyn = h->v.dyn;
    a.K_ptr = h->v.K_ptr;
    a.K_col = h->v.K_col;
    a.Kval = reinterpret_cast<const T*>(d.Kval);
    a.Dinv = reinterpret_cast<const T*>(d.Dinv);
    a.b = b;
    a.bnorm = bnorm;
    a.x = reinterpret_cast<T*>(d.cg[0]);
    a.pv = reinterpret_cast<T*>(d.cg[1]);
    for (int q = 0; q < 2; ++q) {
        a.r[q] = reinterpret_cast<T*>(d.cg[2 + q]);
        a.u[q] = reinterpret_cast<T*>(d.cg[4 + q]);
        a.w[q] = reinterpret_cast<T*>(d.cg[6 + q]);
        a.s[q] = reinterpret_cast<T*>(d.cg[8 + q]);
        a.part[q] = d.part[q];
        a.gr[q] = reinterpret_cast<T*>(d.gr[q]);
        a.gs[q] = reinterpret_cast<T*>(d.gs[q]);
    }
    a.part_bb = d.part_bb;
    a.state = h->v.state;
    a.rtol2 = rtol * rtol;
    a.coarse = h->cg_coarse ? 1 : 0;
    a.Ainv = reinterpret_cast<const T*>(d.Ainv);
    a.node_rel = statics<T>(h).node_rel;
    a.tile_agg_ptr = h->v.tile_agg_ptr;
    a.tile_agg = h->v.tile_agg;
    a.tile_cols = h->v.tile_cols;
    a.tile_ncols = h->v.tile_ncols;
    a.tile_rowl = h->v.tile_rowl;
    a.K_lcol = h->v.K_lcol;
    a.prog = h->prog_dev;
    return a;
}

template <typename T>
CoarseArgs<T> coarse_args(amm_handle* h) {
    const Dyn& d = h->v.d;
    CoarseArgs<T> a{};
    a.aggs = h->v.aggs;
    a.nd_tiles = h->v.nd_tiles;
    a.tile_agg_ptr = h->v.tile_agg_ptr;
    a.tile_agg = h->v.tile_agg;
    a.info = h->v.info;
    a.dyn = h->v.dyn;
    a.K_ptr = h->v.K_ptr;
    a.K_col = h->v.K_col;
    a.Kval = reinterpret_cast<const T*>(d.Kval);
    a.node_rel = statics<T>(h).node_rel;
    a.Ac_tile = d.Ac_tile;
    a.Ac = d.Ac;
    a.Ainv = reinterpret_cast<T*>(d.Ainv);
    return a;
}

template <typename T>
void vec_op(amm_handle* h, int flag, int op, const T* src = nullptr, T* dst = nullptr) {
    NodeVecArgs<T> a{};
    a.nd_tiles = h->v.nd_tiles;
    a.dyn = h->v.dyn;
    a.flag = flag;
    a.op = op;
    a.x64 = h->v.d.x64;
    a.src_t = src;
    a.dst_t = dst;
    for (int q = 0; q < 3; ++q) a.X[q] = reinterpret_cast<T*>(h->v.d.X[q]);
    launch_node_vec_op<T>(a, h->L.n_nd_tiles, h->stream);
}

template <typename T>
amm_status evaluate(amm_handle* h, bool use_override = false) {
    TRY(push_dyn(h));
    launch_eval<T>(eval_args<T>(h, use_override), h->L.n_pt_tiles, h->L.n_eg_tiles, h->L.n_nd_tiles,
                   final_args(h), h->L.P, h->stream, tmr(h));
    if ((h->dyn[0].flags & PF_EVAL) && h->dyn[0].eval_dst == 0) h->rho_set0 = true;
    return pull_out(h);
}

// Sum over a pair's node tiles of a [tiles][3] partial array, on the host.
void pair_sums3(const Layout& L, const double* part, int p, double out[3]) {
    const PairInfo& pi = L.info[p];
    out[0] = out[1] = out[2] = 0;
    for (int t = 0; t < pi.nd_ntile; ++t)
        for (int c = 0; c < 3; ++c) out[c] += part[3 * (pi.nd_tile0 + t) + c];
}

struct SolveReport {
    std::vector<int64_t> cg_iters;
    std::vector<int> refine;
    std::vector<double> rel;   // worst final relative residual |B - K X| / |B| over the 3 columns
    bool not_spd = false;
    int bad_pair = -1;
};

// CG over the pairs flagged PF_SOLVE until all their columns converged.
// The host never copies state back inside the loop: the step kernels report
// their progress in coherent pinned host memory, and the host keeps at most
// kCgLookahead steps in flight, stopping as soon as every pair reports
// convergence (steps already queued return at once for converged pairs).
// Adds each pair's iteration count to rep.
template <typename T>
amm_status run_cg(amm_handle* h, const T* b, const T* bnorm, double rtol, int maxit, SolveReport& rep,
                  double floor = 0.0) {
    const Layout& L = h->L;
    const int nt = L.n_nd_tiles;
    const int P = L.P;
    volatile long long* pg = h->prog;
    for (int p = 0; p < P; ++p) {
        pg[2 * p] = -2;
        pg[2 * p + 1] = -1;
    }
    std::atomic_thread_fence(std::memory_order_seq_cst);
    CgArgs<T> a = cg_args<T>(h, b, bnorm, rtol);
    a.floor2 = floor * floor;
    launch_cg_init<T>(a, nt, h->stream, tmr(h));
    // the step at which pair p converged (low 32 bits of its word), or -1
    auto conv_step = [&](int p) { return (int)(unsigned)(pg[2 * p + 1] & 0xffffffffll); };
    auto all_converged = [&]() {
        for (int p = 0; p < P; ++p)
            if ((h->dyn[p].flags & PF_SOLVE) && conv_step(p) < 0) return false;
        return true;
    };
    auto slowest = [&]() {
        long long m = LLONG_MAX;
        for (int p = 0; p < P; ++p)
            if ((h->dyn[p].flags & PF_SOLVE) && conv_step(p) < 0) m = std::min(m, (long long)pg[2 * p]);
        return m;
    };
    int launched = 0;
    bool done = false;
    for (int it = 0; it < maxit && !done; ++it) {
        if (it > 0 && all_converged()) {
            done = true;
            break;
        }
        const auto t_wait = std::chrono::steady_clock::now();
        while (it - slowest() > kCgLookahead) {
            if (all_converged()) {
                done = true;
                break;
            }
            if (std::chrono::steady_clock::now() - t_wait > std::chrono::seconds(60)) {
                (void)hipStreamSynchronize(h->stream);
                return fail(h, AMM_ERR_HIP, "CG steps made no progress for 60 s");
            }
        }
        if (done) break;
        launch_cg_iter<T>(a, nt, it, h->stream, tmr(h));
        launched = it + 1;
    }
    HIPC(hipGetLastError());
    if (!done) {
        // the step budget ran out before every pair converged: wait for the
        // queued steps and read the state back
        HIPC(hipMemcpyAsync(h->h_state, h->v.state, sizeof(CgState) * 2 * P, hipMemcpyDeviceToHost, h->stream));
        HIPC(hipStreamSynchronize(h->stream));
        if (h->timing) h->timer.collect();
        if (launched == 0) return AMM_OK;
        const int last = launched - 1;
        for (int p = 0; p < P; ++p) {
            if (!(h->dyn[p].flags & PF_SOLVE)) continue;
            rep.cg_iters[p] += h->h_state[2 * p + (last & 1)].iters;
        }
        return AMM_OK;
    }
    // every pair converged: iterations and breakdown flags come with the
    // convergence word, no read-back needed
    for (int p = 0; p < P; ++p) {
        if (!(h->dyn[p].flags & PF_SOLVE)) continue;
        const long long w = pg[2 * p + 1];
        rep.cg_iters[p] += (int)((w >> 32) & 0x0fffffff);
        const int brk = (int)((w >> 60) & 7);
        h->h_state[2 * p].breakdown = h->h_state[2 * p + 1].breakdown = brk;
    }
    return AMM_OK;
}

// true residual |r - K dx| / |B| per pair (worst column) of the increment
// system K dx = r = B - K X^k, i.e. |B - K X'| / |B| for X' = X^k + dx.
// Grows the handle's pinned host scratch to at least `bytes`.  Callers
// synchronize before reusing it, so no copy into the old buffer is pending.
amm_status pinned_scratch(amm_handle* h, size_t bytes) {
    const size_t need = (bytes + 7) / 8;
    if (h->h_scratch_cap >= need) return AMM_OK;
    if (h->h_scratch) (void)hipHostFree(h->h_scratch);
    h->h_scratch = nullptr;
    h->h_scratch_cap = 0;
    HIPC(hipHostMalloc((void**)&h->h_scratch, sizeof(double) * need));
    h->h_scratch_cap = need;
    return AMM_OK;
}

template <typename T>
amm_status true_residual(amm_handle* h, T* rhs_out, std::vector<double>& rel) {
    const Layout& L = h->L;
    Dyn& d = h->v.d;
    const int nt = L.n_nd_tiles;
    CgArgs<T> a = cg_args<T>(h, nullptr, nullptr, 0);
    launch_residual64<T>(a, nt, reinterpret_cast<const T*>(d.rvec), reinterpret_cast<const T*>(d.B), d.x64, rhs_out,
                         d.part_rr64, d.part_bb64, h->stream, tmr(h));
    // read back into pinned memory (a pageable destination makes the copy
    // synchronous and staged)
    TRY(pinned_scratch(h, sizeof(double) * 6 * nt));
    double* rr = h->h_scratch;
    double* bb = h->h_scratch + 3 * nt;
    HIPC(hipMemcpyAsync(rr, d.part_rr64, sizeof(double) * 6 * nt, hipMemcpyDeviceToHost, h->stream));
    TRY(sync_spin(h));
    rel.assign(L.P, 0.0);
    for (int p = 0; p < L.P; ++p) {
        if (!(h->dyn[p].flags & PF_SOLVE)) continue;
        double r3[3], b3[3];
        pair_sums3(L, rr, p, r3);
        pair_sums3(L, bb, p, b3);
        for (int c = 0; c < 3; ++c) rel[p] = std::max(rel[p], b3[c] > 0 ? std::sqrt(r3[c] / b3[c]) : std::sqrt(r3[c]));
    }
    return AMM_OK;
}

// Solves the normal equations K X' = B (Eq. 21) for the pairs flagged
// PF_SOLVE as the increment system K dx = r (r = B - K X^k, assembled in
// residual form), X' = X^k + dx; dx is left in x64 (float64).  The stopping
// test is |B - K X'| <= rtol |B| per column.
template <typename T>
amm_status linear_solve(amm_handle* h, double rtol, int maxit, SolveReport& rep) {
    const Layout& L = h->L;
    Dyn& d = h->v.d;
    rep.cg_iters.assign(L.P, 0);
    rep.refine.assign(L.P, 0);
    rep.rel.assign(L.P, 0.0);
    rep.not_spd = false;
    if (h->cg_coarse) launch_coarse<T>(coarse_args<T>(h), L.n_nd_tiles, L.nagg, L.P, h->stream, tmr(h));
    const T* r = reinterpret_cast<const T*>(d.rvec);
    const T* B = reinterpret_cast<const T*>(d.B);
    T* x = reinterpret_cast<T*>(d.cg[0]);
    vec_op<T>(h, PF_SOLVE, 7);   // dx = 0
    if (sizeof(T) == 8) {
        // float64 CG on K dx = r
        TRY(run_cg<T>(h, r, B, rtol, maxit, rep));
        vec_op<T>(h, PF_SOLVE, 0, x, nullptr);
        TRY(true_residual<T>(h, nullptr, rep.rel));
        for (int p = 0; p < L.P; ++p) {
            if (!(h->dyn[p].flags & PF_SOLVE)) continue;
            if ((h->h_state[2 * p].breakdown | h->h_state[2 * p + 1].breakdown) && rep.rel[p] > 1e-3) {
                rep.not_spd = true;
                rep.bad_pair = p;
            }
        }
        return AMM_OK;
    }
    // float32 CG inside float64 iterative refinement.  The first correction
    // solves on the assembled residual itself (the float64 residual of dx = 0
    // is r) and needs no host decision: it stops at |r| <= rtol/2 |B| or once
    // float32 has reduced its residual by kFirstFloor.
    constexpr double kFirstFloor = 1e-6;
    T* rhs = reinterpret_cast<T*>(d.cg[10]);
    std::vector<int32_t> saved(L.P);
    for (int p = 0; p < L.P; ++p) saved[p] = h->dyn[p].flags;
    for (int p = 0; p < L.P; ++p)
        if (h->dyn[p].flags & PF_SOLVE) rep.refine[p] += 1;
    TRY(run_cg<T>(h, r, B, 0.5 * rtol, maxit, rep, kFirstFloor));
    vec_op<T>(h, PF_SOLVE, 0, x, nullptr);   // dx = first correction
    std::vector<double> prev(L.P, std::numeric_limits<double>::infinity()), rel;
    const int max_refine = 30;
    for (int step = 1; step <= max_refine; ++step) {
        TRY(true_residual<T>(h, rhs, rel));
        bool any = false;
        for (int p = 0; p < L.P; ++p) {
            if (!(h->dyn[p].flags & PF_SOLVE)) continue;
            rep.rel[p] = rel[p];
            if (rel[p] <= rtol || step == max_refine || rel[p] > 0.5 * prev[p]) {
                h->dyn[p].flags &= ~PF_SOLVE;   // converged, or refinement stopped improving
            } else {
                any = true;
                rep.refine[p] += 1;
                // reduce the residual just past the target, within float32 reach
                h->dyn[p].cg_rtol = std::min(0.25, std::max(1e-6, 0.5 * rtol / rel[p]));
            }
            prev[p] = rel[p];
        }
        if (!any) break;
        TRY(push_dyn(h));
        TRY(run_cg<T>(h, rhs, nullptr, 1e-4, maxit, rep));
        vec_op<T>(h, PF_SOLVE, 1, x, nullptr);   // dx += correction
    }
    for (int p = 0; p < L.P; ++p) {
        h->dyn[p].flags = saved[p];
        h->dyn[p].cg_rtol = 0;
        if ((h->dyn[p].flags & PF_SOLVE) && rep.rel[p] > 1e-3 &&
            (h->h_state[2 * p].breakdown | h->h_state[2 * p + 1].breakdown)) {
            rep.not_spd = true;
            rep.bad_pair = p;
        }
    }
    return push_dyn(h);
}

struct PairState {
    double nu_a = 0, nu_min = 0, nu_r = 0, alpha = 0, beta = 0;
    double E_cur = 0;
    int stage = 0, it = 0, total = 0;
    bool done = false;
    int hist_count = 0, hist_head = -1;
    int cur = 0;
    amm_stats st{};
};

// Eq. (26); a graph without edges has no regularization term.  The
// squared-norm variants take the small-residual scale of the Welsch terms
// (the Welsch energy times 2 nu_a^2): alpha = k_alpha |V|/|E_G|,
// beta = k_beta |V|/|V_G|.
void term_weights(const PairInfo& pi, double k_alpha, double k_beta, int robust, PairState& s) {
    const double N = (double)pi.N, n = (double)pi.n, E = (double)pi.n_undirected;
    if (robust != AMM_ROBUST_WELSCH) {
        s.alpha = E > 0 ? k_alpha * (N / E) : 0.0;
        s.beta = k_beta * (N / n);
        return;
    }
    s.alpha = E > 0 ? k_alpha * (N / E) * (s.nu_r * s.nu_r) / (s.nu_a * s.nu_a) : 0.0;
    s.beta = k_beta * (N / n) / (2.0 * s.nu_a * s.nu_a);
}

// Sec. 4.1's fixed-parameter variants: the largest, smallest or midway
// (nu_a, nu_r) of the dynamic update from this start (nu_a halves down to
// nu_min, nu_r halves with it); the stage bound becomes the fixed nu_a so
// that the solve runs one stage.
void fix_nu(int mode, PairState& s) {
    double a = s.nu_a, r = s.nu_r;
    while (a != s.nu_min) {
        a = std::max(a / 2.0, s.nu_min);
        r = r / 2.0;
    }
    if (mode == AMM_NU_FIXED_MIN) {
        s.nu_a = a;
        s.nu_r = r;
    } else if (mode == AMM_NU_FIXED_MED) {
        s.nu_a = 0.5 * (s.nu_a + a);
        s.nu_r = 0.5 * (s.nu_r + r);
    }
    s.nu_min = s.nu_a;
}

void set_scalars(PairDyn& d, double nu_a, double nu_r, double alpha, double beta, int robust = AMM_ROBUST_WELSCH) {
    d.robust = robust;
    d.nu_a = nu_a;
    d.nu_r = nu_r;
    d.alpha = alpha;
    d.beta = beta;
}

template <typename T>
amm_status solve_impl(amm_handle* h, const amm_params& prm, void* X_inout, void* v_out, amm_stats* stats) {
    const Layout& L = h->L;
    Dyn& d = h->v.d;
    const int P = L.P;
    const int m = prm.aa_m;
    const double rtol = prm.cg_rtol > 0 ? prm.cg_rtol : 1e-10;
    const int maxit = prm.cg_maxit > 0 ? prm.cg_maxit : 20000;
    const auto t0 = std::chrono::steady_clock::now();
    auto now_ms = [&]() {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    std::vector<PairState> ps(P);
    for (int p = 0; p < P; ++p) {
        PairDyn& dy = h->dyn[p];
        dy = PairDyn{};
        set_scalars(dy, 1.0, 1.0, 0.0, 0.0, prm.robust);
        dy.flags = PF_EVAL;
    }
    if (prm.init_identity || !X_inout) {
        TRY(push_dyn(h));
        vec_op<T>(h, PF_EVAL, 9);   // X[0] = identity
    } else {
        launch_x_import<T, T>(reinterpret_cast<const T*>(X_inout), reinterpret_cast<T*>(d.X[0]), h->v.node_user,
                              L.ntot, h->stream);
    }
    TRY(evaluate<T>(h));
    // start of nu_a: median closest-point distance at the initial
    // transforms (the mean of the two middle ones for even N), from the two
    // middle squared distances selected on the device (the square root
    // keeps the order)
    T* mid2 = reinterpret_cast<T*>(d.cg[0]);   // free until the first solve
    if (!(prm.nu_a0 > 0))
        launch_select_mid<T>(reinterpret_cast<const T*>(d.d2[0]), h->v.info, h->v.pt_tiles, L.n_pt_tiles, P, mid2,
                             d.sel, h->stream);
    TRY(pinned_scratch(h, sizeof(T) * 2 * P));
    const T* m2h = reinterpret_cast<const T*>(h->h_scratch);
    if (!(prm.nu_a0 > 0)) {
        HIPC(hipMemcpyAsync(h->h_scratch, mid2, sizeof(T) * 2 * P, hipMemcpyDeviceToHost, h->stream));
        HIPC(hipStreamSynchronize(h->stream));
    }
    for (int p = 0; p < P; ++p) {
        const PairInfo& pi = L.info[p];
        double med = 0.0;
        if (!(prm.nu_a0 > 0)) {
            const double hi = std::sqrt((double)m2h[2 * p + 1]);
            med = pi.N % 2 == 0 ? 0.5 * (std::sqrt((double)m2h[2 * p]) + hi) : hi;
        }
        PairState& st = ps[p];
        st.nu_min = prm.nu_a_min > 0 ? prm.nu_a_min : h->lbar[p] / std::sqrt(3.0);
        st.nu_a = std::max(prm.nu_a0 > 0 ? prm.nu_a0 : med, st.nu_min);
        st.nu_r = prm.nu_r0 > 0 ? prm.nu_r0 : 3.0 * h->lbar[p];
        if (prm.nu_mode != AMM_NU_DYNAMIC) fix_nu(prm.nu_mode, st);
        if (prm.robust == AMM_ROBUST_L2) st.nu_min = st.nu_a;   // nothing to update: one stage
        term_weights(pi, prm.k_alpha, prm.k_beta, prm.robust, st);
        st.st.stages = 1;
        PairDyn& dy = h->dyn[p];
        set_scalars(dy, st.nu_a, st.nu_r, st.alpha, st.beta, prm.robust);
        dy.has_prev = 1;   // in place: same transforms, same closest points
    }
    TRY(evaluate<T>(h));
    for (int p = 0; p < P; ++p) ps[p].E_cur = h->h_out[p].E;

    const int ring = m + 1;
    SolveReport rep;
    std::vector<char> reject(P), restage(P);
    std::vector<amm_iter_record> rec(P);
    h->iter_log.clear();
    while (true) {
        bool any = false;
        for (int p = 0; p < P; ++p) {
            PairDyn& dy = h->dyn[p];
            PairState& st = ps[p];
            dy = PairDyn{};
            dy.cur = st.cur;
            set_scalars(dy, st.nu_a, st.nu_r, st.alpha, st.beta, prm.robust);
            if (st.done) continue;
            any = true;
            dy.flags = PF_SOLVE;
            st.hist_head = (st.hist_head + 1) % ring;
            st.hist_count = std::min(st.hist_count + 1, ring);
            dy.aa_mk = std::min(st.hist_count - 1, m);
            for (int x = 0; x <= dy.aa_mk; ++x) dy.aa_slot[x] = ((st.hist_head - x) % ring + ring) % ring;
            dy.eval_x = 1 - st.cur;
            dy.eval_dst = 1 - st.cur;
            dy.has_prev = 1;
        }
        if (!any) break;
        TRY(push_dyn(h));
        launch_assemble<T>(asm_args<T>(h), L.ntot, h->stream, tmr(h));
        TRY(linear_solve<T>(h, rtol, maxit, rep));
        if (rep.not_spd)
            return fail(h, AMM_ERR_NOT_SPD,
                        "K is not positive definite (CG breakdown) in pair " + std::to_string(rep.bad_pair) +
                            " at MM iteration " + std::to_string(ps[rep.bad_pair].total) + ", relative residual " +
                            std::to_string(rep.rel[rep.bad_pair]));
        AaArgs<T> aa{};
        aa.nd_tiles = h->v.nd_tiles;
        aa.dyn = h->v.dyn;
        aa.out = h->v.out;
        aa.ntot = L.ntot;
        aa.G = reinterpret_cast<T*>(d.G);
        aa.F = d.F;
        for (int q = 0; q < 3; ++q) aa.X[q] = reinterpret_cast<T*>(d.X[q]);
        aa.dx = d.x64;
        aa.part = d.aa_part;
        AaSolveArgs sa{h->v.info, h->v.dyn, h->v.out, d.aa_part, P};
        launch_aa<T>(aa, sa, L.n_nd_tiles, h->stream, tmr(h));
        // evaluate E at the candidate (X_AA, or G(X^k) itself)
        for (int p = 0; p < P; ++p)
            if (!ps[p].done) h->dyn[p].flags = PF_EVAL;
        TRY(evaluate<T>(h));
        bool any_reject = false;
        for (int p = 0; p < P; ++p) {
            PairState& st = ps[p];
            reject[p] = 0;
            if (st.done) continue;
            const PairOut& o = h->h_out[p];
            amm_iter_record& r = rec[p];
            r = amm_iter_record{};
            r.pair = p;
            r.iter = st.total;
            r.stage = st.stage;
            r.m_k = h->dyn[p].aa_mk;
            r.aa_used = o.aa_used != 0;
            r.energy_before = st.E_cur;
            r.energy_candidate = o.E;
            r.cg_iters = (int32_t)rep.cg_iters[p];
            r.refine_steps = rep.refine[p];
            r.rel_residual = rep.rel[p];
            r.nu_a = st.nu_a;
            r.nu_r = st.nu_r;
            r.alpha = st.alpha;
            r.beta = st.beta;
            bool acc = true;
            if (o.aa_used != 0) {
                acc = o.E < st.E_cur;
                const int64_t fo = (prm.force_per_pair ? (int64_t)p * prm.force_len : 0) + st.total;
                if (prm.force_accept && st.total < prm.force_len && prm.force_accept[fo] >= 0)
                    acc = prm.force_accept[fo] != 0;
                (acc ? st.st.aa_accepted : st.st.aa_rejected) += 1;
            }
            r.accepted = o.aa_used != 0 ? (acc ? 1 : 0) : -1;
            if (!acc) {
                reject[p] = 1;
                any_reject = true;
            }
        }
        if (any_reject) {
            // take G(X^k) without a second test: evaluate it and store it as the new iterate
            for (int p = 0; p < P; ++p) {
                h->dyn[p].flags = reject[p] ? (PF_EVAL | PF_SOLVE) : 0;
                h->dyn[p].eval_x = 2;
            }
            TRY(evaluate<T>(h));
            vec_op<T>(h, PF_SOLVE, 6);   // X[1 - cur] = G(X^k)
        }
        bool any_stage = false;
        for (int p = 0; p < P; ++p) {
            PairState& st = ps[p];
            restage[p] = 0;
            if (st.done) continue;
            const PairOut& o = h->h_out[p];
            st.cur = 1 - st.cur;
            st.E_cur = o.E;
            st.it += 1;
            st.total += 1;
            st.st.iters = st.total;
            st.st.max_disp = o.maxdisp;
            st.st.cg_iters += rep.cg_iters[p];
            st.st.refine_steps += rep.refine[p];
            st.st.max_rel_residual = std::max(st.st.max_rel_residual, rep.rel[p]);
            if (!(rep.rel[p] <= rtol)) st.st.solves_above_rtol += 1;
            rec[p].energy_after = o.E;
            rec[p].max_disp = o.maxdisp;
            h->iter_log.push_back(rec[p]);
            if (!std::isfinite(o.E)) return fail(h, AMM_ERR_NONFINITE, "energy became non-finite");
            const bool budget = prm.max_total_iters > 0 && st.total >= prm.max_total_iters;
            bool end = o.maxdisp < prm.eps || st.it >= prm.imax || budget;
            const int t = st.total - 1;
            const int64_t fo = (prm.force_per_pair ? (int64_t)p * prm.force_len : 0) + t;
            if (prm.force_stage_end && t < prm.force_len && prm.force_stage_end[fo] >= 0)
                end = prm.force_stage_end[fo] != 0;
            if (!end) continue;
            if (st.nu_a == st.nu_min || budget) {
                st.done = true;
                st.st.converged = (o.maxdisp < prm.eps && st.nu_a == st.nu_min) ? 1 : 0;
                st.st.time_ms = now_ms();
                continue;
            }
            st.stage += 1;
            st.st.stages += 1;
            st.nu_a = std::max(st.nu_a / 2.0, st.nu_min);
            st.nu_r = st.nu_r / 2.0;
            term_weights(L.info[p], prm.k_alpha, prm.k_beta, prm.robust, st);
            st.it = 0;
            st.hist_count = 0;
            st.hist_head = -1;
            restage[p] = 1;
            any_stage = true;
        }
        if (any_stage) {
            // the energy at the new nu (same transforms, same closest points)
            for (int p = 0; p < P; ++p) {
                PairDyn& dy = h->dyn[p];
                dy = PairDyn{};
                dy.flags = restage[p] ? PF_EVAL : 0;
                dy.cur = dy.eval_x = dy.eval_dst = ps[p].cur;
                dy.has_prev = 1;
                set_scalars(dy, ps[p].nu_a, ps[p].nu_r, ps[p].alpha, ps[p].beta, prm.robust);
            }
            TRY(evaluate<T>(h));
            for (int p = 0; p < P; ++p)
                if (restage[p]) ps[p].E_cur = h->h_out[p].E;
        }
    }
    // final energies and terms at the returned transforms; collect X and v_hat
    for (int p = 0; p < P; ++p) {
        PairDyn& dy = h->dyn[p];
        dy = PairDyn{};
        dy.flags = PF_EVAL | PF_SOLVE;
        dy.cur = dy.eval_x = dy.eval_dst = ps[p].cur;
        dy.has_prev = 1;
        set_scalars(dy, ps[p].nu_a, ps[p].nu_r, ps[p].alpha, ps[p].beta, prm.robust);
    }
    TRY(evaluate<T>(h));
    vec_op<T>(h, PF_SOLVE, 5);   // X[2] = X[cur]
    if (X_inout)
        launch_x_export<T, T>(reinterpret_cast<const T*>(d.X[2]), reinterpret_cast<T*>(X_inout), h->v.node_user,
                              L.ntot, h->stream);
    if (v_out) {
        const size_t es = 4 * sizeof(T);
        for (int p = 0; p < P; ++p) {
            const PairInfo& pi = L.info[p];
            HIPC(hipMemcpyAsync(reinterpret_cast<char*>(d.pts_out) + pi.src_off * es,
                                reinterpret_cast<char*>(d.vhat[ps[p].cur]) + pi.src_off * es, pi.N * es,
                                hipMemcpyDeviceToDevice, h->stream));
        }
        launch_points_export<T, T>(d.pts_out, reinterpret_cast<T*>(v_out), h->v.src_user, L.Ntot, h->stream);
    }
    HIPC(hipStreamSynchronize(h->stream));
    HIPC(hipGetLastError());
    if (h->timing) h->timer.collect();
    if (stats) {
        for (int p = 0; p < P; ++p) {
            amm_stats& o = stats[p];
            o = ps[p].st;
            o.energy = h->h_out[p].E;
            o.e_align = h->h_out[p].Ea;
            o.e_reg = h->h_out[p].Er;
            o.e_rot = h->h_out[p].Eo;
            o.nu_a = ps[p].nu_a;
            o.nu_r = ps[p].nu_r;
            o.alpha = ps[p].alpha;
            o.beta = ps[p].beta;
        }
    }
    return AMM_OK;
}

template <typename T>
amm_status energy_impl(amm_handle* h, const void* X, const void* src, double nu_a, double nu_r, double alpha,
                       double beta, double* energy, int32_t* rho, void* d2, void* gX, void* gV) {
    const Layout& L = h->L;
    Dyn& d = h->v.d;
    launch_x_import<T, T>(reinterpret_cast<const T*>(X), reinterpret_cast<T*>(d.X[0]), h->v.node_user, L.ntot,
                          h->stream);
    if (src) launch_src_import<T, T>(reinterpret_cast<const T*>(src), d.src_ovr, h->v.src_user, L.Ntot, h->stream);
    PairDyn& dy = h->dyn[0];
    dy = PairDyn{};
    dy.flags = PF_EVAL;
    dy.has_prev = h->rho_set0 ? 1 : 0;   // seeds only: the search is exact either way
    set_scalars(dy, nu_a, nu_r, alpha, beta);
    TRY(evaluate<T>(h, src != nullptr));
    if (energy) {
        energy[0] = h->h_out[0].E;
        energy[1] = h->h_out[0].Ea;
        energy[2] = h->h_out[0].Er;
        energy[3] = h->h_out[0].Eo;
    }
    if (rho || d2)
        launch_nn_export<T, T>(d.rho[0], reinterpret_cast<const T*>(d.d2[0]), h->v.src_user, h->v.tgt_user, rho,
                               reinterpret_cast<T*>(d2), L.Ntot, h->stream);
    if (gX) {
        using V = typename V4Of<T>::type;
        const StaticT<T>& s = statics<T>(h);
        GradArgs<T> g{};
        g.pt_tiles = h->v.pt_tiles;
        g.info = h->v.info;
        g.dyn = h->v.dyn;
        g.node_pair = h->v.node_pair;
        g.src = s.src;
        g.src_override = src ? reinterpret_cast<const V*>(d.src_ovr) : nullptr;
        g.src_user = h->v.src_user;
        g.node_user = h->v.node_user;
        g.iidx = h->v.iidx;
        g.iw = s.iw;
        g.k = L.k;
        g.Ntot = L.Ntot;
        g.nodes = s.nodes;
        g.tgt = s.tgt;
        g.pj_ptr = h->v.pj_ptr;
        g.pj_ent = h->v.pj_ent;
        g.adj_ptr = h->v.adj_ptr;
        g.adj_nbr = h->v.adj_nbr;
        g.adj_rev = h->v.adj_rev;
        g.adj_r = s.adj_r;
        g.X = reinterpret_cast<const T*>(d.X[0]);
        for (int q = 0; q < 2; ++q) {
            g.vhat[q] = reinterpret_cast<const V*>(d.vhat[q]);
            g.rho[q] = d.rho[q];
            g.d2[q] = reinterpret_cast<const T*>(d.d2[q]);
            g.qw[q] = reinterpret_cast<const V*>(d.qw[q]);
            g.Dres[q] = reinterpret_cast<const V*>(d.Dres[q]);
            g.R[q] = reinterpret_cast<const T*>(d.R[q]);
        }
        g.gpt = reinterpret_cast<V*>(d.gpt);
        g.gX = reinterpret_cast<T*>(gX);
        g.gV = reinterpret_cast<T*>(gV);
        launch_grad<T>(g, L.n_pt_tiles, L.ntot, h->stream);
    }
    HIPC(hipStreamSynchronize(h->stream));
    HIPC(hipGetLastError());
    return AMM_OK;
}

template <typename T>
amm_status step_impl(amm_handle* h, const amm_step_in* in, amm_step_out* out) {
    const Layout& L = h->L;
    Dyn& d = h->v.d;
    launch_x_import<T, T>(reinterpret_cast<const T*>(in->X), reinterpret_cast<T*>(d.X[0]), h->v.node_user, L.ntot,
                          h->stream);
    PairDyn& dy = h->dyn[0];
    dy = PairDyn{};
    dy.flags = PF_EVAL;
    dy.has_prev = h->rho_set0 ? 1 : 0;   // seeds only: the search is exact either way
    set_scalars(dy, in->nu_a, in->nu_r, in->alpha, in->beta, in->robust);
    TRY(evaluate<T>(h));
    out->energy[0] = h->h_out[0].E;
    out->energy[1] = h->h_out[0].Ea;
    out->energy[2] = h->h_out[0].Er;
    out->energy[3] = h->h_out[0].Eo;
    if (out->rho || out->d2)
        launch_nn_export<T, T>(d.rho[0], reinterpret_cast<const T*>(d.d2[0]), h->v.src_user, h->v.tgt_user, out->rho,
                               reinterpret_cast<T*>(out->d2), L.Ntot, h->stream);
    if (out->v_hat)
        launch_points_export<T, T>(d.vhat[0], reinterpret_cast<T*>(out->v_hat), h->v.src_user, L.Ntot, h->stream);
    dy.flags = PF_SOLVE;
    TRY(push_dyn(h));
    launch_assemble<T>(asm_args<T>(h), L.ntot, h->stream, tmr(h));
    SolveReport rep;
    TRY(linear_solve<T>(h, in->cg_rtol > 0 ? in->cg_rtol : 1e-10, in->cg_maxit > 0 ? in->cg_maxit : 20000, rep));
    out->cg_iters = (int32_t)rep.cg_iters[0];
    out->rel_residual = rep.rel[0];
    if (out->X_next) {
        vec_op<T>(h, PF_SOLVE, 8);   // X' = X^k + dx
        launch_x_export<T, T>(reinterpret_cast<const T*>(d.X[2]), reinterpret_cast<T*>(out->X_next), h->v.node_user,
                              L.ntot, h->stream);
    }
    if (out->B)
        launch_x_export<T, T>(reinterpret_cast<const T*>(d.B), reinterpret_cast<T*>(out->B), h->v.node_user, L.ntot,
                              h->stream);
    if (out->K_blocks)
        HIPC(hipMemcpyAsync(out->K_blocks, d.Kval, sizeof(T) * 16 * L.nnzb, hipMemcpyDeviceToDevice, h->stream));
    std::vector<int32_t> kr, kc;
    if (out->K_row || out->K_col) {
        kr.resize(L.nnzb);
        kc.resize(L.nnzb);
        for (int64_t j = 0; j < L.ntot; ++j)
            for (int pos = L.K_ptr[j]; pos < L.K_ptr[j + 1]; ++pos) {
                kr[pos] = L.node_user[j];
                kc[pos] = L.node_user[L.K_col[pos]];
            }
        if (out->K_row)
            HIPC(hipMemcpyAsync(out->K_row, kr.data(), 4 * L.nnzb, hipMemcpyHostToDevice, h->stream));
        if (out->K_col)
            HIPC(hipMemcpyAsync(out->K_col, kc.data(), 4 * L.nnzb, hipMemcpyHostToDevice, h->stream));
    }
    HIPC(hipStreamSynchronize(h->stream));
    HIPC(hipGetLastError());
    return AMM_OK;
}

amm_status analyse(amm_handle* h, const amm_problem* probs, int32_t n_pairs, Layout& L, std::vector<double>& lbar) {
    if (!probs || n_pairs < 1) return fail(h, AMM_ERR_INVALID_ARG, "need at least one problem");
    std::vector<HostPair> hps(n_pairs);
    lbar.resize(n_pairs);
    TRY(read_pairs(h, probs, n_pairs, hps));
    for (int p = 0; p < n_pairs; ++p) lbar[p] = hps[p].lbar;
    std::string err;
    amm_status s = validate_pairs(hps, err);
    if (s != AMM_OK) return fail(h, s, err);
    s = build_layout(hps, h->leaf, L, err);
    if (s != AMM_OK) return fail(h, s, err);
    return AMM_OK;
}

}  // namespace

// ---------------------------------------------------------------- allocation-free energy

namespace amm {
namespace {

// Scratch of amm_energy_noalloc: a file-scope device array, one copy per
// GPU, held from the code object's load until the process ends.  Host code
// never uses the array's name as an address (in host code it stands for a
// host-side shadow): the device address of each GPU's copy is looked up
// once, in amm_create with that GPU current, and kept in g_scratch_dev.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
void* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

amm_status scratch_lookup(amm_handle* h, int device) {
    if (device >= kMaxDevices) return AMM_OK;   // amm_energy_noalloc then refuses on this device
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return AMM_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(h, AMM_ERR_HIP, std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                        hipGetErrorString(e));
    g_scratch_dev[device] = ptr;
    return AMM_OK;
}

// Carves the scratch into 256-byte aligned arrays; false when they do not fit.
struct ScratchCarver {
    unsigned char* base;
    size_t off = 0;
    bool ok = true;
    template <typename P>
    P* take(size_t n) {
        off = (off + 255) & ~size_t(255);
        P* r = reinterpret_cast<P*>(base + off);
        off += sizeof(P) * std::max<size_t>(n, 1);
        if (off > kNoAllocScratchBytes) ok = false;
        return r;
    }
};

template <typename T>
amm_status energy_noalloc_impl(amm_handle* h, const void* X, const void* src, double nu_a, double nu_r,
                               double alpha, double beta, double* energy, int32_t* rho, void* d2) {
    using V = typename V4Of<T>::type;
    const Layout& L = h->L;
    void* base = h->device < kMaxDevices ? g_scratch_dev[h->device] : nullptr;
    if (!base) return fail(h, AMM_ERR_STATE, "no scratch address for this device (amm_create not run on it)");
    // per-call arrays: transforms, source override, one evaluation set,
    // tile partials, the pair's parameters and outputs
    ScratchCarver c{reinterpret_cast<unsigned char*>(base)};
    const size_t N = L.Ntot, n = L.ntot, na = L.nadj;
    // first, so that it sits at the same place for every problem: zero at
    // load, and every evaluation leaves it at zero
    int* s_far_count = c.take<int>(1);
    T* sX = c.take<T>(12 * n);
    V* s_src = src ? c.take<V>(N) : nullptr;
    V* s_vhat = c.take<V>(N);
    int* s_rho = c.take<int>(N);
    T* s_d2 = c.take<T>(N);
    V* s_qw = c.take<V>(N);
    T* s_wr = c.take<T>(na);
    V* s_Dres = c.take<V>(na);
    T* s_R = c.take<T>(9 * n);
    double* s_pt_part = c.take<double>(L.n_pt_tiles);
    double* s_pt_max = c.take<double>(L.n_pt_tiles);
    double* s_eg_part = c.take<double>(L.n_eg_tiles);
    double* s_nd_part = c.take<double>(L.n_nd_tiles);
    PairOut* s_out = c.take<PairOut>(1);
    PairDyn* s_dyn = c.take<PairDyn>(1);
    int2* s_far_list = c.take<int2>(N);
    int* s_far_seed = c.take<int>(N);
    T* s_psi = c.take<T>(N);
    T* s_disp = c.take<T>(N);
    if (!c.ok)
        return fail(h, AMM_ERR_INVALID_ARG,
                    "problem too large for the allocation-free scratch (" + std::to_string(c.off) +
                        " bytes needed, " + std::to_string(kNoAllocScratchBytes) + " available)");
    launch_x_import<T, T>(reinterpret_cast<const T*>(X), sX, h->v.node_user, L.ntot, h->stream);
    if (src) launch_src_import<T, T>(reinterpret_cast<const T*>(src), reinterpret_cast<T*>(s_src), h->v.src_user,
                                     L.Ntot, h->stream);
    // a cold search (no warm start: the scratch's last contents may belong
    // to another problem); every array the kernels read is written first
    PairDyn dy{};
    dy.flags = PF_EVAL;
    set_scalars(dy, nu_a, nu_r, alpha, beta);
    launch_dyn_set(&dy, 1, s_dyn, h->stream);
    EvalArgs<T> a = eval_args<T>(h, false);
    a.dyn = s_dyn;
    a.src_override = s_src;
    for (int q = 0; q < 3; ++q) a.X[q] = sX;
    for (int q = 0; q < 2; ++q) {
        a.vhat[q] = s_vhat;
        a.rho[q] = s_rho;
        a.d2[q] = s_d2;
        a.qw[q] = s_qw;
        a.wr[q] = s_wr;
        a.Dres[q] = s_Dres;
        a.R[q] = s_R;
    }
    a.pt_part = s_pt_part;
    a.pt_max = s_pt_max;
    a.eg_part = s_eg_part;
    a.nd_part = s_nd_part;
    a.nn_work = nullptr;
    a.far_count = s_far_count;
    a.far_list = s_far_list;
    a.far_seed = s_far_seed;
    a.pt_psi = s_psi;
    a.pt_disp = s_disp;
    FinalArgs f = final_args(h);
    f.dyn = s_dyn;
    f.out = s_out;
    f.pt_part = s_pt_part;
    f.pt_max = s_pt_max;
    f.eg_part = s_eg_part;
    f.nd_part = s_nd_part;
    launch_eval<T>(a, L.n_pt_tiles, L.n_eg_tiles, L.n_nd_tiles, f, L.P, h->stream, nullptr);
    if (rho || d2)
        launch_nn_export<T, T>(s_rho, s_d2, h->v.src_user, h->v.tgt_user, rho, reinterpret_cast<T*>(d2), L.Ntot,
                               h->stream);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(h->h_out, s_out, sizeof(PairOut), hipMemcpyDeviceToHost, h->stream));
    TRY(sync_spin(h));
    if (energy) {
        energy[0] = h->h_out[0].E;
        energy[1] = h->h_out[0].Ea;
        energy[2] = h->h_out[0].Er;
        energy[3] = h->h_out[0].Eo;
    }
    return AMM_OK;
}

}  // namespace
}  // namespace amm

extern "C" {

void amm_params_default(amm_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->k_alpha = 100.0;
    p->k_beta = 1.0;
    p->eps = 1e-5;
    p->imax = 100;
    p->max_total_iters = 0;
    p->aa_m = 5;
    p->precision = AMM_FP32_REFINE;
    p->cg_rtol = 1e-10;
    p->cg_maxit = 20000;
    p->init_identity = 1;
}

const char* amm_status_string(amm_status s) {
    switch (s) {
        case AMM_OK: return "ok";
        case AMM_ERR_INVALID_ARG: return "invalid argument";
        case AMM_ERR_STATE: return "invalid call order";
        case AMM_ERR_OOM: return "out of device memory";
        case AMM_ERR_HIP: return "HIP runtime error";
        case AMM_ERR_NONFINITE: return "non-finite value";
        case AMM_ERR_GRAPH: return "invalid deformation graph";
        case AMM_ERR_NOT_SPD: return "system not positive definite";
    }
    return "unknown status";
}

const char* amm_last_error(const amm_handle* h) { return h ? h->err.c_str() : g_last_error.c_str(); }

const char* amm_version(void) { return kVersion; }

amm_status amm_create(amm_handle** out, int device, void* stream) {
    if (!out) return fail(nullptr, AMM_ERR_INVALID_ARG, "null handle pointer");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
        return fail(nullptr, AMM_ERR_HIP, "no HIP device available");
    if (device < 0 || device >= count) return fail(nullptr, AMM_ERR_INVALID_ARG, "device index out of range");
    if (hipSetDevice(device) != hipSuccess) return fail(nullptr, AMM_ERR_HIP, "hipSetDevice failed");
    amm_handle* h = new amm_handle();
    h->device = device;
    h->stream = reinterpret_cast<hipStream_t>(stream);
    const amm_status st = scratch_lookup(h, device);
    if (st != AMM_OK) {
        delete h;
        return st;
    }
    *out = h;
    return AMM_OK;
}

void amm_destroy(amm_handle* h) {
    if (!h) return;
    if (h->freer.joinable()) h->freer.join();
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    if (h->prog) (void)hipHostFree(h->prog);
    if (h->nn_work) (void)hipFree(h->nn_work);
    if (h->graph) graph_release(h->graph);
    if (h->tw.buf) (void)hipFree(h->tw.buf);
    if (h->h_scratch) (void)hipHostFree(h->h_scratch);
    if (h->rb_pin) (void)hipHostFree(h->rb_pin);
    if (h->sync_ev) (void)hipEventDestroy(h->sync_ev);
    if (h->ws_own) (void)hipFree(h->ws_own);
    if (h->h_out) (void)hipHostFree(h->h_out);
    if (h->h_state) (void)hipHostFree(h->h_state);
    delete h;
}

amm_status amm_set_stream(amm_handle* h, void* stream) {
    if (!h) return fail(nullptr, AMM_ERR_INVALID_ARG, "null handle");
    h->stream = reinterpret_cast<hipStream_t>(stream);
    return AMM_OK;
}

amm_status amm_check_problem(const amm_problem* p) {
    if (!p) return fail(nullptr, AMM_ERR_INVALID_ARG, "null problem");
    if (p->on_device) return fail(nullptr, AMM_ERR_INVALID_ARG, "amm_check_problem takes host pointers");
    HostPair hp;
    TRY(read_pair(nullptr, *p, hp));
    std::string err;
    const amm_status s = validate_pair(hp, err);
    if (s != AMM_OK) return fail(nullptr, s, err);
    return AMM_OK;
}

amm_status amm_workspace_size(amm_handle* h, const amm_problem* probs, int32_t n_pairs, size_t* bytes) {
    if (!h || !bytes) return fail(h, AMM_ERR_INVALID_ARG, "null argument");
    HIPC(hipSetDevice(h->device));
    Layout L;
    std::vector<double> lb;
    TRY(analyse(h, probs, n_pairs, L, lb));
    Carver c;
    Dev v{};
    plan(L, c, v);
    *bytes = c.off + 256;
    return AMM_OK;
}

amm_status amm_set_workspace(amm_handle* h, void* ptr, size_t bytes) {
    if (!h) return fail(nullptr, AMM_ERR_INVALID_ARG, "null handle");
    if (ptr && (reinterpret_cast<uintptr_t>(ptr) & 255))
        return fail(h, AMM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    h->ws_user = ptr;
    h->ws_user_bytes = ptr ? bytes : 0;
    h->has_problem = false;
    return AMM_OK;
}

amm_status amm_set_problems(amm_handle* h, const amm_problem* probs, int32_t n_pairs) {
    if (!h) return fail(nullptr, AMM_ERR_INVALID_ARG, "null handle");
    HIPC(hipSetDevice(h->device));
    HIPC(hipStreamSynchronize(h->stream));
    h->has_problem = false;
    if (h->nn_work) {
        // the counters are sized for the previous problems' tiles
        (void)hipFree(h->nn_work);
        h->nn_work = nullptr;
        h->nn_work_tiles = 0;
    }
    Layout L;
    std::vector<double> lb;
    TRY(analyse(h, probs, n_pairs, L, lb));
    Carver c;
    Dev v{};
    plan(L, c, v);
    const size_t need = c.off + 256;
    char* base = nullptr;
    if (h->ws_user) {
        if (h->ws_user_bytes < need) return fail(h, AMM_ERR_OOM, "workspace too small");
        base = reinterpret_cast<char*>(h->ws_user);
    } else {
        if (h->ws_own_bytes < need) {
            if (h->ws_own) (void)hipFree(h->ws_own);
            h->ws_own = nullptr;
            h->ws_own_bytes = 0;
            if (hipMalloc(&h->ws_own, need) != hipSuccess)
                return fail(h, AMM_ERR_OOM, "hipMalloc of the workspace failed");
            h->ws_own_bytes = need;
        }
        base = reinterpret_cast<char*>(h->ws_own);
    }
    Carver c2;
    c2.base = base;
    plan(L, c2, v);
    h->v = v;
    // the previous layout (hundreds of MB for a large batch) is freed on a
    // thread of its own, off the set-up's critical path; the handle joins it
    // at the next set-up or when it is destroyed
    {
        if (h->freer.joinable()) h->freer.join();
        Layout old = std::move(h->L);
        h->L = std::move(L);
        h->freer = std::thread([o = std::move(old)]() mutable { Layout gone = std::move(o); });
    }
    h->lbar = lb;
    const Layout& Lr = h->L;
    TRY(ensure_host(h, Lr.P));
    TRY(up(h, v.iidx, Lr.iidx));
    TRY(up(h, v.src_user, Lr.src_user));
    TRY(up(h, v.node_user, Lr.node_user));
    TRY(up(h, v.node_pair, Lr.node_pair));
    TRY(up(h, v.adj_ptr, Lr.adj_ptr));
    TRY(up(h, v.adj_nbr, Lr.adj_nbr));
    TRY(up(h, v.adj_row, Lr.adj_row));
    TRY(up(h, v.adj_rev, Lr.adj_rev));
    TRY(up(h, v.K_ptr, Lr.K_ptr));
    TRY(up(h, v.K_col, Lr.K_col));
    TRY(up(h, v.K_adj, Lr.K_adj));
    TRY(up(h, v.pj_ptr, Lr.pj_ptr));
    TRY(up(h, v.pj_ent, Lr.pj_ent));
    TRY(up(h, v.pj_pos, Lr.pj_pos));
    TRY(up(h, v.tgt_user, Lr.tgt_user));
    TRY(up(h, v.info, Lr.info));
    TRY(up(h, reinterpret_cast<int32_t*>(v.pt_tiles), Lr.pt_tiles));
    TRY(up(h, reinterpret_cast<int32_t*>(v.nd_tiles), Lr.nd_tiles));
    TRY(up(h, reinterpret_cast<int32_t*>(v.eg_tiles), Lr.eg_tiles));
    TRY(up_real(h, v.sf.src, v.sd.src, Lr.src4));
    TRY(up_real(h, v.sf.iw, v.sd.iw, Lr.iw));
    // the point-major copy of the weights, formed on the device
    launch_weights_point_major<float>(v.sf.iw, Lr.k, Lr.Ntot, v.sf.iw_pt, h->stream);
    launch_weights_point_major<double>(v.sd.iw, Lr.k, Lr.Ntot, v.sd.iw_pt, h->stream);
    TRY(up_real(h, v.sf.nodes, v.sd.nodes, Lr.nodes4));
    TRY(up_real(h, v.sf.tgt, v.sd.tgt, Lr.tgt4));
    TRY(up_real(h, v.sf.adj_r, v.sd.adj_r, Lr.adj_r));
    TRY(up_real(h, v.sf.node_rel, v.sd.node_rel, Lr.node_rel));
    TRY(up(h, reinterpret_cast<int32_t*>(v.aggs), Lr.aggs));
    TRY(up(h, v.tile_agg_ptr, Lr.tile_agg_ptr));
    TRY(up(h, v.tile_agg, Lr.tile_agg));
    TRY(up(h, v.grid_cells, Lr.grid_cells));
    TRY(up(h, v.tile_cols, Lr.tile_cols));
    TRY(up(h, v.tile_ncols, Lr.tile_ncols));
    TRY(up(h, v.tile_rowl, Lr.tile_rowl));
    TRY(up(h, v.K_lcol, Lr.K_lcol));
    // the deferred-search count starts at zero (each evaluation leaves it so)
    HIPC(hipMemsetAsync(v.d.far_count, 0, sizeof(int), h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    h->has_problem = true;
    h->rho_set0 = false;
    return AMM_OK;
}

amm_status amm_set_problem(amm_handle* h, const amm_problem* p) { return amm_set_problems(h, p, 1); }

amm_status amm_set_leaf_size(amm_handle* h, int32_t leaf) {
    if (!h) return fail(nullptr, AMM_ERR_INVALID_ARG, "null handle");
    if (leaf < 1 || leaf > 256) return fail(h, AMM_ERR_INVALID_ARG, "leaf size must be in 1..256");
    h->leaf = leaf;
    return AMM_OK;
}

amm_status amm_set_search_budget(amm_handle* h, int32_t steps) {
    if (!h) return fail(nullptr, AMM_ERR_INVALID_ARG, "null handle");
    if (steps < 0 || steps > 1000000) return fail(h, AMM_ERR_INVALID_ARG, "search budget must be in 0..1000000");
    h->nn_budget = steps;
    return AMM_OK;
}

amm_status amm_get_search_budget(const amm_handle* h, int32_t* steps) {
    if (!h || !steps) return fail(nullptr, AMM_ERR_INVALID_ARG, "null argument");
    *steps = h->nn_budget;
    return AMM_OK;
}

namespace amm {
namespace {

// GPU time of one warm-started evaluation (warp, closest points, terms) of
// every pair at X = I, float32: a cold evaluation seeds the closest points,
// then the fastest of three warm ones.
amm_status time_warm_eval(amm_handle* h, double& ms) {
    const Layout& L = h->L;
    Dyn& d = h->v.d;
    std::vector<float> id(12 * L.ntot, 0.0f);
    for (int64_t j = 0; j < L.ntot; ++j) id[12 * j] = id[12 * j + 4] = id[12 * j + 8] = 1.0f;
    HIPC(hipMemcpyAsync(d.X[0], id.data(), id.size() * sizeof(float), hipMemcpyHostToDevice, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    for (int p = 0; p < L.P; ++p) {
        PairDyn& dy = h->dyn[p];
        dy = PairDyn{};
        set_scalars(dy, 1.0, 1.0, 0.0, 0.0);
        dy.flags = PF_EVAL;
    }
    TRY(evaluate<float>(h));
    for (int p = 0; p < L.P; ++p) h->dyn[p].has_prev = 1;
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    ms = 1e30;
    for (int r = 0; r < 3; ++r) {
        TRY(push_dyn(h));
        HIPC(hipEventRecord(e0, h->stream));
        launch_eval<float>(eval_args<float>(h, false), L.n_pt_tiles, L.n_eg_tiles, L.n_nd_tiles, final_args(h), L.P,
                           h->stream, nullptr);
        HIPC(hipEventRecord(e1, h->stream));
        TRY(pull_out(h));
        float t = 0;
        HIPC(hipEventElapsedTime(&t, e0, e1));
        ms = std::min(ms, (double)t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return AMM_OK;
}

}  // namespace
}  // namespace amm

amm_status amm_autotune(amm_handle* h, const amm_problem* probs, int32_t n_pairs, const int32_t* candidates,
                        int32_t n_candidates, int32_t* best_leaf, double* best_ms) {
    if (!h || !probs) return fail(h, AMM_ERR_INVALID_ARG, "null argument");
    static const int32_t kDefault[] = {2, 4, 8, 16};
    if (!candidates) {
        candidates = kDefault;
        n_candidates = 4;
    }
    if (n_candidates < 1) return fail(h, AMM_ERR_INVALID_ARG, "no candidate leaf sizes");
    // with each leaf size, the search budgets (the point at which a search is
    // left to the wave-wide one) are timed too
    static const int32_t kBudgets[] = {32, 48, 64, 96, 128, 0};
    int32_t best = -1, best_budget = kNnBudgetDefault;
    double best_t = 1e30;
    for (int32_t c = 0; c < n_candidates; ++c) {
        if (candidates[c] < 1 || candidates[c] > 256) return fail(h, AMM_ERR_INVALID_ARG, "candidate leaf size out of range");
        h->leaf = candidates[c];
        const amm_status st = amm_set_problems(h, probs, n_pairs);
        if (st == AMM_ERR_OOM && h->ws_user) continue;   // does not fit the caller's workspace
        if (st != AMM_OK) return st;
        for (const int32_t b : kBudgets) {
            h->nn_budget = b;
            double t = 0;
            TRY(time_warm_eval(h, t));
            if (t < best_t) {
                best_t = t;
                best = candidates[c];
                best_budget = b;
            }
        }
    }
    if (best < 0) return fail(h, AMM_ERR_OOM, "no candidate leaf size fits the workspace");
    h->leaf = best;
    h->nn_budget = best_budget;
    TRY(amm_set_problems(h, probs, n_pairs));
    if (best_leaf) *best_leaf = best;
    if (best_ms) *best_ms = best_t;
    return AMM_OK;
}

amm_status amm_solve(amm_handle* h, const amm_params* prm, void* X_inout, void* v_out, amm_stats* stats) {
    if (!h || !prm) return fail(h, AMM_ERR_INVALID_ARG, "null argument");
    if (!h->has_problem) return fail(h, AMM_ERR_STATE, "amm_solve before amm_set_problem");
    if (prm->aa_m < 0 || prm->aa_m > AMM_MAX_AA_M) return fail(h, AMM_ERR_INVALID_ARG, "aa_m out of range");
    if (!(prm->eps >= 0) || prm->imax < 1) return fail(h, AMM_ERR_INVALID_ARG, "bad eps or imax");
    if (!(prm->k_alpha >= 0) || !(prm->k_beta > 0)) return fail(h, AMM_ERR_INVALID_ARG, "bad k_alpha or k_beta");
    if (!prm->init_identity && !X_inout) return fail(h, AMM_ERR_INVALID_ARG, "X_inout needed without init_identity");
    if (prm->cg_precond != AMM_PRECOND_TWO_LEVEL && prm->cg_precond != AMM_PRECOND_BLOCK_JACOBI)
        return fail(h, AMM_ERR_INVALID_ARG, "bad cg_precond");
    if (prm->robust < AMM_ROBUST_WELSCH || prm->robust > AMM_ROBUST_L2_TRUNC)
        return fail(h, AMM_ERR_INVALID_ARG, "bad robust");
    if (prm->nu_mode < AMM_NU_DYNAMIC || prm->nu_mode > AMM_NU_FIXED_MED)
        return fail(h, AMM_ERR_INVALID_ARG, "bad nu_mode");
    HIPC(hipSetDevice(h->device));
    h->cg_coarse = prm->cg_precond == AMM_PRECOND_TWO_LEVEL;
    if (prm->precision == AMM_FP64_PLAIN) return solve_impl<double>(h, *prm, X_inout, v_out, stats);
    if (prm->precision == AMM_FP32_REFINE) return solve_impl<float>(h, *prm, X_inout, v_out, stats);
    return fail(h, AMM_ERR_INVALID_ARG, "unknown precision");
}

amm_status amm_step(amm_handle* h, const amm_step_in* in, amm_step_out* out) {
    if (!h || !in || !out || !in->X) return fail(h, AMM_ERR_INVALID_ARG, "null argument");
    if (!h->has_problem) return fail(h, AMM_ERR_STATE, "amm_step before amm_set_problem");
    if (h->L.P != 1) return fail(h, AMM_ERR_STATE, "amm_step needs exactly one pair");
    if (!(in->nu_a > 0) || !(in->nu_r > 0) || !(in->beta > 0) || !(in->alpha >= 0))
        return fail(h, AMM_ERR_INVALID_ARG, "nu_a, nu_r, beta must be > 0 and alpha >= 0");
    if (in->cg_precond != AMM_PRECOND_TWO_LEVEL && in->cg_precond != AMM_PRECOND_BLOCK_JACOBI)
        return fail(h, AMM_ERR_INVALID_ARG, "bad cg_precond");
    if (in->robust < AMM_ROBUST_WELSCH || in->robust > AMM_ROBUST_L2_TRUNC)
        return fail(h, AMM_ERR_INVALID_ARG, "bad robust");
    HIPC(hipSetDevice(h->device));
    h->cg_coarse = in->cg_precond == AMM_PRECOND_TWO_LEVEL;
    if (in->precision == AMM_FP64_PLAIN) return step_impl<double>(h, in, out);
    if (in->precision == AMM_FP32_REFINE) return step_impl<float>(h, in, out);
    return fail(h, AMM_ERR_INVALID_ARG, "unknown precision");
}

amm_status amm_set_targets(amm_handle* h, int32_t pair, amm_dtype dtype, const void* tgt_xyz, int64_t n_tgt,
                           int32_t on_device) {
    if (!h || !tgt_xyz) return fail(h, AMM_ERR_INVALID_ARG, "null argument");
    if (!h->has_problem) return fail(h, AMM_ERR_STATE, "amm_set_targets before amm_set_problem");
    if (pair < 0 || pair >= h->L.P) return fail(h, AMM_ERR_INVALID_ARG, "pair out of range");
    if (dtype != AMM_F32 && dtype != AMM_F64) return fail(h, AMM_ERR_INVALID_ARG, "bad dtype");
    PairInfo& pi = h->L.info[pair];
    if (n_tgt != pi.M) return fail(h, AMM_ERR_INVALID_ARG, "n_tgt must equal the pair's target count");
    HIPC(hipSetDevice(h->device));
    HIPC(hipStreamSynchronize(h->stream));   // nothing may still read the old targets
    const size_t es = dtype == AMM_F32 ? 4 : 8;
    Dev& v = h->v;
    const void* src = tgt_xyz;
    if (on_device) {
        HIPC(hipDeviceSynchronize());        // the caller's writes to tgt_xyz, on any stream
    } else {
        // the raw coordinates into the float64 staging area (4 M values)
        HIPC(hipMemcpyAsync(v.staging, tgt_xyz, es * 3 * (size_t)n_tgt, hipMemcpyHostToDevice, h->stream));
        src = v.staging;
    }
    // the search structure is rebuilt on the device, bit for bit the host
    // layout's, at the pair's depth (so its tables keep their size); the
    // host copies of the target arrays keep the set-up values
    TargetLayout frame;
    std::string err;
    const amm_status st = device_target_layout(h->stream, h->tw, dtype == AMM_F64, src, n_tgt, pi.grid_bits,
                                               v.sf.tgt + pi.tgt_off, v.sd.tgt + pi.tgt_off,
                                               v.tgt_user + pi.tgt_off, v.grid_cells + pi.grid_off, frame, err);
    if (st != AMM_OK) return fail(h, st, err);
    for (int c = 0; c < 3; ++c) {
        pi.glo[c] = frame.glo[c];
        pi.gscale[c] = frame.gscale[c];
        pi.cs[c] = frame.cs[c];
    }
    pi.gpad = frame.gpad;
    HIPC(hipMemcpyAsync(v.info + pair, &pi, sizeof(PairInfo), hipMemcpyHostToDevice, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    return AMM_OK;
}

amm_status amm_build_graphs(amm_handle* h, const amm_graph_in* in, int32_t n_sets, amm_graph_info* info) {
    if (!h || !in) return fail(h, AMM_ERR_INVALID_ARG, "null argument");
    HIPC(hipSetDevice(h->device));
    GraphBuild* g = nullptr;
    std::string err;
    const amm_status st = graph_build(h->stream, in, n_sets, info, &g, err);
    if (st != AMM_OK) return fail(h, st, err);
    if (h->graph) graph_release(h->graph);
    h->graph = g;
    return AMM_OK;
}

amm_status amm_build_graph(amm_handle* h, const amm_graph_in* in, amm_graph_info* info) {
    return amm_build_graphs(h, in, 1, info);
}

amm_status amm_graph_copy_set(amm_handle* h, int32_t set, int32_t* node_src_idx, int32_t* infl_idx, void* infl_w,
                              int32_t* edges) {
    if (!h) return fail(nullptr, AMM_ERR_INVALID_ARG, "null handle");
    if (!h->graph) return fail(h, AMM_ERR_STATE, "amm_graph_copy before amm_build_graph");
    HIPC(hipSetDevice(h->device));
    std::string err;
    const amm_status st = graph_copy(h->graph, h->stream, set, node_src_idx, infl_idx, infl_w, edges, err);
    if (st != AMM_OK) return fail(h, st, err);
    HIPC(hipStreamSynchronize(h->stream));
    return AMM_OK;
}

amm_status amm_graph_copy(amm_handle* h, int32_t* node_src_idx, int32_t* infl_idx, void* infl_w, int32_t* edges) {
    return amm_graph_copy_set(h, 0, node_src_idx, infl_idx, infl_w, edges);
}

amm_status amm_count_nn_work(amm_handle* h, int32_t enable) {
    if (!h) return fail(nullptr, AMM_ERR_INVALID_ARG, "null handle");
    if (!h->has_problem) return fail(h, AMM_ERR_STATE, "amm_count_nn_work before amm_set_problem");
    HIPC(hipSetDevice(h->device));
    HIPC(hipStreamSynchronize(h->stream));
    if (h->nn_work) (void)hipFree(h->nn_work);
    h->nn_work = nullptr;
    h->nn_work_tiles = 0;
    if (!enable) return AMM_OK;
    const size_t bytes = sizeof(long long) * 4 * std::max(h->L.n_pt_tiles, 1);
    if (hipMalloc((void**)&h->nn_work, bytes) != hipSuccess) {
        h->nn_work = nullptr;
        return fail(h, AMM_ERR_OOM, "search counters");
    }
    HIPC(hipMemsetAsync(h->nn_work, 0, bytes, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    h->nn_work_tiles = h->L.n_pt_tiles;
    return AMM_OK;
}

amm_status amm_nn_work(amm_handle* h, int64_t* queries, int64_t* box_tests, int64_t* distance_evals,
                       int64_t* cell_lookups) {
    if (!h || !queries || !box_tests || !distance_evals) return fail(h, AMM_ERR_INVALID_ARG, "null argument");
    if (!h->nn_work) return fail(h, AMM_ERR_STATE, "search counting is off");
    HIPC(hipSetDevice(h->device));
    std::vector<long long> c(4 * (size_t)h->nn_work_tiles);
    HIPC(hipMemcpyAsync(c.data(), h->nn_work, sizeof(long long) * c.size(), hipMemcpyDeviceToHost, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    long long q = 0, b = 0, d = 0, g = 0;
    for (int t = 0; t < h->nn_work_tiles; ++t) {
        q += c[4 * t];
        b += c[4 * t + 1];
        d += c[4 * t + 2];
        g += c[4 * t + 3];
    }
    *queries = q;
    *box_tests = b;
    *distance_evals = d;
    if (cell_lookups) *cell_lookups = g;
    return AMM_OK;
}

amm_status amm_iter_log(amm_handle* h, amm_iter_record* out, int32_t capacity, int32_t* count) {
    if (!h || !count) return fail(h, AMM_ERR_INVALID_ARG, "null argument");
    *count = (int32_t)h->iter_log.size();
    for (int32_t i = 0; i < *count && i < capacity && out; ++i) out[i] = h->iter_log[i];
    return AMM_OK;
}

amm_status amm_get_sizes(const amm_handle* h, int32_t* n_pairs, int64_t* n_src_total, int64_t* n_nodes_total,
                         int64_t* n_tgt_total, int32_t* k) {
    if (!h) return fail(nullptr, AMM_ERR_INVALID_ARG, "null handle");
    if (!h->has_problem) {
        g_last_error = "no problem set";
        const_cast<amm_handle*>(h)->err = g_last_error;
        return AMM_ERR_STATE;
    }
    if (n_pairs) *n_pairs = h->L.P;
    if (n_src_total) *n_src_total = h->L.Ntot;
    if (n_nodes_total) *n_nodes_total = h->L.ntot;
    if (n_tgt_total) *n_tgt_total = h->L.Mtot;
    if (k) *k = h->L.k;
    return AMM_OK;
}

amm_status amm_k_nnzb(amm_handle* h, int64_t* nnzb) {
    if (!h || !nnzb) return fail(h, AMM_ERR_INVALID_ARG, "null argument");
    if (!h->has_problem) return fail(h, AMM_ERR_STATE, "no problem set");
    *nnzb = h->L.nnzb;
    return AMM_OK;
}

static amm_status energy_entry(amm_handle* h, amm_dtype dtype, const void* X, const void* src, double nu_a,
                               double nu_r, double alpha, double beta, double* energy, int32_t* rho, void* d2,
                               void* gX, void* gV) {
    if (!h || !X) return fail(h, AMM_ERR_INVALID_ARG, "null argument");
    if (!h->has_problem) return fail(h, AMM_ERR_STATE, "no problem set");
    if (h->L.P != 1) return fail(h, AMM_ERR_STATE, "energy and gradient need exactly one pair");
    if (!(nu_a > 0) || !(nu_r > 0)) return fail(h, AMM_ERR_INVALID_ARG, "nu_a and nu_r must be > 0");
    HIPC(hipSetDevice(h->device));
    if (dtype == AMM_F32) return energy_impl<float>(h, X, src, nu_a, nu_r, alpha, beta, energy, rho, d2, gX, gV);
    if (dtype == AMM_F64) return energy_impl<double>(h, X, src, nu_a, nu_r, alpha, beta, energy, rho, d2, gX, gV);
    return fail(h, AMM_ERR_INVALID_ARG, "bad dtype");
}

amm_status amm_energy(amm_handle* h, amm_dtype dtype, const void* X, const void* src, double nu_a, double nu_r,
                      double alpha, double beta, double* energy, int32_t* rho, void* d2) {
    return energy_entry(h, dtype, X, src, nu_a, nu_r, alpha, beta, energy, rho, d2, nullptr, nullptr);
}

amm_status amm_energy_grad(amm_handle* h, amm_dtype dtype, const void* X, const void* src, double nu_a, double nu_r,
                           double alpha, double beta, void* gX, void* gV, double* energy) {
    if (!gX) return fail(h, AMM_ERR_INVALID_ARG, "gX must not be null");
    return energy_entry(h, dtype, X, src, nu_a, nu_r, alpha, beta, energy, nullptr, nullptr, gX, gV);
}

amm_status amm_energy_noalloc(amm_handle* h, amm_dtype dtype, const void* X, const void* src, double nu_a,
                              double nu_r, double alpha, double beta, double* energy, int32_t* rho, void* d2) {
    if (!h || !X) return fail(h, AMM_ERR_INVALID_ARG, "null argument");
    if (!h->has_problem) return fail(h, AMM_ERR_STATE, "no problem set");
    if (h->L.P != 1) return fail(h, AMM_ERR_STATE, "energy needs exactly one pair");
    if (!(nu_a > 0) || !(nu_r > 0)) return fail(h, AMM_ERR_INVALID_ARG, "nu_a and nu_r must be > 0");
    HIPC(hipSetDevice(h->device));
    if (dtype == AMM_F32) return energy_noalloc_impl<float>(h, X, src, nu_a, nu_r, alpha, beta, energy, rho, d2);
    if (dtype == AMM_F64) return energy_noalloc_impl<double>(h, X, src, nu_a, nu_r, alpha, beta, energy, rho, d2);
    return fail(h, AMM_ERR_INVALID_ARG, "bad dtype");
}

amm_status amm_enable_timing(amm_handle* h, int32_t on, const char* only) {
    if (!h) return fail(nullptr, AMM_ERR_INVALID_ARG, "null handle");
    h->timer.collect();
    h->timing = on != 0;
    h->timer.only = only ? only : "";
    h->timer.acc.clear();
    return AMM_OK;
}

amm_status amm_kernel_times(amm_handle* h, const char** names, double* ms, int32_t* launches, int32_t capacity,
                            int32_t* count) {
    if (!h || !count) return fail(h, AMM_ERR_INVALID_ARG, "null argument");
    h->timer.collect();
    const int n = (int)h->timer.acc.size();
    *count = n;
    for (int i = 0; i < n && i < capacity; ++i) {
        if (names) names[i] = h->timer.acc[i].name;
        if (ms) ms[i] = h->timer.acc[i].ms;
        if (launches) launches[i] = h->timer.acc[i].n;
    }
    return AMM_OK;
}

}  // extern "C"
