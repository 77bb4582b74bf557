// Host-side validation of registration problems and construction of the
// device layout: spatial (Morton) ordering of points, nodes and targets, the
// octree run-start tables over each target set, the node adjacency with the edge
// weights of Eq. (8), the block pattern of K (Eq. 21) and the per-node lists
// of influenced points used by the row-wise assembly.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <limits>
#include <numeric>
#include <thread>

#include "amm_internal.h"

namespace amm {

namespace {

std::string fmt(const char* f, long long a = 0, long long b = 0) {
    char buf[256];
    std::snprintf(buf, sizeof buf, f, a, b);
    return buf;
}

uint32_t spread10(uint32_t x) {
    x &= 0x3ff;
    x = (x | (x << 16)) & 0x030000ff;
    x = (x | (x << 8)) & 0x0300f00f;
    x = (x | (x << 4)) & 0x030c30c3;
    x = (x | (x << 2)) & 0x09249249;
    return x;
}

struct Box {
    double lo[3], hi[3];
};

uint32_t morton(const double* p, const Box& b) {
    uint32_t q[3];
    for (int c = 0; c < 3; ++c) {
        double ext = b.hi[c] - b.lo[c];
        double t = ext > 0 ? (p[c] - b.lo[c]) / ext : 0.0;
        int v = (int)std::floor(t * 1023.999);
        q[c] = (uint32_t)std::min(1023, std::max(0, v));
    }
    return (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
}

// Indices 0..n-1 ordered by their 30-bit codes, equal codes in index order
// (a stable least-significant-digit radix sort, three 10-bit passes: the
// order std::stable_sort gives).
std::vector<int32_t> code_order(const std::vector<uint32_t>& code) {
    const int64_t n = (int64_t)code.size();
    std::vector<int32_t> a(n), b(n);
    std::iota(a.begin(), a.end(), 0);
    std::vector<int64_t> cnt(1025);
    for (int pass = 0; pass < 3; ++pass) {
        const int sh = 10 * pass;
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int64_t i = 0; i < n; ++i) ++cnt[((code[a[i]] >> sh) & 1023u) + 1];
        for (int d = 0; d < 1024; ++d) cnt[d + 1] += cnt[d];
        for (int64_t i = 0; i < n; ++i) b[cnt[(code[a[i]] >> sh) & 1023u]++] = a[i];
        a.swap(b);
    }
    return a;
}

std::vector<int32_t> morton_order(const double* pts, int64_t cnt, const Box& b) {
    std::vector<uint32_t> code(cnt);
    for (int64_t i = 0; i < cnt; ++i) code[i] = morton(pts + 3 * i, b);
    return code_order(code);
}

Box bounds(const double* pts, int64_t cnt) {
    Box b;
    for (int c = 0; c < 3; ++c) {
        b.lo[c] = std::numeric_limits<double>::infinity();
        b.hi[c] = -b.lo[c];
    }
    for (int64_t i = 0; i < cnt; ++i)
        for (int c = 0; c < 3; ++c) {
            b.lo[c] = std::min(b.lo[c], pts[3 * i + c]);
            b.hi[c] = std::max(b.hi[c], pts[3 * i + c]);
        }
    return b;
}

bool finite_all(const std::vector<double>& v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

}  // namespace

amm_status validate_pair(const HostPair& hp, std::string& err) {
    if (hp.N < 1 || hp.M < 1 || hp.n < 1) {
        err = "n_src, n_tgt and n_nodes must be >= 1";
        return AMM_ERR_INVALID_ARG;
    }
    if (hp.M >= (1LL << 24) || hp.N >= (1LL << 28)) {
        err = "point count too large";
        return AMM_ERR_INVALID_ARG;
    }
    if (hp.k < 1 || hp.k > kMaxK || hp.k > hp.n) {
        err = fmt("k = %lld must satisfy 1 <= k <= min(8, n_nodes)", hp.k);
        return AMM_ERR_INVALID_ARG;
    }
    if (hp.E < 0) {
        err = "n_edges < 0";
        return AMM_ERR_INVALID_ARG;
    }
    if (!finite_all(hp.src) || !finite_all(hp.tgt) || !finite_all(hp.infl_w) ||
        !finite_all(hp.src_nrm) || !finite_all(hp.tgt_nrm)) {
        err = "non-finite value in the point sets, normals or weights";
        return AMM_ERR_NONFINITE;
    }
    if (!(hp.lbar > 0) || !std::isfinite(hp.lbar)) {
        err = "mean_edge_len must be finite and > 0";
        return AMM_ERR_INVALID_ARG;
    }
    std::vector<char> seen(hp.N, 0);
    for (int64_t j = 0; j < hp.n; ++j) {
        int32_t s = hp.node_idx[j];
        if (s < 0 || s >= hp.N) {
            err = fmt("node_src_idx[%lld] = %lld out of range", j, s);
            return AMM_ERR_INVALID_ARG;
        }
        if (seen[s]) {
            err = fmt("node_src_idx has the source point %lld twice", s);
            return AMM_ERR_GRAPH;
        }
        seen[s] = 1;
    }
    for (int64_t i = 0; i < hp.N; ++i) {
        double sum = 0.0;
        int real = 0;
        for (int a = 0; a < hp.k; ++a) {
            int32_t j = hp.infl_idx[i * hp.k + a];
            double w = hp.infl_w[i * hp.k + a];
            if (j == -1) {   // unused slot
                if (w != 0.0) {
                    err = fmt("unused influence slot (index -1) of point %lld has a nonzero weight", i);
                    return AMM_ERR_INVALID_ARG;
                }
                continue;
            }
            if (j < 0 || j >= hp.n) {
                err = fmt("infl_idx of point %lld out of range (%lld)", i, j);
                return AMM_ERR_INVALID_ARG;
            }
            for (int b = 0; b < a; ++b)
                if (hp.infl_idx[i * hp.k + b] == j) {
                    err = fmt("point %lld lists node %lld twice", i, j);
                    return AMM_ERR_GRAPH;
                }
            if (w < 0) {
                err = fmt("negative influence weight at point %lld", i);
                return AMM_ERR_GRAPH;
            }
            sum += w;
            ++real;
        }
        if (real == 0) {
            err = fmt("point %lld has no influencing node", i);
            return AMM_ERR_GRAPH;
        }
        if (std::fabs(sum - 1.0) > 1e-5) {
            err = fmt("influence weights of point %lld do not sum to 1", i);
            return AMM_ERR_GRAPH;
        }
    }
    std::vector<std::vector<int32_t>> nb(hp.n);
    for (int64_t e = 0; e < hp.E; ++e) {
        int32_t a = hp.edges[2 * e], b = hp.edges[2 * e + 1];
        if (a < 0 || a >= hp.n || b < 0 || b >= hp.n) {
            err = fmt("edge %lld has a node out of range", e);
            return AMM_ERR_INVALID_ARG;
        }
        if (a == b) {
            err = fmt("edge %lld is a self loop", e);
            return AMM_ERR_GRAPH;
        }
        nb[a].push_back(b);
        nb[b].push_back(a);
    }
    for (auto& v : nb) {
        std::sort(v.begin(), v.end());
        if (std::adjacent_find(v.begin(), v.end()) != v.end()) {
            err = "duplicate node edge";
            return AMM_ERR_GRAPH;
        }
    }
    // connectivity (a disconnected graph leaves a free translation when a
    // component's alignment weights all vanish, so K can be singular)
    std::vector<char> vis(hp.n, 0);
    std::vector<int32_t> stack{0};
    vis[0] = 1;
    int64_t cnt = 1;
    while (!stack.empty()) {
        int32_t a = stack.back();
        stack.pop_back();
        for (int32_t b : nb[a])
            if (!vis[b]) {
                vis[b] = 1;
                ++cnt;
                stack.push_back(b);
            }
    }
    if (cnt != hp.n) {
        err = fmt("node graph is disconnected (%lld of %lld nodes reachable)", cnt, hp.n);
        return AMM_ERR_GRAPH;
    }
    return AMM_OK;
}

namespace {

// Runs f(i) for i in [0, n) on up to `threads` host threads (work taken in
// index order from a shared counter).
template <typename F>
void parallel_for(int64_t n, int threads, F&& f) {
    threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, n));
    if (threads == 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&] {
            for (int64_t i = next.fetch_add(1); i < n; i = next.fetch_add(1)) f(i);
        });
    for (auto& th : pool) th.join();
}

int host_threads() {
    const unsigned hc = std::thread::hardware_concurrency();
    return (int)std::min(16u, std::max(1u, hc));
}

// The variable-length parts of one pair's layout, indexed from the pair's
// own start (row pointers local; node ids, point ids and adjacency indices
// already global), concatenated by build_layout in pair order.
struct PairPart {
    PairInfo pi{};
    std::vector<int32_t> K_rowptr;   // [n + 1] local offsets into K_col
    std::vector<int32_t> K_diag;     // [n] local positions of the diagonal blocks
    std::vector<int32_t> K_col, K_adj;
    std::vector<int32_t> pj_rowptr;  // [n + 1] local offsets into the pair's point lists
    std::vector<int32_t> cells;      // octree run-start tables
    std::vector<int32_t> aggs;       // [nagg][4]
    std::vector<int32_t> tile_agg_cnt, tile_agg;
    int max_row_cols = 0;
};

// Everything of pair p: the fixed-size arrays and the point lists (whose
// length, the pair's influence slots that are not padding, is counted
// beforehand) are written in place at the pair's offsets (so, to, no, ao,
// po), the rest goes to `part`.
amm_status build_pair(const HostPair& hp, int p, int k, int leaf, int64_t so, int64_t to, int64_t no, int64_t ao,
                      int64_t po, int64_t pcount, Layout& L, PairPart& part, std::string& err) {
    PairInfo& pi = part.pi;
    pi.src_off = so;
    pi.N = hp.N;
    pi.tgt_off = to;
    pi.M = hp.M;
    pi.node_off = no;
    pi.n = hp.n;
    pi.adj_off = ao;
    pi.nadj = 2 * hp.E;
    pi.n_undirected = (int32_t)hp.E;

    // sources and nodes are ordered within the sources' box, targets
    // within their own (so that new targets leave the source side as is)
    const Box bb = bounds(hp.src.data(), hp.N);

    // source points in Morton order
    std::vector<int32_t> sord = morton_order(hp.src.data(), hp.N, bb);
    // nodes in Morton order of their positions
    std::vector<double> npos(3 * hp.n);
    for (int64_t j = 0; j < hp.n; ++j)
        for (int c = 0; c < 3; ++c) npos[3 * j + c] = hp.src[3 * hp.node_idx[j] + c];
    std::vector<int32_t> nord = morton_order(npos.data(), hp.n, bb);
    std::vector<int32_t> n_inv(hp.n);
    for (int64_t q = 0; q < hp.n; ++q) n_inv[nord[q]] = (int32_t)q;

    for (int64_t q = 0; q < hp.N; ++q) {
        int64_t u = sord[q];
        for (int c = 0; c < 3; ++c) L.src4[4 * (so + q) + c] = hp.src[3 * u + c];
        L.src4[4 * (so + q) + 3] = 0.0;
        L.src_user[so + q] = (int32_t)(so + u);
        L.src_internal[so + u] = (int32_t)(so + q);
        // an unused slot points at the point's first influencing node with
        // weight 0, so the kernels read valid data and add nothing; it takes
        // no part in K's pattern or the node point lists
        int a0 = 0;
        while (hp.infl_idx[u * k + a0] == -1) ++a0;
        for (int a = 0; a < k; ++a) {
            const bool pad = hp.infl_idx[u * k + a] == -1;
            const int32_t j = hp.infl_idx[u * k + (pad ? a0 : a)];
            const double w = pad ? 0.0 : hp.infl_w[u * k + a];
            L.iidx[(size_t)a * L.Ntot + so + q] = (int32_t)(no + n_inv[j]);
            L.ipad[(size_t)a * L.Ntot + so + q] = pad ? 1 : 0;
            L.iw[(size_t)a * L.Ntot + so + q] = w;
        }
    }
    for (int64_t q = 0; q < hp.n; ++q) {
        int64_t u = nord[q];
        for (int c = 0; c < 3; ++c) L.nodes4[4 * (no + q) + c] = npos[3 * u + c];
        L.node_user[no + q] = (int32_t)(no + u);
        L.node_internal[no + u] = (int32_t)(no + q);
        L.node_pair[no + q] = p;
    }

    // adjacency (directed), r_ij of Eq. (8)
    std::vector<std::vector<int32_t>> nb(hp.n);
    for (int64_t e = 0; e < hp.E; ++e) {
        int32_t a = n_inv[hp.edges[2 * e]], b = n_inv[hp.edges[2 * e + 1]];
        nb[a].push_back(b);
        nb[b].push_back(a);
    }
    long double inv_sum = 0.0L;
    for (int64_t e = 0; e < hp.E; ++e) {
        const double* pa = &npos[3 * hp.edges[2 * e]];
        const double* pb = &npos[3 * hp.edges[2 * e + 1]];
        double d = std::sqrt((pa[0] - pb[0]) * (pa[0] - pb[0]) +
                             (pa[1] - pb[1]) * (pa[1] - pb[1]) +
                             (pa[2] - pb[2]) * (pa[2] - pb[2]));
        if (!(d > 0)) {
            err = "node edge of zero length";
            return AMM_ERR_GRAPH;
        }
        inv_sum += 1.0L / d;
    }
    int64_t at = ao;
    for (int64_t q = 0; q < hp.n; ++q) {
        std::sort(nb[q].begin(), nb[q].end());
        L.adj_ptr[no + q] = (int32_t)at;
        for (int32_t b : nb[q]) {
            L.adj_nbr[at] = (int32_t)(no + b);
            L.adj_row[at] = (int32_t)(no + q);
            const double* pa = &L.nodes4[4 * (no + q)];
            const double* pb = &L.nodes4[4 * (no + b)];
            double d = std::sqrt((pa[0] - pb[0]) * (pa[0] - pb[0]) +
                                 (pa[1] - pb[1]) * (pa[1] - pb[1]) +
                                 (pa[2] - pb[2]) * (pa[2] - pb[2]));
            // 2|E| d^-1 / (sum over ordered pairs of d^-1) = |E| d^-1 / sum over edges
            L.adj_r[at] = (double)((long double)hp.E / (long double)d / inv_sum);
            ++at;
        }
    }
    for (int64_t e = ao; e < at; ++e) {
        int32_t a = L.adj_row[e], b = L.adj_nbr[e];
        auto beg = L.adj_nbr.begin() + L.adj_ptr[b];
        auto end = beg + (int64_t)nb[b - no].size();
        auto it = std::lower_bound(beg, end, a);
        L.adj_rev[e] = (int32_t)(L.adj_ptr[b] + (it - beg));
    }

    // points influenced by each node (entries (point << 3) | slot, in point
    // order), by counting
    part.pj_rowptr.assign(hp.n + 1, 0);
    for (int64_t q = 0; q < hp.N; ++q)
        for (int a = 0; a < k; ++a)
            if (!L.ipad[(size_t)a * L.Ntot + so + q]) ++part.pj_rowptr[L.iidx[(size_t)a * L.Ntot + so + q] - no + 1];
    for (int64_t q = 0; q < hp.n; ++q) part.pj_rowptr[q + 1] += part.pj_rowptr[q];
    if (part.pj_rowptr[hp.n] != pcount) {
        err = "point list length differs from the count of influence slots";
        return AMM_ERR_INVALID_ARG;
    }
    int32_t* const pj_ent = L.pj_ent.data() + po;
    uint64_t* const pj_pos = L.pj_pos.data() + po;
    {
        std::vector<int32_t> fill(part.pj_rowptr.begin(), part.pj_rowptr.end() - 1);
        for (int64_t q = 0; q < hp.N; ++q)
            for (int a = 0; a < k; ++a) {
                if (L.ipad[(size_t)a * L.Ntot + so + q]) continue;
                const int64_t ja = L.iidx[(size_t)a * L.Ntot + so + q] - no;
                pj_ent[fill[ja]++] = (int32_t)(((so + q) << 3) | a);
            }
    }
    // block pattern of K, row by row: the diagonal, the nodes that share an
    // influenced point with the row's node, and its graph neighbours
    // (distinct, sorted); then each point entry's k column positions
    part.K_rowptr.assign(hp.n + 1, 0);
    part.K_diag.assign(hp.n, 0);
    {
        std::vector<int32_t> mark(hp.n, -1), posof(hp.n, 0), c;
        c.reserve(256);
        for (int64_t q = 0; q < hp.n; ++q) {
            c.clear();
            auto add = [&](int32_t col) {
                if (mark[col - no] != (int32_t)q) {
                    mark[col - no] = (int32_t)q;
                    c.push_back(col);
                }
            };
            add((int32_t)(no + q));
            for (int32_t e = part.pj_rowptr[q]; e < part.pj_rowptr[q + 1]; ++e) {
                const int64_t i = pj_ent[e] >> 3;
                for (int b = 0; b < k; ++b)
                    if (!L.ipad[(size_t)b * L.Ntot + i]) add(L.iidx[(size_t)b * L.Ntot + i]);
            }
            for (int32_t b : nb[q]) add((int32_t)(no + b));
            std::sort(c.begin(), c.end());
            if ((int)c.size() > kMaxCols) {
                err = fmt("a node is coupled to %lld others (limit %lld)", (long long)c.size(), kMaxCols);
                return AMM_ERR_INVALID_ARG;
            }
            part.max_row_cols = std::max(part.max_row_cols, (int)c.size());
            part.K_rowptr[q] = (int32_t)part.K_col.size();
            for (size_t t = 0; t < c.size(); ++t) {
                const int32_t col = c[t];
                posof[col - no] = (int32_t)t;
                if (col == no + q) part.K_diag[q] = (int32_t)part.K_col.size();
                int32_t adj = -1;
                if (col != no + q) {
                    auto beg = L.adj_nbr.begin() + L.adj_ptr[no + q];
                    auto end = beg + (int64_t)nb[q].size();
                    auto it = std::lower_bound(beg, end, col);
                    if (it != end && *it == col) adj = (int32_t)(it - L.adj_nbr.begin());
                }
                part.K_col.push_back(col);
                part.K_adj.push_back(adj);
            }
            for (int32_t e = part.pj_rowptr[q]; e < part.pj_rowptr[q + 1]; ++e) {
                const int64_t i = pj_ent[e] >> 3;
                uint64_t pos = 0;
                for (int b = 0; b < k; ++b) {
                    uint64_t bpos = kPosUnused;
                    if (!L.ipad[(size_t)b * L.Ntot + i]) bpos = (uint64_t)posof[L.iidx[(size_t)b * L.Ntot + i] - no];
                    pos |= bpos << (8 * b);
                }
                pj_pos[e] = pos;
            }
        }
    }
    part.K_rowptr[hp.n] = (int32_t)part.K_col.size();

    // targets: Morton order and the octree's run-start tables
    {
        TargetLayout tl;
        target_layout(hp.tgt.data(), hp.M, leaf, tl);
        std::copy(tl.tgt4.begin(), tl.tgt4.end(), L.tgt4.begin() + 4 * to);
        std::copy(tl.tgt_user.begin(), tl.tgt_user.end(), L.tgt_user.begin() + to);
        pi.grid_bits = tl.grid_bits;
        for (int c = 0; c < 3; ++c) {
            pi.glo[c] = tl.glo[c];
            pi.gscale[c] = tl.gscale[c];
            pi.cs[c] = tl.cs[c];
        }
        pi.gpad = tl.gpad;
        part.cells = std::move(tl.cells);
    }

    // coarse aggregates: the fewest power-of-two runs of whole node tiles
    // that leave at most kCoarseMaxAgg of them
    int shift = kAggMinShift;
    while (((hp.n + (int64_t(1) << shift) - 1) >> shift) > kCoarseMaxAgg) ++shift;
    const int64_t per = int64_t(1) << shift;
    pi.agg_shift = shift;
    pi.nagg = (int32_t)((hp.n + per - 1) / per);
    for (int32_t a = 0; a < pi.nagg; ++a) {
        const int64_t s0 = a * per, s1 = std::min<int64_t>(s0 + per, hp.n);
        double ctr[3] = {0, 0, 0};
        for (int64_t q = s0; q < s1; ++q)
            for (int c = 0; c < 3; ++c) ctr[c] += L.nodes4[4 * (no + q) + c];
        for (int c = 0; c < 3; ++c) ctr[c] /= (double)(s1 - s0);
        for (int64_t q = s0; q < s1; ++q)
            for (int c = 0; c < 3; ++c) L.node_rel[4 * (no + q) + c] = L.nodes4[4 * (no + q) + c] - ctr[c];
        part.aggs.insert(part.aggs.end(), {p, (int32_t)(no + s0), (int32_t)(no + s1), a});
    }
    // per node tile, the sorted pair-local aggregates its rows of K touch
    const int64_t ntile = (hp.n + kNodeTile - 1) / kNodeTile;
    for (int64_t t = 0; t < ntile; ++t) {
        std::vector<int32_t> ag;
        const int64_t q0 = t * kNodeTile, q1 = std::min<int64_t>(q0 + kNodeTile, hp.n);
        for (int32_t e = part.K_rowptr[q0]; e < part.K_rowptr[q1]; ++e)
            ag.push_back((int32_t)((part.K_col[e] - no) >> shift));
        std::sort(ag.begin(), ag.end());
        ag.erase(std::unique(ag.begin(), ag.end()), ag.end());
        part.tile_agg.insert(part.tile_agg.end(), ag.begin(), ag.end());
        part.tile_agg_cnt.push_back((int32_t)ag.size());
    }
    return AMM_OK;
}

}  // namespace

amm_status validate_pairs(const std::vector<HostPair>& pairs, std::string& err) {
    const int64_t P = (int64_t)pairs.size();
    std::vector<amm_status> sts(P, AMM_OK);
    std::vector<std::string> errs(P);
    parallel_for(P, host_threads(), [&](int64_t p) { sts[p] = validate_pair(pairs[p], errs[p]); });
    for (int64_t p = 0; p < P; ++p)
        if (sts[p] != AMM_OK) {
            err = fmt("problem %lld: ", p) + errs[p];
            return sts[p];
        }
    return AMM_OK;
}

amm_status build_layout(const std::vector<HostPair>& pairs, int leaf, Layout& L,
                        std::string& err) {
    L = Layout();
    L.P = (int)pairs.size();
    L.k = pairs.empty() ? 0 : pairs[0].k;
    std::vector<int64_t> so(L.P + 1, 0), to(L.P + 1, 0), no(L.P + 1, 0), ao(L.P + 1, 0);
    for (int p = 0; p < L.P; ++p) {
        const HostPair& hp = pairs[p];
        if (hp.k != L.k) {
            err = "all pairs of a batch must have the same k";
            return AMM_ERR_INVALID_ARG;
        }
        so[p + 1] = so[p] + hp.N;
        to[p + 1] = to[p] + hp.M;
        no[p + 1] = no[p] + hp.n;
        ao[p + 1] = ao[p] + 2 * hp.E;
    }
    L.Ntot = so[L.P];
    L.Mtot = to[L.P];
    L.ntot = no[L.P];
    L.nadj = ao[L.P];
    const int k = L.k;
    // (written in full by the pairs' threads)
    L.src4.resize(4 * L.Ntot);
    L.src_user.resize(L.Ntot);
    L.src_internal.resize(L.Ntot);
    L.iidx.resize((size_t)k * L.Ntot);
    L.iw.resize((size_t)k * L.Ntot);
    L.ipad.resize((size_t)k * L.Ntot);
    L.nodes4.assign(4 * L.ntot, 0.0);
    L.node_user.resize(L.ntot);
    L.node_internal.resize(L.ntot);
    L.node_pair.resize(L.ntot);
    L.node_rel.assign(4 * L.ntot, 0.0);
    L.adj_ptr.assign(L.ntot + 1, 0);
    L.adj_nbr.resize(L.nadj);
    L.adj_row.resize(L.nadj);
    L.adj_rev.resize(L.nadj);
    L.adj_r.resize(L.nadj);
    L.K_ptr.assign(L.ntot + 1, 0);
    L.K_diag.resize(L.ntot);
    L.pj_ptr.assign(L.ntot + 1, 0);
    L.tgt4.resize(4 * L.Mtot);
    L.tgt_user.resize(L.Mtot);

    // the point lists' offsets: one entry per influence slot that is not
    // padding
    std::vector<int64_t> pb(L.P + 1, 0);
    parallel_for(L.P, host_threads(), [&](int64_t p) {
        const HostPair& hp = pairs[p];
        int64_t c = 0;
        for (size_t e = 0; e < hp.infl_idx.size(); ++e) c += hp.infl_idx[e] != -1;
        pb[p + 1] = c;
    });
    for (int p = 0; p < L.P; ++p) pb[p + 1] += pb[p];
    if (pb[L.P] >= INT32_MAX) {
        err = "the batch's point lists exceed 32-bit indexing";
        return AMM_ERR_INVALID_ARG;
    }
    L.pj_ent.resize(pb[L.P]);
    L.pj_pos.resize(pb[L.P]);

    // pairs in parallel (each writes its own ranges), then merged in order
    std::vector<PairPart> parts(L.P);
    std::vector<amm_status> sts(L.P, AMM_OK);
    std::vector<std::string> errs(L.P);
    // the largest pairs first, so that no large one is left for the end
    std::vector<int32_t> by_size(L.P);
    std::iota(by_size.begin(), by_size.end(), 0);
    std::stable_sort(by_size.begin(), by_size.end(), [&](int32_t a, int32_t b) {
        return pairs[a].N + pairs[a].M > pairs[b].N + pairs[b].M;
    });
    parallel_for(L.P, host_threads(), [&](int64_t r) {
        const int p = by_size[r];
        sts[p] = build_pair(pairs[p], p, k, leaf, so[p], to[p], no[p], ao[p], pb[p], pb[p + 1] - pb[p], L, parts[p],
                            errs[p]);
    });
    for (int p = 0; p < L.P; ++p)
        if (sts[p] != AMM_OK) {
            err = errs[p];
            return sts[p];
        }
    // offsets of every pair's variable-length parts, then the copies (in
    // parallel: disjoint ranges)
    std::vector<int64_t> kb(L.P + 1, 0), cb(L.P + 1, 0), gb(L.P + 1, 0), tb(L.P + 1, 0);
    for (int p = 0; p < L.P; ++p) {
        kb[p + 1] = kb[p] + (int64_t)parts[p].K_col.size();
        cb[p + 1] = cb[p] + (int64_t)parts[p].cells.size();
        gb[p + 1] = gb[p] + (int64_t)parts[p].aggs.size();
        tb[p + 1] = tb[p] + (int64_t)parts[p].tile_agg.size();
    }
    if (kb[L.P] >= INT32_MAX) {
        err = "the batch's blocks of K exceed 32-bit indexing";
        return AMM_ERR_INVALID_ARG;
    }
    L.K_col.resize(kb[L.P]);
    L.K_adj.resize(kb[L.P]);
    L.grid_cells.resize(cb[L.P]);
    L.aggs.resize(gb[L.P]);
    L.tile_agg.resize(tb[L.P]);
    parallel_for(L.P, host_threads(), [&](int64_t r) {
        const int p = by_size[r];
        PairPart& part = parts[p];
        const int64_t n = pairs[p].n;
        for (int64_t q = 0; q < n; ++q) {
            L.K_ptr[no[p] + q] = (int32_t)(kb[p] + part.K_rowptr[q]);
            L.K_diag[no[p] + q] = (int32_t)(kb[p] + part.K_diag[q]);
            L.pj_ptr[no[p] + q] = (int32_t)(pb[p] + part.pj_rowptr[q]);
        }
        std::copy(part.K_col.begin(), part.K_col.end(), L.K_col.begin() + kb[p]);
        std::copy(part.K_adj.begin(), part.K_adj.end(), L.K_adj.begin() + kb[p]);
        std::copy(part.cells.begin(), part.cells.end(), L.grid_cells.begin() + cb[p]);
        std::copy(part.aggs.begin(), part.aggs.end(), L.aggs.begin() + gb[p]);
        std::copy(part.tile_agg.begin(), part.tile_agg.end(), L.tile_agg.begin() + tb[p]);
        // the copied parts are released here, in parallel
        std::vector<int32_t>().swap(part.K_rowptr);
        std::vector<int32_t>().swap(part.K_diag);
        std::vector<int32_t>().swap(part.K_col);
        std::vector<int32_t>().swap(part.K_adj);
        std::vector<int32_t>().swap(part.pj_rowptr);
        std::vector<int32_t>().swap(part.cells);
        std::vector<int32_t>().swap(part.tile_agg);
    });
    L.tile_agg_ptr.push_back(0);
    for (int p = 0; p < L.P; ++p) {
        const PairPart& part = parts[p];
        PairInfo pi = part.pi;
        const int64_t n = pairs[p].n, N = pairs[p].N, E = pairs[p].E;
        L.max_row_cols = std::max(L.max_row_cols, part.max_row_cols);
        pi.grid_off = cb[p];
        // tiles
        pi.pt_tile0 = L.n_pt_tiles;
        for (int64_t s = 0; s < N; s += kPointTile) {
            L.pt_tiles.insert(L.pt_tiles.end(),
                              {p, (int32_t)(so[p] + s), (int32_t)(so[p] + std::min<int64_t>(s + kPointTile, N)), 0});
            ++L.n_pt_tiles;
        }
        pi.pt_ntile = L.n_pt_tiles - pi.pt_tile0;
        pi.nd_tile0 = L.n_nd_tiles;
        for (int64_t s = 0; s < n; s += kNodeTile) {
            L.nd_tiles.insert(L.nd_tiles.end(),
                              {p, (int32_t)(no[p] + s), (int32_t)(no[p] + std::min<int64_t>(s + kNodeTile, n)), 0});
            ++L.n_nd_tiles;
        }
        pi.nd_ntile = L.n_nd_tiles - pi.nd_tile0;
        // coarse level
        pi.agg0 = (int32_t)L.nagg;
        pi.ainv_off = L.ainv_size;
        L.ainv_size += (int64_t)(4 * pi.nagg) * (4 * pi.nagg);
        L.nagg += pi.nagg;
        int64_t o = tb[p];
        for (int32_t c : part.tile_agg_cnt) {
            o += c;
            L.tile_agg_ptr.push_back((int32_t)o);
        }
        pi.eg_tile0 = L.n_eg_tiles;
        for (int64_t s = 0; s < 2 * E; s += kEdgeTile) {
            L.eg_tiles.insert(L.eg_tiles.end(), {p, (int32_t)(ao[p] + s),
                                                 (int32_t)(ao[p] + std::min<int64_t>(s + kEdgeTile, 2 * E)), 0});
            ++L.n_eg_tiles;
        }
        pi.eg_ntile = L.n_eg_tiles - pi.eg_tile0;
        L.info.push_back(pi);
    }
    parts.clear();
    L.adj_ptr[L.ntot] = (int32_t)L.nadj;
    L.K_ptr[L.ntot] = (int32_t)L.K_col.size();
    L.pj_ptr[L.ntot] = (int32_t)L.pj_ent.size();
    L.tile_cols.assign((size_t)L.n_nd_tiles * kTileColCap, 0);
    L.tile_ncols.assign(L.n_nd_tiles, 0);
    L.tile_rowl.assign((size_t)L.n_nd_tiles * kNodeTile, 0);
    L.K_lcol.assign(L.K_col.size(), 0);
    parallel_for(L.n_nd_tiles, host_threads(), [&](int64_t t) {
        const int32_t j0 = L.nd_tiles[4 * (size_t)t + 1], j1 = L.nd_tiles[4 * (size_t)t + 2];
        std::vector<int32_t> cols(L.K_col.begin() + L.K_ptr[j0], L.K_col.begin() + L.K_ptr[j1]);
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        L.tile_ncols[t] = (int32_t)cols.size();
        if ((int)cols.size() > kTileColCap) return;
        int32_t* dst = &L.tile_cols[(size_t)t * kTileColCap];
        for (int q = 0; q < kTileColCap; ++q) dst[q] = cols[q < (int)cols.size() ? q : 0];
        auto local = [&](int32_t node) {
            return (int32_t)(std::lower_bound(cols.begin(), cols.end(), node) - cols.begin());
        };
        for (int32_t j = j0; j < j1; ++j) {
            L.tile_rowl[(size_t)t * kNodeTile + (j - j0)] = local(j);
            for (int32_t e = L.K_ptr[j]; e < L.K_ptr[j + 1]; ++e) L.K_lcol[e] = (uint16_t)local(L.K_col[e]);
        }
    });
    L.nnzb = (int64_t)L.K_col.size();
    L.pj_entries = (int64_t)L.pj_ent.size();
    return AMM_OK;
}

void target_frame(const double lo[3], const double hi[3], TargetLayout& out) {
    double emax = 0, amax = 0;
    for (int c = 0; c < 3; ++c) {
        const double ext = hi[c] - lo[c];
        out.glo[c] = lo[c];
        out.gscale[c] = ext > 0 ? 1023.999 / ext : 0.0;
        // root cell: quantized coordinates 0..1023 span 1024 / gscale
        out.cs[c] = ext > 0 ? 1024.0 / out.gscale[c] : 0.0;
        emax = std::max(emax, ext);
        amax = std::max({amax, std::fabs(lo[c]), std::fabs(hi[c])});
    }
    // the cell bounds are formed in the search's precision (float32 on the
    // FP32 path) from coordinates up to amax: a relative 1e-6 of the extent
    // plus 16 float32 ulps of the largest coordinate covers their rounding
    // and that of the stored targets
    out.gpad = 1e-6 * emax + 16.0 * std::ldexp(amax, -24);
}

void target_layout(const double* tgt, int64_t M, int leaf, TargetLayout& out, int depth) {
    const Box bb = bounds(tgt, M);
    std::vector<uint32_t> code(M);
    for (int64_t i = 0; i < M; ++i) code[i] = morton(tgt + 3 * i, bb);
    const std::vector<int32_t> tord = code_order(code);
    out.tgt4.assign(4 * (size_t)M, 0.0);
    out.tgt_user.resize(M);
    for (int64_t q = 0; q < M; ++q) {
        const int64_t u = tord[q];
        for (int c = 0; c < 3; ++c) out.tgt4[4 * q + c] = tgt[3 * u + c];
        out.tgt4[4 * q + 3] = (double)u;
        out.tgt_user[q] = (int32_t)u;
    }
    // depth: the smallest whose occupied leaf cells average at most `leaf`
    // targets (occupied cells counted as distinct code prefixes)
    int G = depth;
    if (G < 2 || G > kOctMaxDepth) {
        G = kOctMaxDepth;
        for (int g = 2; g < kOctMaxDepth; ++g) {
            const int sh = 3 * (10 - g);
            int64_t occ = 0;
            for (int64_t q = 0; q < M; ++q)
                if (q == 0 || (code[tord[q]] >> sh) != (code[tord[q - 1]] >> sh)) ++occ;
            if (occ > 0 && (double)M <= (double)leaf * (double)occ) {
                G = g;
                break;
            }
        }
    }
    out.grid_bits = G;
    target_frame(bb.lo, bb.hi, out);
    // leaf-level run starts by counting, coarser levels by sampling them
    const size_t nleaf = (size_t)1 << (3 * G);
    std::vector<int32_t> leafst(nleaf + 1, 0);
    for (int64_t q = 0; q < M; ++q) ++leafst[(code[tord[q]] >> (3 * (10 - G))) + 1];
    for (size_t m = 0; m < nleaf; ++m) leafst[m + 1] += leafst[m];
    out.cells.assign((size_t)oct_level_off(G + 1), 0);
    for (int l = 0; l <= G; ++l) {
        int32_t* tab = out.cells.data() + oct_level_off(l);
        const size_t nc = (size_t)1 << (3 * l);
        for (size_t m = 0; m <= nc; ++m) tab[m] = leafst[m << (3 * (G - l))];
    }
}

}  // namespace amm
