// Deformation-graph construction of Sec. 3.1 (Alg. 1) on the device, with
// Euclidean distance in place of the geodesic one.
//
// Alg. 1 walks the source points in the order of their projection onto the
// principal axis and makes a point a node when no earlier node lies within
// R of it.  That is the lexicographically first maximal independent set of
// the graph "distance < R" under this order, which is unique: a point's
// decision depends only on the decisions of the earlier points within R.  It
// is computed here in rounds over all points: a point becomes covered as
// soon as an earlier neighbour is a node, and a node as soon as all its
// earlier neighbours are covered.  Each round decides at least the earliest
// undecided point, and the result equals the sequential pass exactly.
//
// Neighbour queries use a uniform grid stored as points sorted by cell key
// (a stable radix sort), with each occupied cell's 27 neighbour ranges
// precomputed.  "Within R" is ((dx*dx + dy*dy) + dz*dz) < R*R in float64
// with every operation rounded on its own (no contraction), so that the
// integer decisions of the graph match a plain float64 evaluation.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "amm.h"
#include "amm_internal.h"

namespace amm {

namespace {

constexpr int kGT = 256;
constexpr int kKnn = 6;                       // neighbours of the mean-edge-length graph
constexpr uint64_t kNoKey = ~uint64_t(0);

#define TRY_STATUS(x)                   \
    do {                                \
        const amm_status s_ = (x);      \
        if (s_ != AMM_OK) return s_;    \
    } while (0)

#define GCHK(x)                                                   \
    do {                                                          \
        hipError_t e_ = (x);                                      \
        if (e_ != hipSuccess) {                                   \
            err = std::string(#x) + ": " + hipGetErrorString(e_); \
            return e_ == hipErrorOutOfMemory ? AMM_ERR_OOM : AMM_ERR_HIP; \
        }                                                         \
    } while (0)

__device__ __forceinline__ double gd2(const double4& a, const double4& b) {
#pragma clang fp contract(off)
    const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    return (dx * dx + dy * dy) + dz * dz;
}

template <int NT>
__device__ __forceinline__ double bsum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <int NT, bool MAX>
__device__ __forceinline__ double bext(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            sh[threadIdx.x] = MAX ? fmax(sh[threadIdx.x], sh[threadIdx.x + s])
                                  : fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- statistics

// Source points as double4, and per block: min, max and sum of x, y, z and
// the count of non-finite coordinates.
template <typename T>
__global__ void __launch_bounds__(kGT) k_g_load(const T* __restrict__ v, double4* __restrict__ P, int64_t N,
                                                double* __restrict__ part) {
    __shared__ double sh[kGT];
    const int64_t i = (int64_t)blockIdx.x * kGT + threadIdx.x;
    double x = 0, y = 0, z = 0, bad = 0;
    const bool live = i < N;
    if (live) {
        x = (double)v[3 * i];
        y = (double)v[3 * i + 1];
        z = (double)v[3 * i + 2];
        bad = (std::isfinite(x) && std::isfinite(y) && std::isfinite(z)) ? 0.0 : 1.0;
        P[i] = make_double4(x, y, z, 0.0);
    }
    const double inf = __builtin_inf();
    double r[10];
    r[0] = bext<kGT, false>(live ? x : inf, sh);
    r[1] = bext<kGT, false>(live ? y : inf, sh);
    r[2] = bext<kGT, false>(live ? z : inf, sh);
    r[3] = bext<kGT, true>(live ? x : -inf, sh);
    r[4] = bext<kGT, true>(live ? y : -inf, sh);
    r[5] = bext<kGT, true>(live ? z : -inf, sh);
    r[6] = bsum<kGT>(x, sh);
    r[7] = bsum<kGT>(y, sh);
    r[8] = bsum<kGT>(z, sh);
    r[9] = bsum<kGT>(bad, sh);
    if (threadIdx.x < 10) {
        double o = r[0];
#pragma unroll
        for (int m = 1; m < 10; ++m) o = (int)threadIdx.x == m ? r[m] : o;
        part[10 * (size_t)blockIdx.x + threadIdx.x] = o;
    }
}

// Per block: sum of (v - m)(v - m)^T (xx, xy, xz, yy, yz, zz).
__global__ void __launch_bounds__(kGT) k_g_cov(const double4* __restrict__ P, int64_t N, double mx, double my,
                                               double mz, double* __restrict__ part) {
    __shared__ double sh[kGT];
    const int64_t i = (int64_t)blockIdx.x * kGT + threadIdx.x;
    double dx = 0, dy = 0, dz = 0;
    if (i < N) {
        const double4 p = P[i];
        dx = p.x - mx;
        dy = p.y - my;
        dz = p.z - mz;
    }
    double r[6];
    r[0] = bsum<kGT>(dx * dx, sh);
    r[1] = bsum<kGT>(dx * dy, sh);
    r[2] = bsum<kGT>(dx * dz, sh);
    r[3] = bsum<kGT>(dy * dy, sh);
    r[4] = bsum<kGT>(dy * dz, sh);
    r[5] = bsum<kGT>(dz * dz, sh);
    if (threadIdx.x < 6) {
        double o = r[0];
#pragma unroll
        for (int m = 1; m < 6; ++m) o = (int)threadIdx.x == m ? r[m] : o;
        part[6 * (size_t)blockIdx.x + threadIdx.x] = o;
    }
}

// Projection onto the principal axis (+0.0 folds -0.0 into +0.0, so that
// equal projections sort by index).
__global__ void __launch_bounds__(kGT) k_g_project(const double4* __restrict__ P, int64_t N, double mx,
                                                   double my, double mz, double ax, double ay, double az,
                                                   double* __restrict__ key, int* __restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (i >= N) return;
    const double4 p = P[i];
    key[i] = ((p.x - mx) * ax + (p.y - my) * ay + (p.z - mz) * az) + 0.0;
    val[i] = (int)i;
}

__global__ void __launch_bounds__(kGT) k_g_invert(const int* __restrict__ order, int* __restrict__ rank, int64_t N) {
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (s < N) rank[order[s]] = (int)s;
}

// ---------------------------------------------------------------- sorted-cell grid

struct GridDims {
    double x0, y0, z0, h;
    int64_t nx, ny, nz;
};

__device__ __forceinline__ int64_t cell_coord(double v, double v0, double h, int64_t n) {
    int64_t c = (int64_t)floor((v - v0) / h);
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

__global__ void __launch_bounds__(kGT) k_g_cellkey(const double4* __restrict__ P, int64_t N, GridDims g,
                                                   uint64_t* __restrict__ key, int* __restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (i >= N) return;
    const double4 p = P[i];
    const int64_t cx = cell_coord(p.x, g.x0, g.h, g.nx), cy = cell_coord(p.y, g.y0, g.h, g.ny),
                  cz = cell_coord(p.z, g.z0, g.h, g.nz);
    key[i] = (uint64_t)((cz * g.ny + cy) * g.nx + cx);
    val[i] = (int)i;
}

// Points in cell order: position, rank along the axis, and 1 at the first
// point of every occupied cell.
__global__ void __launch_bounds__(kGT) k_g_gather(const uint64_t* __restrict__ ck, const int* __restrict__ cp,
                                                  const double4* __restrict__ P, const int* __restrict__ rank,
                                                  int64_t N, double4* __restrict__ Ps, int* __restrict__ rs,
                                                  int* __restrict__ head) {
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (s >= N) return;
    const int i = cp[s];
    Ps[s] = P[i];
    if (rs) rs[s] = rank[i];
    head[s] = (s == 0 || ck[s] != ck[s - 1]) ? 1 : 0;
}

// Occupied cells: key and first sorted position; cell of every sorted point.
__global__ void __launch_bounds__(kGT) k_g_cells(const uint64_t* __restrict__ ck, const int* __restrict__ head,
                                                 const int* __restrict__ uid_incl, int64_t N,
                                                 uint64_t* __restrict__ ukey, int* __restrict__ ustart,
                                                 int* __restrict__ us) {
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (s >= N) return;
    const int u = uid_incl[s] - 1;
    us[s] = u;
    if (head[s]) {
        ukey[u] = ck[s];
        ustart[u] = (int)s;
    }
}

__device__ __forceinline__ int find_cell(const uint64_t* __restrict__ ukey, int nu, uint64_t key) {
    int lo = 0, hi = nu;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ukey[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < nu && ukey[lo] == key) ? lo : -1;
}

// For every occupied cell the sorted-position ranges of its 27 neighbour
// cells (itself included), empty ones as (0, 0).
__global__ void __launch_bounds__(kGT) k_g_nbr(const uint64_t* __restrict__ ukey, const int* __restrict__ ustart,
                                               int nu, int64_t N, GridDims g, int2* __restrict__ nb) {
    const int u = blockIdx.x * kGT + threadIdx.x;
    if (u >= nu) return;
    const uint64_t key = ukey[u];
    const int64_t cx = (int64_t)(key % (uint64_t)g.nx);
    const int64_t cy = (int64_t)((key / (uint64_t)g.nx) % (uint64_t)g.ny);
    const int64_t cz = (int64_t)(key / ((uint64_t)g.nx * (uint64_t)g.ny));
    int o = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx, ++o) {
                const int64_t x = cx + dx, y = cy + dy, z = cz + dz;
                int2 r = make_int2(0, 0);
                if (x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz) {
                    const int c = find_cell(ukey, nu, (uint64_t)((z * g.ny + y) * g.nx + x));
                    if (c >= 0) r = make_int2(ustart[c], c + 1 < nu ? ustart[c + 1] : (int)N);
                }
                nb[27 * (size_t)u + o] = r;
            }
}

// ---------------------------------------------------------------- node selection

// One round over the undecided points (cell order).  state: 0 undecided,
// 1 node, 2 covered.  Reads of other points' states may see the value of
// the previous round or of this one; both are final or undecided, so a
// decision taken is always the sequential pass's.
__global__ void __launch_bounds__(kGT) k_g_round(const double4* __restrict__ Ps, const int* __restrict__ rs,
                                                 const int* __restrict__ us, const int2* __restrict__ nb,
                                                 int* state, int64_t N, double R2, int* __restrict__ remaining) {
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    bool undecided = false;
    if (s < N && __hip_atomic_load(&state[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        const double4 q = Ps[s];
        const int rq = rs[s];
        const int2* cells = nb + 27 * (size_t)us[s];
        bool covered = false, pending = false;
        for (int o = 0; o < 27 && !covered; ++o) {
            const int2 r = cells[o];
            for (int t = r.x; t < r.y; ++t) {
                if (rs[t] >= rq) continue;
                if (!(gd2(Ps[t], q) < R2)) continue;
                const int st = __hip_atomic_load(&state[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (st == 1) {
                    covered = true;
                    break;
                }
                if (st == 0) pending = true;
            }
        }
        if (covered)
            __hip_atomic_store(&state[s], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else if (!pending)
            __hip_atomic_store(&state[s], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            undecided = true;
    }
    const int cnt = __syncthreads_count(undecided);
    if (threadIdx.x == 0 && cnt) atomicAdd(remaining, cnt);
}

// Axis order -> node flag (for the node numbering scan).
__global__ void __launch_bounds__(kGT) k_g_nodeflag(const int* __restrict__ rs, const int* __restrict__ state,
                                                    int64_t N, int* __restrict__ flag_by_rank,
                                                    int* __restrict__ pos_by_rank) {
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (s >= N) return;
    flag_by_rank[rs[s]] = state[s] == 1 ? 1 : 0;
    pos_by_rank[rs[s]] = (int)s;
}

// exclusive = inclusive - own flag
__global__ void __launch_bounds__(kGT) k_g_excl_from_incl(const int* __restrict__ incl, const int* __restrict__ flag,
                                                          int64_t N, int* __restrict__ excl) {
    const int64_t r = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (r < N) excl[r] = incl[r] - flag[r];
}

__global__ void __launch_bounds__(kGT) k_g_nodeid(const int* __restrict__ flag_by_rank,
                                                  const int* __restrict__ nid_by_rank,
                                                  const int* __restrict__ pos_by_rank, const int* __restrict__ cp,
                                                  int64_t N, int* __restrict__ nid_s, int* __restrict__ node_src) {
    const int64_t r = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (r >= N) return;
    const int s = pos_by_rank[r];
    if (flag_by_rank[r]) {
        nid_s[s] = nid_by_rank[r];
        node_src[nid_by_rank[r]] = cp[s];
    } else {
        nid_s[s] = -1;
    }
}

// ---------------------------------------------------------------- influence sets

// (d, id) ordered by distance, then id.
__device__ __forceinline__ bool before(double d1, int i1, double d2, int i2) {
    return d1 < d2 || (d1 == d2 && i1 < i2);
}

// Inserts (d, id) into the ascending list (bd, bi) of capacity cap (<= 8),
// compile-time indices only.
__device__ __forceinline__ void topk_insert(double (&bd)[kMaxK], int (&bi)[kMaxK], int cap, double d, int id) {
    int pos = 0;
#pragma unroll
    for (int a = 0; a < kMaxK; ++a) pos += (a < cap && before(bd[a], bi[a], d, id)) ? 1 : 0;
    if (pos >= cap) return;
#pragma unroll
    for (int a = kMaxK - 1; a > 0; --a) {
        if (a < cap && a > pos) {
            bd[a] = bd[a - 1];
            bi[a] = bi[a - 1];
        }
    }
#pragma unroll
    for (int a = 0; a < kMaxK; ++a)
        if (a == pos) {
            bd[a] = d;
            bi[a] = id;
        }
}

// Per point (cell order): its k nearest nodes within R, weights of Eq. (3)
// normalized over them, the pair keys of its kept nodes (for the edges),
// and block partials of the capped count and the largest count.
template <typename TW>
__global__ void __launch_bounds__(kGT) k_g_influence(const double4* __restrict__ Ps, const int* __restrict__ us,
                                                     const int2* __restrict__ nb, const int* __restrict__ nid_s,
                                                     const int* __restrict__ cp, int64_t N, int64_t n_nodes,
                                                     double R2, int k, int* __restrict__ infl_idx,
                                                     TW* __restrict__ infl_w, uint64_t* __restrict__ pair_key,
                                                     int* __restrict__ stats) {
    __shared__ double sh[kGT];
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    double capped = 0, most = 0;
    if (s < N) {
        const double4 q = Ps[s];
        const int2* cells = nb + 27 * (size_t)us[s];
        double bd[kMaxK];
        int bi[kMaxK];
#pragma unroll
        for (int a = 0; a < kMaxK; ++a) {
            bd[a] = __builtin_inf();
            bi[a] = INT32_MAX;
        }
        int cnt = 0;
        for (int o = 0; o < 27; ++o) {
            const int2 r = cells[o];
            for (int t = r.x; t < r.y; ++t) {
                const int id = nid_s[t];
                if (id < 0) continue;
                const double d = gd2(Ps[t], q);
                if (!(d < R2)) continue;
                ++cnt;
                topk_insert(bd, bi, k, d, id);
            }
        }
        capped = cnt > k ? 1.0 : 0.0;
        most = (double)cnt;
        const int kept = cnt < k ? cnt : k;
        double w[kMaxK];
        double sw = 0;
#pragma unroll
        for (int a = 0; a < kMaxK; ++a) {
            double x;
            {
#pragma clang fp contract(off)
                x = 1.0 - bd[a] / R2;
                x = x * x * x;
            }
            w[a] = a < kept ? x : 0.0;
            sw += w[a];
        }
        const int i = cp[s];
        for (int a = 0; a < k; ++a) {
            double wa = 0;
            int ia = -1;
#pragma unroll
            for (int b = 0; b < kMaxK; ++b)
                if (b == a) {
                    wa = w[b];
                    ia = b < kept ? bi[b] : -1;
                }
            infl_idx[(size_t)i * k + a] = ia;
            infl_w[(size_t)i * k + a] = (TW)(ia >= 0 ? wa / sw : 0.0);
        }
        // node pairs through kept slots: key = lo * n_nodes + hi
        const int npair = k * (k - 1) / 2;
        int t = 0;
#pragma unroll
        for (int a = 0; a < kMaxK; ++a)
#pragma unroll
            for (int b = a + 1; b < kMaxK; ++b) {
                if (b < k) {
                    uint64_t key = kNoKey;
                    if (b < kept) {
                        const int lo = bi[a] < bi[b] ? bi[a] : bi[b];
                        const int hi = bi[a] < bi[b] ? bi[b] : bi[a];
                        key = (uint64_t)lo * (uint64_t)n_nodes + (uint64_t)hi;
                    }
                    pair_key[(size_t)i * npair + t] = key;
                    ++t;
                }
            }
    }
    const double c = bsum<kGT>(capped, sh);
    const double m = bext<kGT, true>(most, sh);
    if (threadIdx.x == 0) {
        atomicAdd(&stats[0], (int)c);
        atomicMax(&stats[1], (int)m);
    }
}

// Unique sorted keys -> (lo, hi) edges.
__global__ void __launch_bounds__(kGT) k_g_headflag(const uint64_t* __restrict__ key, int64_t M,
                                                    int* __restrict__ flag) {
    const int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (e >= M) return;
    const uint64_t v = key[e];
    flag[e] = (v != kNoKey && (e == 0 || v != key[e - 1])) ? 1 : 0;
}

__global__ void __launch_bounds__(kGT) k_g_edges(const uint64_t* __restrict__ key, const int* __restrict__ flag,
                                                 const int* __restrict__ incl, int64_t M, int64_t n_nodes,
                                                 int* __restrict__ edges) {
    const int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (e >= M || !flag[e]) return;
    const int o = incl[e] - 1;
    edges[2 * (size_t)o] = (int)(key[e] / (uint64_t)n_nodes);
    edges[2 * (size_t)o + 1] = (int)(key[e] % (uint64_t)n_nodes);
}

// ---------------------------------------------------------------- mean edge length

// kKnn nearest other points (ties to the lower source index) by growing
// shells of cells: after the shell at Chebyshev distance r every point
// within r*h of the query has been seen, so the search stops once the
// kKnn-th distance is below (r*h)^2 or every cell is covered.
__global__ void __launch_bounds__(kGT) k_g_knn(const double4* __restrict__ Ps, const int* __restrict__ cp,
                                               const uint64_t* __restrict__ ukey, const int* __restrict__ ustart,
                                               int nu, int64_t N, GridDims g, uint64_t* __restrict__ pair_key) {
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (s >= N) return;
    const double4 q = Ps[s];
    const int self = cp[s];
    const int64_t cx = cell_coord(q.x, g.x0, g.h, g.nx), cy = cell_coord(q.y, g.y0, g.h, g.ny),
                  cz = cell_coord(q.z, g.z0, g.h, g.nz);
    double bd[kMaxK];
    int bi[kMaxK];
#pragma unroll
    for (int a = 0; a < kMaxK; ++a) {
        bd[a] = __builtin_inf();
        bi[a] = INT32_MAX;
    }
    const int want = N - 1 < kKnn ? (int)(N - 1) : kKnn;
    int cnt = 0;
    const int64_t rmax = g.nx > g.ny ? (g.nx > g.nz ? g.nx : g.nz) : (g.ny > g.nz ? g.ny : g.nz);
    for (int64_t r = 0; r <= rmax; ++r) {
        for (int64_t dz = -r; dz <= r; ++dz)
            for (int64_t dy = -r; dy <= r; ++dy)
                for (int64_t dx = -r; dx <= r; ++dx) {
                    const int64_t ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy, az = dz < 0 ? -dz : dz;
                    const int64_t ring = ax > ay ? (ax > az ? ax : az) : (ay > az ? ay : az);
                    if (ring != r) continue;
                    const int64_t x = cx + dx, y = cy + dy, z = cz + dz;
                    if (x < 0 || x >= g.nx || y < 0 || y >= g.ny || z < 0 || z >= g.nz) continue;
                    const int c = find_cell(ukey, nu, (uint64_t)((z * g.ny + y) * g.nx + x));
                    if (c < 0) continue;
                    const int e = c + 1 < nu ? ustart[c + 1] : (int)N;
                    for (int t = ustart[c]; t < e; ++t) {
                        const int j = cp[t];
                        if (j == self) continue;
                        ++cnt;
                        topk_insert(bd, bi, kKnn, gd2(Ps[t], q), j);
                    }
                }
        const double reach = (double)r * g.h;
        if (cnt >= want && (want == 0 || bd[want - 1] < reach * reach)) break;
    }
#pragma unroll
    for (int a = 0; a < kKnn; ++a) {
        uint64_t key = kNoKey;
        if (a < want) {
            const int lo = self < bi[a] ? self : bi[a];
            const int hi = self < bi[a] ? bi[a] : self;
            key = (uint64_t)lo * (uint64_t)N + (uint64_t)hi;
        }
        pair_key[(size_t)self * kKnn + a] = key;
    }
}

// Per block: sum of the lengths of the unique edges it holds (sorted keys).
__global__ void __launch_bounds__(kGT) k_g_edge_len(const uint64_t* __restrict__ key, const int* __restrict__ flag,
                                                    int64_t M, int64_t N, const double4* __restrict__ P,
                                                    double* __restrict__ part) {
    __shared__ double sh[kGT];
    const int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x;
    double len = 0;
    if (e < M && flag[e]) {
        const int a = (int)(key[e] / (uint64_t)N), b = (int)(key[e] % (uint64_t)N);
        len = sqrt(gd2(P[a], P[b]));
    }
    const double t = bsum<kGT>(len, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kGT - 1) / kGT); }

// Eigenvector of the largest eigenvalue of a symmetric 3x3 matrix by cyclic
// Jacobi rotations.
void sym3_top_eigvec(const double C[3][3], double out[3]) {
    double A[3][3], V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) A[r][c] = C[r][c];
    for (int sweep = 0; sweep < 64; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-300 || off <= 1e-32 * dia) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    int best = 0;
    for (int c = 1; c < 3; ++c)
        if (A[c][c] > A[best][best]) best = c;
    double n = 0;
    for (int r = 0; r < 3; ++r) n += V[r][best] * V[r][best];
    n = std::sqrt(n);
    for (int r = 0; r < 3; ++r) out[r] = V[r][best] / n;
    int big = 0;
    for (int r = 1; r < 3; ++r)
        if (std::fabs(out[r]) > std::fabs(out[big])) big = r;
    if (out[big] < 0)
        for (int r = 0; r < 3; ++r) out[r] = -out[r];
}

// Device scratch owned by one build call (freed when it returns).
struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    hipError_t bytes(void*& out, size_t n) {
        void* p = nullptr;
        const hipError_t e = hipMalloc(&p, std::max<size_t>(n, 1));
        if (e != hipSuccess) return e;
        ptrs.push_back(p);
        out = p;
        return hipSuccess;
    }
    template <typename P>
    hipError_t get(P*& out, size_t count) {
        void* p = nullptr;
        const hipError_t e = bytes(p, count * sizeof(P));
        out = reinterpret_cast<P*>(p);
        return e;
    }
};

template <typename K, typename V>
hipError_t sort_pairs(Scratch& sc, const K* kin, K* kout, const V* vin, V* vout, int64_t n, hipStream_t st) {
    size_t bytes = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, kin, kout, vin, vout, (int)n, 0,
                                                      (int)(8 * sizeof(K)), st);
    if (e != hipSuccess) return e;
    void* tmp = nullptr;
    e = sc.bytes(tmp, bytes);
    if (e != hipSuccess) return e;
    return hipcub::DeviceRadixSort::SortPairs(tmp, bytes, kin, kout, vin, vout, (int)n, 0, (int)(8 * sizeof(K)), st);
}

hipError_t sort_keys(Scratch& sc, const uint64_t* kin, uint64_t* kout, int64_t n, hipStream_t st) {
    size_t bytes = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, kin, kout, (int)n, 0, 64, st);
    if (e != hipSuccess) return e;
    void* tmp = nullptr;
    e = sc.bytes(tmp, bytes);
    if (e != hipSuccess) return e;
    return hipcub::DeviceRadixSort::SortKeys(tmp, bytes, kin, kout, (int)n, 0, 64, st);
}

hipError_t incl_sum(Scratch& sc, const int* in, int* out, int64_t n, hipStream_t st) {
    size_t bytes = 0;
    hipError_t e = hipcub::DeviceScan::InclusiveSum(nullptr, bytes, in, out, (int)n, st);
    if (e != hipSuccess) return e;
    void* tmp = nullptr;
    e = sc.bytes(tmp, bytes);
    if (e != hipSuccess) return e;
    return hipcub::DeviceScan::InclusiveSum(tmp, bytes, in, out, (int)n, st);
}

GridDims grid_for(const double lo[3], const double hi[3], double h) {
    GridDims g;
    g.x0 = lo[0];
    g.y0 = lo[1];
    g.z0 = lo[2];
    g.h = h;
    g.nx = (int64_t)std::floor((hi[0] - lo[0]) / h) + 1;
    g.ny = (int64_t)std::floor((hi[1] - lo[1]) / h) + 1;
    g.nz = (int64_t)std::floor((hi[2] - lo[2]) / h) + 1;
    return g;
}

// Points sorted by grid cell: cell keys and source ids in cell order, the
// occupied cells' keys and first positions, each point's cell, positions
// (and axis ranks when given) in cell order.
struct CellGrid {
    uint64_t* ck = nullptr;
    int* cp = nullptr;
    double4* Ps = nullptr;
    int* rs = nullptr;
    int* us = nullptr;
    uint64_t* ukey = nullptr;
    int* ustart = nullptr;
    int nu = 0;
};

amm_status build_cells(Scratch& sc, const double4* P, const int* rank, int64_t N, const GridDims& g,
                       hipStream_t st, CellGrid& G, std::string& err) {
    uint64_t* key = nullptr;
    int* val = nullptr;
    int *head = nullptr, *incl = nullptr;
    GCHK(sc.get(key, N));
    GCHK(sc.get(val, N));
    GCHK(sc.get(G.ck, N));
    GCHK(sc.get(G.cp, N));
    GCHK(sc.get(G.Ps, N));
    if (rank) GCHK(sc.get(G.rs, N));
    GCHK(sc.get(G.us, N));
    GCHK(sc.get(head, N));
    GCHK(sc.get(incl, N));
    hipLaunchKernelGGL(k_g_cellkey, dim3(nblk(N)), dim3(kGT), 0, st, P, N, g, key, val);
    GCHK(sort_pairs(sc, key, G.ck, val, G.cp, N, st));
    hipLaunchKernelGGL(k_g_gather, dim3(nblk(N)), dim3(kGT), 0, st, G.ck, G.cp, P, rank, N, G.Ps, G.rs, head);
    GCHK(incl_sum(sc, head, incl, N, st));
    int nu = 0;
    GCHK(hipMemcpyAsync(&nu, incl + (N - 1), sizeof(int), hipMemcpyDeviceToHost, st));
    GCHK(hipStreamSynchronize(st));
    G.nu = nu;
    GCHK(sc.get(G.ukey, nu));
    GCHK(sc.get(G.ustart, nu));
    hipLaunchKernelGGL(k_g_cells, dim3(nblk(N)), dim3(kGT), 0, st, G.ck, head, incl, N, G.ukey, G.ustart, G.us);
    GCHK(hipGetLastError());
    return AMM_OK;
}

}  // namespace

struct GraphBuild {
    int64_t N = 0;
    int k = 0;
    amm_dtype dtype = AMM_F64;
    amm_graph_info info{};
    int* node_src = nullptr;
    int* infl_idx = nullptr;
    void* infl_w = nullptr;
    int* edges = nullptr;
    ~GraphBuild() {
        if (node_src) (void)hipFree(node_src);
        if (infl_idx) (void)hipFree(infl_idx);
        if (infl_w) (void)hipFree(infl_w);
        if (edges) (void)hipFree(edges);
    }
};

void graph_release(GraphBuild* g) { delete g; }

amm_status graph_build(void* stream, const amm_graph_in& in, amm_graph_info* info_out, GraphBuild** out,
                       std::string& err) {
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t N = in.n_src;
    const int k = in.k;
    if (!in.src_xyz || N < 2 || N > (int64_t)INT32_MAX / 32 || k < 1 || k > kMaxK ||
        (in.dtype != AMM_F32 && in.dtype != AMM_F64)) {
        err = "graph: bad source pointer, size, k or dtype";
        return AMM_ERR_INVALID_ARG;
    }
    Scratch sc;
    double4* P = nullptr;
    double* part = nullptr;
    const unsigned nb1 = nblk(N);
    GCHK(sc.get(P, N));
    GCHK(sc.get(part, 10 * (size_t)nb1));
    if (in.dtype == AMM_F64)
        hipLaunchKernelGGL(k_g_load<double>, dim3(nb1), dim3(kGT), 0, st, (const double*)in.src_xyz, P, N, part);
    else
        hipLaunchKernelGGL(k_g_load<float>, dim3(nb1), dim3(kGT), 0, st, (const float*)in.src_xyz, P, N, part);
    std::vector<double> hp(10 * (size_t)nb1);
    GCHK(hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st));
    GCHK(hipStreamSynchronize(st));
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, sum[3] = {0, 0, 0};
    double bad = 0;
    for (unsigned b = 0; b < nb1; ++b) {
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], hp[10 * b + c]);
            hi[c] = std::max(hi[c], hp[10 * b + 3 + c]);
            sum[c] += hp[10 * b + 6 + c];
        }
        bad += hp[10 * b + 9];
    }
    if (bad > 0) {
        err = "graph: non-finite source coordinate";
        return AMM_ERR_NONFINITE;
    }
    const double mean[3] = {sum[0] / (double)N, sum[1] / (double)N, sum[2] / (double)N};
    hipLaunchKernelGGL(k_g_cov, dim3(nb1), dim3(kGT), 0, st, P, N, mean[0], mean[1], mean[2], part);
    GCHK(hipMemcpyAsync(hp.data(), part, sizeof(double) * 6 * nb1, hipMemcpyDeviceToHost, st));
    GCHK(hipStreamSynchronize(st));
    double cs[6] = {0, 0, 0, 0, 0, 0};
    for (unsigned b = 0; b < nb1; ++b)
        for (int m = 0; m < 6; ++m) cs[m] += hp[6 * b + m];
    const double C[3][3] = {{cs[0] / N, cs[1] / N, cs[2] / N},
                            {cs[1] / N, cs[3] / N, cs[4] / N},
                            {cs[2] / N, cs[4] / N, cs[5] / N}};
    double ax[3];
    sym3_top_eigvec(C, ax);

    // order along the axis
    double *tk = nullptr, *tks = nullptr;
    int *tv = nullptr, *order = nullptr, *rank = nullptr;
    GCHK(sc.get(tk, N));
    GCHK(sc.get(tks, N));
    GCHK(sc.get(tv, N));
    GCHK(sc.get(order, N));
    GCHK(sc.get(rank, N));
    hipLaunchKernelGGL(k_g_project, dim3(nb1), dim3(kGT), 0, st, P, N, mean[0], mean[1], mean[2], ax[0], ax[1],
                       ax[2], tk, tv);
    GCHK(sort_pairs(sc, tk, tks, tv, order, N, st));
    hipLaunchKernelGGL(k_g_invert, dim3(nb1), dim3(kGT), 0, st, order, rank, N);

    const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]});
    const double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                  (hi[2] - lo[2]) * (hi[2] - lo[2]));
    if (!(ext > 0)) {
        err = "graph: all source points coincide";
        return AMM_ERR_INVALID_ARG;
    }

    // mean edge length of the 6-NN graph
    double lbar = 0;
    {
        const double h = diag / std::cbrt((double)N);
        const GridDims g = grid_for(lo, hi, h);
        CellGrid G;
        TRY_STATUS(build_cells(sc, P, nullptr, N, g, st, G, err));
        const int64_t M = N * kKnn;
        uint64_t *pk = nullptr, *pks = nullptr;
        int *flag = nullptr, *incl = nullptr;
        double* lp = nullptr;
        GCHK(sc.get(pk, M));
        GCHK(sc.get(pks, M));
        GCHK(sc.get(flag, M));
        GCHK(sc.get(incl, M));
        GCHK(sc.get(lp, nblk(M)));
        hipLaunchKernelGGL(k_g_knn, dim3(nb1), dim3(kGT), 0, st, G.Ps, G.cp, G.ukey, G.ustart, G.nu, N, g, pk);
        GCHK(sort_keys(sc, pk, pks, M, st));
        hipLaunchKernelGGL(k_g_headflag, dim3(nblk(M)), dim3(kGT), 0, st, pks, M, flag);
        GCHK(incl_sum(sc, flag, incl, M, st));
        hipLaunchKernelGGL(k_g_edge_len, dim3(nblk(M)), dim3(kGT), 0, st, pks, flag, M, N, P, lp);
        int ne = 0;
        std::vector<double> hl(nblk(M));
        GCHK(hipMemcpyAsync(&ne, incl + (M - 1), sizeof(int), hipMemcpyDeviceToHost, st));
        GCHK(hipMemcpyAsync(hl.data(), lp, sizeof(double) * hl.size(), hipMemcpyDeviceToHost, st));
        GCHK(hipStreamSynchronize(st));
        double tot = 0;
        for (double v : hl) tot += v;
        lbar = ne > 0 ? tot / ne : 0.0;
    }
    const double R = in.radius > 0 ? in.radius : (in.radius_factor > 0 ? in.radius_factor : 5.0) * lbar;
    if (!(R > 0) || !std::isfinite(R)) {
        err = "graph: radius is not positive";
        return AMM_ERR_INVALID_ARG;
    }
    const double R2 = R * R;

    // grid of cell size R (slightly enlarged, so that rounding in the cell
    // index never hides a point within R from the 27 neighbour cells)
    const GridDims g = grid_for(lo, hi, R * (1.0 + 1e-9));
    CellGrid G;
    TRY_STATUS(build_cells(sc, P, rank, N, g, st, G, err));
    int2* nb = nullptr;
    GCHK(sc.get(nb, 27 * (size_t)G.nu));
    hipLaunchKernelGGL(k_g_nbr, dim3(nblk(G.nu)), dim3(kGT), 0, st, G.ukey, G.ustart, G.nu, N, g, nb);

    // node selection in rounds
    int *state = nullptr, *remaining = nullptr;
    GCHK(sc.get(state, N));
    GCHK(sc.get(remaining, 1));
    GCHK(hipMemsetAsync(state, 0, sizeof(int) * N, st));
    int rounds = 0;
    for (;;) {
        int left = 0;
        // a few rounds per read-back; extra rounds after the last decision do nothing
        for (int r = 0; r < 4; ++r) {
            GCHK(hipMemsetAsync(remaining, 0, sizeof(int), st));
            hipLaunchKernelGGL(k_g_round, dim3(nb1), dim3(kGT), 0, st, G.Ps, G.rs, G.us, nb, state, N, R2,
                               remaining);
            ++rounds;
        }
        GCHK(hipMemcpyAsync(&left, remaining, sizeof(int), hipMemcpyDeviceToHost, st));
        GCHK(hipStreamSynchronize(st));
        if (left == 0) break;
        if (rounds > N + 8) {
            err = "graph: node selection did not finish";
            return AMM_ERR_HIP;
        }
    }

    // node ids in axis order
    int *flag_r = nullptr, *pos_r = nullptr, *nid_r = nullptr, *nid_s = nullptr;
    GCHK(sc.get(flag_r, N));
    GCHK(sc.get(pos_r, N));
    GCHK(sc.get(nid_r, N));
    GCHK(sc.get(nid_s, N));
    hipLaunchKernelGGL(k_g_nodeflag, dim3(nb1), dim3(kGT), 0, st, G.rs, state, N, flag_r, pos_r);
    GCHK(incl_sum(sc, flag_r, nid_r, N, st));
    int n_nodes = 0;
    GCHK(hipMemcpyAsync(&n_nodes, nid_r + (N - 1), sizeof(int), hipMemcpyDeviceToHost, st));
    GCHK(hipStreamSynchronize(st));
    // inclusive sums -> ids: a node's id is the count before it
    auto res = new GraphBuild();
    std::unique_ptr<GraphBuild> keep(res);
    res->N = N;
    res->k = k;
    res->dtype = in.dtype;
    GCHK(hipMalloc((void**)&res->node_src, sizeof(int) * std::max(n_nodes, 1)));
    GCHK(hipMalloc((void**)&res->infl_idx, sizeof(int) * (size_t)N * k));
    GCHK(hipMalloc(&res->infl_w, (in.dtype == AMM_F64 ? 8 : 4) * (size_t)N * k));
    {
        int* nid_excl = nullptr;
        GCHK(sc.get(nid_excl, N));
        hipLaunchKernelGGL(k_g_excl_from_incl, dim3(nb1), dim3(kGT), 0, st, nid_r, flag_r, N, nid_excl);
        hipLaunchKernelGGL(k_g_nodeid, dim3(nb1), dim3(kGT), 0, st, flag_r, nid_excl, pos_r, G.cp, N, nid_s,
                           res->node_src);
    }

    // influence sets, weights, node pairs
    const int npair = k * (k - 1) / 2;
    const int64_t M = N * npair;
    uint64_t *pk = nullptr, *pks = nullptr;
    int* stats = nullptr;
    GCHK(sc.get(stats, 2));
    GCHK(hipMemsetAsync(stats, 0, 2 * sizeof(int), st));
    GCHK(sc.get(pk, std::max<int64_t>(M, 1)));
    GCHK(sc.get(pks, std::max<int64_t>(M, 1)));
    if (in.dtype == AMM_F64)
        hipLaunchKernelGGL(k_g_influence<double>, dim3(nb1), dim3(kGT), 0, st, G.Ps, G.us, nb, nid_s, G.cp, N,
                           (int64_t)n_nodes, R2, k, res->infl_idx, (double*)res->infl_w, pk, stats);
    else
        hipLaunchKernelGGL(k_g_influence<float>, dim3(nb1), dim3(kGT), 0, st, G.Ps, G.us, nb, nid_s, G.cp, N,
                           (int64_t)n_nodes, R2, k, res->infl_idx, (float*)res->infl_w, pk, stats);
    int n_edges = 0;
    if (M > 0) {
        int *flag = nullptr, *incl = nullptr;
        GCHK(sc.get(flag, M));
        GCHK(sc.get(incl, M));
        GCHK(sort_keys(sc, pk, pks, M, st));
        hipLaunchKernelGGL(k_g_headflag, dim3(nblk(M)), dim3(kGT), 0, st, pks, M, flag);
        GCHK(incl_sum(sc, flag, incl, M, st));
        GCHK(hipMemcpyAsync(&n_edges, incl + (M - 1), sizeof(int), hipMemcpyDeviceToHost, st));
        GCHK(hipStreamSynchronize(st));
        GCHK(hipMalloc((void**)&res->edges, sizeof(int) * 2 * std::max(n_edges, 1)));
        hipLaunchKernelGGL(k_g_edges, dim3(nblk(M)), dim3(kGT), 0, st, pks, flag, incl, M, (int64_t)n_nodes,
                           res->edges);
    } else {
        GCHK(hipMalloc((void**)&res->edges, sizeof(int) * 2));
    }
    int hs[2] = {0, 0};
    GCHK(hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, st));
    GCHK(hipStreamSynchronize(st));
    GCHK(hipGetLastError());
    amm_graph_info& info = res->info;
    info.n_nodes = n_nodes;
    info.n_edges = n_edges;
    info.radius = R;
    info.mean_edge_len = lbar;
    info.n_capped = hs[0];
    info.max_influences = hs[1];
    info.rounds = rounds;
    if (info_out) *info_out = info;
    *out = keep.release();
    return AMM_OK;
}

amm_status graph_copy(const GraphBuild* g, void* stream, int32_t* node_src_idx, int32_t* infl_idx, void* infl_w,
                      int32_t* edges, std::string& err) {
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t ws = g->dtype == AMM_F64 ? 8 : 4;
    if (node_src_idx)
        GCHK(hipMemcpyAsync(node_src_idx, g->node_src, sizeof(int) * g->info.n_nodes, hipMemcpyDeviceToDevice, st));
    if (infl_idx)
        GCHK(hipMemcpyAsync(infl_idx, g->infl_idx, sizeof(int) * (size_t)g->N * g->k, hipMemcpyDeviceToDevice, st));
    if (infl_w) GCHK(hipMemcpyAsync(infl_w, g->infl_w, ws * (size_t)g->N * g->k, hipMemcpyDeviceToDevice, st));
    if (edges && g->info.n_edges)
        GCHK(hipMemcpyAsync(edges, g->edges, sizeof(int) * 2 * g->info.n_edges, hipMemcpyDeviceToDevice, st));
    return AMM_OK;
}

}  // namespace amm
