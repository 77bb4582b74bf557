// Deformation-graph construction of Sec. 3.1 (Alg. 1) on the device, with
// Euclidean distance or the geodesic distance of Eq. (1) over the point
// cloud's nearest-neighbour edges, for one or many point sets (independent
// registration pairs) at once.
//
// Alg. 1 walks a set's source points in the order of their projection onto
// the principal axis and makes a point a node when no earlier node lies
// within R of it.  That is the lexicographically first maximal independent
// set of the graph "distance < R" under this order, which is unique: a
// point's decision depends only on the decisions of the earlier points
// within R.  It is computed here in rounds over all points of all sets: a
// point becomes covered as soon as an earlier neighbour is a node (the new
// node marks its later neighbours), and a node as soon as all its earlier
// neighbours are covered.  Each round decides at least the earliest
// undecided point of every set, and the result equals the sequential pass
// exactly.
//
// Neighbour queries use a uniform grid per set, stored as points sorted by
// (set, cell) keys (a stable radix sort), with each occupied cell's 27
// neighbour ranges precomputed.  "Within R" is ((dx*dx + dy*dy) + dz*dz) <
// R*R in float64 with every operation rounded on its own (no contraction),
// so that the integer decisions of the graph match a plain float64
// evaluation.  Sets are concatenated; every key carries the set in its high
// bits, so no query crosses sets.
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
constexpr int kSetShift = 44;                 // cell keys: set << 44 | cell
constexpr uint64_t kCellMask = (uint64_t(1) << kSetShift) - 1;
constexpr int kMaxSets = 1 << (64 - kSetShift - 1);

#define TRY_STATUS(x)                   \
    do {                                \
        const amm_status s_ = (x);      \
        if (s_ != AMM_OK) return s_;    \
    } while (0)

#define GCHK(x)                                                          \
    do {                                                                 \
        hipError_t e_ = (x);                                             \
        if (e_ != hipSuccess) {                                          \
            err = std::string(#x) + ": " + hipGetErrorString(e_);        \
            return e_ == hipErrorOutOfMemory ? AMM_ERR_OOM : AMM_ERR_HIP; \
        }                                                                \
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

struct GridDims {
    double x0, y0, z0, h;
    int64_t nx, ny, nz;
};

// Block b of G -> a block index such that each of the 8 XCDs (blocks are
// dealt round-robin over them) covers one contiguous range.
__device__ __forceinline__ int xcd_block(int b, int G) {
    const int per = G >> 3, rem = G & 7;
    const int x = b & 7, q = b >> 3;
    return x * per + min(x, rem) + q;
}

// ---------------------------------------------------------------- per-set statistics

template <typename T>
__global__ void __launch_bounds__(kGT) k_g_load(const T* __restrict__ v, double4* __restrict__ P, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (i < n) P[i] = make_double4((double)v[3 * i], (double)v[3 * i + 1], (double)v[3 * i + 2], 0.0);
}

// Set of every concatenated point.
__global__ void __launch_bounds__(kGT) k_g_setid(const int64_t* __restrict__ off, int n_sets, int64_t N,
                                                 int* __restrict__ sid) {
    const int64_t i = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (i >= N) return;
    int lo = 0, hi = n_sets - 1;
    while (lo < hi) {   // last set whose offset is <= i
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    sid[i] = lo;
}

// One block per set: bounding box, sum, and sum of (v - mean)(v - mean)^T
// (xx, xy, xz, yy, yz, zz), in a fixed order.  A non-finite coordinate
// makes the sums non-finite.
__global__ void __launch_bounds__(kGT) k_g_setstats(const double4* __restrict__ P, const int64_t* __restrict__ off,
                                                    double* __restrict__ stats) {
    __shared__ double sh[kGT];
    const int s = blockIdx.x;
    const int64_t a = off[s], b = off[s + 1];
    const double inf = __builtin_inf();
    double lo[3] = {inf, inf, inf}, hi[3] = {-inf, -inf, -inf}, sm[3] = {0, 0, 0};
    for (int64_t i = a + threadIdx.x; i < b; i += kGT) {
        const double4 p = P[i];
        const double c[3] = {p.x, p.y, p.z};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            lo[q] = fmin(lo[q], c[q]);
            hi[q] = fmax(hi[q], c[q]);
            sm[q] += c[q];
        }
    }
    double r[9];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        r[q] = bext<kGT, false>(lo[q], sh);
        r[3 + q] = bext<kGT, true>(hi[q], sh);
        r[6 + q] = bsum<kGT>(sm[q], sh);
    }
    const double n = (double)(b - a);
    const double m[3] = {r[6] / n, r[7] / n, r[8] / n};
    double cv[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = a + threadIdx.x; i < b; i += kGT) {
        const double4 p = P[i];
        const double dx = p.x - m[0], dy = p.y - m[1], dz = p.z - m[2];
        cv[0] += dx * dx;
        cv[1] += dx * dy;
        cv[2] += dx * dz;
        cv[3] += dy * dy;
        cv[4] += dy * dz;
        cv[5] += dz * dz;
    }
    double c6[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) c6[q] = bsum<kGT>(cv[q], sh);
    if (threadIdx.x == 0) {
        double* o = stats + 15 * (size_t)s;
#pragma unroll
        for (int q = 0; q < 9; ++q) o[q] = r[q];
#pragma unroll
        for (int q = 0; q < 6; ++q) o[9 + q] = c6[q];
    }
}

// Projection onto the set's principal axis (+0.0 folds -0.0 into +0.0, so
// that equal projections sort by index).  ax[s] = (mean, axis).
__global__ void __launch_bounds__(kGT) k_g_project(const double4* __restrict__ P, const int* __restrict__ sid,
                                                   const double* __restrict__ ax, int64_t N,
                                                   double* __restrict__ key, int* __restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (i >= N) return;
    const double4 p = P[i];
    const double* a = ax + 6 * (size_t)sid[i];
    key[i] = ((p.x - a[0]) * a[3] + (p.y - a[1]) * a[4] + (p.z - a[2]) * a[5]) + 0.0;
    val[i] = (int)i;
}

__global__ void __launch_bounds__(kGT) k_g_take(const int* __restrict__ idx, const int* __restrict__ src, int64_t N,
                                                int* __restrict__ dst) {
    const int64_t p = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (p < N) dst[p] = src[idx[p]];
}

__global__ void __launch_bounds__(kGT) k_g_invert(const int* __restrict__ order, int* __restrict__ rank, int64_t N) {
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (s < N) rank[order[s]] = (int)s;
}

// ---------------------------------------------------------------- sorted-cell grids

__device__ __forceinline__ int64_t cell_coord(double v, double v0, double h, int64_t n) {
    int64_t c = (int64_t)floor((v - v0) / h);
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

__device__ __forceinline__ uint64_t cell_key(int set, const GridDims& g, int64_t x, int64_t y, int64_t z) {
    return ((uint64_t)set << kSetShift) | (uint64_t)((z * g.ny + y) * g.nx + x);
}

__global__ void __launch_bounds__(kGT) k_g_cellkey(const double4* __restrict__ P, const int* __restrict__ sid,
                                                   const GridDims* __restrict__ gd, int64_t N,
                                                   uint64_t* __restrict__ key, int* __restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (i >= N) return;
    const double4 p = P[i];
    const int s = sid[i];
    const GridDims g = gd[s];
    key[i] = cell_key(s, g, cell_coord(p.x, g.x0, g.h, g.nx), cell_coord(p.y, g.y0, g.h, g.ny),
                      cell_coord(p.z, g.z0, g.h, g.nz));
    val[i] = (int)i;
}

// Points in cell order: position, set, rank along the axis (when given),
// and 1 at the first point of every occupied cell.
__global__ void __launch_bounds__(kGT) k_g_gather(const uint64_t* __restrict__ ck, const int* __restrict__ cp,
                                                  const double4* __restrict__ P, const int* __restrict__ sid,
                                                  const int* __restrict__ rank, int64_t N, double4* __restrict__ Ps,
                                                  int* __restrict__ ss, int* __restrict__ rs, int* __restrict__ head) {
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (s >= N) return;
    const int i = cp[s];
    Ps[s] = P[i];
    ss[s] = sid[i];
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
// cells of the same set (itself included), empty ones as (0, 0).
__global__ void __launch_bounds__(kGT) k_g_nbr(const uint64_t* __restrict__ ukey, const int* __restrict__ ustart,
                                               int nu, int64_t N, const GridDims* __restrict__ gd,
                                               int2* __restrict__ nb) {
    const int u = blockIdx.x * kGT + threadIdx.x;
    if (u >= nu) return;
    const uint64_t key = ukey[u];
    const int set = (int)(key >> kSetShift);
    const GridDims g = gd[set];
    const uint64_t lin = key & kCellMask;
    const int64_t cx = (int64_t)(lin % (uint64_t)g.nx);
    const int64_t cy = (int64_t)((lin / (uint64_t)g.nx) % (uint64_t)g.ny);
    const int64_t cz = (int64_t)(lin / ((uint64_t)g.nx * (uint64_t)g.ny));
    int o = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx, ++o) {
                const int64_t x = cx + dx, y = cy + dy, z = cz + dz;
                int2 r = make_int2(0, 0);
                if (x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz) {
                    const int c = find_cell(ukey, nu, cell_key(set, g, x, y, z));
                    if (c >= 0) r = make_int2(ustart[c], c + 1 < nu ? ustart[c + 1] : (int)N);
                }
                nb[27 * (size_t)u + o] = r;
            }
}

// ---------------------------------------------------------------- mean edge length

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

// kKnn nearest other points of the same set (ties to the lower index) by
// growing shells of cells: after the shell at Chebyshev distance r every
// point within r*h of the query has been seen, so the search stops once the
// kKnn-th distance is below (r*h)^2 or every cell is covered.  Writes the
// undirected pair keys lo * N + hi (global indices).
__global__ void __launch_bounds__(kGT) k_g_knn(const double4* __restrict__ Ps, const int* __restrict__ cp,
                                               const int* __restrict__ ss, const uint64_t* __restrict__ ukey,
                                               const int* __restrict__ ustart, int nu, int64_t N,
                                               const GridDims* __restrict__ gd, const int64_t* __restrict__ off,
                                               uint64_t* __restrict__ pair_key) {
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (s >= N) return;
    const double4 q = Ps[s];
    const int self = cp[s];
    const int set = ss[s];
    const GridDims g = gd[set];
    const int64_t n_set = off[set + 1] - off[set];
    const int64_t cx = cell_coord(q.x, g.x0, g.h, g.nx), cy = cell_coord(q.y, g.y0, g.h, g.ny),
                  cz = cell_coord(q.z, g.z0, g.h, g.nz);
    double bd[kMaxK];
    int bi[kMaxK];
#pragma unroll
    for (int a = 0; a < kMaxK; ++a) {
        bd[a] = __builtin_inf();
        bi[a] = INT32_MAX;
    }
    const int want = n_set - 1 < kKnn ? (int)(n_set - 1) : kKnn;
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
                    const int c = find_cell(ukey, nu, cell_key(set, g, x, y, z));
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

__global__ void __launch_bounds__(kGT) k_g_headflag(const uint64_t* __restrict__ key, int64_t M,
                                                    int* __restrict__ flag) {
    const int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (e >= M) return;
    const uint64_t v = key[e];
    flag[e] = (v != kNoKey && (e == 0 || v != key[e - 1])) ? 1 : 0;
}

// Per set, the first sorted position whose key is >= bound[s] (the key
// ranges of the sets are contiguous and ordered).
__global__ void __launch_bounds__(kGT) k_g_bounds(const uint64_t* __restrict__ key, int64_t M,
                                                  const uint64_t* __restrict__ bound, int nb,
                                                  int64_t* __restrict__ at) {
    const int s = blockIdx.x * kGT + threadIdx.x;
    if (s >= nb) return;
    const uint64_t b = bound[s];
    int64_t lo = 0, hi = M;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (key[mid] < b)
            lo = mid + 1;
        else
            hi = mid;
    }
    at[s] = lo;
}

// One block per set: sum of the lengths of its unique edges and their count,
// over its range of the sorted keys, in a fixed order.
__global__ void __launch_bounds__(kGT) k_g_edge_len(const uint64_t* __restrict__ key, const int* __restrict__ flag,
                                                    const int64_t* __restrict__ at, int64_t N,
                                                    const double4* __restrict__ P, double* __restrict__ out) {
    __shared__ double sh[kGT];
    const int s = blockIdx.x;
    double len = 0, cnt = 0;
    for (int64_t e = at[s] + threadIdx.x; e < at[s + 1]; e += kGT) {
        if (!flag[e]) continue;
        const int a = (int)(key[e] / (uint64_t)N), b = (int)(key[e] % (uint64_t)N);
        len += sqrt(gd2(P[a], P[b]));
        cnt += 1;
    }
    const double tl = bsum<kGT>(len, sh);
    const double tc = bsum<kGT>(cnt, sh);
    if (threadIdx.x == 0) {
        out[2 * s] = tl;
        out[2 * s + 1] = tc;
    }
}

// ---------------------------------------------------------------- node selection

// One round over the undecided points (cell order).  state: 0 undecided,
// 1 node, 2 covered.  Reads of other points' states may see the value of
// the previous round or of this one; both are final or undecided, so a
// decision taken is always the sequential pass's.  A new node marks the
// later points within R of it covered (`cov`) at once, so coverage needs
// no scan; and a point remembers the earlier neighbour that kept it
// undecided (`wait`) and skips its scan while that one is undecided (it
// cannot become a node before).  No ordering across XCDs is needed inside
// a round (every state seen is either final or undecided), so the state
// accesses are workgroup-scope atomics that stay in the caches; with blocks
// on contiguous ranges per XCD most neighbours' updates still show within
// the round, and a launch boundary shows all of them to the next.
__global__ void __launch_bounds__(kGT) k_g_round(const double4* __restrict__ Ps, const int* __restrict__ rs,
                                                 const int* __restrict__ ss, const int* __restrict__ us,
                                                 const int2* __restrict__ nb, int* state, int* cov,
                                                 int* __restrict__ wait, int64_t N, const double* __restrict__ R2s,
                                                 int* __restrict__ remaining) {
    // blocks take contiguous ranges of the cell order per XCD, so that most
    // neighbours' states sit in the same L2
    const int64_t s = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kGT + threadIdx.x;
    bool undecided = false;
    bool open = s < N && __hip_atomic_load(&state[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0;
    if (open && __hip_atomic_load(&cov[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
        __hip_atomic_store(&state[s], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        open = false;
    }
    if (open) {
        const int wt = wait[s];
        if (wt >= 0 && __hip_atomic_load(&state[wt], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) {
            undecided = true;
            open = false;
        }
    }
    if (open) {
        const double4 q = Ps[s];
        const int rq = rs[s];
        const double R2 = R2s[ss[s]];
        const int2* cells = nb + 27 * (size_t)us[s];
        // every candidate's rank, position and state are loaded up front (no
        // load waits on an earlier test), so the loads of consecutive
        // candidates are in flight together
        bool covered = false;
        int pending = -1;
        for (int o = 0; o < 27 && !covered; ++o) {
            const int2 r = cells[o];
#pragma unroll 8
            for (int t = r.x; t < r.y; ++t) {
                const int rt = rs[t];
                const double4 pt = Ps[t];
                const int st = __hip_atomic_load(&state[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (rt < rq && gd2(pt, q) < R2) {
                    covered = covered || st == 1;
                    if (st == 0 && pending < 0) pending = t;
                }
            }
        }
        if (covered) {
            __hip_atomic_store(&state[s], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else if (pending < 0) {
            __hip_atomic_store(&state[s], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            for (int o = 0; o < 27; ++o) {
                const int2 r = cells[o];
                for (int t = r.x; t < r.y; ++t)
                    if (rs[t] > rq && gd2(Ps[t], q) < R2)
                        __hip_atomic_store(&cov[t], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        } else {
            wait[s] = pending;
            undecided = true;
        }
    }
    const int cnt = __syncthreads_count(undecided);
    if (threadIdx.x == 0 && cnt) atomicAdd(remaining, cnt);
}

// Axis order -> node flag and cell-order position.
__global__ void __launch_bounds__(kGT) k_g_nodeflag(const int* __restrict__ rs, const int* __restrict__ state,
                                                    int64_t N, int* __restrict__ flag_by_rank,
                                                    int* __restrict__ pos_by_rank) {
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (s >= N) return;
    flag_by_rank[rs[s]] = state[s] == 1 ? 1 : 0;
    pos_by_rank[rs[s]] = (int)s;
}

// Per set: global id of its first node (the nodes before it), and the
// total at the end.  Ranks of set s are off[s] .. off[s+1]-1.
__global__ void __launch_bounds__(kGT) k_g_setnodes(const int* __restrict__ incl, const int* __restrict__ flag,
                                                    const int64_t* __restrict__ off, int n_sets,
                                                    int64_t* __restrict__ node_off) {
    const int s = blockIdx.x * kGT + threadIdx.x;
    if (s > n_sets) return;
    const int64_t r = off[s];
    node_off[s] = s < n_sets ? (int64_t)(incl[r] - flag[r]) : (int64_t)incl[r - 1];
}

// Node ids: global in cell order (-1 for non-nodes), the node's source
// point as an index within its set, and the node's set.
__global__ void __launch_bounds__(kGT) k_g_nodeid(const int* __restrict__ flag_by_rank, const int* __restrict__ incl,
                                                  const int* __restrict__ pos_by_rank, const int* __restrict__ cp,
                                                  const int* __restrict__ ss, const int64_t* __restrict__ off,
                                                  int64_t N, int* __restrict__ nid_s, int* __restrict__ node_src,
                                                  int* __restrict__ nset) {
    const int64_t r = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (r >= N) return;
    const int s = pos_by_rank[r];
    if (flag_by_rank[r]) {
        const int g = incl[r] - 1;
        const int set = ss[s];
        nid_s[s] = g;
        node_src[g] = (int)(cp[s] - off[set]);
        nset[g] = set;
    } else {
        nid_s[s] = -1;
    }
}

// ---------------------------------------------------------------- influence sets

// Per point (cell order): its k nearest nodes within R, weights of Eq. (3)
// normalized over them, the pair keys lo * n_nodes + hi (global node ids)
// of its kept nodes, and per set the number of points with more than k
// nodes within R and the largest such number.  Node ids written are
// local to the set.
template <typename TW>
__global__ void __launch_bounds__(kGT) k_g_influence(const double4* __restrict__ Ps, const int* __restrict__ ss,
                                                     const int* __restrict__ us, const int2* __restrict__ nb,
                                                     const int* __restrict__ nid_s, const int* __restrict__ cp,
                                                     const int64_t* __restrict__ node_off,
                                                     const double* __restrict__ R2s, int64_t N, int64_t n_nodes,
                                                     int k, int* __restrict__ infl_idx, TW* __restrict__ infl_w,
                                                     uint64_t* __restrict__ pair_key, int* __restrict__ stats) {
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (s >= N) return;
    const double4 q = Ps[s];
    const int set = ss[s];
    const double R2 = R2s[set];
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
    if (cnt > k) atomicAdd(&stats[2 * set], 1);
    atomicMax(&stats[2 * set + 1], cnt);
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
    const int base = (int)node_off[set];
    for (int a = 0; a < k; ++a) {
        double wa = 0;
        int ia = -1;
#pragma unroll
        for (int b = 0; b < kMaxK; ++b)
            if (b == a) {
                wa = w[b];
                ia = b < kept ? bi[b] - base : -1;
            }
        infl_idx[(size_t)i * k + a] = ia;
        infl_w[(size_t)i * k + a] = (TW)(ia >= 0 ? wa / sw : 0.0);
    }
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

// Unique sorted keys -> edges with node ids local to their set.
__global__ void __launch_bounds__(kGT) k_g_edges(const uint64_t* __restrict__ key, const int* __restrict__ flag,
                                                 const int* __restrict__ incl, int64_t M, int64_t n_nodes,
                                                 const int* __restrict__ nset, const int64_t* __restrict__ node_off,
                                                 uint64_t* __restrict__ ukey, int* __restrict__ edges) {
    const int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (e >= M || !flag[e]) return;
    const int o = incl[e] - 1;
    const int lo = (int)(key[e] / (uint64_t)n_nodes), hi = (int)(key[e] % (uint64_t)n_nodes);
    const int base = (int)node_off[nset[lo]];
    ukey[o] = key[e];
    edges[2 * (size_t)o] = lo - base;
    edges[2 * (size_t)o + 1] = hi - base;
}

// ---------------------------------------------------------------- geodesic distance (Eq. 1)
//
// On a point cloud the edge set is the symmetrized k-NN graph (kKnn
// neighbours, ties to the lower index), an edge as long as its Euclidean
// length, and the geodesic distance is the shortest path over it.  A path
// shorter than R stays inside the Euclidean ball of radius R around its
// start, so each point's geodesic neighbourhood is found inside that ball:
// the ball's points go to LDS and the shortest paths from the point follow
// by relaxing every edge inside the ball until nothing changes (the fixed
// point d(v) = min over edges (u, v) of d(u) + |uv|, which is what a
// label-setting search computes: each value is the left-to-right sum along
// a shortest path, so both agree bitwise).

constexpr int kGeoThreads = 64;   // one wave per point
constexpr int kGeoCap = 1024;     // points of one Euclidean ball held in LDS
constexpr int kGeoHash = 2048;    // open-addressing slots, power of two

// Directed entries a -> b and b -> a (key a << 32 | b) of the unique
// undirected k-NN edges (sorted keys lo * N + hi with head flags).
__global__ void __launch_bounds__(kGT) k_g_directed(const uint64_t* __restrict__ key, const int* __restrict__ flag,
                                                    const int* __restrict__ incl, int64_t M, int64_t N,
                                                    uint64_t* __restrict__ dkey) {
    const int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (e >= M || !flag[e]) return;
    const int64_t o = incl[e] - 1;
    const uint64_t a = key[e] / (uint64_t)N, b = key[e] % (uint64_t)N;
    dkey[2 * o] = (a << 32) | b;
    dkey[2 * o + 1] = (b << 32) | a;
}

// Adjacency rows of the sorted directed entries: row[a] = the first entry
// whose source is >= a (a binary search, so a point without entries gets an
// empty row), for a = 0..N; col = the entries' targets.
__global__ void __launch_bounds__(kGT) k_g_rows(const uint64_t* __restrict__ dkey, int64_t E2, int64_t N,
                                                int* __restrict__ row, int* __restrict__ col) {
    const int64_t i = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (i < E2) col[i] = (int)(dkey[i] & 0xffffffffull);
    if (i > N) return;
    const uint64_t b = (uint64_t)i << 32;
    int64_t lo = 0, hi = E2;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (dkey[mid] < b)
            lo = mid + 1;
        else
            hi = mid;
    }
    row[i] = (int)lo;
}

__device__ __forceinline__ unsigned geo_hash(int g) { return ((unsigned)g * 2654435761u) & (kGeoHash - 1); }

// Geodesic neighbourhood of point s (cell order of the R grid): the points
// at geodesic distance < R (s itself included, at 0).  COUNT: their number
// into cnt[s]; else their cell positions and distances at off[s], in the
// order the ball was gathered (the 27 neighbour cells, then cell order).
template <bool COUNT>
__global__ void __launch_bounds__(kGeoThreads) k_g_geoball(
    const double4* __restrict__ Ps, const double4* __restrict__ P, const int* __restrict__ cp,
    const int* __restrict__ ss, const int* __restrict__ us, const int2* __restrict__ nb, const int* __restrict__ row,
    const int* __restrict__ col, const double* __restrict__ R2s, const double* __restrict__ Rs,
    int* __restrict__ cnt, const int* __restrict__ off, int* __restrict__ gpos, double* __restrict__ gdist,
    int* __restrict__ overflow) {
    __shared__ int lpos[kGeoCap], lgid[kGeoCap];
    __shared__ unsigned long long ldist[kGeoCap];
    __shared__ int hkey[kGeoHash], hval[kGeoHash];
    __shared__ int s_n;
    const int64_t s = blockIdx.x;
    const int lane = threadIdx.x;
    const double4 q = Ps[s];
    const int set = ss[s];
    const double R2 = R2s[set], R = Rs[set];
    constexpr unsigned long long kInf = 0x7ff0000000000000ull;   // +inf
    for (int i = lane; i < kGeoHash; i += kGeoThreads) hkey[i] = -1;
    if (lane == 0) s_n = 0;
    __syncthreads();
    // the Euclidean ball, compacted in gathering order
    const int2* cells = nb + 27 * (size_t)us[s];
    for (int o = 0; o < 27; ++o) {
        const int2 r = cells[o];
        for (int t0 = r.x; t0 < r.y; t0 += kGeoThreads) {
            const int t = t0 + lane;
            const bool in = t < r.y && gd2(Ps[t], q) < R2;
            const unsigned long long m = __ballot(in);
            const int base = s_n;
            if (in) {
                const int i = base + (int)__popcll(m & ((1ull << lane) - 1ull));
                if (i < kGeoCap) {
                    lpos[i] = t;
                    lgid[i] = cp[t];
                }
            }
            __syncthreads();
            if (lane == 0) s_n = base + (int)__popcll(m);
            __syncthreads();
        }
    }
    const int n = s_n;
    if (n > kGeoCap) {   // uniform over the block
        if (lane == 0) {
            atomicOr(overflow, 1);
            if (COUNT) cnt[s] = 0;
        }
        return;
    }
    for (int i = lane; i < n; i += kGeoThreads) {
        const int g = lgid[i];
        unsigned h = geo_hash(g);
        while (atomicCAS(&hkey[h], -1, g) != -1) h = (h + 1) & (kGeoHash - 1);
        hval[h] = i;
        ldist[i] = lpos[i] == (int)s ? 0ull : kInf;
    }
    __syncthreads();
    // relax every edge inside the ball until nothing changes
    while (true) {
        int changed = 0;
        for (int u = lane; u < n; u += kGeoThreads) {
            const unsigned long long bu = ldist[u];
            if (bu == kInf) continue;
            const double du = __longlong_as_double((long long)bu);
            const int g = lgid[u];
            const double4 pu = P[g];
            for (int e = row[g]; e < row[g + 1]; ++e) {
                const int v = col[e];
                unsigned h = geo_hash(v);
                int lv = -1;
                while (true) {
                    const int key = hkey[h];
                    if (key == v) {
                        lv = hval[h];
                        break;
                    }
                    if (key == -1) break;
                    h = (h + 1) & (kGeoHash - 1);
                }
                if (lv < 0) continue;   // outside the ball: no path shorter than R passes there
                const double nd = du + sqrt(gd2(pu, P[v]));
                if (nd < R) {
                    const unsigned long long nbits = (unsigned long long)__double_as_longlong(nd);
                    if (nbits < ldist[lv]) {
                        atomicMin(&ldist[lv], nbits);
                        changed = 1;
                    }
                }
            }
        }
        if (!__syncthreads_or(changed)) break;
    }
    if (COUNT) {
        int c = 0;
        for (int i = lane; i < n; i += kGeoThreads) c += ldist[i] != kInf ? 1 : 0;
        for (int w = 32; w > 0; w >>= 1) c += __shfl_xor(c, w);
        if (lane == 0) cnt[s] = c;
    } else {
        int o = off[s];
        for (int i0 = 0; i0 < n; i0 += kGeoThreads) {
            const int i = i0 + lane;
            const bool in = i < n && ldist[i] != kInf;
            const unsigned long long m = __ballot(in);
            if (in) {
                const int w = o + (int)__popcll(m & ((1ull << lane) - 1ull));
                gpos[w] = lpos[i];
                gdist[w] = __longlong_as_double((long long)ldist[i]);
            }
            o += (int)__popcll(m);
        }
    }
}

// One round of the node selection over the geodesic neighbourhoods (the
// same decisions as k_g_round, with "within R" read from the lists).
__global__ void __launch_bounds__(kGT) k_g_round_geo(const int* __restrict__ rs, const int* __restrict__ goff,
                                                     const int* __restrict__ gpos, int* state, int* cov,
                                                     int* __restrict__ wait, int64_t N, int* __restrict__ remaining) {
    const int64_t s = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kGT + threadIdx.x;
    bool undecided = false;
    bool open = s < N && __hip_atomic_load(&state[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0;
    if (open && __hip_atomic_load(&cov[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
        __hip_atomic_store(&state[s], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        open = false;
    }
    if (open) {
        const int wt = wait[s];
        if (wt >= 0 && __hip_atomic_load(&state[wt], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) {
            undecided = true;
            open = false;
        }
    }
    if (open) {
        const int rq = rs[s];
        const int e0 = goff[s], e1 = goff[s + 1];
        bool covered = false;
        int pending = -1;
        for (int e = e0; e < e1 && !covered; ++e) {
            const int t = gpos[e];
            const int st = __hip_atomic_load(&state[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (rs[t] < rq) {
                covered = covered || st == 1;
                if (st == 0 && pending < 0) pending = t;
            }
        }
        if (covered) {
            __hip_atomic_store(&state[s], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else if (pending < 0) {
            __hip_atomic_store(&state[s], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            for (int e = e0; e < e1; ++e) {
                const int t = gpos[e];
                if (rs[t] > rq) __hip_atomic_store(&cov[t], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        } else {
            wait[s] = pending;
            undecided = true;
        }
    }
    const int cnt = __syncthreads_count(undecided);
    if (threadIdx.x == 0 && cnt) atomicAdd(remaining, cnt);
}

// Influence sets from the geodesic neighbourhoods: as k_g_influence with
// the geodesic distance D (kept nodes the k nearest by D, ties to the lower
// node id; Eq. (3) with D^2 = D * D).
template <typename TW>
__global__ void __launch_bounds__(kGT) k_g_influence_geo(const int* __restrict__ ss, const int* __restrict__ goff,
                                                         const int* __restrict__ gpos,
                                                         const double* __restrict__ gdist,
                                                         const int* __restrict__ nid_s, const int* __restrict__ cp,
                                                         const int64_t* __restrict__ node_off,
                                                         const double* __restrict__ R2s, int64_t N, int64_t n_nodes,
                                                         int k, int* __restrict__ infl_idx, TW* __restrict__ infl_w,
                                                         uint64_t* __restrict__ pair_key, int* __restrict__ stats) {
    const int64_t s = (int64_t)blockIdx.x * kGT + threadIdx.x;
    if (s >= N) return;
    const int set = ss[s];
    const double R2 = R2s[set];
    double bd[kMaxK];
    int bi[kMaxK];
#pragma unroll
    for (int a = 0; a < kMaxK; ++a) {
        bd[a] = __builtin_inf();
        bi[a] = INT32_MAX;
    }
    int cnt = 0;
    for (int e = goff[s]; e < goff[s + 1]; ++e) {
        const int id = nid_s[gpos[e]];
        if (id < 0) continue;
        ++cnt;
        topk_insert(bd, bi, k, gdist[e], id);
    }
    if (cnt > k) atomicAdd(&stats[2 * set], 1);
    atomicMax(&stats[2 * set + 1], cnt);
    const int kept = cnt < k ? cnt : k;
    double w[kMaxK];
    double sw = 0;
#pragma unroll
    for (int a = 0; a < kMaxK; ++a) {
        double x;
        {
#pragma clang fp contract(off)
            x = 1.0 - (bd[a] * bd[a]) / R2;
            x = x * x * x;
        }
        w[a] = a < kept ? x : 0.0;
        sw += w[a];
    }
    const int i = cp[s];
    const int base = (int)node_off[set];
    for (int a = 0; a < k; ++a) {
        double wa = 0;
        int ia = -1;
#pragma unroll
        for (int b = 0; b < kMaxK; ++b)
            if (b == a) {
                wa = w[b];
                ia = b < kept ? bi[b] - base : -1;
            }
        infl_idx[(size_t)i * k + a] = ia;
        infl_w[(size_t)i * k + a] = (TW)(ia >= 0 ? wa / sw : 0.0);
    }
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
                pair_key[(size_t)i * (k * (k - 1) / 2) + t] = key;
                ++t;
            }
        }
}

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kGT - 1) / kGT); }

// Eigenvector of the largest eigenvalue of a symmetric 3x3 matrix by cyclic
// Jacobi rotations, its largest component made positive.
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
hipError_t sort_pairs(Scratch& sc, const K* kin, K* kout, const V* vin, V* vout, int64_t n, hipStream_t st,
                      int end_bit = 8 * sizeof(K)) {
    size_t bytes = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, kin, kout, vin, vout, (int)n, 0, end_bit, st);
    if (e != hipSuccess) return e;
    void* tmp = nullptr;
    e = sc.bytes(tmp, bytes);
    if (e != hipSuccess) return e;
    return hipcub::DeviceRadixSort::SortPairs(tmp, bytes, kin, kout, vin, vout, (int)n, 0, end_bit, st);
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

bool grid_for(const double lo[3], const double hi[3], double h, GridDims& g) {
    g.x0 = lo[0];
    g.y0 = lo[1];
    g.z0 = lo[2];
    g.h = h;
    g.nx = (int64_t)std::floor((hi[0] - lo[0]) / h) + 1;
    g.ny = (int64_t)std::floor((hi[1] - lo[1]) / h) + 1;
    g.nz = (int64_t)std::floor((hi[2] - lo[2]) / h) + 1;
    const double cells = (double)g.nx * (double)g.ny * (double)g.nz;
    return cells < (double)kCellMask;
}

// Points sorted by (set, grid cell): cell keys and source ids in cell
// order, the occupied cells' keys and first positions, each point's cell,
// set, position, and axis rank when given.
struct CellGrid {
    uint64_t* ck = nullptr;
    int* cp = nullptr;
    double4* Ps = nullptr;
    int* ss = nullptr;
    int* rs = nullptr;
    int* us = nullptr;
    uint64_t* ukey = nullptr;
    int* ustart = nullptr;
    int nu = 0;
};

amm_status build_cells(Scratch& sc, const double4* P, const int* sid, const int* rank, int64_t N,
                       const GridDims* gd_dev, hipStream_t st, CellGrid& G, std::string& err) {
    uint64_t* key = nullptr;
    int* val = nullptr;
    int *head = nullptr, *incl = nullptr;
    GCHK(sc.get(key, N));
    GCHK(sc.get(val, N));
    GCHK(sc.get(G.ck, N));
    GCHK(sc.get(G.cp, N));
    GCHK(sc.get(G.Ps, N));
    GCHK(sc.get(G.ss, N));
    if (rank) GCHK(sc.get(G.rs, N));
    GCHK(sc.get(G.us, N));
    GCHK(sc.get(head, N));
    GCHK(sc.get(incl, N));
    hipLaunchKernelGGL(k_g_cellkey, dim3(nblk(N)), dim3(kGT), 0, st, P, sid, gd_dev, N, key, val);
    GCHK(sort_pairs(sc, key, G.ck, val, G.cp, N, st));
    hipLaunchKernelGGL(k_g_gather, dim3(nblk(N)), dim3(kGT), 0, st, G.ck, G.cp, P, sid, rank, N, G.Ps, G.ss, G.rs,
                       head);
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

template <typename T>
hipError_t upload(Scratch& sc, const std::vector<T>& v, T*& out, hipStream_t st) {
    hipError_t e = sc.get(out, v.size());
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(out, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st);
}

}  // namespace

struct GraphBuild {
    int n_sets = 0;
    int k = 0;
    amm_dtype dtype = AMM_F64;
    std::vector<int64_t> pt_off, node_off, edge_off;
    std::vector<amm_graph_info> info;
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

amm_status graph_build(void* stream, const amm_graph_in* in, int n_sets, amm_graph_info* info_out, GraphBuild** out,
                       std::string& err) {
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (n_sets < 1 || n_sets > kMaxSets) {
        err = "graph: bad number of point sets";
        return AMM_ERR_INVALID_ARG;
    }
    const int k = in[0].k;
    const amm_dtype dt = in[0].dtype;
    std::vector<int64_t> off(n_sets + 1, 0);
    for (int s = 0; s < n_sets; ++s) {
        const amm_graph_in& g = in[s];
        if (!g.src_xyz || g.n_src < 2 || g.k != k || k < 1 || k > kMaxK || g.dtype != dt ||
            (dt != AMM_F32 && dt != AMM_F64) || (g.geodesic != 0) != (in[0].geodesic != 0)) {
            err = "graph: bad source pointer, size, k or dtype (k, dtype and the distance must agree over the sets)";
            return AMM_ERR_INVALID_ARG;
        }
        off[s + 1] = off[s] + g.n_src;
    }
    const int64_t N = off[n_sets];
    if (N > (int64_t)INT32_MAX / 32) {
        err = "graph: too many points";
        return AMM_ERR_INVALID_ARG;
    }
    Scratch sc;
    const unsigned nb1 = nblk(N);
    double4* P = nullptr;
    int64_t* off_d = nullptr;
    int* sid = nullptr;
    double* stats = nullptr;
    GCHK(sc.get(P, N));
    GCHK(sc.get(sid, N));
    GCHK(sc.get(stats, 15 * (size_t)n_sets));
    GCHK(upload(sc, off, off_d, st));
    for (int s = 0; s < n_sets; ++s) {
        if (dt == AMM_F64)
            hipLaunchKernelGGL(k_g_load<double>, dim3(nblk(in[s].n_src)), dim3(kGT), 0, st,
                               (const double*)in[s].src_xyz, P + off[s], in[s].n_src);
        else
            hipLaunchKernelGGL(k_g_load<float>, dim3(nblk(in[s].n_src)), dim3(kGT), 0, st,
                               (const float*)in[s].src_xyz, P + off[s], in[s].n_src);
    }
    hipLaunchKernelGGL(k_g_setid, dim3(nb1), dim3(kGT), 0, st, off_d, n_sets, N, sid);
    hipLaunchKernelGGL(k_g_setstats, dim3(n_sets), dim3(kGT), 0, st, P, off_d, stats);
    std::vector<double> hs(15 * (size_t)n_sets);
    GCHK(hipMemcpyAsync(hs.data(), stats, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, st));
    GCHK(hipStreamSynchronize(st));

    // per set: axis, bounding box, the k-NN grid
    std::vector<double> ax(6 * (size_t)n_sets);
    std::vector<GridDims> gk(n_sets);
    std::vector<double> lo3(3 * (size_t)n_sets), hi3(3 * (size_t)n_sets), diag(n_sets);
    for (int s = 0; s < n_sets; ++s) {
        const double* o = &hs[15 * (size_t)s];
        for (int q = 0; q < 15; ++q)
            if (!std::isfinite(o[q])) {
                err = "graph: non-finite source coordinate";
                return AMM_ERR_NONFINITE;
            }
        const double n = (double)in[s].n_src;
        const double C[3][3] = {{o[9] / n, o[10] / n, o[11] / n},
                                {o[10] / n, o[12] / n, o[13] / n},
                                {o[11] / n, o[13] / n, o[14] / n}};
        double a[3];
        sym3_top_eigvec(C, a);
        for (int q = 0; q < 3; ++q) {
            ax[6 * s + q] = o[6 + q] / n;
            ax[6 * s + 3 + q] = a[q];
            lo3[3 * s + q] = o[q];
            hi3[3 * s + q] = o[3 + q];
        }
        const double ex = o[3] - o[0], ey = o[4] - o[1], ez = o[5] - o[2];
        if (!(std::max({ex, ey, ez}) > 0)) {
            err = "graph: all source points of a set coincide";
            return AMM_ERR_INVALID_ARG;
        }
        diag[s] = std::sqrt(ex * ex + ey * ey + ez * ez);
        if (!grid_for(&lo3[3 * s], &hi3[3 * s], diag[s] / std::cbrt(n), gk[s])) {
            err = "graph: grid too fine";
            return AMM_ERR_INVALID_ARG;
        }
    }
    double* ax_d = nullptr;
    GCHK(upload(sc, ax, ax_d, st));

    // order along each set's axis: by projection, then (stably) by set
    double *tk = nullptr, *tks = nullptr;
    int *tv = nullptr, *o1 = nullptr, *s1 = nullptr, *s2 = nullptr, *order = nullptr, *rank = nullptr;
    GCHK(sc.get(tk, N));
    GCHK(sc.get(tks, N));
    GCHK(sc.get(tv, N));
    GCHK(sc.get(o1, N));
    GCHK(sc.get(s1, N));
    GCHK(sc.get(s2, N));
    GCHK(sc.get(order, N));
    GCHK(sc.get(rank, N));
    hipLaunchKernelGGL(k_g_project, dim3(nb1), dim3(kGT), 0, st, P, sid, ax_d, N, tk, tv);
    GCHK(sort_pairs(sc, tk, tks, tv, o1, N, st));
    hipLaunchKernelGGL(k_g_take, dim3(nb1), dim3(kGT), 0, st, o1, sid, N, s1);
    int set_bits = 1;
    while ((1 << set_bits) < n_sets) ++set_bits;
    GCHK(sort_pairs(sc, s1, s2, o1, order, N, st, set_bits));
    hipLaunchKernelGGL(k_g_invert, dim3(nb1), dim3(kGT), 0, st, order, rank, N);

    // host copies of uploaded bounds live until the function returns (the
    // uploads are asynchronous)
    std::vector<uint64_t> knn_bounds(n_sets + 1), edge_bounds(n_sets + 1);

    // mean edge length per set (6-NN graph); its sorted unique keys stay
    // for the geodesic build
    std::vector<double> lbar(n_sets);
    const bool geo = in[0].geodesic != 0;
    uint64_t* knn_keys = nullptr;
    int* knn_flag = nullptr;
    const int64_t knn_M = N * kKnn;
    {
        GridDims* gk_d = nullptr;
        GCHK(upload(sc, gk, gk_d, st));
        CellGrid G;
        TRY_STATUS(build_cells(sc, P, sid, nullptr, N, gk_d, st, G, err));
        const int64_t M = N * kKnn;
        uint64_t *pk = nullptr, *pks = nullptr, *bnd = nullptr;
        int* flag = nullptr;
        int64_t* at = nullptr;
        double* lp = nullptr;
        GCHK(sc.get(pk, M));
        GCHK(sc.get(pks, M));
        GCHK(sc.get(flag, M));
        GCHK(sc.get(at, n_sets + 1));
        GCHK(sc.get(lp, 2 * (size_t)n_sets));
        for (int s = 0; s <= n_sets; ++s) knn_bounds[s] = (uint64_t)off[s] * (uint64_t)N;
        GCHK(upload(sc, knn_bounds, bnd, st));
        hipLaunchKernelGGL(k_g_knn, dim3(nb1), dim3(kGT), 0, st, G.Ps, G.cp, G.ss, G.ukey, G.ustart, G.nu, N, gk_d,
                           off_d, pk);
        GCHK(sort_keys(sc, pk, pks, M, st));
        hipLaunchKernelGGL(k_g_headflag, dim3(nblk(M)), dim3(kGT), 0, st, pks, M, flag);
        hipLaunchKernelGGL(k_g_bounds, dim3(nblk(n_sets + 1)), dim3(kGT), 0, st, pks, M, bnd, n_sets + 1, at);
        hipLaunchKernelGGL(k_g_edge_len, dim3(n_sets), dim3(kGT), 0, st, pks, flag, at, N, P, lp);
        std::vector<double> hl(2 * (size_t)n_sets);
        GCHK(hipMemcpyAsync(hl.data(), lp, sizeof(double) * hl.size(), hipMemcpyDeviceToHost, st));
        GCHK(hipStreamSynchronize(st));
        for (int s = 0; s < n_sets; ++s) lbar[s] = hl[2 * s + 1] > 0 ? hl[2 * s] / hl[2 * s + 1] : 0.0;
        knn_keys = pks;
        knn_flag = flag;
    }

    // per set: R and the grid of cell size R (slightly enlarged, so that
    // rounding in the cell index never hides a point within R from the 27
    // neighbour cells)
    std::vector<double> Rs(n_sets), R2s(n_sets);
    std::vector<GridDims> gr(n_sets);
    for (int s = 0; s < n_sets; ++s) {
        const double R = in[s].radius > 0 ? in[s].radius
                                          : (in[s].radius_factor > 0 ? in[s].radius_factor : 5.0) * lbar[s];
        if (!(R > 0) || !std::isfinite(R)) {
            err = "graph: radius is not positive";
            return AMM_ERR_INVALID_ARG;
        }
        Rs[s] = R;
        R2s[s] = R * R;
        if (!grid_for(&lo3[3 * s], &hi3[3 * s], R * (1.0 + 1e-9), gr[s])) {
            err = "graph: grid too fine for R";
            return AMM_ERR_INVALID_ARG;
        }
    }
    GridDims* gr_d = nullptr;
    double* R2_d = nullptr;
    GCHK(upload(sc, gr, gr_d, st));
    GCHK(upload(sc, R2s, R2_d, st));
    CellGrid G;
    TRY_STATUS(build_cells(sc, P, sid, rank, N, gr_d, st, G, err));
    int2* nb = nullptr;
    GCHK(sc.get(nb, 27 * (size_t)G.nu));
    hipLaunchKernelGGL(k_g_nbr, dim3(nblk(G.nu)), dim3(kGT), 0, st, G.ukey, G.ustart, G.nu, N, gr_d, nb);

    // geodesic neighbourhoods (Eq. 1): the k-NN edge graph as adjacency
    // rows over the points' global ids, then each point's points within R
    int *goff = nullptr, *gpos = nullptr;
    double* gdist = nullptr;
    if (geo) {
        int *incl = nullptr, *row = nullptr, *col = nullptr, *cnt = nullptr, *ovf = nullptr;
        uint64_t *dkey = nullptr, *dkey_s = nullptr;
        double* Rs_d = nullptr;
        GCHK(sc.get(incl, knn_M));
        GCHK(incl_sum(sc, knn_flag, incl, knn_M, st));
        int n_und = 0;
        GCHK(hipMemcpyAsync(&n_und, incl + (knn_M - 1), sizeof(int), hipMemcpyDeviceToHost, st));
        GCHK(hipStreamSynchronize(st));
        const int64_t E2 = 2 * (int64_t)n_und;
        GCHK(sc.get(dkey, E2));
        GCHK(sc.get(dkey_s, E2));
        GCHK(sc.get(row, N + 1));
        GCHK(sc.get(col, E2));
        hipLaunchKernelGGL(k_g_directed, dim3(nblk(knn_M)), dim3(kGT), 0, st, knn_keys, knn_flag, incl, knn_M, N,
                           dkey);
        GCHK(sort_keys(sc, dkey, dkey_s, E2, st));
        hipLaunchKernelGGL(k_g_rows, dim3(nblk(std::max<int64_t>(E2, N + 1))), dim3(kGT), 0, st, dkey_s, E2, N, row,
                           col);
        GCHK(upload(sc, Rs, Rs_d, st));
        GCHK(sc.get(cnt, N));
        GCHK(sc.get(ovf, 1));
        GCHK(hipMemsetAsync(ovf, 0, sizeof(int), st));
        hipLaunchKernelGGL(k_g_geoball<true>, dim3((unsigned)N), dim3(kGeoThreads), 0, st, G.Ps, P, G.cp, G.ss,
                           G.us, nb, row, col, R2_d, Rs_d, cnt, nullptr, nullptr, nullptr, ovf);
        GCHK(sc.get(goff, N + 1));
        GCHK(hipMemsetAsync(goff, 0, sizeof(int), st));
        GCHK(incl_sum(sc, cnt, goff + 1, N, st));
        int total = 0, over = 0;
        GCHK(hipMemcpyAsync(&total, goff + N, sizeof(int), hipMemcpyDeviceToHost, st));
        GCHK(hipMemcpyAsync(&over, ovf, sizeof(int), hipMemcpyDeviceToHost, st));
        GCHK(hipStreamSynchronize(st));
        if (over) {
            err = "graph: more than 1024 points within R of a point (geodesic build)";
            return AMM_ERR_INVALID_ARG;
        }
        GCHK(sc.get(gpos, std::max(total, 1)));
        GCHK(sc.get(gdist, std::max(total, 1)));
        hipLaunchKernelGGL(k_g_geoball<false>, dim3((unsigned)N), dim3(kGeoThreads), 0, st, G.Ps, P, G.cp, G.ss,
                           G.us, nb, row, col, R2_d, Rs_d, cnt, goff, gpos, gdist, ovf);
        GCHK(hipGetLastError());
    }

    // node selection in rounds
    int *state = nullptr, *remaining = nullptr, *wait = nullptr, *cov = nullptr;
    GCHK(sc.get(state, N));
    GCHK(sc.get(wait, N));
    GCHK(sc.get(cov, N));
    GCHK(hipMemsetAsync(cov, 0, sizeof(int) * N, st));
    GCHK(sc.get(remaining, 1));
    GCHK(hipMemsetAsync(state, 0, sizeof(int) * N, st));
    GCHK(hipMemsetAsync(wait, 0xff, sizeof(int) * N, st));   // -1: nothing to wait for
    int rounds = 0;
    for (;;) {
        int left = 0;
        // a few rounds per read-back; extra rounds after the last decision do nothing
        for (int r = 0; r < 4; ++r) {
            GCHK(hipMemsetAsync(remaining, 0, sizeof(int), st));
            if (geo)
                hipLaunchKernelGGL(k_g_round_geo, dim3(nb1), dim3(kGT), 0, st, G.rs, goff, gpos, state, cov, wait, N,
                                   remaining);
            else
                hipLaunchKernelGGL(k_g_round, dim3(nb1), dim3(kGT), 0, st, G.Ps, G.rs, G.ss, G.us, nb, state, cov,
                                   wait, N, R2_d, remaining);
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

    // node ids in axis order (global over the sets, then local)
    int *flag_r = nullptr, *pos_r = nullptr, *nid_r = nullptr, *nid_s = nullptr;
    int64_t* node_off_d = nullptr;
    GCHK(sc.get(flag_r, N));
    GCHK(sc.get(pos_r, N));
    GCHK(sc.get(nid_r, N));
    GCHK(sc.get(nid_s, N));
    GCHK(sc.get(node_off_d, n_sets + 1));
    hipLaunchKernelGGL(k_g_nodeflag, dim3(nb1), dim3(kGT), 0, st, G.rs, state, N, flag_r, pos_r);
    GCHK(incl_sum(sc, flag_r, nid_r, N, st));
    hipLaunchKernelGGL(k_g_setnodes, dim3(nblk(n_sets + 1)), dim3(kGT), 0, st, nid_r, flag_r, off_d, n_sets,
                       node_off_d);
    std::vector<int64_t> node_off(n_sets + 1);
    GCHK(hipMemcpyAsync(node_off.data(), node_off_d, sizeof(int64_t) * (n_sets + 1), hipMemcpyDeviceToHost, st));
    GCHK(hipStreamSynchronize(st));
    const int64_t n_nodes = node_off[n_sets];
    auto res = std::make_unique<GraphBuild>();
    res->n_sets = n_sets;
    res->k = k;
    res->dtype = dt;
    res->pt_off = off;
    res->node_off = node_off;
    int* nset = nullptr;
    GCHK(sc.get(nset, std::max<int64_t>(n_nodes, 1)));
    GCHK(hipMalloc((void**)&res->node_src, sizeof(int) * std::max<int64_t>(n_nodes, 1)));
    GCHK(hipMalloc((void**)&res->infl_idx, sizeof(int) * (size_t)N * k));
    GCHK(hipMalloc(&res->infl_w, (dt == AMM_F64 ? 8 : 4) * (size_t)N * k));
    hipLaunchKernelGGL(k_g_nodeid, dim3(nb1), dim3(kGT), 0, st, flag_r, nid_r, pos_r, G.cp, G.ss, off_d, N, nid_s,
                       res->node_src, nset);

    // influence sets, weights, node pairs
    const int npair = k * (k - 1) / 2;
    const int64_t M = N * npair;
    uint64_t *pk = nullptr, *pks = nullptr;
    int* gst = nullptr;
    GCHK(sc.get(gst, 2 * (size_t)n_sets));
    GCHK(hipMemsetAsync(gst, 0, 2 * sizeof(int) * n_sets, st));
    GCHK(sc.get(pk, std::max<int64_t>(M, 1)));
    GCHK(sc.get(pks, std::max<int64_t>(M, 1)));
    if (geo && dt == AMM_F64)
        hipLaunchKernelGGL(k_g_influence_geo<double>, dim3(nb1), dim3(kGT), 0, st, G.ss, goff, gpos, gdist, nid_s,
                           G.cp, node_off_d, R2_d, N, n_nodes, k, res->infl_idx, (double*)res->infl_w, pk, gst);
    else if (geo)
        hipLaunchKernelGGL(k_g_influence_geo<float>, dim3(nb1), dim3(kGT), 0, st, G.ss, goff, gpos, gdist, nid_s,
                           G.cp, node_off_d, R2_d, N, n_nodes, k, res->infl_idx, (float*)res->infl_w, pk, gst);
    else if (dt == AMM_F64)
        hipLaunchKernelGGL(k_g_influence<double>, dim3(nb1), dim3(kGT), 0, st, G.Ps, G.ss, G.us, nb, nid_s, G.cp,
                           node_off_d, R2_d, N, n_nodes, k, res->infl_idx, (double*)res->infl_w, pk, gst);
    else
        hipLaunchKernelGGL(k_g_influence<float>, dim3(nb1), dim3(kGT), 0, st, G.Ps, G.ss, G.us, nb, nid_s, G.cp,
                           node_off_d, R2_d, N, n_nodes, k, res->infl_idx, (float*)res->infl_w, pk, gst);
    std::vector<int64_t> edge_off(n_sets + 1, 0);
    int n_edges = 0;
    if (M > 0) {
        int *flag = nullptr, *incl = nullptr;
        uint64_t *ukey = nullptr, *bnd = nullptr;
        int64_t* at = nullptr;
        GCHK(sc.get(flag, M));
        GCHK(sc.get(incl, M));
        GCHK(sort_keys(sc, pk, pks, M, st));
        hipLaunchKernelGGL(k_g_headflag, dim3(nblk(M)), dim3(kGT), 0, st, pks, M, flag);
        GCHK(incl_sum(sc, flag, incl, M, st));
        GCHK(hipMemcpyAsync(&n_edges, incl + (M - 1), sizeof(int), hipMemcpyDeviceToHost, st));
        GCHK(hipStreamSynchronize(st));
        GCHK(sc.get(ukey, std::max(n_edges, 1)));
        GCHK(hipMalloc((void**)&res->edges, sizeof(int) * 2 * std::max(n_edges, 1)));
        hipLaunchKernelGGL(k_g_edges, dim3(nblk(M)), dim3(kGT), 0, st, pks, flag, incl, M, n_nodes, nset,
                           node_off_d, ukey, res->edges);
        for (int s = 0; s <= n_sets; ++s) edge_bounds[s] = (uint64_t)node_off[s] * (uint64_t)n_nodes;
        GCHK(upload(sc, edge_bounds, bnd, st));
        GCHK(sc.get(at, n_sets + 1));
        hipLaunchKernelGGL(k_g_bounds, dim3(nblk(n_sets + 1)), dim3(kGT), 0, st, ukey, (int64_t)n_edges, bnd,
                           n_sets + 1, at);
        GCHK(hipMemcpyAsync(edge_off.data(), at, sizeof(int64_t) * (n_sets + 1), hipMemcpyDeviceToHost, st));
    } else {
        GCHK(hipMalloc((void**)&res->edges, sizeof(int) * 2));
    }
    std::vector<int> hg(2 * (size_t)n_sets);
    GCHK(hipMemcpyAsync(hg.data(), gst, sizeof(int) * hg.size(), hipMemcpyDeviceToHost, st));
    GCHK(hipStreamSynchronize(st));
    GCHK(hipGetLastError());
    edge_off[n_sets] = n_edges;
    res->edge_off = edge_off;
    res->info.resize(n_sets);
    for (int s = 0; s < n_sets; ++s) {
        amm_graph_info& fo = res->info[s];
        fo.n_nodes = node_off[s + 1] - node_off[s];
        fo.n_edges = edge_off[s + 1] - edge_off[s];
        fo.radius = Rs[s];
        fo.mean_edge_len = lbar[s];
        fo.n_capped = hg[2 * s];
        fo.max_influences = hg[2 * s + 1];
        fo.rounds = rounds;
        if (info_out) info_out[s] = fo;
    }
    *out = res.release();
    return AMM_OK;
}

amm_status graph_copy(const GraphBuild* g, void* stream, int set, int32_t* node_src_idx, int32_t* infl_idx,
                      void* infl_w, int32_t* edges, std::string& err) {
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (set < 0 || set >= g->n_sets) {
        err = "graph: set out of range";
        return AMM_ERR_INVALID_ARG;
    }
    const size_t ws = g->dtype == AMM_F64 ? 8 : 4;
    const int64_t p0 = g->pt_off[set], np = g->pt_off[set + 1] - p0;
    const int64_t n0 = g->node_off[set], nn = g->node_off[set + 1] - n0;
    const int64_t e0 = g->edge_off[set], ne = g->edge_off[set + 1] - e0;
    if (node_src_idx && nn)
        GCHK(hipMemcpyAsync(node_src_idx, g->node_src + n0, sizeof(int) * nn, hipMemcpyDeviceToDevice, st));
    if (infl_idx)
        GCHK(hipMemcpyAsync(infl_idx, g->infl_idx + (size_t)p0 * g->k, sizeof(int) * (size_t)np * g->k,
                            hipMemcpyDeviceToDevice, st));
    if (infl_w)
        GCHK(hipMemcpyAsync(infl_w, (char*)g->infl_w + ws * (size_t)p0 * g->k, ws * (size_t)np * g->k,
                            hipMemcpyDeviceToDevice, st));
    if (edges && ne)
        GCHK(hipMemcpyAsync(edges, g->edges + 2 * e0, sizeof(int) * 2 * ne, hipMemcpyDeviceToDevice, st));
    return AMM_OK;
}

}  // namespace amm
