// Exact closest-point search over the implicit box tree (shared by the
// kernels and host-side checks; plain arithmetic only).
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "amm_internal.h"

namespace amm {

template <typename T> __host__ __device__ inline T nn_inf() { return (T)INFINITY; }

// Squared length with one fixed evaluation shape (explicit fma chain).  The
// point distance and the box lower bound use the same shape, so the computed
// box bound never exceeds the computed distance of a point inside the box
// (every step is monotone in |dx|, |dy|, |dz|): pruning with `box > best`
// is therefore exact in floating point.
template <typename T>
__host__ __device__ inline T sq3(T dx, T dy, T dz) {
    T s = dz * dz;
    s = fma(dy, dy, s);
    s = fma(dx, dx, s);
    return s;
}

template <typename T, typename V>
__host__ __device__ inline T box_d2(const V& lo, const V& hi, T qx, T qy, T qz) {
    T dx = fmax(fmax(lo.x - qx, qx - hi.x), T(0));
    T dy = fmax(fmax(lo.y - qy, qy - hi.y), T(0));
    T dz = fmax(fmax(lo.z - qz, qz - hi.z), T(0));
    return sq3(dx, dy, dz);
}

// ---------------------------------------------------------------- closest point

// Work of one search, counted only where asked for (COUNT = true): box
// lower-bound tests, target distance evaluations and grid cell lookups.
struct NnWork {
    int boxes;
    int points;
    int cells;
};

// Exact closest target of query q among the pair's targets, by depth-first
// traversal of the implicit complete binary tree of boxes (heap layout: node
// 1 is the root, children 2i and 2i+1, leaves L..2L-1 each holding `leaf`
// consecutive Morton-sorted targets).  Near child first; pending far
// children are kept as one bit per level (no stack).  `prev` (a target
// position from the previous evaluation, or -1) seeds the bound.  Ties in
// distance go to the lowest user target index (stored in .w).  With COUNT,
// `work` accumulates the box tests and distance evaluations.
template <typename T, typename V, bool COUNT = false>
__host__ __device__ inline void nn_search(const PairInfo& pi, const V* __restrict__ tgt,
                                          const V* __restrict__ blo,
                                          const V* __restrict__ bhi, T qx, T qy,
                                          T qz, int prev, int& best_pos, T& best_d2,
                                          NnWork* work = nullptr) {
    const V* lo = blo + pi.tree_off;
    const V* hi = bhi + pi.tree_off;
    const V* tg = tgt + pi.tgt_off;
    const unsigned L = (unsigned)pi.L;
    const int LB = pi.leaf;
    const int M = (int)pi.M;
    T bd = nn_inf<T>();
    int bid = INT_MAX, bpos = -1;
    if (prev >= 0) {
        V u = tg[prev];
        bd = sq3(u.x - qx, u.y - qy, u.z - qz);
        bid = (int)u.w;
        bpos = prev;
        if constexpr (COUNT) work->points += 1;
    }
    unsigned node = 1, trail = 0;
    int depth = 0;
    while (true) {
        if (node < L) {
            const unsigned c0 = node << 1, c1 = c0 | 1u;
            const T d0 = box_d2<T>(lo[c0], hi[c0], qx, qy, qz);
            const T d1 = box_d2<T>(lo[c1], hi[c1], qx, qy, qz);
            if constexpr (COUNT) work->boxes += 2;
            const bool first0 = d0 <= d1;
            const T dn = first0 ? d0 : d1, df = first0 ? d1 : d0;
            if (dn <= bd) {
                if (df <= bd) trail |= 1u << (depth + 1);
                node = first0 ? c0 : c1;
                ++depth;
                continue;
            }
        } else {
            const int s = (int)(node - L) * LB;
            const int e = min(s + LB, M);
            if constexpr (COUNT) work->points += e - s;
            for (int t = s; t < e; ++t) {
                V u = tg[t];
                T d = sq3(u.x - qx, u.y - qy, u.z - qz);
                int id = (int)u.w;
                if (d < bd || (d == bd && id < bid)) {
                    bd = d;
                    bid = id;
                    bpos = t;
                }
            }
        }
        bool next = false;
        while (trail) {
            const int lvl = 31 - __builtin_clz(trail);
            trail &= ~(1u << lvl);
            node = (node >> (depth - lvl)) ^ 1u;
            depth = lvl;
            if constexpr (COUNT) work->boxes += 1;
            if (box_d2<T>(lo[node], hi[node], qx, qy, qz) <= bd) {
                next = true;
                break;
            }
        }
        if (!next) break;
    }
    // a non-finite query matches nothing; keep the index in range
    best_pos = bpos < 0 ? 0 : bpos;
    best_d2 = bd;
}

// ---------------------------------------------------------------- grid

__host__ __device__ inline uint32_t nn_spread10(uint32_t x) {
    x &= 0x3ff;
    x = (x | (x << 16)) & 0x030000ff;
    x = (x | (x << 8)) & 0x0300f00f;
    x = (x | (x << 4)) & 0x030c30c3;
    x = (x | (x << 2)) & 0x09249249;
    return x;
}

constexpr int kGridMaxCells = 32;

// Cell range of one axis covered by [q - r, q + r] (clamped to the grid).
template <typename T>
__host__ __device__ inline void grid_axis(T q, T r, double glo, double gscale, int sh, int& lo, int& hi) {
    const T o = (T)glo, s = (T)gscale;
    T a = (q - r - o) * s, b = (q + r - o) * s;
    a = fmin(fmax(a, T(0)), T(1023));
    b = fmin(fmax(b, T(0)), T(1023));
    lo = (int)floor(a) >> sh;
    hi = (int)floor(b) >> sh;
}

// Exact closest target of q when a target position `prev` bounds it: every
// target at computed squared distance <= bd = |u_prev - q|^2 lies within
// sqrt(bd) (times 1 + 3 ulp) of q on each axis, hence in the grid cells that
// [q - r, q + r] covers, r = sqrt(bd) widened by a relative 1e-5 and by
// pi.gpad (the cell bounds' rounding).  Those cells are scanned with the
// tree search's distance shape and tie rule (the lowest user index), and
// the lexicographic minimum of (distance, index) does not depend on the
// order of visits, so the result is the tree search's.  Returns false,
// leaving the outputs alone, when the range covers more than kGridMaxCells
// cells or the bound is not finite (then the tree is searched).
template <typename T, typename V, bool COUNT = false>
__host__ __device__ inline bool grid_search(const PairInfo& pi, const int* __restrict__ cells,
                                            const V* __restrict__ tgt, T qx, T qy, T qz, int prev,
                                            int& best_pos, T& best_d2, NnWork* work = nullptr) {
    const V* tg = tgt + pi.tgt_off;
    const V u = tg[prev];
    T bd = sq3(u.x - qx, u.y - qy, u.z - qz);
    if (!(bd < nn_inf<T>())) return false;
    const T r = sqrt(bd) * T(1.00001) + (T)pi.gpad;
    const int sh = 10 - pi.grid_bits;
    int x0, x1, y0, y1, z0, z1;
    grid_axis<T>(qx, r, pi.glo[0], pi.gscale[0], sh, x0, x1);
    grid_axis<T>(qy, r, pi.glo[1], pi.gscale[1], sh, y0, y1);
    grid_axis<T>(qz, r, pi.glo[2], pi.gscale[2], sh, z0, z1);
    if ((x1 - x0 + 1) * (y1 - y0 + 1) * (z1 - z0 + 1) > kGridMaxCells) return false;
    const int* cl = cells + pi.grid_off;
    int bid = (int)u.w, bpos = prev;
    for (int cz = z0; cz <= z1; ++cz)
        for (int cy = y0; cy <= y1; ++cy)
            for (int cx = x0; cx <= x1; ++cx) {
                const uint32_t m = (nn_spread10((uint32_t)cx) << 2) | (nn_spread10((uint32_t)cy) << 1) |
                                   nn_spread10((uint32_t)cz);
                const int s0 = cl[m], s1 = cl[m + 1];
                if constexpr (COUNT) {
                    work->cells += 1;
                    work->points += s1 - s0;
                }
                for (int t = s0; t < s1; ++t) {
                    const V w = tg[t];
                    const T d = sq3(w.x - qx, w.y - qy, w.z - qz);
                    const int id = (int)w.w;
                    if (d < bd || (d == bd && id < bid)) {
                        bd = d;
                        bid = id;
                        bpos = t;
                    }
                }
            }
    if constexpr (COUNT) work->points += 1;   // the bound's own target
    best_pos = bpos;
    best_d2 = bd;
    return true;
}

}  // namespace amm
