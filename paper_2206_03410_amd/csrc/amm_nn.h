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
// lower-bound tests and target distance evaluations.
struct NnWork {
    int boxes;
    int points;
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

}  // namespace amm
