// Exact closest-point search over an implicit octree of the targets (shared
// by the kernels and host-side checks; plain arithmetic only).
//
// The targets of a pair are sorted by a 30-bit Morton code (10 bits per axis
// of the coordinate quantized over the targets' bounding box).  A cell of
// level l (0 = the whole box, G = the leaves) is a prefix of 3 l code bits,
// so its targets are one contiguous run of the sorted array.  Level l keeps
// a table of 8^l + 1 run starts (cell m spans [T_l[m], T_l[m + 1])), and the
// eight children of cell m are cells 8 m .. 8 m + 7 of level l + 1: one
// contiguous read of nine starts gives every child's occupancy.  A cell's
// box is not stored: it is computed from the cell's integer coordinates.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "amm_internal.h"

namespace amm {

template <typename T> __host__ __device__ inline T nn_inf() { return (T)INFINITY; }

// Squared length with one fixed evaluation shape (explicit fma chain).  The
// point distance and the cell lower bound use the same shape, and every
// step is monotone in |dx|, |dy|, |dz|, so a cell bound that does not exceed
// the per-axis distances of the cell's targets does not exceed their
// computed squared distances either: pruning with `bound > best` is exact in
// floating point.
template <typename T>
__host__ __device__ inline T sq3(T dx, T dy, T dz) {
    T s = dz * dz;
    s = fma(dy, dy, s);
    s = fma(dx, dx, s);
    return s;
}


// ---------------------------------------------------------------- closest point

// Work of one search, counted only where asked for (COUNT = true): cell
// lower-bound tests (arithmetic only), target distance evaluations (each
// reads one target) and cell expansions that read nine run starts from
// memory (expansions served from the LDS copy are not counted).
struct NnWork {
    int boxes;
    int points;
    int cells;
};

// Lower bound of the distance from q to the cell of integer coordinate j
// (a float holding an integer) along one axis, for cells of size s:
// a = glo - pad - q and b = q - glo - pad, so the cell spans
// [glo + j s, glo + (j + 1) s] widened by pad (which covers the rounding of
// these products and of the targets' stored coordinates).
template <typename T>
__host__ __device__ inline T oct_axis(T a, T b, T s, T j) {
    return (T)fmax(fmax((T)fma(j, s, a), (T)fma(-(j + T(1)), s, b)), T(0));
}

// Exact closest target of q among the pair's targets: depth-first search of
// the octree.  Expanding a cell reads its children's nine run starts and
// keeps the occupied children whose lower bound does not exceed the best
// squared distance so far; they are visited in the order of their octant
// relative to the query (its own octant first, the opposite one last), and
// a child's bound is tested again when its turn comes (the best distance
// only shrinks).  `prev` (a sorted target position from an earlier
// evaluation, or -1) seeds the bound.  Ties in distance go to the lowest
// user target index (stored in .w), and the minimum of (distance, index)
// does not depend on the visiting order, so the result is that of a
// brute-force scan with the same distance shape.
//
// cells: this pair's tables (levels 0..G); near: a copy of levels
// 0..min(G, kOctLdsLevels) (LDS on the device, or `cells` itself).  The
// children still to visit are one byte per level of a 64-bit mask (bit j =
// child j ^ octant), the query's octant three bits per level, so the
// search keeps no stack.
//
// budget > 0 bounds the search's steps (expansions and visits): past it the
// search stops and returns false, best_pos / best_d2 holding the best
// target found so far (an upper bound to hand to another search).
template <typename T, typename V, bool COUNT = false>
__host__ __device__ inline bool oct_search(const PairInfo& pi, const int* __restrict__ cells,
                                           const int* __restrict__ near, const V* __restrict__ tgt, T qx, T qy,
                                           T qz, int prev, int& best_pos, T& best_d2, NnWork* work = nullptr,
                                           int budget = 0) {
    const V* tg = tgt + pi.tgt_off;
    T bd = nn_inf<T>();
    int bid = INT_MAX, bpos = -1;
    if (prev >= 0) {
        const V u = tg[prev];
        bd = sq3(u.x - qx, u.y - qy, u.z - qz);
        bid = (int)u.w;
        bpos = prev;
        if constexpr (COUNT) work->points += 1;
    }
    const int G = pi.grid_bits;
    const T pad = (T)pi.gpad;
    const T ax = ((T)pi.glo[0] - pad) - qx, bx = qx - ((T)pi.glo[0] + pad);
    const T ay = ((T)pi.glo[1] - pad) - qy, by = qy - ((T)pi.glo[1] + pad);
    const T az = ((T)pi.glo[2] - pad) - qz, bz = qz - ((T)pi.glo[2] + pad);
    // the query's coordinates in units of the root cell (for its octant)
    const T ux = pi.cs[0] > 0 ? (qx - (T)pi.glo[0]) / (T)pi.cs[0] : T(0);
    const T uy = pi.cs[1] > 0 ? (qy - (T)pi.glo[1]) / (T)pi.cs[1] : T(0);
    const T uz = pi.cs[2] > 0 ? (qz - (T)pi.glo[2]) / (T)pi.cs[2] : T(0);
    // Start cell: every target whose computed distance does not exceed the
    // seed's lies within r of q on each axis (r = the seed distance widened
    // by a relative 1e-5 and by pad, which cover the rounding of the squared
    // distance, of its root and of the quantization below), so its
    // quantized coordinates lie in [lo, hi] per axis, and the deepest cell
    // holding that whole box (the common leading bits of lo and hi) holds
    // every target the search can accept: the search starts there, at most
    // at level G - 1 (a cold search starts at the root).
    int l0 = 0;
    uint32_t c0x = 0, c0y = 0, c0z = 0;
    if (prev >= 0 && bd < nn_inf<T>()) {
        const T r = sqrt(bd) * T(1.00001) + pad;
        int lz = G - 1;
        uint32_t lo3[3], hi3[3];
        const T qv[3] = {qx, qy, qz};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T gl = (T)pi.glo[c], gs = (T)pi.gscale[c];
            T a = (qv[c] - r - gl) * gs, b = (qv[c] + r - gl) * gs;
            a = fmin(fmax(a, T(0)), T(1023));
            b = fmin(fmax(b, T(0)), T(1023));
            lo3[c] = (uint32_t)floor(a);
            hi3[c] = (uint32_t)floor(b);
            const uint32_t x = lo3[c] ^ hi3[c];
            const int common = x == 0 ? 10 : __builtin_clz(x) - 22;
            lz = common < lz ? common : lz;
        }
        l0 = lz < 0 ? 0 : lz;
        c0x = lo3[0] >> (10 - l0);
        c0y = lo3[1] >> (10 - l0);
        c0z = lo3[2] >> (10 - l0);
    }
    // children's size at the current level (halved on the way down, doubled
    // on the way up: powers of two, exact); children's first coordinate 2 c
    T sx = ldexp((T)pi.cs[0], -(l0 + 1)), sy = ldexp((T)pi.cs[1], -(l0 + 1)), sz = ldexp((T)pi.cs[2], -(l0 + 1));
    T jx = T(2 * c0x), jy = T(2 * c0y), jz = T(2 * c0z);   // 2 x the current cell's coordinates
    int l = l0;                       // level of the current cell
    uint32_t m = 0;                   // its Morton index
    for (int b = l0 - 1; b >= 0; --b)
        m = (m << 3) | (((c0x >> b) & 1u) << 2) | (((c0y >> b) & 1u) << 1) | ((c0z >> b) & 1u);
    uint64_t pend = 0;                // children still to visit, one byte per level
    uint32_t oct = 0;                 // the query's octant, three bits per level
    // run starts of the current level G - 1 cell's children
    int ls0 = 0, ls1 = 0, ls2 = 0, ls3 = 0, ls4 = 0, ls5 = 0, ls6 = 0, ls7 = 0, ls8 = 0;
    bool expand = true;
    bool finished = true;
    int steps = 0;
    while (true) {
        if (budget > 0 && ++steps > budget) {
            finished = false;
            break;
        }
        if (expand) {
            // (two branches, so each read keeps its own address space)
            const int64_t o = oct_level_off(l + 1) + 8 * (int64_t)m;
            int st[9];
            if (l < kOctLdsLevels) {
#pragma unroll
                for (int q = 0; q < 9; ++q) st[q] = near[o + q];
            } else {
#pragma unroll
                for (int q = 0; q < 9; ++q) st[q] = cells[o + q];
                if constexpr (COUNT) work->cells += 1;
            }
            if (l == G - 1) {
                ls0 = st[0];
                ls1 = st[1];
                ls2 = st[2];
                ls3 = st[3];
                ls4 = st[4];
                ls5 = st[5];
                ls6 = st[6];
                ls7 = st[7];
                ls8 = st[8];
            }
            // the eight children's bounds from two values per axis
            const T dx0 = oct_axis(ax, bx, sx, jx), dx1 = oct_axis(ax, bx, sx, jx + T(1));
            const T dy0 = oct_axis(ay, by, sy, jy), dy1 = oct_axis(ay, by, sy, jy + T(1));
            const T dz0 = oct_axis(az, bz, sz, jz), dz1 = oct_axis(az, bz, sz, jz + T(1));
            const T z0 = dz0 * dz0, z1 = dz1 * dz1;
            const T y00 = (T)fma(dy0, dy0, z0), y01 = (T)fma(dy0, dy0, z1), y10 = (T)fma(dy1, dy1, z0),
                    y11 = (T)fma(dy1, dy1, z1);
            const T cb[8] = {(T)fma(dx0, dx0, y00), (T)fma(dx0, dx0, y01), (T)fma(dx0, dx0, y10),
                             (T)fma(dx0, dx0, y11), (T)fma(dx1, dx1, y00), (T)fma(dx1, dx1, y01),
                             (T)fma(dx1, dx1, y10), (T)fma(dx1, dx1, y11)};
            // the query's octant in this cell: which half of each axis
            const T half = ldexp(T(1), -(l + 1));
            const uint32_t qo = (ux >= (jx + T(1)) * half ? 4u : 0u) | (uy >= (jy + T(1)) * half ? 2u : 0u) |
                                (uz >= (jz + T(1)) * half ? 1u : 0u);
            uint32_t keep = 0;
#pragma unroll
            for (int c = 0; c < 8; ++c) keep |= (st[c + 1] > st[c] && cb[c] <= bd ? 1u : 0u) << c;
            // bit j of the visiting mask = child j ^ qo
            keep = (qo & 4u) ? ((keep >> 4) | (keep << 4)) & 0xffu : keep;
            keep = (qo & 2u) ? ((keep >> 2) & 0x33u) | ((keep << 2) & 0xccu) : keep;
            keep = (qo & 1u) ? ((keep >> 1) & 0x55u) | ((keep << 1) & 0xaau) : keep;
            if constexpr (COUNT) {
#pragma unroll
                for (int c = 0; c < 8; ++c) work->boxes += st[c + 1] > st[c] ? 1 : 0;
            }
            pend = (pend & ~(0xffull << (8 * l))) | ((uint64_t)keep << (8 * l));
            oct = (oct & ~(7u << (3 * l))) | (qo << (3 * l));
        }
        const uint32_t pm = (uint32_t)(pend >> (8 * l)) & 0xffu;
        if (pm == 0) {
            if (l == l0) break;
            m >>= 3;
            jx = T(2) * floor(jx * T(0.25));
            jy = T(2) * floor(jy * T(0.25));
            jz = T(2) * floor(jz * T(0.25));
            sx *= T(2);
            sy *= T(2);
            sz *= T(2);
            --l;
            expand = false;
            continue;
        }
        const int j = __builtin_ctz(pm);
        pend &= ~(1ull << (8 * l + j));
        const uint32_t c = (uint32_t)j ^ ((oct >> (3 * l)) & 7u);
        const T cjx = jx + (T)((c >> 2) & 1u), cjy = jy + (T)((c >> 1) & 1u), cjz = jz + (T)(c & 1u);
        const T cbd = sq3(oct_axis(ax, bx, sx, cjx), oct_axis(ay, by, sy, cjy), oct_axis(az, bz, sz, cjz));
        if (cbd > bd) {
            expand = false;
            continue;
        }
        if (l == G - 1) {
            // the child is a leaf: scan its run (starts kept from this
            // cell's expansion; selects, not an indexed array, so they stay
            // in registers), then go on at this level
            const int s = c < 4 ? (c < 2 ? (c == 0 ? ls0 : ls1) : (c == 2 ? ls2 : ls3))
                                : (c < 6 ? (c == 4 ? ls4 : ls5) : (c == 6 ? ls6 : ls7));
            const int e = c < 4 ? (c < 2 ? (c == 0 ? ls1 : ls2) : (c == 2 ? ls3 : ls4))
                                : (c < 6 ? (c == 4 ? ls5 : ls6) : (c == 6 ? ls7 : ls8));
            if constexpr (COUNT) work->points += e - s;
            // four targets per round: the loads are independent and issued
            // together (indices past the run repeat its last target, whose
            // second visit changes nothing)
            for (int t = s; t < e; t += 4) {
                const int t1 = min(t + 1, e - 1), t2 = min(t + 2, e - 1), t3 = min(t + 3, e - 1);
                const V u0 = tg[t], u1 = tg[t1], u2 = tg[t2], u3 = tg[t3];
                const T d0 = sq3(u0.x - qx, u0.y - qy, u0.z - qz);
                const T d1 = sq3(u1.x - qx, u1.y - qy, u1.z - qz);
                const T d2 = sq3(u2.x - qx, u2.y - qy, u2.z - qz);
                const T d3 = sq3(u3.x - qx, u3.y - qy, u3.z - qz);
                const int i0 = (int)u0.w, i1 = (int)u1.w, i2 = (int)u2.w, i3 = (int)u3.w;
                if (d0 < bd || (d0 == bd && i0 < bid)) {
                    bd = d0;
                    bid = i0;
                    bpos = t;
                }
                if (d1 < bd || (d1 == bd && i1 < bid)) {
                    bd = d1;
                    bid = i1;
                    bpos = t1;
                }
                if (d2 < bd || (d2 == bd && i2 < bid)) {
                    bd = d2;
                    bid = i2;
                    bpos = t2;
                }
                if (d3 < bd || (d3 == bd && i3 < bid)) {
                    bd = d3;
                    bid = i3;
                    bpos = t3;
                }
            }
            expand = false;
            continue;
        }
        m = 8 * m + c;
        jx = T(2) * cjx;
        jy = T(2) * cjy;
        jz = T(2) * cjz;
        sx *= T(0.5);
        sy *= T(0.5);
        sz *= T(0.5);
        ++l;
        expand = true;
    }
    // a non-finite query matches nothing; keep the index in range
    best_pos = bpos < 0 ? 0 : bpos;
    best_d2 = bd;
    return finished;
}

}  // namespace amm
