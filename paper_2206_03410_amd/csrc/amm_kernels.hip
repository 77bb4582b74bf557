// HIP kernels for gfx950 (MI355X) implementing one MM iteration of robust
// non-rigid registration (arXiv 2206.03410, Sec. 3.3) and its gradient.
//
// Every kernel is batched: tiles never straddle pairs, and per-pair scalars
// (nu, alpha, beta, flags) come from a small PairDyn array.  All reductions
// are fixed-order trees (no floating-point atomics), so results are
// bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <algorithm>
#include <climits>
#include <type_traits>

#include "amm_device.h"
#include "amm_kernels.h"
#include "amm_nn.h"

namespace amm {

// ---------------------------------------------------------------- evaluation

// Warp of source point i (Eq. 2): v_hat (absolute, for the search) and, for
// the residual, the small parts s = sum_j w_ij ((A_j - I)(v_i - p_j) + t_j)
// and sw1 = sum_j w_ij - 1 (the weights' sum in float64: exact for k <= 8
// terms).
template <typename T, typename V>
__device__ __forceinline__ void warp_point(const EvalArgs<T>& a, const T* __restrict__ X, int i, const V& v, T& vx,
                                           T& vy, T& vz, T& sx, T& sy, T& sz, T& sw1) {
    vx = vy = vz = sx = sy = sz = 0;
    double sw = 0;
    for (int s = 0; s < a.k; ++s) {
        const int j = a.iidx[(size_t)s * a.Ntot + i];
        const T w = a.iw[(size_t)s * a.Ntot + i];
        const V pj = a.nodes[j];
        const T* Xj = X + 12 * (size_t)j;
        const T dx = v.x - pj.x, dyy = v.y - pj.y, dz = v.z - pj.z;
        const T gx = dx * (Xj[0] - T(1)) + dyy * Xj[3] + dz * Xj[6] + Xj[9];
        const T gy = dx * Xj[1] + dyy * (Xj[4] - T(1)) + dz * Xj[7] + Xj[10];
        const T gz = dx * Xj[2] + dyy * Xj[5] + dz * (Xj[8] - T(1)) + Xj[11];
        vx += w * (dx * Xj[0] + dyy * Xj[3] + dz * Xj[6] + Xj[9] + pj.x);
        vy += w * (dx * Xj[1] + dyy * Xj[4] + dz * Xj[7] + Xj[10] + pj.y);
        vz += w * (dx * Xj[2] + dyy * Xj[5] + dz * Xj[8] + Xj[11] + pj.z);
        sx += w * gx;
        sy += w * gy;
        sz += w * gz;
        sw += (double)w;
    }
    sw1 = (T)(sw - 1.0);
}

// Everything of point i that follows its closest target (sorted position
// bpos of pair p): the residual e_i, the alignment term and weight, the
// outputs, and the point's energy term and displacement for the tile sums.
template <typename T, typename V>
__device__ __forceinline__ void finish_point(const EvalArgs<T>& a, const PairDyn& dy, const PairInfo& pi, int i,
                                             const V& v, T vx, T vy, T vz, T sx, T sy, T sz, T sw1, int bpos) {
    const int dst = dy.eval_dst, cur = dy.cur;
    const V u = a.tgt[pi.tgt_off + bpos];
    // e_i = v_hat_i - u_rho(i)
    //     = sum_j w_ij ((A_j - I) d_ij + t_j) + (v_i - u) + (sum_j w_ij - 1) v_i
    // (Eq. 2 rearranged): every operand is small, so e_i keeps its relative
    // accuracy where v_hat_i - u would cancel; d^2 is taken from it
    V q;
    q.x = sx + (v.x - u.x) + sw1 * v.x;
    q.y = sy + (v.y - u.y) + sw1 * v.y;
    q.z = sz + (v.z - u.z) + sw1 * v.z;
    const T d2 = sq3(q.x, q.y, q.z);
    T wa, psi;
    if (dy.robust == AMM_ROBUST_WELSCH) {
        const T inv = T(1) / (T(2) * (T)dy.nu_a * (T)dy.nu_a);
        const T t = d2 * inv;
        psi = -expm1(-t);
        wa = exp(-t) * inv;
    } else if (dy.robust == AMM_ROBUST_L2) {
        psi = d2;
        wa = T(1);
    } else {
        // truncated quadratic: weight 1 inside 3 nu_a, constant outside
        const T tau2 = T(9) * (T)dy.nu_a * (T)dy.nu_a;
        const bool in = d2 < tau2;
        psi = in ? d2 : tau2;
        wa = in ? T(1) : T(0);
    }
    q.w = wa;
    a.qw[dst][i] = q;
    a.rho[dst][i] = (int)pi.tgt_off + bpos;
    a.d2[dst][i] = d2;
    T disp = 0;
    if (dy.has_prev) {
        const V o = a.vhat[cur][i];
        disp = sqrt(sq3(vx - o.x, vy - o.y, vz - o.z));
    }
    a.pt_psi[i] = psi;
    a.pt_disp[i] = disp;
}

// Per source point: warp (Eq. 2), closest target, Welsch value and weight
// (Eqs. 5, 6 and the weight w_a of Eq. 16) or those of a squared-norm
// variant of Sec. 4.1, the alignment residual e_i = v_hat_i - u_rho(i), and
// the max displacement against the accepted iterate.  One thread per point.
// A search that exceeds the step budget (a.nn_budget) leaves its point to
// k_eval_far (one wave per point); the tile sums follow in k_eval_sums.
// COUNT adds the search's work to the tile's counters (reporting only).
template <typename T, bool COUNT>
__global__ void __launch_bounds__(kPointTile) k_eval_points(EvalArgs<T> a) {
    using V = typename V4Of<T>::type;
    __shared__ long long shc[COUNT ? kPointTile : 1];
    __shared__ int oct[kOctLdsInts];
    NnWork wk{0, 0, 0};
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int4 td = a.pt_tiles[tile];
    const int p = td.x;
    const PairDyn dy = a.dyn[p];
    if (!(dy.flags & PF_EVAL)) return;                 // uniform over the block
    const PairInfo pi = a.info[p];
    // the octree's upper levels (every search starts there) into LDS
    const int* cells = a.grid + pi.grid_off;
    {
        const int nl = (int)oct_level_off(min(pi.grid_bits, kOctLdsLevels) + 1);
        for (int q = (int)threadIdx.x; q < nl; q += kPointTile) oct[q] = cells[q];
        __syncthreads();
    }
    const int i = td.y + (int)threadIdx.x;
    const int dst = dy.eval_dst;
    const T* X = a.X[dy.eval_x];
    const V* src = a.src_override ? (const V*)a.src_override : (const V*)a.src;
    bool far = false;
    if (i < td.z) {
        const V v = src[i];
        T vx, vy, vz, sx, sy, sz, sw1;
        warp_point<T, V>(a, X, i, v, vx, vy, vz, sx, sy, sz, sw1);
        V vh;
        vh.x = vx;
        vh.y = vy;
        vh.z = vz;
        vh.w = 0;
        const int prev = dy.has_prev ? a.rho[dy.cur][i] - (int)pi.tgt_off : -1;
        int bpos;
        T d2;
        const bool done = oct_search<T, V, COUNT>(pi, cells, oct, a.tgt, vx, vy, vz, prev, bpos, d2, &wk, a.nn_budget);
        if (done) {
            finish_point<T, V>(a, dy, pi, i, v, vx, vy, vz, sx, sy, sz, sw1, bpos);
            a.vhat[dst][i] = vh;   // after the displacement has read set cur
        } else {
            // the best target so far seeds the wave-wide search, which
            // finishes the point (v_hat included)
            far = true;
            a.far_seed[i] = d2 < nn_inf<T>() ? bpos : -1;
        }
    }
    // deferred points, appended wave by wave (the order does not matter:
    // each is finished on its own)
    const unsigned long long fm = __ballot(far);
    if (fm) {
        const int lane = (int)(threadIdx.x & 63);
        int base = 0;
        if (lane == __ffsll((long long)fm) - 1) base = atomicAdd(a.far_count, (int)__popcll(fm));
        base = __shfl(base, __ffsll((long long)fm) - 1);
        const int slot = base + (int)__popcll(fm & ((1ull << lane) - 1ull));
        if (far && slot < a.Ntot) a.far_list[slot] = make_int2(i, p);
    }
    if constexpr (COUNT) {
        const long long nb = block_sum<long long, kPointTile>(wk.boxes, shc);
        const long long np = block_sum<long long, kPointTile>(wk.points, shc);
        const long long nc = block_sum<long long, kPointTile>(wk.cells, shc);
        if (threadIdx.x == 0) {
            // one block per tile and launch, launches in stream order
            long long* c = a.nn_work + 4 * (size_t)tile;
            c[0] += td.z - td.y;
            c[1] += nb;
            c[2] += np;
            c[3] += nc;
        }
    }
}

// ---------------------------------------------------------------- deferred closest points

constexpr int kFarWaves = 4;       // waves per block of k_eval_far
constexpr int kFarGroup = 16;      // lanes per deferred point
constexpr int kFarPts = 64 / kFarGroup;   // points per wave
constexpr int kFarCap = 128;       // cells per frontier level (per point)
constexpr int kFarRuns = 8 * kFarGroup;   // leaf runs per scan round (one cell per lane, 8 children)

__device__ __forceinline__ uint32_t compact3(uint32_t x) {
    x &= 0x09249249u;
    x = (x ^ (x >> 2)) & 0x030c30c3u;
    x = (x ^ (x >> 4)) & 0x0300f00fu;
    x = (x ^ (x >> 8)) & 0xff0000ffu;
    x = (x ^ (x >> 16)) & 0x000003ffu;
    return x;
}

// orders one wave's shared-memory accesses across its lanes (the waves of
// a k_eval_far block work on different points and do not meet)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// exclusive prefix sum over a group of kFarGroup lanes, and the group's total
__device__ __forceinline__ int group_excl_scan(int v, int gl, int& total) {
    int x = v;
#pragma unroll
    for (int o = 1; o < kFarGroup; o <<= 1) {
        const int y = __shfl_up(x, o, kFarGroup);
        if (gl >= o) x += y;
    }
    total = __shfl(x, kFarGroup - 1, kFarGroup);
    return x - v;
}

// The points whose search ran past the step budget, kFarGroup lanes per
// point (kFarPts points per wave): the same exact search as oct_search (same
// bounds, same distance shape, ties to the lowest user index), but
// breadth-first, the group's lanes working on the cells of a level together
// and scanning the leaves' targets together, pruned by the best distance so
// far (seeded by the budgeted search's best).  A level with more cells than
// the frontier holds falls back to one lane running oct_search from the
// best so far.  The point is then finished as in k_eval_points.
template <typename T>
__device__ void eval_edges_tile(const EvalArgs<T>& a, int tile);
template <typename T>
__device__ void eval_nodes_group(const EvalArgs<T>& a, int tile, int gl, int n_nd_tiles);
constexpr int kNodeGroups = 64 * kFarWaves / kNodeTile;   // node tiles per block of k_eval_far
static_assert(64 * kFarWaves == kEdgeTile, "an edge tile is one block of k_eval_far");

// Blocks past the first far_blocks evaluate the regularization terms (one
// edge tile per block, then kNodeGroups node tiles per block): they depend
// on the transforms only, and run on the compute units that the few long
// deferred searches leave idle.
template <typename T, bool COUNT>
__global__ void __launch_bounds__(64 * kFarWaves) k_eval_far(EvalArgs<T> a, int far_blocks, int n_eg_tiles,
                                                              int n_nd_tiles) {
    using V = typename V4Of<T>::type;
    __shared__ uint32_t fr[kFarWaves * kFarPts][2][kFarCap];
    __shared__ int2 runs[kFarWaves * kFarPts][kFarRuns];
    if ((int)blockIdx.x >= far_blocks) {
        const int b = (int)blockIdx.x - far_blocks;
        if (b < n_eg_tiles)
            eval_edges_tile<T>(a, b);
        else
            eval_nodes_group<T>(a, (b - n_eg_tiles) * kNodeGroups + (int)threadIdx.x / kNodeTile,
                                (int)threadIdx.x % kNodeTile, n_nd_tiles);
        return;
    }
    const int lane = (int)threadIdx.x & 63;
    const int gl = lane & (kFarGroup - 1);
    const int g = (int)threadIdx.x / kFarGroup;    // group slot in the block
    const int nfar = (int)min((int64_t)*a.far_count, a.Ntot);
    const V* src = a.src_override ? (const V*)a.src_override : (const V*)a.src;
    const int stride = far_blocks * kFarWaves * kFarPts;
    for (int h = (int)blockIdx.x * kFarWaves * kFarPts + g; h < nfar; h += stride) {
        const int2 e = a.far_list[h];
        const int i = e.x, p = e.y;
        const PairDyn dy = a.dyn[p];
        const PairInfo pi = a.info[p];
        const int* cells = a.grid + pi.grid_off;
        const V* tg = a.tgt + pi.tgt_off;
        const V v = src[i];
        T vx, vy, vz, sx, sy, sz, sw1;
        warp_point<T, V>(a, a.X[dy.eval_x], i, v, vx, vy, vz, sx, sy, sz, sw1);
        long long n_box = 0, n_pts = 0, n_cells = 0;
        // the seed: the budgeted search's best
        const int seed = a.far_seed[i];
        T bd = nn_inf<T>();
        int bid = INT_MAX, bpos = -1;
        if (seed >= 0) {
            const V u = tg[seed];
            bd = sq3(u.x - vx, u.y - vy, u.z - vz);
            bid = (int)u.w;
            bpos = seed;
        }
        const int G = pi.grid_bits;
        const T pad = (T)pi.gpad;
        const T ax = ((T)pi.glo[0] - pad) - vx, bx = vx - ((T)pi.glo[0] + pad);
        const T ay = ((T)pi.glo[1] - pad) - vy, by = vy - ((T)pi.glo[1] + pad);
        const T az = ((T)pi.glo[2] - pad) - vz, bz = vz - ((T)pi.glo[2] + pad);
        // start cell: the deepest holding the seed's box (as oct_search)
        int l0 = 0;
        uint32_t m0 = 0;
        if (bd < nn_inf<T>()) {
            const T r = sqrt(bd) * T(1.00001) + pad;
            int lz = G - 1;
            uint32_t lo3[3];
            const T qv[3] = {vx, vy, vz};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T gl0 = (T)pi.glo[c], gs = (T)pi.gscale[c];
                T lo = (qv[c] - r - gl0) * gs, hi = (qv[c] + r - gl0) * gs;
                lo = fmin(fmax(lo, T(0)), T(1023));
                hi = fmin(fmax(hi, T(0)), T(1023));
                lo3[c] = (uint32_t)floor(lo);
                const uint32_t x = lo3[c] ^ (uint32_t)floor(hi);
                const int common = x == 0 ? 10 : __builtin_clz(x) - 22;
                lz = common < lz ? common : lz;
            }
            l0 = lz < 0 ? 0 : lz;
            for (int b = l0 - 1; b >= 0; --b)
                m0 = (m0 << 3) | ((((lo3[0] >> (10 - l0)) >> b) & 1u) << 2) |
                     ((((lo3[1] >> (10 - l0)) >> b) & 1u) << 1) | (((lo3[2] >> (10 - l0)) >> b) & 1u);
        }
        if (gl == 0) fr[g][0][0] = m0;
        wave_sync();
        int n = 1, cur = 0;
        bool overflow = false;
        for (int l = l0; l < G && n > 0 && !overflow; ++l) {
            const T sxl = ldexp((T)pi.cs[0], -(l + 1)), syl = ldexp((T)pi.cs[1], -(l + 1)),
                    szl = ldexp((T)pi.cs[2], -(l + 1));
            const int64_t toff = oct_level_off(l + 1);
            const bool leaves = l == G - 1;
            int nn = 0;
            for (int base = 0; base < n && !overflow; base += kFarGroup) {
                const int k = base + gl;
                uint32_t keep = 0, m = 0;
                int st[9];
                if (k < n) {
                    m = fr[g][cur][k];
#pragma unroll
                    for (int q = 0; q < 9; ++q) st[q] = cells[toff + 8 * (int64_t)m + q];
                    const T jx = T(2 * compact3(m >> 2)), jy = T(2 * compact3(m >> 1)), jz = T(2 * compact3(m));
                    const T dx0 = oct_axis(ax, bx, sxl, jx), dx1 = oct_axis(ax, bx, sxl, jx + T(1));
                    const T dy0 = oct_axis(ay, by, syl, jy), dy1 = oct_axis(ay, by, syl, jy + T(1));
                    const T dz0 = oct_axis(az, bz, szl, jz), dz1 = oct_axis(az, bz, szl, jz + T(1));
                    const T z0 = dz0 * dz0, z1 = dz1 * dz1;
                    const T y00 = (T)fma(dy0, dy0, z0), y01 = (T)fma(dy0, dy0, z1), y10 = (T)fma(dy1, dy1, z0),
                            y11 = (T)fma(dy1, dy1, z1);
                    const T cb[8] = {(T)fma(dx0, dx0, y00), (T)fma(dx0, dx0, y01), (T)fma(dx0, dx0, y10),
                                     (T)fma(dx0, dx0, y11), (T)fma(dx1, dx1, y00), (T)fma(dx1, dx1, y01),
                                     (T)fma(dx1, dx1, y10), (T)fma(dx1, dx1, y11)};
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        keep |= (st[c + 1] > st[c] && cb[c] <= bd ? 1u : 0u) << c;
                        if constexpr (COUNT) n_box += st[c + 1] > st[c] ? 1 : 0;
                    }
                    if constexpr (COUNT) n_cells += 1;
                }
                int tot = 0;
                const int off = group_excl_scan((int)__popc(keep), gl, tot);
                if (!leaves) {
                    if (nn + tot > kFarCap) {
                        overflow = true;   // uniform over the group
                        break;
                    }
                    int o = nn + off;
                    for (uint32_t km = keep; km; km &= km - 1) fr[g][cur ^ 1][o++] = 8 * m + (uint32_t)__builtin_ctz(km);
                    nn += tot;
                } else {
                    // the kept leaves' runs, then their targets across the group
                    int o = off;
                    for (uint32_t km = keep; km; km &= km - 1) {
                        const int c = __builtin_ctz(km);
                        int s0 = st[0], s1 = st[1];
#pragma unroll
                        for (int q = 1; q < 8; ++q)
                            if (c == q) {
                                s0 = st[q];
                                s1 = st[q + 1];
                            }
                        runs[g][o++] = make_int2(s0, s1);
                    }
                    wave_sync();
                    // each lane scans whole runs, four targets per round (the
                    // loads issued together; indices past a run repeat its
                    // last target, whose second visit changes nothing)
                    T ld = nn_inf<T>();
                    int lid = INT_MAX, lpos = -1;
                    for (int r = gl; r < tot; r += kFarGroup) {
                        const int s0 = runs[g][r].x, s1 = runs[g][r].y;
                        if constexpr (COUNT) n_pts += s1 - s0;
                        for (int t = s0; t < s1; t += 4) {
                            const int t1 = min(t + 1, s1 - 1), t2 = min(t + 2, s1 - 1), t3 = min(t + 3, s1 - 1);
                            const V u0 = tg[t], u1 = tg[t1], u2 = tg[t2], u3 = tg[t3];
                            const T d0 = sq3(u0.x - vx, u0.y - vy, u0.z - vz);
                            const T d1 = sq3(u1.x - vx, u1.y - vy, u1.z - vz);
                            const T d2 = sq3(u2.x - vx, u2.y - vy, u2.z - vz);
                            const T d3 = sq3(u3.x - vx, u3.y - vy, u3.z - vz);
                            const int i0 = (int)u0.w, i1 = (int)u1.w, i2 = (int)u2.w, i3 = (int)u3.w;
                            if (d0 < ld || (d0 == ld && i0 < lid)) {
                                ld = d0;
                                lid = i0;
                                lpos = t;
                            }
                            if (d1 < ld || (d1 == ld && i1 < lid)) {
                                ld = d1;
                                lid = i1;
                                lpos = t1;
                            }
                            if (d2 < ld || (d2 == ld && i2 < lid)) {
                                ld = d2;
                                lid = i2;
                                lpos = t2;
                            }
                            if (d3 < ld || (d3 == ld && i3 < lid)) {
                                ld = d3;
                                lid = i3;
                                lpos = t3;
                            }
                        }
                    }
                    // group minimum of (distance, user index)
#pragma unroll
                    for (int o2 = kFarGroup / 2; o2 > 0; o2 >>= 1) {
                        const T od = __shfl_xor(ld, o2, kFarGroup);
                        const int oid = __shfl_xor(lid, o2, kFarGroup), opos = __shfl_xor(lpos, o2, kFarGroup);
                        if (od < ld || (od == ld && oid < lid)) {
                            ld = od;
                            lid = oid;
                            lpos = opos;
                        }
                    }
                    if (ld < bd || (ld == bd && lid < bid)) {
                        bd = ld;
                        bid = lid;
                        bpos = lpos;
                    }
                    wave_sync();
                }
            }
            wave_sync();
            n = nn;
            cur ^= 1;
        }
        if (overflow) {
            // one lane finishes the search from the best so far
            int fp = bpos;
            T fd = bd;
            if (gl == 0) oct_search<T, V, false>(pi, cells, cells, a.tgt, vx, vy, vz, bpos, fp, fd);
            bpos = __shfl(fp, 0, kFarGroup);
        }
        if (bpos < 0) bpos = 0;   // a non-finite query matches nothing
        if (gl == 0) {
            finish_point<T, V>(a, dy, pi, i, v, vx, vy, vz, sx, sy, sz, sw1, bpos);
            V vh;
            vh.x = vx;
            vh.y = vy;
            vh.z = vz;
            vh.w = 0;
            a.vhat[dy.eval_dst][i] = vh;   // after the displacement has read set cur
        }
        if constexpr (COUNT) {
            // the group's work into tile 0's counters (totals over tiles are reported)
            for (int o2 = kFarGroup / 2; o2 > 0; o2 >>= 1) {
                n_box += __shfl_xor(n_box, o2, kFarGroup);
                n_pts += __shfl_xor(n_pts, o2, kFarGroup);
                n_cells += __shfl_xor(n_cells, o2, kFarGroup);
            }
            if (gl == 0) {
                atomicAdd((unsigned long long*)&a.nn_work[1], (unsigned long long)n_box);
                atomicAdd((unsigned long long*)&a.nn_work[2], (unsigned long long)n_pts);
                atomicAdd((unsigned long long*)&a.nn_work[3], (unsigned long long)n_cells);
            }
        }
    }
}

// Tile sums of the points' energy terms and displacements (the same tree as
// a fused per-tile sum), after every point is finished; resets the count of
// deferred points for the next evaluation.
template <typename T>
__global__ void __launch_bounds__(kPointTile) k_eval_sums(EvalArgs<T> a) {
    __shared__ T sh[kPointTile];
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.far_count = 0;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int4 td = a.pt_tiles[tile];
    if (!(a.dyn[td.x].flags & PF_EVAL)) return;        // uniform over the block
    const int i = td.y + (int)threadIdx.x;
    const T psi = i < td.z ? a.pt_psi[i] : T(0);
    const T disp = i < td.z ? a.pt_disp[i] : T(0);
    const T tot = block_sum<T, kPointTile>(psi, sh);
    const T mx = block_max<T, kPointTile>(disp, sh);
    if (threadIdx.x == 0) {
        a.pt_part[tile] = (double)tot;
        a.pt_max[tile] = (double)mx;
    }
}

// Per directed node pair (a, b): D_ab of Eq. (7) (transform of b applied at
// p_a), Welsch value and weight (Eqs. 9, 14).  Evaluated as
// r ((A_b - I)(p_a - p_b) + t_b - t_a), equal to Eq. (7) and free of the
// cancellation between p_a and p_b.
// (one block of kEdgeTile threads per edge tile)
template <typename T>
__device__ void eval_edges_tile(const EvalArgs<T>& a, int tile) {
    using V = typename V4Of<T>::type;
    __shared__ T sh[kEdgeTile];
    const int4 td = a.eg_tiles[tile];
    const int p = td.x;
    const PairDyn dy = a.dyn[p];
    if (!(dy.flags & PF_EVAL)) return;
    const int e = td.y + (int)threadIdx.x;
    const T* X = a.X[dy.eval_x];
    T psi = 0;
    if (e < td.z) {
        const int ia = a.adj_row[e], ib = a.adj_nbr[e];
        const T r = a.adj_r[e];
        const V pa = a.nodes[ia], pb = a.nodes[ib];
        const T* Xa = X + 12 * (size_t)ia;
        const T* Xb = X + 12 * (size_t)ib;
        const T dx = pa.x - pb.x, dyy = pa.y - pb.y, dz = pa.z - pb.z;
        const T Dx = r * (dx * (Xb[0] - T(1)) + dyy * Xb[3] + dz * Xb[6] + (Xb[9] - Xa[9]));
        const T Dy = r * (dx * Xb[1] + dyy * (Xb[4] - T(1)) + dz * Xb[7] + (Xb[10] - Xa[10]));
        const T Dz = r * (dx * Xb[2] + dyy * Xb[5] + dz * (Xb[8] - T(1)) + (Xb[11] - Xa[11]));
        const T D2 = sq3(Dx, Dy, Dz);
        if (dy.robust == AMM_ROBUST_WELSCH) {
            const T inv = T(1) / (T(2) * (T)dy.nu_r * (T)dy.nu_r);
            psi = -expm1(-D2 * inv);
            a.wr[dy.eval_dst][e] = exp(-D2 * inv) * inv;
        } else {
            // both squared-norm variants: plain |D|^2, unit weight
            psi = D2;
            a.wr[dy.eval_dst][e] = T(1);
        }
        V D;
        D.x = Dx;
        D.y = Dy;
        D.z = Dz;
        D.w = D2;
        a.Dres[dy.eval_dst][e] = D;
    }
    const T tot = block_sum<T, kEdgeTile>(psi, sh);
    if (threadIdx.x == 0) a.eg_part[tile] = (double)tot;
}

template <typename T>
__global__ void __launch_bounds__(kEdgeTile) k_eval_edges(EvalArgs<T> a) {
    eval_edges_tile<T>(a, (int)blockIdx.x);
}

// Closest rotation to a 3x3 matrix A (rotation term, Sec. 3.2): one-sided
// Jacobi SVD (Hestenes) of A, U completed to a right-handed frame, then
// R = U diag(1, 1, det V) V^T, which equals U' diag(1,1,det(U'V^T)) V^T for
// any SVD A = U' S V^T.  Returns |A - R|_F^2.
template <typename T>
__device__ T proj_rot(const T A[3][3], T R[3][3]) {
    T B[3][3], Vm[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            B[r][c] = A[r][c];
            Vm[r][c] = (r == c) ? T(1) : T(0);
        }
    const T tol = sizeof(T) == 4 ? T(1e-7) : T(1e-15);
    for (int sweep = 0; sweep < 12; ++sweep) {
        bool rotated = false;
        for (int pq = 0; pq < 3; ++pq) {
            const int pp = pq == 2 ? 1 : 0;
            const int qq = pq == 0 ? 1 : 2;
            T al = 0, be = 0, ga = 0;
            for (int r = 0; r < 3; ++r) {
                al += B[r][pp] * B[r][pp];
                be += B[r][qq] * B[r][qq];
                ga += B[r][pp] * B[r][qq];
            }
            if (fabs(ga) <= tol * sqrt(al * be) || ga == T(0)) continue;
            rotated = true;
            const T zeta = (be - al) / (T(2) * ga);
            const T t = (zeta >= 0 ? T(1) : T(-1)) / (fabs(zeta) + sqrt(T(1) + zeta * zeta));
            const T c = T(1) / sqrt(T(1) + t * t);
            const T s = c * t;
            for (int r = 0; r < 3; ++r) {
                const T bp = B[r][pp], bq = B[r][qq];
                B[r][pp] = c * bp - s * bq;
                B[r][qq] = s * bp + c * bq;
                const T vp = Vm[r][pp], vq = Vm[r][qq];
                Vm[r][pp] = c * vp - s * vq;
                Vm[r][qq] = s * vp + c * vq;
            }
        }
        if (!rotated) break;
    }
    T sig[3];
    int ord[3] = {0, 1, 2};
    for (int c = 0; c < 3; ++c) sig[c] = sqrt(B[0][c] * B[0][c] + B[1][c] * B[1][c] + B[2][c] * B[2][c]);
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2 - x; ++y)
            if (sig[ord[y]] < sig[ord[y + 1]]) {
                int tmp = ord[y];
                ord[y] = ord[y + 1];
                ord[y + 1] = tmp;
            }
    T U[3][3], V[3][3];
    for (int c = 0; c < 3; ++c)
        for (int r = 0; r < 3; ++r) V[r][c] = Vm[r][ord[c]];
    // u0, u1 by Gram-Schmidt of the two largest columns, u2 = u0 x u1
    T u0[3], u1[3];
    {
        const T s0 = sig[ord[0]];
        if (s0 > T(0)) {
            for (int r = 0; r < 3; ++r) u0[r] = B[r][ord[0]] / s0;
        } else {
            u0[0] = 1;
            u0[1] = 0;
            u0[2] = 0;
        }
        T b1[3];
        for (int r = 0; r < 3; ++r) b1[r] = B[r][ord[1]];
        const T dp = u0[0] * b1[0] + u0[1] * b1[1] + u0[2] * b1[2];
        for (int r = 0; r < 3; ++r) b1[r] -= dp * u0[r];
        T n1 = sqrt(b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2]);
        if (!(n1 > T(0))) {
            // any unit vector orthogonal to u0
            const T ax = fabs(u0[0]) < T(0.9) ? T(1) : T(0);
            const T ay = T(1) - ax;
            b1[0] = ax - u0[0] * (u0[0] * ax + u0[1] * ay);
            b1[1] = ay - u0[1] * (u0[0] * ax + u0[1] * ay);
            b1[2] = -u0[2] * (u0[0] * ax + u0[1] * ay);
            n1 = sqrt(b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2]);
        }
        for (int r = 0; r < 3; ++r) u1[r] = b1[r] / n1;
    }
    for (int r = 0; r < 3; ++r) {
        U[r][0] = u0[r];
        U[r][1] = u1[r];
    }
    U[0][2] = u0[1] * u1[2] - u0[2] * u1[1];
    U[1][2] = u0[2] * u1[0] - u0[0] * u1[2];
    U[2][2] = u0[0] * u1[1] - u0[1] * u1[0];
    const T detV = V[0][0] * (V[1][1] * V[2][2] - V[1][2] * V[2][1]) -
                   V[0][1] * (V[1][0] * V[2][2] - V[1][2] * V[2][0]) +
                   V[0][2] * (V[1][0] * V[2][1] - V[1][1] * V[2][0]);
    const T d3 = detV >= 0 ? T(1) : T(-1);
    T e = 0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            R[r][c] = U[r][0] * V[c][0] + U[r][1] * V[c][1] + d3 * U[r][2] * V[c][2];
            const T dd = A[r][c] - R[r][c];
            e += dd * dd;
        }
    return e;
}

// Per node: closest rotation and |A_j - proj(A_j)|_F^2, in float64 for both
// arithmetics (A_j is exact in float64): A_j lies within ~1e-3 of a rotation,
// so float32 rounding of proj(A_j) would be amplified in the squared
// difference.  Stores proj(A_j) - A_j (small, accurate in T) for the
// assembly and the gradient.
template <typename T>
__global__ void __launch_bounds__(kNodeTile) k_eval_nodes(EvalArgs<T> a) {
    __shared__ double sh[kNodeTile];
    const int tile = blockIdx.x;
    const int4 td = a.nd_tiles[tile];
    const int p = td.x;
    const PairDyn dy = a.dyn[p];
    if (!(dy.flags & PF_EVAL)) return;
    const int j = td.y + (int)threadIdx.x;
    const T* X = a.X[dy.eval_x];
    double er = 0;
    if (j < td.z) {
        double A[3][3], R[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) A[c][r] = (double)X[12 * (size_t)j + 3 * r + c];
        er = proj_rot<double>(A, R);
        T* Ro = a.R[dy.eval_dst] + 9 * (size_t)j;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Ro[3 * r + c] = (T)(R[r][c] - A[r][c]);
    }
    const double tot = block_sum<double, kNodeTile>(er, sh);
    if (threadIdx.x == 0) a.nd_part[tile] = tot;
}

// k_eval_nodes for one node tile on a group of kNodeTile lanes of a wider
// block (lane gl of the group on node gl of the tile): the same terms, and
// the tile's sum by shuffles in block_sum's order (lane i adds lane i + 8,
// then i + 4, i + 2, i + 1), so nd_part is bitwise the same.
template <typename T>
__device__ void eval_nodes_group(const EvalArgs<T>& a, int tile, int gl, int n_nd_tiles) {
    static_assert(kNodeTile == 16, "the shuffle tree below is written for 16 lanes");
    if (tile >= n_nd_tiles) return;   // uniform over the group
    const int4 td = a.nd_tiles[tile];
    const PairDyn dy = a.dyn[td.x];
    if (!(dy.flags & PF_EVAL)) return;
    const int j = td.y + gl;
    const T* X = a.X[dy.eval_x];
    double er = 0;
    if (j < td.z) {
        double A[3][3], R[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) A[c][r] = (double)X[12 * (size_t)j + 3 * r + c];
        er = proj_rot<double>(A, R);
        T* Ro = a.R[dy.eval_dst] + 9 * (size_t)j;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Ro[3 * r + c] = (T)(R[r][c] - A[r][c]);
    }
    er += __shfl_down(er, 8, kNodeTile);
    er += __shfl_down(er, 4, kNodeTile);
    er += __shfl_down(er, 2, kNodeTile);
    er += __shfl_down(er, 1, kNodeTile);
    if (gl == 0) a.nd_part[tile] = er;
}

// Per pair: E = E_align + alpha E_reg + beta E_rot (Eq. 4) from the tile
// partials in a fixed order, and the max displacement.
__global__ void __launch_bounds__(64) k_energy_final(FinalArgs a) {
    const int p = blockIdx.x;
    const PairDyn dy = a.dyn[p];
    if (!(dy.flags & PF_EVAL)) return;
    const PairInfo pi = a.info[p];
    double sa = 0, sr = 0, so = 0, mx = 0;
    // unrolled so that several partials are loaded before their (in-order) sum
#pragma unroll 8
    for (int t = threadIdx.x; t < pi.pt_ntile; t += 64) {
        sa += a.pt_part[pi.pt_tile0 + t];
        mx = fmax(mx, a.pt_max[pi.pt_tile0 + t]);
    }
#pragma unroll 4
    for (int t = threadIdx.x; t < pi.eg_ntile; t += 64) sr += a.eg_part[pi.eg_tile0 + t];
#pragma unroll 4
    for (int t = threadIdx.x; t < pi.nd_ntile; t += 64) so += a.nd_part[pi.nd_tile0 + t];
    sa = wave_sum(sa);
    sr = wave_sum(sr);
    so = wave_sum(so);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (threadIdx.x == 0) {
        PairOut& out = a.out[p];
        out.Ea = sa;
        out.Er = sr;
        out.Eo = so;
        out.E = sa + dy.alpha * sr + dy.beta * so;
        out.maxdisp = mx;
    }
}

// ---------------------------------------------------------------- assembly


// The 16 x 16 x 4 matrix-core product used by the assembly, D = A B + C with
// A 16 x 4 and B 4 x 16: lane l supplies A(l % 16, l / 16) and B(l / 16,
// l % 16), and its accumulator value r is D(row(l, r), l % 16).
template <typename T>
struct AsmMfma;
template <>
struct AsmMfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float x, float y, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
    // row stride of the staged columns, 4 words past a multiple of 64: the
    // 16-byte reads of 16 lanes from 16 rows hit distinct banks
    static constexpr int kStride = 68;
};
template <>
struct AsmMfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double x, double y, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int r) { return 4 * r + (l >> 4); }
    static constexpr int kStride = 66;
};

constexpr int kAsmGroup = 32;   // column blocks per pass of the assembly (two 16-column tiles)
// an unused influence slot (column byte 255) lands outside every pass's columns
static_assert(kMaxCols <= (int)kPosUnused + 1 - kAsmGroup, "column bytes of unused slots");
// the staged rows hold 64 points and at least two padding columns (where
// influence slots outside the pass write), and the pass's sums per column
// block (kAsmGroup x 10) fit in the first five moment rows
static_assert(AsmMfma<float>::kStride >= 66 && AsmMfma<double>::kStride >= 66, "padding columns");
static_assert(5 * AsmMfma<float>::kStride >= 10 * kAsmGroup && 5 * AsmMfma<double>::kStride >= 10 * kAsmGroup,
              "per-pass sums in the moment rows");
static_assert(kMaxK <= kAsmGroup, "padding rows of the influence slots");

// Eight consecutive staged values of one row, as 16-byte reads.
__device__ __forceinline__ void asm_load8(const float* r, float (&v)[8]) {
    const float4 x = reinterpret_cast<const float4*>(r)[0], y = reinterpret_cast<const float4*>(r)[1];
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
}
__device__ __forceinline__ void asm_load8(const double* r, double (&v)[8]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const double2 x = reinterpret_cast<const double2*>(r)[u];
        v[2 * u] = x.x;
        v[2 * u + 1] = x.y;
    }
}

// A staged point: loaded for the chunk after the one being multiplied.
template <typename T>
struct AsmPoint {
    using V = typename V4Of<T>::type;
    V v, q, w0, w1;   // point, (e, w_a), influence weights 0-3 and 4-7
};

template <typename T>
__device__ __forceinline__ void asm_gather(const AsmArgs<T>& a, const typename V4Of<T>::type* qw, int ent,
                                           AsmPoint<T>& g) {
    using V = typename V4Of<T>::type;
    if (ent < 0) return;
    const int i = ent >> 3;
    g.v = a.src[i];
    g.q = qw[i];
    const V* wp = reinterpret_cast<const V*>(a.iw_pt + (size_t)kMaxK * i);
    g.w0 = wp[0];
    g.w1 = wp[1];
}

// Row j of K and B (Eq. 21) and of the residual r = B - K X^k, one wave per
// node.  Alignment blocks K_jl = sum_i w_a,i w_ij w_il [v_i - p_j; 1]
// [v_i - p_l; 1]^T are formed as moments anchored at p_j,
// M_jl = sum c_i w_il x x^T with x = [v_i - p_j; 1] and c_i = w_a,i w_ij,
// then shifted: K_jl = M_jl S^T, S = [[I, p_j - p_l], [0, 1]].  The ten
// distinct moments of all column blocks of the row are one product
// W^T Mom over the row's points: W (points x columns) holds w_il in the
// column of each influence l of point i and zero elsewhere, Mom (points x
// 10) holds c_i times the products of the entries of x.  Chunks of 64
// points are staged in LDS (a point per lane) and multiplied on the matrix
// cores, four points per instruction, in a fixed order; rows coupled to
// more than 32 nodes take one pass per 32 columns.  Lanes then own the
// columns of the row and shift, add the edge and rotation blocks
// (Eqs. (7), (14), the matrix H and beta J^T J) and write them.  The
// residual is assembled from the residuals at X^k themselves --
// r = -sum w_a F^T e - alpha sum w_r H^T D + beta J(Z - X^k) -- instead of
// as the difference B - K X^k of two large rounded quantities, so its
// relative accuracy does not degrade as the iteration converges;
// B = r + K X^k.  The inverse of the 4x4 diagonal block (block-Jacobi
// preconditioner) is written alongside.
template <typename T>
__global__ void __launch_bounds__(64) k_assemble(AsmArgs<T> a) {
    using V = typename V4Of<T>::type;
    using M = AsmMfma<T>;
    using acc_t = typename M::acc_t;
    __shared__ int scol[kMaxCols];                             // the row's column node ids (sorted)
    __shared__ __align__(16) T swT[kAsmGroup][M::kStride];     // W^T of the staged points
    // Mom^T of the staged points in rows 0-9, zero rows 10-15 (the product's
    // unused moment columns); after a pass's products rows 0-4 hold its sums
    // per column block (sacc)
    __shared__ __align__(16) T smomT[16][M::kStride];
    T* const sacc = &smomT[0][0];
    // neighbouring nodes share most of their points: keep them on one XCD
    const int j = xcd_tile(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    const int lr = lane & 15, lq = lane >> 4;
    const int p = a.node_pair[j];
    const PairDyn dy = a.dyn[p];
    if (!(dy.flags & PF_SOLVE)) return;
    const int cur = dy.cur;
    const V* qw = a.qw[cur];
    const T* wr = a.wr[cur];
    const V* Dr = a.Dres[cur];
    const V pj = a.nodes[j];
    const int kb = a.K_ptr[j], ke = a.K_ptr[j + 1];
    const int ncol = ke - kb;
    const int k = a.k;
    const T alpha = (T)dy.alpha, beta = (T)dy.beta;
    const int ab = a.adj_ptr[j], ae = a.adj_ptr[j + 1];
    const T* Xk = a.X[cur];
    const int e0 = a.pj_ptr[j], e1 = a.pj_ptr[j + 1];
    // the first two chunks' entries and the first chunk's points, then every
    // chunk loads the next one's while it is multiplied
    int entA = -1, entB = -1;
    uint64_t posA = ~0ull, posB = ~0ull;   // ~0: every slot unused
    if (e0 + lane < e1) {
        entA = a.pj_ent[e0 + lane];
        posA = a.pj_pos[e0 + lane];
    }
    if (e0 + 64 + lane < e1) {
        entB = a.pj_ent[e0 + 64 + lane];
        posB = a.pj_pos[e0 + 64 + lane];
    }
    AsmPoint<T> gA = {};
    asm_gather(a, qw, entA, gA);
    for (int c = lane; c < ncol; c += 64) scol[c] = a.K_col[kb + c];
#pragma unroll
    for (int c = 0; c < kAsmGroup; ++c) swT[c][lane] = 0;   // each lane keeps its own point's column zero
#pragma unroll
    for (int m = 10; m < 16; ++m) smomT[m][lane] = 0;

    // Edge terms of the row, summed over the wave: the diagonal block's sum
    // over edges (j, l2) of the entry l2->j's weight times [p_l2 - p_j; 1]
    // [p_l2 - p_j; 1]^T plus the entry j->l2's weight in its last element
    // (ed, upper triangle row-major), and the edges' part of -r (re):
    // -f1 [p_l2 - p_j; 1] D_l2j^T, and f2 D_jl2^T in the last row.
    T ed[10], re[12];
    auto add_edge = [&](T rr, T we, T wv, V q2, V D1, V D2) {
        const T om_e = alpha * we * rr * rr;
        const T om_r = alpha * wv * rr * rr;
        const T x[4] = {q2.x - pj.x, q2.y - pj.y, q2.z - pj.z, T(1)};
        int m = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c2 = r; c2 < 4; ++c2) ed[m++] += om_r * x[r] * x[c2];
        ed[9] += om_e;
        const T f1 = alpha * wv * rr;
        const T f2 = alpha * we * rr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            re[3 * r + 0] -= f1 * x[r] * D1.x;
            re[3 * r + 1] -= f1 * x[r] * D1.y;
            re[3 * r + 2] -= f1 * x[r] * D1.z;
        }
        re[9] += f2 * D2.x;
        re[10] += f2 * D2.y;
        re[11] += f2 * D2.z;
    };

    for (int m = 0; m < 10; ++m) ed[m] = 0;
    for (int m = 0; m < 12; ++m) re[m] = 0;
    for (int e = ab + lane; e < ae; e += 64) {
        const int rev = a.adj_rev[e];
        add_edge(a.adj_r[e], wr[e], wr[rev], a.nodes[a.adj_nbr[e]], Dr[rev], Dr[e]);
    }
#pragma unroll
    for (int m = 0; m < 10; ++m) ed[m] = wave_sum(ed[m]);
#pragma unroll
    for (int m = 0; m < 12; ++m) re[m] = wave_sum(re[m]);

    T racc[12];
#pragma unroll
    for (int m = 0; m < 12; ++m) racc[m] = 0;
    T kx[12];
#pragma unroll
    for (int m = 0; m < 12; ++m) kx[m] = 0;
    __syncthreads();
    for (int g0 = 0; g0 < ncol; g0 += kAsmGroup) {
        // this lane's column block of the pass: its node, edge weights and X
        const int cp = g0 + lane;
        const bool own = lane < kAsmGroup && cp < ncol;
        int l = 0;
        V pl = {};
        T om_e = 0, om_r = 0;
        bool edge = false;
        T Xl[12];
#pragma unroll
        for (int m = 0; m < 12; ++m) Xl[m] = 0;
        if (own) {
            l = scol[cp];
            pl = a.nodes[l];
            const int adj = a.K_adj[kb + cp];
            if (adj >= 0) {
                // D_jl (entry j->l, transform of l) and D_lj (entry l->j, transform of j)
                const int rev = a.adj_rev[adj];
                const T rr = a.adj_r[adj];
                om_e = alpha * wr[adj] * rr * rr;
                om_r = alpha * wr[rev] * rr * rr;
                edge = true;
            }
            const T* xp = Xk + 12 * (size_t)l;
#pragma unroll
            for (int m = 0; m < 12; ++m) Xl[m] = xp[m];
        }
        if (g0 > 0) {
            // a later pass reads the row's entries again from the start
            entA = entB = -1;
            posA = posB = ~0ull;
            if (e0 + lane < e1) {
                entA = a.pj_ent[e0 + lane];
                posA = a.pj_pos[e0 + lane];
            }
            if (e0 + 64 + lane < e1) {
                entB = a.pj_ent[e0 + 64 + lane];
                posB = a.pj_pos[e0 + 64 + lane];
            }
            asm_gather(a, qw, entA, gA);
        }
        acc_t acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
        for (int base = e0; base < e1; base += 64) {
            // this chunk's entry and point; then the next chunk's loads
            const int ent = entA;
            const uint64_t pos = posA;
            const AsmPoint<T> g = gA;
            asm_gather(a, qw, entB, gA);
            entA = entB;
            posA = posB;
            entB = -1;
            posB = ~0ull;
            if (base + 128 + lane < e1) {
                entB = a.pj_ent[base + 128 + lane];
                posB = a.pj_pos[base + 128 + lane];
            }
            T mom[10];
#pragma unroll
            for (int m = 0; m < 10; ++m) mom[m] = 0;
            const T wv[kMaxK] = {g.w0.x, g.w0.y, g.w0.z, g.w0.w, g.w1.x, g.w1.y, g.w1.z, g.w1.w};
            if (ent >= 0) {
                const int s = ent & 7;
                T ws = wv[0];
#pragma unroll
                for (int b = 1; b < kMaxK; ++b) ws = s == b ? wv[b] : ws;
                const T c = g.q.w * ws;
                const T dx = g.v.x - pj.x, dyy = g.v.y - pj.y, dz = g.v.z - pj.z;
                mom[0] = c * dx * dx;
                mom[1] = c * dx * dyy;
                mom[2] = c * dx * dz;
                mom[3] = c * dx;
                mom[4] = c * dyy * dyy;
                mom[5] = c * dyy * dz;
                mom[6] = c * dyy;
                mom[7] = c * dz * dz;
                mom[8] = c * dz;
                mom[9] = c;
                if (g0 == 0) {
                    // alignment part of -r: c [v_i - p_j; 1] e_i^T
                    const T ax = c * dx, ay = c * dyy, az = c * dz;
                    racc[0] += ax * g.q.x;
                    racc[1] += ax * g.q.y;
                    racc[2] += ax * g.q.z;
                    racc[3] += ay * g.q.x;
                    racc[4] += ay * g.q.y;
                    racc[5] += ay * g.q.z;
                    racc[6] += az * g.q.x;
                    racc[7] += az * g.q.y;
                    racc[8] += az * g.q.z;
                    racc[9] += c * g.q.x;
                    racc[10] += c * g.q.y;
                    racc[11] += c * g.q.z;
                }
            }
#pragma unroll
            for (int m = 0; m < 10; ++m) smomT[m][lane] = mom[m];
            // an influence's column within this pass; slots outside it (unused
            // ones have byte 255) write a padding column past the 64 points,
            // which is never read
            T* const swf = &swT[0][0];
            int woff[kMaxK];
#pragma unroll
            for (int b = 0; b < kMaxK; ++b) {
                const unsigned cb = ((unsigned)(pos >> (8 * b)) & 255u) - (unsigned)g0;
                const bool in = b < k && cb < (unsigned)kAsmGroup;
                woff[b] = in ? (int)cb * M::kStride + lane : b * M::kStride + 64 + (lane & 1);
                swf[woff[b]] = wv[b];
            }
            __syncthreads();
            // step u multiplies the staged points u, 16 + u, 32 + u and 48 + u
            // (lane group lq supplies point 16 lq + u), in a fixed order; points
            // past the row's end are zero.  Both tiles are multiplied whatever
            // the row's width (a second tile past the row's columns multiplies
            // zero rows): the products run unconditionally, with no branch
            // around the matrix-core accumulators, which this compiler has
            // been seen to get wrong.
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                T bv[8], a0[8], a1[8];
                asm_load8(smomT[lr] + 16 * lq + 8 * h, bv);
                asm_load8(swT[lr] + 16 * lq + 8 * h, a0);
                asm_load8(swT[16 + lr] + 16 * lq + 8 * h, a1);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    acc0 = M::mma(a0[u], bv[u], acc0);
                    acc1 = M::mma(a1[u], bv[u], acc1);
                }
            }
            __syncthreads();
#pragma unroll
            for (int b = 0; b < kMaxK; ++b) swf[woff[b]] = 0;
        }
        // the pass's moment sums per column block (rows 0-9 of smomT are free:
        // the last products' reads completed before the barrier above)
        if (lr < 10) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sacc[10 * M::row(lane, r) + lr] = acc0[r];
                sacc[10 * (16 + M::row(lane, r)) + lr] = acc1[r];
            }
        }
        __syncthreads();
        if (own) {
            const T* m = sacc + 10 * lane;
            const T S[4][4] = {{m[0], m[1], m[2], m[3]},
                               {m[1], m[4], m[5], m[6]},
                               {m[2], m[5], m[7], m[8]},
                               {m[3], m[6], m[8], m[9]}};
            const T del[3] = {pj.x - pl.x, pj.y - pl.y, pj.z - pl.z};
            T Kb[4][4];
            for (int r = 0; r < 4; ++r) {
                for (int s = 0; s < 3; ++s) Kb[r][s] = S[r][s] + S[r][3] * del[s];
                Kb[r][3] = S[r][3];
            }
            if (edge) {
                const T ext[4] = {-del[0], -del[1], -del[2], T(1)};   // [p_l - p_j; 1]
                const T exj[4] = {del[0], del[1], del[2], T(1)};      // [p_j - p_l; 1]
                for (int r = 0; r < 4; ++r) Kb[r][3] -= om_r * ext[r];
                for (int s = 0; s < 4; ++s) Kb[3][s] -= om_e * exj[s];
            }
            if (l == j) {
                int m2 = 0;
                for (int r = 0; r < 4; ++r)
                    for (int c2 = r; c2 < 4; ++c2) {
                        Kb[r][c2] += ed[m2];
                        if (c2 != r) Kb[c2][r] += ed[m2];
                        ++m2;
                    }
                for (int s = 0; s < 3; ++s) Kb[s][s] += beta;
                spd_inverse4<T>(Kb, a.Dinv + 16 * (size_t)j);
            }
            T* Ko = a.Kval + 16 * (size_t)(kb + cp);
            for (int r = 0; r < 4; ++r)
                for (int s = 0; s < 4; ++s) Ko[4 * r + s] = Kb[r][s];
            // (K X^k)_j contribution of this column block
            for (int r = 0; r < 4; ++r)
                for (int c2 = 0; c2 < 3; ++c2)
                    kx[3 * r + c2] += Kb[r][0] * Xl[c2] + Kb[r][1] * Xl[3 + c2] + Kb[r][2] * Xl[6 + c2] +
                                      Kb[r][3] * Xl[9 + c2];
        }
        __syncthreads();   // rows 0-9 of smomT are staged again by the next pass
    }
#pragma unroll
    for (int m = 0; m < 12; ++m) racc[m] = wave_sum(racc[m]);
#pragma unroll
    for (int m = 0; m < 12; ++m) kx[m] = wave_sum(kx[m]);
    if (lane == 0) {
        T rj[12];
        for (int m2 = 0; m2 < 12; ++m2) rj[m2] = re[m2] - racc[m2];
        // rotation term: beta J (Z - X^k), row r of block j = beta (proj(A_j) - A_j)^T
        const T* Rd = a.R[cur] + 9 * (size_t)j;
        for (int r = 0; r < 3; ++r)
            for (int c2 = 0; c2 < 3; ++c2) rj[3 * r + c2] += beta * Rd[3 * c2 + r];
        T* Ro = a.rvec + 12 * (size_t)j;
        T* Bo = a.B + 12 * (size_t)j;
        for (int m2 = 0; m2 < 12; ++m2) {
            Ro[m2] = rj[m2];
            Bo[m2] = rj[m2] + kx[m2];
        }
    }
}

// ---------------------------------------------------------------- iterative refinement

// res64 = rhs - K x64 in float64 (K, rhs in T, upcast exactly); the T copy of
// res64 is the right-hand side of the next inner solve.  Partials (res,res)
// and (n,n) of the vector n that scales the stopping test.
template <typename T>
__global__ void __launch_bounds__(4 * kNodeTile) k_residual64(CgArgs<T> a, const T* B, const T* Bn,
                                                              const double* x64, T* rhs_out, double* part_rr,
                                                              double* part_bb) {
    __shared__ double sh[4 * kNodeTile];
    const int tile = blockIdx.x;
    const int4 td = a.nd_tiles[tile];
    const int p = td.x;
    if (!(a.dyn[p].flags & PF_SOLVE)) return;
    const int lr = threadIdx.x >> 2, r = threadIdx.x & 3;
    const int j = td.y + lr;
    double rv[3] = {0, 0, 0}, bv[3] = {0, 0, 0};
    if (j < td.z) {
        double acc[3] = {0, 0, 0};
        const int kb = a.K_ptr[j], ke = a.K_ptr[j + 1];
        for (int pos = kb; pos < ke; ++pos) {
            const int l = a.K_col[pos];
            const T* kr = a.Kval + 16 * (size_t)pos + 4 * r;
            const double* xl = x64 + 12 * (size_t)l;
            for (int c = 0; c < 3; ++c)
                acc[c] += (double)kr[0] * xl[c] + (double)kr[1] * xl[3 + c] + (double)kr[2] * xl[6 + c] +
                          (double)kr[3] * xl[9 + c];
        }
        for (int c = 0; c < 3; ++c) {
            const size_t o = 12 * (size_t)j + 3 * r + c;
            bv[c] = (double)Bn[o];
            rv[c] = (double)B[o] - acc[c];
            if (rhs_out) rhs_out[o] = (T)rv[c];
        }
    }
    for (int c = 0; c < 3; ++c) {
        const double s = block_sum<double, 4 * kNodeTile>(rv[c] * rv[c], sh);
        const double s2 = block_sum<double, 4 * kNodeTile>(bv[c] * bv[c], sh);
        if (threadIdx.x == 0) {
            part_rr[3 * tile + c] = s;
            part_bb[3 * tile + c] = s2;
        }
    }
}

// ---------------------------------------------------------------- vector utilities

template <typename T>
__global__ void k_node_vec_op(NodeVecArgs<T> a) {
    // 0: x64 = src_t        1: x64 += src_t       2: dst_t = (T) x64      3: dst_t = src_t
    // 4: x64 = X[cur]       5: X[2] = X[cur]      6: X[1 - cur] = X[2]
    // 7: x64 = 0            8: X[2] = X[cur] + x64   9: X[0] = identity
    const int tile = blockIdx.x;
    const int4 td = a.nd_tiles[tile];
    const PairDyn dy = a.dyn[td.x];
    if (!(dy.flags & a.flag)) return;
    const size_t b0 = 12 * (size_t)td.y, b1 = 12 * (size_t)td.z;
    for (size_t o = b0 + threadIdx.x; o < b1; o += blockDim.x) {
        switch (a.op) {
            case 0: a.x64[o] = (double)a.src_t[o]; break;
            case 1: a.x64[o] += (double)a.src_t[o]; break;
            case 2: a.dst_t[o] = (T)a.x64[o]; break;
            case 3: a.dst_t[o] = a.src_t[o]; break;
            case 4: a.x64[o] = (double)a.X[dy.cur][o]; break;
            case 5: a.X[2][o] = a.X[dy.cur][o]; break;
            case 6: a.X[1 - dy.cur][o] = a.X[2][o]; break;
            case 7: a.x64[o] = 0.0; break;
            case 8: a.X[2][o] = (T)((double)a.X[dy.cur][o] + a.x64[o]); break;
            default: {
                const int m = (int)(o % 12);
                a.X[0][o] = (m == 0 || m == 4 || m == 8) ? T(1) : T(0);
                break;
            }
        }
    }
}

// ---------------------------------------------------------------- Anderson acceleration

// G^(k) = X' = X^k + dX and F^(k) = dX into the ring slot of the newest
// entry; X' also goes to transform set 2.
template <typename T>
__global__ void k_aa_push(AaArgs<T> a) {
    const int tile = blockIdx.x;
    const int4 td = a.nd_tiles[tile];
    const PairDyn& dy = a.dyn[td.x];
    if (!(dy.flags & PF_SOLVE)) return;
    const size_t n12 = 12 * (size_t)a.ntot;
    T* G = a.G + (size_t)dy.aa_slot[0] * n12;
    double* F = a.F + (size_t)dy.aa_slot[0] * n12;
    const T* Xc = a.X[dy.cur];
    const size_t b0 = 12 * (size_t)td.y, b1 = 12 * (size_t)td.z;
    for (size_t o = b0 + threadIdx.x; o < b1; o += blockDim.x) {
        const double dx = a.dx[o];
        const T g = (T)((double)Xc[o] + dx);
        G[o] = g;
        F[o] = dx;
        a.X[2][o] = g;
    }
}

// Tile partials of the Gram matrix dF^T dF and of dF^T F^(k) in float64,
// dF_a = F^(k-a+1) - F^(k-a), a = 1..m_k.
template <typename T>
__global__ void __launch_bounds__(256) k_aa_gram(AaArgs<T> a) {
    __shared__ double sdf[AMM_MAX_AA_M + 1][12 * 32];
    const int tile = blockIdx.x;
    const int4 td = a.nd_tiles[tile];
    const PairDyn& dy = a.dyn[td.x];
    if (!(dy.flags & PF_SOLVE)) return;
    const int mk = dy.aa_mk;
    const int ng = mk * (mk + 1) / 2 + mk;
    const size_t n12 = 12 * (size_t)a.ntot;
    double acc = 0;
    // entry index -> (a, b) of the Gram or the right-hand side
    int ea = 0, eb = 0;
    bool is_rhs = false;
    {
        int t = threadIdx.x, cnt = 0;
        if (t < ng) {
            for (int x = 0; x < mk; ++x)
                for (int y = 0; y <= x; ++y) {
                    if (cnt == t) {
                        ea = x;
                        eb = y;
                    }
                    ++cnt;
                }
            if (t >= cnt) {
                is_rhs = true;
                ea = t - cnt;
            }
        }
    }
    const size_t b0 = 12 * (size_t)td.y, b1 = 12 * (size_t)td.z;
    for (size_t base = b0; base < b1; base += 12 * 32) {
        const int cnt = (int)min((size_t)(12 * 32), b1 - base);
        for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
            const size_t o = base + q;
            const double f0 = (double)a.F[(size_t)dy.aa_slot[0] * n12 + o];
            sdf[mk][q] = f0;
            for (int x = 0; x < mk; ++x) {
                const double fa = (double)a.F[(size_t)dy.aa_slot[x] * n12 + o];
                const double fb = (double)a.F[(size_t)dy.aa_slot[x + 1] * n12 + o];
                sdf[x][q] = fa - fb;
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < ng) {
            const double* va = sdf[ea];
            const double* vb = is_rhs ? sdf[mk] : sdf[eb];
            for (int q = 0; q < cnt; ++q) acc += va[q] * vb[q];
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < ng) a.part[(size_t)tile * kAaParts + threadIdx.x] = acc;
}

// Per pair: Gram matrix from the tile partials (one lane per entry, tiles
// in order), Cholesky in float64; a pivot <= 1e-14 * max diag falls back to
// theta = 0 (plain MM step).  The factorization is unrolled over the
// largest window with compile-time indices, so it stays in registers.
__global__ void __launch_bounds__(512) k_aa_solve(AaSolveArgs a) {
    constexpr int M = AMM_MAX_AA_M;
    constexpr int NG = 8;    // tile groups
    __shared__ double v[kAaParts];
    __shared__ double vg[NG][kAaParts];
    const int p = blockIdx.x;
    const PairDyn dy = a.dyn[p];
    if (!(dy.flags & PF_SOLVE)) return;
    PairOut& out = a.out[p];
    const int mk = dy.aa_mk;
    const PairInfo pi = a.info[p];
    const int ng = mk * (mk + 1) / 2 + mk;
    // entry g of group grp sums tiles grp, grp + NG, ...; the groups are then
    // added in order
    for (int e = threadIdx.x; e < NG * kAaParts; e += 512) {
        const int grp = e / kAaParts, g = e - grp * kAaParts;
        double s = 0;
        // unrolled so that several partials are loaded before their (in-order) sum
        if (g < ng)
#pragma unroll 8
            for (int t = grp; t < pi.nd_ntile; t += NG) s += a.part[(size_t)(pi.nd_tile0 + t) * kAaParts + g];
        vg[grp][g] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < ng) {
        double s = 0;
        for (int grp = 0; grp < NG; ++grp) s += vg[grp][threadIdx.x];
        v[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int x = 0; x < M; ++x) out.theta[x] = 0;
    out.aa_used = 0;
    if (mk == 0) return;
    // packed lower triangle: G[x][y] (y <= x) = v[x (x + 1) / 2 + y]; rhs = v[mk(mk+1)/2 + x]
    double dmax = 0;
#pragma unroll
    for (int x = 0; x < M; ++x)
        if (x < mk) dmax = fmax(dmax, v[x * (x + 1) / 2 + x]);
    const double tol = 1e-14 * dmax;
    double L[M][M];
    bool ok = true;
#pragma unroll
    for (int jj = 0; jj < M; ++jj) {
        if (jj < mk) {
            double piv = v[jj * (jj + 1) / 2 + jj];
#pragma unroll
            for (int q = 0; q < jj; ++q) piv -= L[jj][q] * L[jj][q];
            ok = ok && piv > tol;
            L[jj][jj] = sqrt(fmax(piv, 1e-300));
#pragma unroll
            for (int ii = jj + 1; ii < M; ++ii) {
                if (ii < mk) {
                    double sv = v[ii * (ii + 1) / 2 + jj];
#pragma unroll
                    for (int q = 0; q < jj; ++q) sv -= L[ii][q] * L[jj][q];
                    L[ii][jj] = sv / L[jj][jj];
                }
            }
        }
    }
    if (!ok) return;
    const int r0 = mk * (mk + 1) / 2;
    double y[M], th[M];
#pragma unroll
    for (int ii = 0; ii < M; ++ii) {
        if (ii < mk) {
            double sv = v[r0 + ii];
#pragma unroll
            for (int q = 0; q < ii; ++q) sv -= L[ii][q] * y[q];
            y[ii] = sv / L[ii][ii];
        }
    }
#pragma unroll
    for (int ii = M - 1; ii >= 0; --ii) {
        if (ii < mk) {
            double sv = y[ii];
#pragma unroll
            for (int q = ii + 1; q < M; ++q)
                if (q < mk) sv -= L[q][ii] * th[q];
            th[ii] = sv / L[ii][ii];
        }
    }
#pragma unroll
    for (int x = 0; x < M; ++x)
        if (x < mk) out.theta[x] = th[x];
    out.aa_used = 1;
}

// X_AA = G^(k) - sum_a theta_a (G^(k-a+1) - G^(k-a)) (Eq. 23) into the
// candidate transform set; equals G^(k) when Anderson is not used.
template <typename T>
__global__ void k_aa_mix(AaArgs<T> a) {
    const int tile = blockIdx.x;
    const int4 td = a.nd_tiles[tile];
    const int p = td.x;
    const PairDyn& dy = a.dyn[p];
    if (!(dy.flags & PF_SOLVE)) return;
    const PairOut& out = a.out[p];
    const bool used = out.aa_used != 0;
    const int mk = dy.aa_mk;
    const size_t n12 = 12 * (size_t)a.ntot;
    T* Xc = a.X[1 - dy.cur];
    const size_t b0 = 12 * (size_t)td.y, b1 = 12 * (size_t)td.z;
    for (size_t o = b0 + threadIdx.x; o < b1; o += blockDim.x) {
        double g = (double)a.G[(size_t)dy.aa_slot[0] * n12 + o];
        if (used) {
            for (int x = 0; x < mk; ++x) {
                const double ga = (double)a.G[(size_t)dy.aa_slot[x] * n12 + o];
                const double gb = (double)a.G[(size_t)dy.aa_slot[x + 1] * n12 + o];
                g -= out.theta[x] * (ga - gb);
            }
            Xc[o] = (T)g;
        } else {
            Xc[o] = a.X[2][o];
        }
    }
}

// ---------------------------------------------------------------- gradient

// Per point: g_i = dE/dv_hat_i = exp(-d^2/(2 nu_a^2)) (v_hat_i - u_rho(i)) / nu_a^2
// and dE/dv_i = sum_j w_ij A_j^T g_i (graph frozen).
template <typename T>
__global__ void __launch_bounds__(kPointTile) k_grad_points(GradArgs<T> a) {
    using V = typename V4Of<T>::type;
    const int tile = blockIdx.x;
    const int4 td = a.pt_tiles[tile];
    const int p = td.x;
    const PairDyn dy = a.dyn[p];
    if (!(dy.flags & PF_EVAL)) return;
    const int i = td.y + (int)threadIdx.x;
    if (i >= td.z) return;
    const int set = dy.eval_dst;
    const V e = a.qw[set][i];   // (v_hat_i - u_rho(i), w_a,i = exp(-d^2/(2 nu^2)) / (2 nu^2))
    const T f = T(2) * e.w;
    V g;
    g.x = f * e.x;
    g.y = f * e.y;
    g.z = f * e.z;
    g.w = 0;
    a.gpt[i] = g;
    if (a.gV) {
        const T* X = a.X;
        T gx = 0, gy = 0, gz = 0;
        for (int s = 0; s < a.k; ++s) {
            const int j = a.iidx[(size_t)s * a.Ntot + i];
            const T w = a.iw[(size_t)s * a.Ntot + i];
            const T* Xj = X + 12 * (size_t)j;
            // A^T g: row r of A^T is X_j row r
            gx += w * (Xj[0] * g.x + Xj[1] * g.y + Xj[2] * g.z);
            gy += w * (Xj[3] * g.x + Xj[4] * g.y + Xj[5] * g.z);
            gz += w * (Xj[6] * g.x + Xj[7] * g.y + Xj[8] * g.z);
        }
        const int iu = a.src_user[i];
        a.gV[3 * (size_t)iu + 0] = gx;
        a.gV[3 * (size_t)iu + 1] = gy;
        a.gV[3 * (size_t)iu + 2] = gz;
    }
}

// Per node: dE/dX_j = sum_i w_ij [v_i - p_j; 1] g_i^T
//   + alpha sum over D_lj of r [p_l - p_j; 1] h^T - alpha sum over D_jl of r e4 h^T
//   + 2 beta [(A_j - R_j)^T; 0],   h = exp(-|D|^2/(2 nu_r^2)) D / nu_r^2.
template <typename T>
__global__ void __launch_bounds__(64) k_grad_nodes(GradArgs<T> a) {
    using V = typename V4Of<T>::type;
    // neighbouring nodes share most of their points: keep them on one XCD
    const int j = xcd_tile(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    const int p = a.node_pair[j];
    const PairDyn dy = a.dyn[p];
    if (!(dy.flags & PF_EVAL)) return;
    const V pj = a.nodes[j];
    const int src_set = dy.eval_dst;
    const V* src = a.src_override ? (const V*)a.src_override : (const V*)a.src;
    T acc[12];
    for (int m = 0; m < 12; ++m) acc[m] = 0;
    const int e0 = a.pj_ptr[j], e1 = a.pj_ptr[j + 1];
    for (int e = e0 + lane; e < e1; e += 64) {
        const int ent = a.pj_ent[e];
        const int i = ent >> 3, s = ent & 7;
        const T w = a.iw[(size_t)s * a.Ntot + i];
        const V v = src[i];
        const V g = a.gpt[i];
        const T x4[4] = {v.x - pj.x, v.y - pj.y, v.z - pj.z, T(1)};
        for (int r = 0; r < 4; ++r) {
            acc[3 * r + 0] += w * x4[r] * g.x;
            acc[3 * r + 1] += w * x4[r] * g.y;
            acc[3 * r + 2] += w * x4[r] * g.z;
        }
    }
    for (int m = 0; m < 12; ++m) acc[m] = wave_sum(acc[m]);
    if (lane != 0) return;
    const T nur2 = (T)dy.nu_r * (T)dy.nu_r;
    const T alpha = (T)dy.alpha, beta = (T)dy.beta;
    const V* Dr = a.Dres[src_set];
    for (int e = a.adj_ptr[j]; e < a.adj_ptr[j + 1]; ++e) {
        const int l = a.adj_nbr[e], rev = a.adj_rev[e];
        const T rr = a.adj_r[e];
        // D_lj (entry rev = l->j): transform of j applied at p_l
        const V D1 = Dr[rev];
        const T f1 = exp(-D1.w / (T(2) * nur2)) / nur2;
        const V pl = a.nodes[l];
        const T x4[4] = {pl.x - pj.x, pl.y - pj.y, pl.z - pj.z, T(1)};
        for (int r = 0; r < 4; ++r) {
            acc[3 * r + 0] += alpha * rr * x4[r] * f1 * D1.x;
            acc[3 * r + 1] += alpha * rr * x4[r] * f1 * D1.y;
            acc[3 * r + 2] += alpha * rr * x4[r] * f1 * D1.z;
        }
        // D_jl (entry e = j->l): t_j enters with -r
        const V D2 = Dr[e];
        const T f2 = exp(-D2.w / (T(2) * nur2)) / nur2;
        acc[9] -= alpha * rr * f2 * D2.x;
        acc[10] -= alpha * rr * f2 * D2.y;
        acc[11] -= alpha * rr * f2 * D2.z;
    }
    const T* Rd = a.R[src_set] + 9 * (size_t)j;   // proj(A_j) - A_j
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) acc[3 * r + c] -= T(2) * beta * Rd[3 * c + r];
    T* out = a.gX + 12 * (size_t)a.node_user[j];
    for (int m = 0; m < 12; ++m) out[m] = acc[m];
}

// ---------------------------------------------------------------- layout conversion

// X (user node order, type U) -> internal order (type T) and back.
template <typename T, typename U>
__global__ void k_x_import(const U* __restrict__ xu, T* __restrict__ xi, const int* __restrict__ node_user,
                           int64_t ntot) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= 12 * ntot) return;
    const int64_t j = o / 12, m = o % 12;
    xi[o] = (T)xu[12 * (int64_t)node_user[j] + m];
}

template <typename T, typename U>
__global__ void k_x_export(const T* __restrict__ xi, U* __restrict__ xu, const int* __restrict__ node_user,
                           int64_t ntot) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= 12 * ntot) return;
    const int64_t j = o / 12, m = o % 12;
    xu[12 * (int64_t)node_user[j] + m] = (U)xi[o];
}

template <typename T, typename U>
__global__ void k_src_import(const U* __restrict__ su, typename V4Of<T>::type* __restrict__ si,
                             const int* __restrict__ src_user, int64_t Ntot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Ntot) return;
    const int64_t u = src_user[i];
    typename V4Of<T>::type v;
    v.x = (T)su[3 * u];
    v.y = (T)su[3 * u + 1];
    v.z = (T)su[3 * u + 2];
    v.w = 0;
    si[i] = v;
}

template <typename T, typename U>
__global__ void k_points_export(const typename V4Of<T>::type* __restrict__ vi, U* __restrict__ vu,
                                const int* __restrict__ src_user, int64_t Ntot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Ntot) return;
    const int64_t u = src_user[i];
    const typename V4Of<T>::type v = vi[i];
    vu[3 * u] = (U)v.x;
    vu[3 * u + 1] = (U)v.y;
    vu[3 * u + 2] = (U)v.z;
}

template <typename T, typename U>
__global__ void k_nn_export(const int* __restrict__ rho, const T* __restrict__ d2, const int* __restrict__ src_user,
                            const int* __restrict__ tgt_user, int32_t* __restrict__ rho_u, U* __restrict__ d2_u,
                            int64_t Ntot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Ntot) return;
    const int64_t u = src_user[i];
    if (rho_u) rho_u[u] = tgt_user[rho[i]];
    if (d2_u) d2_u[u] = (U)d2[i];
}

// Exact selection of the two middle squared distances of every pair (ranks
// N/2 - 1 and N/2 of its points in increasing order; for odd N the first is
// unused), for the median start rule of nu_a: a radix select over the
// values' bit patterns, which order non-negative floats like their values,
// 8 bits per pass from the top.  Per pass, every point tile counts its
// points whose higher bits match the prefix chosen so far into 256 bins
// (one per-wave vote per distinct bin, then one global atomic per bin and
// tile: integer counts, exact in any order), and one thread per (pair,
// rank) then picks the bin holding the rank.  The result is the element
// itself, bitwise.
template <typename T>
struct SelUint {
    using type = typename std::conditional<sizeof(T) == 8, unsigned long long, unsigned>::type;
};

struct SelState {
    unsigned long long prefix;
    long long k;
};

__global__ void k_sel_init(const PairInfo* __restrict__ info, int P, SelState* __restrict__ st,
                           unsigned* __restrict__ hist) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < 2 * P * 256) hist[e] = 0;
    if (e < 2 * P) {
        const long long N = info[e >> 1].N, k = N / 2 - 1 + (e & 1);
        st[e].prefix = 0;
        st[e].k = k < 0 ? 0 : k;
    }
}

template <typename T>
__global__ void __launch_bounds__(kPointTile) k_sel_hist(const T* __restrict__ d2, const int4* __restrict__ tiles,
                                                         const SelState* __restrict__ st, int shift,
                                                         unsigned* __restrict__ hist) {
    using U = typename SelUint<T>::type;
    __shared__ unsigned h[2][256];
    const int4 td = tiles[blockIdx.x];
    const int p = td.x;
    h[0][threadIdx.x] = 0;
    h[1][threadIdx.x] = 0;
    __syncthreads();
    const U mask = shift + 8 >= 8 * (int)sizeof(T) ? U(0) : (~U(0)) << (shift + 8);
    const int i = td.y + (int)threadIdx.x;
    U u = 0;
    const bool live = i < td.z;
    if (live) {
        const T x = d2[i];
        __builtin_memcpy(&u, &x, sizeof u);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const U prefix = (U)st[2 * p + r].prefix;
        int bin = live && (u & mask) == prefix ? (int)((u >> shift) & 255u) : -1;
        while (true) {
            const unsigned long long want = __ballot(bin >= 0);
            if (!want) break;
            const int lead = __ffsll((long long)want) - 1;
            const int b = __shfl(bin, lead);
            const unsigned long long same = __ballot(bin == b);
            if ((int)(threadIdx.x & 63) == lead) atomicAdd(&h[r][b], (unsigned)__popcll(same));
            if (bin == b) bin = -1;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 2; ++r)
        if (h[r][threadIdx.x]) atomicAdd(&hist[(2 * p + r) * 256 + threadIdx.x], h[r][threadIdx.x]);
}

__global__ void k_sel_scan(int P, int shift, SelState* __restrict__ st, unsigned* __restrict__ hist) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * P) return;
    unsigned* h = hist + 256 * (size_t)e;
    long long k = st[e].k, cum = 0;
    int b = 0;
    for (; b < 255; ++b) {
        if (cum + h[b] > k) break;
        cum += h[b];
    }
    st[e].k = k - cum;
    st[e].prefix |= (unsigned long long)b << shift;
    for (int q = 0; q < 256; ++q) h[q] = 0;
}

template <typename T>
__global__ void k_sel_out(int P, const SelState* __restrict__ st, T* __restrict__ out) {
    using U = typename SelUint<T>::type;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * P) return;
    const U u = (U)st[e].prefix;
    T x;
    __builtin_memcpy(&x, &u, sizeof x);
    out[e] = x;
}

template <typename T>
__global__ void k_cast_static(const double* __restrict__ in, T* __restrict__ out, int64_t n) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o < n) out[o] = (T)in[o];
}

// ---------------------------------------------------------------- launchers

static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <typename T>
void launch_eval(const EvalArgs<T>& a, int n_pt_tiles, int n_eg_tiles, int n_nd_tiles, const FinalArgs& f,
                 int P, hipStream_t s, KernelTimer* tm) {
    if (n_pt_tiles) {
        // budgeted searches, then the deferred points one wave each, then the
        // tile sums (the deferred points' count is only known on the device:
        // a fixed grid strides over it)
        // (the edge and node terms ride on the deferred searches' launch)
        const int far_blocks = (int)std::min<int64_t>(1024, (a.Ntot + kFarWaves * kFarPts - 1) / (kFarWaves * kFarPts));
        const unsigned grid = (unsigned)(far_blocks + n_eg_tiles + (n_nd_tiles + kNodeGroups - 1) / kNodeGroups);
        if (a.nn_work) {
            launch_one(tm, "eval_points", k_eval_points<T, true>, dim3(n_pt_tiles), dim3(kPointTile), s, a);
            launch_one(tm, "eval_far", k_eval_far<T, true>, dim3(grid), dim3(64 * kFarWaves), s, a, far_blocks,
                       n_eg_tiles, n_nd_tiles);
        } else {
            launch_one(tm, "eval_points", k_eval_points<T, false>, dim3(n_pt_tiles), dim3(kPointTile), s, a);
            launch_one(tm, "eval_far", k_eval_far<T, false>, dim3(grid), dim3(64 * kFarWaves), s, a, far_blocks,
                       n_eg_tiles, n_nd_tiles);
        }
        launch_one(tm, "eval_sums", k_eval_sums<T>, dim3(n_pt_tiles), dim3(kPointTile), s, a);
    } else {
        if (n_eg_tiles) launch_one(tm, "eval_edges", k_eval_edges<T>, dim3(n_eg_tiles), dim3(kEdgeTile), s, a);
        if (n_nd_tiles) launch_one(tm, "eval_nodes", k_eval_nodes<T>, dim3(n_nd_tiles), dim3(kNodeTile), s, a);
    }
    launch_one(tm, "energy_final", k_energy_final, dim3(P), dim3(64), s, f);
}

template <typename T>
void launch_assemble(const AsmArgs<T>& a, int64_t ntot, hipStream_t s, KernelTimer* tm) {
    launch_one(tm, "assemble", k_assemble<T>, dim3((unsigned)ntot), dim3(64), s, a);
}

template <typename T>
void launch_residual64(const CgArgs<T>& a, int n_nd_tiles, const T* B, const T* Bn, const double* x64,
                       T* rhs_out, double* part_rr, double* part_bb, hipStream_t s, KernelTimer* tm) {
    if (tm) tm->begin("residual64", s);
    hipLaunchKernelGGL(k_residual64<T>, dim3(n_nd_tiles), dim3(4 * kNodeTile), 0, s, a, B, Bn, x64, rhs_out,
                       part_rr, part_bb);
    if (tm) tm->end(s);
}

template <typename T>
void launch_node_vec_op(const NodeVecArgs<T>& a, int n_nd_tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_node_vec_op<T>, dim3(n_nd_tiles), dim3(4 * kNodeTile), 0, s, a);
}

template <typename T>
void launch_aa(const AaArgs<T>& a, const AaSolveArgs& sa, int n_nd_tiles, hipStream_t s, KernelTimer* tm) {
    if (tm) tm->begin("anderson", s);
    hipLaunchKernelGGL(k_aa_push<T>, dim3(n_nd_tiles), dim3(4 * kNodeTile), 0, s, a);
    hipLaunchKernelGGL(k_aa_gram<T>, dim3(n_nd_tiles), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_aa_solve, dim3(sa.P), dim3(512), 0, s, sa);
    hipLaunchKernelGGL(k_aa_mix<T>, dim3(n_nd_tiles), dim3(4 * kNodeTile), 0, s, a);
    if (tm) tm->end(s);
}

template <typename T>
void launch_grad(const GradArgs<T>& a, int n_pt_tiles, int64_t ntot, hipStream_t s) {
    hipLaunchKernelGGL(k_grad_points<T>, dim3(n_pt_tiles), dim3(kPointTile), 0, s, a);
    hipLaunchKernelGGL(k_grad_nodes<T>, dim3((unsigned)ntot), dim3(64), 0, s, a);
}

template <typename T, typename U>
void launch_x_import(const U* xu, T* xi, const int* node_user, int64_t ntot, hipStream_t s) {
    if (ntot) hipLaunchKernelGGL((k_x_import<T, U>), dim3(blocks_for(12 * ntot, 256)), dim3(256), 0, s, xu, xi, node_user, ntot);
}
template <typename T, typename U>
void launch_x_export(const T* xi, U* xu, const int* node_user, int64_t ntot, hipStream_t s) {
    if (ntot) hipLaunchKernelGGL((k_x_export<T, U>), dim3(blocks_for(12 * ntot, 256)), dim3(256), 0, s, xi, xu, node_user, ntot);
}
template <typename T, typename U>
void launch_src_import(const U* su, void* si, const int* src_user, int64_t Ntot, hipStream_t s) {
    hipLaunchKernelGGL((k_src_import<T, U>), dim3(blocks_for(Ntot, 256)), dim3(256), 0, s, su,
                       (typename V4Of<T>::type*)si, src_user, Ntot);
}
template <typename T, typename U>
void launch_points_export(const void* vi, U* vu, const int* src_user, int64_t Ntot, hipStream_t s) {
    hipLaunchKernelGGL((k_points_export<T, U>), dim3(blocks_for(Ntot, 256)), dim3(256), 0, s,
                       (const typename V4Of<T>::type*)vi, vu, src_user, Ntot);
}
template <typename T, typename U>
void launch_nn_export(const int* rho, const T* d2, const int* src_user, const int* tgt_user, int32_t* rho_u,
                      U* d2_u, int64_t Ntot, hipStream_t s) {
    hipLaunchKernelGGL((k_nn_export<T, U>), dim3(blocks_for(Ntot, 256)), dim3(256), 0, s, rho, d2, src_user,
                       tgt_user, rho_u, d2_u, Ntot);
}
template <typename T>
__global__ void __launch_bounds__(256) k_weights_point_major(const T* __restrict__ iw, int k, int64_t N,
                                                            T* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
#pragma unroll
    for (int a = 0; a < kMaxK; ++a) out[(size_t)kMaxK * i + a] = a < k ? iw[(size_t)a * N + i] : T(0);
}

template <typename T>
void launch_weights_point_major(const T* iw, int k, int64_t N, T* out, hipStream_t s) {
    if (N) hipLaunchKernelGGL(k_weights_point_major<T>, dim3(blocks_for(N, 256)), dim3(256), 0, s, iw, k, N, out);
}

template <typename T>
void launch_cast_static(const double* in, T* out, int64_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_cast_static<T>, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
}

template <int N>
__global__ void __launch_bounds__(64) k_dyn_set(DynPack<N> pk) {
    static_assert(sizeof(PairDyn) % 4 == 0, "PairDyn is copied in 32-bit words");
    const int words = pk.n * (int)(sizeof(PairDyn) / 4);
    const unsigned* src = reinterpret_cast<const unsigned*>(pk.d);
    unsigned* dst = reinterpret_cast<unsigned*>(pk.dst);
    for (int i = threadIdx.x; i < words; i += 64) dst[i] = src[i];
}

template <int N>
void dyn_set_pack(const PairDyn* src, int n, PairDyn* dst, hipStream_t s) {
    DynPack<N> pk;
    for (int i = 0; i < n; ++i) pk.d[i] = src[i];
    pk.dst = dst;
    pk.n = n;
    hipLaunchKernelGGL(k_dyn_set<N>, dim3(1), dim3(64), 0, s, pk);
}

void launch_dyn_set(const PairDyn* src, int n, PairDyn* dst, hipStream_t s) {
    if (n <= 1)
        dyn_set_pack<1>(src, n, dst, s);
    else if (n <= 8)
        dyn_set_pack<8>(src, n, dst, s);
    else
        dyn_set_pack<kDynPerLaunch>(src, n, dst, s);
}


template <typename T>
void launch_select_mid(const T* d2, const PairInfo* info, const int4* pt_tiles, int n_pt_tiles, int P, T* out,
                       void* work, hipStream_t s) {
    if (P <= 0) return;
    SelState* st = reinterpret_cast<SelState*>(work);
    unsigned* hist = reinterpret_cast<unsigned*>(st + 2 * P);
    hipLaunchKernelGGL(k_sel_init, dim3(blocks_for(2 * (int64_t)P * 256, 256)), dim3(256), 0, s, info, P, st, hist);
    for (int shift = 8 * (int)sizeof(T) - 8; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_sel_hist<T>, dim3(n_pt_tiles), dim3(kPointTile), 0, s, d2, pt_tiles,
                           (const SelState*)st, shift, hist);
        hipLaunchKernelGGL(k_sel_scan, dim3(blocks_for(2 * (int64_t)P, 64)), dim3(64), 0, s, P, shift, st, hist);
    }
    hipLaunchKernelGGL(k_sel_out<T>, dim3(blocks_for(2 * (int64_t)P, 64)), dim3(64), 0, s, P, (const SelState*)st,
                       out);
}

size_t select_mid_work_bytes(int P) { return (sizeof(SelState) + 256 * sizeof(unsigned)) * 2 * (size_t)P; }

#define AMM_INSTANTIATE(T)                                                                                     \
    template void launch_select_mid<T>(const T*, const PairInfo*, const int4*, int, int, T*, void*, hipStream_t); \
    template void launch_eval<T>(const EvalArgs<T>&, int, int, int, const FinalArgs&, int, hipStream_t,        \
                                 KernelTimer*);                                                               \
    template void launch_assemble<T>(const AsmArgs<T>&, int64_t, hipStream_t, KernelTimer*);                   \
    template void launch_residual64<T>(const CgArgs<T>&, int, const T*, const T*, const double*, T*, double*,  \
                                       double*, hipStream_t, KernelTimer*);                                   \
    template void launch_node_vec_op<T>(const NodeVecArgs<T>&, int, hipStream_t);                             \
    template void launch_aa<T>(const AaArgs<T>&, const AaSolveArgs&, int, hipStream_t, KernelTimer*);          \
    template void launch_grad<T>(const GradArgs<T>&, int, int64_t, hipStream_t);                              \
    template void launch_cast_static<T>(const double*, T*, int64_t, hipStream_t);                              \
    template void launch_weights_point_major<T>(const T*, int, int64_t, T*, hipStream_t);                      \
    template void launch_x_import<T, float>(const float*, T*, const int*, int64_t, hipStream_t);              \
    template void launch_x_import<T, double>(const double*, T*, const int*, int64_t, hipStream_t);            \
    template void launch_x_export<T, float>(const T*, float*, const int*, int64_t, hipStream_t);              \
    template void launch_x_export<T, double>(const T*, double*, const int*, int64_t, hipStream_t);            \
    template void launch_src_import<T, float>(const float*, void*, const int*, int64_t, hipStream_t);         \
    template void launch_src_import<T, double>(const double*, void*, const int*, int64_t, hipStream_t);       \
    template void launch_points_export<T, float>(const void*, float*, const int*, int64_t, hipStream_t);      \
    template void launch_points_export<T, double>(const void*, double*, const int*, int64_t, hipStream_t);    \
    template void launch_nn_export<T, float>(const int*, const T*, const int*, const int*, int32_t*, float*,    \
                                             int64_t, hipStream_t);                                           \
    template void launch_nn_export<T, double>(const int*, const T*, const int*, const int*, int32_t*, double*,  \
                                              int64_t, hipStream_t);

AMM_INSTANTIATE(float)
AMM_INSTANTIATE(double)

}  // namespace amm
