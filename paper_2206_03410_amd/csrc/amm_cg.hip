// Preconditioned conjugate gradients for the normal equations K X = B of
// Eq. (21) -- three right-hand sides sharing K -- batched over pairs, and the
// coarse level of its preconditioner.
//
// CG variant: Chronopoulos-Gear, one reduction phase per step.  With
// u = M^{-1} r and w = K u, step i takes gamma = (r, u) and delta = (w, u) of
// the current vectors and forms
//   beta = gamma_i / gamma_{i-1},  alpha = gamma_i / (delta_i - beta gamma_i / alpha_{i-1}),
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
// then the new u and w = K u.  One kernel per step over solver tiles of 16
// node rows, 256 threads (16 lanes per row).  A step needs the new u of
// every column node of its rows; instead of a separate launch, each lane
// recomputes u_l for the column block it multiplies from the previous step's
// r, w, s (r, u, w, s and the partials are double-buffered by step parity).
// Owner and halo recomputation call the same helpers, so both give identical
// values.
//
// Preconditioner: block Jacobi on the 4x4 diagonal blocks of K, optionally
// plus a coarse correction (two-level additive):
//   M^{-1} = D^{-1} + P A_c^{-1} P^T,  A_c = P^T K P,
// where P maps one affine field per aggregate of consecutive (Morton-ordered)
// nodes onto the node transforms: with x -> M x + b on the aggregate, node j
// gets A_j = M, t_j = (M - I) p_j + b, i.e. per column the 4-vector of
// node j is P_j (m, b') with P_j = [[I, 0], [d_j^T, 1]], d_j = p_j - centroid.
// These fields are the smooth modes that block Jacobi damps slowest (the
// regularization term of Eq. (9) vanishes on a common affine map).  P^T r
// of the new residual is carried by the recurrences
//   P^T s_i = P^T w_i + beta P^T s_{i-1},  P^T r_{i+1} = P^T r_i - alpha P^T s_i,
// whose P^T w term is a tile partial of the previous step, so the coarse
// correction needs no extra grid-wide synchronization: every block forms the
// (small) coarse vectors of its pair itself, in a fixed order.
#include <hip/hip_runtime.h>

#include "amm_coarse_inv.h"
#include "amm_device.h"
#include "amm_kernels.h"

namespace amm {

namespace {

constexpr int kCgThreads = 16 * kNodeTile;
constexpr int kSlotCap = 8;   // coarse aggregates per tile whose A_c^{-1} rows are staged in LDS

// wave sums land in lane 63 (DPP reduction)
template <typename T>
__device__ __forceinline__ T wsum(T v) {
    return wave_total63(v);
}

// u = D_l^{-1} r for one node (r, u: [4][3]; Di row-major 4x4)
template <typename T>
__device__ __forceinline__ void apply_dinv(const T* __restrict__ Di, const T rn[12], T u[12]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T acc = Di[4 * q] * rn[c];
            acc = fma(Di[4 * q + 1], rn[3 + c], acc);
            acc = fma(Di[4 * q + 2], rn[6 + c], acc);
            u[3 * q + c] = fma(Di[4 * q + 3], rn[9 + c], acc);
        }
}

// u += P_l cc: rows 0..2 take the aggregate's linear part, row 3 its
// translation plus d_l . linear part
template <typename T, typename V>
__device__ __forceinline__ void prolong_add(const V& d, const T* cc, T u[12]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        u[c] += cc[c];
        u[3 + c] += cc[3 + c];
        u[6 + c] += cc[6 + c];
        T t = fma(d.x, cc[c], cc[9 + c]);
        t = fma(d.y, cc[3 + c], t);
        t = fma(d.z, cc[6 + c], t);
        u[9 + c] += t;
    }
}

// new r of a node from the step's scalars: r - alpha (w + beta s)
template <typename T>
__device__ __forceinline__ T new_r(T r0, T w0, T s0, T al, T be, bool act, bool first) {
    if (!act) return r0;
    const T sn = first ? w0 : fma(be, s0, w0);
    return fma(-al, sn, r0);
}

template <typename T>
__device__ __forceinline__ T new_s(T w0, T s0, T be, bool first) {
    return first ? w0 : fma(be, s0, w0);
}

// v[c] for a lane-dependent c without indexing the register array
template <typename T>
__device__ __forceinline__ T pick3(const T v[3], int c) {
    return c == 0 ? v[0] : (c == 1 ? v[1] : v[2]);
}

}  // namespace

// One CG step (START = false, it >= 0) or the start (r = b, x = 0, u = M^{-1} b,
// w = K u).  Writes the new r, u, w, s into buffer (it+1) & 1 (the start into
// buffer 0) and the tile partials of the new vectors.
template <typename T, bool COARSE, bool START>
__global__ void __launch_bounds__(kCgThreads) k_cg(CgArgs<T> a, int it) {
    using V = typename V4Of<T>::type;
    constexpr int NA = COARSE ? kCoarseMaxAgg : 1;
    __shared__ double wred[4][12];
    __shared__ double scal[3][3];   // alpha, beta, active
    __shared__ int brk_mask;
    __shared__ T rs[kNodeTile][12];
    __shared__ T ys[kNodeTile][12];
    __shared__ T wp[4][kCgPart];
    __shared__ T gw[NA][12], gro[NA][12], gso[NA][12], gcur[NA][12], cco[NA][12];
    __shared__ T bbw[4][3];
    // float64 steps stage the tile's rows of A_c^{-1} in LDS and fetch their
    // first column block early; in float32 both measured slower than reading
    // the rows from L2 where they are used
    constexpr bool kEarly = sizeof(T) == 8;
    constexpr int NCM = COARSE && kEarly ? 4 * kCoarseMaxAgg : 1;
    // staged rows of A_c^{-1} (row length padded by one element so that
    // rows read together fall in different LDS banks)
    __shared__ T ainv_s[COARSE && kEarly ? 4 * kSlotCap : 1][NCM + 1];
    __shared__ int tl[COARSE ? kCoarseMaxAgg : 1];          // this tile's aggregates
    __shared__ T us[START ? 1 : kTileColCap][12];              // u' of the tile's column nodes

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int4 td = a.nd_tiles[tile];
    const int p = td.x;
    const PairDyn& dy = a.dyn[p];
    if (!(dy.flags & PF_SOLVE)) return;
    const int tid = threadIdx.x;
    const int par = START ? 0 : (it & 1);            // buffer read
    const int nxt = START ? 0 : ((it + 1) & 1);      // buffer written
    // previous step's state (read through the pointer: a local copy indexed
    // by thread would live in scratch memory)
    const CgState* prv = a.state + 2 * (size_t)p + ((it + 1) & 1);
    if (!START) {
        if (prv->conv[0] && prv->conv[1] && prv->conv[2]) {
            // converged before this step: x is final and no later step reads
            // the vectors; carry the state to this step's slot
            if (tid == 0 && tile == a.info[p].nd_tile0) a.state[2 * (size_t)p + (it & 1)] = *prv;
            return;
        }
    }
    const PairInfo& pi = a.info[p];
    const int t0 = pi.nd_tile0, ntl = pi.nd_ntile;
    const int row = tid >> 4, lane = tid & 15;
    const int j = td.y + row;
    const bool live = j < td.z;
    const bool first = !START && it == 0;

    // ---- loads that do not depend on this step's scalars
    int kb = 0, ke = 0;
    if (live) {
        kb = a.K_ptr[j] + lane;
        ke = a.K_ptr[j + 1];
    }
    T own_r = 0, own_u = 0, own_w = 0, own_s = 0, own_p = 0;
    if (live && lane < 12) {
        const size_t o = 12 * (size_t)j + lane;
        if (START) {
            own_r = a.b[o];
        } else {
            own_r = a.r[par][o];
            own_u = a.u[par][o];
            own_w = a.w[par][o];
            own_s = a.s[par][o];
            if (!first) own_p = a.pv[o];
        }
    }
    // ---- pair sums of the previous step's tile partials -> step scalars
    if (!START) {
        double v[12];
#pragma unroll
        for (int m = 0; m < 12; ++m) v[m] = 0;
        for (int t = tid; t < ntl; t += kCgThreads) {
            const double* q = a.part[par] + (size_t)(t0 + t) * kCgPart;
#pragma unroll
            for (int m = 0; m < 9; ++m) v[m] += q[m];
            const double* qb = a.part_bb + 3 * (size_t)(t0 + t);
#pragma unroll
            for (int c = 0; c < 3; ++c) v[9 + c] += qb[c];
        }
#pragma unroll
        for (int m = 0; m < 12; ++m) v[m] = wsum(v[m]);
        if ((tid & 63) == 63)
#pragma unroll
            for (int m = 0; m < 12; ++m) wred[tid >> 6][m] = v[m];
    }
    if (COARSE) {
        // P^T w_i (or P^T b at the start) per aggregate from the tile partials,
        // and the carried P^T r_i, P^T s_{i-1}
        const int per = 1 << (pi.agg_shift - 4);   // node tiles per aggregate
        const double* src = a.part[START ? 1 : par];
        for (int e = tid; e < pi.nagg * 12; e += kCgThreads) {
            const int al = e / 12, m = e - 12 * al;
            const int ta = al * per, tb = min(ta + per, ntl);
            double acc = 0;
            for (int t = ta; t < tb; ++t) acc += src[(size_t)(t0 + t) * kCgPart + 9 + m];
            gw[al][m] = (T)acc;
            if (!START) {
                const size_t go = 12 * (size_t)(pi.agg0 + al) + m;
                gro[al][m] = a.gr[par][go];
                gso[al][m] = a.gs[par][go];
            }
        }
    }
    // Issued after the loads the scalars need (a wave waits for its loads in
    // issue order).  A step forms u' of each distinct column node of the
    // tile once, in LDS (at most two tasks per thread: node e / 3, column
    // e % 3): here the previous step's r, w, s of those columns, the nodes'
    // diagonal inverses and positions, and this lane's first two K blocks
    // with their local column indices.  A tile with more column nodes than
    // fit recomputes u' for every block instead.
    static_assert(2 * kCgThreads >= 3 * kTileColCap, "two shared-u' tasks per thread");
    bool shr = false;
    int nct = 0, hl[2] = {0, 0}, slc[2] = {0, 0}, rowl = 0;
    T h_r[2][4], h_w[2][4], h_s[2][4], h_d[2][16], sk[2][16];
    V h_rel[2] = {};
    if (!START) {
        nct = a.tile_ncols[tile];
        shr = nct <= kTileColCap;
    }
    if (!START && shr) {
        rowl = a.tile_rowl[(size_t)tile * kNodeTile + row];
#pragma unroll
        for (int k2 = 0; k2 < 2; ++k2) {
            const int e = tid + kCgThreads * k2;
            if (e < 3 * nct) {
                const int li = e / 3, c = e - 3 * li;
                const int l = a.tile_cols[(size_t)tile * kTileColCap + li];
                hl[k2] = l;
                const size_t ol = 12 * (size_t)l + c;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    h_r[k2][k] = a.r[par][ol + 3 * k];
                    h_w[k2][k] = a.w[par][ol + 3 * k];
                    h_s[k2][k] = a.s[par][ol + 3 * k];
                }
#pragma unroll
                for (int m = 0; m < 16; ++m) h_d[k2][m] = a.Dinv[16 * (size_t)l + m];
                if (COARSE) h_rel[k2] = a.node_rel[l];
            }
        }
#pragma unroll
        for (int k2 = 0; k2 < 2; ++k2) {
            const int pos = kb + 16 * k2;
            if (pos < ke) {
                slc[k2] = a.K_lcol[pos];
#pragma unroll
                for (int m = 0; m < 16; ++m) sk[k2][m] = a.Kval[16 * (size_t)pos + m];
            }
        }
    }
    int l0 = -1;
    T f_r[12], f_w[12], f_s[12], f_d[16], f_k[16];
    V f_rel{};
    if (kEarly && !START && !shr && kb < ke) {
        l0 = a.K_col[kb];
        const size_t ol = 12 * (size_t)l0;
#pragma unroll
        for (int m = 0; m < 12; ++m) {
            f_r[m] = a.r[par][ol + m];
            f_w[m] = a.w[par][ol + m];
            f_s[m] = a.s[par][ol + m];
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            f_d[m] = a.Dinv[16 * (size_t)l0 + m];
            f_k[m] = a.Kval[16 * (size_t)kb + m];
        }
        if (COARSE) f_rel = a.node_rel[l0];
    }
    // rows of A_c^{-1} of this tile's first kSlotCap aggregates (staged in
    // LDS after the first barrier); thread t covers column t % 128 of rows
    // t / 128, t / 128 + 2, ...
    int q0 = 0, nsl = 0, nc = 0;
    constexpr int APRE = COARSE && kEarly ? (4 * kSlotCap * 4 * kCoarseMaxAgg) / kCgThreads : 1;
    T apre[APRE];
    if (COARSE) {
        q0 = a.tile_agg_ptr[tile];
        nsl = a.tile_agg_ptr[tile + 1] - q0;
        nc = 4 * pi.nagg;
        if (tid < nsl) tl[tid] = a.tile_agg[q0 + tid];
        const int nrow = kEarly ? 4 * min(nsl, kSlotCap) : 0;
        const int col = tid & 127, r0 = tid >> 7;
        const T* Ai = a.Ainv + pi.ainv_off;
#pragma unroll
        for (int rr = 0; rr < APRE; ++rr) {
            const int rw = r0 + 2 * rr;
            apre[rr] = 0;
            if (rw < nrow && col < nc) {
                const int ag = a.tile_agg[q0 + (rw >> 2)];
                apre[rr] = Ai[(size_t)(4 * ag + (rw & 3)) * nc + col];
            }
        }
    }

    if (tid == 0) brk_mask = 0;
    __syncthreads();
    if (!START) {
        if (tid < 3) {
            const int c = tid;
            const double gam = ((wred[0][c] + wred[1][c]) + wred[2][c]) + wred[3][c];
            const double del = ((wred[0][3 + c] + wred[1][3 + c]) + wred[2][3 + c]) + wred[3][3 + c];
            const double rr = ((wred[0][6 + c] + wred[1][6 + c]) + wred[2][6 + c]) + wred[3][6 + c];
            const double bb = ((wred[0][9 + c] + wred[1][9 + c]) + wred[2][9 + c]) + wred[3][9 + c];
            const double rtol2 = dy.cg_rtol > 0 ? dy.cg_rtol * dy.cg_rtol : a.rtol2;
            int conv = prv->conv[c];
            int brk = 0;
            double al = 0, be = 0;
            const double rr0 = it == 0 ? rr : prv->rr0[c];
            if (!conv) {
                if (rr <= rtol2 * bb || bb == 0.0 || rr <= a.floor2 * rr0) {
                    conv = 1;
                } else if (it == 0) {
                    al = gam / del;
                } else {
                    be = gam / prv->gamma[c];
                    al = gam / (del - be * gam / prv->alpha[c]);
                }
                if (!conv && !(al > 0.0 && gam > 0.0 && al < 1e300)) {
                    conv = 1;
                    brk = 1;
                    al = be = 0;
                }
            }
            scal[c][0] = al;
            scal[c][1] = be;
            scal[c][2] = conv ? 0.0 : 1.0;
            if (tile == t0) {
                CgState& st = a.state[2 * (size_t)p + (it & 1)];
                st.alpha[c] = al;
                st.gamma[c] = gam;
                st.rr[c] = rr;
                st.bb[c] = bb;
                st.rr0[c] = rr0;
                st.conv[c] = conv;
            }
            if (brk) atomicOr(&brk_mask, 1 << c);
        }
        __syncthreads();
        if (tid == 0 && tile == t0) {
            CgState& st = a.state[2 * (size_t)p + (it & 1)];
            const bool any = scal[0][2] != 0.0 || scal[1][2] != 0.0 || scal[2][2] != 0.0;
            st.iters = prv->iters + (any ? 1 : 0);
            st.breakdown = prv->breakdown | brk_mask;
            // progress for the host (coherent pinned memory), every 4th step
            // and at convergence: a store to host memory delays the kernel's
            // completion, so most steps skip it.  The convergence word carries
            // the iteration count and breakdown flags in the same store.
            volatile long long* pg = a.prog + 2 * p;
            if (!any)
                pg[1] = ((long long)st.iters << 32) | ((long long)(st.breakdown & 7) << 60) |
                        (long long)(unsigned)it;
            if (!any || (it & 3) == 3) pg[0] = it;
        }
    } else {
        if (tid < 3) {
            scal[tid][0] = scal[tid][1] = 0;
            scal[tid][2] = 1.0;
        }
        if (tid < 3 && tile == t0) {
            CgState* st = a.state + 2 * (size_t)p;
            st[0].conv[tid] = 0;
            st[1].conv[tid] = 0;
            if (tid == 0) {
                st[0].iters = st[1].iters = 0;
                st[0].breakdown = st[1].breakdown = 0;
            }
        }
        __syncthreads();
    }
    T al[3], be[3];
    bool act[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        al[c] = (T)scal[c][0];
        be[c] = (T)scal[c][1];
        act[c] = scal[c][2] != 0.0;
    }
    if (COARSE && kEarly) {
        const int nrow = 4 * min(nsl, kSlotCap);
        const int col = tid & 127, r0 = tid >> 7;
#pragma unroll
        for (int rr = 0; rr < APRE; ++rr) {
            const int rw = r0 + 2 * rr;
            if (rw < nrow && col < nc) ainv_s[rw][col] = apre[rr];
        }
    }

    // ---- coarse level: P^T s_i, P^T r_{i+1}, then A_c^{-1} P^T r_{i+1} for
    // the aggregates this tile's rows touch
    if (COARSE) {
        for (int e = tid; e < pi.nagg * 12; e += kCgThreads) {
            const int ag = e / 12, m = e - 12 * ag, c = m % 3;
            T g, gsn;
            if (START) {
                g = gw[ag][m];
                gsn = 0;
            } else if (pick3(act, c)) {
                gsn = first ? gw[ag][m] : fma(pick3(be, c), gso[ag][m], gw[ag][m]);
                g = fma(-pick3(al, c), gsn, gro[ag][m]);
            } else {
                gsn = gso[ag][m];
                g = gro[ag][m];
            }
            gcur[ag][m] = g;
            if (tile == t0) {
                const size_t go = 12 * (size_t)(pi.agg0 + ag) + m;
                a.gr[nxt][go] = g;
                a.gs[nxt][go] = gsn;
            }
        }
        __syncthreads();
        // (A_c^{-1} g)[aggregate, q, c] in four interleaved parts over the
        // coarse columns, combined across 4 consecutive lanes in a fixed order
        // (every block forms the same values for an aggregate)
        const T* Ai = a.Ainv + pi.ainv_off;
        for (int e = tid; e < nsl * 48; e += kCgThreads) {
            const int sl = e / 48, rem = e - 48 * sl, m = rem >> 2, part = rem & 3;
            const int q = m / 3, c = m - 3 * q;
            const int ag = tl[sl];
            T acc = 0;
            if (kEarly && sl < kSlotCap) {
                const T* rw = &ainv_s[4 * sl + q][0];
                for (int bq = part; bq < pi.nagg; bq += 4) {
                    acc = fma(rw[4 * bq], gcur[bq][c], acc);
                    acc = fma(rw[4 * bq + 1], gcur[bq][3 + c], acc);
                    acc = fma(rw[4 * bq + 2], gcur[bq][6 + c], acc);
                    acc = fma(rw[4 * bq + 3], gcur[bq][9 + c], acc);
                }
            } else {
                const T* rw = Ai + (size_t)(4 * ag + q) * nc;
                for (int bq = part; bq < pi.nagg; bq += 4) {
                    acc = fma(rw[4 * bq], gcur[bq][c], acc);
                    acc = fma(rw[4 * bq + 1], gcur[bq][3 + c], acc);
                    acc = fma(rw[4 * bq + 2], gcur[bq][6 + c], acc);
                    acc = fma(rw[4 * bq + 3], gcur[bq][9 + c], acc);
                }
            }
            acc = quad_sum(acc);
            if (part == 0) cco[ag][m] = acc;
        }
        __syncthreads();
    }

    // ---- u' of the tile's column nodes, once each (the arithmetic of the
    // per-block recomputation below, so both give identical values)
    if (!START && shr) {
#pragma unroll
        for (int k2 = 0; k2 < 2; ++k2) {
            const int e = tid + kCgThreads * k2;
            if (e < 3 * nct) {
                const int li = e / 3, c = e - 3 * li;
                const T alc = pick3(al, c), bec = pick3(be, c);
                const bool ac = pick3(act, c);
                T rn[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) rn[k] = new_r(h_r[k2][k], h_w[k2][k], h_s[k2][k], alc, bec, ac, first);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    T v = h_d[k2][4 * q] * rn[0];
                    v = fma(h_d[k2][4 * q + 1], rn[1], v);
                    v = fma(h_d[k2][4 * q + 2], rn[2], v);
                    v = fma(h_d[k2][4 * q + 3], rn[3], v);
                    if (COARSE) {
                        const T* cc = cco[(hl[k2] - (int)pi.node_off) >> pi.agg_shift];
                        if (q < 3) {
                            v += cc[3 * q + c];
                        } else {
                            T t = fma(h_rel[k2].x, cc[c], cc[9 + c]);
                            t = fma(h_rel[k2].y, cc[3 + c], t);
                            t = fma(h_rel[k2].z, cc[6 + c], t);
                            v += t;
                        }
                    }
                    us[li][3 * q + c] = v;
                }
            }
        }
    }

    // ---- own rows: p, s, x, r
    if (live && lane < 12) {
        const size_t o = 12 * (size_t)j + lane;
        const int c = lane % 3;
        T rn;
        if (START) {
            rn = own_r;
            a.x[o] = 0;
            a.s[nxt][o] = 0;
        } else if (pick3(act, c)) {
            const T bec = pick3(be, c), alc = pick3(al, c);
            const T pn = first ? own_u : fma(bec, own_p, own_u);
            const T sn = new_s(own_w, own_s, bec, first);
            a.pv[o] = pn;
            a.s[nxt][o] = sn;
            a.x[o] = fma(alc, pn, a.x[o]);
            rn = fma(-alc, sn, own_r);
        } else {
            rn = own_r;
            a.s[nxt][o] = own_s;
        }
        a.r[nxt][o] = rn;
        rs[row][lane] = rn;
    }

    // ---- w = K u' with u' recomputed for every column block
    T y[12];
#pragma unroll
    for (int m = 0; m < 12; ++m) y[m] = 0;
    // y += K_jl u'_l
    auto block = [&](int l, const T* rn, const T* Dl, const T* kv, const V& rel) {
        T ul[12];
        apply_dinv(Dl, rn, ul);
        if (COARSE) prolong_add(rel, cco[(l - (int)pi.node_off) >> pi.agg_shift], ul);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T acc = y[3 * q + c];
                acc = fma(kv[4 * q], ul[c], acc);
                acc = fma(kv[4 * q + 1], ul[3 + c], acc);
                acc = fma(kv[4 * q + 2], ul[6 + c], acc);
                y[3 * q + c] = fma(kv[4 * q + 3], ul[9 + c], acc);
            }
    };
    int pos0 = kb;
    if (!START && shr) {
        __syncthreads();   // us complete
        auto sblock = [&](const T* kv, int li) {
            const T* ul = us[li];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    T acc = y[3 * q + c];
                    acc = fma(kv[4 * q], ul[c], acc);
                    acc = fma(kv[4 * q + 1], ul[3 + c], acc);
                    acc = fma(kv[4 * q + 2], ul[6 + c], acc);
                    y[3 * q + c] = fma(kv[4 * q + 3], ul[9 + c], acc);
                }
        };
        if (kb < ke) sblock(sk[0], slc[0]);
        if (kb + 16 < ke) sblock(sk[1], slc[1]);
        for (int pos = kb + 32; pos < ke; pos += 16) {
            T kv[16];
#pragma unroll
            for (int m = 0; m < 16; ++m) kv[m] = a.Kval[16 * (size_t)pos + m];
            sblock(kv, a.K_lcol[pos]);
        }
        pos0 = ke;
    } else if (!START && l0 >= 0) {
        T rn[12];
#pragma unroll
        for (int m = 0; m < 12; ++m)
            rn[m] = new_r(f_r[m], f_w[m], f_s[m], al[m % 3], be[m % 3], act[m % 3], first);
        block(l0, rn, f_d, f_k, f_rel);
        pos0 = kb + 16;
    }
    for (int pos = pos0; pos < ke; pos += 16) {
        const int l = a.K_col[pos];
        const size_t ol = 12 * (size_t)l;
        T rn[12];
        if (START) {
#pragma unroll
            for (int m = 0; m < 12; ++m) rn[m] = a.b[ol + m];
        } else {
#pragma unroll
            for (int m = 0; m < 12; ++m)
                rn[m] = new_r(a.r[par][ol + m], a.w[par][ol + m], a.s[par][ol + m], al[m % 3], be[m % 3],
                              act[m % 3], first);
        }
        T kv[16];
        const T* kbk = a.Kval + 16 * (size_t)pos;
#pragma unroll
        for (int m = 0; m < 16; ++m) kv[m] = kbk[m];
        V rel{};
        if (COARSE) rel = a.node_rel[l];
        block(l, rn, a.Dinv + 16 * (size_t)l, kv, rel);
    }
#pragma unroll
    for (int m = 0; m < 12; ++m) y[m] = row_sum(y[m]);
    if (lane == 0)
#pragma unroll
        for (int m = 0; m < 12; ++m) ys[row][m] = y[m];
    __syncthreads();

    // ---- own rows: u', w', partials of the new vectors
    T pc[kCgPart];
#pragma unroll
    for (int m = 0; m < kCgPart; ++m) pc[m] = 0;
    T bn[3] = {0, 0, 0};
    if (live && lane < 12) {
        const size_t o = 12 * (size_t)j + lane;
        const int c = lane % 3;
        V dj{};
        if (COARSE) dj = a.node_rel[j];
        T un;
        if (!START && shr) {
            un = us[rowl][lane];   // the row's own node in the shared table
        } else {
            T rrow[12], urow[12];
#pragma unroll
            for (int m = 0; m < 12; ++m) rrow[m] = rs[row][m];
            apply_dinv(a.Dinv + 16 * (size_t)j, rrow, urow);
            if (COARSE) prolong_add(dj, cco[(j - (int)pi.node_off) >> pi.agg_shift], urow);
            un = urow[0];
#pragma unroll
            for (int m = 1; m < 12; ++m)
                if (lane == m) un = urow[m];
        }
        const T wn = ys[row][lane];
        a.u[nxt][o] = un;
        a.w[nxt][o] = wn;
        const T rn = rs[row][lane];
        const T ru = rn * un, wu = wn * un, rr = rn * rn;
        // (compile-time register indices only: a lane-dependent index would
        // put the array in scratch memory)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            pc[cc] = c == cc ? ru : T(0);
            pc[3 + cc] = c == cc ? wu : T(0);
            pc[6 + cc] = c == cc ? rr : T(0);
        }
        if (COARSE) {
            // P_j^T w': rows 0..2 add d_j times the translation row
            const int q = lane / 3;
            T v = wn;
            if (q < 3) {
                const T dq = q == 0 ? dj.x : (q == 1 ? dj.y : dj.z);
                v = fma(dq, ys[row][9 + c], wn);
            }
#pragma unroll
            for (int m = 0; m < 12; ++m) pc[9 + m] = lane == m ? v : T(0);
        }
        if (START) {
            const T bv = a.bnorm ? a.bnorm[o] : own_r;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) bn[cc] = c == cc ? bv * bv : T(0);
        }
    }
#pragma unroll
    for (int m = 0; m < kCgPart; ++m)
        if (m < 9 || COARSE) pc[m] = wsum(pc[m]);
    if (START)
#pragma unroll
        for (int c = 0; c < 3; ++c) bn[c] = wsum(bn[c]);
    if ((tid & 63) == 63) {
#pragma unroll
        for (int m = 0; m < kCgPart; ++m) wp[tid >> 6][m] = pc[m];
        if (START)
#pragma unroll
            for (int c = 0; c < 3; ++c) bbw[tid >> 6][c] = bn[c];
    }
    __syncthreads();
    if (tid < kCgPart) {
        const int m = tid;
        const double v = (((double)wp[0][m] + (double)wp[1][m]) + (double)wp[2][m]) + (double)wp[3][m];
        a.part[nxt][(size_t)tile * kCgPart + m] = v;
    }
    if (START && tid < 3)
        a.part_bb[3 * (size_t)tile + tid] =
            (((double)bbw[0][tid] + (double)bbw[1][tid]) + (double)bbw[2][tid]) + (double)bbw[3][tid];
}

// Tile partials of P^T b into part[1][tile][9..20], read by the coarse start.
template <typename T>
__global__ void __launch_bounds__(64) k_cg_restrict(CgArgs<T> a) {
    __shared__ T sh[kNodeTile][12];
    const int tile = blockIdx.x;
    const int4 td = a.nd_tiles[tile];
    if (!(a.dyn[td.x].flags & PF_SOLVE)) return;
    const int tid = threadIdx.x;
    const int row = tid >> 2, q = tid & 3;
    const int j = td.y + row;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T v = 0;
        if (j < td.z) {
            const size_t o = 12 * (size_t)j;
            v = a.b[o + 3 * q + c];
            if (q < 3) {
                const auto d = a.node_rel[j];
                const T dq = q == 0 ? d.x : (q == 1 ? d.y : d.z);
                v = fma(dq, a.b[o + 9 + c], v);
            }
        }
        sh[row][3 * q + c] = v;
    }
    __syncthreads();
    if (tid < 12) {
        double acc = 0;
        for (int r = 0; r < kNodeTile; ++r) acc += (double)sh[r][tid];
        a.part[1][(size_t)tile * kCgPart + 9 + tid] = acc;
    }
}

// A_c = P^T K P in two passes.  Pass 1, per solver tile: the contribution
// P_j^T K_jl P_l of every K block of the tile's rows, summed per coarse
// column aggregate of l (the tile's aggregate list gives the slots), in a
// fixed order.  Pass 2, per aggregate: the sum of its tiles' slots.
template <typename T>
__global__ void __launch_bounds__(256) k_coarse_tiles(CoarseArgs<T> a) {
    using V = typename V4Of<T>::type;
    __shared__ double contrib[256][17];   // padded against bank conflicts
    __shared__ int slot_of[256];
    __shared__ int kp[kNodeTile + 1];
    __shared__ int list[kCoarseMaxAgg];
    const int tile = blockIdx.x;
    const int4 td = a.nd_tiles[tile];
    const int p = td.x;
    if (!(a.dyn[p].flags & PF_SOLVE)) return;
    const PairInfo& pi = a.info[p];
    const int tid = threadIdx.x;
    const int nrow = td.z - td.y;
    if (tid <= nrow) kp[tid] = a.K_ptr[td.y + tid];
    const int q0 = a.tile_agg_ptr[tile], ns = a.tile_agg_ptr[tile + 1] - q0;
    if (tid < ns) list[tid] = a.tile_agg[q0 + tid];
    __syncthreads();
    const int e0 = kp[0], e1 = kp[nrow];
    // (slot, entry m) pairs owned by this thread: tid and tid + 256
    double acc0 = 0, acc1 = 0;
    for (int base = e0; base < e1; base += 256) {
        const int e = base + tid;
        int sl = -1;
        if (e < e1) {
            int r = 0;
            while (kp[r + 1] <= e) ++r;
            const int j = td.y + r;
            const int l = a.K_col[e];
            const int al = (l - (int)pi.node_off) >> pi.agg_shift;
            sl = 0;
            while (list[sl] != al) ++sl;
            const V dj = a.node_rel[j];
            const V dl = a.node_rel[l];
            const T* kb = a.Kval + 16 * (size_t)e;
            double kpm[16];
            // K P_l: column m < 3 gains K[q][3] d_l[m]
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double k3 = (double)kb[4 * q + 3];
                kpm[4 * q + 0] = (double)kb[4 * q + 0] + k3 * (double)dl.x;
                kpm[4 * q + 1] = (double)kb[4 * q + 1] + k3 * (double)dl.y;
                kpm[4 * q + 2] = (double)kb[4 * q + 2] + k3 * (double)dl.z;
                kpm[4 * q + 3] = k3;
            }
            // P_j^T (K P_l): row q < 3 gains d_j[q] times row 3
            const double djv[3] = {(double)dj.x, (double)dj.y, (double)dj.z};
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int m = 0; m < 4; ++m) contrib[tid][4 * q + m] = kpm[4 * q + m] + djv[q] * kpm[12 + m];
#pragma unroll
            for (int m = 0; m < 4; ++m) contrib[tid][12 + m] = kpm[12 + m];
        }
        slot_of[tid] = sl;
        __syncthreads();
        const int cnt = min(256, e1 - base);
        for (int h = 0; h < 2; ++h) {
            const int o = tid + 256 * h;
            const int s2 = o >> 4, m = o & 15;
            if (s2 < ns) {
                // entries in order; one of another slot adds +0.0, which
                // leaves the sum's bits as skipping it would (the sum only
                // reaches acc0/acc1, which never hold -0), and lets eight
                // reads be in flight together
                double v = 0;
                int t = 0;
                for (; t + 8 <= cnt; t += 8) {
                    double x[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const double c = contrib[t + u][m];
                        x[u] = slot_of[t + u] == s2 ? c : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) v += x[u];
                }
                for (; t < cnt; ++t) {
                    const double c = contrib[t][m];
                    v += slot_of[t] == s2 ? c : 0.0;
                }
                if (h == 0) acc0 += v;
                else acc1 += v;
            }
        }
        __syncthreads();
    }
    double* out = a.Ac_tile + (size_t)tile * kCoarseMaxAgg * 16;
    if ((tid >> 4) < ns) out[tid] = acc0;
    if (((tid + 256) >> 4) < ns) out[tid + 256] = acc1;
}

template <typename T>
__global__ void __launch_bounds__(256) k_coarse_sum(CoarseArgs<T> a) {
    constexpr int MT = 64;   // tiles staged per pass
    __shared__ int lst[MT][kCoarseMaxAgg + 1];   // [0] = count, then the aggregates
    const int4 ag = a.aggs[blockIdx.x];   // pair, first node, end node, local id
    const int p = ag.x;
    if (!(a.dyn[p].flags & PF_SOLVE)) return;
    const PairInfo& pi = a.info[p];
    const int nc = 4 * pi.nagg;
    const int t_first = pi.nd_tile0 + ((ag.y - (int)pi.node_off) >> 4);
    const int t_end = pi.nd_tile0 + ((ag.z - (int)pi.node_off + kNodeTile - 1) >> 4);
    double acc0 = 0, acc1 = 0;   // outputs tid and tid + 256
    for (int tb = t_first; tb < t_end; tb += MT) {
        const int nt = min(MT, t_end - tb);
        for (int o = threadIdx.x; o < nt * (kCoarseMaxAgg + 1); o += 256) {
            const int t = o / (kCoarseMaxAgg + 1), q = o - t * (kCoarseMaxAgg + 1);
            const int q0 = a.tile_agg_ptr[tb + t], cnt = a.tile_agg_ptr[tb + t + 1] - q0;
            lst[t][q] = q == 0 ? cnt : (q <= cnt ? a.tile_agg[q0 + q - 1] : -1);
        }
        __syncthreads();
        for (int h = 0; h < 2; ++h) {
            const int o = threadIdx.x + 256 * h;
            if (o >= pi.nagg * 16) continue;
            const int b = o >> 4, m = o & 15;
            // unrolled so that the tiles' loads are in flight together; a tile
            // without a slot for b adds +0.0, which leaves the sum's bits alone
            // (it starts at +0 and an in-order sum never turns into -0)
            double v = 0;
#pragma unroll 8
            for (int t = 0; t < nt; ++t) {
                const int cnt = lst[t][0];
                int sl = -1;
                for (int s2 = 0; s2 < cnt; ++s2)
                    if (sl < 0 && lst[t][1 + s2] == b) sl = s2;
                const double x = sl >= 0 ? a.Ac_tile[(size_t)(tb + t) * kCoarseMaxAgg * 16 + 16 * sl + m] : 0.0;
                v += x;
            }
            if (h == 0) acc0 += v;
            else acc1 += v;
        }
        __syncthreads();
    }
    double* out = a.Ac + pi.ainv_off;
    for (int h = 0; h < 2; ++h) {
        const int o = threadIdx.x + 256 * h;
        if (o >= pi.nagg * 16) continue;
        const int b = o >> 4, m = o & 15, q = m >> 2, mm = m & 3;
        out[(size_t)(4 * ag.w + q) * nc + 4 * b + mm] = h == 0 ? acc0 : acc1;
    }
}

template <typename T>
__global__ void __launch_bounds__(kCinvThreads) k_coarse_invert(CoarseArgs<T> a) {
    const int p = blockIdx.x;
    if (!(a.dyn[p].flags & PF_SOLVE)) return;
    const PairInfo& pi = a.info[p];
    coarse_invert_mfma<T>(a.Ac + pi.ainv_off, a.Ainv + pi.ainv_off, pi.nagg);
}

template <typename T>
void launch_cg_init(const CgArgs<T>& a, int n_nd_tiles, hipStream_t s, KernelTimer* tm) {
    if (tm) tm->begin("cg_init", s);
    if (a.coarse) {
        hipLaunchKernelGGL(k_cg_restrict<T>, dim3(n_nd_tiles), dim3(4 * kNodeTile), 0, s, a);
        hipLaunchKernelGGL((k_cg<T, true, true>), dim3(n_nd_tiles), dim3(kCgThreads), 0, s, a, -1);
    } else {
        hipLaunchKernelGGL((k_cg<T, false, true>), dim3(n_nd_tiles), dim3(kCgThreads), 0, s, a, -1);
    }
    if (tm) tm->end(s);
}

template <typename T>
void launch_cg_iter(const CgArgs<T>& a, int n_nd_tiles, int it, hipStream_t s, KernelTimer* tm) {
    if (a.coarse)
        launch_one(tm, "cg_step", k_cg<T, true, false>, dim3(n_nd_tiles), dim3(kCgThreads), s, a, it);
    else
        launch_one(tm, "cg_step", k_cg<T, false, false>, dim3(n_nd_tiles), dim3(kCgThreads), s, a, it);
}

template <typename T>
void launch_coarse(const CoarseArgs<T>& a, int n_nd_tiles, int64_t nagg, int P, hipStream_t s, KernelTimer* tm) {
    if (tm) tm->begin("coarse_matrix", s);
    hipLaunchKernelGGL(k_coarse_tiles<T>, dim3(n_nd_tiles), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_coarse_sum<T>, dim3((unsigned)nagg), dim3(256), 0, s, a);
    if (tm) tm->end(s);
    if (tm) tm->begin("coarse_invert", s);
    hipLaunchKernelGGL(k_coarse_invert<T>, dim3(P), dim3(kCinvThreads), 0, s, a);
    if (tm) tm->end(s);
}

#define AMM_CG_INSTANTIATE(T)                                                                    \
    template void launch_cg_init<T>(const CgArgs<T>&, int, hipStream_t, KernelTimer*);           \
    template void launch_cg_iter<T>(const CgArgs<T>&, int, int, hipStream_t, KernelTimer*);      \
    template void launch_coarse<T>(const CoarseArgs<T>&, int, int64_t, int, hipStream_t, KernelTimer*);

AMM_CG_INSTANTIATE(float)
AMM_CG_INSTANTIATE(double)

}  // namespace amm
