// Inverse of each pair's coarse matrix A_c (the aggregates' affine block of
// the two-level preconditioner), in float64 on the FP64 matrix cores.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "amm_internal.h"

namespace amm {

typedef double cinv_d4 __attribute__((ext_vector_type(4)));

constexpr int kCinvOrder = 4 * kCoarseMaxAgg;   // largest coarse order
constexpr int kCinvTiles = kCinvOrder / 16;  // tiles per side at the largest order
constexpr int kCinvThreads = 64 * (kCinvTiles + 1);   // tile rows + the pivot wave

// The matrix, zero-padded to order 16 m, is held as m x m tiles of 16 x 16
// in the accumulators of v_mfma_f64_16x16x4f64: lane l's value r of a tile
// is the tile's element (4 r + l / 16, l % 16).  Wave w owns tile row w, so
// the products of its tiles share one left operand.
struct CinvLane {
    int nc, m;        // order, tiles per side
    int ti;           // tile row
    int lr, lq;       // lane % 16, lane / 16
    bool active;      // the wave owns tiles
};

// Publish rows and columns k0 .. k0 + 3 (k0 = 16 tk + 4 S) to LDS and, when
// `dnext`, the diagonal block of the pivot after them (rows and columns
// k0 + 4 .. k0 + 7).  Tiles and tile entries past the order hold zero (they
// start at zero and every product adds zero to them; after a failed pivot
// the result is discarded anyway), so whole tile rows and columns are written.
template <int S>
__device__ __forceinline__ void cinv_publish(const cinv_d4 (&acc)[kCinvTiles], const CinvLane& L, int tk,
                                             bool dnext, double (*rowK)[kCinvOrder], double (*colK)[4],
                                             double (*dK)[4]) {
    if (!L.active) return;
    if (L.ti == tk) {
#pragma unroll
        for (int t = 0; t < kCinvTiles; ++t) rowK[L.lq][16 * t + L.lr] = acc[t][S];
    }
    constexpr int SD = (S + 1) & 3;
    const int tkd = S == 3 ? tk + 1 : tk;
#pragma unroll
    for (int t = 0; t < kCinvTiles; ++t) {
        if (t == tk && (L.lr >> 2) == S) {   // t == tk is uniform over the block
#pragma unroll
            for (int r = 0; r < 4; ++r) colK[16 * L.ti + 4 * r + L.lq][L.lr & 3] = acc[t][r];
        }
        if (dnext && t == tkd && L.ti == tkd && (L.lr >> 2) == SD) dK[L.lq][L.lr & 3] = acc[t][SD];
    }
}

// Inverse of a symmetric 4x4 pivot block (lower triangle of m read) as its
// adjugate over its determinant, both from the 2x2 minors of rows 0-1 (s)
// and rows 2-3 (c) (Laplace expansion along the first two rows): a short
// dependency chain with one division.  The block is positive definite when
// its leading principal minors m00, s0, the leading 3x3 minor and the
// determinant are positive (Sylvester's criterion); false otherwise or when
// the inverse is not finite.
__host__ __device__ __forceinline__ bool cinv_pivot_inverse(const double m[4][4], double out[16]) {
    const double m00 = m[0][0], m10 = m[1][0], m11 = m[1][1], m20 = m[2][0], m21 = m[2][1];
    const double m22 = m[2][2], m30 = m[3][0], m31 = m[3][1], m32 = m[3][2], m33 = m[3][3];
    // rows 0-1 minors (m01 = m10, m02 = m20, m03 = m30, m12 = m21, m13 = m31)
    const double s0 = m00 * m11 - m10 * m10, s1 = m00 * m21 - m20 * m10, s2 = m00 * m31 - m30 * m10;
    const double s3 = m10 * m21 - m20 * m11, s4 = m10 * m31 - m30 * m11, s5 = m20 * m31 - m30 * m21;
    // rows 2-3 minors (m23 = m32)
    const double c0 = m20 * m31 - m21 * m30, c1 = m20 * m32 - m22 * m30, c2 = m20 * m33 - m32 * m30;
    const double c3 = m21 * m32 - m22 * m31, c4 = m21 * m33 - m32 * m31, c5 = m22 * m33 - m32 * m32;
    const double det = (s0 * c5 - s1 * c4) + (s2 * c3 + s3 * c2) + (s5 * c0 - s4 * c1);
    // adjugate, lower triangle
    const double a00 = m11 * c5 - m21 * c4 + m31 * c3;
    const double a10 = -m10 * c5 + m21 * c2 - m31 * c1;
    const double a11 = m00 * c5 - m20 * c2 + m30 * c1;
    const double a20 = m10 * c4 - m11 * c2 + m31 * c0;
    const double a21 = -m00 * c4 + m10 * c2 - m30 * c0;
    const double a22 = m30 * s4 - m31 * s2 + m33 * s0;
    const double a30 = -m10 * c3 + m11 * c1 - m21 * c0;
    const double a31 = m00 * c3 - m10 * c1 + m20 * c0;
    const double a32 = -m30 * s3 + m31 * s1 - m32 * s0;
    const double a33 = m20 * s3 - m21 * s1 + m22 * s0;   // the leading 3x3 minor
    const double id = 1.0 / det;
    out[0] = a00 * id;
    out[4] = out[1] = a10 * id;
    out[5] = a11 * id;
    out[8] = out[2] = a20 * id;
    out[9] = out[6] = a21 * id;
    out[10] = a22 * id;
    out[12] = out[3] = a30 * id;
    out[13] = out[7] = a31 * id;
    out[14] = out[11] = a32 * id;
    out[15] = a33 * id;
    bool ok = m00 > 0.0 && s0 > 0.0 && a33 > 0.0 && det > 0.0;
#pragma unroll
    for (int e = 0; e < 16; ++e) ok = ok && fabs(out[e]) < 1e300;
    return ok;
}

// One Gauss-Jordan step on pivot block K = 4 tk + S (k0 = 4 K), with the
// rows and columns k0 .. k0 + 3 as they were before the step in rowK/colK
// and the pivot block's inverse in piK.  With P = A[K][K]:
//   A[K][K] = P^-1,  A[K][J] = P^-1 A[K][J],  A[I][K] = -A[I][K] P^-1,
//   A[I][J] -= A[I][K] P^-1 A[K][J],
// as one rank-4 product A <- A~ + L R per tile, where L holds -A[I][K] P^-1
// in the rows I != K and P^-1 in the pivot rows, R holds A[K][J] in the
// columns J != K and the identity in the pivot columns, and A~ is A with the
// pivot rows and columns cleared.
template <int S>
__device__ __forceinline__ void cinv_step(cinv_d4 (&acc)[kCinvTiles], const CinvLane& L, int tk,
                                          const double (*rowK)[kCinvOrder], const double (*colK)[4],
                                          const double* piK) {
    // every operand read up front (entries past the order are zero)
    double bk[kCinvTiles];
#pragma unroll
    for (int t = 0; t < kCinvTiles; ++t) bk[t] = rowK[L.lq][16 * t + L.lr];
    const int arow = 16 * L.ti + L.lr;
    const double c0 = colK[arow][0], c1 = colK[arow][1], c2 = colK[arow][2], c3 = colK[arow][3];
    const int q = L.lr & 3;
    // column lq of P^-1, and element (q, lq)
    const double p0 = piK[L.lq], p1 = piK[4 + L.lq], p2 = piK[8 + L.lq], p3 = piK[12 + L.lq];
    const double pq = piK[4 * q + L.lq];
    // left operand: element (lr, lq) of this tile row's L
    const bool prow = L.ti == tk && (L.lr >> 2) == S;
    const double av = prow ? pq : -(c0 * p0 + c1 * p1 + c2 * p2 + c3 * p3);
#pragma unroll
    for (int t = 0; t < kCinvTiles; ++t) {
        if (t >= L.m) continue;   // uniform over the wave
        const bool pcol = t == tk && (L.lr >> 2) == S;
        const double bv = pcol ? (L.lq == q ? 1.0 : 0.0) : bk[t];
        cinv_d4 c = acc[t];
        if (pcol) c = cinv_d4{0.0, 0.0, 0.0, 0.0};
        if (L.ti == tk) c[S] = 0.0;
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c, 0, 0, 0);
    }
}

// The pivot block after step K (rows and columns k1 .. k1 + 3, k1 = k0 + 4),
// A[K+1][K+1] - A[K+1][K] P^-1 A[K][K+1], from that block before the step
// (dK), the step's rows and columns and P^-1 (Pv); its inverse replaces Pv.
// Every LDS read is issued before the arithmetic that needs it.
__device__ __forceinline__ bool cinv_next_pivot(int k1, const double (*rowK)[kCinvOrder],
                                                const double (*colK)[4], const double (*dK)[4],
                                                double (&Pv)[16]) {
    double C[4][4], R[4][4], D[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            C[i][j] = colK[k1 + i][j];
            R[i][j] = rowK[i][k1 + j];
            D[i][j] = dK[i][j];
        }
    double G[4][4];   // A[K+1][K] P^-1
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            G[i][j] = (C[i][0] * Pv[j] + C[i][1] * Pv[4 + j]) + (C[i][2] * Pv[8 + j] + C[i][3] * Pv[12 + j]);
    double Kn[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            Kn[i][j] = D[i][j] - ((G[i][0] * R[0][j] + G[i][1] * R[1][j]) + (G[i][2] * R[2][j] + G[i][3] * R[3][j]));
    return cinv_pivot_inverse(Kn, Pv);
}

// In-place block Gauss-Jordan inversion of one symmetric positive definite
// matrix of order 4 nagg (nagg <= kCoarseMaxAgg; no pivoting: every pivot
// block is a Schur complement of an SPD matrix), pivoting on one 4x4
// diagonal block at a time, by one block of kCinvThreads threads.  `in` is
// read, `out` written (row-major, order 4 nagg); a pivot block that is not
// positive definite in floating point writes an all-zero inverse.
// One barrier per step: rows, columns and pivot inverses of consecutive steps
// go to alternating LDS buffers.  The tile-row waves apply step K while the
// last wave forms the pivot inverse of step K + 1 from the same buffers.
template <typename T>
__device__ __forceinline__ void coarse_invert_mfma(const double* __restrict__ in, T* __restrict__ out,
                                                   int nagg) {
    __shared__ double rowK[2][4][kCinvOrder];
    __shared__ double colK[2][kCinvOrder][4];
    __shared__ double dK[2][4][4];
    __shared__ double piK[2][16];
    __shared__ int bad;
    if (nagg <= 0 || nagg > kCoarseMaxAgg) return;
    CinvLane L;
    L.nc = 4 * nagg;
    L.m = (L.nc + 15) >> 4;
    const int l = threadIdx.x & 63;
    L.lr = l & 15;
    L.lq = l >> 4;
    L.ti = threadIdx.x >> 6;
    L.active = L.ti < L.m;
    if (threadIdx.x == 0) bad = 0;
    // zero both buffers: entries past the order are read as operands
    for (int e = threadIdx.x; e < 2 * 4 * kCinvOrder; e += kCinvThreads) {
        (&rowK[0][0][0])[e] = 0.0;
        (&colK[0][0][0])[e] = 0.0;
    }
    // Both roles below pass the same barriers: one here, one after the first
    // publication, one per pivot step and one at the end.
    if (L.ti == kCinvTiles) {
        // the pivot wave: inverse of pivot 0, then during step K that of K + 1
        __syncthreads();
        __syncthreads();
        double Pn[16];
        {
            double Kb[4][4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int q = 0; q <= r; ++q) Kb[r][q] = rowK[0][r][q];
            const bool ok = cinv_pivot_inverse(Kb, Pn);
            if (l == 0) {
#pragma unroll
                for (int e = 0; e < 16; ++e) piK[0][e] = Pn[e];
                if (!ok) bad = 1;
            }
        }
        for (int K = 0; K < nagg; ++K) {
            const int b = K & 1;
            __syncthreads();
            if (K + 1 < nagg) {
                const bool ok = cinv_next_pivot(4 * K + 4, rowK[b], colK[b], dK[b], Pn);
                if (l == 0) {
#pragma unroll
                    for (int e = 0; e < 16; ++e) piK[b ^ 1][e] = Pn[e];
                    if (!ok) bad = 1;
                }
            }
        }
        __syncthreads();
        return;
    }
    cinv_d4 acc[kCinvTiles];
#pragma unroll
    for (int t = 0; t < kCinvTiles; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * L.ti + 4 * r + L.lq, col = 16 * t + L.lr;
            acc[t][r] = L.active && t < L.m && row < L.nc && col < L.nc ? in[(size_t)row * L.nc + col] : 0.0;
        }
    __syncthreads();
    cinv_publish<0>(acc, L, 0, nagg > 1, rowK[0], colK[0], dK[0]);
    __syncthreads();
    for (int tk = 0; tk < L.m; ++tk) {
#define AMM_CINV_SUBSTEP(S)                                                                       \
        {                                                                                         \
            const int K = 4 * tk + (S);                                                           \
            if (K >= nagg) break;                                                                 \
            const int b = K & 1;                                                                  \
            __syncthreads();                                                                      \
            if (L.active) {                                                                       \
                cinv_step<S>(acc, L, tk, rowK[b], colK[b], piK[b]);                               \
                if (K + 1 < nagg) {                                                               \
                    if ((S) < 3)                                                                  \
                        cinv_publish<((S) + 1) & 3>(acc, L, tk, K + 2 < nagg, rowK[b ^ 1],        \
                                                    colK[b ^ 1], dK[b ^ 1]);                      \
                    else                                                                          \
                        cinv_publish<0>(acc, L, tk + 1, K + 2 < nagg, rowK[b ^ 1], colK[b ^ 1],   \
                                        dK[b ^ 1]);                                               \
                }                                                                                 \
            }                                                                                     \
        }
        AMM_CINV_SUBSTEP(0)
        AMM_CINV_SUBSTEP(1)
        AMM_CINV_SUBSTEP(2)
        AMM_CINV_SUBSTEP(3)
#undef AMM_CINV_SUBSTEP
    }
    __syncthreads();
    if (!L.active) return;
    const bool zero = bad != 0;
#pragma unroll
    for (int t = 0; t < kCinvTiles; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * L.ti + 4 * r + L.lq, col = 16 * t + L.lr;
            if (t < L.m && row < L.nc && col < L.nc)
                out[(size_t)row * L.nc + col] = zero ? T(0) : (T)acc[t][r];
        }
}

}  // namespace amm
