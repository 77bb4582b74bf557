// Inverse of each pair's coarse matrix A_c (the aggregates' affine block of
// the two-level preconditioner), in float64 on the FP64 matrix cores.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "amm_internal.h"

namespace amm {

// Inverse of a symmetric positive definite 4x4 matrix (lower triangle of K
// read) by its 2x2 block partition [[A, B], [B^T, D]]: with the Schur
// complement S = D - B^T A^-1 B, the inverse is
//   [[A^-1 + A^-1 B S^-1 B^T A^-1, -A^-1 B S^-1], [-S^-1 B^T A^-1, S^-1]].
// False when A or S is not positive definite in floating point.
__device__ __forceinline__ bool spd_inverse4_schur(const double K[4][4], double out[16]) {
    const double a = K[0][0], b = K[1][0], c = K[1][1];
    const double da = a * c - b * b;
    bool ok = a > 0.0 && da > 0.0;
    const double ia = 1.0 / da;
    const double a00 = c * ia, a01 = -b * ia, a11 = a * ia;          // A^-1
    const double b00 = K[2][0], b01 = K[3][0], b10 = K[2][1], b11 = K[3][1];   // B = K[0:2][2:4]
    const double g00 = a00 * b00 + a01 * b10, g01 = a00 * b01 + a01 * b11;     // G = A^-1 B
    const double g10 = a01 * b00 + a11 * b10, g11 = a01 * b01 + a11 * b11;
    const double s00 = K[2][2] - (b00 * g00 + b10 * g10);
    const double s01 = K[3][2] - (b00 * g01 + b10 * g11);
    const double s11 = K[3][3] - (b01 * g01 + b11 * g11);
    const double ds = s00 * s11 - s01 * s01;
    ok = ok && s00 > 0.0 && ds > 0.0;
    const double is = 1.0 / ds;
    const double t00 = s11 * is, t01 = -s01 * is, t11 = s00 * is;    // S^-1
    const double h00 = g00 * t00 + g01 * t01, h01 = g00 * t01 + g01 * t11;     // H = G S^-1
    const double h10 = g10 * t00 + g11 * t01, h11 = g10 * t01 + g11 * t11;
    out[0] = a00 + (h00 * g00 + h01 * g01);
    out[1] = a01 + (h00 * g10 + h01 * g11);
    out[5] = a11 + (h10 * g10 + h11 * g11);
    out[4] = out[1];
    out[2] = -h00;
    out[3] = -h01;
    out[6] = -h10;
    out[7] = -h11;
    out[8] = -h00;
    out[9] = -h10;
    out[12] = -h01;
    out[13] = -h11;
    out[10] = t00;
    out[11] = t01;
    out[14] = t01;
    out[15] = t11;
    return ok;
}

typedef double cinv_d4 __attribute__((ext_vector_type(4)));

constexpr int kCinvOrder = 4 * kCoarseMaxAgg;   // largest coarse order
constexpr int kCinvTiles = kCinvOrder / 16;  // tiles per side at the largest order
constexpr int kCinvThreads = 64 * kCinvTiles;

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

// Publish rows and columns k0 .. k0 + 3 (k0 = 16 tk + 4 S) to LDS.
template <int S>
__device__ __forceinline__ void cinv_publish(const cinv_d4 (&acc)[kCinvTiles], const CinvLane& L, int tk,
                                             double (*rowK)[kCinvOrder], double (*colK)[4]) {
    if (!L.active) return;
    if (L.ti == tk) {
#pragma unroll
        for (int t = 0; t < kCinvTiles; ++t) {
            const int col = 16 * t + L.lr;
            if (t < L.m && col < L.nc) rowK[L.lq][col] = acc[t][S];
        }
    }
#pragma unroll
    for (int t = 0; t < kCinvTiles; ++t) {
        if (t != tk || (L.lr >> 2) != S) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * L.ti + 4 * r + L.lq;
            if (row < L.nc) colK[row][L.lr & 3] = acc[t][r];
        }
    }
}

// One Gauss-Jordan step on pivot block K = 4 tk + S (k0 = 4 K), with the
// rows and columns k0 .. k0 + 3 as they were before the step in rowK/colK.
// With P = A[K][K]:
//   A[K][K] = P^-1,  A[K][J] = P^-1 A[K][J],  A[I][K] = -A[I][K] P^-1,
//   A[I][J] -= A[I][K] P^-1 A[K][J],
// as one rank-4 product A <- A~ + L R per tile, where L holds -A[I][K] P^-1
// in the rows I != K and P^-1 in the pivot rows, R holds A[K][J] in the
// columns J != K and the identity in the pivot columns, and A~ is A with the
// pivot rows and columns cleared.  Every wave forms P^-1 itself (same inputs,
// same result).  Returns false when P is not positive definite.
template <int S>
__device__ __forceinline__ bool cinv_step(cinv_d4 (&acc)[kCinvTiles], const CinvLane& L, int tk,
                                          const double (*rowK)[kCinvOrder], const double (*colK)[4]) {
    const int k0 = 16 * tk + 4 * S;
    double Kb[4][4], Pv[16];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q <= r; ++q) Kb[r][q] = rowK[r][k0 + q];
    bool ok = spd_inverse4_schur(Kb, Pv);
#pragma unroll
    for (int e = 0; e < 16; ++e) ok = ok && fabs(Pv[e]) < 1e300;
    if (!L.active) return ok;
    // column lq of P^-1
    double pc[4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
        pc[p] = L.lq == 0 ? Pv[4 * p] : (L.lq == 1 ? Pv[4 * p + 1] : (L.lq == 2 ? Pv[4 * p + 2] : Pv[4 * p + 3]));
    // left operand: element (lr, lq) of this tile row's L
    const int arow = 16 * L.ti + L.lr;
    double av = 0.0;
    if (L.ti == tk && (L.lr >> 2) == S) {
        const int q = L.lr & 3;
        av = q == 0 ? pc[0] : (q == 1 ? pc[1] : (q == 2 ? pc[2] : pc[3]));
    } else if (arow < L.nc) {
        av = -(colK[arow][0] * pc[0] + colK[arow][1] * pc[1] + colK[arow][2] * pc[2] + colK[arow][3] * pc[3]);
    }
#pragma unroll
    for (int t = 0; t < kCinvTiles; ++t) {
        if (t >= L.m) continue;   // uniform over the wave
        const bool pcol = t == tk && (L.lr >> 2) == S;
        const int bcol = 16 * t + L.lr;
        const double bv = pcol ? (L.lq == (L.lr & 3) ? 1.0 : 0.0) : (bcol < L.nc ? rowK[L.lq][bcol] : 0.0);
        cinv_d4 c = acc[t];
        if (pcol) c = cinv_d4{0.0, 0.0, 0.0, 0.0};
        if (L.ti == tk) c[S] = 0.0;
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c, 0, 0, 0);
    }
    return ok;
}

// In-place block Gauss-Jordan inversion of one symmetric positive definite
// matrix of order 4 nagg (nagg <= kCoarseMaxAgg; no pivoting: every pivot
// block is a Schur complement of an SPD matrix), pivoting on one 4x4
// diagonal block at a time, by one block of kCinvThreads threads.  `in` is
// read, `out` written (row-major, order 4 nagg); a pivot block that is not
// positive definite in floating point writes an all-zero inverse.  One
// barrier per step: rows and columns of consecutive steps go to alternating
// LDS buffers.
template <typename T>
__device__ __forceinline__ void coarse_invert_mfma(const double* __restrict__ in, T* __restrict__ out,
                                                   int nagg) {
    __shared__ double rowK[2][4][kCinvOrder];
    __shared__ double colK[2][kCinvOrder][4];
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
    cinv_d4 acc[kCinvTiles];
#pragma unroll
    for (int t = 0; t < kCinvTiles; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * L.ti + 4 * r + L.lq, col = 16 * t + L.lr;
            acc[t][r] = L.active && t < L.m && row < L.nc && col < L.nc ? in[(size_t)row * L.nc + col] : 0.0;
        }
    if (threadIdx.x == 0) bad = 0;
    cinv_publish<0>(acc, L, 0, rowK[0], colK[0]);
    for (int tk = 0; tk < L.m; ++tk) {
#define AMM_CINV_SUBSTEP(S)                                                              \
        {                                                                                \
            const int K = 4 * tk + (S);                                                  \
            if (K >= nagg) break;                                                        \
            const int b = K & 1;                                                         \
            __syncthreads();                                                             \
            const bool ok = cinv_step<S>(acc, L, tk, rowK[b], colK[b]);                  \
            if (!ok && threadIdx.x == 0) bad = 1;                                        \
            if (K + 1 < nagg) {                                                          \
                if ((S) < 3)                                                             \
                    cinv_publish<((S) + 1) & 3>(acc, L, tk, rowK[b ^ 1], colK[b ^ 1]);   \
                else                                                                     \
                    cinv_publish<0>(acc, L, tk + 1, rowK[b ^ 1], colK[b ^ 1]);           \
            }                                                                            \
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
