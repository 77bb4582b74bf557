// Device helpers shared by the kernel translation units (internal).
#pragma once

#include <hip/hip_runtime.h>

namespace amm {


template <typename T> __device__ __forceinline__ T dev_inf();
template <> __device__ __forceinline__ float dev_inf<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double dev_inf<double>() { return __builtin_inf(); }

// Maps block b of G to a tile so that each of the 8 XCDs (blocks are
// dispatched round-robin over XCDs) works on one contiguous range of tiles,
// which keeps the target data a range touches inside one XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
    const int per = G >> 3, rem = G & 7;
    const int x = b & 7, q = b >> 3;
    return x * per + min(x, rem) + q;
}

template <typename T, int NT>
__device__ __forceinline__ T block_sum(T v, T* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    T r = sh[0];
    __syncthreads();
    return r;
}

template <typename T, int NT>
__device__ __forceinline__ T block_max(T v, T* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    T r = sh[0];
    __syncthreads();
    return r;
}


// Cross-lane moves by DPP (a modifier of ordinary VALU moves: no LDS round
// trip, unlike the permutes behind __shfl_xor).  CTRL: 0xB1 quad_perm
// [1,0,3,2], 0x4E quad_perm [2,3,0,1], 0x141 row_half_mirror, 0x140
// row_mirror, 0x142 row_bcast:15, 0x143 row_bcast:31.  Rows outside RMASK
// (and lanes without a source) receive 0.
template <int CTRL, int RMASK = 0xf>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, RMASK, 0xf, false));
}
template <int CTRL, int RMASK = 0xf>
__device__ __forceinline__ double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, RMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, RMASK, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over each aligned group of 4 lanes, in all 4 (fixed order).
template <typename T>
__device__ __forceinline__ T quad_sum(T v) {
    v += dpp_mov<0xB1>(v);
    return v + dpp_mov<0x4E>(v);
}

// Sum over each row of 16 lanes, in all 16 (fixed order per lane).
template <typename T>
__device__ __forceinline__ T row_sum(T v) {
    v = quad_sum(v);
    v += dpp_mov<0x141>(v);
    return v + dpp_mov<0x140>(v);
}

// Sum over the 64 lanes of a wave, valid in lane 63 (fixed order).  Every
// lane of the wave must be active.
template <typename T>
__device__ __forceinline__ T wave_total63(T v) {
    v = row_sum(v);
    v += dpp_mov<0x142, 0xa>(v);
    return v + dpp_mov<0x143, 0xc>(v);
}

__device__ __forceinline__ float lane63(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double lane63(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes of a wave, in every lane (fixed order).  Every lane
// of the wave must be active.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    return lane63(wave_total63(v));
}

// Inverse of a symmetric positive definite 4x4 block through its Cholesky
// factor, fully unrolled.  Returns false on a non-positive pivot, and then
// writes the inverse of the diagonal instead.
template <typename T>
__device__ __forceinline__ bool spd_inverse4(const T K[4][4], T* out) {
    T L[4][4] = {};
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        T d = K[c][c];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < c) d -= L[c][q] * L[c][q];
        ok = ok && d > T(0);
        const T lc = sqrt(fmax(d, T(1e-300)));
        L[c][c] = lc;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r > c) {
                T v = K[r][c];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (q < c) v -= L[r][q] * L[c][q];
                L[r][c] = v / lc;
            }
    }
    // W = L^{-1} (lower triangular), then K^{-1} = W^T W
    T W[4][4] = {};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        W[c][c] = T(1) / L[c][c];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r > c) {
                T v = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (q >= c && q < r) v -= L[r][q] * W[q][c];
                W[r][c] = v / L[r][r];
            }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            T v = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) v += W[q][r] * W[q][c];
            out[4 * r + c] = ok ? v : (r == c ? T(1) / fmax(fabs(K[r][r]), T(1e-30)) : T(0));
        }
    return ok;
}

}  // namespace amm
