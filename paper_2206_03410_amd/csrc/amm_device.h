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

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
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
