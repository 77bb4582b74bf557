// The target side of the closest-point structure built on the device, for a
// pair whose targets are replaced between solves (the frames of a sequence,
// Sec. 4): the same Morton order, sorted arrays and octree run-start tables
// as the host layout builds at set-up, bit for bit, so that replacing the
// targets costs a few kernels instead of a copy to the host, a sort there
// and an upload.
//
// Steps: bounding box (exact min / max per axis), 30-bit Morton codes of
// the coordinates quantized over it (the host's arithmetic: (p - lo) / ext
// scaled by 1023.999, floored and clamped), a stable radix sort of (code,
// index), the sorted targets and their user indices, and the run starts of
// every level: the leaf level by a binary search of each cell's first code
// among the sorted codes, coarser levels by sampling it.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <climits>
#include <cmath>
#include <cstring>
#include <string>

#include "amm_internal.h"

namespace amm {

namespace {

constexpr int kTT = 256;

inline int blocks(int64_t n) { return (int)((n + kTT - 1) / kTT); }

// float64 coordinates, non-finite flag and per-block bounds
template <typename In>
__global__ void __launch_bounds__(kTT) k_tl_load(const In* __restrict__ raw, int64_t M, double* __restrict__ xyz,
                                                 double* __restrict__ part, int* __restrict__ bad) {
    __shared__ double sh[6][kTT];
    const int64_t i = (int64_t)blockIdx.x * kTT + threadIdx.x;
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    if (i < M) {
        bool fin = true;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double x = (double)raw[3 * i + c];
            xyz[3 * i + c] = x;
            fin = fin && isfinite(x);
            v[c] = x;
            v[3 + c] = x;
        }
        if (!fin) atomicOr(bad, 1);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) sh[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int s = kTT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sh[c][threadIdx.x] = fmin(sh[c][threadIdx.x], sh[c][threadIdx.x + s]);
                sh[3 + c][threadIdx.x] = fmax(sh[3 + c][threadIdx.x], sh[3 + c][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[6 * (size_t)blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// bounds of the whole set from the block bounds (min and max are exact, so
// the order does not matter)
__global__ void __launch_bounds__(kTT) k_tl_box(const double* __restrict__ part, int nb, double* __restrict__ box) {
    __shared__ double sh[6][kTT];
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nb; b += kTT)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[c] = fmin(v[c], part[6 * (size_t)b + c]);
            v[3 + c] = fmax(v[3 + c], part[6 * (size_t)b + 3 + c]);
        }
#pragma unroll
    for (int c = 0; c < 6; ++c) sh[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int s = kTT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sh[c][threadIdx.x] = fmin(sh[c][threadIdx.x], sh[c][threadIdx.x + s]);
                sh[3 + c][threadIdx.x] = fmax(sh[3 + c][threadIdx.x], sh[3 + c][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) box[threadIdx.x] = sh[threadIdx.x][0];
}

__device__ __forceinline__ uint32_t spread10(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

struct Box6 {
    double lo[3], hi[3];
};

// Morton code of each target (x, y, z bits interleaved, x highest)
__global__ void __launch_bounds__(kTT) k_tl_codes(const double* __restrict__ xyz, int64_t M, Box6 b,
                                                  uint32_t* __restrict__ code, int* __restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * kTT + threadIdx.x;
    if (i >= M) return;
    uint32_t q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double ext = b.hi[c] - b.lo[c];
        // correctly rounded quotient and product (no contraction possible)
        const double t = ext > 0 ? __ddiv_rn(xyz[3 * i + c] - b.lo[c], ext) : 0.0;
        const int v = (int)floor(__dmul_rn(t, 1023.999));
        q[c] = (uint32_t)min(1023, max(0, v));
    }
    code[i] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    idx[i] = (int)i;
}

// sorted targets in both precisions (.w = user index) and user indices
__global__ void __launch_bounds__(kTT) k_tl_gather(const double* __restrict__ xyz, const int* __restrict__ ord,
                                                   int64_t M, float4* __restrict__ tf, double4* __restrict__ td,
                                                   int* __restrict__ user) {
    const int64_t q = (int64_t)blockIdx.x * kTT + threadIdx.x;
    if (q >= M) return;
    const int u = ord[q];
    const double x = xyz[3 * (size_t)u], y = xyz[3 * (size_t)u + 1], z = xyz[3 * (size_t)u + 2];
    const double w = (double)u;
    td[q] = make_double4(x, y, z, w);
    tf[q] = make_float4((float)x, (float)y, (float)z, (float)w);
    user[q] = u;
}

// leaf level: T_G[m] = number of targets whose leaf cell precedes m
__global__ void __launch_bounds__(kTT) k_tl_leaf(const uint32_t* __restrict__ code, int64_t M, int G,
                                                 int* __restrict__ tab) {
    const int64_t m = (int64_t)blockIdx.x * kTT + threadIdx.x;
    const int64_t nc = (int64_t)1 << (3 * G);
    if (m > nc) return;
    const int sh = 3 * (10 - G);
    int64_t lo = 0, hi = M;   // first position whose cell is >= m
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)(code[mid] >> sh) < m)
            lo = mid + 1;
        else
            hi = mid;
    }
    tab[m] = (int)lo;
}

// coarser levels: T_l[m] = T_G[m 8^(G - l)]
__global__ void __launch_bounds__(kTT) k_tl_levels(int* __restrict__ cells, int G) {
    const int64_t e = (int64_t)blockIdx.x * kTT + threadIdx.x;
    if (e >= oct_level_off(G)) return;
    int l = 0;
    while (oct_level_off(l + 1) <= e) ++l;
    const int64_t m = e - oct_level_off(l);
    cells[e] = cells[oct_level_off(G) + (m << (3 * (G - l)))];
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

amm_status device_target_layout(void* stream, DeviceTargetWork& w, bool f64, const void* tgt, int64_t M, int depth,
                                void* tgt_f4, void* tgt_d4, int32_t* tgt_user, int32_t* cells, TargetLayout& frame,
                                std::string& err) {
    hipStream_t s = (hipStream_t)stream;
    if (M <= 0 || M > INT32_MAX || depth < 2 || depth > kOctMaxDepth) {
        err = "device target layout: bad size or depth";
        return AMM_ERR_INVALID_ARG;
    }
    const int nb = blocks(M);
    size_t sort_bytes = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (const int*)nullptr, (int*)nullptr, (int)M, 0, 30, s) != hipSuccess) {
        err = "device target layout: sort size query failed";
        return AMM_ERR_HIP;
    }
    // xyz | block bounds | box + flag | codes x 2 | indices x 2 | sort temp
    const size_t o_part = align256(24 * (size_t)M);
    const size_t o_box = o_part + align256(48 * (size_t)nb);
    const size_t o_code = o_box + 256;
    const size_t o_code2 = o_code + align256(4 * (size_t)M);
    const size_t o_idx = o_code2 + align256(4 * (size_t)M);
    const size_t o_idx2 = o_idx + align256(4 * (size_t)M);
    const size_t o_tmp = o_idx2 + align256(4 * (size_t)M);
    const size_t need = o_tmp + align256(sort_bytes);
    if (w.bytes < need) {
        if (w.buf && hipFree(w.buf) != hipSuccess) {
            err = "device target layout: hipFree failed";
            return AMM_ERR_HIP;
        }
        w.buf = nullptr;
        w.bytes = 0;
        if (hipMalloc(&w.buf, need) != hipSuccess) {
            err = "device target layout: out of device memory";
            return AMM_ERR_OOM;
        }
        w.bytes = need;
    }
    char* base = (char*)w.buf;
    double* xyz = (double*)base;
    double* part = (double*)(base + o_part);
    double* box = (double*)(base + o_box);
    int* bad = (int*)(base + o_box + 64);
    uint32_t* code = (uint32_t*)(base + o_code);
    uint32_t* code2 = (uint32_t*)(base + o_code2);
    int* idx = (int*)(base + o_idx);
    int* idx2 = (int*)(base + o_idx2);
    void* tmp = base + o_tmp;
    auto ok = [&](hipError_t e, const char* what) {
        if (e == hipSuccess) return true;
        err = std::string("device target layout: ") + what + ": " + hipGetErrorString(e);
        return false;
    };
    if (!ok(hipMemsetAsync(bad, 0, sizeof(int), s), "flag clear")) return AMM_ERR_HIP;
    if (f64)
        hipLaunchKernelGGL(k_tl_load<double>, dim3(nb), dim3(kTT), 0, s, (const double*)tgt, M, xyz, part, bad);
    else
        hipLaunchKernelGGL(k_tl_load<float>, dim3(nb), dim3(kTT), 0, s, (const float*)tgt, M, xyz, part, bad);
    hipLaunchKernelGGL(k_tl_box, dim3(1), dim3(kTT), 0, s, part, nb, box);
    double hb[9];   // six bounds, one spare, the flag
    if (!ok(hipMemcpyAsync(hb, box, 64 + sizeof(int), hipMemcpyDeviceToHost, s), "bounds copy") ||
        !ok(hipStreamSynchronize(s), "bounds"))
        return AMM_ERR_HIP;
    int hbad = 0;
    std::memcpy(&hbad, reinterpret_cast<const char*>(hb) + 64, sizeof(int));
    if (hbad) {
        err = "non-finite target coordinate";
        return AMM_ERR_NONFINITE;
    }
    Box6 b;
    for (int c = 0; c < 3; ++c) {
        b.lo[c] = hb[c];
        b.hi[c] = hb[3 + c];
    }
    target_frame(b.lo, b.hi, frame);
    frame.grid_bits = depth;
    hipLaunchKernelGGL(k_tl_codes, dim3(nb), dim3(kTT), 0, s, xyz, M, b, code, idx);
    size_t tb = sort_bytes;
    if (!ok(hipcub::DeviceRadixSort::SortPairs(tmp, tb, code, code2, idx, idx2, (int)M, 0, 30, s), "sort"))
        return AMM_ERR_HIP;
    hipLaunchKernelGGL(k_tl_gather, dim3(nb), dim3(kTT), 0, s, xyz, idx2, M, (float4*)tgt_f4, (double4*)tgt_d4,
                       tgt_user);
    const int64_t nleaf = (int64_t)1 << (3 * depth);
    hipLaunchKernelGGL(k_tl_leaf, dim3(blocks(nleaf + 1)), dim3(kTT), 0, s, code2, M, depth,
                       cells + oct_level_off(depth));
    hipLaunchKernelGGL(k_tl_levels, dim3(blocks(oct_level_off(depth))), dim3(kTT), 0, s, cells, depth);
    if (!ok(hipGetLastError(), "launch")) return AMM_ERR_HIP;
    return AMM_OK;
}

}  // namespace amm
