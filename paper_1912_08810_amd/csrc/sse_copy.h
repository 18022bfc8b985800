// sse_copy.h -- asynchronous global -> LDS copies (gfx950's global_load_lds)
// used by the MFMA kernels to stage their G windows and A fragments, and the
// small exact division shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sse {

typedef __attribute__((address_space(3))) void lds_void;

// s_waitcnt immediate (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt in
// 6:4, lgkmcnt in 11:8) that waits for lgkmcnt to reach 0 (LDS and scalar
// memory) and leaves vmcnt and expcnt at their maxima, i.e. not waited for.
constexpr unsigned kWaitLgkm0 = 0xC07F;

// x / d for 0 <= x < 2^20 and 1 <= d < 2^11, rd = 1 / d within an ulp: the
// float product is within 2^20 (2^-23 + 2^-24) < 0.2 of x / d, so its
// truncation is off by at most one and a single correction makes it exact.
// (The integer division it replaces is a long instruction sequence on the GPU.)
__device__ __forceinline__ int small_div(int x, int d, float rd)
{
    int q = (int)((float)x * rd);
    const int r = x - q * d;
    q += (r >= d ? 1 : 0) - (r < 0 ? 1 : 0);
    return q;
}

// One lane's global -> LDS copy of U words (U = 4 or 1) to the wave's base d:
// lane i's data lands at d + i U words.
template <int U>
__device__ __forceinline__ void lds_copy(const void *src, uint32_t *d)
{
    if constexpr (U == 4)
        __builtin_amdgcn_global_load_lds(src, (lds_void *)d, 16, 0, 0);
    else
        __builtin_amdgcn_global_load_lds(src, (lds_void *)d, 4, 0, 0);
}

// Copy n units of U 32-bit words, unit u from src_of(u) to dst + u U words, by a
// workgroup of NT threads.  The copy engine writes each wave's 64 units
// contiguously, so the LDS base of a wave's instruction is wave-uniform.
// Completion is awaited with the vector-memory counter (a following
// __syncthreads() waits for it).
template <int U, int NT, typename SrcOf>
__device__ __forceinline__ void copy_to_lds(uint32_t *dst, int n, SrcOf src_of)
{
    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int base = 0; base < n; base += NT) {
        const int u = base + tid;
        uint32_t *d = dst + (size_t)(base + wv * 64) * U;
        if (u < n)
            lds_copy<U>(src_of(u), d);
    }
}

// Copy a window of nrow rows of rowW words into LDS at dst (NT threads): row r
// is energy ebase + r of a row sequence starting at g0 with stride strideW
// words per energy; rows outside [0, NE) come from zero (>= 16 zero bytes).
// Units of U words (rowW % U == 0) are walked incrementally (no division per
// unit).
template <int U, int NT>
__device__ __forceinline__ void copy_window(uint32_t *dst, const uint32_t *g0, int64_t strideW,
                                            int ebase, int NE, int nrow, int rowW,
                                            const uint32_t *zero)
{
    const int upr = rowW / U;
    const int n = nrow * upr;
    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const float rupr = __builtin_amdgcn_rcpf((float)upr);
    const int dr = small_div(NT, upr, rupr), dc = NT - dr * upr;
    int r = small_div(tid, upr, rupr), c = tid - r * upr;
    for (int base = 0; base < n; base += NT) {
        uint32_t *d = dst + (size_t)(base + wv * 64) * U;
        if (base + tid < n) {
            const int e = ebase + r;
            const uint32_t *src = (e >= 0 && e < NE) ? g0 + (int64_t)e * strideW + c * U : zero;
            lds_copy<U>(src, d);
        }
        r += dr;
        c += dc;
        if (c >= upr) {
            c -= upr;
            ++r;
        }
    }
}

}  // namespace sse
