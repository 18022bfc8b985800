// sse_copy.h -- asynchronous global -> LDS copies (gfx950's global_load_lds)
// used by the MFMA kernels to stage their G windows and A fragments.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sse {

typedef __attribute__((address_space(3))) void lds_void;

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
    const int dr = NT / upr, dc = NT - (NT / upr) * upr;
    int r = tid / upr, c = tid - (tid / upr) * upr;
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
