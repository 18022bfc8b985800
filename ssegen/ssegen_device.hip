// ssegen_device.hip -- device side of the seeded input generator (see
// ssegen_core.h): fills resident device tensors with the same bits the host
// generator produces, and applies the per-iteration perturbation in place.
// Built with -ffp-contract=off so no multiply-add is fused.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SSEGEN_FN static __device__ inline
#include "ssegen_core.h"

namespace {

__global__ void k_fill_dH(uint64_t seed, int64_t n, double *out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = ssegen_normal(seed, (uint64_t)i, SSEGEN_S_DH, 0);
}

// One thread per complex element of every n_side x n_side block.
template <typename T>
__global__ void k_fill_antiherm(uint64_t seed, uint32_t stream, uint32_t scale_stream, int scaled,
                                int n_side, int64_t nblk, T *out)
{
    const int nn = n_side * n_side;
    const int64_t n = nblk * nn;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t B = (uint64_t)(i / nn);
        int e = (int)(i - (int64_t)B * nn);
        double re, im;
        ssegen_antiherm(seed, B * nn, n_side, e / n_side, e % n_side, stream, &re, &im);
        if (scaled) {
            double s = ssegen_block_scale(seed, B, scale_stream);
            re = re * s;
            im = im * s;
        }
        out[2 * i] = (T)re;
        out[2 * i + 1] = (T)im;
    }
}

// One wavefront per block: X <- X + 0.01 * (|X|_F / |N|_F) * N, N the
// anti-Hermitian part of the block's raw complex normals.  The wave draws the
// raw normals once into LDS (element (m, n) of N needs raw (m, n) and (n, m),
// and both passes need N), then forms N from pairs: a quarter of the draws of
// forming each element independently in each pass, with the same arithmetic
// and summation order.
template <typename T>
__global__ __launch_bounds__(256) void k_perturb(uint64_t seed, uint32_t st, int n_side,
                                                 int64_t nblk, T *data)
{
    extern __shared__ double2 raw_all[];  // 4 waves x n_side^2
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t B = blockIdx.x * (int64_t)(blockDim.x >> 6) + wv;
    const int nn = n_side * n_side;
    double2 *raw = raw_all + (size_t)wv * nn;
    const bool live = B < nblk;
    if (live) {
        const uint64_t base = (uint64_t)B * nn;
        for (int e = lane; e < nn; e += 64) {
            double re, im;
            ssegen_cnormal(seed, base + (uint64_t)e, st, &re, &im);
            raw[e] = make_double2(re, im);
        }
    }
    __syncthreads();
    if (!live)
        return;
    T *x = data + (size_t)B * nn * 2;
    double nx = 0.0, nr = 0.0;
    for (int e = lane; e < nn; e += 64) {
        const int m = e / n_side, n = e - m * n_side;
        const double2 a = raw[e], b = raw[n * n_side + m];
        /* X[m,n] - conj(X[n,m]) = (ar - br) + i (ai + bi), halved */
        const double re = (a.x - b.x) * 0.5, im = (a.y + b.y) * 0.5;
        const double xr = (double)x[2 * e], xi = (double)x[2 * e + 1];
        nx = nx + (xr * xr + xi * xi);
        nr = nr + (re * re + im * im);
    }
    for (int o = 32; o > 0; o >>= 1) {
        nx = nx + __shfl_xor(nx, o, 64);
        nr = nr + __shfl_xor(nr, o, 64);
    }
    const double f = nr > 0.0 ? 0.01 * (sqrt(nx) / sqrt(nr)) : 0.0;
    for (int e = lane; e < nn; e += 64) {
        const int m = e / n_side, n = e - m * n_side;
        const double2 a = raw[e], b = raw[n * n_side + m];
        const double re = (a.x - b.x) * 0.5, im = (a.y + b.y) * 0.5;
        x[2 * e] = (T)((double)x[2 * e] + f * re);
        x[2 * e + 1] = (T)((double)x[2 * e + 1] + f * im);
    }
}

inline unsigned grid_for(int64_t n, int bs)
{
    int64_t g = (n + bs - 1) / bs;
    if (g > (1 << 20))
        g = 1 << 20;
    if (g < 1)
        g = 1;
    return (unsigned)g;
}

} // namespace

extern "C" {

int ssegen_dev_fill_dH(uint64_t seed, int64_t n, double *out, void *stream)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_fill_dH, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, seed, n,
                       out);
    return (int)hipGetLastError();
}

// G: every block of [Nkz, NE, NA] (nblk = Nkz * NE * NA), side Norb.
int ssegen_dev_fill_G(uint64_t seed, int comp, int Norb, int64_t nblk, int scaled, int fp32,
                      void *out, void *stream)
{
    const int64_t n = nblk * Norb * Norb;
    if (fp32) {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_fill_antiherm<float>, dim3(grid_for(n, 256)), dim3(256), 0,
                           (hipStream_t)stream, seed, (uint32_t)(SSEGEN_S_G + comp),
                           (uint32_t)(SSEGEN_S_GSCALE + comp), scaled, Norb, nblk, (float *)out);
    } else {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_fill_antiherm<double>, dim3(grid_for(n, 256)), dim3(256), 0,
                           (hipStream_t)stream, seed, (uint32_t)(SSEGEN_S_G + comp),
                           (uint32_t)(SSEGEN_S_GSCALE + comp), scaled, Norb, nblk, (double *)out);
    }
    return (int)hipGetLastError();
}

// D~: every block of [Nqz, Nw, NA, NB] (nblk), side N3D.
int ssegen_dev_fill_D(uint64_t seed, int comp, int N3D, int64_t nblk, int fp32, void *out,
                      void *stream)
{
    const int64_t n = nblk * N3D * N3D;
    if (fp32) {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_fill_antiherm<float>, dim3(grid_for(n, 256)), dim3(256), 0,
                           (hipStream_t)stream, seed, (uint32_t)(SSEGEN_S_D + comp), 0u, 0, N3D,
                           nblk, (float *)out);
    } else {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_fill_antiherm<double>, dim3(grid_for(n, 256)), dim3(256), 0,
                           (hipStream_t)stream, seed, (uint32_t)(SSEGEN_S_D + comp), 0u, 0, N3D,
                           nblk, (double *)out);
    }
    return (int)hipGetLastError();
}

// In-place perturbation of nblk contiguous n_side x n_side blocks; block t is
// keyed by flat index t (the whole tensor is perturbed).
int ssegen_dev_perturb(uint64_t seed, int iteration, uint32_t stream_word, int n_side, int64_t nblk,
                       int fp32, void *data, void *stream)
{
    const uint32_t st = stream_word | ((uint32_t)(iteration + 1) << 8);
    const int64_t nwg = (nblk + 3) / 4;
    if (nwg > 0x7fffffff)
        return (int)hipErrorInvalidValue;
    const size_t lds = (size_t)4 * n_side * n_side * sizeof(double2);
    if (lds > 64 * 1024)
        return (int)hipErrorInvalidValue;
    if (fp32) {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_perturb<float>, dim3((unsigned)nwg), dim3(256), lds,
                           (hipStream_t)stream, seed, st, n_side, nblk, (float *)data);
    } else {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_perturb<double>, dim3((unsigned)nwg), dim3(256), lds,
                           (hipStream_t)stream, seed, st, n_side, nblk, (double *)data);
    }
    return (int)hipGetLastError();
}

} // extern "C"
