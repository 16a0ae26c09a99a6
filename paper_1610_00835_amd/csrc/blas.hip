// FP64 vector kernels for the Krylov solver (HBM-bound level-1/level-2 work).
// Reductions are two-pass with a fixed block count and fixed order, so every
// result is bitwise reproducible from run to run.
#include "common.hpp"

namespace ertvie {

namespace {

constexpr int kBlk = 256;
constexpr int kRedBlocks = 240;   // partial sums per column
constexpr int kColGroup = 8;      // columns reduced together per pass over w

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kBlk) void k_multidot_partial(const double* __restrict__ V, long ldv, int ncols,
                                                           const double* __restrict__ w, long N,
                                                           double* __restrict__ partial)
{
    __shared__ double sh[kBlk];
    const long chunk = (N + gridDim.x - 1) / gridDim.x;
    const long lo = blockIdx.x * chunk;
    const long hi = (lo + chunk) < N ? (lo + chunk) : N;
    for (int c0 = 0; c0 < ncols; c0 += kColGroup) {
        double acc[kColGroup];
#pragma unroll
        for (int c = 0; c < kColGroup; ++c) acc[c] = 0.0;
        for (long i = lo + threadIdx.x; i < hi; i += kBlk) {
            const double wi = w[i];
#pragma unroll
            for (int c = 0; c < kColGroup; ++c)
                if (c0 + c < ncols) acc[c] += V[(long)(c0 + c) * ldv + i] * wi;
        }
#pragma unroll
        for (int c = 0; c < kColGroup; ++c) {
            if (c0 + c < ncols) {
                double s = block_sum(acc[c], sh);
                if (threadIdx.x == 0) partial[(long)blockIdx.x * ncols + c0 + c] = s;
            }
        }
    }
}

__global__ void k_multidot_final(const double* __restrict__ partial, int nblk, int ncols, double* __restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(long)b * ncols + c];
    out[c] = s;
}

__global__ __launch_bounds__(kBlk) void k_gemv(const double* __restrict__ V, long ldv, int ncols,
                                               const double* __restrict__ coef, double* __restrict__ w, long N,
                                               double sign)
{
    const long i = blockIdx.x * (long)kBlk + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    for (int c = 0; c < ncols; ++c) s += V[(long)c * ldv + i] * coef[c];
    w[i] += sign * s;
}

__global__ void k_scale(double* __restrict__ y, const double* __restrict__ x, double a, long N)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < N) y[i] = a * x[i];
}

__global__ void k_sub(double* __restrict__ y, const double* __restrict__ a, const double* __restrict__ b, long N)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < N) y[i] = a[i] - b[i];
}

__global__ void k_add(double* __restrict__ y, const double* __restrict__ x, long N)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < N) y[i] += x[i];
}

__global__ void k_zero(double* __restrict__ y, long N)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < N) y[i] = 0.0;
}

inline unsigned nblocks(long N) { return (unsigned)((N + kBlk - 1) / kBlk); }

}  // namespace

ert_status dev_multidot(hipStream_t s, const double* V, long ldv, int ncols, const double* w, long N,
                        double* partial, double* out)
{
    if (ncols <= 0) return ERT_OK;
    int nb = kRedBlocks;
    if ((long)nb * 64 > N) nb = (int)((N + 63) / 64);
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_multidot_partial, dim3(nb), dim3(kBlk), 0, s, V, ldv, ncols, w, N, partial);
    ERT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_multidot_final, dim3((ncols + 63) / 64), dim3(64), 0, s, partial, nb, ncols, out);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ert_status dev_gemv_sub(hipStream_t s, const double* V, long ldv, int ncols, const double* coef, double* w,
                        long N)
{
    if (ncols <= 0) return ERT_OK;
    hipLaunchKernelGGL(k_gemv, dim3(nblocks(N)), dim3(kBlk), 0, s, V, ldv, ncols, coef, w, N, -1.0);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ert_status dev_gemv_add(hipStream_t s, const double* V, long ldv, int ncols, const double* coef, double* x,
                        long N)
{
    if (ncols <= 0) return ERT_OK;
    hipLaunchKernelGGL(k_gemv, dim3(nblocks(N)), dim3(kBlk), 0, s, V, ldv, ncols, coef, x, N, 1.0);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ert_status dev_scale(hipStream_t s, double* y, const double* x, double alpha, long N)
{
    hipLaunchKernelGGL(k_scale, dim3(nblocks(N)), dim3(kBlk), 0, s, y, x, alpha, N);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ert_status dev_sub(hipStream_t s, double* y, const double* a, const double* b, long N)
{
    hipLaunchKernelGGL(k_sub, dim3(nblocks(N)), dim3(kBlk), 0, s, y, a, b, N);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ert_status dev_add(hipStream_t s, double* y, const double* x, long N)
{
    hipLaunchKernelGGL(k_add, dim3(nblocks(N)), dim3(kBlk), 0, s, y, x, N);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ert_status dev_zero(hipStream_t s, double* y, long N)
{
    hipLaunchKernelGGL(k_zero, dim3(nblocks(N)), dim3(kBlk), 0, s, y, N);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ert_status dev_small_add(hipStream_t s, double* dst, const double* src, int n)
{
    hipLaunchKernelGGL(k_add, dim3(nblocks(n)), dim3(kBlk), 0, s, dst, src, (long)n);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

}  // namespace ertvie
