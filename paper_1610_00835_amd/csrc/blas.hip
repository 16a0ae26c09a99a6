// FP64 vector kernels for the Krylov solver (HBM-bound level-1/level-2 work).
// Reductions are two-pass with a fixed block count and fixed order, so every
// result is bitwise reproducible from run to run.
#include <algorithm>

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

// ------------------------------------------------------------ level 3 ----
// C = beta C + alpha A B with element strides (A(i,k) = A[i*sAi + k*sAk], ...).
// 64 x 64 output tiles, 4 x 4 per thread, reduction chunks of 16 staged in LDS.
// Long reductions (tall-skinny products) are split over gridDim.z slices whose
// partial tiles go to a workspace and are summed in slice order (deterministic).
namespace ertvie {
namespace {

struct DG {
    int M, N;
    long K;
    double alpha, beta;
    const double* A; long sAi, sAk;
    const double* B; long sBk, sBj;
    double* C; long sCi, sCj;
    double* part;      // split-K workspace [nz][M][N] (row-major), or null
    long kchunk;       // reduction length per slice
};

__global__ __launch_bounds__(256) void k_dgemm(DG g)
{
    __shared__ double As[16][65], Bs[16][65];
    const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const long klo = (long)blockIdx.z * g.kchunk;
    const long khi = (klo + g.kchunk) < g.K ? (klo + g.kchunk) : g.K;
    double acc[4][4] = {};
    for (long k0 = klo; k0 < khi; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e / 64, r = e % 64;
            const long k = k0 + kk;
            const int i = i0 + r, j = j0 + r;
            As[kk][r] = (i < g.M && k < khi) ? g.A[i * g.sAi + k * g.sAk] : 0.0;
            Bs[kk][r] = (j < g.N && k < khi) ? g.B[k * g.sBk + j * g.sBj] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[kk][ty * 4 + u];
                b[u] = Bs[kk][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + ty * 4 + u, j = j0 + tx * 4 + v;
            if (i >= g.M || j >= g.N) continue;
            if (g.part) {
                g.part[((long)blockIdx.z * g.M + i) * g.N + j] = acc[u][v];
            } else {
                double* c = g.C + i * g.sCi + j * g.sCj;
                *c = (g.beta == 0.0 ? 0.0 : g.beta * *c) + g.alpha * acc[u][v];
            }
        }
}

__global__ void k_dgemm_reduce(DG g, int nz)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)g.M * g.N) return;
    const int i = (int)(t / g.N), j = (int)(t % g.N);
    double s = 0.0;
    for (int z = 0; z < nz; ++z) s += g.part[((long)z * g.M + i) * g.N + j];
    double* c = g.C + i * g.sCi + j * g.sCj;
    *c = (g.beta == 0.0 ? 0.0 : g.beta * *c) + g.alpha * s;
}

}  // namespace

ert_status dev_dgemm(hipStream_t s, int M, int N, long K, double alpha, const double* A, long sAi, long sAk,
                     const double* B, long sBk, long sBj, double beta, double* C, long sCi, long sCj, double* work,
                     size_t work_elems)
{
    if (M <= 0 || N <= 0) return ERT_OK;
    DG g{M, N, K, alpha, beta, A, sAi, sAk, B, sBk, sBj, C, sCi, sCj, nullptr, K};
    const long tiles = (long)((M + 63) / 64) * ((N + 63) / 64);
    int nz = 1;
    if (tiles < 256 && K > 4096 && work) {
        nz = (int)std::min<long>(std::max<long>(1, 512 / tiles), (K + 4095) / 4096);
        while (nz > 1 && (size_t)nz * M * N > work_elems) --nz;
    }
    if (nz > 1) {
        g.part = work;
        g.kchunk = ((K + nz - 1) / nz + 15) / 16 * 16;
        nz = (int)((K + g.kchunk - 1) / g.kchunk);
    }
    dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64), (unsigned)nz);
    hipLaunchKernelGGL(k_dgemm, grid, dim3(256), 0, s, g);
    ERT_HIP(hipGetLastError());
    if (nz > 1) {
        const long n = (long)M * N;
        hipLaunchKernelGGL(k_dgemm_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, nz);
        ERT_HIP(hipGetLastError());
    }
    return ERT_OK;
}

}  // namespace ertvie
