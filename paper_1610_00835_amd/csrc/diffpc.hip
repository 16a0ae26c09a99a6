// Diffusion preconditioner (Sec. 4.4, eq. EQ:DA): the diffusion approximation
//   -div(D grad U) + mu_a U = f,  U + l dU/dn = 0,  D = 1/(d sigma_t), l = 2 D,
// models f -> U = (I - K)^{-1} A f, so (I - K)^{-1} = I + (I - K)^{-1} A S is
// approximated by  M r = r + L^{-1} (sigma_s r),  L^{-1} by two V-cycles.
//
// Cell-centred finite differences per unit volume on the solver's grid:
//   (L U)_j = sum_interior faces Df (U_j - U_k) / h^2 + sum_boundary faces 2 D_j / (h (h + 2 l_j)) U_j
//           + mu_a_j U_j,   Df = harmonic mean of D_j, D_k.
// Multigrid: levels by halving each axis (ceil) down to at most 4 cells per
// axis, coarse sigma_t / sigma_s the averages of the children, rediscretised
// with 2h; red-black Gauss-Seidel (red = even i0+i1+i2 first), 2 sweeps before
// and after the coarse correction; restriction by averaging the children,
// constant prolongation; the coarsest level gets 60 sweeps in one workgroup.
// All FP64 (the smoother's sums in a fixed order: per axis z, y, x, the upper
// neighbour before the lower).
#include "common.hpp"

#include <algorithm>
#include <vector>

namespace ertvie {

struct DiffLevel {
    int n[3] = {1, 1, 1};
    double h = 0.0;
    long N = 0;
    double* st = nullptr;
    double* ss = nullptr;
    double* diag = nullptr;
    double* df[3] = {nullptr, nullptr, nullptr};   // face to the upper neighbour along axis a
    double* U = nullptr;
    double* B = nullptr;
};

struct DiffPc {
    int dim = 0;
    std::vector<DiffLevel> lv;
    double* rhs = nullptr;
    long bytes = 0;
};

namespace {

constexpr int kPre = 2, kPost = 2, kCoarseSweeps = 60, kCoarsest = 4, kCycles = 2;

struct LvArgs {
    int dim, n0, n1, n2;
    double h;
    const double* st;
    const double* ss;
    double* diag;
    double* dfx;
    double* dfy;
    double* dfz;
};

__device__ __forceinline__ void unravel(long j, int n0, int n1, int i[3])
{
    i[0] = (int)(j % n0);
    i[1] = (int)((j / n0) % n1);
    i[2] = (int)(j / ((long)n0 * n1));
}

__global__ void k_avg_children(int dim, int f0, int f1, int f2, const double* __restrict__ fine, int c0, int c1,
                               int c2, double* __restrict__ coarse)
{
    const long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= (long)c0 * c1 * c2) return;
    int ic[3];
    unravel(c, c0, c1, ic);
    double s = 0.0;
    int cnt = 0;
    for (int oz = 0; oz < (dim > 2 ? 2 : 1); ++oz)
        for (int oy = 0; oy < 2; ++oy)
            for (int ox = 0; ox < 2; ++ox) {
                const int a = 2 * ic[0] + ox, b = 2 * ic[1] + oy, z = 2 * ic[2] + oz;
                if (a < f0 && b < f1 && z < f2) {
                    s += fine[a + (long)f0 * (b + (long)f1 * z)];
                    ++cnt;
                }
            }
    coarse[c] = s / cnt;
}

__global__ void k_faces(LvArgs a)
{
    const long N = (long)a.n0 * a.n1 * a.n2;
    const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (j >= N) return;
    int i[3];
    unravel(j, a.n0, a.n1, i);
    const int n[3] = {a.n0, a.n1, a.n2};
    const long s[3] = {1, a.n0, (long)a.n0 * a.n1};
    double* df[3] = {a.dfx, a.dfy, a.dfz};
    const double Dj = 1.0 / (a.dim * a.st[j]);
    for (int ax = 0; ax < 3; ++ax) {
        double v = 0.0;
        if (ax < a.dim && i[ax] < n[ax] - 1) {
            const double Dk = 1.0 / (a.dim * a.st[j + s[ax]]);
            v = 2.0 * Dj * Dk / (Dj + Dk);
        }
        df[ax][j] = v;
    }
}

__global__ void k_diag(LvArgs a)
{
    const long N = (long)a.n0 * a.n1 * a.n2;
    const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (j >= N) return;
    int i[3];
    unravel(j, a.n0, a.n1, i);
    const int n[3] = {a.n0, a.n1, a.n2};
    const long s[3] = {1, a.n0, (long)a.n0 * a.n1};
    const double* df[3] = {a.dfx, a.dfy, a.dfz};
    const double h2 = a.h * a.h;
    const double Dj = 1.0 / (a.dim * a.st[j]);
    const double rob = 2.0 * Dj / (a.h * (a.h + 4.0 * Dj));
    double d = a.st[j] - a.ss[j];
    for (int ax = a.dim - 1; ax >= 0; --ax) {
        if (i[ax] < n[ax] - 1) d += df[ax][j] / h2;
        if (i[ax] > 0) d += df[ax][j - s[ax]] / h2;
        if (i[ax] == 0) d += rob;
        if (i[ax] == n[ax] - 1) d += rob;
    }
    a.diag[j] = d;
}

// sum over interior faces of Df U_k / h^2, per axis z, y, x: upper then lower neighbour
__device__ __forceinline__ double offdiag(const LvArgs& a, const double* __restrict__ U, long j, const int i[3])
{
    const int n[3] = {a.n0, a.n1, a.n2};
    const long s[3] = {1, a.n0, (long)a.n0 * a.n1};
    const double* df[3] = {a.dfx, a.dfy, a.dfz};
    const double h2 = a.h * a.h;
    double o = 0.0;
    for (int ax = a.dim - 1; ax >= 0; --ax) {
        if (i[ax] < n[ax] - 1) o += df[ax][j] * U[j + s[ax]] / h2;
        if (i[ax] > 0) o += df[ax][j - s[ax]] * U[j - s[ax]] / h2;
    }
    return o;
}

__global__ __launch_bounds__(256) void k_rbgs(LvArgs a, double* __restrict__ U, const double* __restrict__ B,
                                              int colour)
{
    const long N = (long)a.n0 * a.n1 * a.n2;
    const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (j >= N) return;
    int i[3];
    unravel(j, a.n0, a.n1, i);
    if (((i[0] + i[1] + i[2]) & 1) != colour) return;
    U[j] = (B[j] + offdiag(a, U, j, i)) / a.diag[j];
}

// B_c = average over the children of the fine residual B - (diag U - offdiag U), and
// U_c = 0 (the coarser correction starts from zero): coarse cell q
__device__ __forceinline__ void restrict_residual(const LvArgs& a, const double* __restrict__ U,
                                                  const double* __restrict__ B, long q, int c0, int c1,
                                                  double* __restrict__ Bc, double* __restrict__ Uc)
{
    int ic[3];
    unravel(q, c0, c1, ic);
    double s = 0.0;
    int cnt = 0;
    for (int oz = 0; oz < (a.dim > 2 ? 2 : 1); ++oz)
        for (int oy = 0; oy < 2; ++oy)
            for (int ox = 0; ox < 2; ++ox) {
                const int i[3] = {2 * ic[0] + ox, 2 * ic[1] + oy, 2 * ic[2] + oz};
                if (i[0] < a.n0 && i[1] < a.n1 && i[2] < a.n2) {
                    const long j = i[0] + (long)a.n0 * (i[1] + (long)a.n1 * i[2]);
                    s += B[j] - (a.diag[j] * U[j] - offdiag(a, U, j, i));
                    ++cnt;
                }
            }
    Bc[q] = s / cnt;
    Uc[q] = 0.0;
}

__global__ __launch_bounds__(256) void k_restrict_residual(LvArgs a, const double* __restrict__ U,
                                                           const double* __restrict__ B, int c0, int c1, int c2,
                                                           double* __restrict__ Bc, double* __restrict__ Uc)
{
    const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (q < (long)c0 * c1 * c2) restrict_residual(a, U, B, q, c0, c1, Bc, Uc);
}

__global__ void k_prolong_add(int f0, int f1, int f2, double* __restrict__ Uf, int c0, int c1,
                              const double* __restrict__ Ec)
{
    const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (j >= (long)f0 * f1 * f2) return;
    int i[3];
    unravel(j, f0, f1, i);
    Uf[j] += Ec[(i[0] / 2) + (long)c0 * ((i[1] / 2) + (long)c1 * (i[2] / 2))];
}

// The V-cycle below a level of at most kSmallCells cells, in one workgroup: the
// same steps as the per-level launches (smoothing, residual, restriction, the
// coarser cycle, prolongation, smoothing), each a workgroup-stride loop closed by
// a barrier.  Red-black colours, residuals, averages and prolongations are per
// cell, so the results equal the per-level launches bit for bit.
constexpr int kSmallCells = 256;
constexpr int kMaxSmall = 12;

struct SmallLevel {
    LvArgs a;
    long N;
    double* U;
    double* B;
};

struct SmallCycle {
    int nl;                       // levels k0 .. k0 + nl - 1, the last the coarsest
    SmallLevel lv[kMaxSmall];
};

__device__ __forceinline__ void small_rbgs(const SmallLevel& L, int sweeps)
{
    for (int sw = 0; sw < sweeps; ++sw)
        for (int colour = 0; colour < 2; ++colour) {
            for (long j = threadIdx.x; j < L.N; j += blockDim.x) {
                int i[3];
                unravel(j, L.a.n0, L.a.n1, i);
                if (((i[0] + i[1] + i[2]) & 1) == colour) L.U[j] = (L.B[j] + offdiag(L.a, L.U, j, i)) / L.a.diag[j];
            }
            __syncthreads();
        }
}

__global__ __launch_bounds__(256) void k_small_cycle(SmallCycle c)
{
    // down: smooth, residual, restrict (the first level's U is the caller's)
    for (int k = 0; k + 1 < c.nl; ++k) {
        const SmallLevel& L = c.lv[k];
        const SmallLevel& C = c.lv[k + 1];
        small_rbgs(L, kPre);
        for (long q = threadIdx.x; q < C.N; q += blockDim.x) restrict_residual(L.a, L.U, L.B, q, C.a.n0, C.a.n1, C.B, C.U);
        __syncthreads();
    }
    // coarsest: sweeps on the correction equation from zero (zeroed above); a single-level
    // hierarchy's only level is the finest, whose cycles continue from the current iterate
    small_rbgs(c.lv[c.nl - 1], kCoarseSweeps);
    // up: prolongate and smooth
    for (int k = c.nl - 2; k >= 0; --k) {
        const SmallLevel& L = c.lv[k];
        const SmallLevel& C = c.lv[k + 1];
        for (long j = threadIdx.x; j < L.N; j += blockDim.x) {
            int i[3];
            unravel(j, L.a.n0, L.a.n1, i);
            L.U[j] += C.U[(i[0] / 2) + (long)C.a.n0 * ((i[1] / 2) + (long)C.a.n1 * (i[2] / 2))];
        }
        __syncthreads();
        small_rbgs(L, kPost);
    }
}

__global__ void k_scaled(const double* __restrict__ r, const double* __restrict__ ss, long N, double* __restrict__ b)
{
    const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (j < N) b[j] = ss[j] * r[j];
}

__global__ void k_add_out(const double* __restrict__ r, const double* __restrict__ u, long N, double* __restrict__ z)
{
    const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (j < N) z[j] = r[j] + u[j];
}

inline unsigned nblk(long n) { return (unsigned)((n + 255) / 256); }

LvArgs args_of(const DiffPc* d, const DiffLevel& L)
{
    return LvArgs{d->dim, L.n[0], L.n[1], L.n[2], L.h, L.st, L.ss, L.diag, L.df[0], L.df[1], L.df[2]};
}

__global__ void k_zero(double* __restrict__ p, long n)
{
    const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (j < n) p[j] = 0.0;
}

ert_status zero(hipStream_t s, double* p, long n)
{
    hipLaunchKernelGGL(k_zero, dim3(nblk(n)), dim3(256), 0, s, p, n);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ert_status vcycle(hipStream_t s, DiffPc* d, int k)
{
    DiffLevel& L = d->lv[k];
    const LvArgs a = args_of(d, L);
    const int nl = (int)d->lv.size() - k;
    if (k + 1 == (int)d->lv.size() || (L.N <= kSmallCells && nl <= kMaxSmall)) {
        // this level and the coarser ones in one workgroup (the coarsest level always goes here)
        SmallCycle c{};
        c.nl = nl;
        for (int q = 0; q < nl; ++q) {
            DiffLevel& Q = d->lv[k + q];
            c.lv[q] = SmallLevel{args_of(d, Q), Q.N, Q.U, Q.B};
        }
        hipLaunchKernelGGL(k_small_cycle, dim3(1), dim3(256), 0, s, c);
        ERT_HIP(hipGetLastError());
        return ERT_OK;
    }
    for (int sw = 0; sw < kPre; ++sw)
        for (int c = 0; c < 2; ++c) hipLaunchKernelGGL(k_rbgs, dim3(nblk(L.N)), dim3(256), 0, s, a, L.U, L.B, c);
    DiffLevel& C = d->lv[k + 1];
    hipLaunchKernelGGL(k_restrict_residual, dim3(nblk(C.N)), dim3(256), 0, s, a, (const double*)L.U,
                       (const double*)L.B, C.n[0], C.n[1], C.n[2], C.B, C.U);
    ERT_HIP(hipGetLastError());
    ERT_TRY(vcycle(s, d, k + 1));
    hipLaunchKernelGGL(k_prolong_add, dim3(nblk(L.N)), dim3(256), 0, s, L.n[0], L.n[1], L.n[2], L.U, C.n[0], C.n[1],
                       (const double*)C.U);
    for (int sw = 0; sw < kPost; ++sw)
        for (int c = 0; c < 2; ++c) hipLaunchKernelGGL(k_rbgs, dim3(nblk(L.N)), dim3(256), 0, s, a, L.U, L.B, c);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ert_status diffpc_build(ert_plan_impl* p)
{
    if (p->diffpc) return ERT_OK;
    DiffPc* d = new DiffPc();
    d->dim = p->o.dim;
    hipStream_t s = p->stream;
    int n[3] = {p->geo.n0, p->geo.n1, d->dim == 3 ? p->geo.n2 : 1};
    double h = p->geo.h;
    ert_status st = ERT_OK;
    auto alloc = [&](double** q, long cnt) {
        if (st != ERT_OK) return;
        if (hipMalloc(q, sizeof(double) * std::max<long>(1, cnt)) != hipSuccess) {
            record_error("diffusion preconditioner: allocation failed");
            st = ERT_ENOMEM;
        }
        d->bytes += sizeof(double) * cnt;
    };
    while (st == ERT_OK) {
        DiffLevel L;
        for (int a = 0; a < 3; ++a) L.n[a] = n[a];
        L.h = h;
        L.N = (long)n[0] * n[1] * n[2];
        alloc(&L.st, L.N);
        alloc(&L.ss, L.N);
        alloc(&L.diag, L.N);
        for (int a = 0; a < 3; ++a) alloc(&L.df[a], L.N);
        alloc(&L.U, L.N);
        alloc(&L.B, L.N);
        d->lv.push_back(L);
        if (st != ERT_OK) break;
        const int mx = std::max(n[0], std::max(n[1], n[2]));
        if (mx <= kCoarsest) break;
        for (int a = 0; a < 3; ++a) n[a] = (n[a] + 1) / 2;
        h *= 2.0;
    }
    if (st == ERT_OK) alloc(&d->rhs, p->N);
    if (st == ERT_OK) {
        DiffLevel& L0 = d->lv[0];
        st = ERT_HIPST(hipMemcpyAsync(L0.st, p->d_st, sizeof(double) * L0.N, hipMemcpyDeviceToDevice, s));
        if (st == ERT_OK)
            st = ERT_HIPST(hipMemcpyAsync(L0.ss, p->d_ss, sizeof(double) * L0.N, hipMemcpyDeviceToDevice, s));
        for (size_t k = 1; k < d->lv.size() && st == ERT_OK; ++k) {
            DiffLevel& F = d->lv[k - 1];
            DiffLevel& C = d->lv[k];
            hipLaunchKernelGGL(k_avg_children, dim3(nblk(C.N)), dim3(256), 0, s, d->dim, F.n[0], F.n[1], F.n[2],
                               (const double*)F.st, C.n[0], C.n[1], C.n[2], C.st);
            hipLaunchKernelGGL(k_avg_children, dim3(nblk(C.N)), dim3(256), 0, s, d->dim, F.n[0], F.n[1], F.n[2],
                               (const double*)F.ss, C.n[0], C.n[1], C.n[2], C.ss);
            st = ERT_HIPST(hipGetLastError());
        }
        for (size_t k = 0; k < d->lv.size() && st == ERT_OK; ++k) {
            const LvArgs a = args_of(d, d->lv[k]);
            hipLaunchKernelGGL(k_faces, dim3(nblk(d->lv[k].N)), dim3(256), 0, s, a);
            hipLaunchKernelGGL(k_diag, dim3(nblk(d->lv[k].N)), dim3(256), 0, s, a);
            st = ERT_HIPST(hipGetLastError());
        }
        if (st == ERT_OK) st = ERT_HIPST(hipStreamSynchronize(s));
    }
    if (st != ERT_OK) {
        diffpc_destroy(d);
        return st;
    }
    p->diffpc = d;
    return ERT_OK;
}

}  // namespace

void diffpc_destroy(DiffPc* d)
{
    if (!d) return;
    for (auto& L : d->lv) {
        (void)hipFree(L.st);
        (void)hipFree(L.ss);
        (void)hipFree(L.diag);
        for (auto* q : L.df) (void)hipFree(q);
        (void)hipFree(L.U);
        (void)hipFree(L.B);
    }
    (void)hipFree(d->rhs);
    delete d;
}

ert_status diffpc_apply(ert_plan_impl* p, const double* r, double* z, int nrhs)
{
    ERT_TRY(diffpc_build(p));
    DiffPc* d = p->diffpc;
    hipStream_t s = p->stream;
    DiffLevel& L0 = d->lv[0];
    for (int c = 0; c < nrhs; ++c) {
        const double* rc = r + (size_t)c * p->N;
        double* zc = z + (size_t)c * p->N;
        hipLaunchKernelGGL(k_scaled, dim3(nblk(p->N)), dim3(256), 0, s, rc, (const double*)p->d_ss, p->N, L0.B);
        ERT_HIP(hipGetLastError());
        ERT_TRY(zero(s, L0.U, L0.N));
        for (int cy = 0; cy < kCycles; ++cy) ERT_TRY(vcycle(s, d, 0));
        hipLaunchKernelGGL(k_add_out, dim3(nblk(p->N)), dim3(256), 0, s, rc, (const double*)L0.U, p->N, zc);
        ERT_HIP(hipGetLastError());
    }
    return ERT_OK;
}

}  // namespace ertvie
