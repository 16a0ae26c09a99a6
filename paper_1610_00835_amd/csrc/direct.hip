// Dense summation of the collocation matrix (Sec. 3.2, approach (M-iii)) and
// the singular diagonal entry, both on the GPU.
//
//   y_j = h^d sum_{k != j} G(x_j, x_k) w_k + A_jj w_j,   w = x or sigma_s x,
//   G(x,y) = exp(-tau) / (|S^{d-1}| |x-y|^{d-1})            (eq. EQ:Kernel)
//
// One thread per target; source weights are staged through LDS in tiles of
// 256 and the source cell coordinates advance incrementally (uniform across
// the wave, so they live in scalar registers).  Offsets between collocation
// points are integers, so |x-y|^2 = h^2 K with K exact and the ray step count
// m = ceil(2 sqrt K) is exact as well.
#include "common.hpp"

namespace ertvie {

namespace {

constexpr int kTile = 256;

// ---------------------------------------------------------- self cell -----

// sigma_at for points inside cell c, reading the cell's 3^3 neighbourhood nb
// (nb[a0 + 3 a1 + 9 a2] = sigma_t of cell c + a - 1, indices clamped to the grid):
// every interpolation cell such a point can fall in has its corners there.  The
// clamp, cell search and interpolation are sigma_at's, done in FP64 (max, min,
// floor give the same integers and fractions), so the values agree bit for bit.
// An axis of one cell (or the third axis in 2D) takes k = 0, t = 0 and a zero
// corner offset: its terms add exact zeros.
struct NbAxes {
    double hi[3], km[3], cl[3];  // n - 1, max(n - 2, 0), c - 1 (inactive axis: 0, 0, -1)
    int d0, d1, d2;              // corner offsets in nb
};

__device__ __forceinline__ NbAxes nb_axes(const Geo& g, const int c[3])
{
    const int n[3] = {g.n0, g.n1, g.n2};
    NbAxes A;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool on = a < g.dim && n[a] > 1;
        A.hi[a] = on ? double(n[a] - 1) : 0.0;
        A.km[a] = on ? double(n[a] - 2) : 0.0;
        A.cl[a] = on ? double(c[a] - 1) : -1.0;
    }
    A.d0 = n[0] > 1 ? 1 : 0;
    A.d1 = n[1] > 1 ? 3 : 0;
    A.d2 = (g.dim > 2 && n[2] > 1) ? 9 : 0;
    return A;
}

__device__ __forceinline__ double sigma_nb(const double* nb, const NbAxes& A, double inv_h, double p0, double p1,
                                           double p2)
{
    const double p[3] = {p0, p1, p2};
    double t[3], l[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = fmin(fmax(p[a] * inv_h - 0.5, 0.0), A.hi[a]);
        const double k = fmin(floor(u), A.km[a]);
        t[a] = u - k;
        l[a] = k - A.cl[a];
    }
    const int b0 = (int)fma(9.0, l[2], fma(3.0, l[1], l[0]));
    const int d0 = A.d0, d1 = A.d1, d2 = A.d2;
    double c00 = nb[b0] + t[0] * (nb[b0 + d0] - nb[b0]);
    double c10 = nb[b0 + d1] + t[0] * (nb[b0 + d1 + d0] - nb[b0 + d1]);
    double c0 = c00 + t[1] * (c10 - c00);
    double c01 = nb[b0 + d2] + t[0] * (nb[b0 + d2 + d0] - nb[b0 + d2]);
    double c11 = nb[b0 + d2 + d1] + t[0] * (nb[b0 + d2 + d1 + d0] - nb[b0 + d2 + d1]);
    double c1 = c01 + t[1] * (c11 - c01);
    return c0 + t[2] * (c1 - c0);
}

// integral_0^rho E(x, x + r v) dr (same step rule as the off-diagonal kernel:
// one midpoint step for r <= h/2, two beyond; rho < h always).  Every sample
// lies in the cell of x, whose neighbourhood nb holds sigma_t.
__device__ double radial_integral(const Geo& g, int ray, double sigma, const double* nb, const NbAxes& A,
                                  const double x[3], const double v[3], double rho,
                                  const double* __restrict__ rx, const double* __restrict__ rw, int nrad)
{
    if (!ray) {
        double a = sigma * rho;
        return a < 1e-300 ? rho : -expm1(-a) / sigma;
    }
    const double half = 0.5 * g.h, inv_h = 1.0 / g.h;
    double acc = 0.0;
    double b0 = rho < half ? rho : half;
    for (int q = 0; q < nrad; ++q) {
        double r = 0.5 * b0 * (rx[q] + 1.0);
        double s = sigma_nb(nb, A, inv_h, x[0] + 0.5 * r * v[0], x[1] + 0.5 * r * v[1],
                                    x[2] + 0.5 * r * v[2]);
        acc += 0.5 * b0 * rw[q] * exp(-r * s);
    }
    if (rho > half) {
        double len = rho - half;
        for (int q = 0; q < nrad; ++q) {
            double r = half + 0.5 * len * (rx[q] + 1.0);
            double s1 = sigma_nb(nb, A, inv_h, x[0] + 0.25 * r * v[0], x[1] + 0.25 * r * v[1],
                                         x[2] + 0.25 * r * v[2]);
            double s2 = sigma_nb(nb, A, inv_h, x[0] + 0.75 * r * v[0], x[1] + 0.75 * r * v[1],
                                         x[2] + 0.75 * r * v[2]);
            acc += 0.5 * len * rw[q] * exp(-0.5 * r * (s1 + s2));
        }
    }
    return acc;
}

// One workgroup per cell: the directions are split into patches on which the
// integrand is smooth (2D: eight arcs of pi/4; 3D: six faces x four quadrants,
// parametrised by the face point with solid-angle Jacobian (h/2)/R^3), with
// tensor Gauss-Legendre per patch.  Fixed-order block reduction.
__global__ __launch_bounds__(256) void k_selfcell(Geo g, int ray, double sigma, const double* __restrict__ st,
                                                  const double* __restrict__ ax, const double* __restrict__ aw,
                                                  int nang, const double* __restrict__ rx,
                                                  const double* __restrict__ rw, int nrad, long j0,
                                                  double* __restrict__ diag)
{
    __shared__ double red[256];
    __shared__ double nb[27];
    const long j = j0 + blockIdx.x;
    const int i0 = (int)(j % g.n0);
    const int i1 = (int)((j / g.n0) % g.n1);
    const int i2 = (int)(j / ((long)g.n0 * g.n1));
    const int cell[3] = {i0, i1, i2};
    if (ray && threadIdx.x < 27) {
        const int n[3] = {g.n0, g.n1, g.n2};
        int q[3];
        for (int a = 0; a < 3; ++a) {
            const int k = cell[a] + (int)(a == 0 ? threadIdx.x % 3 : a == 1 ? (threadIdx.x / 3) % 3 : threadIdx.x / 9) - 1;
            q[a] = k < 0 ? 0 : (k > n[a] - 1 ? n[a] - 1 : k);
        }
        nb[threadIdx.x] = st[q[0] + (long)g.n0 * (q[1] + (long)g.n1 * q[2])];
    }
    __syncthreads();
    const NbAxes A = nb_axes(g, cell);
    const double half = 0.5 * g.h;
    const double x[3] = {g.h * (i0 + 0.5), g.h * (i1 + 0.5), g.dim > 2 ? g.h * (i2 + 0.5) : 0.0};
    double acc = 0.0;
    if (g.dim == 2) {
        const int total = 8 * nang;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            int arc = t / nang, q = t % nang;
            double t0 = arc * (kPi / 4.0);
            double th = t0 + (kPi / 8.0) * (ax[q] + 1.0);
            double v[3] = {cos(th), sin(th), 0.0};
            double c = fabs(v[0]) > fabs(v[1]) ? fabs(v[0]) : fabs(v[1]);
            acc += (kPi / 8.0) * aw[q] * radial_integral(g, ray, sigma, nb, A, x, v, half / c, rx, rw, nrad);
        }
    } else {
        const int per = nang * nang;
        const int total = 24 * per;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            int patch = t / per, q = t % per;
            int axis = patch / 8, sgn = ((patch / 4) & 1) ? 1 : -1, quad = patch & 3;
            int qa = q / nang, qb = q % nang;
            double u = ((quad & 1) ? 0.0 : -half) + 0.5 * half * (ax[qa] + 1.0);
            double w = ((quad & 2) ? 0.0 : -half) + 0.5 * half * (ax[qb] + 1.0);
            double R = sqrt(u * u + w * w + half * half);
            double v[3];
            v[axis] = sgn * half / R;
            v[(axis + 1) % 3] = u / R;
            v[(axis + 2) % 3] = w / R;
            double wq = 0.25 * half * half * aw[qa] * aw[qb] * half / (R * R * R);
            acc += wq * radial_integral(g, ray, sigma, nb, A, x, v, R, rx, rw, nrad);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) diag[j] = red[0] / surface_area(g.dim);
}

__global__ void k_fill(double* __restrict__ d, long N, const double* __restrict__ src)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < N) d[i] = src[0];
}

// (M-ii): cell integrals at the grid's integer offsets, itab[o0 + n0 (o1 + n1 o2)]
// = cell_int(o) for 0 <= o_a < n_a (the integral is even in every component).
__global__ void k_itab(int dim, int n0, int n1, int n2, double* __restrict__ itab)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= (long)n0 * n1 * n2) return;
    const int o0 = (int)(i % n0), o1 = (int)((i / n0) % n1), o2 = (int)(i / ((long)n0 * n1));
    itab[i] = cell_int(dim, o0, o1, dim > 2 ? o2 : 0);
}

// (M-ii) diagonal: h cell_int(0) / |S^{d-1}| for every cell.
__global__ void k_fill_scaled(double* __restrict__ d, long N, const double* __restrict__ src, double scale)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < N) d[i] = src[0] * scale;
}

// ------------------------------------------------------- dense apply -----

template <typename T, bool RAY, int RB>
__global__ __launch_bounds__(kTile) void k_direct(Geo g, const T* __restrict__ st, T sigma, T hd_over_area,
                                                  const double* __restrict__ x, const double* __restrict__ ss,
                                                  int weighted, long N, const double* __restrict__ diag,
                                                  const double* __restrict__ itab, int op, double* __restrict__ y)
{
    __shared__ T sw[kTile * RB];
    const long j = blockIdx.x * (long)kTile + threadIdx.x;
    const bool active = j < N;
    const int j0 = active ? (int)(j % g.n0) : 0;
    const int j1 = active ? (int)((j / g.n0) % g.n1) : 0;
    const int j2 = active ? (int)(j / ((long)g.n0 * g.n1)) : 0;
    const T h = T(g.h), inv_h = T(1.0 / g.h);
    T acc[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) acc[b] = T(0);

    for (long k0 = 0; k0 < N; k0 += kTile) {
        const long k = k0 + threadIdx.x;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            double v = 0.0;
            if (k < N) v = weighted ? ss[k] * x[k + b * N] : x[k + b * N];
            sw[threadIdx.x * RB + b] = T(v);
        }
        __syncthreads();
        const int cnt = (N - k0) < kTile ? (int)(N - k0) : kTile;
        int c0 = (int)(k0 % g.n0), c1 = (int)((k0 / g.n0) % g.n1), c2 = (int)(k0 / ((long)g.n0 * g.n1));
        if (active) {
            for (int t = 0; t < cnt; ++t) {
                const long kk = k0 + t;
                if (kk != j) {
                    const int d0 = j0 - c0, d1 = j1 - c1, d2 = j2 - c2;
                    const int K = d0 * d0 + d1 * d1 + d2 * d2;
                    const T r = h * sqrt(T(K));
                    T tau;
                    if (RAY) {
                        const bool lo = j < kk;
                        const T a0 = h * (T(lo ? j0 : c0) + T(0.5)), a1 = h * (T(lo ? j1 : c1) + T(0.5));
                        const T a2 = h * (T(lo ? j2 : c2) + T(0.5));
                        const T b0 = h * (T(lo ? c0 : j0) + T(0.5)), b1 = h * (T(lo ? c1 : j1) + T(0.5));
                        const T b2 = h * (T(lo ? c2 : j2) + T(0.5));
                        tau = tau_march<T>(st, g, inv_h, a0, a1, a2, b0, b1, b2, steps_grid(K), r);
                    } else {
                        tau = sigma * r;
                    }
                    T gk;
                    if (itab) {
                        // (M-ii): the cell integral replaces |offset|^{1-d}
                        const int a0 = d0 < 0 ? -d0 : d0, a1 = d1 < 0 ? -d1 : d1, a2 = d2 < 0 ? -d2 : d2;
                        gk = exp(-tau) * T(itab[a0 + (long)g.n0 * (a1 + (long)g.n1 * a2)]);
                    } else {
                        const T rp = (g.dim == 2) ? T(sqrt(T(K))) : T(K);
                        gk = exp(-tau) / rp;
                    }
#pragma unroll
                    for (int b = 0; b < RB; ++b) acc[b] += gk * sw[t * RB + b];
                }
                if (++c0 == g.n0) {
                    c0 = 0;
                    if (++c1 == g.n1) { c1 = 0; ++c2; }
                }
            }
        }
        __syncthreads();
    }
    if (active) {
        // entries are h^d G = h^d exp(-tau) / (area h^{d-1} K^{(d-1)/2}) = (h / area) exp(-tau)/rp
        const double wself_scale = weighted ? ss[j] : 1.0;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const double xj = x[j + b * N];
            double v = (double)hd_over_area * (double)acc[b] + diag[j] * wself_scale * xj;
            y[j + b * N] = (op == ERT_OP_A) ? xj - v : v;
        }
    }
}

template <typename T, bool RAY>
ert_status launch_direct(ert_plan_impl* p, const T* st, int op, const double* x, double* y, int nrhs)
{
    const long N = p->N;
    const int weighted = (op != ERT_OP_G);
    const T sigma = T(p->sigma_const);
    const T scale = T(p->geo.h / surface_area(p->geo.dim));
    dim3 grid((unsigned)((N + kTile - 1) / kTile));
    int b = 0;
    while (b < nrhs) {
        const int left = nrhs - b;
        const double* xb = x + (long)b * N;
        double* yb = y + (long)b * N;
        if (left >= 4) {
            hipLaunchKernelGGL((k_direct<T, RAY, 4>), grid, dim3(kTile), 0, p->stream, p->geo, st, sigma, scale,
                               xb, p->d_ss, weighted, N, p->d_diag, p->d_itab, op, yb);
            b += 4;
        } else if (left >= 2) {
            hipLaunchKernelGGL((k_direct<T, RAY, 2>), grid, dim3(kTile), 0, p->stream, p->geo, st, sigma, scale,
                               xb, p->d_ss, weighted, N, p->d_diag, p->d_itab, op, yb);
            b += 2;
        } else {
            hipLaunchKernelGGL((k_direct<T, RAY, 1>), grid, dim3(kTile), 0, p->stream, p->geo, st, sigma, scale,
                               xb, p->d_ss, weighted, N, p->d_diag, p->d_itab, op, yb);
            b += 1;
        }
        ERT_HIP(hipGetLastError());
    }
    return ERT_OK;
}

}  // namespace

namespace {

// Launch k_selfcell for cells [0, ncell) (ray rule: the plan's sigma_t; else
// the constant `sigma`) into diag, with the plan's angular and radial rules.
ert_status selfcell_launch(ert_plan_impl* p, int ray, double sigma, long ncell, double* diag)
{
    const int nang = 16, nrad = 10;
    std::vector<double> ax, aw, rx, rw;
    gauss_legendre(nang, ax, aw);
    gauss_legendre(nrad, rx, rw);
    std::vector<double> pack;
    pack.insert(pack.end(), ax.begin(), ax.end());
    pack.insert(pack.end(), aw.begin(), aw.end());
    pack.insert(pack.end(), rx.begin(), rx.end());
    pack.insert(pack.end(), rw.begin(), rw.end());
    double* d = nullptr;
    ERT_HIP(hipMalloc(&d, pack.size() * sizeof(double)));
    ert_status st = ERT_HIPST(hipMemcpyAsync(d, pack.data(), pack.size() * sizeof(double), hipMemcpyHostToDevice,
                                             p->stream));
    // chunk the launch so one dispatch never holds the GPU for long
    const long chunk = 65536;
    for (long j0 = 0; j0 < ncell && st == ERT_OK; j0 += chunk) {
        long cnt = (ncell - j0) < chunk ? (ncell - j0) : chunk;
        hipLaunchKernelGGL(k_selfcell, dim3((unsigned)cnt), dim3(256), 0, p->stream, p->geo, ray, sigma, p->d_st, d,
                           d + nang, nang, d + 2 * nang, d + 2 * nang + nrad, nrad, j0, diag);
        st = ERT_HIPST(hipGetLastError());
    }
    if (st == ERT_OK) st = ERT_HIPST(hipStreamSynchronize(p->stream));
    (void)hipFree(d);
    return st;
}

}  // namespace

ert_status selfcell_compute(ert_plan_impl* p)
{
    if (p->o.scheme == 1) {
        // (M-ii): the table of cell integrals, and A_jj = h cell_int(0) / |S^{d-1}|
        const long M = (long)p->geo.n0 * p->geo.n1 * p->geo.n2;
        ERT_HIP(hipMalloc(&p->d_itab, M * sizeof(double)));
        hipLaunchKernelGGL(k_itab, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, p->stream, p->geo.dim, p->geo.n0,
                           p->geo.n1, p->geo.n2, p->d_itab);
        ERT_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_fill_scaled, dim3((unsigned)((p->N + 255) / 256)), dim3(256), 0, p->stream, p->d_diag,
                           p->N, p->d_itab, p->geo.h / surface_area(p->geo.dim));
        ERT_HIP(hipGetLastError());
        ERT_HIP(hipStreamSynchronize(p->stream));
        return ERT_OK;
    }
    const int ray = p->o.kernel == ERT_K_RAY_MIDPOINT;
    ERT_TRY(selfcell_launch(p, ray, p->sigma_const, ray ? p->N : 1, p->d_diag));
    if (!ray) {
        hipLaunchKernelGGL(k_fill, dim3((unsigned)((p->N + 255) / 256)), dim3(256), 0, p->stream, p->d_diag, p->N,
                           p->d_diag);
        ERT_HIP(hipGetLastError());
        ERT_HIP(hipStreamSynchronize(p->stream));
    }
    return ERT_OK;
}

ert_status selfcell_constant(ert_plan_impl* p, double sigma, double* value)
{
    double* d = nullptr;
    ERT_HIP(hipMalloc(&d, sizeof(double)));
    ert_status st = selfcell_launch(p, 0, sigma, 1, d);
    if (st == ERT_OK) st = ERT_HIPST(hipMemcpy(value, d, sizeof(double), hipMemcpyDeviceToHost));
    (void)hipFree(d);
    return st;
}

ert_status direct_apply(ert_plan_impl* p, int op, int prec, const double* x, double* y, int nrhs)
{
    const bool ray = p->o.kernel == ERT_K_RAY_MIDPOINT;
    if (prec == ERT_FP64) {
        return ray ? launch_direct<double, true>(p, p->d_st, op, x, y, nrhs)
                   : launch_direct<double, false>(p, p->d_st, op, x, y, nrhs);
    }
    return ray ? launch_direct<float, true>(p, p->d_st32, op, x, y, nrhs)
               : launch_direct<float, false>(p, p->d_st32, op, x, y, nrhs);
}

}  // namespace ertvie
