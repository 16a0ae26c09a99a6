// FFT-based preconditioner (Sec. 4.4, eqs. EQ: FFT and EQ:SOL FFT): the
// equation in the mean medium, solved on a periodic grid twice the size of the
// domain with zero extension of the residual and restriction of the result,
//
//   z = P IDFT( DFT(E r) / c ),   c = 1 - sbar_s DFT(w),
//
// w the constant-medium kernel h^d G on the periodic offsets with the self-cell
// integral at offset 0.  Everything runs as line transforms in LDS: a workgroup
// takes a few lines of one axis, loads them (coalesced along the contiguous
// axis of the line set), runs a mixed-radix Stockham FFT (radices 8, 4, 2, 3,
// 5, 7) between two LDS buffers and stores the part that is needed.  Zero
// padding and restriction never touch memory: the forward passes read only the
// n_a input positions and the inverse passes write only the n_a kept ones.
//
// Apply, 3D (T1: n2 x n1 x H0, T2: n2 x m1 x H0 complex FP32, H0 = m0/2 + 1):
//   x forward (real input, half spectrum out)     r  -> T1
//   y forward (n1 of m1 inputs)                   T1 -> T2
//   z forward, times 1/c, z inverse (n2 kept)     T2 -> T2
//   y inverse (n1 kept)                           T2 -> T1
//   x inverse (Hermitian half in, real out)       T1 -> z
// 2D drops the y passes and does forward / 1/c / inverse along y.
// The symbol is built once in FP64 by the same line kernels on the full
// periodic grid (w has no zero padding) and folded to its distinct values
// (c is even along every axis): 1/c on (m2/2 + 1) x (m1/2 + 1) x H0, FP32.
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace ertvie {

template <typename R>
struct Cx {
    R re, im;
};

struct FftPc {
    int dim = 0;
    int n[3] = {1, 1, 1};
    int m[3] = {1, 1, 1};
    int H[3] = {1, 1, 1};        // m_a / 2 + 1
    int nfac[3] = {0, 0, 0};
    int fac[3][12];
    double sbar_t = 0, sbar_s = 0, dself = 0, cmin = 0, cmax = 0;
    float* invc = nullptr;       // folded 1/c
    Cx<float>* tw[3] = {nullptr, nullptr, nullptr};   // exp(-2 pi i j / m_a), FP32
    Cx<float>* t1 = nullptr;
    Cx<float>* t2 = nullptr;
    long bytes = 0;
};

namespace {

constexpr int kThreads = 256;
constexpr size_t kLdsMax = 64 * 1024;
constexpr int kMaxPeriod = 1024;

// Smallest integer >= 2 n with no prime factor above 7.
int smooth_period(int n)
{
    for (int m = 2 * n;; ++m) {
        int k = m;
        for (int p : {2, 3, 5, 7})
            while (k % p == 0) k /= p;
        if (k == 1) return m;
    }
}

int factorize(int m, int* f)
{
    int c = 0;
    for (int r : {8, 4, 2, 3, 5, 7})
        while (m % r == 0) {
            f[c++] = r;
            m /= r;
        }
    return c;
}

// One batch of line transforms.  Line (a, b), a in [0, A), b in [0, B), element
// i at base + a * sa + b * sb + i * si (source) and likewise for the destination.
struct Lines {
    int m, nin, nout;
    int A, B, TX;
    long sa, sb, si;
    long da, db, di;
    int nfac;
    int fac[12];
    double scale;
    const float* invc;           // mid pass: 1/c at fold(i) * ci + fold_b(b) * cb + a * ca
    long ca, cb, ci;
    int mb;                      // b folds as min(b, mb - b) when mb > 0
};

enum { kFwdReal = 0, kCplx = 1, kMid = 2, kInvReal = 3 };

template <typename R>
__device__ __forceinline__ Cx<R> twmul(Cx<R> x, Cx<R> w, bool inv)
{
    // x * w, or x * conj(w) for the inverse direction
    const R wi = inv ? -w.im : w.im;
    return {x.re * w.re - x.im * wi, x.re * wi + x.im * w.re};
}

template <typename R, int RAD>
__device__ void fft_stage(const Cx<R>* __restrict__ in, Cx<R>* __restrict__ out, const Cx<R>* __restrict__ tw,
                          int m, int p, int TX, int TXP, bool inv)
{
    const int mr = m / RAD, step = m / (p * RAD);
    for (int e = threadIdx.x; e < TX * mr; e += kThreads) {
        const int t = e % TX, j = e / TX, k = j % p;
        Cx<R> x[RAD];
#pragma unroll
        for (int q = 0; q < RAD; ++q) x[q] = in[(j + q * mr) * TXP + t];
#pragma unroll
        for (int q = 1; q < RAD; ++q) x[q] = twmul(x[q], tw[q * k * step], inv);   // q k step < m
        const int base = (j - k) * RAD + k;
#pragma unroll
        for (int s = 0; s < RAD; ++s) {
            Cx<R> acc = x[0];
#pragma unroll
            for (int q = 1; q < RAD; ++q) {
                const Cx<R> v = twmul(x[q], tw[((q * s) % RAD) * mr], inv);
                acc.re += v.re;
                acc.im += v.im;
            }
            out[(base + s * p) * TXP + t] = acc;
        }
    }
}

// All stages; returns the buffer holding the result.
template <typename R>
__device__ Cx<R>* fft_lines(Cx<R>* a, Cx<R>* b, const Cx<R>* tw, const Lines& L, int TXP, bool inv)
{
    int p = 1;
    for (int s = 0; s < L.nfac; ++s) {
        const int r = L.fac[s];
        switch (r) {
        case 8: fft_stage<R, 8>(a, b, tw, L.m, p, L.TX, TXP, inv); break;
        case 4: fft_stage<R, 4>(a, b, tw, L.m, p, L.TX, TXP, inv); break;
        case 2: fft_stage<R, 2>(a, b, tw, L.m, p, L.TX, TXP, inv); break;
        case 3: fft_stage<R, 3>(a, b, tw, L.m, p, L.TX, TXP, inv); break;
        case 5: fft_stage<R, 5>(a, b, tw, L.m, p, L.TX, TXP, inv); break;
        default: fft_stage<R, 7>(a, b, tw, L.m, p, L.TX, TXP, inv); break;
        }
        __syncthreads();
        Cx<R>* t = a;
        a = b;
        b = t;
        p *= r;
    }
    return a;
}

__device__ __forceinline__ int fold(int i, int m) { return i <= m - i ? i : m - i; }

// MODE kFwdReal: real FP64 source, forward, half spectrum out (nout = H).
// kCplx: complex source and destination, one direction (INV).
// kMid: forward, times 1/c, inverse.  kInvReal: Hermitian half in (nin = H),
// inverse, real part times `scale` out as FP64.
template <typename R, int MODE, bool INV>
__global__ __launch_bounds__(kThreads) void k_lines(Lines L, const void* src_, void* dst_,
                                                    const Cx<R>* __restrict__ tw)
{
    extern __shared__ unsigned char lds_raw[];
    const int m = L.m, TX = L.TX, TXP = TX == 1 ? 1 : TX + 1;
    Cx<R>* tws = reinterpret_cast<Cx<R>*>(lds_raw);
    Cx<R>* b0 = tws + m;
    Cx<R>* b1 = b0 + (size_t)m * TXP;
    const int tiles = (L.A + TX - 1) / TX;
    const int a0 = (int)(blockIdx.x % tiles) * TX;
    const long b = blockIdx.x / tiles;
    const int tv = min(TX, L.A - a0);     // valid lines in this tile
    for (int i = threadIdx.x; i < m; i += kThreads) tws[i] = tw[i];

    // load (zeros beyond nin and for missing lines)
    const bool rows = L.si == 1;          // lines run along the contiguous axis
    const long sbase = a0 * L.sa + b * L.sb;
    for (int e = threadIdx.x; e < TX * m; e += kThreads) {
        const int i = rows ? e % m : e / TX;
        const int t = rows ? e / m : e % TX;
        Cx<R> v = {R(0), R(0)};
        if (t < tv && i < L.nin) {
            const long off = sbase + t * L.sa + i * L.si;
            if (MODE == kFwdReal) {
                v.re = (R)static_cast<const double*>(src_)[off];
            } else {
                v = static_cast<const Cx<R>*>(src_)[off];
            }
        }
        b0[i * TXP + t] = v;
    }
    __syncthreads();
    if (MODE == kInvReal) {
        // X[k] = conj(X[m - k]) above the stored half
        for (int e = threadIdx.x; e < TX * m; e += kThreads) {
            const int i = e / TX, t = e % TX;
            if (i >= L.nin) {
                Cx<R> v = b0[(m - i) * TXP + t];
                b0[i * TXP + t] = {v.re, -v.im};
            }
        }
        __syncthreads();
    }

    Cx<R>* res = fft_lines<R>(b0, b1, tws, L, TXP, MODE == kInvReal || (MODE == kCplx && INV));
    if (MODE == kMid) {
        const long fb = L.mb > 0 ? fold((int)b, L.mb) : b;
        for (int e = threadIdx.x; e < TX * m; e += kThreads) {
            const int i = e / TX, t = e % TX;
            const R s = (t < tv) ? (R)L.invc[fold(i, m) * L.ci + fb * L.cb + (a0 + t) * L.ca] : R(0);
            Cx<R> v = res[i * TXP + t];
            res[i * TXP + t] = {v.re * s, v.im * s};
        }
        __syncthreads();
        Cx<R>* other = res == b0 ? b1 : b0;
        res = fft_lines<R>(res, other, tws, L, TXP, true);
    }

    // store the kept positions
    const long dbase = a0 * L.da + b * L.db;
    const bool drows = L.di == 1;
    for (int e = threadIdx.x; e < TX * L.nout; e += kThreads) {
        const int i = drows ? e % L.nout : e / TX;
        const int t = drows ? e / L.nout : e % TX;
        if (t >= tv) continue;
        const long off = dbase + t * L.da + i * L.di;
        const Cx<R> v = res[i * TXP + t];
        if (MODE == kInvReal)
            static_cast<double*>(dst_)[off] = (double)v.re * L.scale;
        else
            static_cast<Cx<R>*>(dst_)[off] = v;
    }
}

// Sums of sigma_t and sigma_s: per-block partials, then one block, fixed order.
__global__ __launch_bounds__(kThreads) void k_sum2(const double* __restrict__ a, const double* __restrict__ c,
                                                   long N, double* __restrict__ part)
{
    __shared__ double sa[kThreads], sc[kThreads];
    double x = 0.0, y = 0.0;
    for (long i = blockIdx.x * (long)kThreads + threadIdx.x; i < N; i += (long)gridDim.x * kThreads) {
        x += a[i];
        y += c[i];
    }
    sa[threadIdx.x] = x;
    sc[threadIdx.x] = y;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sa[threadIdx.x] += sa[threadIdx.x + s];
            sc[threadIdx.x] += sc[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sa[0];
        part[2 * blockIdx.x + 1] = sc[0];
    }
}

__global__ __launch_bounds__(kThreads) void k_sum2_final(double* __restrict__ part, int nb)
{
    __shared__ double sa[kThreads], sc[kThreads];
    double x = 0.0, y = 0.0;
    for (int i = threadIdx.x; i < nb; i += kThreads) {
        x += part[2 * i];
        y += part[2 * i + 1];
    }
    sa[threadIdx.x] = x;
    sc[threadIdx.x] = y;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sa[threadIdx.x] += sa[threadIdx.x + s];
            sc[threadIdx.x] += sc[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[0] = sa[0];
        part[1] = sc[0];
    }
}

// Kernel array of the constant medium on the periodic grid [m2][m1][m0]: the
// matrix entry of the plan's discretisation at each periodic offset, (M-iii)
// h^d G or (M-ii) h E cell_int / |S^{d-1}|.
__global__ __launch_bounds__(kThreads) void k_kernel_array(int dim, int m0, int m1, int m2, double h, double sigma,
                                                           double dself, int mii, double* __restrict__ w)
{
    const long M = (long)m0 * m1 * m2;
    const long i = blockIdx.x * (long)kThreads + threadIdx.x;
    if (i >= M) return;
    const int i0 = (int)(i % m0), i1 = (int)((i / m0) % m1), i2 = (int)(i / ((long)m0 * m1));
    const double o0 = i0 <= m0 / 2 ? i0 : i0 - m0;
    const double o1 = i1 <= m1 / 2 ? i1 : i1 - m1;
    const double o2 = i2 <= m2 / 2 ? i2 : i2 - m2;
    const double K = o0 * o0 + o1 * o1 + o2 * o2;
    if (K == 0.0) {
        w[i] = dself;
        return;
    }
    const double r = h * sqrt(K);
    if (mii) {
        w[i] = h * exp(-sigma * r) * cell_int(dim, o0, o1, o2) / surface_area(dim);
        return;
    }
    const double hd = dim == 2 ? h * h : h * h * h;
    w[i] = hd * exp(-sigma * r) / (surface_area(dim) * (dim == 2 ? r : r * r));
}

// 1/c on the folded grid [H2][H1][H0] from the full spectrum T [m2][m1][H0];
// per-block extremes of c for the positivity check.
__global__ __launch_bounds__(kThreads) void k_symbol(const Cx<double>* __restrict__ T, int H0, int H1, int H2, int m1,
                                                     double sbar_s, float* __restrict__ invc,
                                                     double* __restrict__ ext)
{
    __shared__ double smin[kThreads], smax[kThreads];
    const long M = (long)H0 * H1 * H2;
    const long i = blockIdx.x * (long)kThreads + threadIdx.x;
    double lo = 1e300, hi = -1e300;
    if (i < M) {
        const int k0 = (int)(i % H0), k1 = (int)((i / H0) % H1), k2 = (int)(i / ((long)H0 * H1));
        const double c = 1.0 - sbar_s * T[((long)k2 * m1 + k1) * H0 + k0].re;
        invc[i] = (float)(1.0 / c);
        lo = hi = c;
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ext[2 * blockIdx.x] = smin[0];
        ext[2 * blockIdx.x + 1] = smax[0];
    }
}

template <typename R>
size_t lds_bytes(int m, int TX)
{
    const int TXP = TX == 1 ? 1 : TX + 1;
    return sizeof(Cx<R>) * (size_t)m * (1 + 2 * (size_t)TXP);
}

template <typename R>
int lines_per_group(int m)
{
    int TX = 16;
    while (TX > 1 && lds_bytes<R>(m, TX) > kLdsMax) TX /= 2;
    return TX;
}

template <typename R, int MODE, bool INV>
ert_status launch_lines(hipStream_t s, Lines L, const void* src, void* dst, const Cx<R>* tw)
{
    L.TX = lines_per_group<R>(L.m);
    const size_t lds = lds_bytes<R>(L.m, L.TX);
    if (lds > kLdsMax) {
        record_error("ert_vie_fft_precond: line transform does not fit in LDS");
        return ERT_EUNSUPPORTED;
    }
    const long tiles = (L.A + L.TX - 1) / L.TX;
    const long blocks = tiles * L.B;
    if (blocks <= 0) return ERT_OK;
    if (blocks > 0x7fffffffL) return ERT_EUNSUPPORTED;
    hipLaunchKernelGGL((k_lines<R, MODE, INV>), dim3((unsigned)blocks), dim3(kThreads), lds, s, L, src, dst, tw);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

Lines make_lines(const FftPc* f, int axis, int nin, int nout, int A, int B)
{
    Lines L;
    std::memset(&L, 0, sizeof(L));
    L.m = f->m[axis];
    L.nin = nin;
    L.nout = nout;
    L.A = A;
    L.B = B;
    L.nfac = f->nfac[axis];
    for (int i = 0; i < L.nfac; ++i) L.fac[i] = f->fac[axis][i];
    L.scale = 1.0;
    return L;
}

template <typename R>
ert_status upload_twiddles(hipStream_t s, int m, Cx<R>** out)
{
    std::vector<Cx<R>> h(m);
    for (int j = 0; j < m; ++j) {
        const double a = -2.0 * kPi * (double)j / (double)m;
        h[j] = {(R)std::cos(a), (R)std::sin(a)};
    }
    ERT_HIP(hipMalloc(out, sizeof(Cx<R>) * m));
    ERT_HIP(hipMemcpyAsync(*out, h.data(), sizeof(Cx<R>) * m, hipMemcpyHostToDevice, s));
    ERT_HIP(hipStreamSynchronize(s));
    return ERT_OK;
}

// The symbol: kernel array (FP64), its DFT along every axis, 1/c folded.
ert_status build_symbol(ert_plan_impl* p, FftPc* f)
{
    hipStream_t s = p->stream;
    const int dim = f->dim;
    const int m0 = f->m[0], m1 = f->m[1], m2 = f->m[2], H0 = f->H[0];
    const long M = (long)m0 * m1 * m2;
    const long MH = (long)H0 * m1 * m2;
    double* w = nullptr;
    Cx<double>* T = nullptr;
    Cx<double>* tw[3] = {nullptr, nullptr, nullptr};
    double* ext = nullptr;
    ert_status st = ERT_OK;
    const long nsym = (long)f->H[0] * f->H[1] * f->H[2];
    const long eblocks = (nsym + kThreads - 1) / kThreads;
    do {
        if (hipMalloc(&w, sizeof(double) * M) != hipSuccess || hipMalloc(&T, sizeof(Cx<double>) * MH) != hipSuccess ||
            hipMalloc(&ext, sizeof(double) * 2 * eblocks) != hipSuccess) {
            record_error("ert_vie_fft_precond: symbol build allocation failed");
            st = ERT_ENOMEM;
            break;
        }
        for (int a = 0; a < dim && st == ERT_OK; ++a) st = upload_twiddles<double>(s, f->m[a], &tw[a]);
        if (st != ERT_OK) break;
        hipLaunchKernelGGL(k_kernel_array, dim3((unsigned)((M + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, dim,
                           m0, m1, m2, p->geo.h, f->sbar_t, f->dself, p->o.scheme, w);
        st = ERT_HIPST(hipGetLastError());
        if (st != ERT_OK) break;
        // x: every row of w, real in, half spectrum out
        Lines L = make_lines(f, 0, m0, H0, m1 * m2, 1);
        L.sa = m0;
        L.si = 1;
        L.da = H0;
        L.di = 1;
        st = launch_lines<double, kFwdReal, false>(s, L, w, T, tw[0]);
        if (st != ERT_OK) break;
        // y: lines (k0, i2), in place
        L = make_lines(f, 1, m1, m1, H0, m2);
        L.sa = 1;
        L.sb = (long)m1 * H0;
        L.si = H0;
        L.da = 1;
        L.db = (long)m1 * H0;
        L.di = H0;
        st = launch_lines<double, kCplx, false>(s, L, T, T, tw[1]);
        if (st != ERT_OK) break;
        if (dim == 3) {
            L = make_lines(f, 2, m2, m2, H0, m1);
            L.sa = 1;
            L.sb = H0;
            L.si = (long)m1 * H0;
            L.da = 1;
            L.db = H0;
            L.di = (long)m1 * H0;
            st = launch_lines<double, kCplx, false>(s, L, T, T, tw[2]);
            if (st != ERT_OK) break;
        }
        hipLaunchKernelGGL(k_symbol, dim3((unsigned)eblocks), dim3(kThreads), 0, s, T, H0, f->H[1], f->H[2], m1,
                           f->sbar_s, f->invc, ext);
        st = ERT_HIPST(hipGetLastError());
        if (st != ERT_OK) break;
        std::vector<double> e(2 * eblocks);
        st = ERT_HIPST(hipMemcpyAsync(e.data(), ext, sizeof(double) * 2 * eblocks, hipMemcpyDeviceToHost, s));
        if (st == ERT_OK) st = ERT_HIPST(hipStreamSynchronize(s));
        if (st != ERT_OK) break;
        f->cmin = 1e300;
        f->cmax = -1e300;
        for (long i = 0; i < eblocks; ++i) {
            f->cmin = std::min(f->cmin, e[2 * i]);
            f->cmax = std::max(f->cmax, e[2 * i + 1]);
        }
        if (!(f->cmin > 0.0) || !std::isfinite(f->cmax)) {
            record_error("ert_vie_fft_precond: the symbol of the mean medium is not positive");
            st = ERT_EUNSUPPORTED;
        }
    } while (0);
    (void)hipStreamSynchronize(s);
    (void)hipFree(w);
    (void)hipFree(T);
    (void)hipFree(ext);
    for (auto* t : tw) (void)hipFree(t);
    return st;
}

ert_status fftpc_build(ert_plan_impl* p)
{
    if (p->fftpc) return ERT_OK;
    FftPc* f = new FftPc();
    f->dim = p->o.dim;
    f->n[0] = p->geo.n0;
    f->n[1] = p->geo.n1;
    f->n[2] = f->dim == 3 ? p->geo.n2 : 1;
    for (int a = 0; a < 3; ++a) {
        f->m[a] = a < f->dim ? smooth_period(f->n[a]) : 1;
        f->H[a] = a < f->dim ? f->m[a] / 2 + 1 : 1;
        f->nfac[a] = a < f->dim ? factorize(f->m[a], f->fac[a]) : 0;
        if (f->m[a] > kMaxPeriod) {
            delete f;
            record_error("ert_vie_fft_precond: a periodic grid axis would exceed 1024 cells");
            return ERT_EUNSUPPORTED;
        }
    }
    ert_status st = ERT_OK;
    double* part = nullptr;
    do {
        // mean medium
        const int nb = 1024;
        if (hipMalloc(&part, sizeof(double) * 2 * nb) != hipSuccess) {
            st = ERT_ENOMEM;
            break;
        }
        hipLaunchKernelGGL(k_sum2, dim3(nb), dim3(kThreads), 0, p->stream, p->d_st, p->d_ss, p->N, part);
        hipLaunchKernelGGL(k_sum2_final, dim3(1), dim3(kThreads), 0, p->stream, part, nb);
        st = ERT_HIPST(hipGetLastError());
        if (st != ERT_OK) break;
        double sums[2];
        st = ERT_HIPST(hipMemcpyAsync(sums, part, sizeof(sums), hipMemcpyDeviceToHost, p->stream));
        if (st == ERT_OK) st = ERT_HIPST(hipStreamSynchronize(p->stream));
        if (st != ERT_OK) break;
        f->sbar_t = sums[0] / (double)p->N;
        f->sbar_s = sums[1] / (double)p->N;
        if (p->o.scheme == 1)   // (M-ii): the diagonal does not depend on the medium
            st = ERT_HIPST(hipMemcpy(&f->dself, p->d_diag, sizeof(double), hipMemcpyDeviceToHost));
        else
            st = selfcell_constant(p, f->sbar_t, &f->dself);
        if (st != ERT_OK) break;
        const long nsym = (long)f->H[0] * f->H[1] * f->H[2];
        const long n1 = (long)f->n[2] * f->n[1] * f->H[0];
        const long n2 = f->dim == 3 ? (long)f->n[2] * f->m[1] * f->H[0] : 0;
        if (hipMalloc(&f->invc, sizeof(float) * nsym) != hipSuccess ||
            hipMalloc(&f->t1, sizeof(Cx<float>) * n1) != hipSuccess ||
            (n2 > 0 && hipMalloc(&f->t2, sizeof(Cx<float>) * n2) != hipSuccess)) {
            record_error("ert_vie_fft_precond: allocation failed");
            st = ERT_ENOMEM;
            break;
        }
        f->bytes = (long)(sizeof(float) * nsym + sizeof(Cx<float>) * (n1 + n2));
        for (int a = 0; a < f->dim && st == ERT_OK; ++a) {
            st = upload_twiddles<float>(p->stream, f->m[a], &f->tw[a]);
            f->bytes += (long)sizeof(Cx<float>) * f->m[a];
        }
        if (st != ERT_OK) break;
        st = build_symbol(p, f);
    } while (0);
    (void)hipFree(part);
    if (st != ERT_OK) {
        fftpc_destroy(f);
        return st;
    }
    p->fftpc = f;
    return ERT_OK;
}

// One column.
ert_status fftpc_column(ert_plan_impl* p, const FftPc* f, const double* r, double* z)
{
    hipStream_t s = p->stream;
    const int n0 = f->n[0], n1 = f->n[1], n2 = f->n[2];
    const int m0 = f->m[0], m1 = f->m[1], m2 = f->m[2], H0 = f->H[0];
    // x forward: rows (i1, i2) of r -> T1 [n2][n1][H0]
    Lines L = make_lines(f, 0, n0, H0, n1 * n2, 1);
    L.sa = n0;
    L.si = 1;
    L.da = H0;
    L.di = 1;
    ERT_TRY((launch_lines<float, kFwdReal, false>(s, L, r, f->t1, f->tw[0])));
    if (f->dim == 2) {
        // y: forward, 1/c, inverse, in place on T1 [n1][H0]
        L = make_lines(f, 1, n1, n1, H0, 1);
        L.sa = L.da = 1;
        L.si = L.di = H0;
        L.invc = f->invc;
        L.ci = H0;
        L.ca = 1;
        L.cb = 0;
        L.mb = 0;
        ERT_TRY((launch_lines<float, kMid, false>(s, L, f->t1, f->t1, f->tw[1])));
    } else {
        // y forward: T1 [n2][n1][H0] -> T2 [n2][m1][H0]
        L = make_lines(f, 1, n1, m1, H0, n2);
        L.sa = 1;
        L.sb = (long)n1 * H0;
        L.si = H0;
        L.da = 1;
        L.db = (long)m1 * H0;
        L.di = H0;
        ERT_TRY((launch_lines<float, kCplx, false>(s, L, f->t1, f->t2, f->tw[1])));
        // z: forward, 1/c, inverse on lines (k0, k1), n2 of m2 positions in and out
        L = make_lines(f, 2, n2, n2, H0, m1);
        L.sa = L.da = 1;
        L.sb = L.db = H0;
        L.si = L.di = (long)m1 * H0;
        L.invc = f->invc;
        L.ci = (long)f->H[1] * H0;
        L.cb = H0;
        L.ca = 1;
        L.mb = m1;
        ERT_TRY((launch_lines<float, kMid, false>(s, L, f->t2, f->t2, f->tw[2])));
        // y inverse: T2 -> T1, n1 kept
        L = make_lines(f, 1, m1, n1, H0, n2);
        L.sa = 1;
        L.sb = (long)m1 * H0;
        L.si = H0;
        L.da = 1;
        L.db = (long)n1 * H0;
        L.di = H0;
        ERT_TRY((launch_lines<float, kCplx, true>(s, L, f->t2, f->t1, f->tw[1])));
    }
    // x inverse: T1 rows -> z rows, n0 kept, 1 / (m0 m1 m2)
    L = make_lines(f, 0, H0, n0, n1 * n2, 1);
    L.sa = H0;
    L.si = 1;
    L.da = n0;
    L.di = 1;
    L.scale = 1.0 / ((double)m0 * m1 * m2);
    ERT_TRY((launch_lines<float, kInvReal, false>(s, L, f->t1, z, f->tw[0])));
    return ERT_OK;
}

}  // namespace

void fftpc_destroy(FftPc* f)
{
    if (!f) return;
    (void)hipFree(f->invc);
    (void)hipFree(f->t1);
    (void)hipFree(f->t2);
    for (auto* t : f->tw) (void)hipFree(t);
    delete f;
}

ert_status fftpc_apply(ert_plan_impl* p, const double* r, double* z, int nrhs)
{
    ERT_TRY(fftpc_build(p));
    for (int c = 0; c < nrhs; ++c) ERT_TRY(fftpc_column(p, p->fftpc, r + (size_t)c * p->N, z + (size_t)c * p->N));
    return ERT_OK;
}

ert_status fftpc_info(ert_plan_impl* p, ert_fft_info* info)
{
    ERT_TRY(fftpc_build(p));
    const FftPc* f = p->fftpc;
    std::memset(info, 0, sizeof(*info));
    for (int a = 0; a < 3; ++a) info->m[a] = f->m[a];
    info->sigma_t_mean = f->sbar_t;
    info->sigma_s_mean = f->sbar_s;
    info->self_cell = f->dself;
    info->symbol_min = f->cmin;
    info->symbol_max = f->cmax;
    info->bytes = f->bytes;
    return ERT_OK;
}

}  // namespace ertvie
