// Internal definitions shared by the library's translation units: the plan
// object, launch helpers and the device functions that evaluate the transport
// kernel.  Not part of the ABI (include/ertvie.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "ertvie.h"

namespace ertvie {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- errors ---

// Failure bookkeeping behind ert_vie_last_error (thread-local text).
void record_hip_error(const char* what, hipError_t e, const char* file, int line);
void record_error(const char* msg);

#define ERT_HIP(call)                                              \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) {                                    \
            ::ertvie::record_hip_error(#call, e_, __FILE__, __LINE__); \
            return ERT_EDEVICE;                                    \
        }                                                          \
    } while (0)

// hipError_t -> ert_status with bookkeeping, for code that cannot return early
#define ERT_HIPST(call) (((call) == hipSuccess) ? ERT_OK : (::ertvie::record_hip_error(#call, hipGetLastError(), __FILE__, __LINE__), ERT_EDEVICE))

#define ERT_TRY(call)                                              \
    do {                                                           \
        ert_status s_ = (call);                                    \
        if (s_ != ERT_OK) return s_;                               \
    } while (0)

// --------------------------------------------------------------- geometry ---

// Grid seen by device code.  n[2] == 1 for dim 2.
struct Geo {
    int dim;
    int n0, n1, n2;
    double h;
};

// |S^{d-1}|
__host__ __device__ inline double surface_area(int dim) { return dim == 2 ? 2.0 * kPi : 4.0 * kPi; }

// Clamped d-linear interpolation of cell-centred sigma_t at point p (real T).
template <typename T>
__device__ __forceinline__ T sigma_at(const T* __restrict__ st, const Geo& g, T inv_h, T p0, T p1,
                                      T p2)
{
    const int n[3] = {g.n0, g.n1, g.n2};
    const T p[3] = {p0, p1, p2};
    int i0[3] = {0, 0, 0};
    T t[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a < g.dim && n[a] > 1) {
            T u = p[a] * inv_h - T(0.5);
            T hi = T(n[a] - 1);
            u = u < T(0) ? T(0) : (u > hi ? hi : u);
            int k = (int)floor(u);
            k = k > n[a] - 2 ? n[a] - 2 : k;
            i0[a] = k;
            t[a] = u - T(k);
        }
    }
    const int b0 = i0[0] + n[0] * (i0[1] + n[1] * i0[2]);
    const int d0 = n[0] > 1 ? 1 : 0;
    const int d1 = n[1] > 1 ? n[0] : 0;
    const int d2 = (g.dim > 2 && n[2] > 1) ? n[0] * n[1] : 0;
    T c00 = st[b0] + t[0] * (st[b0 + d0] - st[b0]);
    T c10 = st[b0 + d1] + t[0] * (st[b0 + d1 + d0] - st[b0 + d1]);
    T c0 = c00 + t[1] * (c10 - c00);
    if (g.dim == 2) return c0;
    T c01 = st[b0 + d2] + t[0] * (st[b0 + d2 + d0] - st[b0 + d2]);
    T c11 = st[b0 + d2 + d1] + t[0] * (st[b0 + d2 + d1 + d0] - st[b0 + d2 + d1]);
    T c1 = c01 + t[1] * (c11 - c01);
    return c0 + t[2] * (c1 - c0);
}

// Smallest m >= 1 with m*m >= 4K: steps of the midpoint rule between two
// collocation points whose integer offsets square-sum to K (step <= h/2).
__host__ __device__ inline int steps_grid(int K)
{
    int m = (int)(2.0 * sqrt((double)K));
    while (m * m < 4 * K) ++m;
    while (m > 1 && (m - 1) * (m - 1) >= 4 * K) --m;
    return m < 1 ? 1 : m;
}

// Midpoint-rule optical depth between points a and b with m steps.
template <typename T>
__device__ __forceinline__ T tau_march(const T* __restrict__ st, const Geo& g, T inv_h, T a0, T a1,
                                       T a2, T b0, T b1, T b2, int m, T r)
{
    T e0 = b0 - a0, e1 = b1 - a1, e2 = b2 - a2;
    T inv_m = T(1) / T(m);
    T s = T(0);
    for (int q = 1; q <= m; ++q) {
        T f = (T(q) - T(0.5)) * inv_m;
        s += sigma_at<T>(st, g, inv_h, a0 + f * e0, a1 + f * e1, a2 + f * e2);
    }
    return r * inv_m * s;
}

// --------------------------------------------------------------- the plan ---

struct FmmData;   // fmm.hip
struct HetCache;  // fmm.hip
struct FftPc;     // fftpc.hip

// Per-stage event timing (ert_vie_profile).
struct Profiler {
    bool on = false;
    struct Rec { int stage; hipEvent_t a, b; };
    std::vector<Rec> recs;
    double ms[ERT_NSTAGES] = {};
    int launches[ERT_NSTAGES] = {};
    std::vector<hipEvent_t> pool;
    hipEvent_t get();
    ert_status begin(hipStream_t s, int stage, hipEvent_t* ev);
    ert_status end(hipStream_t s, int stage, hipEvent_t ev0);
    ert_status resolve();
    void clear();
    ~Profiler();
};

// RAII bracket for one stage of an apply
struct StageTimer {
    Profiler* p;
    hipStream_t s;
    int stage;
    hipEvent_t ev0 = nullptr;
    StageTimer(Profiler* p_, hipStream_t s_, int st) : p(p_), s(s_), stage(st)
    {
        if (p && p->on) p->begin(s, stage, &ev0);
    }
    // close the bracket now
    void stop()
    {
        if (p && p->on && ev0) p->end(s, stage, ev0);
        ev0 = nullptr;
    }
    // drop the bracket (an inner bracket takes over)
    void pause()
    {
        if (p && p->on && ev0) p->pool.push_back(ev0);
        ev0 = nullptr;
    }
    ~StageTimer()
    {
        if (p && p->on && ev0) p->end(s, stage, ev0);
    }
};

struct ert_plan_impl {
    ert_vie_opts o;
    Geo geo;
    long N;
    int nrhs_max;
    hipStream_t stream;
    double sigma_const;          // homogeneous kernel: the constant sigma_t
    std::vector<double> h_st, h_ss;
    double* d_st = nullptr;      // sigma_t FP64
    float* d_st32 = nullptr;     // sigma_t FP32
    double* d_ss = nullptr;      // sigma_s FP64
    double* d_diag = nullptr;    // A_jj FP64
    // GMRES workspace (grown on demand)
    double* d_ws = nullptr;
    size_t ws_elems = 0;
    double* d_red = nullptr;     // reduction partials / small vectors
    size_t red_elems = 0;
    FmmData* fmm[3] = {nullptr, nullptr, nullptr};   // per ert_prec
    HetCache* het[2] = {nullptr, nullptr};   // heterogeneous kernel caches (per Chebyshev order)
    FftPc* fftpc = nullptr;      // FFT-based preconditioner (built on first use)
    Profiler prof;
    bool use_graphs = true;      // FMM applies replay captured graphs
};

// ------------------------------------------------------ launchers (.hip) ---

ert_status selfcell_compute(ert_plan_impl* p);
// A_jj of the constant medium sigma (homogeneous kernel), to host `value`.
ert_status selfcell_constant(ert_plan_impl* p, double sigma, double* value);
ert_status direct_apply(ert_plan_impl* p, int op, int prec, const double* x, double* y, int nrhs);
ert_status fmm_apply(ert_plan_impl* p, int op, int prec, const double* x, double* y, int nrhs);
ert_status fmm_info(ert_plan_impl* p, int prec, ert_fmm_info* info);
void fmm_destroy(FmmData* f);
void het_destroy(HetCache* c);
// FFT-based preconditioner of the mean medium (fftpc.hip): z = M r for nrhs
// columns (device FP64), stream-ordered; builds the symbol on first use.
ert_status fftpc_apply(ert_plan_impl* p, const double* r, double* z, int nrhs);
ert_status fftpc_info(ert_plan_impl* p, ert_fft_info* info);
void fftpc_destroy(FftPc* f);

// BLAS-1 helpers for GMRES (blas.hip); all stream-ordered on `s`.
// out[c] = <V[:,c], w> for c < ncols; V has leading dimension ldv.
ert_status dev_multidot(hipStream_t s, const double* V, long ldv, int ncols, const double* w, long N,
                        double* partial, double* out);
// w -= V[:, :ncols] * coef   (coef device vector)
ert_status dev_gemv_sub(hipStream_t s, const double* V, long ldv, int ncols, const double* coef,
                        double* w, long N);
// x += V[:, :ncols] * coef   (coef device vector)
ert_status dev_gemv_add(hipStream_t s, const double* V, long ldv, int ncols, const double* coef,
                        double* x, long N);
// y = alpha * x
ert_status dev_scale(hipStream_t s, double* y, const double* x, double alpha, long N);
// y = a - b
ert_status dev_sub(hipStream_t s, double* y, const double* a, const double* b, long N);
// y += x
ert_status dev_add(hipStream_t s, double* y, const double* x, long N);
// y = 0
ert_status dev_zero(hipStream_t s, double* y, long N);
// dst[i] += src[i] for a small vector of length n (device)
ert_status dev_small_add(hipStream_t s, double* dst, const double* src, int n);

// C = beta C + alpha A B (FP64, element strides); `work` (may be null) lets long
// reductions split over several workgroup slices.
ert_status dev_dgemm(hipStream_t s, int M, int N, long K, double alpha, const double* A, long sAi, long sAk,
                     const double* B, long sBk, long sBj, double beta, double* C, long sCi, long sCj, double* work,
                     size_t work_elems);

// Learned preconditioner (unet.hip): z = net(r) on the media st / ss (device FP64,
// one column), ordered on stream s.
struct NetImpl;
NetImpl* net_impl(ert_net_t net);
ert_status net_precond(NetImpl* n, const double* r, const double* st, const double* ss, double* z, hipStream_t s);
const int* net_grid(const NetImpl* n);

// Gauss-Legendre nodes/weights on [-1,1] (host).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

}  // namespace ertvie

struct ert_vie_plan_s : public ertvie::ert_plan_impl {};
