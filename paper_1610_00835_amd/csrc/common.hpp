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

// The same interpolant read from a table of corner octets: entry b holds the
// eight values st[b], st[b + d0], st[b + d1], st[b + d1 + d0], st[b + d2],
// st[b + d2 + d0], st[b + d2 + d1], st[b + d2 + d1 + d0] (64 bytes, aligned),
// so that a sample costs four 16-byte loads from one cache line instead of
// eight gathers over four lines.  The arithmetic is sigma_at's, term for term.
__device__ __forceinline__ double sigma_at8(const double* __restrict__ st8, const Geo& g, double inv_h, double p0,
                                            double p1, double p2)
{
    const int n[3] = {g.n0, g.n1, g.n2};
    const double p[3] = {p0, p1, p2};
    int i0[3] = {0, 0, 0};
    double t[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a < g.dim && n[a] > 1) {
            double u = p[a] * inv_h - 0.5;
            double hi = double(n[a] - 1);
            u = u < 0.0 ? 0.0 : (u > hi ? hi : u);
            int k = (int)floor(u);
            k = k > n[a] - 2 ? n[a] - 2 : k;
            i0[a] = k;
            t[a] = u - double(k);
        }
    }
    const long b0 = i0[0] + (long)n[0] * (i0[1] + (long)n[1] * i0[2]);
    const double2* q = reinterpret_cast<const double2*>(st8) + 4 * b0;
    const double2 v01 = q[0], v23 = q[1];
    double c00 = v01.x + t[0] * (v01.y - v01.x);
    double c10 = v23.x + t[0] * (v23.y - v23.x);
    double c0 = c00 + t[1] * (c10 - c00);
    if (g.dim == 2) return c0;
    const double2 v45 = q[2], v67 = q[3];
    double c01 = v45.x + t[0] * (v45.y - v45.x);
    double c11 = v67.x + t[0] * (v67.y - v67.x);
    double c1 = c01 + t[1] * (c11 - c01);
    return c0 + t[2] * (c1 - c0);
}

// Midpoint-rule optical depth from the corner-octet table (tau_march's rule and
// sum order, the same values bit for bit).  On a 3D grid with every side > 1
// the cell searches of U consecutive samples come first and their 4U loads are
// issued together, so the march does not wait one memory latency per sample;
// samples past m repeat the last one and are added with weight 0.  The clamp
// and floor are done in FP64 (max, min, floor: the same integers and
// fractions as sigma_at's compare-select form and integer minimum).
template <int U = 2>
__device__ __forceinline__ double tau_march8(const double* __restrict__ st8, const Geo& g, double inv_h, double a0,
                                             double a1, double a2, double b0, double b1, double b2, int m, double r)
{
    double e0 = b0 - a0, e1 = b1 - a1, e2 = b2 - a2;
    double inv_m = 1.0 / double(m);
    double s = 0.0;
    const long ncell = (long)g.n0 * g.n1 * g.n2;
    if (g.dim != 3 || g.n0 < 2 || g.n1 < 2 || g.n2 < 2 || ncell > (0x7fffffffL >> 6)) {
        for (int q = 1; q <= m; ++q) {
            double f = (double(q) - 0.5) * inv_m;
            s += sigma_at8(st8, g, inv_h, a0 + f * e0, a1 + f * e1, a2 + f * e2);
        }
        return r * inv_m * s;
    }
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)st8, 0, (int)(ncell << 6), 0x00020000);
    const double hi0 = double(g.n0 - 1), hi1 = double(g.n1 - 1), hi2 = double(g.n2 - 1);
    const double km0 = double(g.n0 - 2), km1 = double(g.n1 - 2), km2 = double(g.n2 - 2);
    const double nxd = double(g.n0), nyd = double(g.n1);
    const double last = double(m) - 0.5;
    double hq = 0.5;  // q0 - 0.5
    for (int q0 = 1; q0 <= m; q0 += U, hq += double(U)) {
        double t0[U], t1[U], t2[U];
        v4u raw[U][4];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const double hj = fmin(hq + double(j), last);
            const double f = hj * inv_m;
            const double u0 = fmin(fmax((a0 + f * e0) * inv_h - 0.5, 0.0), hi0);
            const double u1 = fmin(fmax((a1 + f * e1) * inv_h - 0.5, 0.0), hi1);
            const double u2 = fmin(fmax((a2 + f * e2) * inv_h - 0.5, 0.0), hi2);
            const double k0 = fmin(floor(u0), km0), k1 = fmin(floor(u1), km1), k2 = fmin(floor(u2), km2);
            t0[j] = u0 - k0;
            t1[j] = u1 - k1;
            t2[j] = u2 - k2;
            const unsigned c = (unsigned)fma(nxd, fma(nyd, k2, k1), k0);  // exact: integers below 2^25
#pragma unroll
            for (int w = 0; w < 4; ++w) raw[j][w] = __builtin_amdgcn_raw_buffer_load_b128(rs, (c << 6) + 16 * w, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);  // every load of the group issued before the first use
#pragma unroll
        for (int j = 0; j < U; ++j) {
            double v[8];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const double2 d = __builtin_bit_cast(double2, raw[j][w]);
                v[2 * w] = d.x;
                v[2 * w + 1] = d.y;
            }
            double c00 = v[0] + t0[j] * (v[1] - v[0]);
            double c10 = v[2] + t0[j] * (v[3] - v[2]);
            double c0 = c00 + t1[j] * (c10 - c00);
            double c01 = v[4] + t0[j] * (v[5] - v[4]);
            double c11 = v[6] + t0[j] * (v[7] - v[6]);
            double c1 = c01 + t1[j] * (c11 - c01);
            const double sv = c0 + t2[j] * (c1 - c0);
            s = fma(sv, q0 + j <= m ? 1.0 : 0.0, s);
        }
    }
    return r * inv_m * s;
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

// ------------------------------------------------- (M-ii) cell integrals ---

// Approach (M-ii) (Sec. 3.2, Remark 3.1) replaces h^d |x - y|^{1-d} by the
// integral of |z|^{1-d} over the source cell, centred at t = y - x.  For a
// cell of side h this is h * cell_int(t / h), cell_int being the integral over
// the unit cell:
//   2D: the closed form of Remark 3.1, sum over corners of +-F(r, s);
//   3D, |t|^2 >= 144: the Taylor expansion of the cell average of |z|^-2,
//       1/r^2 + 1/(12 r^4) + P4/(240 r^10) + P6/(20160 r^14) (relative error
//       below 2e-11, falling as r^-8);
//   3D, closer: the divergence theorem (div(z / |z|^2) = 1/|z|^2) turns the
//       cell integral into six face integrals of |z|^-2 times the face offset;
//       each is done in closed form along one face axis (arctangent) and by
//       12-point Gauss-Legendre panels growing by 3x away from the peak at the
//       foot of the perpendicular along the other.
__device__ __forceinline__ double mii_F(double r, double s)
{
    if (r == 0.0 || s == 0.0) return 0.0;
    const double ar = fabs(r), as = fabs(s), q = sqrt(r * r + s * s);
    const double v = ar * log(as + q) + as * log(ar + q) - ar * log(ar) - as * log(as);
    return ((r > 0.0) == (s > 0.0)) ? v : -v;
}

__device__ __forceinline__ double mii_face_piece(double c, double a, double b, double v0, double v1)
{
    // integral over u in [a, b] (0 <= a < b) of (atan(v1/q) - atan(v0/q)) / q, q = sqrt(c^2 + u^2)
    const double gx[6] = {0.12523340851146891, 0.36783149899818018, 0.58731795428661748, 0.76990267419430469,
                          0.9041172563704748, 0.98156063424671924};
    const double gw[6] = {0.24914704581340269, 0.23349253653835464, 0.20316742672306565, 0.16007832854334611,
                          0.10693932599531888, 0.047175336386512022};
    const double ac = fabs(c);
    double acc = 0.0;
    double lo = a;
    for (int pnl = 0; pnl < 40 && lo < b; ++pnl) {
        double hi = (lo < ac) ? ac : 3.0 * lo;
        if (hi > b) hi = b;
        const double m = 0.5 * (hi + lo), d = 0.5 * (hi - lo);
        for (int q = 0; q < 6; ++q)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                const double u = m + sgn * d * gx[q];
                const double qq = sqrt(c * c + u * u);
                acc += d * gw[q] * (atan(v1 / qq) - atan(v0 / qq)) / qq;
            }
        lo = hi;
    }
    return acc;
}

__device__ __forceinline__ double mii_face(double c, double u0, double u1, double v0, double v1)
{
    // the integrand is even in u: fold [u0, u1] onto u >= 0
    if (u0 >= 0.0) return mii_face_piece(c, u0, u1, v0, v1);
    if (u1 <= 0.0) return mii_face_piece(c, -u1, -u0, v0, v1);
    return mii_face_piece(c, 0.0, -u0, v0, v1) + mii_face_piece(c, 0.0, u1, v0, v1);
}

// far2: squared distance (in cells) from which the 3D expansion is used; the
// far-field interpolation nodes use 64 (relative error below 3e-10 there).
__device__ __forceinline__ double cell_int(int dim, double t0, double t1, double t2, double far2 = 144.0)
{
    if (dim == 2) {
        return mii_F(t0 + 0.5, t1 + 0.5) - mii_F(t0 + 0.5, t1 - 0.5) - mii_F(t0 - 0.5, t1 + 0.5) +
               mii_F(t0 - 0.5, t1 - 0.5);
    }
    const double x2 = t0 * t0, y2 = t1 * t1, z2 = t2 * t2, r2 = x2 + y2 + z2;
    if (r2 >= far2) {
        const double i2 = 1.0 / r2, i4 = i2 * i2, i8 = i4 * i4;
        const double p4 = -9.0 * (x2 * x2 + y2 * y2 + z2 * z2) + 46.0 * (x2 * y2 + x2 * z2 + y2 * z2);
        const double p6 = x2 * x2 * x2 + y2 * y2 * y2 + z2 * z2 * z2 -
                          317.0 * (x2 * x2 * (y2 + z2) + y2 * y2 * (x2 + z2) + z2 * z2 * (x2 + y2)) +
                          14406.0 * x2 * y2 * z2;
        return i2 + i4 / 12.0 + p4 * i8 * i2 / 240.0 + p6 * i8 * i4 * i2 / 20160.0;
    }
    const double t[3] = {t0, t1, t2};
    double acc = 0.0;
    for (int a = 0; a < 3; ++a) {
        const int b = (a + 1) % 3, c = (a + 2) % 3;
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            const double off = t[a] + 0.5 * sgn;
            if (off == 0.0) continue;
            acc += sgn * off * mii_face(off, t[b] - 0.5, t[b] + 0.5, t[c] - 0.5, t[c] + 0.5);
        }
    }
    return acc;
}

// --------------------------------------------------------------- the plan ---

struct FmmData;   // fmm.hip
struct HetCache;  // fmm.hip
struct FftPc;     // fftpc.hip
struct DiffPc;    // diffpc.hip

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
    int device = 0;              // the device current when the plan was made (its memory lives there)
    double sigma_const;          // homogeneous kernel: the constant sigma_t
    std::vector<double> h_st, h_ss;
    double* d_st = nullptr;      // sigma_t FP64
    float* d_st32 = nullptr;     // sigma_t FP32
    double* d_ss = nullptr;      // sigma_s FP64
    double* d_diag = nullptr;    // A_jj FP64
    double* d_itab = nullptr;    // (M-ii): cell_int at integer offsets |o| (n0 x n1 x n2, FP64), else null
    // GMRES workspace (grown on demand)
    double* d_ws = nullptr;
    size_t ws_elems = 0;
    double* d_red = nullptr;     // reduction partials / small vectors
    size_t red_elems = 0;
    // solve vectors beside the Krylov workspace (phi, residual, correction, trial
    // iterate and its residual), grown on demand and kept for the next solve
    double* d_solve = nullptr;
    size_t solve_elems = 0;
    FmmData* fmm[3] = {nullptr, nullptr, nullptr};   // per ert_prec
    HetCache* het[2] = {nullptr, nullptr};   // heterogeneous kernel caches (per Chebyshev order)
    FftPc* fftpc = nullptr;      // FFT-based preconditioner (built on first use)
    DiffPc* diffpc = nullptr;    // diffusion preconditioner (built on first use)
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
// Build the FMM data of precision `prec` if not built yet (tree, operators, caches).
ert_status fmm_build(ert_plan_impl* p, int prec);
void fmm_destroy(FmmData* f);
void het_destroy(HetCache* c);
// FFT-based preconditioner of the mean medium (fftpc.hip): z = M r for nrhs
// columns (device FP64), stream-ordered; builds the symbol on first use.
ert_status fftpc_apply(ert_plan_impl* p, const double* r, double* z, int nrhs);
// Diffusion preconditioner (diffpc.hip): z = r + (two V-cycles for L e = sigma_s r).
ert_status diffpc_apply(ert_plan_impl* p, const double* r, double* z, int nrhs);
void diffpc_destroy(DiffPc* d);
// Right preconditioner by kind (ERT_PRECOND_FFT or ERT_PRECOND_DIFFUSION), nrhs columns.
inline ert_status precond_apply(ert_plan_impl* p, int kind, const double* r, double* z, int nrhs)
{
    return kind == ERT_PRECOND_DIFFUSION ? diffpc_apply(p, r, z, nrhs) : fftpc_apply(p, r, z, nrhs);
}
// Algorithm 1 S.3 (transport.hip): phi[:, d] = the angular solution for direction d.
ert_status transport_sweep(ert_plan_impl* p, const double* U, const double* f, const double* dirs_host, int ndir,
                           double* phi);
// The same with the device scratch of the library instead of an allocation.
ert_status transport_sweep_noalloc(ert_plan_impl* p, const double* U, const double* f, const double* dirs_host,
                                   int ndir, double* phi);
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
// pn: the plan's grid, the network's grid times f >= 1 on every axis (f > 1: the network acts
// on cell averages over f^3 blocks and its output is extended piecewise constant).
ert_status net_precond(NetImpl* n, const double* r, const double* st, const double* ss, double* z, hipStream_t s,
                       const int* pn);
// y = cell averages of x over f^3 blocks of the grid n (nrhs columns; unet.hip).
ert_status restrict_avg(hipStream_t s, const double* x, const int n[3], int f, double* y, int nrhs);
const int* net_grid(const NetImpl* n);

// Gauss-Legendre nodes/weights on [-1,1] (host).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

}  // namespace ertvie

struct ert_vie_plan_s : public ertvie::ert_plan_impl {};
