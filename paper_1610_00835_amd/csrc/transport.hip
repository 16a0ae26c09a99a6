// Algorithm 1 step S.3: the angular solution Phi(x, v) from U by the
// scattering-free transport equation v . grad Phi + sigma_t Phi = Q,
// Q = sigma_s U + f, with no inflow, solved along characteristics: from each
// cell centre the ray is followed backwards to the boundary of the box
// [0, n_a h]^d in m = ceil(s_b / (h/2)) equal steps (with a 1e-12 relative margin); on each step sigma_t and Q
// take their (clamped d-linear) values at the step midpoint and the step is
// integrated exactly for those constants (step characteristics), so a constant
// medium and source give Q (1 - exp(-sigma_t s_b)) / sigma_t exactly.
//
// One thread per (cell, direction), FP64; the medium and the source are read
// through the d-linear interpolation the kernel's ray rule uses (L2-resident
// gathers of the two fields interleaved per cell).  exp(-tau) is carried as a
// running product of the steps' factors.
#include "common.hpp"

#include <cmath>
#include <mutex>

namespace ertvie {

// Device scratch of the allocation-free entry point (ert_vie_transport_noalloc):
// the interleaved (sigma_t, Q) pairs, 2 N doubles, then the directions, dim * ndir
// doubles.  32.5 MiB per device, held from the library's first use of it on that
// device until the process ends.  Host code never passes this name to a kernel
// or a copy: it uses the device address from hipGetSymbolAddress (scratch_base).
constexpr size_t kTransportScratch = (size_t(1) << 22) + (size_t(1) << 16);   // doubles
static __device__ __align__(256) double scratch[kTransportScratch];

namespace {

// (sigma_t, Q) per cell, interleaved so that one 16-byte load serves both fields
__global__ __launch_bounds__(256) void k_source(const double* __restrict__ U, const double* __restrict__ f,
                                                const double* __restrict__ st, const double* __restrict__ ss, long N,
                                                double2* __restrict__ sq)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    sq[i] = make_double2(st[i], (U ? ss[i] * U[i] : 0.0) + (f ? f[i] : 0.0));
}

// The clamped d-linear interpolation of the ray rule (as for sigma_t alone), applied to
// both interleaved fields with one set of weights: the same operations per field.
__device__ __forceinline__ double2 pair_at(const double2* __restrict__ v, const Geo& g, double inv_h, double p0,
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
            const double hi = (double)(n[a] - 1);
            u = u < 0.0 ? 0.0 : (u > hi ? hi : u);
            int k = (int)floor(u);
            k = k > n[a] - 2 ? n[a] - 2 : k;
            i0[a] = k;
            t[a] = u - (double)k;
        }
    }
    const int b0 = i0[0] + n[0] * (i0[1] + n[1] * i0[2]);
    const int d0 = n[0] > 1 ? 1 : 0;
    const int d1 = n[1] > 1 ? n[0] : 0;
    const int d2 = (g.dim > 2 && n[2] > 1) ? n[0] * n[1] : 0;
    auto lerp2 = [&](int b) {
        const double2 a = v[b], c = v[b + d0];
        return make_double2(a.x + t[0] * (c.x - a.x), a.y + t[0] * (c.y - a.y));
    };
    const double2 c00 = lerp2(b0), c10 = lerp2(b0 + d1);
    const double2 c0 = make_double2(c00.x + t[1] * (c10.x - c00.x), c00.y + t[1] * (c10.y - c00.y));
    if (g.dim == 2) return c0;
    const double2 c01 = lerp2(b0 + d2), c11 = lerp2(b0 + d2 + d1);
    const double2 c1 = make_double2(c01.x + t[1] * (c11.x - c01.x), c01.y + t[1] * (c11.y - c01.y));
    return make_double2(c0.x + t[2] * (c1.x - c0.x), c0.y + t[2] * (c1.y - c0.y));
}

__global__ __launch_bounds__(256) void k_sweep(Geo g, const double2* __restrict__ sq,
                                               const double* __restrict__ dirs, long N, double* __restrict__ phi)
{
    const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int d = blockIdx.y;
    const double h = g.h, inv_h = 1.0 / g.h;
    const int i0 = (int)(j % g.n0), i1 = (int)((j / g.n0) % g.n1), i2 = (int)(j / ((long)g.n0 * g.n1));
    const double x[3] = {h * (i0 + 0.5), h * (i1 + 0.5), g.dim > 2 ? h * (i2 + 0.5) : 0.0};
    const double v[3] = {dirs[g.dim * d], dirs[g.dim * d + 1], g.dim > 2 ? dirs[g.dim * d + 2] : 0.0};
    const int n[3] = {g.n0, g.n1, g.n2};
    // distance backwards along -v to the box boundary
    double sb = 1e300;
    for (int a = 0; a < g.dim; ++a) {
        if (v[a] > 0.0) sb = fmin(sb, x[a] / v[a]);
        else if (v[a] < 0.0) sb = fmin(sb, (n[a] * h - x[a]) / (-v[a]));
    }
    // the relative margin keeps the count of an exact multiple of h/2 (every
    // axis-parallel ray) independent of the last bit of sb
    const double q0 = ceil(sb / (0.5 * h) * (1.0 - 1e-12));
    const long m = q0 < 1.0 ? 1 : (long)q0;
    const double D = sb / (double)m;
    double acc = 0.0, att = 1.0;     // att = exp(-tau) before the step
    for (long k = 1; k <= m; ++k) {
        const double t = ((double)k - 0.5) * D;
        const double p0 = x[0] - t * v[0], p1 = x[1] - t * v[1], p2 = x[2] - t * v[2];
        const double2 sqk = pair_at(sq, g, inv_h, p0, p1, p2);
        const double s = sqk.x, qk = sqk.y;
        const double sd = s * D;
        const double em = expm1(-sd);                 // exp(-sigma D) - 1
        const double step = sd > 1e-300 ? -em / s : D;
        acc += att * qk * step;
        att *= 1.0 + em;
    }
    phi[(long)d * N + j] = acc;
}

// Directions (host, ndir x dim): finite unit vectors.
ert_status check_dirs(int dim, const double* dirs_host, int ndir)
{
    for (int d = 0; d < ndir; ++d) {
        double nn = 0.0;
        for (int a = 0; a < dim; ++a) {
            const double c = dirs_host[(size_t)d * dim + a];
            if (!std::isfinite(c)) {
                record_error("ert_vie_transport: non-finite direction");
                return ERT_EINVAL;
            }
            nn += c * c;
        }
        if (std::fabs(nn - 1.0) > 1e-10) {
            record_error("ert_vie_transport: directions must be unit vectors");
            return ERT_EINVAL;
        }
    }
    return ERT_OK;
}

// The sweep with caller-provided device buffers: sq (N pairs) and dd (dim * ndir),
// which receives the directions.  Synchronises the plan's stream before returning
// (the directions are copied from the caller's host array).
ert_status sweep_into(ert_plan_impl* p, const double* U, const double* f, const double* dirs_host, int ndir,
                      double* phi, double2* sq, double* dd)
{
    const long N = p->N;
    const int dim = p->o.dim;
    ert_status st = ERT_HIPST(hipMemcpyAsync(dd, dirs_host, sizeof(double) * dim * (size_t)ndir,
                                             hipMemcpyHostToDevice, p->stream));
    if (st == ERT_OK) {
        hipLaunchKernelGGL(k_source, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, p->stream, U, f, p->d_st,
                           p->d_ss, N, sq);
        st = ERT_HIPST(hipGetLastError());
    }
    // directions in slabs of at most 65535 (grid.y)
    for (int d0 = 0; d0 < ndir && st == ERT_OK; d0 += 65535) {
        const int nd = std::min(65535, ndir - d0);
        hipLaunchKernelGGL(k_sweep, dim3((unsigned)((N + 255) / 256), (unsigned)nd), dim3(256), 0, p->stream, p->geo,
                           sq, dd + (size_t)dim * d0, N, phi + (size_t)d0 * N);
        st = ERT_HIPST(hipGetLastError());
    }
    const ert_status ss = ERT_HIPST(hipStreamSynchronize(p->stream));
    return st != ERT_OK ? st : ss;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (made current by the caller), looked
// up once per device.
ert_status scratch_base(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        record_error("ert_vie_transport_noalloc: device index out of range");
        return ERT_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            record_hip_error("hipGetSymbolAddress(scratch)", e != hipSuccess ? e : hipErrorInvalidSymbol, __FILE__,
                             __LINE__);
            return ERT_EDEVICE;
        }
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return ERT_OK;
}

}  // namespace

ert_status transport_sweep(ert_plan_impl* p, const double* U, const double* f, const double* dirs_host, int ndir,
                           double* phi)
{
    ERT_TRY(check_dirs(p->o.dim, dirs_host, ndir));
    const long N = p->N;
    double* buf = nullptr;
    ERT_HIP(hipMalloc(&buf, sizeof(double) * (2 * N + (size_t)p->o.dim * ndir)));
    const ert_status st = sweep_into(p, U, f, dirs_host, ndir, phi, reinterpret_cast<double2*>(buf), buf + 2 * N);
    (void)hipFree(buf);
    return st;
}

ert_status transport_sweep_noalloc(ert_plan_impl* p, const double* U, const double* f, const double* dirs_host,
                                   int ndir, double* phi)
{
    ERT_TRY(check_dirs(p->o.dim, dirs_host, ndir));
    const size_t need = 2 * (size_t)p->N + (size_t)p->o.dim * ndir;
    if (need > kTransportScratch) {
        record_error("ert_vie_transport_noalloc: 2 N + dim * ndir exceeds the scratch of 4259840 doubles");
        return ERT_EINVAL;
    }
    int cur = 0;
    ERT_HIP(hipGetDevice(&cur));
    if (cur != p->device) ERT_HIP(hipSetDevice(p->device));
    double* base = nullptr;
    ert_status st = scratch_base(p->device, &base);
    if (st == ERT_OK)
        st = sweep_into(p, U, f, dirs_host, ndir, phi, reinterpret_cast<double2*>(base), base + 2 * p->N);
    if (cur != p->device) {
        const hipError_t e = hipSetDevice(cur);
        if (st == ERT_OK && e != hipSuccess) {
            record_hip_error("hipSetDevice", e, __FILE__, __LINE__);
            st = ERT_EDEVICE;
        }
    }
    return st;
}

}  // namespace ertvie
