// C ABI of the library (include/ertvie.h): plan construction and validation,
// operator dispatch, and the Krylov solvers of Algorithm 1 step S.2 driven
// from the host with FP64 device vectors.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"

namespace ertvie {

namespace {
thread_local std::string g_last_error;
}

void record_hip_error(const char* what, hipError_t e, const char* file, int line)
{
    g_last_error = std::string(what) + " failed: " + hipGetErrorString(e) + " (" + file + ":" +
                   std::to_string(line) + ")";
}

void record_error(const char* msg) { g_last_error = msg; }

// Gauss-Legendre rule on [-1,1]: Newton iteration on P_n from Chebyshev-like
// initial guesses, weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double pn = 0.0, dpn = 1.0;
        for (int it = 0; it < 200; ++it) {
            double pm1 = 1.0, p = z;
            for (int k = 1; k < n; ++k) {
                double pk1 = ((2 * k + 1) * z * p - k * pm1) / (k + 1);
                pm1 = p;
                p = pk1;
            }
            pn = p;
            dpn = n * (z * p - pm1) / (z * z - 1.0);
            double dz = pn / dpn;
            z -= dz;
            if (std::fabs(dz) <= 1e-16 * std::fabs(z) + 1e-300) break;
        }
        {
            double pm1 = 1.0, p = z;
            for (int k = 1; k < n; ++k) {
                double pk1 = ((2 * k + 1) * z * p - k * pm1) / (k + 1);
                pm1 = p;
                p = pk1;
            }
            dpn = n * (z * p - pm1) / (z * z - 1.0);
        }
        double wi = 2.0 / ((1.0 - z * z) * dpn * dpn);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = wi;
        w[n - 1 - i] = wi;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

hipEvent_t Profiler::get()
{
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ert_status Profiler::begin(hipStream_t s, int stage, hipEvent_t* ev)
{
    (void)stage;
    *ev = get();
    if (!*ev) return ERT_EDEVICE;
    ERT_HIP(hipEventRecord(*ev, s));
    return ERT_OK;
}

ert_status Profiler::end(hipStream_t s, int stage, hipEvent_t ev0)
{
    hipEvent_t e1 = get();
    if (!e1) return ERT_EDEVICE;
    ERT_HIP(hipEventRecord(e1, s));
    recs.push_back({stage, ev0, e1});
    return ERT_OK;
}

ert_status Profiler::resolve()
{
    for (auto& r : recs) {
        ERT_HIP(hipEventSynchronize(r.b));
        float t = 0.f;
        ERT_HIP(hipEventElapsedTime(&t, r.a, r.b));
        ms[r.stage] += t;
        launches[r.stage] += 1;
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    recs.clear();
    return ERT_OK;
}

void Profiler::clear()
{
    (void)resolve();
    for (int i = 0; i < ERT_NSTAGES; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
}

Profiler::~Profiler()
{
    for (auto& r : recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
}

ert_status plan_apply(ert_plan_impl* p, int op, int method, int prec, const double* x, double* y, int nrhs)
{
    if (method == ERT_DIRECT) {
        StageTimer t(&p->prof, p->stream, ERT_STAGE_DIRECT);
        return direct_apply(p, op, prec, x, y, nrhs);
    }
    return fmm_apply(p, op, prec, x, y, nrhs);
}

ert_status block_gmres(ert_plan_impl* pl, int method, int prec, const double* Phi, double* X, int nb, double rtol,
                       int maxit, int restart, bool check_true, int* iters_out, int* cycles_out, int* matvecs_out,
                       double* est_out, double* true_out, bool* conv_out, int pk, bool* breakdown_out);

namespace {

ert_status apply_dispatch(ert_plan_impl* p, int op, int method, int prec, const double* x, double* y, int nrhs)
{
    return plan_apply(p, op, method, prec, x, y, nrhs);
}

ert_status ensure_workspace(ert_plan_impl* p, size_t vec_elems, size_t red_elems)
{
    if (vec_elems > p->ws_elems) {
        if (p->d_ws) (void)hipFree(p->d_ws);
        p->d_ws = nullptr;
        p->ws_elems = 0;
        if (hipMalloc(&p->d_ws, vec_elems * sizeof(double)) != hipSuccess) return ERT_ENOMEM;
        p->ws_elems = vec_elems;
    }
    if (red_elems > p->red_elems) {
        if (p->d_red) (void)hipFree(p->d_red);
        p->d_red = nullptr;
        p->red_elems = 0;
        if (hipMalloc(&p->d_red, red_elems * sizeof(double)) != hipSuccess) return ERT_ENOMEM;
        p->red_elems = red_elems;
    }
    return ERT_OK;
}

ert_status ensure_solve_scratch(ert_plan_impl* p, size_t elems)
{
    if (elems <= p->solve_elems) return ERT_OK;
    if (p->d_solve) (void)hipFree(p->d_solve);
    p->d_solve = nullptr;
    p->solve_elems = 0;
    if (hipMalloc(&p->d_solve, elems * sizeof(double)) != hipSuccess) {
        record_error("ert_vie_solve: device allocation of the solve vectors failed");
        return ERT_ENOMEM;
    }
    p->solve_elems = elems;
    return ERT_OK;
}

constexpr int kPartials = 240;   // matches the reduction block count of blas.hip (upper bound)

double dev_norm(ert_plan_impl* p, const double* v, double* partial, double* out_dev, ert_status* st)
{
    *st = dev_multidot(p->stream, v, p->N, 1, v, p->N, partial, out_dev);
    if (*st != ERT_OK) return 0.0;
    double h = 0.0;
    if (hipMemcpyAsync(&h, out_dev, sizeof(double), hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
        hipStreamSynchronize(p->stream) != hipSuccess) {
        *st = ERT_EDEVICE;
        return 0.0;
    }
    return std::sqrt(h);
}

// Iterate/residual pairs recorded at the start of every GMRES cycle.
struct History {
    double* buf = nullptr;   // N x 2 cap
    int cap = 0;
    int count = 0;
};

// Right preconditioner of a GMRES run: a fixed one (kind: FFT-based of the mean
// medium, or diffusion), the network, or the network acting on the fixed one's output.
struct Precond {
    NetImpl* net = nullptr;
    int kind = ERT_PRECOND_NONE;
    bool active() const { return net != nullptr || kind != ERT_PRECOND_NONE; }
};

struct RunStats {
    int iters = 0, matvecs = 0, cycles = 0, precond = 0;
    double est = 0.0, true_rel = -1.0;
    bool converged = false;
};

// GMRES (x0 = 0) for (I - K) u = b with the operator (method, prec).  Arnoldi by
// classical Gram-Schmidt with one re-orthogonalisation on the device, Givens
// rotations and the small triangular solve on the host.  Stops when the
// recurrence estimate reaches rtol ||b||; with check_true it then confirms the
// true residual with the same operator and restarts from u if needed.
// With a preconditioner: flexible GMRES with right preconditioning (Saad 1993),
// the operator applied to z_j = M(v_j) and the update built from the z_j.
ert_status gmres_run(ert_plan_impl* p, int method, int prec, const double* b, double* u, double rtol, int maxit,
                     int restart, bool check_true, RunStats* rs, const Precond* pc = nullptr, History* hist = nullptr)
{
    const long N = p->N;
    const int m = (restart > 0 && restart < maxit) ? restart : maxit;
    const bool flex = pc && pc->active();
    const int nz = flex ? m : 0;
    // workspace: V (m+1 vectors), Z (m, flexible only), w, r
    ERT_TRY(ensure_workspace(p, (size_t)(m + nz + 3) * N, (size_t)kPartials * (m + 2) + 4 * (size_t)(m + 2)));
    double* V = p->d_ws;
    double* Z = V + (size_t)(m + 1) * N;
    double* w = Z + (size_t)nz * N;
    double* r = w + N;
    double* partial = p->d_red;
    double* dh = partial + (size_t)kPartials * (m + 2);    // h1 (m+1) then h2 (m+1) then norm
    double* dh2 = dh + (m + 2);
    double* dy = dh2 + (m + 2);
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), hh(m + 2);
    ert_status st = ERT_OK;

    ERT_TRY(dev_zero(p->stream, u, N));
    double bnorm = dev_norm(p, b, partial, dh, &st);
    ERT_TRY(st);
    if (bnorm == 0.0) {
        rs->converged = true;
        rs->true_rel = 0.0;
        return ERT_OK;
    }
    double beta = bnorm;
    const double* rsrc = b;
    for (int cycle = 0; rs->iters < maxit; ++cycle) {
        rs->cycles = cycle + 1;
        if (hist && hist->count < hist->cap) {
            double* hb = hist->buf + (size_t)2 * hist->count * N;
            ERT_HIP(hipMemcpyAsync(hb, u, N * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
            ERT_HIP(hipMemcpyAsync(hb + N, rsrc, N * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
            hist->count++;
        }
        ERT_TRY(dev_scale(p->stream, V, rsrc, 1.0 / beta, N));
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        bool done = false;
        for (int j = 0; j < m && rs->iters < maxit; ++j) {
            double* vj = V + (size_t)j * N;
            if (flex) {
                double* zj = Z + (size_t)j * N;
                if (pc->kind && pc->net) {
                    ERT_TRY(precond_apply(p, pc->kind, vj, w, 1));
                    ERT_TRY(net_precond(pc->net, w, p->d_st, p->d_ss, zj, p->stream, p->o.n));
                } else if (pc->kind) {
                    ERT_TRY(precond_apply(p, pc->kind, vj, zj, 1));
                } else {
                    ERT_TRY(net_precond(pc->net, vj, p->d_st, p->d_ss, zj, p->stream, p->o.n));
                }
                if (pc->net) rs->precond++;
                vj = zj;
            }
            ERT_TRY(apply_dispatch(p, ERT_OP_A, method, prec, vj, w, 1));
            rs->matvecs++;
            ERT_TRY(dev_multidot(p->stream, V, N, j + 1, w, N, partial, dh));
            ERT_TRY(dev_gemv_sub(p->stream, V, N, j + 1, dh, w, N));
            ERT_TRY(dev_multidot(p->stream, V, N, j + 1, w, N, partial, dh2));
            ERT_TRY(dev_gemv_sub(p->stream, V, N, j + 1, dh2, w, N));
            ERT_TRY(dev_small_add(p->stream, dh, dh2, j + 1));
            ERT_TRY(dev_multidot(p->stream, w, N, 1, w, N, partial, dh + j + 1));
            ERT_HIP(hipMemcpyAsync(hh.data(), dh, sizeof(double) * (j + 2), hipMemcpyDeviceToHost, p->stream));
            ERT_HIP(hipStreamSynchronize(p->stream));
            const double hn = std::sqrt(hh[j + 1] > 0.0 ? hh[j + 1] : 0.0);
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh[i];
            for (int i = 0; i < j; ++i) {
                double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[(size_t)j * m + j];
            double den = std::hypot(a, hn);
            cs[j] = den == 0.0 ? 1.0 : a / den;
            sn[j] = den == 0.0 ? 0.0 : hn / den;
            H[(size_t)j * m + j] = den;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            rs->iters++;
            k = j + 1;
            rs->est = std::fabs(g[j + 1]) / bnorm;
            if (rs->est <= rtol || hn == 0.0) { done = true; break; }
            ERT_TRY(dev_scale(p->stream, V + (size_t)(j + 1) * N, w, 1.0 / hn, N));
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int c = i + 1; c < k; ++c) s -= H[(size_t)i * m + c] * y[c];
            // a zero pivot only arises from a zero search direction (breakdown of a
            // flexible step): that direction takes no weight
            y[i] = H[(size_t)i * m + i] != 0.0 ? s / H[(size_t)i * m + i] : 0.0;
        }
        ERT_HIP(hipMemcpyAsync(dy, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, p->stream));
        ERT_TRY(dev_gemv_add(p->stream, flex ? Z : V, N, k, dy, u, N));
        if (!check_true) {
            if (done) rs->converged = true;
            if (done) break;
            // restart from the recurrence residual direction: recompute r with the operator
        }
        ERT_TRY(apply_dispatch(p, ERT_OP_A, method, prec, u, w, 1));
        rs->matvecs++;
        ERT_TRY(dev_sub(p->stream, r, b, w, N));
        beta = dev_norm(p, r, partial, dh, &st);
        ERT_TRY(st);
        rs->true_rel = beta / bnorm;
        if (rs->true_rel <= rtol) { rs->converged = true; break; }
        if (beta == 0.0) { rs->converged = true; break; }
        rsrc = r;
    }
    ERT_HIP(hipStreamSynchronize(p->stream));
    return ERT_OK;
}

// Refinement with the learned preconditioner and its residual check: each
// step computes a correction d by flexible GMRES (at most precond_steps Arnoldi
// steps, stopping at inner_tol) on the inner operator, and keeps U + d only if
// the true residual phi - (I - K)(U + d) decreases, with the residual taken
// with the FP64 operator whatever the inner precision; a rejected step is
// redone without the network (plain GMRES, or with the fixed preconditioner
// `kind` alone) with the same budget, and when that step does not lower the
// residual either the refinement stops (ERT_ENOCONV from the caller).
// r, d: caller scratch (N each); trial: caller scratch (2 N).
ert_status learned_refine(ert_plan_impl* p, int method, int prec_inner, NetImpl* net, int kind, const double* phi,
                          double* U, double* r, double* d, double* trial, const ert_solve_opts& so,
                          ert_solve_info* inf)
{
    const long N = p->N;
    const int prec_outer = ERT_FP64;
    const int steps = so.precond_steps > 0 ? so.precond_steps : 10;
    ERT_TRY(dev_zero(p->stream, U, N));
    ERT_HIP(hipMemcpyAsync(r, phi, N * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
    double* rt = trial + N;
    ert_status st = ERT_OK;
    auto norm = [&](const double* v) {
        ert_status s2 = ensure_workspace(p, 3 * N, (size_t)kPartials * 4 + 16);
        if (s2 != ERT_OK) { st = s2; return 0.0; }
        return dev_norm(p, v, p->d_red, p->d_red + (size_t)kPartials * 4, &st);
    };
    const double pnorm = norm(phi);
    double rnorm = pnorm;
    int used = 0;
    bool stalled = false;
    for (int outer = 0; outer < 1000 && st == ERT_OK && !stalled; ++outer) {
        inf->rel_resid_true = pnorm > 0 ? rnorm / pnorm : 0.0;
        if (rnorm <= so.tol * pnorm) { inf->converged = 1; break; }
        if (used >= so.max_iter) break;
        const int budget = std::min(steps, so.max_iter - used);
        bool accepted = false;
        for (int attempt = 0; attempt < 2 && !accepted && st == ERT_OK; ++attempt) {
            RunStats rs;
            Precond pc;
            pc.net = attempt == 0 ? net : nullptr;
            pc.kind = kind;
            st = gmres_run(p, method, prec_inner, r, d, so.inner_tol, budget, budget, false, &rs, &pc);
            if (st != ERT_OK) break;
            used += rs.iters;
            inf->iters += rs.iters;
            inf->matvecs += rs.matvecs;
            inf->precond_applies += rs.precond;
            inf->rel_resid_est = rs.est;
            st = ERT_HIPST(hipMemcpyAsync(trial, U, N * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
            if (st == ERT_OK) st = dev_add(p->stream, trial, d, N);
            if (st == ERT_OK) st = apply_dispatch(p, ERT_OP_A, method, prec_outer, trial, rt, 1);
            if (st != ERT_OK) break;
            inf->matvecs++;
            st = dev_sub(p->stream, rt, phi, rt, N);
            if (st != ERT_OK) break;
            const double tn = norm(rt);
            if (st != ERT_OK) break;
            // the check: keep the step only if the true residual went down
            if (tn < rnorm) {
                accepted = true;
                st = ERT_HIPST(hipMemcpyAsync(U, trial, N * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
                if (st == ERT_OK)
                    st = ERT_HIPST(hipMemcpyAsync(r, rt, N * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
                rnorm = tn;
            } else if (attempt == 0 && net) {
                inf->rejected++;
            } else {
                stalled = true;   // the step without the network made no progress either
            }
        }
        inf->restarts = outer + 1;
    }
    if (st == ERT_OK) {
        inf->rel_resid_true = pnorm > 0 ? rnorm / pnorm : 0.0;
        if (rnorm <= so.tol * pnorm) inf->converged = 1;
    }
    (void)hipStreamSynchronize(p->stream);
    return st;
}

// Column-by-column completion of a block solve after a block breakdown (a zero,
// repeated or already solved column leaves the residual block without an
// orthonormal basis): with R = Phi - (I - K) X, every column whose residual
// exceeds tol ||Phi_b|| is finished by GMRES on (I - K) d = R_b with the same
// operator and fixed right preconditioner, X_b += d.  R and d are scratch
// (N nrhs and N).  Fills iters, matvecs, rel_resid_true (worst column) and
// converged of inf.
ert_status finish_columns(ert_plan_impl* p, int method, int prec, const double* Phi, double* X, double* R, double* d,
                          int nrhs, const ert_solve_opts& so, int kind, ert_solve_info* inf)
{
    const long N = p->N;
    ERT_TRY(apply_dispatch(p, ERT_OP_A, method, prec, X, R, nrhs));
    inf->matvecs++;
    ERT_TRY(dev_sub(p->stream, R, Phi, R, N * nrhs));
    ert_status st = ERT_OK;
    auto norm = [&](const double* v) {
        ert_status s2 = ensure_workspace(p, 3 * N, (size_t)kPartials * 4 + 16);
        if (s2 != ERT_OK) { st = s2; return 0.0; }
        return dev_norm(p, v, p->d_red, p->d_red + (size_t)kPartials * 4, &st);
    };
    Precond pc;
    pc.kind = kind;
    double worst = 0.0;
    for (int b = 0; b < nrhs; ++b) {
        const double pn = norm(Phi + (size_t)b * N);
        const double rn = norm(R + (size_t)b * N);
        ERT_TRY(st);
        if (rn <= so.tol * pn) {
            worst = std::max(worst, pn > 0.0 ? rn / pn : 0.0);
            continue;
        }
        RunStats rs;
        const int budget = std::max(1, so.max_iter - inf->iters);
        ERT_TRY(gmres_run(p, method, prec, R + (size_t)b * N, d, std::min(0.5, so.tol * pn / rn), budget, so.restart,
                          true, &rs, &pc));
        inf->iters += rs.iters;
        inf->matvecs += rs.matvecs;
        ERT_TRY(dev_add(p->stream, X + (size_t)b * N, d, N));
        worst = std::max(worst, rs.true_rel * rn / pn);
    }
    inf->rel_resid_true = worst;
    inf->converged = worst <= so.tol ? 1 : 0;
    return ERT_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace
}  // namespace ertvie

using namespace ertvie;

extern "C" {

const char* ert_vie_last_error(void) { return g_last_error.c_str(); }

const char* ert_vie_strerror(ert_status s)
{
    switch (s) {
    case ERT_OK: return "ok";
    case ERT_EINVAL: return "invalid argument";
    case ERT_ENOMEM: return "out of memory";
    case ERT_EDEVICE: return "HIP device error";
    case ERT_ENOCONV: return "solver did not converge within max_iter";
    case ERT_EUNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

long ert_vie_size(ert_vie_plan_t plan) { return plan ? plan->N : -1; }

void ert_vie_destroy(ert_vie_plan_t p)
{
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    for (auto& f : p->fmm) {
        if (f) fmm_destroy(f);
        f = nullptr;
    }
    for (auto& c : p->het) {
        het_destroy(c);
        c = nullptr;
    }
    fftpc_destroy(p->fftpc);
    p->fftpc = nullptr;
    diffpc_destroy(p->diffpc);
    p->diffpc = nullptr;
    (void)hipFree(p->d_st);
    (void)hipFree(p->d_st32);
    (void)hipFree(p->d_ss);
    (void)hipFree(p->d_diag);
    (void)hipFree(p->d_itab);
    (void)hipFree(p->d_ws);
    (void)hipFree(p->d_red);
    (void)hipFree(p->d_solve);
    delete p;
}

ert_status ert_vie_plan(const ert_vie_opts* opts, const double* sigma_t, const double* sigma_s, void* hip_stream,
                        ert_vie_plan_t* out)
{
    record_error("ert_vie_plan: invalid argument");
    if (!opts || !sigma_t || !sigma_s || !out) return ERT_EINVAL;
    const ert_vie_opts& o = *opts;
    if (o.dim != 2 && o.dim != 3) return ERT_EINVAL;
    if (!finite_pos(o.h) || (o.scheme != 0 && o.scheme != 1)) return ERT_EINVAL;
    if (o.kernel != ERT_K_HOMOGENEOUS && o.kernel != ERT_K_RAY_MIDPOINT) return ERT_EINVAL;
    if (o.method != ERT_DIRECT && o.method != ERT_FMM) return ERT_EINVAL;
    if (o.prec != ERT_FP64 && o.prec != ERT_FP32 && o.prec != ERT_BF16X3) return ERT_EINVAL;
    if (o.cheb_n != 0 && (o.cheb_n < 2 || o.cheb_n > 8)) return ERT_EINVAL;
    if (o.leaf < 0 || o.leaf > 8 || o.nrhs_max < 0 || !std::isfinite(o.svd_tol) || o.svd_tol >= 1.0)
        return ERT_EINVAL;
    if ((o.inner_cheb_n != 0 && (o.inner_cheb_n < 2 || o.inner_cheb_n > 8)) || (o.inner_near16 != 0 && o.inner_near16 != 1)) return ERT_EINVAL;
    for (int i = 0; i < 2; ++i)
        if (o.form[i] < 0 || o.form[i] > 6) return ERT_EINVAL;   // execution forms 0..5, stored as f + 1
    if (!std::isfinite(o.far_cache_gb) || o.far_cache_gb < 0.0) return ERT_EINVAL;
    long N = 1;
    for (int a = 0; a < o.dim; ++a) {
        if (o.n[a] < 1 || o.n[a] > (1 << 20)) return ERT_EINVAL;
        N *= o.n[a];
        if (N > (1L << 30)) return ERT_EINVAL;
    }
    if (N < 2) return ERT_EINVAL;
    record_error("ert_vie_plan: invalid coefficients (need finite sigma_t > 0, 0 <= sigma_s <= sigma_t, "
                 "constant sigma_t for the homogeneous kernel)");
    for (long j = 0; j < N; ++j) {
        const double t = sigma_t[j], s = sigma_s[j];
        if (!finite_pos(t) || !std::isfinite(s) || s < 0.0 || s > t * (1.0 + 1e-12)) return ERT_EINVAL;
        if (o.kernel == ERT_K_HOMOGENEOUS && t != sigma_t[0]) return ERT_EINVAL;
    }
    int ndev = 0;
    hipError_t de = hipGetDeviceCount(&ndev);
    if (de != hipSuccess || ndev < 1) {
        record_hip_error("hipGetDeviceCount", de != hipSuccess ? de : hipErrorNoDevice, __FILE__, __LINE__);
        return ERT_EDEVICE;
    }

    int dev = 0;
    de = hipGetDevice(&dev);
    if (de != hipSuccess) {
        record_hip_error("hipGetDevice", de, __FILE__, __LINE__);
        return ERT_EDEVICE;
    }
    record_error("");
    ert_vie_plan_s* p = new (std::nothrow) ert_vie_plan_s();
    if (!p) return ERT_ENOMEM;
    p->o = o;
    p->device = dev;
    if (p->o.dim == 2) p->o.n[2] = 1;
    p->geo.dim = o.dim;
    p->geo.n0 = o.n[0];
    p->geo.n1 = o.n[1];
    p->geo.n2 = o.dim > 2 ? o.n[2] : 1;
    p->geo.h = o.h;
    p->N = N;
    p->nrhs_max = o.nrhs_max > 0 ? o.nrhs_max : 1;
    p->stream = (hipStream_t)hip_stream;
    p->sigma_const = sigma_t[0];
    p->h_st.assign(sigma_t, sigma_t + N);
    p->h_ss.assign(sigma_s, sigma_s + N);
    std::vector<float> st32(N);
    for (long j = 0; j < N; ++j) st32[j] = (float)sigma_t[j];

    ert_status st = ERT_OK;
    do {
        if (hipMalloc(&p->d_st, N * sizeof(double)) != hipSuccess ||
            hipMalloc(&p->d_st32, N * sizeof(float)) != hipSuccess ||
            hipMalloc(&p->d_ss, N * sizeof(double)) != hipSuccess ||
            hipMalloc(&p->d_diag, N * sizeof(double)) != hipSuccess) {
            record_error("ert_vie_plan: device allocation failed");
            st = ERT_ENOMEM;
            break;
        }
        st = ERT_HIPST(hipMemcpyAsync(p->d_st, sigma_t, N * sizeof(double), hipMemcpyHostToDevice, p->stream));
        if (st == ERT_OK)
            st = ERT_HIPST(hipMemcpyAsync(p->d_st32, st32.data(), N * sizeof(float), hipMemcpyHostToDevice,
                                          p->stream));
        if (st == ERT_OK)
            st = ERT_HIPST(hipMemcpyAsync(p->d_ss, sigma_s, N * sizeof(double), hipMemcpyHostToDevice, p->stream));
        if (st != ERT_OK) break;
        st = selfcell_compute(p);
    } while (0);
    if (st != ERT_OK) {
        ert_vie_destroy(p);
        return st;
    }
    *out = p;
    return ERT_OK;
}

ert_status ert_vie_apply_ex(ert_vie_plan_t p, int op, int method, int prec, const double* x, double* y, int nrhs)
{
    if (!p || !x || !y) return ERT_EINVAL;
    if (op < ERT_OP_G || op > ERT_OP_A) return ERT_EINVAL;
    if (method != ERT_DIRECT && method != ERT_FMM) return ERT_EINVAL;
    if (prec != ERT_FP64 && prec != ERT_FP32 && prec != ERT_BF16X3) return ERT_EINVAL;
    if (nrhs < 1 || nrhs > p->nrhs_max) return ERT_EINVAL;
    return apply_dispatch(p, op, method, prec, x, y, nrhs);
}

ert_status ert_vie_apply(ert_vie_plan_t p, int op, const double* x, double* y, int nrhs)
{
    if (!p) return ERT_EINVAL;
    return ert_vie_apply_ex(p, op, p->o.method, p->o.prec, x, y, nrhs);
}

ert_status ert_vie_profile(ert_vie_plan_t p, int enable, double* stage_ms, int* stage_launches)
{
    if (!p) return ERT_EINVAL;
    ERT_TRY(p->prof.resolve());
    if (stage_ms)
        for (int i = 0; i < ERT_NSTAGES; ++i) stage_ms[i] = p->prof.ms[i];
    if (stage_launches)
        for (int i = 0; i < ERT_NSTAGES; ++i) stage_launches[i] = p->prof.launches[i];
    if (enable && !p->prof.on) p->prof.clear();
    p->prof.on = enable != 0;
    return ERT_OK;
}

ert_status ert_vie_fmm_info(ert_vie_plan_t p, int prec, ert_fmm_info* info)
{
    if (!p || !info || prec < ERT_FP64 || prec > ERT_BF16X3) return ERT_EINVAL;
    return fmm_info(p, prec, info);
}

ert_status ert_vie_fft_precond(ert_vie_plan_t p, const double* r, double* z, int nrhs)
{
    if (!p || !r || !z || nrhs < 1 || nrhs > p->nrhs_max) return ERT_EINVAL;
    return fftpc_apply(p, r, z, nrhs);
}

ert_status ert_vie_transport(ert_vie_plan_t p, const double* U, const double* f, const double* dirs, int ndir,
                             double* phi)
{
    if (!p || !dirs || !phi || ndir < 1) return ERT_EINVAL;
    return transport_sweep(p, U, f, dirs, ndir, phi);
}

ert_status ert_vie_transport_noalloc(ert_vie_plan_t p, const double* U, const double* f, const double* dirs,
                                     int ndir, double* phi)
{
    if (!p || !dirs || !phi || ndir < 1) return ERT_EINVAL;
    return transport_sweep_noalloc(p, U, f, dirs, ndir, phi);
}

ert_status ert_vie_net_apply(ert_vie_plan_t p, ert_net_t net, const double* r, double* z)
{
    if (!p || !net || !r || !z) return ERT_EINVAL;
    NetImpl* n = net_impl(net);
    const int* g = net_grid(n);
    const int f = p->o.dim == 3 && g[0] > 0 ? p->geo.n0 / g[0] : 0;
    if (p->o.dim != 3 || f < 1 || g[0] * f != p->geo.n0 || g[1] * f != p->geo.n1 || g[2] * f != p->geo.n2) {
        record_error("ert_vie_net_apply: the network's grid is not the plan's grid coarsened by one factor");
        return ERT_EINVAL;
    }
    return net_precond(n, r, p->d_st, p->d_ss, z, p->stream, p->o.n);
}

ert_status ert_vie_restrict(ert_vie_plan_t p, int factor, const double* x, double* y, int nrhs)
{
    if (!p || !x || !y || nrhs < 1 || factor < 1) return ERT_EINVAL;
    if (p->o.dim != 3) {
        record_error("ert_vie_restrict: three-dimensional grids only");
        return ERT_EUNSUPPORTED;
    }
    const int n[3] = {p->geo.n0, p->geo.n1, p->geo.n2};
    for (int a = 0; a < 3; ++a)
        if (n[a] % factor != 0) {
            record_error("ert_vie_restrict: the grid is not a multiple of the factor");
            return ERT_EINVAL;
        }
    return restrict_avg(p->stream, x, n, factor, y, nrhs);
}

ert_status ert_vie_diff_precond(ert_vie_plan_t p, const double* r, double* z, int nrhs)
{
    if (!p || !r || !z || nrhs < 1 || nrhs > p->nrhs_max) return ERT_EINVAL;
    return diffpc_apply(p, r, z, nrhs);
}

ert_status ert_vie_fft_info(ert_vie_plan_t p, ert_fft_info* info)
{
    if (!p || !info) return ERT_EINVAL;
    return fftpc_info(p, info);
}

ert_status ert_vie_diag(ert_vie_plan_t p, double* d)
{
    if (!p || !d) return ERT_EINVAL;
    ERT_HIP(hipMemcpyAsync(d, p->d_diag, p->N * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    ERT_HIP(hipStreamSynchronize(p->stream));
    return ERT_OK;
}

ert_status ert_vie_solve(ert_vie_plan_t p, const double* f, double* U, int nrhs, const ert_solve_opts* sopts,
                         ert_solve_info* info)
{
    if (!p || !f || !U) return ERT_EINVAL;
    if (nrhs < 1 || nrhs > p->nrhs_max) return ERT_EINVAL;
    ert_solve_opts so;
    std::memset(&so, 0, sizeof(so));
    if (sopts) so = *sopts;
    if (so.tol == 0.0) so.tol = 1e-8;
    if (so.max_iter == 0) so.max_iter = 500;
    if (so.inner_tol == 0.0) so.inner_tol = 1e-5;
    if (!(so.tol > 0.0) || so.max_iter < 1 || so.restart < 0 || !(so.inner_tol > 0.0) || so.inner_tol >= 1.0)
        return ERT_EINVAL;
    if (so.precond_kind < ERT_PRECOND_NONE || so.precond_kind > ERT_PRECOND_DIFFUSION) return ERT_EINVAL;
    if (so.precond_steps < 0 || so.history_max < 0 || (so.history_max > 0 && !so.history)) return ERT_EINVAL;
    NetImpl* net = so.precond ? net_impl(so.precond) : nullptr;
    if (net) {
        const int* g = net_grid(net);
        const int f = p->o.dim == 3 && g[0] > 0 ? p->geo.n0 / g[0] : 0;
        if (p->o.dim != 3 || f < 1 || g[0] * f != p->geo.n0 || g[1] * f != p->geo.n1 || g[2] * f != p->geo.n2) {
            record_error("ert_vie_solve: the preconditioner's grid is not the plan's grid coarsened by one factor");
            return ERT_EINVAL;
        }
        if (so.block && nrhs > 1) {
            record_error("ert_vie_solve: a learned preconditioner is not combined with block GMRES");
            return ERT_EUNSUPPORTED;
        }
    }
    const long N = p->N;
    const int method = p->o.method;
    const int prec_outer = so.mixed ? ERT_FP64 : p->o.prec;
    const int prec_inner = (p->o.prec == ERT_FP64) ? ERT_FP32 : p->o.prec;

    ert_solve_info inf;
    std::memset(&inf, 0, sizeof(inf));
    ert_status result = ERT_OK;
    // the FMM data of every operator this solve applies are built (on first use of a
    // precision) before the timed solve starts; that time is reported as t_setup
    double t_setup = 0.0;
    {
        const auto ts = std::chrono::steady_clock::now();
        if (method == ERT_FMM) {
            ERT_TRY(fmm_build(p, prec_outer));
            if (so.mixed) ERT_TRY(fmm_build(p, prec_inner));
            if (net) ERT_TRY(fmm_build(p, ERT_FP64));   // the learned steps' FP64 residual check
        }
        ERT_TRY(ERT_HIPST(hipStreamSynchronize(p->stream)));
        t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count();
        inf.t_setup = t_setup;
    }
    auto t0 = std::chrono::steady_clock::now();
    // vectors beyond the Krylov workspace: phi, r, d, and the trial iterate with its
    // residual of the learned refinement (per column, reused; plan-owned)
    ERT_TRY(ensure_solve_scratch(p, (size_t)5 * N));
    double* phi = p->d_solve;
    double* r = phi + N;
    double* d = phi + 2 * N;
    double* trial = phi + 3 * N;
    ert_status st = ERT_OK;
    if (so.block && nrhs > 1) {
        // all columns at once: phi = A f batched, then block GMRES (or block refinement)
        double* blk = nullptr;
        if (hipMalloc(&blk, (size_t)3 * N * nrhs * sizeof(double)) != hipSuccess) {
            record_error("ert_vie_solve: block workspace allocation failed");
            return ERT_ENOMEM;
        }
        double* Phi = blk;
        double* Rb = blk + (size_t)N * nrhs;
        double* Db = blk + (size_t)2 * N * nrhs;
        do {
            if (so.rhs_is_phi)
                st = ERT_HIPST(hipMemcpyAsync(Phi, f, sizeof(double) * N * nrhs, hipMemcpyDeviceToDevice, p->stream));
            else
                st = apply_dispatch(p, ERT_OP_G, method, prec_outer, f, Phi, nrhs);
            if (st != ERT_OK) break;
            inf.matvecs++;
            int it = 0, cy = 0, mv = 0;
            double est = 0.0, tr = 0.0;
            bool conv = false, brk = false;
            if (!so.mixed) {
                st = block_gmres(p, method, prec_outer, Phi, U, nrhs, so.tol, so.max_iter, so.restart, true, &it, &cy,
                                 &mv, &est, &tr, &conv, so.precond_kind, &brk);
                if (st != ERT_OK) break;
                inf.iters = it;
                inf.restarts = cy > 0 ? cy - 1 : 0;
                inf.matvecs += mv;
                inf.rel_resid_est = est;
                inf.rel_resid_true = tr;
                inf.converged = conv ? 1 : 0;
                if (brk) st = finish_columns(p, method, prec_outer, Phi, U, Rb, d, nrhs, so, so.precond_kind, &inf);
            } else {
                // block refinement: R = Phi - A64 U, inner block GMRES on the FP32 operator
                st = dev_zero(p->stream, U, N * nrhs);
                if (st != ERT_OK) break;
                st = ERT_HIPST(hipMemcpyAsync(Rb, Phi, sizeof(double) * N * nrhs, hipMemcpyDeviceToDevice, p->stream));
                if (st != ERT_OK) break;
                std::vector<double> pn(nrhs), rn(nrhs);
                st = ensure_workspace(p, 3 * N, (size_t)kPartials * 4 + 16);
                if (st != ERT_OK) break;
                double* dn = p->d_red + (size_t)kPartials * 4;
                for (int b = 0; b < nrhs && st == ERT_OK; ++b) pn[b] = dev_norm(p, Phi + (size_t)b * N, p->d_red, dn, &st);
                int used = 0;
                double worst = 1.0, prev_worst = 0.0;
                for (int outer = 0; outer < 200 && st == ERT_OK; ++outer) {
                    worst = 0.0;
                    for (int b = 0; b < nrhs && st == ERT_OK; ++b) {
                        st = ensure_workspace(p, 3 * N, (size_t)kPartials * 4 + 16);
                        if (st != ERT_OK) break;
                        rn[b] = dev_norm(p, Rb + (size_t)b * N, p->d_red, p->d_red + (size_t)kPartials * 4, &st);
                        worst = std::max(worst, pn[b] > 0 ? rn[b] / pn[b] : 0.0);
                    }
                    if (st != ERT_OK) break;
                    inf.rel_resid_true = worst;
                    if (worst <= so.tol) { inf.converged = 1; break; }
                    if (used >= so.max_iter) break;
                    if (outer > 0 && !(worst < prev_worst)) break;   // no progress: stop (ERT_ENOCONV)
                    prev_worst = worst;
                    st = block_gmres(p, method, prec_inner, Rb, Db, nrhs, so.inner_tol, so.max_iter - used, so.restart,
                                     false, &it, &cy, &mv, &est, &tr, &conv, so.precond_kind, &brk);
                    if (st != ERT_OK) break;
                    used += it;
                    inf.iters += it;
                    inf.matvecs += mv;
                    inf.rel_resid_est = est;
                    if (brk) {
                        // no block basis for this residual: inner solves column by column
                        // (columns already within tol get no correction)
                        Precond pcb;
                        pcb.kind = so.precond_kind;
                        for (int b = 0; b < nrhs && st == ERT_OK; ++b) {
                            double* Db_b = Db + (size_t)b * N;
                            if (rn[b] <= so.tol * pn[b]) {
                                st = dev_zero(p->stream, Db_b, N);
                                continue;
                            }
                            RunStats rs;
                            st = gmres_run(p, method, prec_inner, Rb + (size_t)b * N, Db_b, so.inner_tol,
                                           std::max(1, so.max_iter - used), so.restart, false, &rs, &pcb);
                            used += rs.iters;
                            inf.iters += rs.iters;
                            inf.matvecs += rs.matvecs;
                        }
                        if (st != ERT_OK) break;
                    }
                    st = dev_add(p->stream, U, Db, N * nrhs);
                    if (st != ERT_OK) break;
                    st = apply_dispatch(p, ERT_OP_A, method, ERT_FP64, U, Db, nrhs);
                    if (st != ERT_OK) break;
                    inf.matvecs++;
                    st = dev_sub(p->stream, Rb, Phi, Db, N * nrhs);
                    inf.restarts = outer + 1;
                }
            }
            if (st == ERT_OK && !inf.converged) result = ERT_ENOCONV;
        } while (0);
        (void)hipStreamSynchronize(p->stream);
        (void)hipFree(blk);
        inf.t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (info) *info = inf;
        return st != ERT_OK ? st : result;
    }
    Precond pc;
    pc.kind = so.precond_kind;
    if (pc.kind) st = precond_apply(p, pc.kind, nullptr, nullptr, 0);   // build it before the first column
    for (int c = 0; c < nrhs && st == ERT_OK; ++c) {
        std::memset(&inf, 0, sizeof(inf));
        inf.t_setup = t_setup;
        const double* fc = f + (size_t)c * N;
        double* Uc = U + (size_t)c * N;
        if (so.rhs_is_phi) {
            st = (hipMemcpyAsync(phi, fc, N * sizeof(double), hipMemcpyDeviceToDevice, p->stream) == hipSuccess)
                     ? ERT_OK : ERT_EDEVICE;
        } else {
            // the learned refinement judges its steps with the FP64 operator: phi in FP64 too
            st = apply_dispatch(p, ERT_OP_G, method, net ? ERT_FP64 : prec_outer, fc, phi, 1);
            inf.matvecs++;
        }
        if (st != ERT_OK) break;
        if (net) {
            st = learned_refine(p, method, so.mixed ? prec_inner : p->o.prec, net, so.precond_kind, phi, Uc, r, d,
                                trial, so, &inf);
        } else if (!so.mixed) {
            RunStats rs;
            History hist;
            if (c == 0 && so.history && so.history_max > 0) {
                hist.buf = so.history;
                hist.cap = so.history_max;
            }
            st = gmres_run(p, method, prec_outer, phi, Uc, so.tol, so.max_iter, so.restart, true, &rs, &pc,
                           hist.buf ? &hist : nullptr);
            inf.history_count = hist.count;
            inf.iters = rs.iters;
            inf.matvecs += rs.matvecs;
            inf.restarts = rs.cycles > 0 ? rs.cycles - 1 : 0;
            inf.rel_resid_est = rs.est;
            inf.rel_resid_true = rs.true_rel;
            inf.converged = rs.converged ? 1 : 0;
        } else {
            // iterative refinement: r = phi - A64 U (FP64), inner GMRES on the FP32 operator
            st = dev_zero(p->stream, Uc, N);
            if (st != ERT_OK) break;
            st = (hipMemcpyAsync(r, phi, N * sizeof(double), hipMemcpyDeviceToDevice, p->stream) == hipSuccess)
                     ? ERT_OK : ERT_EDEVICE;
            if (st != ERT_OK) break;
            st = ensure_workspace(p, 3 * N, (size_t)kPartials * 4 + 16);
            if (st != ERT_OK) break;
            double* dn = p->d_red + (size_t)kPartials * 4;
            double pnorm = dev_norm(p, phi, p->d_red, dn, &st);
            if (st != ERT_OK) break;
            double rnorm = pnorm;
            int used = 0;
            for (int outer = 0; outer < 200; ++outer) {
                inf.rel_resid_true = pnorm > 0 ? rnorm / pnorm : 0.0;
                if (rnorm <= so.tol * pnorm) { inf.converged = 1; break; }
                if (used >= so.max_iter) break;
                RunStats rs;
                // the inner solve only needs to reduce this residual by inner_tol
                st = gmres_run(p, method, prec_inner, r, d, so.inner_tol, so.max_iter - used, so.restart, false, &rs,
                               &pc);
                if (st != ERT_OK) break;
                used += rs.iters;
                inf.iters += rs.iters;
                inf.matvecs += rs.matvecs;
                inf.rel_resid_est = rs.est;
                st = dev_add(p->stream, Uc, d, N);
                if (st != ERT_OK) break;
                st = apply_dispatch(p, ERT_OP_A, method, ERT_FP64, Uc, d, 1);
                if (st != ERT_OK) break;
                inf.matvecs++;
                st = dev_sub(p->stream, r, phi, d, N);
                if (st != ERT_OK) break;
                st = ensure_workspace(p, 3 * N, (size_t)kPartials * 4 + 16);
                if (st != ERT_OK) break;
                dn = p->d_red + (size_t)kPartials * 4;
                rnorm = dev_norm(p, r, p->d_red, dn, &st);
                if (st != ERT_OK) break;
                inf.restarts = outer + 1;
            }
            if (st == ERT_OK) inf.rel_resid_true = pnorm > 0 ? rnorm / pnorm : 0.0;
            if (st == ERT_OK && rnorm <= so.tol * pnorm) inf.converged = 1;
        }
        if (st == ERT_OK && !inf.converged) result = ERT_ENOCONV;
    }
    (void)hipStreamSynchronize(p->stream);
    inf.t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return st != ERT_OK ? st : result;
}

}  // extern "C"
