// Block GMRES for many right-hand sides at once (Algorithm 1 step S.2 with the
// nrhs columns of Phi sharing one block Krylov space).  Every operator
// application is one batched apply of all columns, so the near field and the
// far-field translations run as matrix-matrix products.
//
//   R0 = Phi - A X0 = V_0 B0                       (Cholesky QR, twice)
//   W  = A V_j;  H_ij = V_i^T W, W -= V_i H_ij      (block classical Gram-Schmidt, twice)
//   W  = V_{j+1} H_{j+1,j}                         (Cholesky QR, twice)
//   min || E1 B0 - Hbar_j Y ||_F                   (Householder QR of the block
//                                                   Hessenberg matrix, updated per block column)
//   X  = X0 + [V_0 .. V_j] Y
//
// The level-3 work (inner products, updates, Cholesky QR) runs on the device in
// FP64; the small block Hessenberg least-squares problem on the host.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace ertvie {

namespace {

struct DevBuf {
    double* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    ert_status alloc(size_t n)
    {
        if (hipMalloc(&p, std::max<size_t>(1, n) * sizeof(double)) != hipSuccess) {
            record_error("block GMRES: device allocation failed");
            return ERT_ENOMEM;
        }
        return ERT_OK;
    }
};

// Upper Cholesky factor of a symmetric positive definite p x p (row-major); false if not SPD.
bool cholesky_upper(int p, const std::vector<double>& G, std::vector<double>& R)
{
    R.assign((size_t)p * p, 0.0);
    for (int i = 0; i < p; ++i) {
        double d = G[(size_t)i * p + i];
        for (int k = 0; k < i; ++k) d -= R[(size_t)k * p + i] * R[(size_t)k * p + i];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        const double rii = std::sqrt(d);
        R[(size_t)i * p + i] = rii;
        for (int j = i + 1; j < p; ++j) {
            double s = G[(size_t)i * p + j];
            for (int k = 0; k < i; ++k) s -= R[(size_t)k * p + i] * R[(size_t)k * p + j];
            R[(size_t)i * p + j] = s / rii;
        }
    }
    return true;
}

// inverse of an upper-triangular p x p (row-major)
void upper_inverse(int p, const std::vector<double>& R, std::vector<double>& Ri)
{
    Ri.assign((size_t)p * p, 0.0);
    for (int c = 0; c < p; ++c) {
        for (int i = c; i >= 0; --i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = i + 1; k <= c; ++k) s -= R[(size_t)i * p + k] * Ri[(size_t)k * p + c];
            Ri[(size_t)i * p + c] = s / R[(size_t)i * p + i];
        }
    }
}

struct Ctx {
    ert_plan_impl* pl;
    hipStream_t s;
    long N;
    int p;
    double* work;       // split-K workspace
    size_t work_elems;
    double* small;      // device p x p / (m+1)p x p scratch
};

// Upper Cholesky factor of the Gram matrix G after scaling it to unit diagonal
// (G = D Gs D, D = diag(sqrt(G_ii)), Gs = Rs^T Rs, R = Rs D): columns of very
// different norms (a converged column beside an unconverged one) then keep a
// well-conditioned factorisation.  False for a zero column or a Gram matrix that
// is not numerically positive definite (linearly dependent columns).
bool cholesky_scaled(int p, const std::vector<double>& G, std::vector<double>& R)
{
    std::vector<double> d(p), Gs((size_t)p * p);
    for (int i = 0; i < p; ++i) {
        const double gi = G[(size_t)i * p + i];
        if (!(gi > 0.0) || !std::isfinite(gi)) return false;
        d[i] = std::sqrt(gi);
    }
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) Gs[(size_t)i * p + j] = G[(size_t)i * p + j] / (d[i] * d[j]);
    if (!cholesky_upper(p, Gs, R)) return false;
    // a pivot far below the unit diagonal: the column is numerically dependent on the others
    for (int i = 0; i < p; ++i)
        if (!(R[(size_t)i * p + i] > 1e-7)) return false;
    for (int i = 0; i < p; ++i)
        for (int j = i; j < p; ++j) R[(size_t)i * p + j] *= d[j];
    return true;
}

// out (N x p) = in orthonormalised; R (host, p x p upper) with in = out R.
// Two passes of Cholesky QR; returns false on breakdown (rank-deficient block).
ert_status chol_qr2(Ctx& c, const double* in, double* out, double* tmp, std::vector<double>& R, bool* ok)
{
    const int p = c.p;
    const long N = c.N;
    std::vector<double> G((size_t)p * p), R1, R2, Ri;
    const double* src = in;
    double* dst[2] = {tmp, out};
    *ok = true;
    for (int pass = 0; pass < 2; ++pass) {
        ERT_TRY(dev_dgemm(c.s, p, p, N, 1.0, src, N, 1, src, 1, N, 0.0, c.small, p, 1, c.work, c.work_elems));
        ERT_HIP(hipMemcpyAsync(G.data(), c.small, sizeof(double) * p * p, hipMemcpyDeviceToHost, c.s));
        ERT_HIP(hipStreamSynchronize(c.s));
        std::vector<double>& Rk = pass == 0 ? R1 : R2;
        if (!cholesky_scaled(p, G, Rk)) {
            *ok = false;
            return ERT_OK;
        }
        upper_inverse(p, Rk, Ri);
        ERT_HIP(hipMemcpyAsync(c.small, Ri.data(), sizeof(double) * p * p, hipMemcpyHostToDevice, c.s));
        // dst = src * Ri  (N x p)
        ERT_TRY(dev_dgemm(c.s, (int)N, p, p, 1.0, src, 1, N, c.small, p, 1, 0.0, dst[pass], 1, N, nullptr, 0));
        src = dst[pass];
    }
    // in = out * (R2 R1)
    R.assign((size_t)p * p, 0.0);
    for (int i = 0; i < p; ++i)
        for (int j = i; j < p; ++j) {
            double s = 0.0;
            for (int k = i; k <= j; ++k) s += R2[(size_t)i * p + k] * R1[(size_t)k * p + j];
            R[(size_t)i * p + j] = s;
        }
    return ERT_OK;
}

}  // namespace

ert_status plan_apply(ert_plan_impl* p, int op, int method, int prec, const double* x, double* y, int nrhs);

// Block GMRES with x0 = 0 for (I - K) X = Phi, all nb columns in one block.
// Converged when every column's residual estimate reaches rtol ||Phi_b||; the
// true residual (same operator) is then checked and the method restarts if needed.
// With a preconditioner kind pk (FFT-based or diffusion, fixed linear maps):
// right preconditioning, i.e. the Krylov space of (I - K) M and the update
// X += M [V_0 .. V_j] Y.
// Breakdown: when the residual block at the start of a cycle has a zero or
// linearly dependent column (a zero right-hand side, two equal ones, a column
// solved exactly), no orthonormal block basis exists; the method then stops with
// *breakdown_out set, *conv_out false and X holding the iterate reached so far,
// and the caller finishes the columns one by one.  Convergence is only reported
// when every column's residual met rtol (the true residual with check_true).
ert_status block_gmres(ert_plan_impl* pl, int method, int prec, const double* Phi, double* X, int nb, double rtol,
                       int maxit, int restart, bool check_true, int* iters_out, int* cycles_out, int* matvecs_out,
                       double* est_out, double* true_out, bool* conv_out, int pk, bool* breakdown_out)
{
    const bool fft = pk != 0;     // right preconditioner of that kind (ERT_PRECOND_*)
    const long N = pl->N;
    const int p = nb;
    // Krylov dimension in blocks: restart, or (unrestarted) as many blocks as fit in 4 GiB
    // (134 MB per block at 64 columns of 64^3), beyond which the method restarts
    const long fit = std::max<long>(2, (4L << 30) / ((long)p * N * (long)sizeof(double)) - 1);
    const int m = std::max(1, std::min<int>(restart > 0 ? restart : (int)std::min<long>(maxit, fit), maxit));
    hipStream_t s = pl->stream;
    DevBuf V, W, R, T, small, work;
    ERT_TRY(V.alloc((size_t)(m + 1) * p * N));
    ERT_TRY(W.alloc((size_t)p * N));
    ERT_TRY(R.alloc((size_t)p * N));
    ERT_TRY(T.alloc((size_t)p * N));
    ERT_TRY(small.alloc((size_t)(m + 1) * p * p + (size_t)p * p));
    const size_t work_elems = (size_t)64 * (m + 1) * p * p;
    ERT_TRY(work.alloc(work_elems));
    Ctx c{pl, s, N, p, work.p, work_elems, small.p};
    int iters = 0, cycles = 0, matvecs = 0;
    double est = 1.0, truer = -1.0;
    bool converged = false, breakdown = false;

    // column norms of Phi
    std::vector<double> pnorm(p), G((size_t)p * p);
    ERT_TRY(dev_dgemm(s, p, p, N, 1.0, Phi, N, 1, Phi, 1, N, 0.0, small.p, p, 1, work.p, work_elems));
    ERT_HIP(hipMemcpyAsync(G.data(), small.p, sizeof(double) * p * p, hipMemcpyDeviceToHost, s));
    ERT_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < p; ++b) pnorm[b] = std::sqrt(std::max(0.0, G[(size_t)b * p + b]));
    ERT_TRY(dev_zero(s, X, N * p));
    ERT_HIP(hipMemcpyAsync(R.p, Phi, sizeof(double) * N * p, hipMemcpyDeviceToDevice, s));

    const int LD = (m + 1) * p;           // leading dimension of the host block Hessenberg (column-major)
    std::vector<double> H((size_t)LD * m * p), g((size_t)LD * p), Hc((size_t)(m + 1) * p * p), Y;
    std::vector<std::vector<double>> refl((size_t)m * p);
    std::vector<double> tau((size_t)m * p);
    std::vector<double> B0;
    while (iters < maxit) {
        ++cycles;
        bool ok = true;
        ERT_TRY(chol_qr2(c, R.p, V.p, T.p, B0, &ok));
        if (!ok) {       // residual block rank deficient: no block basis (see above)
            breakdown = true;
            break;
        }
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        for (int i = 0; i < p; ++i)
            for (int b = 0; b < p; ++b) g[(size_t)b * LD + i] = B0[(size_t)i * p + b];
        int k = 0;
        bool cyc_conv = false;
        for (int j = 0; j < m && iters < maxit; ++j) {
            double* Vj = V.p + (size_t)j * p * N;
            if (fft) {
                ERT_TRY(precond_apply(pl, pk, Vj, T.p, p));    // T is free until the block QR below
                ERT_TRY(plan_apply(pl, ERT_OP_A, method, prec, T.p, W.p, p));
            } else {
                ERT_TRY(plan_apply(pl, ERT_OP_A, method, prec, Vj, W.p, p));
            }
            ++matvecs;
            const int rows = (j + 1) * p;
            std::fill(Hc.begin(), Hc.end(), 0.0);
            std::vector<double> hpass((size_t)rows * p);
            for (int pass = 0; pass < 2; ++pass) {
                ERT_TRY(dev_dgemm(s, rows, p, N, 1.0, V.p, N, 1, W.p, 1, N, 0.0, small.p, p, 1, work.p, work_elems));
                ERT_TRY(dev_dgemm(s, (int)N, p, rows, -1.0, V.p, 1, N, small.p, p, 1, 1.0, W.p, 1, N, nullptr, 0));
                ERT_HIP(hipMemcpyAsync(hpass.data(), small.p, sizeof(double) * rows * p, hipMemcpyDeviceToHost, s));
                ERT_HIP(hipStreamSynchronize(s));
                for (size_t q = 0; q < hpass.size(); ++q) Hc[q] += hpass[q];
            }
            std::vector<double> Rj;
            ERT_TRY(chol_qr2(c, W.p, V.p + (size_t)(j + 1) * p * N, T.p, Rj, &ok));
            // block column j of Hbar: Hc (rows x p, row-major) above, Rj below
            for (int col = 0; col < p; ++col) {
                double* hc = &H[(size_t)(j * p + col) * LD];
                for (int r = 0; r < rows; ++r) hc[r] = Hc[(size_t)r * p + col];
                for (int r = 0; r < p; ++r) hc[rows + r] = ok ? Rj[(size_t)r * p + col] : 0.0;
            }
            // previous reflectors
            for (int jc = 0; jc < j; ++jc)
                for (int kk = 0; kk < p; ++kk) {
                    const std::vector<double>& v = refl[(size_t)jc * p + kk];
                    const double t = tau[(size_t)jc * p + kk];
                    const int r0 = jc * p + kk;
                    if (t == 0.0) continue;
                    for (int col = 0; col < p; ++col) {
                        double* hc = &H[(size_t)(j * p + col) * LD];
                        double w = 0.0;
                        for (size_t q = 0; q < v.size(); ++q) w += v[q] * hc[r0 + q];
                        w *= t;
                        for (size_t q = 0; q < v.size(); ++q) hc[r0 + q] -= w * v[q];
                    }
                }
            // new reflectors for the columns of block j
            for (int kk = 0; kk < p; ++kk) {
                const int col = j * p + kk, r0 = col, r1 = (j + 2) * p;
                double* hc = &H[(size_t)col * LD];
                double nrm = 0.0;
                for (int r = r0; r < r1; ++r) nrm += hc[r] * hc[r];
                nrm = std::sqrt(nrm);
                std::vector<double> v(r1 - r0, 0.0);
                double t = 0.0;
                if (nrm > 0.0) {
                    const double alpha = hc[r0] > 0 ? -nrm : nrm;
                    for (int r = r0; r < r1; ++r) v[r - r0] = hc[r];
                    v[0] -= alpha;
                    double vv = 0.0;
                    for (double e : v) vv += e * e;
                    t = vv > 0.0 ? 2.0 / vv : 0.0;
                    hc[r0] = alpha;
                    for (int r = r0 + 1; r < r1; ++r) hc[r] = 0.0;
                    for (int kc = kk + 1; kc < p; ++kc) {
                        double* h2 = &H[(size_t)(j * p + kc) * LD];
                        double w = 0.0;
                        for (int r = r0; r < r1; ++r) w += v[r - r0] * h2[r];
                        w *= t;
                        for (int r = r0; r < r1; ++r) h2[r] -= w * v[r - r0];
                    }
                    for (int b = 0; b < p; ++b) {
                        double* gb = &g[(size_t)b * LD];
                        double w = 0.0;
                        for (int r = r0; r < r1; ++r) w += v[r - r0] * gb[r];
                        w *= t;
                        for (int r = r0; r < r1; ++r) gb[r] -= w * v[r - r0];
                    }
                }
                refl[(size_t)j * p + kk] = v;
                tau[(size_t)j * p + kk] = t;
            }
            ++iters;
            k = j + 1;
            // residual estimates: rows (j+1)p .. (j+2)p of g
            est = 0.0;
            for (int b = 0; b < p; ++b) {
                double r2 = 0.0;
                for (int r = (j + 1) * p; r < (j + 2) * p; ++r) r2 += g[(size_t)b * LD + r] * g[(size_t)b * LD + r];
                const double rel = pnorm[b] > 0 ? std::sqrt(r2) / pnorm[b] : 0.0;
                est = std::max(est, rel);
            }
            if (est <= rtol || !ok) {
                // !ok: the new block direction is dependent on the basis; the least-squares
                // solution over the basis so far is still the best update of this cycle
                cyc_conv = est <= rtol;
                break;
            }
        }
        // Y = T^{-1} g_top, T = leading k p x k p upper triangle
        const int n = k * p;
        Y.assign((size_t)n * p, 0.0);   // row-major n x p
        for (int b = 0; b < p; ++b)
            for (int i = n - 1; i >= 0; --i) {
                double sacc = g[(size_t)b * LD + i];
                for (int q = i + 1; q < n; ++q) sacc -= H[(size_t)q * LD + i] * Y[(size_t)q * p + b];
                const double d = H[(size_t)i * LD + i];
                Y[(size_t)i * p + b] = d != 0.0 ? sacc / d : 0.0;
            }
        DevBuf Yd;
        ERT_TRY(Yd.alloc((size_t)n * p));
        ERT_HIP(hipMemcpyAsync(Yd.p, Y.data(), sizeof(double) * n * p, hipMemcpyHostToDevice, s));
        if (fft) {
            ERT_TRY(dev_dgemm(s, (int)N, p, n, 1.0, V.p, 1, N, Yd.p, p, 1, 0.0, T.p, 1, N, nullptr, 0));
            ERT_TRY(precond_apply(pl, pk, T.p, W.p, p));
            ERT_TRY(dev_add(s, X, W.p, N * p));
        } else {
            ERT_TRY(dev_dgemm(s, (int)N, p, n, 1.0, V.p, 1, N, Yd.p, p, 1, 1.0, X, 1, N, nullptr, 0));
        }
        ERT_HIP(hipStreamSynchronize(s));
        if (!check_true && cyc_conv) {
            converged = true;
            break;
        }
        // true residual R = Phi - A X
        ERT_TRY(plan_apply(pl, ERT_OP_A, method, prec, X, T.p, p));
        ++matvecs;
        ERT_TRY(dev_sub(s, R.p, Phi, T.p, N * p));
        ERT_TRY(dev_dgemm(s, p, p, N, 1.0, R.p, N, 1, R.p, 1, N, 0.0, small.p, p, 1, work.p, work_elems));
        ERT_HIP(hipMemcpyAsync(G.data(), small.p, sizeof(double) * p * p, hipMemcpyDeviceToHost, s));
        ERT_HIP(hipStreamSynchronize(s));
        truer = 0.0;
        for (int b = 0; b < p; ++b)
            truer = std::max(truer, pnorm[b] > 0 ? std::sqrt(std::max(0.0, G[(size_t)b * p + b])) / pnorm[b] : 0.0);
        if (truer <= rtol) {
            converged = true;
            break;
        }
    }
    *iters_out = iters;
    *cycles_out = cycles;
    *matvecs_out = matvecs;
    *est_out = est;
    *true_out = truer;
    *conv_out = converged;
    if (breakdown_out) *breakdown_out = breakdown && !converged;
    return ERT_OK;
}

}  // namespace ertvie
