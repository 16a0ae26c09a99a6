// Dense symmetric eigen-decomposition on the host (FP64), used at plan time to
// compress the far-field translations: Householder reduction to tridiagonal
// form, then the implicit QL iteration with Wilkinson-type shifts, with the
// orthogonal transformations accumulated into the eigenvector matrix.  The QL
// stage follows the published tridiagonal QL algorithm with implicit shifts
// (Bowdler, Martin, Reinsch and Wilkinson, Numer. Math. 11 (1968), the EISPACK
// routine tql2), step for step: the shift from the leading 2 x 2 block, the
// chase of the bulge by plane rotations, and the rotations applied to Z.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace ertvie {

// A: n x n symmetric, row-major; on return the columns of Z (row-major n x n)
// are orthonormal eigenvectors and w the eigenvalues, sorted descending.
void sym_eig(int n, const std::vector<double>& A, std::vector<double>& w, std::vector<double>& Z)
{
    std::vector<double> a(A);
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n), p(n), q(n);
    // Householder: column k below the subdiagonal is annihilated by H = I - 2 v v^T
    for (int k = 0; k + 2 < n; ++k) {
        double norm = 0.0;
        for (int i = k + 1; i < n; ++i) norm += a[(size_t)i * n + k] * a[(size_t)i * n + k];
        norm = std::sqrt(norm);
        if (norm == 0.0) continue;
        const double x0 = a[(size_t)(k + 1) * n + k];
        const double alpha = x0 > 0 ? -norm : norm;
        double vn = 0.0;
        for (int i = 0; i < n; ++i) v[i] = 0.0;
        for (int i = k + 1; i < n; ++i) v[i] = a[(size_t)i * n + k];
        v[k + 1] -= alpha;
        for (int i = k + 1; i < n; ++i) vn += v[i] * v[i];
        vn = std::sqrt(vn);
        if (vn == 0.0) continue;
        for (int i = k + 1; i < n; ++i) v[i] /= vn;
        // p = A v (trailing block), w = p - (v.p) v, A <- A - 2 v w^T - 2 w v^T
        double vp = 0.0;
        for (int i = k; i < n; ++i) {
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += a[(size_t)i * n + j] * v[j];
            p[i] = s;
        }
        for (int i = k + 1; i < n; ++i) vp += v[i] * p[i];
        for (int i = k; i < n; ++i) q[i] = p[i] - vp * v[i];
        for (int i = k; i < n; ++i)
            for (int j = k; j < n; ++j) a[(size_t)i * n + j] -= 2.0 * (v[i] * q[j] + q[i] * v[j]);
        // accumulate Z <- Z H
        for (int r = 0; r < n; ++r) {
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += Z[(size_t)r * n + j] * v[j];
            for (int j = k + 1; j < n; ++j) Z[(size_t)r * n + j] -= 2.0 * s * v[j];
        }
    }
    std::vector<double> d(n), e(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = a[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = a[(size_t)(i + 1) * n + i];   // couples i and i+1
    // implicit QL on (d, e)
    for (int l = 0; l < n; ++l) {
        for (int iter = 0; iter < 200; ++iter) {
            int m = l;
            for (; m + 1 < n; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-300 + 2.2e-16 * dd) break;
            }
            if (m == l) break;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double s = 1.0, c = 1.0, pp = 0.0;
            int i = m - 1;
            bool early = false;
            for (; i >= l; --i) {
                const double f = s * e[i];
                const double b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= pp;
                    e[m] = 0.0;
                    early = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - pp;
                r = (d[i] - g) * s + 2.0 * c * b;
                pp = s * r;
                d[i + 1] = g + pp;
                g = c * r - b;
                for (int k = 0; k < n; ++k) {
                    const double zf = Z[(size_t)k * n + i + 1];
                    Z[(size_t)k * n + i + 1] = s * Z[(size_t)k * n + i] + c * zf;
                    Z[(size_t)k * n + i] = c * Z[(size_t)k * n + i] - s * zf;
                }
            }
            if (early) continue;
            d[l] -= pp;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    // sort descending
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] > d[y]; });
    std::vector<double> Zs((size_t)n * n);
    w.resize(n);
    for (int c = 0; c < n; ++c) {
        w[c] = d[idx[c]];
        for (int r = 0; r < n; ++r) Zs[(size_t)r * n + c] = Z[(size_t)r * n + idx[c]];
    }
    Z.swap(Zs);
}

}  // namespace ertvie
