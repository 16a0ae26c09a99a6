/*
 * oracle.c -- plain, slow, FP64 CPU reference for the isotropic-ERT
 * volume-integral operator and its GMRES solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only tests/, the smoke check and the CPU-baseline leg of
 * bench.py do.  It shares no code, header, table or helper with the HIP
 * library; the only thing both sides consume is the seeded input generator.
 *
 * What it computes, and where the paper defines it:
 *
 *   Collocation (Sec. 3.1, "Discretization"): a uniform cell-centred grid of
 *   n[0] x n[1] (x n[2]) cells of side h; collocation point of cell
 *   (i0,i1,i2) is x = h (i + 1/2) per axis; linear index j = i0 + n0 (i1 + n1 i2).
 *
 *   Kernel (Sec. 2, eq. EQ:Kernel without the mu_s factor):
 *       G(x,y) = E(x,y) / (|S^{d-1}| |x-y|^{d-1}),   |S^1| = 2 pi, |S^2| = 4 pi,
 *       E(x,y) = exp(-tau(x,y)),  tau = line integral of sigma_t from x to y.
 *   Homogeneous media (eq. EQ:Kernel Cons):  tau = sigma_t |x-y|.
 *   Gridded media (Sec. 4.2 leaves the line-integral rule open as long as it is
 *   second-order): midpoint rule with m = smallest integer such that the
 *   step |x-y|/m <= h/2, applied to the d-linear interpolant of the
 *   cell-centred sigma_t, each coordinate clamped to [h/2, n_a h - h/2].
 *
 *   Matrix (Sec. 3.2, approach (M-iii) with the diagonal "computed
 *   explicitly"):  A_jk = h^d G(x_j,x_k) for j != k;
 *   A_jj = (1/|S^{d-1}|) * integral over the own cell of E(x_j,y)/|x_j-y|^{d-1} dy,
 *   done in polar form around x_j:  integral over directions v of
 *   integral_0^{rho(v)} E(x_j, x_j + r v) dr, rho = distance to the cell wall.
 *
 *   Apply (Sec. 3.2, eq. EQ: LINEAR SYSTEM; the paper's K is A diag(sigma_s)):
 *       op 0: y = A x        (phi = K(mu_s^{-1} f) = A f,  Algorithm 1 S.1)
 *       op 1: y = A (s .* x) (s = sigma_s)
 *       op 2: y = x - A (s .* x)   (the operator I - K of eq. EQ:ERT Intgrl FMM)
 *
 *   Matrix, approach (M-ii) (Sec. 3.2 and Remark 3.1, selected by bit 1 of the
 *   kernel argument): the kernel is split as a(x,y) |x-y|^{1-d} with
 *   a = E / |S^{d-1}| and only the singular factor is integrated over the
 *   source cell:  A_jk = E(x_j,x_k) / |S^{d-1}| * I(x_k - x_j)  for every j, k
 *   (E(x,x) = 1), with I(t) = integral over the cell of side h centred at t of
 *   |z|^{1-d} dz.  2D: the closed form of Remark 3.1.  3D: by the divergence
 *   theorem (div(z / |z|^2) = 1 / |z|^2 in 3D) a sum over the six faces of
 *   (signed face offset) * integral over the face of |z|^-2, each face integral
 *   done in one variable in closed form (arctangent) and in the other by
 *   composite Gauss-Legendre.
 *
 *   Solve (Algorithm 1, step S.2): GMRES for (I - A S) U = A f with x0 = 0,
 *   modified Gram-Schmidt with one re-orthogonalisation, Givens rotations,
 *   stop on the recurrence estimate, then confirm with the true residual.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ---- grid description -------------------------------------------------- */

typedef struct {
    int dim;
    long n[3];
    double h;
    int kernel;            /* 0: homogeneous exp(-sigma r); 1: midpoint ray rule */
    int scheme;            /* 0: (M-iii); 1: (M-ii) */
    const double* st;      /* sigma_t, one value per cell */
    double* itab;          /* (M-ii): I(h o) for o_a = 0..n_a-1 (by symmetry |o_a|), or NULL */
} og_t;

static long og_count(const og_t* g)
{
    long N = 1;
    for (int a = 0; a < g->dim; ++a) N *= g->n[a];
    return N;
}

static void og_index(const og_t* g, long j, long i[3])
{
    i[0] = j % g->n[0];
    long r = j / g->n[0];
    i[1] = (g->dim > 1) ? r % g->n[1] : 0;
    i[2] = (g->dim > 2) ? r / g->n[1] : 0;
}

static void og_centre(const og_t* g, long j, double x[3])
{
    long i[3];
    og_index(g, j, i);
    for (int a = 0; a < 3; ++a) x[a] = (a < g->dim) ? g->h * ((double)i[a] + 0.5) : 0.0;
}

static double surface_area(int dim) { return dim == 2 ? 2.0 * OR_PI : 4.0 * OR_PI; }

/* ---- d-linear interpolation of cell-centred sigma_t (clamped) ----------- */

static double og_sigma(const og_t* g, const double p[3])
{
    long i0[3];
    double t[3];
    for (int a = 0; a < 3; ++a) { i0[a] = 0; t[a] = 0.0; }
    for (int a = 0; a < g->dim; ++a) {
        double u = p[a] / g->h - 0.5;               /* cell-centre coordinates */
        double hi = (double)(g->n[a] - 1);
        if (u < 0.0) u = 0.0;
        if (u > hi) u = hi;
        long k = (long)floor(u);
        if (k > g->n[a] - 2) k = g->n[a] - 2;
        if (k < 0) k = 0;
        i0[a] = k;
        t[a] = (g->n[a] > 1) ? u - (double)k : 0.0;
    }
    double acc = 0.0;
    int corners = 1 << g->dim;
    for (int c = 0; c < corners; ++c) {
        double w = 1.0;
        long idx[3] = {0, 0, 0};
        for (int a = 0; a < g->dim; ++a) {
            int bit = (c >> a) & 1;
            long ia = i0[a] + bit;
            if (ia > g->n[a] - 1) ia = g->n[a] - 1;  /* only when n_a == 1, where t = 0 */
            idx[a] = ia;
            w *= bit ? t[a] : 1.0 - t[a];
        }
        long j = idx[0] + g->n[0] * (idx[1] + g->n[1] * idx[2]);
        acc += w * g->st[j];
    }
    return acc;
}

/* Midpoint rule with m equal steps for the line integral of sigma_t from xa to xb. */
static double og_tau(const og_t* g, const double xa[3], const double xb[3], long m)
{
    double r2 = 0.0;
    for (int a = 0; a < g->dim; ++a) r2 += (xb[a] - xa[a]) * (xb[a] - xa[a]);
    double r = sqrt(r2);
    double s = 0.0;
    for (long k = 1; k <= m; ++k) {
        double f = ((double)k - 0.5) / (double)m;
        double p[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < g->dim; ++a) p[a] = xa[a] + f * (xb[a] - xa[a]);
        s += og_sigma(g, p);
    }
    return r / (double)m * s;
}

/* number of steps for a segment of length r: smallest m >= 1 with r/m <= h/2 */
static long og_steps_real(double r, double h)
{
    double q = ceil(r / (0.5 * h));
    return q < 1.0 ? 1 : (long)q;
}

/* the same rule for two grid points whose integer offsets square-sum to K:
 * r = h sqrt(K), so r/m <= h/2  <=>  m*m >= 4K (exact integer arithmetic). */
static long og_steps_grid(long K)
{
    long m = (long)floor(2.0 * sqrt((double)K));
    while (m * m < 4 * K) ++m;
    while (m > 1 && (m - 1) * (m - 1) >= 4 * K) --m;
    return m < 1 ? 1 : m;
}

/* G between two arbitrary points (x != y). */
static double og_kernel_points(const og_t* g, const double x[3], const double y[3])
{
    double r2 = 0.0;
    for (int a = 0; a < g->dim; ++a) r2 += (x[a] - y[a]) * (x[a] - y[a]);
    double r = sqrt(r2);
    double tau;
    if (g->kernel == 0) tau = g->st[0] * r;
    else tau = og_tau(g, x, y, og_steps_real(r, g->h));
    double rp = (g->dim == 2) ? r : r2;
    return exp(-tau) / (surface_area(g->dim) * rp);
}

/* E = exp(-tau) between collocation points j != k.  The ray is always marched
 * from the lower linear index so that E(x_j,x_k) == E(x_k,x_j) bit for bit. */
static double og_atten_cells(const og_t* g, long j, long k)
{
    long ij[3], ik[3];
    og_index(g, j, ij);
    og_index(g, k, ik);
    long K = 0;
    for (int a = 0; a < g->dim; ++a) K += (ij[a] - ik[a]) * (ij[a] - ik[a]);
    double r = g->h * sqrt((double)K);
    double tau;
    if (g->kernel == 0) {
        tau = g->st[0] * r;
    } else {
        long lo = j < k ? j : k, hi = j < k ? k : j;
        double xa[3], xb[3];
        og_centre(g, lo, xa);
        og_centre(g, hi, xb);
        long m = og_steps_grid(K);
        double s = 0.0;
        for (long q = 1; q <= m; ++q) {
            double f = ((double)q - 0.5) / (double)m;
            double p[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < g->dim; ++a) p[a] = xa[a] + f * (xb[a] - xa[a]);
            s += og_sigma(g, p);
        }
        tau = r / (double)m * s;
    }
    return exp(-tau);
}

/* G between collocation points j != k. */
static double og_kernel_cells(const og_t* g, long j, long k)
{
    long ij[3], ik[3];
    og_index(g, j, ij);
    og_index(g, k, ik);
    long K = 0;
    for (int a = 0; a < g->dim; ++a) K += (ij[a] - ik[a]) * (ij[a] - ik[a]);
    double r = g->h * sqrt((double)K);
    double rp = (g->dim == 2) ? r : r * r;
    return og_atten_cells(g, j, k) / (surface_area(g->dim) * rp);
}

/* ---- Gauss-Legendre nodes on [-1,1] by Newton's method -------------------- */

static void gauss_legendre(int n, double* x, double* w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(OR_PI * ((double)i + 0.75) / ((double)n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / (double)k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = (double)n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / (double)k;
            p0 = p1;
            p1 = p2;
        }
        dp = (double)n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* ---- (M-ii): integral of |z|^{1-d} over a cell ---------------------------- */

/* Remark 3.1's F(r, s), with 0 log 0 = 0. */
static double og_F(double r, double s)
{
    if (r == 0.0 || s == 0.0) return 0.0;
    double ar = fabs(r), as = fabs(s), q = sqrt(r * r + s * s);
    double v = ar * log(as + q) + as * log(ar + q) - ar * log(ar) - as * log(as);
    return ((r > 0) == (s > 0)) ? v : -v;
}

#define OR_FACE_PANELS 4
#define OR_FACE_NODES 20

/* integral over u in [u0,u1], v in [v0,v1] of 1 / (c^2 + u^2 + v^2), c != 0:
 * the v integral in closed form, the u integral by composite Gauss-Legendre
 * with panels split at u = 0 (where the integrand peaks). */
static double og_face(double c, double u0, double u1, double v0, double v1, const double* gx, const double* gw)
{
    double cuts[3] = {u0, u1, u1};
    int ncut = 2;
    if (u0 < 0.0 && u1 > 0.0) { cuts[1] = 0.0; cuts[2] = u1; ncut = 3; }
    double acc = 0.0;
    for (int piece = 0; piece + 1 < ncut; ++piece) {
        double a = cuts[piece], b = cuts[piece + 1];
        for (int pnl = 0; pnl < OR_FACE_PANELS; ++pnl) {
            double pa = a + (b - a) * pnl / OR_FACE_PANELS, pb = a + (b - a) * (pnl + 1) / OR_FACE_PANELS;
            for (int q = 0; q < OR_FACE_NODES; ++q) {
                double u = 0.5 * (pb - pa) * gx[q] + 0.5 * (pb + pa);
                double qq = sqrt(c * c + u * u);
                acc += 0.5 * (pb - pa) * gw[q] * (atan(v1 / qq) - atan(v0 / qq)) / qq;
            }
        }
    }
    return acc;
}

/* I(t) = integral over the cell of side h centred at t of |z|^{1-d} dz. */
static double og_cell_integral(int dim, double h, const double t[3])
{
    double gx[OR_FACE_NODES], gw[OR_FACE_NODES];
    gauss_legendre(OR_FACE_NODES, gx, gw);
    double hh = 0.5 * h;
    if (dim == 2) {
        double acc = 0.0;
        for (int i = -1; i <= 1; i += 2)
            for (int j = -1; j <= 1; j += 2) acc += (double)(i * j) * og_F(t[0] + i * hh, t[1] + j * hh);
        return acc;
    }
    /* sum over faces of (z . n) * integral_face |z|^-2; z . n is the face plane's offset */
    double acc = 0.0;
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            double off = t[a] + sgn * hh;
            if (off == 0.0) continue;
            acc += sgn * off * og_face(off, t[b] - hh, t[b] + hh, t[c] - hh, t[c] + hh, gx, gw);
        }
    }
    return acc;
}

/* Matrix entry A_jk of the selected approach (j != k). */
static double og_entry(const og_t* g, long j, long k)
{
    if (g->scheme == 0) {
        double hd = (g->dim == 2) ? g->h * g->h : g->h * g->h * g->h;
        return hd * og_kernel_cells(g, j, k);
    }
    long ij[3], ik[3];
    og_index(g, j, ij);
    og_index(g, k, ik);
    long o[3] = {0, 0, 0};
    for (int a = 0; a < g->dim; ++a) o[a] = labs(ik[a] - ij[a]);
    double I;
    if (g->itab) {
        I = g->itab[o[0] + g->n[0] * (o[1] + g->n[1] * o[2])];
    } else {
        double t[3] = {g->h * (double)o[0], g->h * (double)o[1], g->h * (double)o[2]};
        I = og_cell_integral(g->dim, g->h, t);
    }
    return og_atten_cells(g, j, k) * I / surface_area(g->dim);
}

/* (M-ii): tabulate I over the grid's offsets (I is even in every component). */
static void og_prepare(og_t* g)
{
    g->itab = NULL;
    if (g->scheme != 1) return;
    long M = g->n[0] * g->n[1] * g->n[2];
    g->itab = (double*)malloc(sizeof(double) * (size_t)M);
#pragma omp parallel for schedule(dynamic, 64)
    for (long i = 0; i < M; ++i) {
        long o0 = i % g->n[0], o1 = (i / g->n[0]) % g->n[1], o2 = i / (g->n[0] * g->n[1]);
        double t[3] = {g->h * (double)o0, g->h * (double)o1, g->h * (double)o2};
        g->itab[i] = og_cell_integral(g->dim, g->h, t);
    }
}

static void og_release(og_t* g)
{
    free(g->itab);
    g->itab = NULL;
}

#define OR_NANG 16   /* Gauss-Legendre nodes per angular patch axis */
#define OR_NRAD 10   /* Gauss-Legendre nodes per radial piece */

/* integral_0^rho E(x, x + r v) dr.  Homogeneous: closed form.  Ray rule: the
 * step count is 1 for r <= h/2 and 2 beyond (rho < h always), so the radial
 * integral is split at h/2 and each smooth piece gets Gauss-Legendre. */
static double og_radial(const og_t* g, const double x[3], const double v[3], double rho,
                        const double* gx, const double* gw)
{
    if (g->kernel == 0) {
        double s = g->st[0];
        if (s * rho < 1e-300) return rho;
        return -expm1(-s * rho) / s;
    }
    double half = 0.5 * g->h;
    double acc = 0.0;
    double a0 = 0.0, b0 = rho < half ? rho : half;
    for (int q = 0; q < OR_NRAD; ++q) {
        double r = 0.5 * (b0 - a0) * gx[q] + 0.5 * (b0 + a0);
        double p[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < g->dim; ++a) p[a] = x[a] + 0.5 * r * v[a];
        double tau = r * og_sigma(g, p);
        acc += 0.5 * (b0 - a0) * gw[q] * exp(-tau);
    }
    if (rho > half) {
        double a1 = half, b1 = rho;
        for (int q = 0; q < OR_NRAD; ++q) {
            double r = 0.5 * (b1 - a1) * gx[q] + 0.5 * (b1 + a1);
            double p1[3] = {0.0, 0.0, 0.0}, p2[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < g->dim; ++a) {
                p1[a] = x[a] + 0.25 * r * v[a];
                p2[a] = x[a] + 0.75 * r * v[a];
            }
            double tau = 0.5 * r * (og_sigma(g, p1) + og_sigma(g, p2));
            acc += 0.5 * (b1 - a1) * gw[q] * exp(-tau);
        }
    }
    return acc;
}

/* Diagonal entry A_jj: (1/|S^{d-1}|) integral over directions of the radial
 * integral up to the cell wall.  2D: eight arcs of pi/4.  3D: each of the six
 * faces split in four quadrants, parametrised by the face point (u,w) with the
 * solid-angle Jacobian (h/2)/R^3.  Each patch stays inside one octant of the
 * d-linear interpolant, so every integrand is smooth on its patch. */
static double og_self(const og_t* g, long j)
{
    if (g->scheme == 1) {
        double t0[3] = {0.0, 0.0, 0.0};
        return og_cell_integral(g->dim, g->h, t0) / surface_area(g->dim);
    }
    double ax[OR_NANG], aw[OR_NANG], rx[OR_NRAD], rw[OR_NRAD];
    gauss_legendre(OR_NANG, ax, aw);
    gauss_legendre(OR_NRAD, rx, rw);
    double x[3];
    og_centre(g, j, x);
    double half = 0.5 * g->h;
    double total = 0.0;
    if (g->dim == 2) {
        for (int arc = 0; arc < 8; ++arc) {
            double t0 = arc * OR_PI / 4.0, t1 = (arc + 1) * OR_PI / 4.0;
            for (int q = 0; q < OR_NANG; ++q) {
                double th = 0.5 * (t1 - t0) * ax[q] + 0.5 * (t1 + t0);
                double v[3] = {cos(th), sin(th), 0.0};
                double c = fabs(v[0]) > fabs(v[1]) ? fabs(v[0]) : fabs(v[1]);
                double rho = half / c;
                total += 0.5 * (t1 - t0) * aw[q] * og_radial(g, x, v, rho, rx, rw);
            }
        }
    } else {
        for (int axis = 0; axis < 3; ++axis) {
            int a1 = (axis + 1) % 3, a2 = (axis + 2) % 3;
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                for (int quad = 0; quad < 4; ++quad) {
                    double u0 = (quad & 1) ? 0.0 : -half, u1 = (quad & 1) ? half : 0.0;
                    double w0 = (quad & 2) ? 0.0 : -half, w1 = (quad & 2) ? half : 0.0;
                    for (int qa = 0; qa < OR_NANG; ++qa) {
                        double u = 0.5 * (u1 - u0) * ax[qa] + 0.5 * (u1 + u0);
                        for (int qb = 0; qb < OR_NANG; ++qb) {
                            double wv = 0.5 * (w1 - w0) * ax[qb] + 0.5 * (w1 + w0);
                            double R = sqrt(u * u + wv * wv + half * half);
                            double v[3];
                            v[axis] = sgn * half / R;
                            v[a1] = u / R;
                            v[a2] = wv / R;
                            double jac = half / (R * R * R);
                            double wq = 0.25 * (u1 - u0) * (w1 - w0) * aw[qa] * aw[qb];
                            total += wq * jac * og_radial(g, x, v, R, rx, rw);
                        }
                    }
                }
            }
        }
    }
    return total / surface_area(g->dim);
}

/* ---- exported: building blocks, for the pins in tests/ ------------------- */

static og_t og_make(int dim, const long* n, double h, int kernel, const double* st)
{
    og_t g;
    g.dim = dim;
    g.n[0] = n[0];
    g.n[1] = dim > 1 ? n[1] : 1;
    g.n[2] = dim > 2 ? n[2] : 1;
    g.h = h;
    g.kernel = kernel & 1;
    g.scheme = (kernel >> 1) & 1;
    g.st = st;
    g.itab = NULL;
    return g;
}

double oracle_cell_integral(int dim, double h, const double* t)
{
    double tt[3] = {t[0], t[1], dim > 2 ? t[2] : 0.0};
    return og_cell_integral(dim, h, tt);
}

double oracle_entry(int dim, const long* n, double h, int kernel, const double* st, long j, long k)
{
    og_t g = og_make(dim, n, h, kernel, st);
    return j == k ? og_self(&g, j) : og_entry(&g, j, k);
}

double oracle_sigma_interp(int dim, const long* n, double h, const double* st, const double* p)
{
    og_t g = og_make(dim, n, h, 1, st);
    double q[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; ++a) q[a] = p[a];
    return og_sigma(&g, q);
}

double oracle_tau(int dim, const long* n, double h, const double* st,
                  const double* xa, const double* xb, long m)
{
    og_t g = og_make(dim, n, h, 1, st);
    double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) { a[k] = xa[k]; b[k] = xb[k]; }
    return og_tau(&g, a, b, m);
}

long oracle_steps_real(double r, double h) { return og_steps_real(r, h); }
long oracle_steps_grid(long K) { return og_steps_grid(K); }

double oracle_kernel_points(int dim, const long* n, double h, int kernel, const double* st,
                            const double* x, const double* y)
{
    og_t g = og_make(dim, n, h, kernel, st);
    double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) { a[k] = x[k]; b[k] = y[k]; }
    return og_kernel_points(&g, a, b);
}

double oracle_kernel_cells(int dim, const long* n, double h, int kernel, const double* st,
                           long j, long k)
{
    og_t g = og_make(dim, n, h, kernel, st);
    return og_kernel_cells(&g, j, k);
}

double oracle_self_cell(int dim, const long* n, double h, int kernel, const double* st, long j)
{
    og_t g = og_make(dim, n, h, kernel, st);
    return og_self(&g, j);
}

/* all diagonal entries (homogeneous: one value repeated) */
void oracle_diag(int dim, const long* n, double h, int kernel, const double* st,
                 double* d, int nthreads)
{
    og_t g = og_make(dim, n, h, kernel, st);
    long N = og_count(&g);
    if (g.kernel == 0 || g.scheme == 1) {
        double v = og_self(&g, 0);
        for (long j = 0; j < N; ++j) d[j] = v;
        return;
    }
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (long j = 0; j < N; ++j) d[j] = og_self(&g, j);
}

/* dense matrix A (row-major, N x N) -- small N only */
void oracle_matrix(int dim, const long* n, double h, int kernel, const double* st,
                   const double* diag, double* A, int nthreads)
{
    og_t g = og_make(dim, n, h, kernel, st);
    og_prepare(&g);
    long N = og_count(&g);
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
    for (long j = 0; j < N; ++j)
        for (long k = 0; k < N; ++k)
            A[j * N + k] = (j == k) ? diag[j] : og_entry(&g, j, k);
    og_release(&g);
}

/* ---- the apply ------------------------------------------------------------ */

/* One row of the apply for every right-hand side.  x is N x nrhs column-major;
 * each entry A_jk is formed once and applied to all columns; the sum over k
 * runs in index order with Neumaier compensation per column. */
static void og_row(const og_t* g, const double* ss, int op, const double* x, long N, int nrhs,
                   const double* diag, long j, double* out /* nrhs, stride ostride */, long ostride)
{
    double* sum = (double*)calloc((size_t)nrhs * 2, sizeof(double));
    double* comp = sum + nrhs;
    for (long k = 0; k < N; ++k) {
        double a = (k == j) ? diag[j] : og_entry(g, j, k);
        double sk = (op == 0) ? 1.0 : ss[k];
        for (int b = 0; b < nrhs; ++b) {
            double term = a * (sk * x[(long)b * N + k]);
            double t = sum[b] + term;
            if (fabs(sum[b]) >= fabs(term)) comp[b] += (sum[b] - t) + term;
            else comp[b] += (term - t) + sum[b];
            sum[b] = t;
        }
    }
    for (int b = 0; b < nrhs; ++b) {
        double y = sum[b] + comp[b];
        out[(long)b * ostride] = (op == 2) ? x[(long)b * N + j] - y : y;
    }
    free(sum);
}

void oracle_apply(int dim, const long* n, double h, int kernel, const double* st,
                  const double* ss, const double* diag, int op,
                  const double* x, double* y, int nrhs, int nthreads)
{
    og_t g = og_make(dim, n, h, kernel, st);
    og_prepare(&g);
    long N = og_count(&g);
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (long j = 0; j < N; ++j) og_row(&g, ss, op, x, N, nrhs, diag, j, y + j, N);
    og_release(&g);
}

/* rows[i] of the apply, i < nrows; y_rows is nrows x nrhs column-major.
 * diag may be NULL: the needed diagonal entries are then computed here. */
void oracle_apply_rows(int dim, const long* n, double h, int kernel, const double* st,
                       const double* ss, const double* diag, int op,
                       const double* x, const long* rows, long nrows,
                       double* y_rows, int nrhs, int nthreads)
{
    og_t g = og_make(dim, n, h, kernel, st);
    og_prepare(&g);
    long N = og_count(&g);
    (void)nthreads;
    /* one row per scheduling chunk: a row costs O(N) kernel evaluations, so a few
     * sampled rows still spread over every thread */
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (long i = 0; i < nrows; ++i) {
        long j = rows[i];
        double dj;
        const double* dptr = diag;
        double* tmp = NULL;
        if (!diag) {
            dj = og_self(&g, j);
            tmp = (double*)calloc((size_t)N, sizeof(double));
            tmp[j] = dj;
            dptr = tmp;
        }
        og_row(&g, ss, op, x, N, nrhs, dptr, j, y_rows + i, nrows);
        free(tmp);
    }
    og_release(&g);
}

/* ---- GMRES (Algorithm 1, step S.2) --------------------------------------- */

typedef struct {
    int iters;          /* Arnoldi steps taken */
    int matvecs;        /* applications of I - A S (incl. true-residual checks) */
    int converged;
    int restarts;
    double rel_resid_est;
    double rel_resid_true;
} oracle_gmres_info;

static double dotp(const double* a, const double* b, long N)
{
    double s = 0.0, c = 0.0;
    for (long i = 0; i < N; ++i) {
        double term = a[i] * b[i];
        double t = s + term;
        if (fabs(s) >= fabs(term)) c += (s - t) + term;
        else c += (term - t) + s;
        s = t;
    }
    return s + c;
}

/* Solve (I - A S) U = phi, phi = A f.  One right-hand side.  restart <= 0
 * means unrestarted (Krylov space up to maxit).  Returns 0 on convergence. */
int oracle_gmres(int dim, const long* n, double h, int kernel, const double* st,
                 const double* ss, const double* diag, const double* f, double* U,
                 double* phi_out, double tol, int maxit, int restart, int nthreads,
                 oracle_gmres_info* info)
{
    og_t g = og_make(dim, n, h, kernel, st);
    long N = og_count(&g);
    int m = (restart > 0 && restart < maxit) ? restart : maxit;
    double* phi = (double*)malloc(sizeof(double) * N);
    double* r = (double*)malloc(sizeof(double) * N);
    double* w = (double*)malloc(sizeof(double) * N);
    double* V = (double*)malloc(sizeof(double) * N * (size_t)(m + 1));
    double* H = (double*)calloc((size_t)(m + 1) * m, sizeof(double));
    double* cs = (double*)malloc(sizeof(double) * m);
    double* sn = (double*)malloc(sizeof(double) * m);
    double* gv = (double*)malloc(sizeof(double) * (m + 1));
    double* yv = (double*)malloc(sizeof(double) * m);
    oracle_gmres_info inf;
    memset(&inf, 0, sizeof(inf));

    oracle_apply(dim, n, h, kernel, st, ss, diag, 0, f, phi, 1, nthreads);
    if (phi_out) memcpy(phi_out, phi, sizeof(double) * N);
    double beta0 = sqrt(dotp(phi, phi, N));
    for (long i = 0; i < N; ++i) U[i] = 0.0;
    int status = 1;
    if (beta0 == 0.0) {
        inf.converged = 1;
        status = 0;
        goto done;
    }
    memcpy(r, phi, sizeof(double) * N);
    for (int cycle = 0;; ++cycle) {
        double beta = sqrt(dotp(r, r, N));
        inf.rel_resid_true = beta / beta0;
        if (beta / beta0 <= tol) { inf.converged = 1; status = 0; break; }
        if (inf.iters >= maxit || cycle > 1000) break;
        inf.restarts = cycle;
        for (long i = 0; i < N; ++i) V[i] = r[i] / beta;
        memset(H, 0, sizeof(double) * (size_t)(m + 1) * m);
        for (int i = 0; i <= m; ++i) gv[i] = 0.0;
        gv[0] = beta;
        int k = 0;
        for (int j = 0; j < m && inf.iters < maxit; ++j) {
            oracle_apply(dim, n, h, kernel, st, ss, diag, 2, V + (long)j * N, w, 1, nthreads);
            inf.matvecs++;
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = 0; i <= j; ++i) {
                    double hij = dotp(V + (long)i * N, w, N);
                    H[i * m + j] += hij;
                    for (long q = 0; q < N; ++q) w[q] -= hij * V[(long)i * N + q];
                }
            }
            double hn = sqrt(dotp(w, w, N));
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], b = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * b;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            double a = H[j * m + j], b = H[(j + 1) * m + j];
            double den = hypot(a, b);
            cs[j] = den == 0.0 ? 1.0 : a / den;
            sn[j] = den == 0.0 ? 0.0 : b / den;
            H[j * m + j] = den;
            H[(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            inf.iters++;
            k = j + 1;
            inf.rel_resid_est = fabs(gv[j + 1]) / beta0;
            if (inf.rel_resid_est <= tol || hn == 0.0) break;
            for (long q = 0; q < N; ++q) V[(long)(j + 1) * N + q] = w[q] / hn;
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = gv[i];
            for (int c = i + 1; c < k; ++c) s -= H[i * m + c] * yv[c];
            yv[i] = s / H[i * m + i];
        }
        for (int i = 0; i < k; ++i)
            for (long q = 0; q < N; ++q) U[q] += yv[i] * V[(long)i * N + q];
        /* true residual r = phi - (I - A S) U */
        oracle_apply(dim, n, h, kernel, st, ss, diag, 2, U, w, 1, nthreads);
        inf.matvecs++;
        for (long q = 0; q < N; ++q) r[q] = phi[q] - w[q];
    }
done:
    if (info) *info = inf;
    free(phi); free(r); free(w); free(V); free(H); free(cs); free(sn); free(gv); free(yv);
    return status;
}
