/*
 * ertvie.h -- C ABI of the MI355X volume-integral solver for isotropic
 * radiative transport (Ren, Zhang, Zhong, "A fast algorithm for radiative
 * transport in isotropic media").
 *
 * Problem (Sec. 2): on a uniform cell-centred grid, the angular density U
 * solves the second-kind integral equation (I - K) U = phi with
 * K u = G(sigma_s u) and phi = G f (eq. EQ:ERT Intgrl U / EQ:ERT Intgrl FMM,
 * Algorithm 1 step S.1 "analytically"), where G is the integral operator with
 * the transport kernel
 *
 *     G(x,y) = exp(-tau(x,y)) / (|S^{d-1}| |x-y|^{d-1}),   |S^1| = 2 pi, |S^2| = 4 pi,
 *
 * and tau(x,y) the line integral of sigma_t along the segment (eq. EQ:Kernel
 * without the sigma_s factor).  The discrete operator is the collocation
 * matrix of Sec. 3.2, approach (M-iii): A_jk = h^d G(x_j,x_k) for j != k and
 * an explicitly integrated singular diagonal A_jj = (1/|S^{d-1}|) * integral
 * over the own cell of E(x_j,y)/|x_j-y|^{d-1} dy.
 *
 * Grid convention: dim 2 or 3, n[a] cells per axis, side h, domain
 * [0, n[a] h]; cell (i0,i1,i2) has centre h (i + 1/2) and linear index
 * j = i0 + n0 (i1 + n1 i2) (x fastest).  N = product of n[a].
 * Vectors are FP64, N x nrhs, column-major (column b starts at b*N).
 *
 * Memory ownership: sigma_t / sigma_s passed to ert_vie_plan are HOST arrays
 * that the plan copies; every vector passed to apply/solve is a DEVICE
 * pointer owned by the caller (e.g. a torch tensor's data_ptr()).  The plan
 * owns every internal buffer (grids, expansions, operators, caches,
 * workspaces) and frees them in ert_vie_destroy.  All device work of a plan
 * is ordered on the HIP stream given at plan time; apply returns without
 * synchronising, solve synchronises (it needs scalars on the host).
 * A plan is not thread-safe: one host thread at a time per plan.
 *
 * Errors: every call returns an ert_status; nothing throws across the ABI.
 * Invalid arguments return ERT_EINVAL and leave outputs untouched.
 */
#ifndef ERTVIE_H
#define ERTVIE_H

#include <stddef.h>

#if defined(__GNUC__) || defined(__clang__)
#define ERT_API __attribute__((visibility("default")))
#else
#define ERT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ert_vie_plan_s* ert_vie_plan_t;
typedef struct ert_net_s* ert_net_t;      /* learned preconditioner (see the end of this file) */

typedef enum {
    ERT_OK = 0,
    ERT_EINVAL = -1,        /* bad argument: dim, sizes, h, coefficients, nrhs, null pointer */
    ERT_ENOMEM = -2,        /* device or host allocation failed */
    ERT_EDEVICE = -3,       /* a HIP call failed (no device, launch error, ...) */
    ERT_ENOCONV = -4,       /* solve stopped at max_iter; best iterate and info are written */
    ERT_EUNSUPPORTED = -5   /* valid request this build does not provide */
} ert_status;

typedef enum {
    /* tau = sigma_t |x-y| with constant sigma_t (eq. EQ:Kernel Cons); every
     * sigma_t value must be equal */
    ERT_K_HOMOGENEOUS = 0,
    /* tau by the midpoint rule with m = smallest integer such that |x-y|/m <= h/2,
     * sampling the d-linear interpolant of the cell-centred sigma_t with each
     * coordinate clamped to [h/2, n_a h - h/2] (Sec. 4.2: a local second-order
     * rule for the line integral of gridded sigma_t) */
    ERT_K_RAY_MIDPOINT = 1
} ert_kernel;

typedef enum {
    ERT_DIRECT = 0,   /* dense O(N^2) summation of the collocation matrix */
    ERT_FMM = 1       /* Chebyshev-interpolation fast multipole method (Sec. 3.3) */
} ert_method;

typedef enum {
    ERT_FP64 = 0,     /* everything in FP64 */
    ERT_FP32 = 1,     /* near and far field in FP32, self term and assembly in FP64 */
    ERT_BF16X3 = 2    /* as FP32, with the far-field translations (Sec. 3.3 eq. EQ: M2L) as
                         split-BF16x3 MFMA products accumulated in FP32, in homogeneous media
                         (shared per-offset operators) and heterogeneous ones (cached per-pair
                         matrices, for any number of right-hand sides); near field in FP32 */
} ert_prec;

typedef enum {
    ERT_OP_G = 0,     /* y = A x             (phi = A f: Algorithm 1, step S.1) */
    ERT_OP_GS = 1,    /* y = A (sigma_s x)   (the paper's K applied to x) */
    ERT_OP_A = 2      /* y = x - A (sigma_s x)  (the operator I - K of step S.2) */
} ert_op;

typedef enum {
    ERT_PRECOND_NONE = 0,
    ERT_PRECOND_FFT = 1,        /* FFT-based preconditioner of the mean medium (Sec. 4.4) */
    ERT_PRECOND_DIFFUSION = 2   /* diffusion approximation, multigrid V-cycles (Sec. 4.4) */
} ert_precond;

typedef struct {
    int dim;          /* 2 or 3 */
    int n[3];         /* cells per axis (n[2] ignored for dim 2), each >= 1, N >= 2 */
    double h;         /* cell side, > 0 */
    int kernel;       /* ert_kernel */
    int method;       /* ert_method used by ert_vie_apply and the solver */
    int prec;         /* ert_prec used by ert_vie_apply and the solver */
    int cheb_n;       /* FMM: Chebyshev nodes per axis (Sec. 3.3, n); 0 -> 8; 2..8 */
    int leaf;         /* FMM: cells per leaf-box side; 0 -> 8; 1..8 */
    int nrhs_max;     /* largest nrhs later passed to apply/solve; 0 -> 1 */
    int scheme;       /* discretisation of the integral operator (Sec. 3.2):
                         0 (M-iii): A_jk = h^d G(x_j, x_k) for j != k, A_jj the singular
                           self-cell integral of E / (|S^{d-1}| r^{d-1}) (polar quadrature);
                         1 (M-ii), with Remark 3.1's smooth kernel: A_jk = E(x_j, x_k)
                           / |S^{d-1}| * integral over the cell of side h centred at x_k - x_j
                           of |z|^{1-d} dz, for every j, k (E(x, x) = 1).  The FMM evaluates
                           the same kernel at its interpolation nodes.  Homogeneous FMM needs
                           leaf^dim to be a multiple of 32 */
    double svd_tol;   /* FMM, homogeneous media: relative singular-value cutoff of the
                         compressed far-field translations (shared orthonormal basis per
                         level from the SVD of all translation matrices); 0 -> 1e-6
                         (rank 256 of 512 at n = 8), < 0 -> no compression.  A looser cutoff
                         lowers the rank (1e-5: rank 160) and the error grows with the number
                         of compressed levels */
    int inner_cheb_n; /* FMM: Chebyshev nodes per axis of the FP32 and BF16x3 applies (the
                         inner operator of mixed solves); 0 -> cheb_n; 2..8.  The far-field
                         translations cost n^(2d) per box pair, so a lower order makes the inner
                         solves cheaper; the FP64 outer residual keeps the accuracy */
    int inner_near16; /* heterogeneous media, FMM: 1 -> the FP32 and BF16x3 applies (the inner
                         operator of mixed solves) read the near-field kernel cache rounded to
                         BF16 (2 bytes per value instead of 4; relative rounding <= 2^-9 per
                         value).  The cache always holds each FP32 value as two 16-bit planes,
                         the high half rounded to BF16 and the exact remainder: FP64 applies,
                         and FP32 applies without this option, read both and rebuild the FP32
                         value exactly.  0 or 1 */
    int form[2];      /* FMM, homogeneous media: execution form of the box-offset products,
                         [0] for the near field and [1] for the far-field translations.
                         0 -> timed on first use per right-hand-side count (the fastest of
                         the forms that apply is kept); f + 1 -> always form f:
                         0 target-tile GEMM, 1 offset-stationary 32x16 tiles, 2 32x64,
                         3 16x64, 4 (FP32) 64x16 tiles with the source columns staged in LDS,
                         5 (FP32, reduction length <= 252) 64-column tiles over all rows with
                         the source columns staged in LDS
                         (a form that does not apply to a product leaves it to the timing).
                         Fixed forms make runs reproducible bit for bit across plans */
    double far_cache_gb; /* heterogeneous media, FMM: device memory, in GB (1e9 bytes), that
                         the plan's stored far-field translation matrices (of every order the
                         plan builds) may take; 0 -> 90 % of the device memory free when a level
                         is built.  A level that does not fit keeps the box pairs that fit
                         stored; every apply rebuilds the others by the same ray march (Sec.
                         4.2's kernel evaluations), in chunks of whole pairs written to a
                         scratch buffer (a sixteenth of the level's room, at least one pair,
                         at most 2 GB) and used right away.  The results are those of a fully
                         stored level bit for bit; each apply then costs the rebuilt pairs' ray
                         marches (seconds at 128^3 instead of milliseconds).  The near-field
                         blocks are always stored (ERT_ENOMEM when they do not fit).  >= 0 and
                         finite */
} ert_vie_opts;

typedef struct {
    double tol;       /* stop when ||phi - (I - K) U||_2 <= tol ||phi||_2 (true residual); 0 -> 1e-8 */
    int max_iter;     /* total Arnoldi steps (all restarts / inner solves); 0 -> 500 */
    int restart;      /* Krylov dimension per cycle; 0 -> unrestarted (max_iter) */
    int mixed;        /* 1: iterative refinement -- FP64 outer residual with the plan's
                         FP64 operator, inner GMRES on the FP32 operator */
    double inner_tol; /* mixed: relative tolerance of each inner solve; 0 -> 1e-5 */
    int rhs_is_phi;   /* 1: the f argument already holds phi (skip step S.1) */
    int block;        /* 1: block GMRES -- the nrhs columns share one block Krylov space and
                         every operator application is one batched apply (0: column by column);
                         with restart = 0 the block basis is capped at 4 GiB */
    int precond_steps;/* with precond: Arnoldi steps per preconditioned correction; 0 -> 10 */
    int history_max;  /* columns of `history` (0: no history) */
    int precond_kind; /* ert_precond: right-precondition every GMRES solve (the inner solves
                         with `mixed`, each correction with `precond`) by a fixed preconditioner
                         M, in flexible GMRES: ERT_PRECOND_FFT (ert_vie_fft_precond) or
                         ERT_PRECOND_DIFFUSION (ert_vie_diff_precond).  With `precond` the
                         network acts on M's output, z_j = net(M v_j), and the fallback of a
                         rejected step keeps M; with `block`, block GMRES on (I - K) M with
                         U = M Y.  ERT_PRECOND_NONE (0): none */
    ert_net_t precond;/* NULL, or a learned right preconditioner (dim 3) on the plan's grid or on
                         that grid coarsened by one integer factor f on every axis (the network
                         then sees the cell averages of the vector and of the media over f^3
                         blocks, and its correction is extended piecewise constant:
                         z = v + P(s y(R v))): the solve
                         becomes a refinement loop.  Each step solves (I - K) d = r by flexible
                         GMRES with z_j = net(v_j) (inner operator: FP32 with `mixed`, else the
                         plan's), and is kept only if the true residual phi - (I - K)(U + d),
                         taken with the FP64 operator (phi = A f in FP64 as well), is smaller
                         than before; otherwise plain GMRES with the same budget replaces it,
                         and when that step does not lower the residual either the solve stops
                         with ERT_ENOCONV.  rel_resid_true is that FP64 residual.
                         Not combined with `block`. */
    double* history;  /* NULL, or DEVICE N x 2 history_max FP64: the plain solve (no mixed,
                         block or precond) of the first column stores, at the start of every
                         GMRES cycle k < history_max, the iterate U_k in column 2k and its
                         residual phi - (I - K) U_k in column 2k + 1 (training pairs for the
                         preconditioner: the correction of U_k is U - U_k) */
} ert_solve_opts;

typedef struct {
    int iters;            /* Arnoldi steps taken (inner steps for mixed) */
    int matvecs;          /* operator applications, including phi and true residuals */
    int converged;        /* 1 if the true relative residual met tol */
    int restarts;         /* GMRES cycles after the first (refinement steps for mixed) */
    double rel_resid_est; /* last Arnoldi estimate */
    double rel_resid_true;/* ||phi - (I - K) U|| / ||phi|| with the plan's operator */
    double t_solve;       /* seconds, host wall clock, phi included (FMM data built before) */
    int rejected;         /* preconditioned corrections rejected by the residual check */
    int precond_applies;  /* network applications */
    int history_count;    /* (iterate, residual) pairs written to opts->history */
    double t_setup;       /* seconds this call spent building FMM data for its operators
                             (first use of a precision: the inner operator of mixed solves,
                             or an FMM not yet built by an apply or ert_vie_fmm_info); not
                             part of t_solve */
} ert_solve_info;

/* Build a plan: validate and copy the media, place the collocation grid and
 * integrate the singular diagonal (FP64, on the device).  FMM data (tree,
 * translation operators, caches) are built on first FMM use of each precision.
 *   opts     : host pointer, read only.
 *   sigma_t  : host, N values, finite and > 0 (total attenuation, Sec. 2 mu).
 *   sigma_s  : host, N values, 0 <= sigma_s <= sigma_t (1 + 1e-12) (scattering, mu_s;
 *              absorption mu_a = sigma_t - sigma_s >= 0).
 *   hip_stream: hipStream_t for all work of the plan (NULL = default stream).
 *   out      : receives the plan handle.
 * Returns ERT_EINVAL for dim not 2/3, n < 1, N < 2, h <= 0, bad coefficients,
 * non-constant sigma_t with ERT_K_HOMOGENEOUS, cheb_n outside 2..8 or scheme not 0/1. */
ERT_API ert_status ert_vie_plan(const ert_vie_opts* opts, const double* sigma_t, const double* sigma_s,
                        void* hip_stream, ert_vie_plan_t* out);

/* y = op(x) with the plan's method and precision (Sec. 3.2 eq. EQ: LINEAR SYSTEM;
 * FMM per Sec. 3.3).  x, y: device, N x nrhs column-major FP64, must not
 * overlap.  1 <= nrhs <= nrhs_max.  Stream-ordered, asynchronous. */
ERT_API ert_status ert_vie_apply(ert_vie_plan_t plan, int op, const double* x, double* y, int nrhs);

/* As ert_vie_apply with an explicit method (ert_method) and precision (ert_prec). */
ERT_API ert_status ert_vie_apply_ex(ert_vie_plan_t plan, int op, int method, int prec,
                            const double* x, double* y, int nrhs);

/* Algorithm 1 steps S.1-S.2: phi = A f, then GMRES (x0 = 0) for (I - K) U = phi.
 *   f, U : device, N x nrhs column-major FP64 (solved one after another, or together with
 *          opts->block; a block solve reports the worst column in info).
 *   opts : host, may be NULL for defaults.  info: host, may be NULL (last column's info).
 * Returns ERT_ENOCONV when max_iter is reached first; U then holds the best iterate. */
ERT_API ert_status ert_vie_solve(ert_vie_plan_t plan, const double* f, double* U, int nrhs,
                         const ert_solve_opts* opts, ert_solve_info* info);

/* FFT-based preconditioner (Sec. 4.4, eqs. EQ: FFT and EQ:SOL FFT): the solve
 * of the same equation in the constant medium sigma_t_mean, sigma_s_mean (the
 * means of the plan's coefficients over the cells), done by FFT on a periodic
 * grid of m_a cells per axis with the residual extended by zeros and the
 * result restricted to the grid:
 *   z = P IDFT( DFT(E r) / c ),   c = 1 - sigma_s_mean DFT(w),
 * w[i] = h^d G(h o(i)) for the constant-medium kernel G at the periodic offset
 * o(i)_a = i_a (i_a <= m_a / 2) or i_a - m_a, and w[0] = the self-cell integral
 * of that medium (the diagonal of its M-iii matrix).  m_a is the smallest
 * integer >= 2 n_a with no prime factor above 7 (2 n_a, the paper's [0, 2]^d,
 * whenever 2 n_a has none), at most 1024.  For a constant medium, P C E with C
 * the periodic operator of symbol c is exactly the plan's I - K.
 * Arithmetic: the symbol is computed in FP64 (kernel array and its DFT) and
 * kept as 1/c in FP32 on the half-grid of distinct values (c is even along every
 * axis); the per-residual transforms are FP32 with FP32 twiddles from FP64
 * tables.  Built on the plan's stream on first use (symbol plus work buffers:
 * about 24 bytes per periodic cell for the build, 8 per cell of the
 * n_2 x m_1 x (m_0/2 + 1) work grid after it). */
typedef struct {
    int m[3];             /* periodic grid, cells per axis (1 beyond dim) */
    double sigma_t_mean;  /* the constant medium */
    double sigma_s_mean;
    double self_cell;     /* diagonal of the constant medium's matrix */
    double symbol_min;    /* extremes of c (positive for sigma_s <= sigma_t) */
    double symbol_max;
    long bytes;           /* device memory held by the preconditioner */
} ert_fft_info;

/* z = M r for nrhs columns: r, z device N x nrhs column-major FP64 (may be the
 * same buffer), 1 <= nrhs <= nrhs_max.  Stream-ordered, asynchronous after the
 * first call.  ERT_EUNSUPPORTED when a period would exceed 1024 or the symbol is
 * not positive. */
ERT_API ert_status ert_vie_fft_precond(ert_vie_plan_t plan, const double* r, double* z, int nrhs);

/* Build (if needed) and describe the FFT-based preconditioner (host struct). */
ERT_API ert_status ert_vie_fft_info(ert_vie_plan_t plan, ert_fft_info* info);

/* Algorithm 1 step S.3: the angular solution Phi(x_j, v_k) from U, i.e. the
 * scattering-free transport equation v . grad Phi + sigma_t Phi = Q with
 * Q = sigma_s U + f and no inflow, solved along characteristics.  From each cell
 * centre the ray is followed backwards to the boundary of [0, n_a h]^dim in
 * m = ceil(s / (h/2) (1 - 1e-12)) equal steps; on each step sigma_t and Q take their values at
 * the step midpoint (d-linear interpolation of the cell values, clamped to the
 * cell-centre box, as the kernel's ray rule does) and the step is integrated
 * exactly for those constants, so a constant medium and source give
 * Q (1 - exp(-sigma_t s)) / sigma_t.  The angular average of Phi approximates U.
 *   U, f : device, N values FP64; either may be NULL (taken as zero).
 *   dirs : host, ndir x dim unit vectors (|v| = 1 within 1e-10), row per direction.
 *   phi  : device, N x ndir column-major FP64 (column k for dirs[k]).
 * FP64 throughout; stream-ordered, synchronises before returning (it frees its
 * scratch).  ERT_EINVAL for a non-unit or non-finite direction or ndir < 1. */
ERT_API ert_status ert_vie_transport(ert_vie_plan_t plan, const double* U, const double* f, const double* dirs,
                                     int ndir, double* phi);

/* ert_vie_transport without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results (bit for bit) and errors as
 * ert_vie_transport, plus ERT_EINVAL when 2 N + dim * ndir exceeds 4,259,840
 * doubles (32.5 MiB; e.g. N = 128^3 with up to 21,845 directions in 3D).
 * Its work buffer (the interleaved sigma_t and Q of every cell, and the
 * directions) is one static device array per GPU, held from the first call on
 * that GPU until the process ends and shared by every call on it: calls that
 * overlap on one GPU (plans on different streams, several host threads) race
 * on it and must be serialised by the caller.  Runs on the plan's device and
 * stream and synchronises that stream before returning. */
ERT_API ert_status ert_vie_transport_noalloc(ert_vie_plan_t plan, const double* U, const double* f,
                                             const double* dirs, int ndir, double* phi);

/* The learned right preconditioner as the solver applies it (ert_solve_opts.precond): z =
 * M(r) for one column on the plan's media, with the network on the plan's grid or on that
 * grid coarsened by one integer factor f (cell averages of r and the media over f^3 blocks
 * in, the correction extended piecewise constant out).  r, z: device N FP64 (may not
 * overlap).  Stream-ordered on the plan's stream.  Not part of the paper's method. */
ERT_API ert_status ert_vie_net_apply(ert_vie_plan_t plan, ert_net_t net, const double* r, double* z);

/* Cell averages over blocks of factor^3 cells (3D grids whose sides are multiples of
 * factor): y[c] = factor^-3 * sum of x over the cells of coarse cell c, the coarse grid
 * (n_a / factor per axis) in the same x-fastest order; the restriction a coarse-grid
 * learned preconditioner applies to its inputs (not part of the paper's method).
 * x: device N x nrhs, y: device (N / factor^3) x nrhs, column-major FP64; nrhs >= 1
 * (any count: no plan buffer is used).  Stream-ordered, asynchronous.  ERT_EUNSUPPORTED
 * in 2D. */
ERT_API ert_status ert_vie_restrict(ert_vie_plan_t plan, int factor, const double* x, double* y, int nrhs);

/* Diffusion preconditioner (Sec. 4.4, eq. EQ:DA).  The diffusion approximation
 *   -div(D grad U) + mu_a U = f,  U + l dU/dn = 0 on the boundary,
 *   D = 1 / (dim sigma_t),  mu_a = sigma_t - sigma_s,  l = 2 / (dim sigma_t),
 * models f -> U = (I - K)^{-1} A f, so (I - K)^{-1} = I + (I - K)^{-1} A S is
 * approximated by  z = M r = r + L^{-1} (sigma_s r).  L: cell-centred finite
 * differences per unit volume on the plan's grid (harmonic-mean face
 * coefficients; each boundary face adds 2 D / (h (h + 2 l)) from the Robin
 * condition with the boundary value extrapolated from the cell centre).
 * L^{-1}: two multigrid V-cycles from zero (levels by halving every axis down to
 * 4 cells per axis, coarse coefficients averaged over the children, red-black
 * Gauss-Seidel with 2 + 2 sweeps, averaging restriction, constant prolongation,
 * 60 sweeps on the coarsest level).  FP64.  r, z: device N x nrhs (may be the
 * same buffer), 1 <= nrhs <= nrhs_max.  Built on the plan's stream on first use
 * (about 9 vectors of N doubles over all levels).  The approximation holds for
 * optically thin cells (sigma_t h well below 1) in optically thick domains. */
ERT_API ert_status ert_vie_diff_precond(ert_vie_plan_t plan, const double* r, double* z, int nrhs);

/* Stages of one FMM apply, for ert_vie_profile. */
typedef enum {
    ERT_STAGE_GATHER = 0,   /* weights into leaf-major order */
    ERT_STAGE_NEAR = 1,     /* near field over neighbouring leaves (P2P) */
    ERT_STAGE_P2M = 2,
    ERT_STAGE_M2M = 3,
    ERT_STAGE_M2L = 4,      /* far-field translations (Sec. 3.3 eq. EQ: M2L) */
    ERT_STAGE_L2L = 5,
    ERT_STAGE_L2P = 6,
    ERT_STAGE_ASSEMBLE = 7, /* scaling, self term, I - K */
    ERT_STAGE_DIRECT = 8,   /* dense apply */
    ERT_STAGE_BASIS = 9,    /* change of basis of the compressed translations */
    ERT_STAGE_REDUCE = 10,  /* fixed-order sums of staged pair products (offset-stationary form) */
    ERT_NSTAGES = 11
} ert_stage;

/* Shape of a plan's FMM for one precision (built on first use). */
typedef struct {
    int levels;           /* leaf level L of the tree; far field on levels 2..L */
    int leaf;             /* cells per leaf side */
    int cheb_n;           /* Chebyshev nodes per axis */
    int nodes;            /* nodes per box (cheb_n^dim) */
    int nodes_padded;     /* nodes per box as stored (multiple of 32) */
    int rank[16];         /* per level: compressed translation rank as stored, 0 = uncompressed */
    long far_pairs[16];   /* per level: (target, source) box pairs of the interaction lists */
    long near_pairs;      /* point pairs of the near field (self pairs excluded) */
    int form_near;        /* execution form of the homogeneous near-field product for one
                             right-hand side: -1 not tuned yet / not a box-offset product,
                             0 target-tile GEMM, 1 offset-stationary 32x16 tiles, 2 32x64, 3 16x64,
                             4 (FP32) 64x16 tiles with the source columns staged in LDS,
                             5 (FP32) 64-column tiles over all rows, source columns in LDS */
    int form_far[16];     /* per level: the same for the far-field translations */
    long near_table;      /* homogeneous media, leaf a power of two >= 4: the offset-stationary
                             near-field products read one table of (4 leaf - 1)^dim values over
                             cell offsets (this count) instead of the 3^dim explicit blocks;
                             0 = no table */
    int far_rebuilt[16];  /* heterogeneous media, per level: 1 when the level's translation
                             matrices are not stored and every apply rebuilds them
                             (ert_vie_opts.far_cache_gb) */
    double cache_bytes;   /* heterogeneous media: device bytes of the kernel caches this
                             precision's operator uses (near blocks, stored translation
                             matrices, scratch and corner table of rebuilt levels) */
} ert_fmm_info;

/* Device timing of applies by stage, with HIP events recorded on the plan's
 * stream around every kernel launch of a stage.
 *   enable = 1: clear the totals and start recording; 0: stop recording.
 *   stage_ms / stage_launches (host, ERT_NSTAGES entries each, may be NULL):
 *   receive the totals recorded so far (synchronises the stream).
 * Recording adds an event pair per launch; leave it off for timed runs. */
ERT_API ert_status ert_vie_profile(ert_vie_plan_t plan, int enable, double* stage_ms, int* stage_launches);

/* Build (if needed) the FMM of precision `prec` and describe it (host struct). */
ERT_API ert_status ert_vie_fmm_info(ert_vie_plan_t plan, int prec, ert_fmm_info* info);

/* Copy the diagonal A_jj (N values, FP64) to host memory `d` (synchronises). */
ERT_API ert_status ert_vie_diag(ert_vie_plan_t plan, double* d);

/* Number of collocation points N of a plan, or -1 for a null plan. */
ERT_API long ert_vie_size(ert_vie_plan_t plan);

/* Release the plan and everything it owns.  NULL is a no-op. */
ERT_API void ert_vie_destroy(ert_vie_plan_t plan);

/* Text describing the most recent failure in this thread (the failing HIP call
 * and its error string, or the argument check that rejected a call); "" if none.
 * The pointer stays valid until the next failing call in the same thread. */
ERT_API const char* ert_vie_last_error(void);

/* Static, human-readable text for a status code. */
ERT_API const char* ert_vie_strerror(ert_status status);

/* Diagnostic, for stating the attainable HBM read rate beside the published
 * peak (the cached-pair products are HBM-bound): streams the first
 * floor(bytes / piece) * piece bytes of the DEVICE buffer `buf` once per
 * repetition, one workgroup of 256 lanes per contiguous `piece` (16-byte loads,
 * eight in flight per lane: the access pattern of the cached-pair products),
 * and writes the fastest of `reps` timed passes (after one untimed pass) in
 * milliseconds to *ms_out (HOST).  buf: 16-byte aligned, owned by the caller,
 * only read.  piece: a multiple of 16, at most bytes.  Runs on `hip_stream`
 * (NULL: the null stream) and synchronises.  ERT_EINVAL for bad arguments,
 * ERT_EDEVICE for a failed HIP call. */
ERT_API ert_status ert_vie_read_rate(const void* buf, size_t bytes, size_t piece, int reps, void* hip_stream,
                                     double* ms_out);


/* ------------------------------------------------------------------------
 * Learned right preconditioner (not part of the paper's method).
 *
 * A three-level 3D convolutional U-Net maps a residual r of (I - K) U = phi and
 * the medium to an approximate correction e ~ (I - K)^{-1} r; the solver uses it
 * as a right preconditioner of flexible GMRES (ert_solve_opts.precond).
 *
 * Input channels per cell: r / s (s = root mean square of r), log sigma_t,
 * sigma_s / sigma_t.  Output: z = r + s y with y the network value: the identity
 * part of the correction passes through exactly and the network supplies
 * e - r = K e, the part the transport operator produces.
 * Layers (w1, w2, w3 = width[0..2], default 16, 32, 64):
 *   L1 3x3x3 3 -> w1, ReLU; L2 w1 -> w1, ReLU (= s1); 2x2x2 average pool;
 *   L3 w1 -> w2, ReLU; L4 w2 -> w2, ReLU (= s2); pool;
 *   L5 w2 -> w3, ReLU; L6 w3 -> w3, ReLU; nearest 2x upsampling, concatenate
 *   [upsampled, s2]; L7 (w3 + w2) -> w2, ReLU; L8 w2 -> w2, ReLU; upsample,
 *   concatenate [upsampled, s1]; L9 (w2 + w1) -> w1, ReLU; L10 w1 -> w1, ReLU;
 *   L11 1x1x1 w1 -> 1.
 * 3x3x3 layers are cross-correlations with zero padding:
 *   out[o](z,y,x) = b[o] + sum_{i,a,c,d} W[o][i][a][c][d] in[i](z+a-1, y+c-1, x+d-1).
 * Parameters: one FP32 vector, layer by layer, W as [cout][cin][k][k][k] then
 * b[cout] (ert_net_param_count entries).
 * Arithmetic: 3x3x3 convolutions and their input gradients take BF16 weights
 * (round to nearest even) times activations split into two BF16 parts
 * (hi = bf16(x), lo = bf16(x - hi)) and accumulate in FP32; weight gradients,
 * the 1x1 layer, pooling, loss and Adam are FP32.
 * Loss: mean over the batch of ||y_b - t_b||^2 / ||t_b||^2, t_b = (e_b - r_b) / s_b.
 * Grid: dim 3, every n[a] a multiple of 4 (two poolings), cell order as the
 * solver's (x fastest).  Vectors are DEVICE FP64 N x batch, column-major;
 * sigma_t / sigma_s given to forward/grad/train are DEVICE FP64 N x batch (one
 * medium per column).  A network is not thread-safe; its work is ordered on
 * its stream.
 * ------------------------------------------------------------------------ */
typedef struct {
    int dim;          /* 3 */
    int n[3];         /* cells per axis, each a positive multiple of 4 */
    int batch_max;    /* largest batch of forward/grad/train calls; 0 -> 1 */
    int width[3];     /* channel widths w1, w2, w3; 0 -> 16, 32, 64; multiples of 16, <= 128 */
    int reserved[4];  /* must be 0 */
} ert_net_opts;

typedef struct {
    double lr;        /* Adam step size; 0 -> 1e-3 */
    double beta1;     /* 0 -> 0.9 */
    double beta2;     /* 0 -> 0.999 */
    double eps;       /* 0 -> 1e-8 */
} ert_net_train_opts;

/* Number of parameters of a network with these options, or -1. */
ERT_API long ert_net_param_count(const ert_net_opts* opts);

/* Create a network with zero parameters (set them with ert_net_set_params).
 * Returns ERT_EUNSUPPORTED for dim 2, ERT_EINVAL for bad sizes or widths. */
ERT_API ert_status ert_net_create(const ert_net_opts* opts, void* hip_stream, ert_net_t* out);

/* Number of parameters of `net`, or -1 for NULL. */
ERT_API long ert_net_size(ert_net_t net);

/* Copy parameters from / to HOST memory (ert_net_size floats); set also resets
 * the optimiser state.  Both synchronise. */
ERT_API ert_status ert_net_set_params(ert_net_t net, const float* params);
ERT_API ert_status ert_net_get_params(ert_net_t net, float* params);

/* z = M(r) for `batch` columns (device FP64).  Asynchronous. */
ERT_API ert_status ert_net_forward(ert_net_t net, const double* r, const double* sigma_t, const double* sigma_s,
                                   double* z, int batch);

/* Loss for targets e (the corrections with (I - K) e = r) and its gradient with
 * respect to the parameters: loss -> host double, grad -> host floats
 * (ert_net_size entries); either may be NULL.  Synchronises. */
ERT_API ert_status ert_net_grad(ert_net_t net, const double* r, const double* e, const double* sigma_t,
                                const double* sigma_s, int batch, double* loss, float* grad);

/* One Adam step (Kingma and Ba) on the loss of this batch; loss (host, may be
 * NULL) receives the loss before the step (synchronises only when non-NULL). */
ERT_API ert_status ert_net_train_step(ert_net_t net, const double* r, const double* e, const double* sigma_t,
                                      const double* sigma_s, int batch, const ert_net_train_opts* opts,
                                      double* loss);

/* Release the network.  NULL is a no-op. */
ERT_API void ert_net_destroy(ert_net_t net);

#ifdef __cplusplus
}
#endif

#endif /* ERTVIE_H */
