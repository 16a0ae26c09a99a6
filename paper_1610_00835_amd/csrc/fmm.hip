// Chebyshev-interpolation fast multipole method for the collocation apply
// (Sec. 3.3 with the multilevel tree of Sec. 4.2).
//
//   y_j = h^d * sum_{k != j} G(x_j, x_k) w_k + A_jj w_j
//
// Points are reordered leaf-major (leaf boxes of leaf^d cells, lexicographic);
// far-field interactions go through tensor Chebyshev interpolants with
// S_n(p,q) = prod_i (1/n + 2/n sum_{k=1}^{n-1} T_k(p_i) T_k(q_i))
// (eq. EQ: CHEB), nodes at the roots of T_n:
//   P2M  f1(q_m) = sum_{x_j in box} S_n(R^{-1} x_j, q_m) w_j        (step 1)
//   M2M  parent multipoles by re-anterpolating the children's node charges
//   M2L  f2(p_m) = sum_m' K(L p_m, R q_m') f1(q_m')                 (step 2, m2l.hip)
//   L2L  children's locals by interpolating the parent's local values
//   L2P  phi(x_i) = sum_m S_n(L^{-1} x_i, p_m) f2(p_m)              (step 3)
//   P2P  direct sums over the 3^d neighbouring leaves
// Every transfer is separable, so P2M/M2M/L2L/L2P are three (two in 2D) small
// 1D contractions done in LDS.  The interaction list of a box is the set of
// children of its parent's neighbours that are not its own neighbours
// (at most 6^d - 3^d, Sec. 4.2).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "fmm.hpp"

#include <type_traits>

namespace ertvie {

struct FmmData {
    virtual ~FmmData() {}
    virtual int rank_of(int l) const = 0;
    virtual int form_of(int site) const = 0;   // site -1: near field, l >= 0: far field of level l
    virtual long near_table() const = 0;       // entries of the near-field offset table, 0 = none
    virtual bool far_rebuilt(int l) const = 0; // heterogeneous level l rebuilt by every apply
    virtual double cache_bytes() const = 0;    // device bytes of the heterogeneous caches in use
    virtual ert_status apply(ert_plan_impl* p, int op, const double* x, double* y, int nrhs) = 0;
    virtual ert_status setup(ert_plan_impl* p) = 0;
    FmmTree tr;
};

namespace {

constexpr int kB = 256;

// ------------------------------------------------------------ geometry ----

__host__ __device__ inline void unravel3(long i, const int n[3], int out[3])
{
    out[0] = (int)(i % n[0]);
    long r = i / n[0];
    out[1] = (int)(r % n[1]);
    out[2] = (int)(r / n[1]);
}

struct DevTree {
    int D, nc, K, Kp, leaf, S;
    int nb[3];
    long nleaf, nslot;
    int n[3];       // grid cells per axis
};

// slot -> grid cell (or -1 when the slot lies outside the grid)
__device__ __forceinline__ long slot_cell(const DevTree& t, long slot, int c[3])
{
    long leafi = slot / t.S;
    int li = (int)(slot - leafi * t.S);
    int b[3], l[3];
    unravel3(leafi, t.nb, b);
    int ls[3] = {t.leaf, t.D > 1 ? t.leaf : 1, t.D > 2 ? t.leaf : 1};
    unravel3(li, ls, l);
    for (int a = 0; a < 3; ++a) {
        c[a] = (a < t.D) ? b[a] * t.leaf + l[a] : 0;
        if (c[a] >= t.n[a]) return -1;
    }
    return c[0] + (long)t.n[0] * (c[1] + (long)t.n[1] * c[2]);
}

// ---------------------------------------------------- gather / assemble ----

// Vectors and operator of the current apply, read by the first and last kernel
// so that one captured graph serves every call with the same rhs count.
struct ApplyIO {
    const double* x;
    double* y;
    int op;
    int pad;
};

// The first kernel of an apply receives the apply's vectors as an argument (the
// argument of a replayed graph's root node is updated per call) and stores them
// for the later kernels of the apply, which read them through io.
__device__ __forceinline__ void store_io(const ApplyIO& a, ApplyIO* io)
{
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *io = a;
}

template <typename T>
__global__ void k_gather(ApplyIO a, ApplyIO* io, DevTree t, const double* __restrict__ ss, long N, int B,
                         T* __restrict__ q)
{
    store_io(a, io);
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= t.nslot * B) return;
    const double* x = a.x;
    const int weighted = a.op != ERT_OP_G;
    int b = (int)(i / t.nslot);
    long slot = i - (long)b * t.nslot;
    int c[3];
    long j = slot_cell(t, slot, c);
    double v = 0.0;
    if (j >= 0) v = weighted ? ss[j] * x[j + (long)b * N] : x[j + (long)b * N];
    q[i] = T(v);
}

// y_j = h^d pot_j + A_jj w_j (FP64), op A: x_j - y_j; natural order
template <typename T>
__global__ void k_assemble(DevTree t, const T* __restrict__ pot, const ApplyIO* __restrict__ io,
                           const double* __restrict__ ss, const double* __restrict__ diag, double hd, long N, int B)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= N * B) return;
    const double* x = io->x;
    double* y = io->y;
    const int op = io->op;
    int b = (int)(i / N);
    long j = i - (long)b * N;
    int c[3];
    c[0] = (int)(j % t.n[0]);
    long r = j / t.n[0];
    c[1] = (int)(r % t.n[1]);
    c[2] = (int)(r / t.n[1]);
    int bl[3], l[3];
    for (int a = 0; a < 3; ++a) {
        bl[a] = (a < t.D) ? c[a] / t.leaf : 0;
        l[a] = (a < t.D) ? c[a] - bl[a] * t.leaf : 0;
    }
    long leafi = bl[0] + (long)t.nb[0] * (bl[1] + (long)t.nb[1] * bl[2]);
    long li = l[0] + (long)t.leaf * (l[1] + (long)(t.D > 1 ? t.leaf : 1) * l[2]);
    long slot = leafi * t.S + li;
    const double xj = x[i];
    const double w = (op == ERT_OP_G) ? xj : ss[j] * xj;
    double v = hd * (double)pot[(long)b * t.nslot + slot] + diag[j] * w;
    y[i] = (op == ERT_OP_A) ? xj - v : v;
}

constexpr int kLeafInWaves = 16;               // waves per workgroup of k_leaf_in
constexpr int kLeafWaves = 8;                  // waves per workgroup of k_leaf_out
constexpr int kLeafMaxPairs = kPadPairs;       // pairs per target on a one-level tree (at most 4^3 boxes)

// One-level homogeneous apply, first kernel.  Workgroup (leaf, 64 rows of the
// compressed multipole, rhs): the leaf's weighted charges go to LDS (and, from
// the first row chunk, to q in leaf order for the near-field products), then
// W = leaf_in q (leaf_in = Ut P, R x S) with one lane per row, read through the
// transposed copy [S][R] so that a wave's loads are contiguous; the sixteen
// waves take consecutive sixteenths of the S charges and their partial sums are
// added in wave order.
template <typename T>
__global__ __launch_bounds__(64 * kLeafInWaves) void k_leaf_in(ApplyIO a, ApplyIO* io, DevTree t,
                                                             const double* __restrict__ ss, long N,
                                                             const T* __restrict__ linT, int R, int rch,
                                                             T* __restrict__ q, T* __restrict__ W)
{
    store_io(a, io);
    extern __shared__ __align__(16) unsigned char smem[];
    T* part = (T*)smem;                          // [kLeafInWaves][64]
    T* sq = part + kLeafInWaves * 64;              // [S]
    const long pos = xcd_position(blockIdx.x, gridDim.x);
    const long leafi = pos / rch;
    const int chunk = (int)(pos % rch);
    const int b = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = chunk * 64 + lane;
    const int per = (t.S + kLeafInWaves - 1) / kLeafInWaves;
    const int k0 = wave * per, k1 = min(t.S, k0 + per);
    const T* col = linT + r;
    // a lane's first 16 operator entries, requested before the charges are gathered
    const bool pre = r < R && k1 - k0 >= 16;
    T v0[16];
    if (pre) {
#pragma unroll
        for (int u = 0; u < 16; ++u) v0[u] = col[(long)(k0 + u) * R];
    }
    const double* x = a.x;
    const int weighted = a.op != ERT_OP_G;
    for (int li = threadIdx.x; li < t.S; li += blockDim.x) {
        const long slot = leafi * t.S + li;
        int c[3];
        const long j = slot_cell(t, slot, c);
        double v = 0.0;
        if (j >= 0) v = weighted ? ss[j] * x[j + (long)b * N] : x[j + (long)b * N];
        const T tv = T(v);
        sq[li] = tv;
        if (chunk == 0) q[(long)b * t.nslot + slot] = tv;
    }
    __syncthreads();
    T acc = T(0);
    if (r < R) {
        int k = k0;
        if (pre) {
#pragma unroll
            for (int u = 0; u < 16; ++u) acc += v0[u] * sq[k0 + u];
            k += 16;
        }
        for (; k + 16 <= k1; k += 16) {
            T v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = col[(long)(k + u) * R];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc += v[u] * sq[k + u];
        }
        for (; k < k1; ++k) acc += col[(long)k * R] * sq[k];
    }
    part[wave * 64 + lane] = acc;
    __syncthreads();
    if (wave != 0 || r >= R) return;
    T s = part[lane];
    for (int w = 1; w < kLeafInWaves; ++w) s += part[w * 64 + lane];
    W[((long)b * t.nleaf + leafi) * R + r] = s;
}

// sum over k in [k0, k1) of St[tp[k] * M], in order, eight loads in flight
template <typename T>
__device__ __forceinline__ T staged_sum(const T* __restrict__ St, int M, const int* tp, int k0, int k1)
{
    T s = T(0);
    int k = k0;
    for (; k + 8 <= k1; k += 8) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = St[(long)tp[k + u] * M];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; k < k1; ++k) s += St[(long)tp[k] * M];
    return s;
}

// The same sum with all loads in flight at once when the range holds at most MAXK.
template <typename T, int MAXK>
__device__ __forceinline__ T staged_sum_one(const T* __restrict__ St, int M, const int* tp, int k0, int k1)
{
    if (k1 - k0 > MAXK) return staged_sum(St, M, tp, k0, k1);
    T v[MAXK];
#pragma unroll
    for (int u = 0; u < MAXK; ++u) v[u] = (k0 + u < k1) ? St[(long)tp[k0 + u] * M] : T(0);
    T s = T(0);
#pragma unroll
    for (int u = 0; u < MAXK; ++u)
        if (k0 + u < k1) s += v[u];
    return s;
}

// One-level homogeneous apply, last kernel.  Workgroup (leaf, 64 cells of the
// leaf, rhs): the leaf's far-field local expansion is the sum of its staged
// translation products (the pair list cut into as many consecutive parts as
// the workgroup holds copies of the rank, parts added in order); each lane owns
// one cell, whose potential is the sum of its staged near-field products plus
// the expansion with L2P (leaf_out = P^T Um, S x R, read through the transposed
// copy [R][S]).  The eight waves take consecutive eighths of the near pairs and
// of the rank, partial sums are added in wave order, and wave 0 assembles
// y = h^d pot + A_jj w (op A: x - y) in the natural cell order.
template <typename T>
__global__ __launch_bounds__(64 * kLeafWaves) void k_leaf_out(
    DevTree t, const ApplyIO* __restrict__ io, const double* __restrict__ ss, const double* __restrict__ diag,
    double hd, long N, const T* __restrict__ stn, const int* __restrict__ tcn, const int* __restrict__ tpn, long npn,
    const T* __restrict__ stf, const int* __restrict__ tcf, const int* __restrict__ tpf, long npf, int R,
    const T* __restrict__ loutT, int sch)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int pl_n[kLeafMaxPairs], pl_f[kLeafMaxPairs];
    T* pn = (T*)smem;                            // [kLeafWaves][64] near partial sums
    T* pf = pn + kLeafWaves * 64;                // [kLeafWaves][64] L2P partial sums
    T* sl = pf + kLeafWaves * 64;                // [R] far-field local expansion
    T* fpart = sl + R;                           // [G][R] far partial sums
    const long pos = xcd_position(blockIdx.x, gridDim.x);
    const long leafi = pos / sch;
    const int chunk = (int)(pos % sch);
    const int b = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = chunk * 64 + lane;
    const bool ok = li < t.S;
    // pair lists padded to kLeafMaxPairs per target, and their lengths: one round of loads
    const int nn = tcn[leafi], nf = tcf[leafi];
    if (threadIdx.x < kLeafMaxPairs) pl_n[threadIdx.x] = tpn[leafi * kLeafMaxPairs + threadIdx.x];
    else if (threadIdx.x < 2 * kLeafMaxPairs)
        pl_f[threadIdx.x - kLeafMaxPairs] = tpf[leafi * kLeafMaxPairs + threadIdx.x - kLeafMaxPairs];
    // a lane's first 16 L2P operator entries, requested before the staged sums
    const int perR = (R + kLeafWaves - 1) / kLeafWaves;
    const int r0 = min(R, wave * perR), r1 = min(R, r0 + perR);
    const T* lcol = loutT + li;
    const bool pre = ok && r1 - r0 >= 16;
    T lv[16];
    if (pre) {
#pragma unroll
        for (int u = 0; u < 16; ++u) lv[u] = lcol[(long)(r0 + u) * t.S];
    }
    // the assembly's operands, loaded early
    int c[3];
    long j = -1;
    double xj = 0.0, sj = 0.0, dj = 0.0;
    if (wave == 0 && ok) {
        j = slot_cell(t, leafi * t.S + li, c);
        if (j >= 0) {
            xj = io->x[j + (long)b * N];
            sj = ss[j];
            dj = diag[j];
        }
    }
    __syncthreads();
    const int G = (int)blockDim.x / R;           // copies of the rank in the workgroup (>= 1)
    {
        const int g = (int)threadIdx.x / R, r = (int)threadIdx.x - g * R;
        const int per = (nf + G - 1) / G;
        if (g < G) {
            const int a0 = min(nf, g * per), a1 = min(nf, a0 + per);
            fpart[g * R + r] = staged_sum_one<T, 24>(stf + (long)b * npf * R + r, R, pl_f, a0, a1);
        }
    }
    {
        const int per = (nn + kLeafWaves - 1) / kLeafWaves;
        const int a0 = min(nn, wave * per), a1 = min(nn, a0 + per);
        pn[wave * 64 + lane] = ok ? staged_sum(stn + (long)b * npn * t.S + li, t.S, pl_n, a0, a1) : T(0);
    }
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        T v = fpart[r];
        for (int g = 1; g < G; ++g) v += fpart[g * R + r];
        sl[r] = v;
    }
    __syncthreads();
    {
        T acc = T(0);
        if (ok) {
            int r = r0;
            if (pre) {
#pragma unroll
                for (int u = 0; u < 16; ++u) acc += lv[u] * sl[r0 + u];
                r += 16;
            }
            for (; r + 16 <= r1; r += 16) {
                T v[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) v[u] = lcol[(long)(r + u) * t.S];
#pragma unroll
                for (int u = 0; u < 16; ++u) acc += v[u] * sl[r + u];
            }
            for (; r < r1; ++r) acc += lcol[(long)r * t.S] * sl[r];
        }
        pf[wave * 64 + lane] = acc;
    }
    __syncthreads();
    if (wave != 0 || j < 0) return;
    T near = pn[lane], far = pf[lane];
    for (int w = 1; w < kLeafWaves; ++w) {
        near += pn[w * 64 + lane];
        far += pf[w * 64 + lane];
    }
    const int op = io->op;
    const double w = (op == ERT_OP_G) ? xj : sj * xj;
    const double v = hd * (double)(near + far) + dj * w;
    io->y[j + (long)b * N] = (op == ERT_OP_A) ? xj - v : v;
}

template <typename T>
__global__ void k_zero_t(T* __restrict__ p, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = T(0);
}

// --------------------------------------------------- separable transfers ----

// out = contraction of `in` (dims d0 x d1 x d2, x fastest) along `axis` with a
// 1D matrix: out[.., m, ..] = sum_i M(m, i) in[.., i, ..].  M(m,i) = mat[m*nin + i],
// or mat[i*nout + m] when `tr`.  Cooperative over the block; ends with a barrier.
template <typename T>
__device__ void sep_axis(const T* in, T* out, int d0, int d1, int d2, int axis, int nout, const T* mat, bool tr)
{
    int od[3] = {d0, d1, d2};
    const int nin = od[axis];
    od[axis] = nout;
    const int total = od[0] * od[1] * od[2];
    for (int tix = threadIdx.x; tix < total; tix += blockDim.x) {
        int c[3] = {tix % od[0], (tix / od[0]) % od[1], tix / (od[0] * od[1])};
        const int m = c[axis];
        T acc = T(0);
        for (int i = 0; i < nin; ++i) {
            c[axis] = i;
            const T mv = tr ? mat[i * nout + m] : mat[m * nin + i];
            acc += mv * in[c[0] + d0 * (c[1] + d1 * c[2])];
        }
        out[tix] = acc;
    }
    __syncthreads();
}

// apply the 1D matrices along every axis: input extent nin per axis, output nout
template <typename T>
__device__ const T* sep_all(const T* in, T* b0, T* b1, int D, int nin, int nout, const T* m0, const T* m1,
                            const T* m2, bool tr)
{
    int d[3] = {nin, D > 1 ? nin : 1, D > 2 ? nin : 1};
    sep_axis<T>(in, b0, d[0], d[1], d[2], 0, nout, m0, tr);
    d[0] = nout;
    if (D == 1) return b0;
    sep_axis<T>(b0, b1, d[0], d[1], d[2], 1, nout, m1, tr);
    d[1] = nout;
    if (D == 2) return b1;
    sep_axis<T>(b1, b0, d[0], d[1], d[2], 2, nout, m2, tr);
    return b0;
}

constexpr int kSepBuf = 512;   // largest tensor in a transfer: max(nc, leaf)^3 <= 8^3

// P2M: one block per (leaf, rhs).  P1[m][i] = S_n(xi_i, p_m).
template <typename T>
__global__ __launch_bounds__(kB) void k_p2m(DevTree t, const T* __restrict__ q, const T* __restrict__ P1,
                                            T* __restrict__ W)
{
    __shared__ T in[kSepBuf], b0[kSepBuf], b1[kSepBuf], mat[64];
    const long leafi = blockIdx.x;
    const int b = blockIdx.y;
    for (int i = threadIdx.x; i < t.nc * t.leaf; i += blockDim.x) mat[i] = P1[i];
    for (int i = threadIdx.x; i < t.S; i += blockDim.x) in[i] = q[(long)b * t.nslot + leafi * t.S + i];
    __syncthreads();
    const T* r = sep_all<T>(in, b0, b1, t.D, t.leaf, t.nc, mat, mat, mat, false);
    T* dst = W + ((long)b * t.nleaf + leafi) * t.Kp;
    for (int i = threadIdx.x; i < t.K; i += blockDim.x) dst[i] = r[i];
}

// M2M: one block per (parent box, rhs), the transfer factorised axis by axis over the
// children: W_p = sum_c (M_{c_z} (x) M_{c_y} (x) M_{c_x}) W_c, with M_o[m][m'] =
// S_n(node m' of the child at offset o in the parent frame, p_m).  The x contraction
// of all 2^d children is summed over c_x (2^(d-1) tensors), then the y contraction
// over c_y (2^(d-2)), then z: 2^d + 2^(d-1) + 2^(d-2) one-axis contractions instead
// of 3 per child, three barriers in all.  Children outside the lattice are zero.
template <typename T>
__global__ __launch_bounds__(kB) void k_m2m(int D, int nc, int K, int Kp, int nlp0, int nlp1, int nlp2, long nboxp,
                                            int nlc0, int nlc1, int nlc2, long nboxc, const T* __restrict__ Wc,
                                            const T* __restrict__ M1, T* __restrict__ Wp)
{
    __shared__ T ch[8 * kSepBuf];       // children (x-contracted pairs reuse it)
    __shared__ T zc[4 * kSepBuf];       // x-contracted, summed over c_x
    __shared__ T mat[128];
    const long pbox = blockIdx.x;
    const int b = blockIdx.y;
    const int nlp[3] = {nlp0, nlp1, nlp2}, nlc[3] = {nlc0, nlc1, nlc2};
    const int nchild = 1 << D;
    int pc[3];
    unravel3(pbox, nlp, pc);
    for (int i = threadIdx.x; i < 2 * nc * nc; i += blockDim.x) mat[i] = M1[i];
    for (int i = threadIdx.x; i < nchild * K; i += blockDim.x) {
        const int c = i / K, m = i - c * K;
        int cc[3];
        bool inside = true;
        for (int a = 0; a < 3; ++a) {
            cc[a] = (a < D) ? 2 * pc[a] + ((c >> a) & 1) : 0;
            if (a < D && cc[a] >= nlc[a]) inside = false;
        }
        const long cb = cc[0] + (long)nlc[0] * (cc[1] + (long)nlc[1] * cc[2]);
        ch[i] = inside ? Wc[((long)b * nboxc + cb) * Kp + m] : T(0);
    }
    __syncthreads();
    const int n1 = D > 1 ? nc : 1, n2 = D > 2 ? nc : 1;
    // x: zc[c >> 1][m] = sum_{cx} sum_k M_cx[m0][k] ch[c][.., k]
    for (int i = threadIdx.x; i < (nchild >> 1) * K; i += blockDim.x) {
        const int q = i / K, m = i - q * K;
        const int m0 = m % nc, rest = m - m0;
        T sum = T(0);
        for (int cx = 0; cx < 2; ++cx) {
            const T* mx = mat + cx * nc * nc + m0 * nc;
            const T* in = ch + (2 * q + cx) * K + rest;
            for (int k = 0; k < nc; ++k) sum += mx[k] * in[k];
        }
        zc[i] = sum;
    }
    __syncthreads();
    if (D == 1) {
        T* dst = Wp + ((long)b * nboxp + pbox) * Kp;
        for (int i = threadIdx.x; i < K; i += blockDim.x) dst[i] = zc[i];
        return;
    }
    // y: ch[q >> 1][m] = sum_{cy} sum_k M_cy[m1][k] zc[q][.., k, ..]
    for (int i = threadIdx.x; i < (nchild >> 2) * K; i += blockDim.x) {
        const int q = i / K, m = i - q * K;
        const int m0 = m % nc, m1 = (m / nc) % n1, m2 = m / (nc * n1);
        T sum = T(0);
        for (int cy = 0; cy < 2; ++cy) {
            const T* my = mat + cy * nc * nc + m1 * nc;
            const T* in = zc + (2 * q + cy) * K + m2 * nc * n1 + m0;
            for (int k = 0; k < nc; ++k) sum += my[k] * in[k * nc];
        }
        ch[i] = sum;
    }
    __syncthreads();
    T* dst = Wp + ((long)b * nboxp + pbox) * Kp;
    if (D == 2) {
        for (int i = threadIdx.x; i < K; i += blockDim.x) dst[i] = ch[i];
        return;
    }
    // z: W_p[m] = sum_{cz} sum_k M_cz[m2][k] ch[cz][k, m1, m0]
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
        const int m01 = i % (nc * n1), m2 = i / (nc * n1);
        T sum = T(0);
        for (int cz = 0; cz < 2; ++cz) {
            const T* mz = mat + cz * nc * nc + m2 * nc;
            const T* in = ch + cz * K + m01;
            for (int k = 0; k < n2; ++k) sum += mz[k] * in[k * nc * n1];
        }
        dst[i] = sum;
    }
}

// L2L: one block per (child box, rhs): the child's locals are the parent's
// local interpolant evaluated at the child nodes (written, not accumulated:
// the far-field translations of the child level are added afterwards).
template <typename T>
__global__ __launch_bounds__(kB) void k_l2l(int D, int nc, int K, int Kp, int nlp0, int nlp1, int nlp2, long nboxp,
                                            int nlc0, int nlc1, int nlc2, long nboxc, const T* __restrict__ Lp,
                                            const T* __restrict__ M1, T* __restrict__ Lc)
{
    __shared__ T in[kSepBuf], b0[kSepBuf], b1[kSepBuf], mat[128];
    const long cbox = blockIdx.x;
    const int b = blockIdx.y;
    const int nlp[3] = {nlp0, nlp1, nlp2}, nlc[3] = {nlc0, nlc1, nlc2};
    int cc[3];
    unravel3(cbox, nlc, cc);
    for (int i = threadIdx.x; i < 2 * nc * nc; i += blockDim.x) mat[i] = M1[i];
    long pb = (cc[0] >> 1) + (long)nlp[0] * ((cc[1] >> 1) + (long)nlp[1] * (cc[2] >> 1));
    const T* src = Lp + ((long)b * nboxp + pb) * Kp;
    for (int i = threadIdx.x; i < K; i += blockDim.x) in[i] = src[i];
    __syncthreads();
    const T* r = sep_all<T>(in, b0, b1, D, nc, nc, mat + (cc[0] & 1) * nc * nc, mat + (cc[1] & 1) * nc * nc,
                            mat + (cc[2] & 1) * nc * nc, true);
    T* dst = Lc + ((long)b * nboxc + cbox) * Kp;
    for (int i = threadIdx.x; i < K; i += blockDim.x) dst[i] = r[i];
}

// L2P: one block per (leaf, rhs); adds the far field to the potential.
template <typename T>
__global__ __launch_bounds__(kB) void k_l2p(DevTree t, const T* __restrict__ Lc, const T* __restrict__ P1,
                                            T* __restrict__ pot)
{
    __shared__ T in[kSepBuf], b0[kSepBuf], b1[kSepBuf], mat[64];
    const long leafi = blockIdx.x;
    const int b = blockIdx.y;
    for (int i = threadIdx.x; i < t.nc * t.leaf; i += blockDim.x) mat[i] = P1[i];
    const T* src = Lc + ((long)b * t.nleaf + leafi) * t.Kp;
    for (int i = threadIdx.x; i < t.K; i += blockDim.x) in[i] = src[i];
    __syncthreads();
    const T* r = sep_all<T>(in, b0, b1, t.D, t.nc, t.leaf, mat, mat, mat, true);
    T* dst = pot + (long)b * t.nslot + leafi * t.S;
    for (int i = threadIdx.x; i < t.S; i += blockDim.x) dst[i] += r[i];
}

// ---------------------------------------------------------- near field ----

// Homogeneous media: G between two collocation points depends only on the
// integer K = |offset|^2, so the near field reads a table g[K] (g[0] = 0 drops
// the self pair).  One block per (target leaf, rhs); the 3^d neighbour leaves'
// charges are staged in LDS; threads = targets x source groups.
template <typename T>
__global__ __launch_bounds__(kB) void k_p2p_hom(DevTree t, const T* __restrict__ q, const T* __restrict__ tab,
                                                int ntab, T* __restrict__ pot)
{
    extern __shared__ unsigned char smem[];
    T* stab = (T*)smem;                          // [ntab]
    const int nn = (t.D == 3) ? 27 : 9;
    T* sq = stab + ntab;                         // [nn][S]
    int* nbr = (int*)(sq + nn * t.S);            // [nn] neighbour leaf (or -1), 32 slots
    const long leafi = blockIdx.x;
    const int b = blockIdx.y;
    int lb[3];
    unravel3(leafi, t.nb, lb);
    if (threadIdx.x < nn) {
        int k = threadIdx.x, o[3] = {k % 3 - 1, (k / 3) % 3 - 1, t.D == 3 ? k / 9 - 1 : 0};
        int s[3];
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
            s[a] = lb[a] + ((a < t.D) ? o[a] : 0);
            if (s[a] < 0 || s[a] >= t.nb[a]) ok = false;
        }
        nbr[k] = ok ? (int)(s[0] + (long)t.nb[0] * (s[1] + (long)t.nb[1] * s[2])) : -1;
    }
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) stab[i] = tab[i];
    __syncthreads();
    for (int i = threadIdx.x; i < nn * t.S; i += blockDim.x) {
        int k = i / t.S, li = i - k * t.S;
        sq[i] = nbr[k] >= 0 ? q[(long)b * t.nslot + (long)nbr[k] * t.S + li] : T(0);
    }
    __syncthreads();
    const int ls1 = t.D > 1 ? t.leaf : 1;
    const int tpp = t.S < (int)blockDim.x ? t.S : (int)blockDim.x;     // targets per pass
    const int groups = blockDim.x / tpp;
    const int grp = threadIdx.x / tpp;
    T* red = (T*)(nbr + 32);                     // [groups][tpp]
    for (int tb = 0; tb < t.S; tb += tpp) {
        const int ti = tb + (threadIdx.x % tpp);
        T acc = T(0);
        if (grp < groups && ti < t.S) {
            const int tx = ti % t.leaf, ty = (ti / t.leaf) % ls1, tz = ti / (t.leaf * ls1);
            for (int k = grp; k < nn; k += groups) {
                if (nbr[k] < 0) continue;
                const int ox = (k % 3 - 1) * t.leaf, oy = ((k / 3) % 3 - 1) * t.leaf;
                const int oz = (t.D == 3) ? (k / 9 - 1) * t.leaf : 0;
                const T* qs = sq + k * t.S;
                for (int sz = 0; sz < (t.D == 3 ? t.leaf : 1); ++sz) {
                    const int dz = tz - (sz + oz);
                    for (int sy = 0; sy < ls1; ++sy) {
                        const int dy = ty - (sy + oy);
                        const int ayz = dz * dz + dy * dy;
                        const T* qrow = qs + t.leaf * (sy + ls1 * sz);
                        for (int sx = 0; sx < t.leaf; ++sx) {
                            const int dx = tx - (sx + ox);
                            acc += stab[ayz + dx * dx] * qrow[sx];
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (grp < groups) red[grp * tpp + (threadIdx.x % tpp)] = acc;
        __syncthreads();
        if (threadIdx.x < tpp && tb + (int)threadIdx.x < t.S) {
            T s = red[threadIdx.x];
            for (int g2 = 1; g2 < groups; ++g2) s += red[g2 * tpp + threadIdx.x];
            pot[(long)b * t.nslot + leafi * t.S + tb + threadIdx.x] = s;
        }
        __syncthreads();
    }
}

// Corner-octet table of sigma_t for the ray march of the cache builds (layout
// in sigma_at8).  Cells on the upper face of an axis are never the lower
// corner of an interpolation cell; their octets repeat the face values.
__global__ void k_corner8(Geo g, const double* __restrict__ st, double* __restrict__ st8, long ncell)
{
    const long b = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (b >= ncell) return;
    const int i0 = (int)(b % g.n0), i1 = (int)((b / g.n0) % g.n1);
    const int i2 = (int)(b / ((long)g.n0 * g.n1));
    const long d0 = (g.n0 > 1 && i0 < g.n0 - 1) ? 1 : 0;
    const long d1 = (g.n1 > 1 && i1 < g.n1 - 1) ? g.n0 : 0;
    const long d2 = (g.dim > 2 && g.n2 > 1 && i2 < g.n2 - 1) ? (long)g.n0 * g.n1 : 0;
    double2* q = reinterpret_cast<double2*>(st8) + 4 * b;
    q[0] = make_double2(st[b], st[b + d0]);
    q[1] = make_double2(st[b + d1], st[b + d1 + d0]);
    q[2] = make_double2(st[b + d2], st[b + d2 + d0]);
    q[3] = make_double2(st[b + d2 + d1], st[b + d2 + d1 + d0]);
}

// Cached near-field blocks for the ray kernel, FP64 arithmetic: the same rule
// as the dense apply (exact integer step count, marched from the lower index,
// so the value of a cell pair does not depend on its order).  One workgroup per
// stored pair u (blocks u0 .. ; blk and lo_plane point at block u0): element
// [si][ti] = G(cell ti of leaf ua[u], cell si of leaf ub[u]), zero for a cell
// with itself (the diagonal's term).  FP32 values as a BF16-rounded high plane
// and the exact remainder.  sigma_t over the cells spanned by the two leaves,
// plus one layer above (the upper corner of a sample on the top face), is
// staged in LDS and the march reads it there: samples lie between the two cell
// centres, so every corner they need is in the box.  Cell search and
// interpolation are sigma_at's, term for term.  Leaves have at most
// kNearLdsLeaf cells per side (the plan's limit).
constexpr int kNearLdsLeaf = 8;
constexpr int kNearLdsSide = 2 * kNearLdsLeaf + 1;
constexpr int kNearLdsThreads = 512;

__global__ __launch_bounds__(kNearLdsThreads) void k_near_blocks(
    DevTree t, Geo g, const double* __restrict__ st, const double* __restrict__ itab, const int* __restrict__ ua,
    const int* __restrict__ ub, long u0, uint16_t* __restrict__ blk, int16_t* __restrict__ lo_plane)
{
    constexpr int P = kNearLdsSide;  // LDS pitch of a row and (P * P) of a plane
    __shared__ double sl[P * P * P];
    const long u = u0 + blockIdx.x;
    const int per = t.S * t.S;
    const int n[3] = {g.n0, g.n1, g.n2};
    int bt[3], bs[3], lo[3], ext[3];
    unravel3(ua[u], t.nb, bt);
    unravel3(ub[u], t.nb, bs);
    for (int a = 0; a < 3; ++a) {
        if (a < t.D) {
            // lowest cell: the leaves' first, or n - 2 when the clamped search
            // (k <= n - 2) reaches below a one-cell leaf on the top face
            int l0 = (bt[a] < bs[a] ? bt[a] : bs[a]) * t.leaf;
            l0 = (n[a] > 1 && l0 > n[a] - 2) ? n[a] - 2 : l0;
            int hi = ((bt[a] > bs[a] ? bt[a] : bs[a]) + 1) * t.leaf + 1;
            hi = hi < n[a] ? hi : n[a];
            lo[a] = l0;
            ext[a] = hi - l0;
        } else {
            lo[a] = 0;
            ext[a] = 1;
        }
    }
    // staged box: at least two layers per axis (an axis of one cell repeats it,
    // so its upper corner reads the same value as sigma_at's zero offset)
    const int sx0 = ext[0] > 1 ? ext[0] : 2, sx1 = ext[1] > 1 ? ext[1] : 2, sx2 = ext[2] > 1 ? ext[2] : 2;
    for (int e = threadIdx.x; e < sx0 * sx1 * sx2; e += kNearLdsThreads) {
        const int x0 = e % sx0, x1 = (e / sx0) % sx1, x2 = e / (sx0 * sx1);
        const int c0 = lo[0] + (x0 < ext[0] ? x0 : ext[0] - 1), c1 = lo[1] + (x1 < ext[1] ? x1 : ext[1] - 1);
        const int c2 = lo[2] + (x2 < ext[2] ? x2 : ext[2] - 1);
        sl[x0 + P * (x1 + P * x2)] = st[c0 + (long)g.n0 * (c1 + (long)g.n1 * c2)];
    }
    __syncthreads();
    const double inv_h = 1.0 / g.h;
    const bool d3 = t.D > 2;
    // An axis of one cell (or the third axis in 2D) takes k = 0 and t = 0: its
    // terms add exact zeros, so a 2D value is sigma_at's c0.
    const double hiA[3] = {double(n[0] - 1), double(n[1] - 1), double(n[2] - 1)};
    const double kmA[3] = {double(n[0] > 1 ? n[0] - 2 : 0), double(n[1] > 1 ? n[1] - 2 : 0),
                           double(n[2] > 1 ? n[2] - 2 : 0)};
    const double off = fma(double(P * P), double(lo[2]), fma(double(P), double(lo[1]), double(lo[0])));
    const int L = t.leaf, L1 = t.D > 1 ? t.leaf : 1;
    uint16_t* bo = blk + (u - u0) * (long)per;
    int16_t* lp = lo_plane + (u - u0) * (long)per;
    for (int i = threadIdx.x; i < per; i += kNearLdsThreads) {
        const int si = i / t.S, ti = i - (i / t.S) * t.S;
        double v = 0.0;
        // cells of slot ti of the target leaf and slot si of the source leaf
        const int ct[3] = {bt[0] * L + ti % L, t.D > 1 ? bt[1] * L + (ti / L) % L1 : 0,
                           t.D > 2 ? bt[2] * L + ti / (L * L1) : 0};
        const int cs[3] = {bs[0] * L + si % L, t.D > 1 ? bs[1] * L + (si / L) % L1 : 0,
                           t.D > 2 ? bs[2] * L + si / (L * L1) : 0};
        const bool in = ct[0] < n[0] && ct[1] < n[1] && ct[2] < n[2] && cs[0] < n[0] && cs[1] < n[1] &&
                        cs[2] < n[2];
        const long jt = ct[0] + (long)n[0] * (ct[1] + (long)n[1] * ct[2]);
        const long js = cs[0] + (long)n[0] * (cs[1] + (long)n[1] * cs[2]);
        if (in && jt != js) {
            int K = 0;
            for (int a = 0; a < 3; ++a) K += (ct[a] - cs[a]) * (ct[a] - cs[a]);
            const double r = g.h * sqrt((double)K);
            const int* pa = (jt < js) ? ct : cs;
            const int* pb = (jt < js) ? cs : ct;
            const double a0 = g.h * (pa[0] + 0.5), a1 = g.h * (pa[1] + 0.5), a2 = d3 ? g.h * (pa[2] + 0.5) : 0.0;
            const double e0 = g.h * (pb[0] + 0.5) - a0, e1 = g.h * (pb[1] + 0.5) - a1;
            const double e2 = (d3 ? g.h * (pb[2] + 0.5) : 0.0) - a2;
            const int m = steps_grid(K);
            const double inv_m = 1.0 / double(m);
            double s = 0.0;
            for (int q = 1; q <= m; ++q) {
                const double f = (double(q) - 0.5) * inv_m;
                const double u0 = fmin(fmax((a0 + f * e0) * inv_h - 0.5, 0.0), hiA[0]);
                const double u1 = fmin(fmax((a1 + f * e1) * inv_h - 0.5, 0.0), hiA[1]);
                const double u2 = fmin(fmax((a2 + f * e2) * inv_h - 0.5, 0.0), hiA[2]);
                const double k0 = fmin(floor(u0), kmA[0]), k1 = fmin(floor(u1), kmA[1]);
                const double k2 = fmin(floor(u2), kmA[2]);
                const double t0 = u0 - k0, t1 = u1 - k1, t2 = u2 - k2;
                const double* c = sl + (int)(fma(double(P * P), k2, fma(double(P), k1, k0)) - off);
                double c00 = c[0] + t0 * (c[1] - c[0]);
                double c10 = c[P] + t0 * (c[P + 1] - c[P]);
                double c0 = c00 + t1 * (c10 - c00);
                double c01 = c[P * P] + t0 * (c[P * P + 1] - c[P * P]);
                double c11 = c[P * P + P] + t0 * (c[P * P + P + 1] - c[P * P + P]);
                double c1 = c01 + t1 * (c11 - c01);
                s += c0 + t2 * (c1 - c0);
            }
            const double tau = r * inv_m * s;
            if (itab) {
                const int o0 = abs(ct[0] - cs[0]), o1 = abs(ct[1] - cs[1]), o2 = abs(ct[2] - cs[2]);
                const double hp = (t.D == 2) ? g.h : g.h * g.h;
                v = exp(-tau) * itab[o0 + (long)g.n0 * (o1 + (long)g.n1 * o2)] / (surface_area(t.D) * hp);
            } else {
                const double rp = (t.D == 2) ? r : r * r;
                v = exp(-tau) / (surface_area(t.D) * rp);
            }
        }
        const unsigned X = __float_as_uint((float)v);
        const unsigned hi = (X + 0x8000u) >> 16;
        bo[i] = (uint16_t)hi;
        lp[i] = (int16_t)(int)(X - (hi << 16));
    }
}

// ----------------------------------------------- far-field operators ----

__device__ __forceinline__ void node_multi(int m, int nc, int D, int out[3])
{
    out[0] = m % nc;
    out[1] = D > 1 ? (m / nc) % nc : 0;
    out[2] = D > 2 ? m / (nc * nc) : 0;
}

// Homogeneous translation matrices of one level: ops[o][r][c] =
// G(target node r, source node c) for box offset o (FP64 arithmetic).
template <typename T>
__global__ void k_ops_hom(int D, int nc, int K, int Kp, double w, double sigma, const double* __restrict__ cheb,
                          T* __restrict__ ops, __bf16* __restrict__ lo, int mii, double h)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long per = (long)Kp * Kp;
    int noff = 1;
    for (int a = 0; a < D; ++a) noff *= kOffSide;
    if (i >= noff * per) return;
    int oi = (int)(i / per);
    long rem = i - (long)oi * per;
    int r = (int)(rem / Kp), c = (int)(rem % Kp);
    double v = 0.0;
    int o[3] = {oi % kOffSide - 3, (oi / kOffSide) % kOffSide - 3, D > 2 ? oi / (kOffSide * kOffSide) - 3 : 0};
    bool far = false;
    for (int a = 0; a < D; ++a)
        if (o[a] < -1 || o[a] > 1) far = true;
    if (far && r < K && c < K) {
        int mr[3], mc[3];
        node_multi(r, nc, D, mr);
        node_multi(c, nc, D, mc);
        double r2 = 0.0, dv[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < D; ++a) {
            double d = w * (o[a] + 0.5 * (cheb[mc[a]] - cheb[mr[a]]));
            dv[a] = d;
            r2 += d * d;
        }
        double rr = sqrt(r2);
        if (mii) {
            const double hp = (D == 2) ? h : h * h;
            v = exp(-sigma * rr) * cell_int(D, dv[0] / h, dv[1] / h, dv[2] / h, 64.0) / (surface_area(D) * hp);
        } else {
            double rp = (D == 2) ? rr : r2;
            v = exp(-sigma * rr) / (surface_area(D) * rp);
        }
    }
    if (lo) {
        __bf16 hi = (__bf16)(float)v;
        ((__bf16*)ops)[i] = hi;
        lo[i] = (__bf16)((float)v - (float)hi);
    } else {
        ops[i] = T(v);
    }
}

// Coordinate of Chebyshev node value c in the box of index b (width w), written
// as one fused product so that every kernel building a matrix entry rounds it
// the same way.
__device__ __forceinline__ double node_coord(double w, int b, double c)
{
    return fma(w, double(b) + 0.5, (0.5 * w) * c);
}

// Heterogeneous translation matrices, one per stored (target, source) pair of a
// level, stored source-node major: opsT[pair][c][r] (opsT points at pair p0).  Midpoint ray rule with
// step <= h/2 between the Chebyshev nodes (FP64 arithmetic).  The rule samples the
// same points from either end, so the matrix of (source, target) is the transpose.
template <typename T>
__global__ void k_ops_het(Geo g, const double* __restrict__ st8, int D, int nc, int K, int Kp, double w,
                          int nl0, int nl1, int nl2, const double* __restrict__ cheb, const int* __restrict__ pair_t,
                          const int* __restrict__ pair_s, long p0, long np, T* __restrict__ opsT, int mii)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long per = (long)Kp * Kp;
    if (i >= np * per) return;
    long p = p0 + i / per;
    long rem = i % per;
    int c = (int)(rem / Kp), r = (int)(rem % Kp);
    double v = 0.0;
    if (r < K && c < K) {
        const int nl[3] = {nl0, nl1, nl2};
        int tb[3], sb[3], mr[3], mc[3];
        unravel3(pair_t[p], nl, tb);
        unravel3(pair_s[p], nl, sb);
        node_multi(r, nc, D, mr);
        node_multi(c, nc, D, mc);
        double X[3] = {0, 0, 0}, Y[3] = {0, 0, 0};
        double r2 = 0.0;
        for (int a = 0; a < D; ++a) {
            X[a] = node_coord(w, tb[a], cheb[mr[a]]);
            Y[a] = node_coord(w, sb[a], cheb[mc[a]]);
            r2 = fma(Y[a] - X[a], Y[a] - X[a], r2);
        }
        double rr = sqrt(r2);
        double q = ceil(rr / (0.5 * g.h));
        int m = q < 1.0 ? 1 : (int)q;
        double tau = tau_march8(st8, g, 1.0 / g.h, X[0], X[1], X[2], Y[0], Y[1], Y[2], m, rr);
        if (mii) {
            const double hp = (D == 2) ? g.h : g.h * g.h;
            v = exp(-tau) * cell_int(D, (Y[0] - X[0]) / g.h, (Y[1] - X[1]) / g.h, (Y[2] - X[2]) / g.h, 64.0) /
                (surface_area(D) * hp);
        } else {
            double rp = (D == 2) ? rr : r2;
            v = exp(-tau) / (surface_area(D) * rp);
        }
    }
    opsT[i] = T(v);
}


// The same matrices (3D, every grid side > 1) with sigma_t read from LDS.  A
// workgroup takes kOpsLdsRays x kOpsLdsThreads entries of one pair and marches
// them window by window in the ray parameter: window w holds, for a ray of m
// steps, the samples q in (w m / nwin, (w + 1) m / nwin].  Their points lie in
// the box swept by (1 - f) A + f B for f in [w / nwin - 1/(2m), (w + 1) / nwin]
// (A, B the two boxes; the shift below w / nwin is at most half a step, a
// quarter cell), so sigma_t over that box plus one cell of margin on each side
// is staged before the window.  Each ray keeps its running sum across windows:
// the samples are added in the order q = 1 .. m and every value matches
// k_ops_het bit for bit.  A window whose box exceeds the LDS capacity reads
// the corner-octet table instead.
constexpr int kOpsLdsThreads = 512;
constexpr int kOpsLdsRays = 2;
constexpr int kOpsLdsSide = 18;   // cells per axis of a staged box (LDS pitch; 18^3 doubles = 46.7 KB)

template <typename T, bool MII>
__global__ __launch_bounds__(kOpsLdsThreads) void k_ops_het_lds(
    Geo g, const double* __restrict__ st, const double* __restrict__ st8, int nc, int K, int Kp, double w, int nl0,
    int nl1, int nl2, const double* __restrict__ cheb, const int* __restrict__ pair_t, const int* __restrict__ pair_s,
    long p0, int ngroup, int nwin, T* __restrict__ opsT)
{
    constexpr int R = kOpsLdsRays;
    constexpr int P = kOpsLdsSide;
    __shared__ double sl[P * P * P];
    const long pl = blockIdx.x / ngroup;
    const long p = p0 + pl;
    const int gi = (int)(blockIdx.x - pl * ngroup);
    const int per = Kp * Kp;
    const int nl[3] = {nl0, nl1, nl2};
    int tb[3], sb[3];
    unravel3(pair_t[p], nl, tb);
    unravel3(pair_s[p], nl, sb);
    const double inv_h = 1.0 / g.h;
    const int n[3] = {g.n0, g.n1, g.n2};
    const double hi0 = double(n[0] - 1), hi1 = double(n[1] - 1), hi2 = double(n[2] - 1);
    const double km0 = double(n[0] - 2), km1 = double(n[1] - 2), km2 = double(n[2] - 2);

    double ra[R][3], re[R][3], rinv[R], rs[R], rlen[R], r2s[R];
    int rm[R], ri[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int e = gi * (R * kOpsLdsThreads) + j * kOpsLdsThreads + (int)threadIdx.x;
        ri[j] = e;
        rm[j] = 0;
        rs[j] = 0.0;
        rinv[j] = 1.0;
        rlen[j] = 0.0;
        r2s[j] = 0.0;
        for (int a = 0; a < 3; ++a) ra[j][a] = re[j][a] = 0.0;
        const int c = e / Kp, r = e - (e / Kp) * Kp;
        if (e < per && r < K && c < K) {
            int mr[3], mc[3];
            node_multi(r, nc, 3, mr);
            node_multi(c, nc, 3, mc);
            double X[3], Y[3], r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                X[a] = node_coord(w, tb[a], cheb[mr[a]]);
                Y[a] = node_coord(w, sb[a], cheb[mc[a]]);
                r2 = fma(Y[a] - X[a], Y[a] - X[a], r2);
            }
            const double rr = sqrt(r2);
            const double q = ceil(rr / (0.5 * g.h));
            const int m = q < 1.0 ? 1 : (int)q;
            for (int a = 0; a < 3; ++a) {
                ra[j][a] = X[a];
                re[j][a] = Y[a] - X[a];
            }
            rm[j] = m;
            rinv[j] = 1.0 / double(m);
            rlen[j] = rr;
            r2s[j] = r2;
        }
    }

    const double2* q8 = reinterpret_cast<const double2*>(st8);
    for (int wi = 0; wi < nwin; ++wi) {
        const double F0 = double(wi) / nwin, F1 = double(wi + 1) / nwin;
        int kmin[3], ext[3];
        for (int a = 0; a < 3; ++a) {
            const double Al = w * tb[a], d = w * (sb[a] - tb[a]);
            const double l0 = Al + F0 * d, l1 = Al + F1 * d;
            const double lo_pos = l0 < l1 ? l0 : l1;
            const double hi_pos = (l0 > l1 ? l0 : l1) + w;
            int k0 = (int)floor(lo_pos * inv_h - 0.5) - 1;
            int k1 = (int)floor(hi_pos * inv_h - 0.5) + 2;
            k0 = k0 < 0 ? 0 : (k0 > n[a] - 2 ? n[a] - 2 : k0);
            k1 = k1 > n[a] - 1 ? n[a] - 1 : k1;
            k1 = k1 < k0 + 1 ? k0 + 1 : k1;
            kmin[a] = k0;
            ext[a] = k1 - k0 + 1;
        }
        const int nst = ext[0] * ext[1] * ext[2];
        const bool lds = ext[0] <= P && ext[1] <= P && ext[2] <= P;
        __syncthreads();  // the previous window's reads are done
        if (lds) {
            for (int e = threadIdx.x; e < nst; e += kOpsLdsThreads) {
                const int x0 = e % ext[0], x1 = (e / ext[0]) % ext[1], x2 = e / (ext[0] * ext[1]);
                sl[x0 + P * (x1 + P * x2)] =
                    st[(kmin[0] + x0) + (long)n[0] * ((kmin[1] + x1) + (long)n[1] * (kmin[2] + x2))];
            }
        }
        __syncthreads();
        const double off = fma(double(P * P), double(kmin[2]), fma(double(P), double(kmin[1]), double(kmin[0])));
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int m = rm[j];
            const int qa = (wi * m) / nwin + 1, qb = ((wi + 1) * m) / nwin;
            double s = rs[j];
            // one sample: the cell search of sigma_at and its interpolation over the
            // corners c[0], c[dx], c[dy], c[dy + dx], c[dz], ... (LDS box or octet table)
            auto sample = [&](int q, auto corners) {
                const double f = (double(q) - 0.5) * rinv[j];
                const double u0 = fmin(fmax((ra[j][0] + f * re[j][0]) * inv_h - 0.5, 0.0), hi0);
                const double u1 = fmin(fmax((ra[j][1] + f * re[j][1]) * inv_h - 0.5, 0.0), hi1);
                const double u2 = fmin(fmax((ra[j][2] + f * re[j][2]) * inv_h - 0.5, 0.0), hi2);
                const double k0 = fmin(floor(u0), km0), k1 = fmin(floor(u1), km1), k2 = fmin(floor(u2), km2);
                const double t0 = u0 - k0, t1 = u1 - k1, t2 = u2 - k2;
                double v[8];
                corners(k0, k1, k2, v);
                double c00 = v[0] + t0 * (v[1] - v[0]);
                double c10 = v[2] + t0 * (v[3] - v[2]);
                double c0 = c00 + t1 * (c10 - c00);
                double c01 = v[4] + t0 * (v[5] - v[4]);
                double c11 = v[6] + t0 * (v[7] - v[6]);
                double c1 = c01 + t1 * (c11 - c01);
                s += c0 + t2 * (c1 - c0);
            };
            if (lds) {
                auto from_lds = [&](double k0, double k1, double k2, double* v) {
                    const double* c = sl + (int)(fma(double(P * P), k2, fma(double(P), k1, k0)) - off);
                    v[0] = c[0];
                    v[1] = c[1];
                    v[2] = c[P];
                    v[3] = c[P + 1];
                    v[4] = c[P * P];
                    v[5] = c[P * P + 1];
                    v[6] = c[P * P + P];
                    v[7] = c[P * P + P + 1];
                };
                for (int q = qa; q <= qb; ++q) sample(q, from_lds);
            } else {
                auto from_table = [&](double k0, double k1, double k2, double* v) {
                    const unsigned cc = (unsigned)fma(double(n[0]), fma(double(n[1]), k2, k1), k0);
                    const double2* pq = q8 + 4 * (size_t)cc;
                    for (int x = 0; x < 4; ++x) {
                        const double2 d = pq[x];
                        v[2 * x] = d.x;
                        v[2 * x + 1] = d.y;
                    }
                };
                for (int q = qa; q <= qb; ++q) sample(q, from_table);
            }
            rs[j] = s;
        }
    }

    T* out = opsT + pl * (long)per;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int e = ri[j];
        if (e >= per) continue;
        double v = 0.0;
        if (rm[j] > 0) {
            const double tau = rlen[j] * rinv[j] * rs[j];
            if constexpr (MII) {
                const double hp = g.h * g.h;
                v = exp(-tau) * cell_int(3, re[j][0] / g.h, re[j][1] / g.h, re[j][2] / g.h, 64.0) /
                    (surface_area(3) * hp);
            } else {
                v = exp(-tau) / (surface_area(3) * r2s[j]);
            }
        }
        out[e] = T(v);
    }
}

// Windows per pair for k_ops_het_lds at box width w (in cells): the fewest whose
// boxes fit kOpsLdsSide cells per axis for offsets up to 3 boxes; 0 when none up
// to 32 do.
inline int ops_lds_windows(int wc)
{
    for (int nw = 1; nw <= 32; ++nw) {
        const long side = wc + (3L * wc + nw - 1) / nw + 5;
        if (side <= kOpsLdsSide) return nw;
    }
    return 0;
}

// Near-field coupling of two cells of a homogeneous medium at cell offset dv
// (zero for the self pair, whose term is the diagonal's).
__device__ __forceinline__ double near_value(int D, const int dv[3], double h, double sigma, int mii)
{
    const int K = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
    if (K == 0) return 0.0;
    const double r = h * sqrt((double)K);
    if (mii) {
        const double hp = (D == 2) ? h : h * h;
        return exp(-sigma * r) * cell_int(D, dv[0], dv[1], dv[2]) / (surface_area(D) * hp);
    }
    const double rp = (D == 2) ? r : r * r;
    return exp(-sigma * r) / (surface_area(D) * rp);
}

// The same values over all cell offsets of neighbouring leaves, d_a in
// [-(2 leaf - 1), 2 leaf - 1], index sum_a (d_a + 2 leaf - 1) W^a with
// W = 4 leaf - 1, as four copies: copy r holds entry i + r at position i (zero
// past the end), so that any four consecutive entries are one aligned vector
// of some copy.
template <typename T>
__global__ void k_near_tab(int D, int leaf, double h, double sigma, int mii, int tlen, T* __restrict__ tab)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= 4L * tlen) return;
    const int r = (int)(i / tlen);
    const long e = i - (long)r * tlen + r;          // table entry
    const int W = 4 * leaf - 1, c = 2 * leaf - 1;
    const long n = (D == 3) ? (long)W * W * W : (long)W * W;
    double v = 0.0;
    if (e < n) {
        const int dv[3] = {(int)(e % W) - c, (int)((e / W) % W) - c, D == 3 ? (int)(e / ((long)W * W)) - c : 0};
        v = near_value(D, dv, h, sigma, mii);
    }
    tab[i] = T(v);
}

// Near-field blocks of a homogeneous medium: on a uniform grid the block
// between a target leaf and its neighbour at leaf offset o depends only on o.
// ops[o][target i][source i] = G, zero for the self pair.
template <typename T>
__global__ void k_near_ops(int D, int leaf, int S, double h, double sigma, T* __restrict__ ops, int mii)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long per = (long)S * S;
    const int nop = (D == 3) ? 27 : 9;
    if (i >= nop * per) return;
    int oi = (int)(i / per);
    long rem = i - (long)oi * per;
    int it = (int)(rem / S), is = (int)(rem % S);
    int o[3] = {oi % 3 - 1, (oi / 3) % 3 - 1, D == 3 ? oi / 9 - 1 : 0};
    int ls1 = D > 1 ? leaf : 1;
    int lt[3] = {it % leaf, (it / leaf) % ls1, it / (leaf * ls1)};
    int lsr[3] = {is % leaf, (is / leaf) % ls1, is / (leaf * ls1)};
    int dv[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) dv[a] = o[a] * leaf + lsr[a] - lt[a];
    ops[i] = T(near_value(D, dv, h, sigma, mii));
}

// Batched FP64 GEMM with B transposed, for plan-time work:
//   sumbatch: C(i,j) = sum_b sum_k A_b(i,k) B_b(j,k);  else C_b(i,j) = sum_k A_b(i,k) B_b(j,k)
// with arbitrary strides.  64x64 tiles, 4x4 outputs per thread, k-chunks of 16 in LDS.
struct GemmBT {
    int M, N, Kd, nb, sumbatch;
    const double* A; long sAb, sAi, sAk;
    const double* B; long sBb, sBj, sBk;
    double* C; long sCb, sCi, sCj;
};

__global__ __launch_bounds__(256) void k_gemm_bt(GemmBT g)
{
    __shared__ double As[16][65], Bs[16][65];
    const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4] = {};
    const int b_lo = g.sumbatch ? 0 : blockIdx.z, b_hi = g.sumbatch ? g.nb : blockIdx.z + 1;
    for (int b = b_lo; b < b_hi; ++b) {
        const double* A = g.A + (long)b * g.sAb;
        const double* Bm = g.B + (long)b * g.sBb;
        for (int k0 = 0; k0 < g.Kd; k0 += 16) {
            for (int e = threadIdx.x; e < 16 * 64; e += 256) {
                int kk = e / 64, r = e % 64;
                int i = i0 + r, j = j0 + r, k = k0 + kk;
                As[kk][r] = (i < g.M && k < g.Kd) ? A[i * g.sAi + k * g.sAk] : 0.0;
                Bs[kk][r] = (j < g.N && k < g.Kd) ? Bm[j * g.sBj + k * g.sBk] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                double a[4], bb[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = As[kk][ty * 4 + u];
                    bb[u] = Bs[kk][tx * 4 + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * bb[v];
            }
            __syncthreads();
        }
    }
    double* C = g.C + (g.sumbatch ? 0 : (long)blockIdx.z * g.sCb);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int i = i0 + ty * 4 + u, j = j0 + tx * 4 + v;
            if (i < g.M && j < g.N) C[i * g.sCi + j * g.sCj] = acc[u][v];
        }
}

template <typename T>
__global__ void k_cvt(const double* __restrict__ src, T* __restrict__ dst, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = T(src[i]);
}

__global__ void k_cvt_bf16x2(const double* __restrict__ src, __bf16* __restrict__ hi, __bf16* __restrict__ lo, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) {
        float v = (float)src[i];
        __bf16 h = (__bf16)v;
        hi[i] = h;
        lo[i] = (__bf16)(v - (float)h);
    }
}

// ---------------------------------------------------------- host helpers ----

double cheb_T(int k, double x)
{
    double t0 = 1.0, t1 = x;
    if (k == 0) return 1.0;
    for (int i = 1; i < k; ++i) {
        double t2 = 2.0 * x * t1 - t0;
        t0 = t1;
        t1 = t2;
    }
    return t1;
}

// S_n(p, q) for one axis (eq. EQ: CHEB)
double cheb_S(int n, double p, double q)
{
    double s = 1.0 / n;
    for (int k = 1; k < n; ++k) s += 2.0 / n * cheb_T(k, p) * cheb_T(k, q);
    return s;
}

template <typename T>
ert_status upload(hipStream_t s, T** dst, const std::vector<T>& src)
{
    ERT_HIP(hipMalloc(dst, std::max<size_t>(1, src.size()) * sizeof(T)));
    ERT_HIP(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    ERT_HIP(hipStreamSynchronize(s));
    return ERT_OK;
}

template <typename T>
ert_status upload_cvt(hipStream_t s, T** dst, const std::vector<double>& src)
{
    std::vector<T> tmp(src.size());
    for (size_t i = 0; i < src.size(); ++i) tmp[i] = T(src[i]);
    return upload<T>(s, dst, tmp);
}

inline unsigned blocks(long n) { return (unsigned)((n + kB - 1) / kB); }

ert_status gemm_bt(hipStream_t s, const GemmBT& g)
{
    dim3 grid((unsigned)((g.M + 63) / 64), (unsigned)((g.N + 63) / 64), g.sumbatch ? 1u : (unsigned)g.nb);
    hipLaunchKernelGGL(k_gemm_bt, grid, dim3(256), 0, s, g);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

struct DevPtrs {
    std::vector<void*> p;
    ~DevPtrs()
    {
        for (void* q : p)
            if (q) (void)hipFree(q);
    }
    template <typename T>
    ert_status alloc(T** out, size_t n)
    {
        *out = nullptr;
        if (hipMalloc(out, std::max<size_t>(1, n) * sizeof(T)) != hipSuccess) {
            record_error("FMM: device allocation failed during setup");
            return ERT_ENOMEM;
        }
        p.push_back(*out);
        return ERT_OK;
    }
};

}  // namespace

void sym_eig(int n, const std::vector<double>& A, std::vector<double>& w, std::vector<double>& Z);

namespace {

// One box-offset product of the apply (near field, or the far field of a
// level) with both execution forms and the autotuned choice between them.
struct GemmSite {
    bool used = false;
    PairTiles pl;                         // device arrays of the offset-stationary form
    std::vector<int> h_gstart;            // host copy, to rebuild tiles for a larger rhs capacity
    // per rhs bucket (1, >1): 0 class GEMM; offset-stationary with 1: 32 x 16 tiles per
    // workgroup wave set, 2: 32 x 64, 3: 16 x 64 (twice the workgroups of 2)
    int choice[2] = {-1, -1};
    float tuned_ms[2][kForms] = {};
    void release()
    {
        auto f = [](void* p) { if (p) (void)hipFree(p); };
        f(pl.pt); f(pl.ps); f(pl.gstart); f(pl.gop); f(pl.tile_group); f(pl.tile_col0); f(pl.tstart); f(pl.tpairs);
        f(pl.tile_group4); f(pl.tile_col04); f(pl.tpad); f(pl.tcnt);
        pl = PairTiles();
    }
};

// Pairs of a lattice grouped by offset (offsets in lexicographic order, targets
// lexicographic within an offset).  far: offsets in [-3,3]^d outside the
// neighbour cube with parent adjacency; otherwise the 3^d neighbour offsets.
ert_status build_site(hipStream_t s, int D, const int nl[3], bool far, GemmSite& site)
{
    std::vector<int> pt, ps, gstart, gop;
    const int lo = far ? -3 : -1, hi = far ? 3 : 1, side = far ? kOffSide : 3;
    long nbox = (long)nl[0] * nl[1] * nl[2];
    for (int oz = (D > 2 ? lo : 0); oz <= (D > 2 ? hi : 0); ++oz)
        for (int oy = lo; oy <= hi; ++oy)
            for (int ox = lo; ox <= hi; ++ox) {
                const int o[3] = {ox, oy, oz};
                if (far && ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1 && oz >= -1 && oz <= 1) continue;
                const int op = (ox - lo) + side * ((oy - lo) + (D > 2 ? side * (oz - lo) : 0));
                const size_t before = pt.size();
                for (long t = 0; t < nbox; ++t) {
                    int t3[3];
                    unravel3(t, nl, t3);
                    bool ok = true;
                    int s3[3];
                    for (int a = 0; a < 3; ++a) {
                        s3[a] = t3[a] + o[a];
                        if (s3[a] < 0 || s3[a] >= nl[a]) ok = false;
                        if (far && std::abs((t3[a] >> 1) - (s3[a] >> 1)) > 1) ok = false;
                    }
                    if (!ok) continue;
                    pt.push_back((int)t);
                    ps.push_back((int)(s3[0] + (long)nl[0] * (s3[1] + (long)nl[1] * s3[2])));
                }
                if (pt.size() > before) {
                    gstart.push_back((int)before);
                    gop.push_back(op);
                }
            }
    gstart.push_back((int)pt.size());
    const long np = (long)pt.size();
    std::vector<int> tstart(nbox + 1, 0), tpairs(np), fill(nbox, 0);
    for (long p = 0; p < np; ++p) tstart[pt[p] + 1]++;
    for (long t = 0; t < nbox; ++t) tstart[t + 1] += tstart[t];
    for (long p = 0; p < np; ++p) tpairs[tstart[pt[p]] + fill[pt[p]]++] = (int)p;
    site.release();
    site.pl.npairs = np;
    site.pl.ngroups = (int)gop.size();
    site.h_gstart = gstart;
    ERT_TRY(upload<int>(s, &site.pl.pt, pt));
    ERT_TRY(upload<int>(s, &site.pl.ps, ps));
    ERT_TRY(upload<int>(s, &site.pl.gstart, gstart));
    ERT_TRY(upload<int>(s, &site.pl.gop, gop));
    ERT_TRY(upload<int>(s, &site.pl.tstart, tstart));
    ERT_TRY(upload<int>(s, &site.pl.tpairs, tpairs));
    if (nbox <= kPadPairs) {
        std::vector<int> pad((size_t)nbox * kPadPairs, -1), cnt(nbox);
        for (long t = 0; t < nbox; ++t) {
            cnt[t] = tstart[t + 1] - tstart[t];
            for (int k = 0; k < cnt[t]; ++k) pad[(size_t)t * kPadPairs + k] = tpairs[tstart[t] + k];
        }
        ERT_TRY(upload<int>(s, &site.pl.tpad, pad));
        ERT_TRY(upload<int>(s, &site.pl.tcnt, cnt));
    }
    site.used = true;
    return ERT_OK;
}

// column tiles (16 pair-rhs columns each) for a rhs capacity B
ert_status build_tiles(hipStream_t s, GemmSite& site, int B)
{
    for (int width : {16, 64}) {
        std::vector<int> tg, tc;
        for (int g = 0; g + 1 < (int)site.h_gstart.size(); ++g) {
            const long ncols = (long)(site.h_gstart[g + 1] - site.h_gstart[g]) * B;
            for (long c = 0; c < ncols; c += width) {
                tg.push_back(g);
                tc.push_back((int)c);
            }
        }
        int** grp = width == 16 ? &site.pl.tile_group : &site.pl.tile_group4;
        int** col = width == 16 ? &site.pl.tile_col0 : &site.pl.tile_col04;
        if (*grp) (void)hipFree(*grp);
        if (*col) (void)hipFree(*col);
        *grp = *col = nullptr;
        ERT_TRY(upload<int>(s, grp, tg));
        ERT_TRY(upload<int>(s, col, tc));
        (width == 16 ? site.pl.ntiles : site.pl.ntiles4) = (long)tg.size();
    }
    return ERT_OK;
}

template <typename T>
struct FmmImpl : FmmData {
    int prec = ERT_FP64;
    bool hetero = false;
    bool compress = false;
    int B = 0;                      // rhs capacity of the work buffers
    DevTree dt{};
    T* P1 = nullptr;                // [nc][leaf]
    T* M1 = nullptr;                // [2][nc][nc]
    double* cheb = nullptr;         // nodes (FP64, for operator generation)
    BoxOffset* m2l_offs = nullptr;  // [2^d classes][noff]
    int m2l_noff = 0;
    BoxOffset* near_offs = nullptr; // [3^d]
    BoxOffset* id_off = nullptr;    // [1]: the zero offset
    void* ops[kMaxLevels + 1] = {};     // far translations [7^d][M][M] (bf16 high parts for BF16X3)
    __bf16* ops_lo[kMaxLevels + 1] = {};
    int rp[kMaxLevels + 1] = {};        // compressed rank (padded), 0 = uncompressed
    T* Ut[kMaxLevels + 1] = {};         // [rp][Kp]: multipoles -> compressed
    T* Um[kMaxLevels + 1] = {};         // [Kp][rp]: compressed locals -> locals
    // A tree whose leaves are the only far-field level (L = 2) with compressed
    // translations: P2M and the compression fold into one [rp][S] matrix, the
    // expansion and L2P into one [S][rp] matrix (each applied as one GEMM).
    T* leaf_in = nullptr;               // [rp][S] = Ut P
    T* leaf_out = nullptr;              // [S][rp] = P^T Um
    T* leaf_inT = nullptr;              // [S][rp], leaf_in transposed
    T* leaf_outT = nullptr;             // [rp][S], leaf_out transposed
    HetCache* hc = nullptr;             // heterogeneous caches (owned by the plan)
    T* nearops = nullptr;               // homogeneous near blocks [3^d][S][S]
    T* neartab = nullptr;               // the same values over cell offsets, [4][near_tlen]
    int near_tlen = 0;
    T* tab = nullptr;                   // homogeneous near table (S not a multiple of 32)
    int ntab = 0;
    T* q = nullptr;
    T* pot = nullptr;
    T* W[kMaxLevels + 1] = {};
    T* Lc[kMaxLevels + 1] = {};
    T* Wc[kMaxLevels + 1] = {};         // compressed multipoles
    T* Lh[kMaxLevels + 1] = {};         // compressed locals
    GemmSite far_site[kMaxLevels + 1];  // far field of level l >= 2 (homogeneous)
    GemmSite near_site;                 // near field (homogeneous)
    ApplyIO* io = nullptr;              // device: vectors of the current apply
    ApplyIO cur{};                      // host: vectors of the apply being enqueued
    // the first kernel of an enqueued apply, with its arguments, so that the root node
    // of a captured apply can be given the vectors of each replay
    struct GatherArgs {
        ApplyIO a; ApplyIO* io; DevTree t; const double* ss; long N; int B; T* q;
    };
    struct LeafInArgs {
        ApplyIO a; ApplyIO* io; DevTree t; const double* ss; long N; const T* linT; int R; int rch; T* q; T* W;
    };
    struct FirstLaunch {
        int kind = 0;                   // 1 k_gather, 2 k_leaf_in
        const void* func = nullptr;
        dim3 grid, block;
        size_t shmem = 0;
        GatherArgs g{};
        LeafInArgs l{};
    };
    FirstLaunch first;                  // of the most recent enqueue
    FirstLaunch gfirst[2];              // of the captured applies
    hipGraphNode_t groot[2] = {};
    hipStream_t cap = nullptr;          // internal stream used only to capture graphs
    hipGraph_t graph[2] = {};           // captured applies, per rhs bucket (1, >1)
    hipGraphExec_t gexec[2] = {};
    int graph_nrhs[2] = {0, 0};
    int calls[2] = {0, 0};
    bool no_graph[2] = {false, false};  // the captured apply had an unexpected root: run eagerly
    T* stage = nullptr;                 // staging rows of the far-field products
    T* stage_near = nullptr;            // staging rows of the near-field products (runs concurrently)
    size_t stage_near_elems = 0;
    // the near field and the far-field passes are independent until L2P: after the
    // first (tuning) apply of a rhs bucket the near field runs on a second stream,
    // forked from and joined back to the apply's stream (also inside captured graphs)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool tuned[2] = {false, false};
    T* tune = nullptr;                  // scratch output while autotuning
    size_t stage_elems = 0, tune_elems = 0;

    ~FmmImpl() override
    {
        auto f = [](void* p) { if (p) (void)hipFree(p); };
        f(P1); f(M1); f(cheb); f(m2l_offs); f(near_offs); f(id_off); f(nearops); f(neartab); f(tab); f(q); f(pot); f(leaf_in); f(leaf_out); f(leaf_inT); f(leaf_outT);
        for (int l = 0; l <= kMaxLevels; ++l) {
            f(ops[l]); f(ops_lo[l]); f(Ut[l]); f(Um[l]);
            f(W[l]); f(Lc[l]); f(Wc[l]); f(Lh[l]);
            far_site[l].release();
        }
        near_site.release();
        f(stage); f(stage_near); f(tune); f(io);
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        if (side) (void)hipStreamDestroy(side);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
    }

    ert_status run_site(ert_plan_impl* p, hipStream_t s, GemmSite& site, int gprec, const BoxGemm& g, int nrhs,
                        StageTimer* outer, T* stg);
    // offset-stationary description of a box-offset product in the form `form` (1..5)
    OffsetGemm offset_of(const GemmSite& gs, const BoxGemm& b, T* stg, int form) const
    {
        OffsetGemm o;
        o.nbox = b.nbox;
        o.B = b.B;
        o.M = b.M;
        o.Kd = b.Kd;
        o.ops = b.ops;
        o.ops_lo = b.ops_lo;
        o.W = b.W;
        o.L = b.L;
        o.stage = stg;
        o.accumulate = b.accumulate;
        o.tn = (form == 2 || form == 3) ? 4 : 1;
        o.tm = form == 3 ? 1 : 2;
        o.lds = form == 4 ? 1 : form == 5 ? 2 : 0;
        o.pl = gs.pl;
        if (&gs == &near_site && neartab && b.ops == nearops) {
            o.atab = neartab;
            o.tlen = near_tlen;
            o.tw = 4 * tr.leaf - 1;
            o.leaf = tr.leaf;
            while ((1 << o.lshift) < tr.leaf) ++o.lshift;
            o.dim = tr.D;
        }
        return o;
    }
    ert_status enqueue_grouped(ert_plan_impl* p, hipStream_t s, int nrhs);
    ert_status set_root_args(int bucket);
    ert_status enqueue(ert_plan_impl* p, hipStream_t s, int nrhs);
    void drop_graphs()
    {
        for (int b = 0; b < 2; ++b) {
            if (gexec[b]) (void)hipGraphExecDestroy(gexec[b]);
            if (graph[b]) (void)hipGraphDestroy(graph[b]);
            gexec[b] = nullptr;
            graph[b] = nullptr;
            graph_nrhs[b] = 0;
            groot[b] = nullptr;
        }
    }

    int rank_of(int l) const override { return rp[l]; }
    bool far_rebuilt(int l) const override { return hc && l >= 0 && l <= kMaxLevels && hc->rebuilt[l]; }
    double cache_bytes() const override { return hc ? (double)hc->bytes : 0.0; }
    long near_table() const override
    {
        const long W = 4L * tr.leaf - 1;
        return neartab ? (tr.D == 3 ? W * W * W : W * W) : 0;
    }
    int form_of(int site) const override
    {
        const GemmSite& gs = site < 0 ? near_site : far_site[site];
        return gs.used ? gs.choice[0] : -1;
    }
    ert_status setup(ert_plan_impl* p) override;
    ert_status setup_far_hom(ert_plan_impl* p, int l, double svd_tol);
    ert_status setup_het(ert_plan_impl* p);
    ert_status ensure_buffers(int nrhs);
    hipStream_t p_stream = nullptr;
    ert_status apply(ert_plan_impl* p, int op, const double* x, double* y, int nrhs) override;

    // one-level homogeneous trees whose tuned near and far products are both
    // offset-stationary run as three fused launches
    bool grouped_form(int bk) const
    {
        return !hetero && leaf_inT && leaf_outT && nearops && tr.L == 2 && tr.nbox[2] <= kLeafMaxPairs &&
               near_site.pl.tpad && far_site[2].pl.tpad &&
               rp[2] <= 64 * kLeafWaves && near_site.used && far_site[2].used &&
               near_site.choice[bk] >= 1 && far_site[2].choice[bk] >= 1;
    }

    BoxGemm gemm_desc(int l, int Mrows, int Kd, int nrhs) const
    {
        BoxGemm g{};
        g.D = tr.D;
        for (int d = 0; d < 3; ++d) g.nl[d] = tr.nl[l][d];
        g.nbox = tr.nbox[l];
        g.B = nrhs;
        g.M = Mrows;
        g.Kd = Kd;
        return g;
    }
};

// Build the tree geometry for a plan.
FmmTree make_tree(const ert_plan_impl* p, int prec)
{
    FmmTree t;
    t.D = p->o.dim;
    t.nc = p->o.cheb_n > 0 ? p->o.cheb_n : 8;
    if (prec != ERT_FP64 && p->o.inner_cheb_n > 0) t.nc = p->o.inner_cheb_n;
    t.K = 1;
    for (int a = 0; a < t.D; ++a) t.K *= t.nc;
    t.Kp = (t.K + 31) / 32 * 32;
    t.leaf = p->o.leaf > 0 ? p->o.leaf : 8;
    t.S = 1;
    for (int a = 0; a < t.D; ++a) t.S *= t.leaf;
    const int n[3] = {p->geo.n0, p->geo.n1, p->geo.n2};
    int mx = 1;
    t.nleaf = 1;
    for (int a = 0; a < 3; ++a) {
        t.nb[a] = (a < t.D) ? (n[a] + t.leaf - 1) / t.leaf : 1;
        mx = std::max(mx, t.nb[a]);
        t.nleaf *= t.nb[a];
    }
    t.nslot = t.nleaf * t.S;
    t.L = 0;
    while ((1 << t.L) < mx) ++t.L;
    for (int l = 0; l <= t.L && l <= kMaxLevels; ++l) {
        t.nbox[l] = 1;
        for (int a = 0; a < 3; ++a) {
            int f = 1 << (t.L - l);
            t.nl[l][a] = (a < t.D) ? (t.nb[a] + f - 1) / f : 1;
            t.nbox[l] *= t.nl[l][a];
        }
        t.width[l] = p->geo.h * t.leaf * (double)(1 << (t.L - l));
    }
    return t;
}

// Homogeneous far field of level l: translation matrices for every box offset
// in [-3,3]^d (FP64 on the GPU); optionally compressed with the orthonormal
// basis U of the dominant left singular vectors of [M_o1 M_o2 ...] (which are
// also the right ones, the kernel being symmetric): M_o ~ U (U^T M_o U) U^T.
template <typename T>
ert_status FmmImpl<T>::setup_far_hom(ert_plan_impl* p, int l, double svd_tol)
{
    hipStream_t s = p->stream;
    const int Kp = tr.Kp;
    int noff = 1;
    for (int a = 0; a < tr.D; ++a) noff *= kOffSide;
    const long KpKp = (long)Kp * Kp;
    DevPtrs tmp;
    double* M64 = nullptr;
    ERT_TRY(tmp.alloc(&M64, (size_t)noff * KpKp));
    hipLaunchKernelGGL(k_ops_hom<double>, dim3(blocks(noff * KpKp)), dim3(kB), 0, s, tr.D, tr.nc, tr.K, Kp,
                       tr.width[l], p->sigma_const, cheb, M64, (__bf16*)nullptr, p->o.scheme, p->geo.h);
    ERT_HIP(hipGetLastError());
    const double* Cd = M64;
    int M = Kp;
    if (svd_tol >= 0.0) {
        // Gram matrix sum_o M_o M_o^T (near offsets are zero matrices)
        double* gram = nullptr;
        ERT_TRY(tmp.alloc(&gram, (size_t)KpKp));
        GemmBT g{Kp, Kp, Kp, noff, 1, M64, KpKp, Kp, 1, M64, KpKp, Kp, 1, gram, 0, Kp, 1};
        ERT_TRY(gemm_bt(s, g));
        std::vector<double> G((size_t)KpKp), w, Z;
        ERT_HIP(hipMemcpyAsync(G.data(), gram, KpKp * sizeof(double), hipMemcpyDeviceToHost, s));
        ERT_HIP(hipStreamSynchronize(s));
        sym_eig(Kp, G, w, Z);
        const double wmax = w.empty() ? 0.0 : w[0];
        int r = 0;
        while (r < Kp && w[r] > 0.0 && std::sqrt(w[r] / wmax) > svd_tol) ++r;
        if (r < 1) r = 1;
        const int R = std::min(Kp, (r + 31) / 32 * 32);
        std::vector<double> Uh((size_t)Kp * R, 0.0);
        for (int i = 0; i < Kp; ++i)
            for (int c = 0; c < r; ++c) Uh[(size_t)i * R + c] = Z[(size_t)i * Kp + c];
        double* U64 = nullptr;
        ERT_TRY(tmp.alloc(&U64, Uh.size()));
        ERT_HIP(hipMemcpyAsync(U64, Uh.data(), Uh.size() * sizeof(double), hipMemcpyHostToDevice, s));
        // T_o = M_o U (Kp x R), C_o = U^T T_o (R x R)
        double *T1 = nullptr, *C64 = nullptr;
        ERT_TRY(tmp.alloc(&T1, (size_t)noff * Kp * R));
        ERT_TRY(tmp.alloc(&C64, (size_t)noff * R * R));
        GemmBT g1{Kp, R, Kp, noff, 0, M64, KpKp, Kp, 1, U64, 0, 1, R, T1, (long)Kp * R, R, 1};
        ERT_TRY(gemm_bt(s, g1));
        GemmBT g2{R, R, Kp, noff, 0, U64, 0, 1, R, T1, (long)Kp * R, 1, R, C64, (long)R * R, R, 1};
        ERT_TRY(gemm_bt(s, g2));
        // change-of-basis matrices in the working precision
        std::vector<double> Ut_h((size_t)R * Kp);
        for (int c = 0; c < R; ++c)
            for (int i = 0; i < Kp; ++i) Ut_h[(size_t)c * Kp + i] = Uh[(size_t)i * R + c];
        ERT_TRY(upload_cvt<T>(s, &Ut[l], Ut_h));
        ERT_TRY(upload_cvt<T>(s, &Um[l], Uh));
        rp[l] = R;
        if (l == 2 && tr.L == 2 && tr.S % 32 == 0) {
            // dense leaf interpolation P[m][j] = prod_a S_n(x_{j_a}, node_{m_a}) (the separable
            // P2M/L2P operator), folded with the basis change
            std::vector<double> node(tr.nc), P1h((size_t)tr.nc * tr.leaf);
            for (int m = 0; m < tr.nc; ++m) node[m] = std::cos((2.0 * m + 1.0) * kPi / (2.0 * tr.nc));
            for (int m = 0; m < tr.nc; ++m)
                for (int i = 0; i < tr.leaf; ++i)
                    P1h[(size_t)m * tr.leaf + i] = cheb_S(tr.nc, (2.0 * i + 1.0) / tr.leaf - 1.0, node[m]);
            const int S = tr.S;
            std::vector<double> P((size_t)Kp * S, 0.0);
            for (int m = 0; m < tr.K; ++m) {
                int mm[3] = {m % tr.nc, tr.D > 1 ? (m / tr.nc) % tr.nc : 0, tr.D > 2 ? m / (tr.nc * tr.nc) : 0};
                for (int j = 0; j < S; ++j) {
                    int jj[3] = {j % tr.leaf, tr.D > 1 ? (j / tr.leaf) % tr.leaf : 0,
                                 tr.D > 2 ? j / (tr.leaf * tr.leaf) : 0};
                    double v = 1.0;
                    for (int a = 0; a < tr.D; ++a) v *= P1h[(size_t)mm[a] * tr.leaf + jj[a]];
                    P[(size_t)m * S + j] = v;
                }
            }
            std::vector<double> fin((size_t)R * S, 0.0), fout((size_t)S * R, 0.0);
            for (int c = 0; c < R; ++c)
                for (int m = 0; m < tr.K; ++m) {
                    const double u = Ut_h[(size_t)c * Kp + m];
                    if (u == 0.0) continue;
                    const double* pm = &P[(size_t)m * S];
                    double* fc = &fin[(size_t)c * S];
                    for (int j = 0; j < S; ++j) fc[j] += u * pm[j];
                }
            for (int m = 0; m < tr.K; ++m) {
                const double* pm = &P[(size_t)m * S];
                const double* um = &Uh[(size_t)m * R];
                for (int j = 0; j < S; ++j) {
                    const double pj = pm[j];
                    double* fj = &fout[(size_t)j * R];
                    for (int c = 0; c < R; ++c) fj[c] += pj * um[c];
                }
            }
            ERT_TRY(upload_cvt<T>(s, &leaf_in, fin));
            ERT_TRY(upload_cvt<T>(s, &leaf_out, fout));
            // transposed copies for the fused one-level apply (lanes over outputs)
            std::vector<double> tin((size_t)S * R), tout((size_t)R * S);
            for (int c = 0; c < R; ++c)
                for (int j = 0; j < S; ++j) {
                    tin[(size_t)j * R + c] = fin[(size_t)c * S + j];
                    tout[(size_t)c * S + j] = fout[(size_t)j * R + c];
                }
            ERT_TRY(upload_cvt<T>(s, &leaf_inT, tin));
            ERT_TRY(upload_cvt<T>(s, &leaf_outT, tout));
        }
        Cd = C64;
        M = R;
    }
    const long n = (long)noff * M * M;
    if (prec == ERT_BF16X3) {
        ERT_HIP(hipMalloc(&ops[l], n * sizeof(__bf16)));
        ERT_HIP(hipMalloc(&ops_lo[l], n * sizeof(__bf16)));
        hipLaunchKernelGGL(k_cvt_bf16x2, dim3(blocks(n)), dim3(kB), 0, s, Cd, (__bf16*)ops[l], ops_lo[l], n);
    } else {
        ERT_HIP(hipMalloc(&ops[l], n * sizeof(T)));
        hipLaunchKernelGGL(k_cvt<T>, dim3(blocks(n)), dim3(kB), 0, s, Cd, (T*)ops[l], n);
    }
    ERT_HIP(hipGetLastError());
    ERT_HIP(hipStreamSynchronize(s));
    return ERT_OK;
}

// Heterogeneous far field of level l: the directed interaction-list pairs grouped by
// target (the staging rows), and one stored matrix per unordered pair {t, s}, t < s,
// for target t and source s (the transpose serves target s).
// The corner-octet table of the plan's sigma_t, held while the caches are built
// (8 doubles per cell); the stream is drained before it is released.
struct CornerTable {
    double* st8 = nullptr;
    hipStream_t s = nullptr;
    ert_status build(ert_plan_impl* p)
    {
        s = p->stream;
        const long n = p->N;
        if (hipMalloc(&st8, std::max<size_t>(1, (size_t)n * 8 * sizeof(double))) != hipSuccess) {
            st8 = nullptr;
            record_error("FMM: sigma_t corner table allocation failed");
            return ERT_ENOMEM;
        }
        hipLaunchKernelGGL(k_corner8, dim3(blocks(n)), dim3(kB), 0, s, p->geo, p->d_st, st8, n);
        return hipGetLastError() == hipSuccess ? ERT_OK : ERT_EDEVICE;
    }
    // hand the table to the caller (levels rebuilt by every apply keep it)
    double* release()
    {
        double* q = st8;
        st8 = nullptr;
        return q;
    }
    ~CornerTable()
    {
        if (!st8) return;
        (void)hipStreamSynchronize(s);
        (void)hipFree(st8);
    }
};

// Translation matrices of stored pairs p0 .. p0 + cnt - 1 of level l into dst
// ([cnt][Kp][Kp]): kernel launches on the stream only (also used inside applies
// for the levels that are rebuilt each time).
ert_status het_fill(ert_plan_impl* p, hipStream_t s, const FmmTree& tr, const double* cheb, const double* st8,
                    const HetCache* hc, int l, long p0, long cnt, float* dst)
{
    const long KpKp = (long)tr.Kp * tr.Kp;
    const long pchunk = std::max<long>(1, (1L << 27) / KpKp);
    const Geo& g = p->geo;
    const int nl[3] = {tr.nl[l][0], tr.nl[l][1], tr.nl[l][2]};
    const int nwin = (tr.D == 3 && g.n0 > 1 && g.n1 > 1 && g.n2 > 1) ? ops_lds_windows(tr.leaf << (tr.L - l)) : 0;
    const long ngroup = (KpKp + kOpsLdsRays * kOpsLdsThreads - 1) / (kOpsLdsRays * kOpsLdsThreads);
    for (long q0 = p0; q0 < p0 + cnt; q0 += pchunk) {
        const long c = std::min(pchunk, p0 + cnt - q0);
        float* out = dst + (size_t)(q0 - p0) * KpKp;
        if (nwin > 0) {
            auto kern = p->o.scheme ? k_ops_het_lds<float, true> : k_ops_het_lds<float, false>;
            hipLaunchKernelGGL(kern, dim3((unsigned)(c * ngroup)), dim3(kOpsLdsThreads), 0, s, g, p->d_st, st8, tr.nc,
                               tr.K, tr.Kp, tr.width[l], nl[0], nl[1], nl[2], cheb, hc->hua[l], hc->hub[l], q0,
                               (int)ngroup, nwin, out);
        } else {
            hipLaunchKernelGGL(k_ops_het<float>, dim3(blocks(c * KpKp)), dim3(kB), 0, s, g, st8, tr.D, tr.nc, tr.K,
                               tr.Kp, tr.width[l], nl[0], nl[1], nl[2], cheb, hc->hua[l], hc->hub[l], q0, c, out,
                               p->o.scheme);
        }
        ERT_HIP(hipGetLastError());
    }
    return ERT_OK;
}

// On-demand translation matrices of a rebuilt level, for pair_stream.
struct HetGenCtx {
    ert_plan_impl* p;
    const FmmTree* tr;
    const double* cheb;
    const HetCache* hc;
    int l;
};

ert_status het_gen_fill(const void* ctx, hipStream_t s, long p0, long cnt, float* dst)
{
    const HetGenCtx* c = static_cast<const HetGenCtx*>(ctx);
    return het_fill(c->p, s, *c->tr, c->cheb, c->hc->st8, c->hc, c->l, p0, cnt, dst);
}

ert_status het_far_level(ert_plan_impl* p, const FmmTree& tr, const double* cheb, const double* st8, HetCache* hc,
                         int l)
{
    hipStream_t s = p->stream;
    const long KpKp = (long)tr.Kp * tr.Kp;
    std::vector<long> start(tr.nbox[l] + 1, 0);
    std::vector<int> src;
    const int* nl = tr.nl[l];
    for (long tb = 0; tb < tr.nbox[l]; ++tb) {
        int t3[3];
        unravel3(tb, nl, t3);
        start[tb] = (long)src.size();
        for (int oz = (tr.D > 2 ? -3 : 0); oz <= (tr.D > 2 ? 3 : 0); ++oz)
            for (int oy = -3; oy <= 3; ++oy)
                for (int ox = -3; ox <= 3; ++ox) {
                    int o[3] = {ox, oy, oz}, s3[3];
                    bool ok = true, adjacent = true;
                    for (int a = 0; a < 3; ++a) {
                        s3[a] = t3[a] + o[a];
                        if (s3[a] < 0 || s3[a] >= nl[a]) ok = false;
                        if ((t3[a] >> 1) - (s3[a] >> 1) > 1 || (s3[a] >> 1) - (t3[a] >> 1) > 1) ok = false;
                        if (o[a] < -1 || o[a] > 1) adjacent = false;
                    }
                    if (!ok || adjacent) continue;
                    src.push_back((int)(s3[0] + (long)nl[0] * (s3[1] + (long)nl[1] * s3[2])));
                }
    }
    start[tr.nbox[l]] = (long)src.size();
    const long nd = (long)src.size();
    // unordered pairs: the directed pair (t, s) with t < s, and the row of (s, t)
    std::vector<int> ua, ub;
    std::vector<long> fwd, bwd;
    for (long tb = 0; tb < tr.nbox[l]; ++tb)
        for (long k = start[tb]; k < start[tb + 1]; ++k) {
            const int sb = src[k];
            if (sb <= tb) continue;
            long back = -1;
            for (long q = start[sb]; q < start[sb + 1]; ++q)
                if (src[q] == (int)tb) back = q;
            if (back < 0) {
                record_error("FMM: interaction lists are not symmetric");
                return ERT_EINVAL;
            }
            ua.push_back((int)tb);
            ub.push_back(sb);
            fwd.push_back(k);
            bwd.push_back(back);
        }
    const long np = (long)ua.size();
    if (2 * np != nd) {
        record_error("FMM: interaction lists are not symmetric");
        return ERT_EINVAL;
    }
    hc->hnp[l] = np;
    hc->hnd[l] = nd;
    ERT_TRY(upload<long>(s, &hc->pstart[l], start));
    ERT_TRY(upload<int>(s, &hc->hua[l], ua));
    ERT_TRY(upload<int>(s, &hc->hub[l], ub));
    ERT_TRY(upload<long>(s, &hc->hfwd[l], fwd));
    ERT_TRY(upload<long>(s, &hc->hbwd[l], bwd));
    const size_t bytes = (size_t)np * KpKp * sizeof(float);
    // budget of the stored translation matrices: the plan's option, else 90 % of the
    // free device memory; both orders' caches count against it
    size_t fr = 0, tot = 0;
    ERT_HIP(hipMemGetInfo(&fr, &tot));
    size_t avail = fr / 10 * 9;
    if (p->o.far_cache_gb > 0.0) {
        size_t used = hc->far_bytes;
        for (int i = 0; i < 2; ++i)
            if (p->het[i] && p->het[i] != hc) used += p->het[i]->far_bytes;
        const double lim = p->o.far_cache_gb * 1e9;
        const size_t left = lim > (double)used ? (size_t)(lim - (double)used) : 0;
        avail = std::min(avail, left);
    }
    const size_t block = (size_t)KpKp * sizeof(float);
    if (bytes <= avail && hipMalloc(&hc->hops[l], std::max<size_t>(1, bytes)) == hipSuccess) {
        ERT_TRY(het_fill(p, s, tr, cheb, st8, hc, l, 0, np, hc->hops[l]));
        hc->hstored[l] = np;
        hc->bytes += bytes;
        hc->far_bytes += bytes;
    } else {
        // the first pairs that fit are stored; every apply rebuilds the others through
        // a scratch buffer of whole blocks (1/16 of the room, at least one block, at
        // most 2 GB, shared by the levels)
        (void)hipGetLastError();
        hc->hops[l] = nullptr;
        hc->rebuilt[l] = true;
        const size_t sbytes = std::max(block, std::min<size_t>(avail / 16, size_t(2) << 30));
        const long chunk = (long)std::min<size_t>((size_t)np, sbytes / block);
        if (chunk > hc->chunk) {
            if (hc->scratch) {
                (void)hipFree(hc->scratch);
                hc->bytes -= (size_t)hc->chunk * block;
            }
            hc->scratch = nullptr;
            hc->chunk = 0;
            if (hipMalloc(&hc->scratch, (size_t)chunk * block) != hipSuccess) {
                record_error("FMM: scratch for the rebuilt translation matrices could not be allocated");
                return ERT_ENOMEM;
            }
            hc->chunk = chunk;
            hc->bytes += (size_t)chunk * block;
        }
        const size_t room = avail > (size_t)chunk * block ? avail - (size_t)chunk * block : 0;
        long ns = (long)std::min<size_t>((size_t)(np - 1), room / block);
        if (ns > 0 && hipMalloc(&hc->hops[l], (size_t)ns * block) != hipSuccess) {
            (void)hipGetLastError();
            hc->hops[l] = nullptr;
            ns = 0;
        }
        if (ns > 0) {
            ERT_TRY(het_fill(p, s, tr, cheb, st8, hc, l, 0, ns, hc->hops[l]));
            hc->bytes += (size_t)ns * block;
            hc->far_bytes += (size_t)ns * block;
        }
        hc->hstored[l] = ns;
    }
    ERT_HIP(hipStreamSynchronize(s));
    return ERT_OK;
}

// Heterogeneous caches of the plan (built by the first precision that needs them).
template <typename T>
ert_status FmmImpl<T>::setup_het(ert_plan_impl* p)
{
    HetCache* other = nullptr;
    int slot = -1;
    for (int i = 0; i < 2; ++i) {
        HetCache* c = p->het[i];
        if (!c) {
            if (slot < 0) slot = i;
            continue;
        }
        if (c->leaf != tr.leaf) {
            record_error("FMM: heterogeneous cache built for another leaf size");
            return ERT_EINVAL;
        }
        if (c->nc == tr.nc) {
            hc = c;
            return ERT_OK;
        }
        other = c;
    }
    if (slot < 0) {
        record_error("FMM: no free heterogeneous cache slot");
        return ERT_EINVAL;
    }
    hipStream_t s = p->stream;
    HetCache* c = new (std::nothrow) HetCache();
    if (!c) return ERT_ENOMEM;
    c->nc = tr.nc;
    c->leaf = tr.leaf;
    auto fail = [&](ert_status e) { delete c; return e; };
    const int nn = tr.D == 3 ? 27 : 9;
    if (other) {
        // the near field does not depend on the Chebyshev order: share it
        c->owns_near = false;
        c->near_hi = other->near_hi;
        c->near_lo = other->near_lo;
        c->near_src = other->near_src;
        c->near_tstart = other->near_tstart;
        c->near_np = other->near_np;
        c->near_ua = other->near_ua;
        c->near_ub = other->near_ub;
        c->near_fwd = other->near_fwd;
        c->near_bwd = other->near_bwd;
        CornerTable t8;
        ert_status st = t8.build(p);
        for (int l = 2; l <= tr.L && st == ERT_OK; ++l) st = het_far_level(p, tr, cheb, t8.st8, c, l);
        if (st != ERT_OK) return fail(st);
        if (c->chunk > 0) {
            c->st8 = t8.release();
            c->bytes += (size_t)p->N * 8 * sizeof(double);
        }
        if (hipStreamSynchronize(s) != hipSuccess) return fail(ERT_EDEVICE);
        p->het[slot] = c;
        hc = c;
        return ERT_OK;
    }
    // directed rows: every leaf and each of its 3^d neighbour offsets (-1 outside the grid)
    std::vector<int> src((size_t)tr.nleaf * nn);
    std::vector<long> ts(tr.nleaf + 1);
    for (long lf = 0; lf < tr.nleaf; ++lf) {
        int lb[3];
        unravel3(lf, tr.nb, lb);
        ts[lf] = lf * nn;
        for (int k = 0; k < nn; ++k) {
            const int o[3] = {k % 3 - 1, (k / 3) % 3 - 1, tr.D == 3 ? k / 9 - 1 : 0};
            int sb[3];
            bool ok = true;
            for (int a = 0; a < 3; ++a) {
                sb[a] = lb[a] + ((a < tr.D) ? o[a] : 0);
                if (sb[a] < 0 || sb[a] >= tr.nb[a]) ok = false;
            }
            src[(size_t)lf * nn + k] = ok ? (int)(sb[0] + (long)tr.nb[0] * (sb[1] + (long)tr.nb[1] * sb[2])) : -1;
        }
    }
    ts[tr.nleaf] = tr.nleaf * nn;
    // stored blocks: the self offset (nn / 2) and the offsets after it; offset index k
    // and nn - 1 - k are opposite offsets
    std::vector<int> ua, ub;
    std::vector<long> fwd, bwd;
    for (long lf = 0; lf < tr.nleaf; ++lf)
        for (int k = nn / 2; k < nn; ++k) {
            const int sl = src[(size_t)lf * nn + k];
            if (sl < 0) continue;
            ua.push_back((int)lf);
            ub.push_back(sl);
            fwd.push_back(lf * nn + k);
            bwd.push_back(k == nn / 2 ? -1 : (long)sl * nn + (nn - 1 - k));
        }
    const long np = (long)ua.size();
    const long per = (long)tr.S * tr.S;
    const size_t plane = (size_t)np * per * sizeof(uint16_t);
    const size_t bytes = 2 * plane;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess && bytes > fr / 10 * 9) {
        record_error("FMM: heterogeneous near-field cache does not fit in device memory");
        return fail(ERT_ENOMEM);
    }
    if (hipMalloc(&c->near_hi, std::max<size_t>(1, plane)) != hipSuccess ||
        hipMalloc(&c->near_lo, std::max<size_t>(1, plane)) != hipSuccess) {
        record_error("FMM: near-field cache allocation failed");
        return fail(ERT_ENOMEM);
    }
    c->bytes += bytes;
    c->near_np = np;
    ert_status st = upload<int>(s, &c->near_src, src);
    if (st == ERT_OK) st = upload<long>(s, &c->near_tstart, ts);
    if (st == ERT_OK) st = upload<int>(s, &c->near_ua, ua);
    if (st == ERT_OK) st = upload<int>(s, &c->near_ub, ub);
    if (st == ERT_OK) st = upload<long>(s, &c->near_fwd, fwd);
    if (st == ERT_OK) st = upload<long>(s, &c->near_bwd, bwd);
    CornerTable t8;
    if (st == ERT_OK) st = t8.build(p);
    if (st != ERT_OK) return fail(st);
    if (tr.leaf > kNearLdsLeaf) {
        record_error("FMM: leaf larger than the near-field block kernel supports");
        return fail(ERT_EINVAL);
    }
    const long chunk = std::max<long>(1, (1L << 28) / per);
    for (long u0 = 0; u0 < np; u0 += chunk) {
        const long cnt = std::min(chunk, np - u0);
        hipLaunchKernelGGL(k_near_blocks, dim3((unsigned)cnt), dim3(kNearLdsThreads), 0, s, dt, p->geo, p->d_st,
                           p->d_itab, c->near_ua, c->near_ub, u0, c->near_hi + (size_t)u0 * per,
                           c->near_lo + (size_t)u0 * per);
        if (hipGetLastError() != hipSuccess) return fail(ERT_EDEVICE);
    }
    for (int l = 2; l <= tr.L && st == ERT_OK; ++l) st = het_far_level(p, tr, cheb, t8.st8, c, l);
    if (st == ERT_OK && hipStreamSynchronize(s) != hipSuccess) st = ERT_EDEVICE;
    if (st != ERT_OK) return fail(st);
    if (c->chunk > 0) {
        c->st8 = t8.release();
        c->bytes += (size_t)p->N * 8 * sizeof(double);
    }
    p->het[slot] = c;
    hc = c;
    return ERT_OK;
}

template <typename T>
ert_status FmmImpl<T>::setup(ert_plan_impl* p)
{
    tr = make_tree(p, prec);
    hetero = p->o.kernel == ERT_K_RAY_MIDPOINT;
    if (tr.L > kMaxLevels) {
        record_error("FMM: grid too large for the tree depth limit");
        return ERT_EUNSUPPORTED;
    }
    if (tr.leaf > 8 || tr.nc > 8) {
        record_error("FMM: leaf side and Chebyshev order must be <= 8");
        return ERT_EUNSUPPORTED;
    }
    dt.D = tr.D; dt.nc = tr.nc; dt.K = tr.K; dt.Kp = tr.Kp; dt.leaf = tr.leaf; dt.S = tr.S;
    for (int a = 0; a < 3; ++a) dt.nb[a] = tr.nb[a];
    dt.nleaf = tr.nleaf;
    dt.nslot = tr.nslot;
    dt.n[0] = p->geo.n0; dt.n[1] = p->geo.n1; dt.n[2] = p->geo.n2;
    hipStream_t s = p->stream;
    p_stream = s;

    // 1D interpolation matrices (FP64 on the host)
    const int nc = tr.nc, leaf = tr.leaf;
    std::vector<double> node(nc), P1h((size_t)nc * leaf), M1h((size_t)2 * nc * nc);
    for (int m = 0; m < nc; ++m) node[m] = std::cos((2.0 * m + 1.0) * kPi / (2.0 * nc));
    for (int m = 0; m < nc; ++m)
        for (int i = 0; i < leaf; ++i) P1h[(size_t)m * leaf + i] = cheb_S(nc, (2.0 * i + 1.0) / leaf - 1.0, node[m]);
    for (int c = 0; c < 2; ++c)
        for (int m = 0; m < nc; ++m)
            for (int mp = 0; mp < nc; ++mp) {
                double xi = 0.5 * node[mp] + (c ? 0.5 : -0.5);
                M1h[((size_t)c * nc + m) * nc + mp] = cheb_S(nc, xi, node[m]);
            }
    ERT_TRY(upload_cvt<T>(s, &P1, P1h));
    ERT_TRY(upload_cvt<T>(s, &M1, M1h));
    ERT_TRY(upload<double>(s, &cheb, node));

    // offset tables: far-field interaction offsets per parity class, near offsets, identity
    {
        const int classes = 1 << tr.D;
        std::vector<BoxOffset> far;
        int per = 0;
        for (int c = 0; c < classes; ++c) {
            int pc[3] = {c & 1, tr.D > 1 ? (c >> 1) & 1 : 0, tr.D > 2 ? (c >> 2) & 1 : 0};
            int cnt = 0;
            for (int oz = (tr.D > 2 ? -2 - pc[2] : 0); oz <= (tr.D > 2 ? 3 - pc[2] : 0); ++oz)
                for (int oy = -2 - pc[1]; oy <= 3 - pc[1]; ++oy)
                    for (int ox = -2 - pc[0]; ox <= 3 - pc[0]; ++ox) {
                        if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1 && oz >= -1 && oz <= 1) continue;
                        // operator slot: lexicographic in [-3,3]^d (no z term in 2D)
                        int op = (ox + 3) + kOffSide * ((oy + 3) + (tr.D > 2 ? kOffSide * (oz + 3) : 0));
                        far.push_back({ox, oy, oz, op});
                        ++cnt;
                    }
            per = cnt;
        }
        m2l_noff = per;
        std::vector<BoxOffset> nr;
        const int nn = tr.D == 3 ? 27 : 9;
        for (int k = 0; k < nn; ++k) nr.push_back({k % 3 - 1, (k / 3) % 3 - 1, tr.D == 3 ? k / 9 - 1 : 0, k});
        // every operator slot must exist: 7^d far matrices, 3^d near blocks
        int nfar = 1;
        for (int a = 0; a < tr.D; ++a) nfar *= kOffSide;
        for (const BoxOffset& o : far)
            if (o.op < 0 || o.op >= nfar || (tr.D < 3 && o.o2 != 0)) {
                record_error("FMM: far-field offset table out of range");
                return ERT_EINVAL;
            }
        for (const BoxOffset& o : nr)
            if (o.op < 0 || o.op >= nn || (tr.D < 3 && o.o2 != 0)) {
                record_error("FMM: near-field offset table out of range");
                return ERT_EINVAL;
            }
        ERT_TRY(upload<BoxOffset>(s, &m2l_offs, far));
        ERT_TRY(upload<BoxOffset>(s, &near_offs, nr));
        std::vector<BoxOffset> id{{0, 0, 0, 0}};
        ERT_TRY(upload<BoxOffset>(s, &id_off, id));
    }

    if (!hetero) {
        const double sigma = p->sigma_const, h = p->geo.h;
        if (tr.S % 32 == 0) {
            const int nn = tr.D == 3 ? 27 : 9;
            const long n = (long)nn * tr.S * tr.S;
            ERT_HIP(hipMalloc(&nearops, n * sizeof(T)));
            hipLaunchKernelGGL(k_near_ops<T>, dim3(blocks(n)), dim3(kB), 0, s, tr.D, leaf, tr.S, h, sigma, nearops,
                               p->o.scheme);
            ERT_HIP(hipGetLastError());
            if (leaf >= 4 && (leaf & (leaf - 1)) == 0) {
                const int W = 4 * leaf - 1;
                const long ne = (tr.D == 3) ? (long)W * W * W : (long)W * W;
                near_tlen = (int)((ne + 3 + 3) / 4 * 4);
                ERT_HIP(hipMalloc(&neartab, 4L * near_tlen * sizeof(T)));
                hipLaunchKernelGGL(k_near_tab<T>, dim3(blocks(4L * near_tlen)), dim3(kB), 0, s, tr.D, leaf, h, sigma,
                                   p->o.scheme, near_tlen, neartab);
                ERT_HIP(hipGetLastError());
            }
        } else {
            if (p->o.scheme != 0) {
                record_error("FMM: approach (M-ii) in homogeneous media needs leaf^dim to be a multiple of 32");
                return ERT_EUNSUPPORTED;
            }
            // near-field table over K = |offset|^2 <= D (2 leaf - 1)^2
            const int span = 2 * leaf - 1;
            ntab = tr.D * span * span + 1;
            std::vector<double> tb(ntab, 0.0);
            for (int K = 1; K < ntab; ++K) {
                double r = h * std::sqrt((double)K);
                double rpw = (tr.D == 2) ? r : r * r;
                tb[K] = std::exp(-sigma * r) / (surface_area(tr.D) * rpw);
            }
            ERT_TRY(upload_cvt<T>(s, &tab, tb));
        }
        const double svd_tol = p->o.svd_tol == 0.0 ? 1e-6 : p->o.svd_tol;
        compress = svd_tol >= 0.0;
        for (int l = 2; l <= tr.L; ++l) ERT_TRY(setup_far_hom(p, l, svd_tol));
        // both execution forms of the box-offset products
        if (nearops) ERT_TRY(build_site(s, tr.D, tr.nl[tr.L], false, near_site));
        for (int l = 2; l <= tr.L; ++l) ERT_TRY(build_site(s, tr.D, tr.nl[l], true, far_site[l]));
    } else {
        ERT_TRY(setup_het(p));
    }
    ERT_HIP(hipStreamSynchronize(s));
    return ensure_buffers(1);
}

template <typename T>
ert_status FmmImpl<T>::ensure_buffers(int nrhs)
{
    if (nrhs <= B) return ERT_OK;
    drop_graphs();
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    if (!io) ERT_HIP(hipMalloc(&io, sizeof(ApplyIO)));
    f(q); f(pot);
    q = pot = nullptr;
    for (int l = 0; l <= kMaxLevels; ++l) {
        f(W[l]); f(Lc[l]); f(Wc[l]); f(Lh[l]);
        W[l] = Lc[l] = Wc[l] = Lh[l] = nullptr;
    }
    B = 0;
    ERT_HIP(hipMalloc(&q, (size_t)nrhs * tr.nslot * sizeof(T)));
    ERT_HIP(hipMalloc(&pot, (size_t)nrhs * tr.nslot * sizeof(T)));
    for (int l = 2; l <= tr.L; ++l) {
        size_t n = (size_t)nrhs * tr.nbox[l] * tr.Kp;
        ERT_HIP(hipMalloc(&W[l], n * sizeof(T)));
        ERT_HIP(hipMalloc(&Lc[l], n * sizeof(T)));
        // node padding (K..Kp) stays zero: the transfers never write it
        ERT_HIP(hipMemset(W[l], 0, n * sizeof(T)));
        ERT_HIP(hipMemset(Lc[l], 0, n * sizeof(T)));
        if (rp[l] > 0) {
            size_t m = (size_t)nrhs * tr.nbox[l] * rp[l];
            ERT_HIP(hipMalloc(&Wc[l], m * sizeof(T)));
            ERT_HIP(hipMalloc(&Lh[l], m * sizeof(T)));
        }
    }
    // offset-stationary form: tiles for this capacity, staging (far and near apart,
    // as they run concurrently) and tuning scratch
    size_t st_need = 0, sn_need = 0, tu_need = 0;
    auto site_need = [&](GemmSite& gs, long nbox, int M, size_t& need) -> ert_status {
        if (!gs.used) return ERT_OK;
        ERT_TRY(build_tiles(p_stream, gs, nrhs));
        need = std::max(need, (size_t)nrhs * gs.pl.npairs * M);
        tu_need = std::max(tu_need, (size_t)nrhs * nbox * M);
        return ERT_OK;
    };
    ERT_TRY(site_need(near_site, tr.nleaf, tr.S, sn_need));
    if (hetero) {
        // staging rows (one per directed pair) per pass: kPairStreamRhs right-hand sides
        // streamed, 64 on the matrix cores (from kPairMfmaMinRhs on, and always for the
        // split-BF16x3 translations)
        const size_t rb = (size_t)std::min(nrhs, nrhs >= kPairMfmaMinRhs ? 64 : kPairStreamRhs);
        const size_t rbf = (size_t)std::min(nrhs, (nrhs >= kPairMfmaMinRhs || prec == ERT_BF16X3) ? 64 : kPairStreamRhs);
        sn_need = std::max(sn_need, rb * tr.nleaf * (tr.D == 3 ? 27 : 9) * tr.S);
        for (int l = 2; l <= tr.L; ++l) st_need = std::max(st_need, rbf * hc->hnd[l] * tr.Kp);
    }
    for (int l = 2; l <= tr.L; ++l)
        ERT_TRY(site_need(far_site[l], tr.nbox[l], rp[l] > 0 ? rp[l] : tr.Kp, st_need));
    auto grow = [](T** buf, size_t* have, size_t need) -> ert_status {
        if (need <= *have) return ERT_OK;
        if (*buf) (void)hipFree(*buf);
        *buf = nullptr;
        *have = 0;
        ERT_HIP(hipMalloc(buf, need * sizeof(T)));
        *have = need;
        return ERT_OK;
    };
    ERT_TRY(grow(&stage, &stage_elems, st_need));
    ERT_TRY(grow(&stage_near, &stage_near_elems, sn_need));
    if (tu_need > tune_elems) {
        if (tune) (void)hipFree(tune);
        tune = nullptr;
        tune_elems = 0;
        ERT_HIP(hipMalloc(&tune, tu_need * sizeof(T)));
        tune_elems = tu_need;
    }
    B = nrhs;
    return ERT_OK;
}

// Run one box-offset product in the form chosen for this rhs bucket; the first
// call of a bucket times both forms (into scratch) and keeps the faster one.
template <typename T>
ert_status FmmImpl<T>::run_site(ert_plan_impl* p, hipStream_t s, GemmSite& gs, int gprec, const BoxGemm& g, int nrhs,
                                StageTimer* outer, T* stg)
{
    if (!gs.used) return box_gemm(s, gprec, g);
    const int bucket = nrhs > 1 ? 1 : 0;
    if (gs.choice[bucket] < 0) {
        BoxGemm gt = g;
        gt.L = tune;
        gt.accumulate = 0;
        OffsetGemm ot[kForms];
        for (int f = 1; f < kForms; ++f) ot[f] = offset_of(gs, gt, stg, f);
        // forms 4 and 5 (LDS-staged source columns) where they apply
        bool ok[kForms];
        for (int f = 0; f < kForms; ++f) ok[f] = f < 4;
        ok[4] = offset_lds_ok(gprec, ot[4]);
        ok[5] = offset_lds64_ok(gprec, ot[5]);
        hipEvent_t e[3];
        for (auto& ev : e) ERT_HIP(hipEventCreate(&ev));
        float ms[kForms] = {};
        ert_status st = ERT_OK;
        auto run = [&](int form) { return form == 0 ? box_gemm(s, gprec, gt) : offset_gemm(s, gprec, ot[form]); };
        for (int form = 0; form < kForms && st == ERT_OK; ++form) {
            if (!ok[form]) continue;
            st = run(form);   // warm-up
            if (st != ERT_OK) break;
            (void)hipEventRecord(e[0], s);
            for (int r = 0; r < 3 && st == ERT_OK; ++r) st = run(form);
            (void)hipEventRecord(e[1], s);
            if (hipEventSynchronize(e[1]) != hipSuccess) st = ERT_EDEVICE;
            else (void)hipEventElapsedTime(&ms[form], e[0], e[1]);
        }
        for (auto& ev : e) (void)hipEventDestroy(ev);
        ERT_TRY(st);
        int best = 0;
        for (int form = 0; form < kForms; ++form) {
            if (!ok[form]) continue;
            gs.tuned_ms[bucket][form] = ms[form] / 3;
            if (ms[form] < ms[best]) best = form;
        }
        // within 5 % of the fastest, take the 64-column tiles: they read each operator
        // block once instead of once per 16 columns (less HBM traffic at the same speed)
        if (best == 1 && ms[2] <= 1.05f * ms[1]) best = 2;
        // a form fixed by the plan's options (near field / far field), where it applies
        const int fixed = p->o.form[&gs == &near_site ? 0 : 1] - 1;
        if (fixed >= 0 && fixed < kForms && ok[fixed]) best = fixed;
        gs.choice[bucket] = best;
    }
    if (gs.choice[bucket] == 0) return box_gemm(s, gprec, g);
    OffsetGemm og = offset_of(gs, g, stg, gs.choice[bucket]);
    ERT_TRY(offset_gemm_products(s, gprec, og));
    if (outer) outer->stop();
    StageTimer sr_(&p->prof, s, ERT_STAGE_REDUCE);
    return offset_gemm_reduce(s, gprec, og);
}

// One-level homogeneous tree with compressed translations, after tuning: the near
// field and the far-field translations are independent products of the same kind;
// they run in one launch (each in its tuned form), and so do their per-target sums:
// gather, P2M with compression, the two products, the two sums, expansion with L2P,
// assembly.
template <typename T>
ert_status FmmImpl<T>::enqueue_grouped(ert_plan_impl* p, hipStream_t s, int nrhs)
{
    const long N = p->N;
    const int nn = tr.D == 3 ? 27 : 9;
    const int L = tr.L, R = rp[L], bk = nrhs > 1 ? 1 : 0;
    const int dprec = (prec == ERT_FP64) ? ERT_FP64 : ERT_FP32;
    Profiler* pf = &p->prof;
    {
        // weighted charges into leaf order and P2M with the compression, one kernel
        StageTimer st_(pf, s, ERT_STAGE_GATHER);
        const int rch = (R + 63) / 64;
        first.kind = 2;
        first.func = (const void*)k_leaf_in<T>;
        first.grid = dim3((unsigned)(tr.nbox[L] * rch), (unsigned)nrhs);
        first.block = dim3(64 * kLeafInWaves);
        first.shmem = (kLeafInWaves * 64 + tr.S) * sizeof(T);
        first.l = LeafInArgs{cur, io, dt, p->d_ss, N, leaf_inT, R, rch, q, Wc[L]};
        const LeafInArgs& A = first.l;
        hipLaunchKernelGGL(k_leaf_in<T>, first.grid, first.block, first.shmem, s, A.a, A.io, A.t, A.ss, A.N, A.linT,
                           A.R, A.rch, A.q, A.W);
        ERT_HIP(hipGetLastError());
    }
    BoxGemm gn = gemm_desc(L, tr.S, tr.S, nrhs);
    gn.stride = 1; gn.nclass = 1; gn.noff = nn; gn.offs = near_offs;
    gn.ops = nearops; gn.W = q; gn.L = pot; gn.accumulate = 0;
    BoxGemm gf = gemm_desc(L, R, R, nrhs);
    gf.stride = 2; gf.nclass = 1 << tr.D; gf.noff = m2l_noff; gf.offs = m2l_offs;
    gf.ops = ops[L]; gf.ops_lo = ops_lo[L]; gf.W = Wc[L]; gf.L = Lh[L]; gf.accumulate = 0;
    const OffsetGemm on = offset_of(near_site, gn, stage_near, near_site.choice[bk]);
    const OffsetGemm of = offset_of(far_site[L], gf, stage, far_site[L].choice[bk]);
    {
        // the near-field blocks are FP32/FP64 like the dense transforms; the
        // translations take the plan's precision (BF16x3 included): one launch needs one
        // precision, so BF16x3 plans keep the products apart
        StageTimer st_(pf, s, ERT_STAGE_NEAR);
        if (dprec == prec) {
            ERT_TRY(offset_gemm_pair_products(s, prec, on, of));
        } else {
            ERT_TRY(offset_gemm_products(s, dprec, on));
            ERT_TRY(offset_gemm_products(s, prec, of));
        }
    }
    // sums of the staged products, expansion with L2P and assembly, one kernel
    const double hd = std::pow(p->geo.h, tr.D);
    StageTimer st_(pf, s, ERT_STAGE_ASSEMBLE);
    const int sch = (tr.S + 63) / 64;
    hipLaunchKernelGGL(k_leaf_out<T>, dim3((unsigned)(tr.nbox[L] * sch), (unsigned)nrhs), dim3(64 * kLeafWaves),
                       (2 * kLeafWaves * 64 + R + (64 * kLeafWaves / R) * R) * sizeof(T), s, dt, io, p->d_ss,
                       p->d_diag, hd, N,
                       (const T*)on.stage, on.pl.tcnt, on.pl.tpad, on.pl.npairs, (const T*)of.stage,
                       of.pl.tcnt, of.pl.tpad, of.pl.npairs, R, leaf_outT, sch);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

template <typename T>
ert_status FmmImpl<T>::enqueue(ert_plan_impl* p, hipStream_t s, int nrhs)
{
    {
        const int bk = nrhs > 1 ? 1 : 0;
        if (grouped_form(bk)) return enqueue_grouped(p, s, nrhs);
    }
    const long N = p->N;
    const int nn = tr.D == 3 ? 27 : 9;
    const int dprec = (prec == ERT_FP64) ? ERT_FP64 : ERT_FP32;   // precision of the dense transforms
    Profiler* pf = &p->prof;
    // a4: weights into leaf-major order
    {
        StageTimer st_(pf, s, ERT_STAGE_GATHER);
        first.kind = 1;
        first.func = (const void*)k_gather<T>;
        first.grid = dim3(blocks(tr.nslot * nrhs));
        first.block = dim3(kB);
        first.shmem = 0;
        first.g = GatherArgs{cur, io, dt, p->d_ss, N, nrhs, q};
        const GatherArgs& A = first.g;
        hipLaunchKernelGGL(k_gather<T>, first.grid, first.block, 0, s, A.a, A.io, A.t, A.ss, A.N, A.B, A.q);
        ERT_HIP(hipGetLastError());
    }
    // a10: near field (writes pot), on the side stream once the forms are tuned; while
    // stages are timed everything runs on one stream, so that each stage's events
    // bracket its own kernels and the stage times add up to the apply's
    const bool fork = tuned[nrhs > 1 ? 1 : 0] && !pf->on;
    hipStream_t sn = s;
    if (fork) {
        if (!side) ERT_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
        if (!ev_fork) ERT_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
        if (!ev_join) ERT_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
        ERT_HIP(hipEventRecord(ev_fork, s));
        ERT_HIP(hipStreamWaitEvent(side, ev_fork, 0));
        sn = side;
    }
    {
        StageTimer st_(pf, sn, ERT_STAGE_NEAR);
        StageTimer* near_timer = &st_;
        if (hetero) {
            PairStream a;
            // the FP32 applies of a plan with inner_near16 read the BF16-rounded plane alone
            a.ops_fmt = (prec != ERT_FP64 && p->o.inner_near16) ? kOpsHi : kOpsSplit;
            a.opsT = hc->near_hi;
            a.opsT_lo = hc->near_lo;
            a.npairs = hc->near_np;
            a.ua = hc->near_ua;
            a.ub = hc->near_ub;
            a.fwd_row = hc->near_fwd;
            a.bwd_row = hc->near_bwd;
            a.nrows = tr.nleaf * nn;
            a.row_src = hc->near_src;
            a.tstart = hc->near_tstart;
            a.ntarget = tr.nleaf;
            a.B = nrhs;
            a.M = tr.S;
            a.nsrc = tr.nleaf;
            a.W = q;
            a.stage = stage_near;
            a.L = pot;
            a.accumulate = 0;
            st_.pause();
            a.prof = pf;
            a.prof_stage = ERT_STAGE_NEAR;
            ERT_TRY(pair_stream(sn, prec == ERT_FP64 ? ERT_FP64 : ERT_FP32, a));
        } else if (nearops) {
            BoxGemm g = gemm_desc(tr.L, tr.S, tr.S, nrhs);
            g.stride = 1;
            g.nclass = 1;
            g.noff = nn;
            g.offs = near_offs;
            g.ops = nearops;
            g.W = q;
            g.L = pot;
            g.accumulate = 0;
            ERT_TRY(run_site(p, sn, near_site, dprec, g, nrhs, near_timer, stage_near));
        } else {
            const int tpp = std::min(tr.S, kB);
            const int groups = kB / tpp;
            size_t sh = (size_t)(ntab + nn * tr.S) * sizeof(T) + 32 * sizeof(int) + (size_t)groups * tpp * sizeof(T);
            hipLaunchKernelGGL(k_p2p_hom<T>, dim3((unsigned)tr.nleaf, nrhs), dim3(kB), sh, sn, dt, q, tab, ntab, pot);
            ERT_HIP(hipGetLastError());
        }
    }
    bool joined = false;
    if (tr.L >= 2) {
        const int L = tr.L;
        // a5: P2M on the leaves (with the compression folded in when the leaves are the
        // only far-field level)
        if (leaf_in) {
            StageTimer st_(pf, s, ERT_STAGE_P2M);
            BoxGemm c = gemm_desc(L, rp[L], tr.S, nrhs);
            c.stride = 1; c.nclass = 1; c.noff = 1; c.offs = id_off;
            c.ops = leaf_in; c.W = q; c.L = Wc[L]; c.accumulate = 0;
            ERT_TRY(box_gemm(s, dprec, c));
        } else {
            StageTimer st_(pf, s, ERT_STAGE_P2M);
            hipLaunchKernelGGL(k_p2m<T>, dim3((unsigned)tr.nleaf, nrhs), dim3(kB), 0, s, dt, q, P1, W[L]);
            ERT_HIP(hipGetLastError());
        }
        // a6: M2M up to level 2
        for (int l = L - 1; l >= 2; --l) {
            StageTimer st_(pf, s, ERT_STAGE_M2M);
            hipLaunchKernelGGL(k_m2m<T>, dim3((unsigned)tr.nbox[l], nrhs), dim3(kB), 0, s, tr.D, tr.nc, tr.K, tr.Kp,
                               tr.nl[l][0], tr.nl[l][1], tr.nl[l][2], tr.nbox[l], tr.nl[l + 1][0], tr.nl[l + 1][1],
                               tr.nl[l + 1][2], tr.nbox[l + 1], W[l + 1], M1, W[l]);
            ERT_HIP(hipGetLastError());
        }
        // a7/a8: downward pass
        for (int l = 2; l <= L; ++l) {
            // the top level has no parent: its locals start at the first far-field
            // product written with accumulate = 0 (no zero fill)
            const int first = (l == 2) ? 1 : 0;
            {
                StageTimer st_(pf, s, ERT_STAGE_L2L);
                if (l == 2) {
                    // nothing to inherit
                } else {
                    hipLaunchKernelGGL(k_l2l<T>, dim3((unsigned)tr.nbox[l], nrhs), dim3(kB), 0, s, tr.D, tr.nc, tr.K,
                                       tr.Kp, tr.nl[l - 1][0], tr.nl[l - 1][1], tr.nl[l - 1][2], tr.nbox[l - 1],
                                       tr.nl[l][0], tr.nl[l][1], tr.nl[l][2], tr.nbox[l], Lc[l - 1], M1, Lc[l]);
                }
                ERT_HIP(hipGetLastError());
            }
            StageTimer st_(pf, s, ERT_STAGE_M2L);
            if (hetero) {
                PairStream a;
                a.ops_fmt = kOpsF32;
                a.opsT = hc->hops[l];
                a.opsT_lo = nullptr;
                a.npairs = hc->hnp[l];
                a.ua = hc->hua[l];
                a.ub = hc->hub[l];
                a.fwd_row = hc->hfwd[l];
                a.bwd_row = hc->hbwd[l];
                a.nrows = hc->hnd[l];
                a.row_src = nullptr;
                a.tstart = hc->pstart[l];
                a.ntarget = tr.nbox[l];
                a.B = nrhs;
                a.M = tr.Kp;
                a.nsrc = tr.nbox[l];
                a.W = W[l];
                a.stage = stage;
                a.L = Lc[l];
                a.accumulate = first ? 0 : 1;
                st_.pause();
                a.prof = pf;
                a.prof_stage = ERT_STAGE_M2L;
                // split-BF16x3 translations run on the matrix cores for any rhs count
                if (hc->rebuilt[l]) {
                    // pairs past the stored ones: rebuilt chunk by chunk for these products
                    const HetGenCtx ctx{p, &tr, cheb, hc, l};
                    PairGen gen;
                    gen.stored = hc->hstored[l];
                    gen.stored_ops = hc->hops[l];
                    gen.chunk = hc->chunk;
                    gen.scratch = hc->scratch;
                    gen.fill = het_gen_fill;
                    gen.ctx = &ctx;
                    ERT_TRY(pair_stream(s, prec, a, &gen));
                } else {
                    ERT_TRY(pair_stream(s, prec, a));
                }
            } else if (rp[l] > 0 && leaf_in) {
                // single compressed level: multipoles already compressed, the expansion
                // is folded into L2P below
                BoxGemm g = gemm_desc(l, rp[l], rp[l], nrhs);
                g.stride = 2; g.nclass = 1 << tr.D; g.noff = m2l_noff; g.offs = m2l_offs;
                g.ops = ops[l]; g.ops_lo = ops_lo[l]; g.W = Wc[l]; g.L = Lh[l]; g.accumulate = 0;
                ERT_TRY(run_site(p, s, far_site[l], prec, g, nrhs, &st_, stage));
            } else if (rp[l] > 0) {
                const int R = rp[l];
                st_.pause();
                {
                    StageTimer sb_(pf, s, ERT_STAGE_BASIS);
                    BoxGemm c = gemm_desc(l, R, tr.Kp, nrhs);   // compress
                    c.stride = 1; c.nclass = 1; c.noff = 1; c.offs = id_off;
                    c.ops = Ut[l]; c.W = W[l]; c.L = Wc[l]; c.accumulate = 0;
                    ERT_TRY(box_gemm(s, dprec, c));
                }
                {
                    StageTimer sm_(pf, s, ERT_STAGE_M2L);
                    BoxGemm g = gemm_desc(l, R, R, nrhs);       // translate
                    g.stride = 2; g.nclass = 1 << tr.D; g.noff = m2l_noff; g.offs = m2l_offs;
                    g.ops = ops[l]; g.ops_lo = ops_lo[l]; g.W = Wc[l]; g.L = Lh[l]; g.accumulate = 0;
                    ERT_TRY(run_site(p, s, far_site[l], prec, g, nrhs, &sm_, stage));
                }
                {
                    StageTimer sb_(pf, s, ERT_STAGE_BASIS);
                    BoxGemm u = gemm_desc(l, tr.Kp, R, nrhs);   // back to the node basis, added to the locals
                    u.stride = 1; u.nclass = 1; u.noff = 1; u.offs = id_off;
                    u.ops = Um[l]; u.W = Lh[l]; u.L = Lc[l]; u.accumulate = first ? 0 : 1;
                    ERT_TRY(box_gemm(s, dprec, u));
                }
            } else {
                BoxGemm g = gemm_desc(l, tr.Kp, tr.Kp, nrhs);
                g.stride = 2; g.nclass = 1 << tr.D; g.noff = m2l_noff; g.offs = m2l_offs;
                g.ops = ops[l]; g.ops_lo = ops_lo[l]; g.W = W[l]; g.L = Lc[l]; g.accumulate = first ? 0 : 1;
                ERT_TRY(run_site(p, s, far_site[l], prec, g, nrhs, &st_, stage));
            }
        }
        // a9: L2P adds the far field (after the near field has written pot)
        if (fork) {
            ERT_HIP(hipEventRecord(ev_join, side));
            ERT_HIP(hipStreamWaitEvent(s, ev_join, 0));
            joined = true;
        }
        StageTimer st_(pf, s, ERT_STAGE_L2P);
        if (leaf_in) {
            BoxGemm u = gemm_desc(L, tr.S, rp[L], nrhs);
            u.stride = 1; u.nclass = 1; u.noff = 1; u.offs = id_off;
            u.ops = leaf_out; u.W = Lh[L]; u.L = pot; u.accumulate = 1;
            ERT_TRY(box_gemm(s, dprec, u));
        } else {
            hipLaunchKernelGGL(k_l2p<T>, dim3((unsigned)tr.nleaf, nrhs), dim3(kB), 0, s, dt, Lc[L], P1, pot);
            ERT_HIP(hipGetLastError());
        }
    }
    if (fork && !joined) {   // no far field: join before the assembly reads pot
        ERT_HIP(hipEventRecord(ev_join, side));
        ERT_HIP(hipStreamWaitEvent(s, ev_join, 0));
    }
    // a11: scale, self term, operator
    {
        const double hd = std::pow(p->geo.h, tr.D);
        StageTimer st_(pf, s, ERT_STAGE_ASSEMBLE);
        hipLaunchKernelGGL(k_assemble<T>, dim3(blocks(N * nrhs)), dim3(kB), 0, s, dt, pot, io, p->d_ss, p->d_diag,
                           hd, N, nrhs);
        ERT_HIP(hipGetLastError());
    }
    // this call chose the forms and they make the fused one-level apply, which sums
    // in another order: recompute with it (x and y do not overlap) so that every
    // call of the bucket, eager or replayed, returns the same bits
    if (grouped_form(nrhs > 1 ? 1 : 0)) return enqueue_grouped(p, s, nrhs);
    return ERT_OK;
}

// y = op(x): one small kernel sets the vectors, then the apply runs from a
// captured graph (third and later calls of a rhs bucket; the first call tunes
// the execution forms, the second captures) or eagerly while profiling.
template <typename T>
ert_status FmmImpl<T>::apply(ert_plan_impl* p, int op, const double* x, double* y, int nrhs)
{
    ERT_TRY(ensure_buffers(nrhs));
    hipStream_t s = p->stream;
    cur = ApplyIO{x, y, op, 0};
    const int bucket = nrhs > 1 ? 1 : 0;
    if (p->prof.on || !p->use_graphs || no_graph[bucket]) return enqueue(p, s, nrhs);
    if (gexec[bucket] && graph_nrhs[bucket] == nrhs) {
        ERT_TRY(set_root_args(bucket));
        ERT_HIP(hipGraphLaunch(gexec[bucket], s));
        return ERT_OK;
    }
    if (calls[bucket]++ == 0) {                             // tunes the forms of this bucket
        ERT_TRY(enqueue(p, s, nrhs));
        tuned[bucket] = true;
        return ERT_OK;
    }
    // capture on the internal stream, ordered after the caller's stream
    if (!cap) ERT_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    if (gexec[bucket]) {
        (void)hipGraphExecDestroy(gexec[bucket]);
        (void)hipGraphDestroy(graph[bucket]);
        gexec[bucket] = nullptr;
        graph[bucket] = nullptr;
    }
    ERT_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    ert_status st = enqueue(p, cap, nrhs);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(cap, &g);
    if (st != ERT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (ce != hipSuccess) {
        record_hip_error("hipStreamEndCapture", ce, __FILE__, __LINE__);
        return ERT_EDEVICE;
    }
    // the root must be the recorded first kernel, whose vectors each replay replaces;
    // otherwise this rhs bucket runs eagerly
    hipGraphNode_t root = nullptr;
    size_t nroot = 0;
    bool root_ok = hipGraphGetRootNodes(g, nullptr, &nroot) == hipSuccess && nroot == 1;
    if (root_ok) root_ok = hipGraphGetRootNodes(g, &root, &nroot) == hipSuccess && nroot == 1 && root;
    if (root_ok) {
        hipGraphNodeType ty;
        hipKernelNodeParams kp{};
        root_ok = hipGraphNodeGetType(root, &ty) == hipSuccess && ty == hipGraphNodeTypeKernel &&
                  hipGraphKernelNodeGetParams(root, &kp) == hipSuccess && kp.func == first.func && first.kind != 0;
    }
    if (!root_ok) {
        (void)hipGraphDestroy(g);
        no_graph[bucket] = true;
        return enqueue(p, s, nrhs);
    }
    hipGraphExec_t ge = nullptr;
    hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        record_hip_error("hipGraphInstantiate", ie, __FILE__, __LINE__);
        return ERT_EDEVICE;
    }
    graph[bucket] = g;
    gexec[bucket] = ge;
    graph_nrhs[bucket] = nrhs;
    gfirst[bucket] = first;
    groot[bucket] = root;
    ERT_HIP(hipGraphLaunch(ge, s));
    return ERT_OK;
}

// Give the root kernel node of a captured apply the vectors of this call.
template <typename T>
ert_status FmmImpl<T>::set_root_args(int bucket)
{
    FirstLaunch& f = gfirst[bucket];
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(f.func);
    kp.gridDim = f.grid;
    kp.blockDim = f.block;
    kp.sharedMemBytes = (unsigned int)f.shmem;
    kp.extra = nullptr;
    if (f.kind == 1) {
        GatherArgs& A = f.g;
        A.a = cur;
        void* args[] = {&A.a, &A.io, &A.t, &A.ss, &A.N, &A.B, &A.q};
        kp.kernelParams = args;
        ERT_HIP(hipGraphExecKernelNodeSetParams(gexec[bucket], groot[bucket], &kp));
    } else {
        LeafInArgs& A = f.l;
        A.a = cur;
        void* args[] = {&A.a, &A.io, &A.t, &A.ss, &A.N, &A.linT, &A.R, &A.rch, &A.q, &A.W};
        kp.kernelParams = args;
        ERT_HIP(hipGraphExecKernelNodeSetParams(gexec[bucket], groot[bucket], &kp));
    }
    return ERT_OK;
}

}  // namespace

ert_status fmm_build(ert_plan_impl* p, int prec)
{
    if (prec < 0 || prec > 2) return ERT_EINVAL;
    if (!p->fmm[prec]) {
        FmmData* f = nullptr;
        if (prec == ERT_FP64) {
            auto* g = new (std::nothrow) FmmImpl<double>();
            if (g) g->prec = ERT_FP64;
            f = g;
        } else {
            auto* g = new (std::nothrow) FmmImpl<float>();
            if (g) g->prec = prec;
            f = g;
        }
        if (!f) return ERT_ENOMEM;
        ert_status st = f->setup(p);
        if (st != ERT_OK) {
            delete f;
            return st;
        }
        p->fmm[prec] = f;
    }
    return ERT_OK;
}

ert_status fmm_apply(ert_plan_impl* p, int op, int prec, const double* x, double* y, int nrhs)
{
    ERT_TRY(fmm_build(p, prec));
    return p->fmm[prec]->apply(p, op, x, y, nrhs);
}

ert_status fmm_info(ert_plan_impl* p, int prec, ert_fmm_info* info)
{
    ERT_TRY(fmm_build(p, prec));
    const FmmData* f = p->fmm[prec];
    const FmmTree& t = f->tr;
    std::memset(info, 0, sizeof(*info));
    info->levels = t.L;
    info->leaf = t.leaf;
    info->cheb_n = t.nc;
    info->nodes = t.K;
    info->nodes_padded = t.Kp;
    for (int l = 0; l <= t.L && l < 16; ++l) info->rank[l] = f->rank_of(l);
    info->form_near = f->form_of(-1);
    info->near_table = f->near_table();
    for (int l = 0; l < 16; ++l) info->form_far[l] = (l <= t.L && l >= 2) ? f->form_of(l) : -1;
    for (int l = 0; l < 16; ++l) info->far_rebuilt[l] = (l <= t.L && l >= 2 && f->far_rebuilt(l)) ? 1 : 0;
    info->cache_bytes = f->cache_bytes();
    // interaction-list pairs per level (separable per axis) and near point pairs
    for (int l = 2; l <= t.L && l < 16; ++l) {
        long par = 1, nr = 1;
        for (int a = 0; a < t.D; ++a) {
            const int n = t.nl[l][a];
            long pa = 0, na = 0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    if (std::abs(i / 2 - j / 2) <= 1) {
                        ++pa;
                        if (std::abs(i - j) <= 1) ++na;
                    }
                }
            par *= pa;
            nr *= na;
        }
        info->far_pairs[l] = par - nr;
    }
    {
        const int n[3] = {p->geo.n0, p->geo.n1, p->geo.n2};
        long tot = 1;
        for (int a = 0; a < t.D; ++a) {
            // point pairs along one axis whose leaves are adjacent
            long c = 0;
            for (int i = 0; i < n[a]; ++i) {
                const int bi = i / t.leaf;
                const int lo = std::max(0, (bi - 1) * t.leaf), hi = std::min(n[a], (bi + 2) * t.leaf);
                c += hi - lo;
            }
            tot *= c;
        }
        info->near_pairs = tot - p->N;
    }
    return ERT_OK;
}

void fmm_destroy(FmmData* f) { delete f; }

HetCache::~HetCache()
{
    auto f = [](void* q) { if (q) (void)hipFree(q); };
    if (owns_near) {
        f(near_hi); f(near_lo); f(near_src); f(near_tstart);
        f(near_ua); f(near_ub); f(near_fwd); f(near_bwd);
    }
    for (int l = 0; l <= kMaxLevels; ++l) {
        f(hops[l]); f(pstart[l]); f(hua[l]); f(hub[l]); f(hfwd[l]); f(hbwd[l]);
    }
    f(scratch);
    f(st8);
}

void het_destroy(HetCache* c) { delete c; }

}  // namespace ertvie
