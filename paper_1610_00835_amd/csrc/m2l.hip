// Box-offset GEMMs on the matrix cores, and the cached-pair far field.
//
// On a uniform grid with a homogeneous medium every interaction between two
// boxes depends only on their offset, so the far-field translations (Sec. 3.3,
// eq. EQ: M2L: f2(p_m) = sum_m' K(L p_m, R q_m') f1(q_m')), the near field over
// neighbouring leaves and the change of basis of the compressed translations
// are all one kind of batched GEMM:
//     L[b][t] (+)= sum_{o in list(class(t))} ops[o] * W[b][t + o].
// A workgroup owns a tile of (output rows) x (target box, right-hand side)
// columns; targets are grouped by index parity when the far-field interaction
// lists are used (all targets of a parity class share one offset list).  The
// four waves of a workgroup run the same offsets and split the reduction
// chunks of each offset; their partial sums are combined in LDS in a fixed
// order, so results are bitwise reproducible.  Operands go straight from
// global memory into MFMA registers: each lane loads 16-32 contiguous bytes
// along the reduction dimension and the order in which reduction indices are
// fed to the MFMA steps is permuted to match (the same permutation for both
// operands, so the product is unchanged).  Output register layouts (checked on
// gfx950): 16x16x4 f32 and 16x16x32 bf16 hold rows 4*(lane/16)+i of column
// lane%16; 16x16x4 f64 holds rows lane/16 + 4*i.
//
// Heterogeneous media (every box pair with its own cached matrix) are in pairs.hip.
#include <algorithm>
#include <type_traits>

#include "fmm.hpp"

namespace ertvie {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kWaves = 4;

template <int PREC>
struct Acc;
template <>
struct Acc<ERT_FP64> { typedef v4d V; typedef double T; };
template <>
struct Acc<ERT_FP32> { typedef v4f V; typedef float T; };
template <>
struct Acc<ERT_BF16X3> { typedef v4f V; typedef float T; };

__device__ __forceinline__ void split_bf16(const v4f& x0, const v4f& x1, v8bf& hi, v8bf& lo)
{
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        __bf16 h0 = (__bf16)x0[e];
        __bf16 h1 = (__bf16)x1[e];
        hi[e] = h0;
        hi[4 + e] = h1;
        lo[e] = (__bf16)(x0[e] - (float)h0);
        lo[4 + e] = (__bf16)(x1[e] - (float)h1);
    }
}


// One reduction chunk of a tile: the operand registers of TM row blocks and TN
// column blocks (bf16x3 keeps the FP32 source values and splits them at use).
template <int PREC, int TM, int TN>
struct Frag {
    typedef typename Acc<PREC>::V V;
    V a[TM], b[TN];              // FP64 / FP32
    v8bf ah[TM], al[TM];         // BF16X3 operator parts
    v4f x0[TN], x1[TN];          // BF16X3 source values
};

template <int PREC, int TM, int TN>
__device__ __forceinline__ void frag_load(Frag<PREC, TM, TN>& f, const void* ops, const void* ops_lo, long abase,
                                          long rowstep, const typename Acc<PREC>::T* const bp[TN], int kk)
{
    typedef typename Acc<PREC>::V V;
    typedef typename Acc<PREC>::T T;
    if constexpr (PREC == ERT_BF16X3) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) {
            const long a = abase + tm * rowstep + kk;
            f.ah[tm] = *(const v8bf*)((const __bf16*)ops + a);
            f.al[tm] = *(const v8bf*)((const __bf16*)ops_lo + a);
        }
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            f.x0[tn] = bp[tn] ? *(const v4f*)(bp[tn] + kk) : v4f{0.f, 0.f, 0.f, 0.f};
            f.x1[tn] = bp[tn] ? *(const v4f*)(bp[tn] + kk + 4) : v4f{0.f, 0.f, 0.f, 0.f};
        }
    } else {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) f.a[tm] = *(const V*)((const T*)ops + abase + tm * rowstep + kk);
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) f.b[tn] = bp[tn] ? *(const V*)(bp[tn] + kk) : V{0, 0, 0, 0};
    }
}

template <int PREC, int TM, int TN>
__device__ __forceinline__ void frag_mma(const Frag<PREC, TM, TN>& f, typename Acc<PREC>::V (&acc)[TM][TN])
{
    if constexpr (PREC == ERT_BF16X3) {
        v8bf bh[TN], bl[TN];
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) split_bf16(f.x0[tn], f.x1[tn], bh[tn], bl[tn]);
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) {
                acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ah[tm], bh[tn], acc[tm][tn], 0, 0, 0);
                acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ah[tm], bl[tn], acc[tm][tn], 0, 0, 0);
                acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.al[tm], bh[tn], acc[tm][tn], 0, 0, 0);
            }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                for (int tn = 0; tn < TN; ++tn) {
                    if constexpr (PREC == ERT_FP64)
                        acc[tm][tn] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.a[tm][e], f.b[tn][e], acc[tm][tn], 0, 0, 0);
                    else
                        acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(f.a[tm][e], f.b[tn][e], acc[tm][tn], 0, 0, 0);
                }
    }
}

// The reduction chunks of one operator, split over the waves (chunk c goes to
// wave c mod 4); U chunks' loads are issued before their products so that
// several loads are in flight per wave.
template <int PREC, int TM, int TN>
__device__ __forceinline__ void tile_reduce(const void* ops, const void* ops_lo, long abase, long rowstep, int Kd,
                                            const typename Acc<PREC>::T* const bp[TN], int wave,
                                            typename Acc<PREC>::V (&acc)[TM][TN])
{
    constexpr int CW = (PREC == ERT_BF16X3) ? 32 : 16;
    constexpr int U = (PREC == ERT_FP32) ? 4 : 2;
    constexpr int STEP = kWaves * CW;
    for (int k0 = wave * CW; k0 < Kd; k0 += U * STEP) {
        Frag<PREC, TM, TN> f[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * STEP < Kd) frag_load<PREC, TM, TN>(f[u], ops, ops_lo, abase, rowstep, bp, k0 + u * STEP);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * STEP < Kd) frag_mma<PREC, TM, TN>(f[u], acc);
    }
}

// Operator read from a table over cell offsets (the near field of a homogeneous
// medium on a uniform grid: the block entry of target cell t and source cell s
// at leaf offset o depends only on o leaf + s - t).  The table index of entry
// (t, s) is tb(t) + lin(s), lin(c) = c0 + W c1 + W^2 c2; a lane's four
// consecutive reduction indices lie on one grid line (leaf a multiple of 4), so
// they are four consecutive table entries, read as one aligned vector from the
// copy of the table shifted by the index modulo 4.
__device__ __forceinline__ int tab_lin(const OffsetGemm& g, int c)
{
    const int sh = g.lshift, m = (1 << sh) - 1;
    if (g.dim == 2) return (c & m) + g.tw * (c >> sh);
    return (c & m) + g.tw * ((c >> sh) & m) + g.tw * g.tw * (c >> (2 * sh));
}

template <int PREC, int TM, int TN>
__device__ __forceinline__ void frag_load_tab(Frag<PREC, TM, TN>& f, const OffsetGemm& g, const int (&tb)[TM],
                                              int kl, const typename Acc<PREC>::T* const bp[TN], int kk)
{
    typedef typename Acc<PREC>::V V;
    typedef typename Acc<PREC>::T T;
    const int ls = tab_lin(g, kk + kl);
    const T* tab = (const T*)g.atab;
#pragma unroll
    for (int tm = 0; tm < TM; ++tm) {
        const int idx = tb[tm] + ls;
        const int r = idx & 3;
        f.a[tm] = *(const V*)(tab + r * g.tlen + (idx - r));
    }
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) f.b[tn] = bp[tn] ? *(const V*)(bp[tn] + kk) : V{0, 0, 0, 0};
}

template <int PREC, int TM, int TN>
__device__ __forceinline__ void tile_reduce_tab(const OffsetGemm& g, const int (&tb)[TM], int kl,
                                                const typename Acc<PREC>::T* const bp[TN], int wave,
                                                typename Acc<PREC>::V (&acc)[TM][TN])
{
    constexpr int CW = 16;
    constexpr int U = (PREC == ERT_FP32) ? 4 : 2;
    constexpr int STEP = kWaves * CW;
    for (int k0 = wave * CW; k0 < g.Kd; k0 += U * STEP) {
        Frag<PREC, TM, TN> f[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * STEP < g.Kd) frag_load_tab<PREC, TM, TN>(f[u], g, tb, kl, bp, k0 + u * STEP);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * STEP < g.Kd) frag_mma<PREC, TM, TN>(f[u], acc);
    }
}

template <int PREC, int TM, int TN>
__global__ __launch_bounds__(64 * kWaves) void k_box_gemm(BoxGemm g, int row_tiles)
{
    typedef typename Acc<PREC>::V V;
    typedef typename Acc<PREC>::T T;
    __shared__ V red[(kWaves - 1) * TM * TN * 64];
    const int cls = blockIdx.y;
    int pc[3], ncl[3];
    long nt = 1;
    for (int d = 0; d < 3; ++d) {
        pc[d] = (g.stride == 2 && d < g.D) ? (cls >> d) & 1 : 0;
        int n = (d < g.D) ? g.nl[d] : 1;
        int c = (n - pc[d] + g.stride - 1) / g.stride;
        ncl[d] = c < 0 ? 0 : c;
        nt *= ncl[d];
    }
    const int rt = blockIdx.x % row_tiles;
    const long col0 = (long)(blockIdx.x / row_tiles) * 16 * TN;
    if (col0 >= nt * g.B) return;                      // uniform over the block
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane >> 4;
    const int row0 = rt * 16 * TM;
    constexpr int LG = (PREC == ERT_BF16X3) ? 8 : 4;    // elements per lane per chunk

    // columns of this lane
    int tc[TN][3];
    long tlin[TN];
    int tb[TN];
    bool ok[TN];
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
        long col = col0 + 16 * tn + (lane & 15);
        ok[tn] = col < nt * g.B;
        long cc = ok[tn] ? col : 0;
        tb[tn] = (int)(cc / nt);
        long tp = cc - (long)tb[tn] * nt;
        int a0 = (int)(tp % ncl[0]);
        long r = tp / ncl[0];
        int a1 = (int)(r % ncl[1]);
        int a2 = (int)(r / ncl[1]);
        tc[tn][0] = g.stride * a0 + pc[0];
        tc[tn][1] = g.stride * a1 + pc[1];
        tc[tn][2] = g.stride * a2 + pc[2];
        tlin[tn] = tc[tn][0] + (long)g.nl[0] * (tc[tn][1] + (long)g.nl[1] * tc[tn][2]);
    }

    // tot: sum over offsets of the per-offset partial sums in acc (shorter
    // FP32 accumulation chains than one running sum)
    V acc[TM][TN], tot[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) tot[i][j] = V{0, 0, 0, 0};

    const BoxOffset* offs = g.offs + (long)cls * g.noff;
    for (int oi = 0; oi < g.noff; ++oi) {
        const BoxOffset o = offs[oi];
        const T* bp[TN];
        bool any = false;
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            const int s0 = tc[tn][0] + o.o0, s1 = tc[tn][1] + o.o1, s2 = tc[tn][2] + o.o2;
            const bool in = ok[tn] && s0 >= 0 && s0 < g.nl[0] && s1 >= 0 && s1 < g.nl[1] && s2 >= 0 &&
                            s2 < g.nl[2];
            const long sl = s0 + (long)g.nl[0] * (s1 + (long)g.nl[1] * s2);
            bp[tn] = in ? (const T*)g.W + ((long)tb[tn] * g.nbox + sl) * g.Kd + LG * grp : nullptr;
            any |= in;
        }
        if (!__any(any)) continue;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = V{0, 0, 0, 0};
        const long abase = ((long)o.op * g.M + row0 + (lane & 15)) * g.Kd + LG * grp;
        tile_reduce<PREC, TM, TN>(g.ops, g.ops_lo, abase, (long)16 * g.Kd, g.Kd, bp, wave, acc);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) tot[i][j] += acc[i][j];
    }
    if (wave > 0) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) red[(((wave - 1) * TM + tm) * TN + tn) * 64 + lane] = tot[tm][tn];
    }
    __syncthreads();
    if (wave != 0) return;
    T* Lo = (T*)g.L;
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            V s = tot[tm][tn];
            for (int w = 1; w < kWaves; ++w) s += red[(((w - 1) * TM + tm) * TN + tn) * 64 + lane];
            if (!ok[tn]) continue;
            T* col = Lo + ((long)tb[tn] * g.nbox + tlin[tn]) * g.M + row0 + 16 * tm;
            if constexpr (PREC == ERT_FP64) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    T* d = col + grp + 4 * i;
                    *d = g.accumulate ? *d + s[i] : s[i];
                }
            } else {
                V* d = (V*)(col + 4 * grp);
                *d = g.accumulate ? *d + s : s;
            }
        }
}

// ---------------------------------------------------- offset-stationary ----

// One tile (column tile `tile`, row tile `rtile`) of an offset-stationary product.
template <int PREC, int TM, int TN, bool TAB = false>
__device__ __forceinline__ void offset_tile(const OffsetGemm& g, long tile, int rtile)
{
    typedef typename Acc<PREC>::V V;
    typedef typename Acc<PREC>::T T;
    __shared__ V red[(kWaves - 1) * TM * TN * 64];
    const int grpi = g.pl.tile_group[tile];
    const long col0 = g.pl.tile_col0[tile];
    const int p0 = g.pl.gstart[grpi], np = g.pl.gstart[grpi + 1] - p0;
    if (col0 >= (long)np * g.B) return;                 // uniform over the block
    const int op = g.pl.gop[grpi];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane >> 4;
    const int row0 = rtile * 16 * TM;
    constexpr int LG = (PREC == ERT_BF16X3) ? 8 : 4;
    long pidx[TN];
    int pb[TN];
    const T* bp[TN];
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
        const long col = col0 + 16 * tn + (lane & 15);
        const bool ok = col < (long)np * g.B;
        const long cc = ok ? col : 0;
        pb[tn] = (int)(cc / np);
        pidx[tn] = ok ? p0 + (cc - (long)pb[tn] * np) : -1;
        bp[tn] = ok ? (const T*)g.W + ((long)pb[tn] * g.nbox + g.pl.ps[pidx[tn]]) * g.Kd + LG * grp : nullptr;
    }
    V acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = V{0, 0, 0, 0};
    if constexpr (TAB) {
        // op = (o0 + 1) + 3 (o1 + 1) + 9 (o2 + 1): the leaf offset of the group
        const int o0 = op % 3 - 1, o1 = (op / 3) % 3 - 1, o2 = g.dim == 3 ? op / 9 - 1 : 0;
        const int c = 2 * g.leaf - 1;
        const int base = (c + g.leaf * o0) + g.tw * (c + g.leaf * o1) + g.tw * g.tw * (g.dim == 3 ? c + g.leaf * o2 : 0);
        int tb[TM];
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) tb[tm] = base - tab_lin(g, row0 + 16 * tm + (lane & 15));
        tile_reduce_tab<PREC, TM, TN>(g, tb, LG * grp, bp, wave, acc);
    } else {
        const long abase = ((long)op * g.M + row0 + (lane & 15)) * g.Kd + LG * grp;
        tile_reduce<PREC, TM, TN>(g.ops, g.ops_lo, abase, (long)16 * g.Kd, g.Kd, bp, wave, acc);
    }
    if (wave > 0) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) red[(((wave - 1) * TM + tm) * TN + tn) * 64 + lane] = acc[tm][tn];
    }
    __syncthreads();
    if (wave != 0) return;
    T* St = (T*)g.stage;
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            V s = acc[tm][tn];
            for (int w = 1; w < kWaves; ++w) s += red[(((w - 1) * TM + tm) * TN + tn) * 64 + lane];
            if (pidx[tn] < 0) continue;
            T* col = St + ((long)pb[tn] * g.pl.npairs + pidx[tn]) * g.M + row0 + 16 * tm;
            if constexpr (PREC == ERT_FP64) {
#pragma unroll
                for (int i = 0; i < 4; ++i) col[grp + 4 * i] = s[i];
            } else {
                *(V*)(col + 4 * grp) = s;
            }
        }
}

template <int PREC, int TM, int TN, bool TAB = false>
__global__ __launch_bounds__(64 * kWaves) void k_offset_gemm(OffsetGemm g)
{
    offset_tile<PREC, TM, TN, TAB>(g, blockIdx.x, blockIdx.y);
}

// Two independent offset-stationary products in one launch (the near field and the
// far-field translations of a one-level tree): blocks [0, na) belong to the first.
template <int PREC, int TMA, int TNA, int TMB, int TNB, bool TABA = false>
__global__ __launch_bounds__(64 * kWaves) void k_offset_gemm2(OffsetGemm a, int rows_a, long na, OffsetGemm b,
                                                              int rows_b)
{
    // the row tiles of one column tile read the same source columns: keep them on one XCD
    const long bid = blockIdx.x;
    if (bid < na) {
        const long p = xcd_position(bid, na);
        offset_tile<PREC, TMA, TNA, TABA>(a, p / rows_a, (int)(p % rows_a));
    } else {
        const long nb = (long)gridDim.x - na;
        const long p = xcd_position(bid - na, nb, (int)(na & 7));
        offset_tile<PREC, TMB, TNB>(b, p / rows_b, (int)(p % rows_b));
    }
}

// Execution form 4 (FP32).  Workgroup = (16-column tile, 64 rows): the tile's 16
// source columns are staged in LDS once (row stride Kd + 4 floats, so that the 16
// lanes of a k-group read distinct banks); each wave reduces its 16 rows over the
// whole reduction length, the operator streamed from memory (or read from the
// offset table), kLdsU chunks of 16 in flight, even and odd chunks in two
// accumulators added at the end; no cross-wave sums.
constexpr int kLdsU = 4;

template <bool TAB>
__device__ __forceinline__ void lds_tile(const OffsetGemm& g, long tile, int rblk, float* sB)
{
    typedef v4f V;
    const int grpi = g.pl.tile_group[tile];
    const long col0 = g.pl.tile_col0[tile];
    const int p0 = g.pl.gstart[grpi], np = g.pl.gstart[grpi + 1] - p0;
    if (col0 >= (long)np * g.B) return;                 // uniform over the block
    const int op = g.pl.gop[grpi];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane >> 4;
    const int ld = g.Kd + 4, kq = g.Kd >> 2;
    for (int e = threadIdx.x; e < 16 * kq; e += blockDim.x) {
        const int c = e / kq, k4 = e - c * kq;
        const long col = col0 + c;
        V v = V{0.f, 0.f, 0.f, 0.f};
        if (col < (long)np * g.B) {
            const int pb = (int)(col / np);
            const long pidx = p0 + (col - (long)pb * np);
            v = *(const V*)((const float*)g.W + ((long)pb * g.nbox + g.pl.ps[pidx]) * g.Kd + 4 * k4);
        }
        *(V*)(sB + c * ld + 4 * k4) = v;
    }
    __syncthreads();
    const int row0 = rblk * 64 + wave * 16;
    if (row0 >= g.M) return;                            // uniform over the wave; no barrier follows
    const float* bl = sB + (lane & 15) * ld + 4 * grp;
    V acc0 = V{0.f, 0.f, 0.f, 0.f}, acc1 = V{0.f, 0.f, 0.f, 0.f};
    int tb = 0;
    const float* ar = nullptr;
    if constexpr (TAB) {
        const int o0 = op % 3 - 1, o1 = (op / 3) % 3 - 1, o2 = g.dim == 3 ? op / 9 - 1 : 0;
        const int c = 2 * g.leaf - 1;
        const int base = (c + g.leaf * o0) + g.tw * (c + g.leaf * o1) + g.tw * g.tw * (g.dim == 3 ? c + g.leaf * o2 : 0);
        tb = base - tab_lin(g, row0 + (lane & 15));
    } else {
        ar = (const float*)g.ops + ((long)op * g.M + row0 + (lane & 15)) * g.Kd + 4 * grp;
    }
    for (int k0 = 0; k0 < g.Kd; k0 += 16 * kLdsU) {
        V a[kLdsU], b[kLdsU];
#pragma unroll
        for (int u = 0; u < kLdsU; ++u) {
            const int kk = k0 + 16 * u;
            if (kk < g.Kd) {
                if constexpr (TAB) {
                    const int idx = tb + tab_lin(g, kk + 4 * grp);
                    const int r = idx & 3;
                    a[u] = *(const V*)((const float*)g.atab + r * g.tlen + (idx - r));
                } else {
                    a[u] = *(const V*)(ar + kk);
                }
                b[u] = *(const V*)(bl + kk);
            }
        }
#pragma unroll
        for (int u = 0; u < kLdsU; ++u) {
            if (k0 + 16 * u < g.Kd) {
                V& acc = (u & 1) ? acc1 : acc0;
#pragma unroll
                for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][e], b[u][e], acc, 0, 0, 0);
            }
        }
    }
    const long col = col0 + (lane & 15);
    if (col < (long)np * g.B) {
        const int pb = (int)(col / np);
        const long pidx = p0 + (col - (long)pb * np);
        *(V*)((float*)g.stage + ((long)pb * g.pl.npairs + pidx) * g.M + row0 + 4 * grp) = acc0 + acc1;
    }
}

template <bool TAB>
__global__ __launch_bounds__(256) void k_offset_lds(OffsetGemm g)
{
    extern __shared__ __align__(16) float lds_b[];
    lds_tile<TAB>(g, blockIdx.x, blockIdx.y, lds_b);
}

// both products of a one-level tree in form 4, in one launch
template <bool TABA>
__global__ __launch_bounds__(256) void k_offset_lds2(OffsetGemm a, int rows_a, long na, OffsetGemm b, int rows_b)
{
    extern __shared__ __align__(16) float lds_b[];
    const long bid = blockIdx.x;
    if (bid < na) {
        const long p = xcd_position(bid, na);
        lds_tile<TABA>(a, p / rows_a, (int)(p % rows_a), lds_b);
    } else {
        const long nb = (long)gridDim.x - na;
        const long p = xcd_position(bid - na, nb, (int)(na & 7));
        lds_tile<false>(b, p / rows_b, (int)(p % rows_b), lds_b);
    }
}

// Execution form 5 (FP32).  Workgroup = one 64-column tile over all rows of the
// product: the tile's 64 source columns are staged in LDS once (row stride Kd + 4
// floats); wave w takes the 16-row blocks w, w + 4, ... and reduces each over the
// whole reduction length against all 64 columns, so every operator fragment feeds
// four MFMA column blocks (a quarter of the operator reads of form 4).  A wave holds
// its block's operator rows in registers (Kd / 16 fragments per lane, read from
// memory or from the offset table) and loads the next block's while it multiplies
// this one; the loads are unconditional (a wave past its last block re-reads that
// block's rows), so the wait before a block leaves the next block's loads in flight.
constexpr int kLds64K = 15;   // fragments of 16 reduction indices per lane: Kd <= 240

// KS = Kd / 16 reduction fragments per lane (a compile-time count: no branch around a load)
template <bool TAB, int KS>
__device__ __forceinline__ void lds64_tile(const OffsetGemm& g, long tile, float* sB)
{
    typedef v4f V;
    const int grpi = g.pl.tile_group4[tile];
    const long col0 = g.pl.tile_col04[tile];
    const int p0 = g.pl.gstart[grpi], np = g.pl.gstart[grpi + 1] - p0;
    if (col0 >= (long)np * g.B) return;                 // uniform over the block
    const int op = g.pl.gop[grpi];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: a scalar loop
    const int lane = threadIdx.x & 63, grp = lane >> 4;
    const int ld = g.Kd + 4, kq = g.Kd >> 2, MB = g.M >> 4;
    int tbase = 0;
    if constexpr (TAB) {
        const int o0 = op % 3 - 1, o1 = (op / 3) % 3 - 1, o2 = g.dim == 3 ? op / 9 - 1 : 0;
        const int c = 2 * g.leaf - 1;
        tbase = (c + g.leaf * o0) + g.tw * (c + g.leaf * o1) + g.tw * g.tw * (g.dim == 3 ? c + g.leaf * o2 : 0);
    }
    // the operator fragments of row block rb (rows 16 rb + lane % 16, reduction indices
    // 16 ks + 4 grp .. + 3)
    auto load_a = [&](int rb, V (&a)[KS]) {
        const int row = 16 * rb + (lane & 15);
        if constexpr (TAB) {
            const int tb = tbase - tab_lin(g, row);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int idx = tb + tab_lin(g, 16 * ks + 4 * grp);
                const int r = idx & 3;
                a[ks] = *(const V*)((const float*)g.atab + r * g.tlen + (idx - r));
            }
        } else {
            const float* ar = (const float*)g.ops + ((long)op * g.M + row) * g.Kd + 4 * grp;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) a[ks] = *(const V*)(ar + 16 * ks);
        }
    };
    V a0[KS], a1[KS];
    load_a(wave < MB ? wave : MB - 1, a0);
    for (int e = threadIdx.x; e < 64 * kq; e += blockDim.x) {
        const int c = e / kq, k4 = e - c * kq;
        const long col = col0 + c;
        V v = V{0.f, 0.f, 0.f, 0.f};
        if (col < (long)np * g.B) {
            const int pb = (int)(col / np);
            const long pidx = p0 + (col - (long)pb * np);
            v = *(const V*)((const float*)g.W + ((long)pb * g.nbox + g.pl.ps[pidx]) * g.Kd + 4 * k4);
        }
        *(V*)(sB + c * ld + 4 * k4) = v;
    }
    __syncthreads();
    long pidx[4];
    int pb[4];
#pragma unroll
    for (int tn = 0; tn < 4; ++tn) {
        const long col = col0 + 16 * tn + (lane & 15);
        const bool ok = col < (long)np * g.B;
        const long cc = ok ? col : 0;
        pb[tn] = (int)(cc / np);
        pidx[tn] = ok ? p0 + (cc - (long)pb[tn] * np) : -1;
    }
    const float* bl = sB + (lane & 15) * ld + 4 * grp;
    auto block = [&](int rb, const V (&a)[KS]) {
        V acc[4];
#pragma unroll
        for (int tn = 0; tn < 4; ++tn) acc[tn] = V{0.f, 0.f, 0.f, 0.f};
        // the source fragments are read from LDS anew for every row block: an offset the
        // compiler cannot see through keeps it from hoisting all KS x 4 of them into
        // registers (which would leave one wave per SIMD)
        int off = 0;
        asm volatile("" : "+v"(off));
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            V b[4];
#pragma unroll
            for (int tn = 0; tn < 4; ++tn) b[tn] = *(const V*)(bl + off + tn * 16 * ld + 16 * ks);
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int tn = 0; tn < 4; ++tn)
                    acc[tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks][e], b[tn][e], acc[tn], 0, 0, 0);
        }
#pragma unroll
        for (int tn = 0; tn < 4; ++tn)
            if (pidx[tn] >= 0)
                *(V*)((float*)g.stage + ((long)pb[tn] * g.pl.npairs + pidx[tn]) * g.M + 16 * rb + 4 * grp) = acc[tn];
    };
    for (int rb = wave; rb < MB; rb += 2 * kWaves) {
        const int r1 = rb + kWaves;
        load_a(r1 < MB ? r1 : rb, a1);
        block(rb, a0);
        if (r1 >= MB) break;                            // uniform over the wave
        const int r2 = r1 + kWaves;
        load_a(r2 < MB ? r2 : r1, a0);
        block(r1, a1);
    }
}

// tiles of one offset group are consecutive: keep them on one XCD (its L2 holds the operator)
template <bool TAB, int KS>
__global__ __launch_bounds__(256) void k_offset_lds64(OffsetGemm g)
{
    extern __shared__ __align__(16) float lds_b[];
    lds64_tile<TAB, KS>(g, xcd_position(blockIdx.x, gridDim.x), lds_b);
}

template <bool TAB, int KS = 1>
void launch_lds64(hipStream_t s, const OffsetGemm& g, size_t sh)
{
    if constexpr (KS <= kLds64K) {
        if (g.Kd == 16 * KS) hipLaunchKernelGGL((k_offset_lds64<TAB, KS>), dim3((unsigned)g.pl.ntiles4), dim3(256), sh, s, g);
        else launch_lds64<TAB, KS + 1>(s, g, sh);
    }
}

// Per-target sums of the staged pair products, in a fixed order: one workgroup
// per (target, 64-row slab, rhs); its four waves sum four consecutive quarters
// of the target's pair list (8 row loads in flight per lane) and wave 0 adds
// the quarters in order.
template <typename T>
__device__ __forceinline__ void stage_reduce_block(const OffsetGemm& g, int rslabs, long blk)
{
    __shared__ T part[3][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rs = (int)(blk % rslabs);
    blk /= rslabs;
    const long t = blk % g.nbox;
    const int b = (int)(blk / g.nbox);
    const int r = rs * 64 + lane;
    const bool ok = r < g.M;
    const T* St = (const T*)g.stage + (long)b * g.pl.npairs * g.M + (ok ? r : 0);
    const int k0 = g.pl.tstart[t], k1 = g.pl.tstart[t + 1];
    const int per = (k1 - k0 + 3) / 4;
    const int a0 = k0 + wave * per;
    const int a1 = (a0 + per) < k1 ? (a0 + per) : k1;
    T s = T(0);
    int k = a0;
    for (; k + 8 <= a1; k += 8) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = St[(long)g.pl.tpairs[k + u] * g.M];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; k < a1; ++k) s += St[(long)g.pl.tpairs[k] * g.M];
    if (wave > 0) part[wave - 1][lane] = s;
    __syncthreads();
    if (wave != 0 || !ok) return;
    s = s + part[0][lane] + part[1][lane] + part[2][lane];
    T* d = (T*)g.L + ((long)b * g.nbox + t) * g.M + r;
    *d = g.accumulate ? *d + s : s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_stage_reduce(OffsetGemm g, int rslabs)
{
    stage_reduce_block<T>(g, rslabs, blockIdx.x);
}

constexpr int kTM = 2, kTN = 2;

}  // namespace

ert_status box_gemm(hipStream_t s, int prec, const BoxGemm& g)
{
    if (g.M % (16 * kTM) != 0 || g.Kd % 32 != 0) {
        record_error("box_gemm: row count must be a multiple of 32 and the reduction length of 32");
        return ERT_EINVAL;
    }
    const int row_tiles = g.M / (16 * kTM);
    long max_nt = 0;
    for (int c = 0; c < g.nclass; ++c) {
        long nt = 1;
        for (int d = 0; d < g.D; ++d) {
            int pc = (g.stride == 2) ? (c >> d) & 1 : 0;
            int n = (g.nl[d] - pc + g.stride - 1) / g.stride;
            nt *= n > 0 ? n : 0;
        }
        max_nt = nt > max_nt ? nt : max_nt;
    }
    const long col_tiles = (max_nt * g.B + 16 * kTN - 1) / (16 * kTN);
    if (col_tiles == 0) return ERT_OK;
    if ((long)row_tiles * col_tiles * g.nclass < 512) {
        // small products: 16 x 16 tiles for four times as many workgroups
        const int rt1 = g.M / 16;
        const long ct1 = (max_nt * g.B + 15) / 16;
        dim3 grid((unsigned)(rt1 * ct1), (unsigned)g.nclass);
        if (prec == ERT_FP64)
            hipLaunchKernelGGL((k_box_gemm<ERT_FP64, 1, 1>), grid, dim3(64 * kWaves), 0, s, g, rt1);
        else if (prec == ERT_FP32)
            hipLaunchKernelGGL((k_box_gemm<ERT_FP32, 1, 1>), grid, dim3(64 * kWaves), 0, s, g, rt1);
        else
            hipLaunchKernelGGL((k_box_gemm<ERT_BF16X3, 1, 1>), grid, dim3(64 * kWaves), 0, s, g, rt1);
        ERT_HIP(hipGetLastError());
        return ERT_OK;
    }
    dim3 grid((unsigned)(row_tiles * col_tiles), (unsigned)g.nclass);
    if (prec == ERT_FP64)
        hipLaunchKernelGGL((k_box_gemm<ERT_FP64, kTM, kTN>), grid, dim3(64 * kWaves), 0, s, g, row_tiles);
    else if (prec == ERT_FP32)
        hipLaunchKernelGGL((k_box_gemm<ERT_FP32, kTM, kTN>), grid, dim3(64 * kWaves), 0, s, g, row_tiles);
    else
        hipLaunchKernelGGL((k_box_gemm<ERT_BF16X3, kTM, kTN>), grid, dim3(64 * kWaves), 0, s, g, row_tiles);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

bool offset_lds_ok(int prec, const OffsetGemm& g)
{
    return prec == ERT_FP32 && g.M % 16 == 0 && g.Kd % 16 == 0 && 16L * (g.Kd + 4) * 4 <= 65536;
}

bool offset_lds64_ok(int prec, const OffsetGemm& g)
{
    return prec == ERT_FP32 && g.M % 16 == 0 && g.Kd % 16 == 0 && g.Kd <= 16 * kLds64K &&
           64L * (g.Kd + 4) * 4 <= 65536;
}

ert_status offset_gemm_products(hipStream_t s, int prec, const OffsetGemm& g)
{
    if (g.M % (16 * kTM) != 0 || g.Kd % 32 != 0) {
        record_error("offset_gemm: row count must be a multiple of 32 and the reduction length of 32");
        return ERT_EINVAL;
    }
    if (g.lds == 2) {
        if (!offset_lds64_ok(prec, g)) {
            record_error("offset_gemm: execution form 5 needs FP32 and a reduction length of at most 240");
            return ERT_EINVAL;
        }
        if (g.pl.ntiles4 > 0) {
            const size_t sh = 64 * (size_t)(g.Kd + 4) * sizeof(float);
            if (g.atab) launch_lds64<true>(s, g, sh);
            else launch_lds64<false>(s, g, sh);
            ERT_HIP(hipGetLastError());
        }
        return ERT_OK;
    }
    if (g.lds) {
        if (!offset_lds_ok(prec, g)) {
            record_error("offset_gemm: execution form 4 needs FP32 and a reduction length of at most 1020");
            return ERT_EINVAL;
        }
        if (g.pl.ntiles > 0) {
            const dim3 grid((unsigned)g.pl.ntiles, (unsigned)((g.M + 63) / 64));
            const size_t sh = 16 * (size_t)(g.Kd + 4) * sizeof(float);
            if (g.atab) hipLaunchKernelGGL(k_offset_lds<true>, grid, dim3(256), sh, s, g);
            else hipLaunchKernelGGL(k_offset_lds<false>, grid, dim3(256), sh, s, g);
            ERT_HIP(hipGetLastError());
        }
        return ERT_OK;
    }
    if (g.tn == 4) {
        if (g.pl.ntiles4 > 0) {
            OffsetGemm g4 = g;
            g4.pl.tile_group = g.pl.tile_group4;
            g4.pl.tile_col0 = g.pl.tile_col04;
            const int tm = g.tm == 1 ? 1 : kTM;
            dim3 grid((unsigned)g.pl.ntiles4, (unsigned)(g.M / (16 * tm)));
#define ERT_OFF4(TM_)                                                                                   \
    if (prec == ERT_FP64 && g.atab) hipLaunchKernelGGL((k_offset_gemm<ERT_FP64, TM_, 4, true>), grid, dim3(64 * kWaves), 0, s, g4); \
    else if (prec == ERT_FP32 && g.atab) hipLaunchKernelGGL((k_offset_gemm<ERT_FP32, TM_, 4, true>), grid, dim3(64 * kWaves), 0, s, g4); \
    else if (prec == ERT_FP64) hipLaunchKernelGGL((k_offset_gemm<ERT_FP64, TM_, 4>), grid, dim3(64 * kWaves), 0, s, g4); \
    else if (prec == ERT_FP32) hipLaunchKernelGGL((k_offset_gemm<ERT_FP32, TM_, 4>), grid, dim3(64 * kWaves), 0, s, g4); \
    else hipLaunchKernelGGL((k_offset_gemm<ERT_BF16X3, TM_, 4>), grid, dim3(64 * kWaves), 0, s, g4);
            if (tm == 1) {
                ERT_OFF4(1)
            } else {
                ERT_OFF4(kTM)
            }
#undef ERT_OFF4
            ERT_HIP(hipGetLastError());
        }
    } else if (g.pl.ntiles > 0) {
        dim3 grid((unsigned)g.pl.ntiles, (unsigned)(g.M / (16 * kTM)));
        if (prec == ERT_FP64 && g.atab)
            hipLaunchKernelGGL((k_offset_gemm<ERT_FP64, kTM, 1, true>), grid, dim3(64 * kWaves), 0, s, g);
        else if (prec == ERT_FP32 && g.atab)
            hipLaunchKernelGGL((k_offset_gemm<ERT_FP32, kTM, 1, true>), grid, dim3(64 * kWaves), 0, s, g);
        else if (prec == ERT_FP64)
            hipLaunchKernelGGL((k_offset_gemm<ERT_FP64, kTM, 1>), grid, dim3(64 * kWaves), 0, s, g);
        else if (prec == ERT_FP32)
            hipLaunchKernelGGL((k_offset_gemm<ERT_FP32, kTM, 1>), grid, dim3(64 * kWaves), 0, s, g);
        else
            hipLaunchKernelGGL((k_offset_gemm<ERT_BF16X3, kTM, 1>), grid, dim3(64 * kWaves), 0, s, g);
        ERT_HIP(hipGetLastError());
    }
    return ERT_OK;
}

ert_status offset_gemm_reduce(hipStream_t s, int prec, const OffsetGemm& g)
{
    const int rslabs = (g.M + 63) / 64;
    const long nblk = g.nbox * rslabs * g.B;
    if (prec == ERT_FP64)
        hipLaunchKernelGGL(k_stage_reduce<double>, dim3((unsigned)nblk), dim3(256), 0, s, g, rslabs);
    else
        hipLaunchKernelGGL(k_stage_reduce<float>, dim3((unsigned)nblk), dim3(256), 0, s, g, rslabs);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

namespace {

// Tile arrays and row-tile count of the form a product runs in.
OffsetGemm with_form(const OffsetGemm& g, int* rows, long* nblk)
{
    OffsetGemm o = g;
    const int tm = (g.tn == 4 && g.tm == 1) ? 1 : kTM;
    if (g.tn == 4) {
        o.pl.tile_group = g.pl.tile_group4;
        o.pl.tile_col0 = g.pl.tile_col04;
    }
    *rows = g.M / (16 * tm);
    *nblk = (g.tn == 4 ? g.pl.ntiles4 : g.pl.ntiles) * (long)*rows;
    return o;
}

template <int PREC, int TMA, int TNA, bool TABA>
void launch_pair_b(hipStream_t s, const OffsetGemm& a, int ra, long na, const OffsetGemm& b, int rb, long nb,
                   int fb)
{
    const dim3 grid((unsigned)(na + nb)), blk(64 * kWaves);
    if (fb == 1)
        hipLaunchKernelGGL((k_offset_gemm2<PREC, TMA, TNA, kTM, 1, TABA>), grid, blk, 0, s, a, ra, na, b, rb);
    else if (fb == 2)
        hipLaunchKernelGGL((k_offset_gemm2<PREC, TMA, TNA, kTM, 4, TABA>), grid, blk, 0, s, a, ra, na, b, rb);
    else
        hipLaunchKernelGGL((k_offset_gemm2<PREC, TMA, TNA, 1, 4, TABA>), grid, blk, 0, s, a, ra, na, b, rb);
}

template <int PREC, bool TABA>
void launch_pair_a(hipStream_t s, const OffsetGemm& a, int ra, long na, int fa, const OffsetGemm& b, int rb, long nb,
                   int fb)
{
    if (fa == 1) launch_pair_b<PREC, kTM, 1, TABA>(s, a, ra, na, b, rb, nb, fb);
    else if (fa == 2) launch_pair_b<PREC, kTM, 4, TABA>(s, a, ra, na, b, rb, nb, fb);
    else launch_pair_b<PREC, 1, 4, TABA>(s, a, ra, na, b, rb, nb, fb);
}

// the first product may read its operator from an offset table (FP32/FP64)
template <int PREC>
void launch_pair(hipStream_t s, const OffsetGemm& a, int ra, long na, int fa, const OffsetGemm& b, int rb, long nb,
                 int fb)
{
    if constexpr (PREC != ERT_BF16X3) {
        if (a.atab) {
            launch_pair_a<PREC, true>(s, a, ra, na, fa, b, rb, nb, fb);
            return;
        }
    }
    launch_pair_a<PREC, false>(s, a, ra, na, fa, b, rb, nb, fb);
}

int form_of(const OffsetGemm& g) { return g.lds == 2 ? 5 : g.lds ? 4 : g.tn == 4 ? (g.tm == 1 ? 3 : 2) : 1; }

}  // namespace

ert_status offset_gemm_pair_products(hipStream_t s, int prec, const OffsetGemm& a, const OffsetGemm& b)
{
    for (const OffsetGemm* g : {&a, &b})
        if (g->M % (16 * kTM) != 0 || g->Kd % 32 != 0) {
            record_error("offset_gemm: row count must be a multiple of 32 and the reduction length of 32");
            return ERT_EINVAL;
        }
    if (b.atab || (a.atab && prec == ERT_BF16X3)) {
        record_error("offset_gemm: only the first product of a pair, in FP32/FP64, reads an offset table");
        return ERT_EINVAL;
    }
    if (a.lds != b.lds || a.lds == 2) {         // forms of both kinds, or form 5: two launches
        ERT_TRY(offset_gemm_products(s, prec, a));
        return offset_gemm_products(s, prec, b);
    }
    if (a.lds) {
        if (!offset_lds_ok(prec, a) || !offset_lds_ok(prec, b)) {
            record_error("offset_gemm: execution form 4 needs FP32 and a reduction length of at most 1020");
            return ERT_EINVAL;
        }
        const int ra4 = (a.M + 63) / 64, rb4 = (b.M + 63) / 64;
        const long na4 = a.pl.ntiles * ra4, nb4 = b.pl.ntiles * rb4;
        if (na4 + nb4 == 0) return ERT_OK;
        const size_t sh = 16 * (size_t)(std::max(a.Kd, b.Kd) + 4) * sizeof(float);
        if (a.atab)
            hipLaunchKernelGGL(k_offset_lds2<true>, dim3((unsigned)(na4 + nb4)), dim3(256), sh, s, a, ra4, na4, b, rb4);
        else
            hipLaunchKernelGGL(k_offset_lds2<false>, dim3((unsigned)(na4 + nb4)), dim3(256), sh, s, a, ra4, na4, b, rb4);
        ERT_HIP(hipGetLastError());
        return ERT_OK;
    }
    int ra, rb;
    long na, nb;
    const OffsetGemm ga = with_form(a, &ra, &na), gb = with_form(b, &rb, &nb);
    if (na + nb == 0) return ERT_OK;
    if (prec == ERT_FP64) launch_pair<ERT_FP64>(s, ga, ra, na, form_of(a), gb, rb, nb, form_of(b));
    else if (prec == ERT_FP32) launch_pair<ERT_FP32>(s, ga, ra, na, form_of(a), gb, rb, nb, form_of(b));
    else launch_pair<ERT_BF16X3>(s, ga, ra, na, form_of(a), gb, rb, nb, form_of(b));
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ert_status offset_gemm(hipStream_t s, int prec, const OffsetGemm& g)
{
    ERT_TRY(offset_gemm_products(s, prec, g));
    return offset_gemm_reduce(s, prec, g);
}

}  // namespace ertvie
