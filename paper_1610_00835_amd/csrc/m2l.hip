// Far-field translations of the Chebyshev FMM (Sec. 3.3, eq. EQ: M2L):
// f2(p_m) = sum_{m'} K(L p_m, R q_m') f1(q_m'), summed over the interaction
// list of every target box.
//
// Homogeneous media: the translation matrix depends only on the level and the
// box offset, so each level is one batched GEMM on the matrix cores.  Targets
// are grouped in the 2^d classes of their index parity: all targets of a class
// share the same 6^d - 3^d interaction offsets, so one workgroup owns a tile
// of (target node rows) x (target box, right-hand side) columns and runs the
// reduction over (offset, source node).  The four waves of a workgroup split
// the offsets and their partial sums are combined in LDS in a fixed order, so
// results are bitwise reproducible.  Operands go straight from global memory
// (L2-resident operators, gathered multipoles) into MFMA registers: each lane
// loads 16 contiguous bytes along the reduction dimension, and the order in
// which the reduction index is fed to the MFMA steps is permuted accordingly
// (the same permutation for both operands, so the product is unchanged).
//
// Heterogeneous media: every (target, source) pair has its own matrix, cached
// at plan time; the translation is a batched GEMV/GEMM that streams those
// matrices once per apply (HBM-bound).
#include "fmm.hpp"

namespace ertvie {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kWaves = 4;

struct ClassInfo {
    int pc[3];      // parity of the class
    int ncl[3];     // targets of the class per axis
    long nt;        // targets in the class
};

__device__ __forceinline__ ClassInfo class_info(const M2LArgs& a, int cls)
{
    ClassInfo ci;
    ci.nt = 1;
    for (int d = 0; d < 3; ++d) {
        ci.pc[d] = (d < a.D) ? (cls >> d) & 1 : 0;
        int n = (d < a.D) ? a.nl[d] : 1;
        int c = (n - ci.pc[d] + 1) / 2;
        ci.ncl[d] = c < 0 ? 0 : c;
        ci.nt *= ci.ncl[d];
    }
    return ci;
}

// number of per-axis offset choices for one class (children of the parent's
// neighbours): o in [-2 - p, 3 - p]
constexpr int kSpan = 6;

template <int TN>
struct Cols {
    int t[TN][3];
    long tlin[TN];
    int b[TN];
    bool ok[TN];
};

template <int TN>
__device__ __forceinline__ void column_setup(const M2LArgs& a, const ClassInfo& ci, long col0, int lane, Cols<TN>& c)
{
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
        long col = col0 + 16 * tn + (lane & 15);
        c.ok[tn] = col < ci.nt * a.B;
        long cc = c.ok[tn] ? col : 0;
        c.b[tn] = (int)(cc / (ci.nt > 0 ? ci.nt : 1));
        long tp = cc - (long)c.b[tn] * ci.nt;
        int t0 = (int)(tp % (ci.ncl[0] > 0 ? ci.ncl[0] : 1));
        long r = tp / (ci.ncl[0] > 0 ? ci.ncl[0] : 1);
        int t1 = (int)(r % (ci.ncl[1] > 0 ? ci.ncl[1] : 1));
        int t2 = (int)(r / (ci.ncl[1] > 0 ? ci.ncl[1] : 1));
        c.t[tn][0] = 2 * t0 + ci.pc[0];
        c.t[tn][1] = 2 * t1 + ci.pc[1];
        c.t[tn][2] = 2 * t2 + ci.pc[2];
        c.tlin[tn] = c.t[tn][0] + (long)a.nl[0] * (c.t[tn][1] + (long)a.nl[1] * c.t[tn][2]);
    }
}

// source box of column tn under offset o; -1 when outside the lattice
template <int TN>
__device__ __forceinline__ long source_box(const M2LArgs& a, const Cols<TN>& c, int tn, const int o[3])
{
    if (!c.ok[tn]) return -1;
    long lin = 0, stride = 1;
    for (int d = 0; d < 3; ++d) {
        int n = (d < a.D) ? a.nl[d] : 1;
        int s = c.t[tn][d] + o[d];
        if (s < 0 || s >= n) return -1;
        lin += stride * s;
        stride *= n;
    }
    return lin;
}

__device__ __forceinline__ bool decode_offset(const M2LArgs& a, const ClassInfo& ci, int idx, int o[3], int* oidx)
{
    int near = 1;
    int lin = 0, stride = 1;
    int rem = idx;
    for (int d = 0; d < 3; ++d) {
        if (d < a.D) {
            int k = rem % kSpan;
            rem /= kSpan;
            o[d] = k - 2 - ci.pc[d];
            if (o[d] < -1 || o[d] > 1) near = 0;
            lin += stride * (o[d] + 3);
            stride *= kOffSide;
        } else {
            o[d] = 0;
        }
    }
    *oidx = lin;
    return !near;
}

// ------------------------------------------------------------------ FP32 ----

template <int TM, int TN>
__global__ __launch_bounds__(64 * kWaves) void k_m2l_f32(M2LArgs a, int row_tiles)
{
    __shared__ v4f red[(kWaves - 1) * TM * TN * 64];
    const int cls = blockIdx.y;
    const ClassInfo ci = class_info(a, cls);
    const int rt = blockIdx.x % row_tiles;
    const long ct = blockIdx.x / row_tiles;
    const long col0 = ct * 16 * TN;
    if (col0 >= ci.nt * a.B) return;                  // uniform over the block
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4;
    const int row0 = rt * 16 * TM;
    Cols<TN> cols;
    column_setup<TN>(a, ci, col0, lane, cols);
    const float* ops = (const float*)a.ops;
    const float* W = (const float*)a.W;
    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    int total = 1;
    for (int d = 0; d < a.D; ++d) total *= kSpan;
    for (int idx = wave; idx < total; idx += kWaves) {
        int o[3], oidx;
        if (!decode_offset(a, ci, idx, o, &oidx)) continue;
        const float* bp[TN];
        bool any = false;
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            long s = source_box<TN>(a, cols, tn, o);
            bp[tn] = s >= 0 ? W + ((long)cols.b[tn] * a.nbox + s) * a.Kp + 4 * g : nullptr;
            any |= (s >= 0);
        }
        if (!__any(any)) continue;
        const float* ap[TM];
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
            ap[tm] = ops + ((long)oidx * a.Kp + row0 + 16 * tm + (lane & 15)) * a.Kp + 4 * g;
        for (int kk = 0; kk < a.Kp; kk += 16) {
            v4f av[TM], bv[TN];
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) av[tm] = *(const v4f*)(ap[tm] + kk);
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) bv[tn] = bp[tn] ? *(const v4f*)(bp[tn] + kk) : v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                    for (int tn = 0; tn < TN; ++tn)
                        acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[tm][e], bv[tn][e], acc[tm][tn], 0, 0, 0);
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) red[(((wave - 1) * TM + tm) * TN + tn) * 64 + lane] = acc[tm][tn];
    }
    __syncthreads();
    if (wave != 0) return;
    float* Lo = (float*)a.L;
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            v4f s = acc[tm][tn];
            for (int w = 1; w < kWaves; ++w) s += red[(((w - 1) * TM + tm) * TN + tn) * 64 + lane];
            if (!cols.ok[tn]) continue;
            // output layout: lane holds rows 4*(lane/16) + i of column lane % 16
            float* dst = Lo + ((long)cols.b[tn] * a.nbox + cols.tlin[tn]) * a.Kp + row0 + 16 * tm + 4 * g;
            v4f cur = *(v4f*)dst;
            *(v4f*)dst = cur + s;
        }
}

// ------------------------------------------------------------------ FP64 ----

template <int TM, int TN>
__global__ __launch_bounds__(64 * kWaves) void k_m2l_f64(M2LArgs a, int row_tiles)
{
    __shared__ v4d red[(kWaves - 1) * TM * TN * 64];
    const int cls = blockIdx.y;
    const ClassInfo ci = class_info(a, cls);
    const int rt = blockIdx.x % row_tiles;
    const long ct = blockIdx.x / row_tiles;
    const long col0 = ct * 16 * TN;
    if (col0 >= ci.nt * a.B) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4;
    const int row0 = rt * 16 * TM;
    Cols<TN> cols;
    column_setup<TN>(a, ci, col0, lane, cols);
    const double* ops = (const double*)a.ops;
    const double* W = (const double*)a.W;
    v4d acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    int total = 1;
    for (int d = 0; d < a.D; ++d) total *= kSpan;
    for (int idx = wave; idx < total; idx += kWaves) {
        int o[3], oidx;
        if (!decode_offset(a, ci, idx, o, &oidx)) continue;
        const double* bp[TN];
        bool any = false;
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            long s = source_box<TN>(a, cols, tn, o);
            bp[tn] = s >= 0 ? W + ((long)cols.b[tn] * a.nbox + s) * a.Kp + 4 * g : nullptr;
            any |= (s >= 0);
        }
        if (!__any(any)) continue;
        const double* ap[TM];
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
            ap[tm] = ops + ((long)oidx * a.Kp + row0 + 16 * tm + (lane & 15)) * a.Kp + 4 * g;
        for (int kk = 0; kk < a.Kp; kk += 16) {
            v4d av[TM], bv[TN];
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) av[tm] = *(const v4d*)(ap[tm] + kk);
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) bv[tn] = bp[tn] ? *(const v4d*)(bp[tn] + kk) : v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                    for (int tn = 0; tn < TN; ++tn)
                        acc[tm][tn] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[tm][e], bv[tn][e], acc[tm][tn], 0, 0, 0);
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) red[(((wave - 1) * TM + tm) * TN + tn) * 64 + lane] = acc[tm][tn];
    }
    __syncthreads();
    if (wave != 0) return;
    double* Lo = (double*)a.L;
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            v4d s = acc[tm][tn];
            for (int w = 1; w < kWaves; ++w) s += red[(((w - 1) * TM + tm) * TN + tn) * 64 + lane];
            if (!cols.ok[tn]) continue;
            // FP64 output layout: lane holds rows (lane/16) + 4*i of column lane % 16
            double* dst = Lo + ((long)cols.b[tn] * a.nbox + cols.tlin[tn]) * a.Kp + row0 + 16 * tm + g;
#pragma unroll
            for (int i = 0; i < 4; ++i) dst[4 * i] += s[i];
        }
}

// --------------------------------------------------------------- BF16x3 ----
// A = A_hi + A_lo (bf16 pair, split at plan time), B split the same way on the
// fly; A B ~ A_hi B_hi + A_hi B_lo + A_lo B_hi accumulated in FP32.

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

template <int TM, int TN>
__global__ __launch_bounds__(64 * kWaves) void k_m2l_bf16x3(M2LArgs a, int row_tiles)
{
    __shared__ v4f red[(kWaves - 1) * TM * TN * 64];
    const int cls = blockIdx.y;
    const ClassInfo ci = class_info(a, cls);
    const int rt = blockIdx.x % row_tiles;
    const long ct = blockIdx.x / row_tiles;
    const long col0 = ct * 16 * TN;
    if (col0 >= ci.nt * a.B) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4;
    const int row0 = rt * 16 * TM;
    Cols<TN> cols;
    column_setup<TN>(a, ci, col0, lane, cols);
    const __bf16* ohi = (const __bf16*)a.ops;
    const __bf16* olo = (const __bf16*)a.ops_lo;
    const float* W = (const float*)a.W;
    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    int total = 1;
    for (int d = 0; d < a.D; ++d) total *= kSpan;
    for (int idx = wave; idx < total; idx += kWaves) {
        int o[3], oidx;
        if (!decode_offset(a, ci, idx, o, &oidx)) continue;
        const float* bp[TN];
        bool any = false;
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            long s = source_box<TN>(a, cols, tn, o);
            bp[tn] = s >= 0 ? W + ((long)cols.b[tn] * a.nbox + s) * a.Kp + 8 * g : nullptr;
            any |= (s >= 0);
        }
        if (!__any(any)) continue;
        long arow[TM];
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
            arow[tm] = ((long)oidx * a.Kp + row0 + 16 * tm + (lane & 15)) * a.Kp + 8 * g;
        for (int kk = 0; kk < a.Kp; kk += 32) {
            v8bf ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) {
                ah[tm] = *(const v8bf*)(ohi + arow[tm] + kk);
                al[tm] = *(const v8bf*)(olo + arow[tm] + kk);
            }
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) {
                v4f x0 = v4f{0.f, 0.f, 0.f, 0.f}, x1 = x0;
                if (bp[tn]) {
                    x0 = *(const v4f*)(bp[tn] + kk);
                    x1 = *(const v4f*)(bp[tn] + kk + 4);
                }
                split_bf16(x0, x1, bh[tn], bl[tn]);
            }
#pragma unroll
            for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                for (int tn = 0; tn < TN; ++tn) {
                    acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[tm], bh[tn], acc[tm][tn], 0, 0, 0);
                    acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[tm], bl[tn], acc[tm][tn], 0, 0, 0);
                    acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[tm], bh[tn], acc[tm][tn], 0, 0, 0);
                }
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) red[(((wave - 1) * TM + tm) * TN + tn) * 64 + lane] = acc[tm][tn];
    }
    __syncthreads();
    if (wave != 0) return;
    float* Lo = (float*)a.L;
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            v4f s = acc[tm][tn];
            for (int w = 1; w < kWaves; ++w) s += red[(((w - 1) * TM + tm) * TN + tn) * 64 + lane];
            if (!cols.ok[tn]) continue;
            float* dst = Lo + ((long)cols.b[tn] * a.nbox + cols.tlin[tn]) * a.Kp + row0 + 16 * tm + 4 * g;
            v4f cur = *(v4f*)dst;
            *(v4f*)dst = cur + s;
        }
}

// ------------------------------------------------- heterogeneous (cached) ----
// One workgroup per (target box, block of right-hand sides).  Thread r owns
// target node r; for each source of the target's list the source multipoles of
// the RHS block are staged in LDS and the cached matrix (stored source-node
// major, so consecutive threads read consecutive rows) is streamed once.

template <typename T, int RB>
__global__ __launch_bounds__(256) void k_m2l_het(M2LArgs a, const T* __restrict__ opsT)
{
    extern __shared__ unsigned char smem[];
    T* ws = (T*)smem;                      // [RB][Kp]
    const long t = blockIdx.x;
    const int b0 = blockIdx.y * RB;
    const int nb = (a.B - b0) < RB ? (a.B - b0) : RB;
    const T* W = (const T*)a.W;
    T* Lo = (T*)a.L;
    const long p0 = a.pair_start[t], p1 = a.pair_start[t + 1];
    for (int r0 = 0; r0 < a.Kp; r0 += 256) {
        const int r = r0 + threadIdx.x;
        T acc[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) acc[b] = T(0);
        for (long p = p0; p < p1; ++p) {
            const long s = a.pair_src[p];
            __syncthreads();
            for (int i = threadIdx.x; i < RB * a.Kp; i += 256) {
                int b = i / a.Kp, k = i - b * a.Kp;
                ws[i] = (b < nb) ? W[((long)(b0 + b) * a.nbox + s) * a.Kp + k] : T(0);
            }
            __syncthreads();
            if (r < a.Kp) {
                const T* col = opsT + (size_t)p * a.Kp * a.Kp + r;
                for (int k = 0; k < a.Kp; ++k) {
                    const T m = col[(size_t)k * a.Kp];
#pragma unroll
                    for (int b = 0; b < RB; ++b) acc[b] += m * ws[b * a.Kp + k];
                }
            }
        }
        if (r < a.Kp) {
#pragma unroll
            for (int b = 0; b < RB; ++b)
                if (b < nb) Lo[((long)(b0 + b) * a.nbox + t) * a.Kp + r] += acc[b];
        }
    }
}

constexpr int kTM = 2, kTN = 2;

}  // namespace

ert_status m2l_launch(hipStream_t s, int prec, bool hetero, const M2LArgs& a)
{
    if (hetero) {
        const int rb = a.B >= 8 ? 8 : (a.B >= 4 ? 4 : 1);
        dim3 grid((unsigned)a.nbox, (unsigned)((a.B + rb - 1) / rb));
        if (prec == ERT_FP64) {
            size_t sh = (size_t)rb * a.Kp * sizeof(double);
            if (rb == 8) hipLaunchKernelGGL((k_m2l_het<double, 8>), grid, dim3(256), sh, s, a, (const double*)a.ops);
            else if (rb == 4) hipLaunchKernelGGL((k_m2l_het<double, 4>), grid, dim3(256), sh, s, a, (const double*)a.ops);
            else hipLaunchKernelGGL((k_m2l_het<double, 1>), grid, dim3(256), sh, s, a, (const double*)a.ops);
        } else {
            size_t sh = (size_t)rb * a.Kp * sizeof(float);
            if (rb == 8) hipLaunchKernelGGL((k_m2l_het<float, 8>), grid, dim3(256), sh, s, a, (const float*)a.ops);
            else if (rb == 4) hipLaunchKernelGGL((k_m2l_het<float, 4>), grid, dim3(256), sh, s, a, (const float*)a.ops);
            else hipLaunchKernelGGL((k_m2l_het<float, 1>), grid, dim3(256), sh, s, a, (const float*)a.ops);
        }
        ERT_HIP(hipGetLastError());
        return ERT_OK;
    }
    const int classes = 1 << a.D;
    const int row_tiles = a.Kp / (16 * kTM);
    long max_nt = 0;
    for (int c = 0; c < classes; ++c) {
        long nt = 1;
        for (int d = 0; d < a.D; ++d) {
            int pc = (c >> d) & 1;
            int n = (a.nl[d] - pc + 1) / 2;
            nt *= n > 0 ? n : 0;
        }
        max_nt = nt > max_nt ? nt : max_nt;
    }
    const long col_tiles = (max_nt * a.B + 16 * kTN - 1) / (16 * kTN);
    if (col_tiles == 0) return ERT_OK;
    dim3 grid((unsigned)(row_tiles * col_tiles), (unsigned)classes);
    if (prec == ERT_FP64)
        hipLaunchKernelGGL((k_m2l_f64<kTM, kTN>), grid, dim3(64 * kWaves), 0, s, a, row_tiles);
    else if (prec == ERT_FP32)
        hipLaunchKernelGGL((k_m2l_f32<kTM, kTN>), grid, dim3(64 * kWaves), 0, s, a, row_tiles);
    else
        hipLaunchKernelGGL((k_m2l_bf16x3<kTM, kTN>), grid, dim3(64 * kWaves), 0, s, a, row_tiles);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

}  // namespace ertvie
