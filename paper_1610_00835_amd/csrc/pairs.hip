// Cached-pair products of a heterogeneous medium: the far-field translations
// (Sec. 3.3 eq. EQ: M2L with one matrix per (target, source) box pair) and the
// near field over neighbouring leaves, both from kernel values cached at plan
// time (Sec. 4.2 caches every kernel evaluation).
//
// The kernel is symmetric, G(x, y) = G(y, x) (the ray rule samples the same
// points from either end of the segment), so one block is stored per unordered
// pair of boxes {a, b}: B[j][i] = G(x_i in a, y_j in b), i fastest.  It serves
// both directed pairs: the forward product for target a,
//     fwd[i] = sum_j B[j][i] w_b[j],
// and the backward product for target b,
//     bwd[j] = sum_i B[j][i] w_a[i]
// (none for a self block, a = b, which is symmetric itself).  Every product
// goes to the staging row of its directed pair; a second pass sums the rows of
// every target in a fixed order, so results are bitwise reproducible.
//
// Forms.  Up to 8 right-hand sides (passes of at most 4): one workgroup per
// block streams it once from HBM into registers and forms both products
// (HBM-bound: each stored value is read once per pass).  From
// kPairMfmaMinRhs right-hand sides on, and for the split-BF16x3 products always,
// the matrix cores take 64 right-hand sides per pass, the forward and the
// backward products as two launches over the blocks (the backward one reads the
// blocks row-wise through LDS).
#include <algorithm>
#include <type_traits>

#include "fmm.hpp"

namespace ertvie {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Tags of the 16-bit plane storage (kOpsSplit, kOpsHi).
struct OpsSplit {};
struct OpsHi {};

// VEC consecutive stored values from element idx, as FP32.  Planes: the FP32 bit
// pattern is (hi << 16) + lo, lo the signed remainder (zero for kOpsHi).
template <typename TS, int VEC>
__device__ __forceinline__ void load_vals(const PairStream& g, size_t idx, float (&o)[VEC])
{
    if constexpr (std::is_same<TS, float>::value) {
        const float* p = (const float*)g.opsT + idx;
        if constexpr (VEC == 4) {
            const v4f v = *(const v4f*)p;
            o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) o[e] = p[e];
        }
    } else {
        const unsigned short* hp = (const unsigned short*)g.opsT + idx;
        const short* lp = (const short*)g.opsT_lo + idx;
        if constexpr (VEC == 4) {
            const uint2 h = *(const uint2*)hp;
            const unsigned hv[4] = {h.x & 0xffffu, h.x >> 16, h.y & 0xffffu, h.y >> 16};
            int lv[4] = {0, 0, 0, 0};
            if constexpr (std::is_same<TS, OpsSplit>::value) {
                const uint2 l = *(const uint2*)lp;
                lv[0] = (short)(l.x & 0xffffu);
                lv[1] = (short)(l.x >> 16);
                lv[2] = (short)(l.y & 0xffffu);
                lv[3] = (short)(l.y >> 16);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = __uint_as_float((hv[e] << 16) + (unsigned)lv[e]);
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const int lo = std::is_same<TS, OpsSplit>::value ? (int)lp[e] : 0;
                o[e] = __uint_as_float(((unsigned)hp[e] << 16) + (unsigned)lo);
            }
        }
    }
}

// Streaming form, RB right-hand sides per pass.  Workgroup = one stored block.
// The block is read in strips of SW = CG CPL columns (one 128-byte piece of a row
// per plane); in a strip, lane (rg, cg) holds the CPL columns i = CPL cg + e of rows
// rg R + r of every chunk of CH = RG R rows, straight from HBM into registers (the
// next chunk in flight while one is used).  Forward: each lane sums its columns over
// its rows in registers; at the strip end the row groups of a wave are combined by a
// butterfly and the four waves in LDS, in a fixed order.  Backward: each row's
// partial over the lane's columns is combined over the CG lanes of the row by a
// butterfly (IEEE addition commutes, so every lane holds the same bits) and added by
// the row's owner lane (cg = 0, the same lane in every strip) to its LDS
// accumulator, strips in order.  R <= RMAX rows per lane.
template <typename T, typename TS, int RB, int VEC>
__global__ __launch_bounds__(256) void k_pair_sym(PairStream g, int b0, int R)
{
    constexpr int CPL = std::is_same<TS, float>::value ? 4 : 8;   // columns per lane: 16 bytes per plane
    constexpr int CG = 8;                               // lanes per row
    constexpr int RG = 256 / CG;                        // row groups (8 per wave)
    constexpr int SW = CPL * CG;                        // strip width (columns)
    constexpr int RMAX = CPL == 4 ? 8 : 4;
    extern __shared__ __align__(16) unsigned char smem[];
    const int M = g.M;
    T* wb = (T*)smem;                                   // [RB][M] forward sources (box b)
    T* wa = wb + RB * M;                                // [RB][M] backward sources (box a)
    T* bacc = wa + RB * M;                              // [RB][M] backward sums
    T* red = bacc + RB * M;                             // [2][4 waves][RB][SW] forward partials of a strip
    const long u = blockIdx.x;
    const int a = g.ua[u], bs = g.ub[u];
    const long frow = g.fwd_row[u], brow = g.bwd_row[u];
    const bool back = brow >= 0;                        // uniform over the workgroup
    const int nb = (g.B - b0) < RB ? (g.B - b0) : RB;
    const int tid = threadIdx.x, cg = tid % CG, rg = tid / CG, wave = tid >> 6;
    const T* W = (const T*)g.W;
    for (int i = tid; i < RB * M; i += 256) {
        const int b = i / M, k = i - b * M;
        wb[i] = b < nb ? W[((long)(b0 + b) * g.nsrc + bs) * M + k] : T(0);
        wa[i] = (back && b < nb) ? W[((long)(b0 + b) * g.nsrc + a) * M + k] : T(0);
        bacc[i] = T(0);
    }
    const int CH = RG * R;                              // rows per chunk
    const int nchunk = (M + CH - 1) / CH;
    const int nstrip = (M + SW - 1) / SW;
    const size_t base = (size_t)u * M * M;
    // one chunk of the lane: rows c CH + rg R + r, columns s SW + CPL cg + e
    auto load_chunk = [&](int s, int c, float (&v)[RMAX][CPL]) {
        const int i0 = s * SW + CPL * cg;
        const int j0 = c * CH + rg * R;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const int j = j0 + r;
            if (r < R && j < M && i0 < M) {
                if constexpr (VEC == 4) {
#pragma unroll
                    for (int h = 0; h < CPL / 4; ++h) {
                        float o[4];
                        load_vals<TS, 4>(g, base + (size_t)j * M + i0 + 4 * h, o);
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[r][4 * h + e] = o[e];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < CPL; ++e) {
                        float o[1] = {0.f};
                        if (i0 + e < M) load_vals<TS, 1>(g, base + (size_t)j * M + i0 + e, o);
                        v[r][e] = o[0];
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < CPL; ++e) v[r][e] = 0.f;
            }
        }
    };
    float cur[RMAX][CPL], nxt[RMAX][CPL];
    T accf[RB][CPL], war[RB][CPL];
    T* stage = (T*)g.stage;
    load_chunk(0, 0, cur);
    __syncthreads();                                    // wb and bacc staged
    for (int s = 0; s < nstrip; ++s) {
        const int i0 = s * SW + CPL * cg;
#pragma unroll
        for (int b = 0; b < RB; ++b)
#pragma unroll
            for (int e = 0; e < CPL; ++e) {
                accf[b][e] = T(0);
                war[b][e] = i0 + e < M ? wa[b * M + i0 + e] : T(0);
            }
        for (int c = 0; c < nchunk; ++c) {
            // the next chunk (of this strip, or the first of the next) in flight
            const int cn = c + 1 < nchunk ? c + 1 : 0;
            const int sn = c + 1 < nchunk ? s : s + 1;
            if (sn < nstrip) load_chunk(sn, cn, nxt);
            const int j0 = c * CH + rg * R;
#pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                if (r >= R) break;                      // uniform
                const int j = j0 + r;
                T x[CPL];
#pragma unroll
                for (int e = 0; e < CPL; ++e) x[e] = (T)cur[r][e];
                // forward: the lane's columns
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    const T w = j < M ? wb[b * M + j] : T(0);
#pragma unroll
                    for (int e = 0; e < CPL; ++e) accf[b][e] += x[e] * w;
                }
                // backward: row j over the strip's columns
                if (back) {
                    T pb[RB];
#pragma unroll
                    for (int b = 0; b < RB; ++b) {
                        T t = T(0);
#pragma unroll
                        for (int e = 0; e < CPL; ++e) t += x[e] * war[b][e];
                        pb[b] = t;
                    }
#pragma unroll
                    for (int off = CG / 2; off >= 1; off >>= 1)
#pragma unroll
                        for (int b = 0; b < RB; ++b) pb[b] += __shfl_xor(pb[b], off, CG);
                    if (cg == 0 && j < M) {
#pragma unroll
                        for (int b = 0; b < RB; ++b) bacc[b * M + j] += pb[b];
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < RMAX; ++r)
#pragma unroll
                for (int e = 0; e < CPL; ++e) cur[r][e] = nxt[r][e];
        }
        // forward sums of the strip: the 8 row groups of a wave by a butterfly over
        // the lanes of one column group, then the four waves in order (two LDS buffers
        // by strip parity, so one barrier per strip separates writes from reads)
#pragma unroll
        for (int b = 0; b < RB; ++b)
#pragma unroll
            for (int e = 0; e < CPL; ++e) {
                T v = accf[b][e];
#pragma unroll
                for (int off = 32; off >= CG; off >>= 1) v += __shfl_xor(v, off, 64);
                accf[b][e] = v;
            }
        T* rs = red + (size_t)(s & 1) * 4 * RB * SW;
        if ((tid & 63) < CG) {
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int e = 0; e < CPL; ++e) rs[(wave * RB + b) * SW + CPL * cg + e] = accf[b][e];
        }
        __syncthreads();
        for (int idx = tid; idx < RB * SW; idx += 256) {
            const int b = idx / SW, col = idx - b * SW, i = s * SW + col;
            const T sum = ((rs[(0 * RB + b) * SW + col] + rs[(1 * RB + b) * SW + col]) + rs[(2 * RB + b) * SW + col]) +
                          rs[(3 * RB + b) * SW + col];
            if (b < nb && i < M) stage[((long)b * g.nrows + frow) * M + i] = sum;
        }
    }
    if (back) {
        __syncthreads();                                // every row's owner lane is done
        for (int idx = tid; idx < RB * M; idx += 256) {
            const int b = idx / M, j = idx - b * M;
            if (b < nb) stage[((long)b * g.nrows + brow) * M + j] = bacc[idx];
        }
    }
}

template <int PREC>
struct Acc;
template <>
struct Acc<ERT_FP64> { typedef v4d V; typedef double T; };
template <>
struct Acc<ERT_FP32> { typedef v4f V; typedef float T; };

// One stored value as FP32 (element idx).
template <typename TS>
__device__ __forceinline__ float load_one(const PairStream& g, size_t idx)
{
    float o[1];
    load_vals<TS, 1>(g, idx, o);
    return o[0];
}

// Matrix-core form, 64 right-hand sides per pass: per block, the (M x M) x (M x 64)
// product of the forward direction (A[r][k] = B[k][r], sources of box b, row
// fwd_row), FP32 or FP64 accumulation over the FP32 values.  Workgroup: one block
// and 64 RT output rows per wave-row block; the 64 source vectors pass through LDS,
// 32 reduction indices at a time, transposed so that lanes read consecutive columns;
// lanes read the block along its rows (consecutive r), coalesced.
template <int PREC, int RT, typename TS>
__global__ __launch_bounds__(256) void k_pair_mfma(PairStream g, int b0, int rblocks)
{
    typedef typename Acc<PREC>::V V;
    typedef typename Acc<PREC>::T T;
    constexpr int KC = 32;
    constexpr int LDW = 80;                       // padded LDS row (columns)
    __shared__ T wsh[KC * LDW];
    const long p = blockIdx.x / rblocks;
    const long row = g.fwd_row[p];
    const int rblk = (int)(blockIdx.x % rblocks);
    const int nb = (g.B - b0) < 64 ? (g.B - b0) : 64;
    const int s = g.ub[p];
    const int M = g.M;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane >> 4, li = lane & 15;
    const int row0 = (rblk * 4 + wave) * 16 * RT;
    const size_t A = (size_t)p * M * M;
    V acc[RT][4];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = V{0, 0, 0, 0};
    for (int k0 = 0; k0 < M; k0 += KC) {
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * KC; i += 256) {
            const int b = i / KC, kk = i - b * KC;
            T v = T(0);
            if (b < nb && k0 + kk < M) v = ((const T*)g.W)[((long)(b0 + b) * g.nsrc + s) * M + k0 + kk];
            wsh[kk * LDW + b] = v;
        }
        __syncthreads();
#pragma unroll 2
        for (int kk = 0; kk < KC; kk += 4) {
            const int k = k0 + kk + grp;
            T av[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const int r = row0 + 16 * rt + li;
                av[rt] = (k < M && r < M) ? (T)load_one<TS>(g, A + (size_t)k * M + r) : T(0);
            }
            T bf[4];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) bf[ct] = wsh[(kk + grp) * LDW + 16 * ct + li];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    if constexpr (PREC == ERT_FP64)
                        acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rt], bf[ct], acc[rt][ct], 0, 0, 0);
                    else
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rt], bf[ct], acc[rt][ct], 0, 0, 0);
                }
        }
    }
    // FP32 tiles: rows 4 grp + i; FP64 tiles: rows grp + 4 i (column li in both)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int b = 16 * ct + li;
        if (b >= nb) continue;
        T* dst = (T*)g.stage + ((long)b * g.nrows + row) * M;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int base = row0 + 16 * rt;
            if constexpr (PREC == ERT_FP64) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (base + grp + 4 * i < M) dst[base + grp + 4 * i] = acc[rt][ct][i];
            } else {
                if (base + 4 * grp + 3 < M) *(V*)(dst + base + 4 * grp) = acc[rt][ct];
            }
        }
    }
}

// The backward direction of the matrix-core form: out[j][b] = sum_i B[j][i] W_a[i][b],
// whose A operand runs along the stored rows (A[r][k] = B[r][k]).  A tile of the
// workgroup's 64 RT rows and 32 reduction indices is read row-wise (eight lanes per
// 128-byte row piece) into LDS, and the lanes take their operands from there.
template <int PREC, int RT, typename TS>
__global__ __launch_bounds__(256) void k_pair_mfma_back(PairStream g, int b0, int rblocks)
{
    typedef typename Acc<PREC>::V V;
    typedef typename Acc<PREC>::T T;
    constexpr int KC = 32;
    constexpr int LDW = 80;                       // padded LDS row of the sources (columns)
    constexpr int ROWS = 64 * RT;                 // rows of the workgroup
    constexpr int TP = KC + 4;                    // tile pitch (floats)
    __shared__ T wsh[KC * LDW];
    __shared__ __align__(16) float tile[ROWS * TP];
    const long p = blockIdx.x / rblocks;
    const long row = g.bwd_row[p];
    if (row < 0) return;                          // self block: no backward product (uniform)
    const int rblk = (int)(blockIdx.x % rblocks);
    const int nb = (g.B - b0) < 64 ? (g.B - b0) : 64;
    const int s = g.ua[p];
    const int M = g.M;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane >> 4, li = lane & 15;
    const int rw0 = rblk * ROWS;                  // first row of the workgroup
    const int row0 = wave * 16 * RT;              // first row of the wave (in the tile)
    const size_t A = (size_t)p * M * M;
    V acc[RT][4];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = V{0, 0, 0, 0};
    for (int k0 = 0; k0 < M; k0 += KC) {
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * KC; i += 256) {
            const int b = i / KC, kk = i - b * KC;
            T v = T(0);
            if (b < nb && k0 + kk < M) v = ((const T*)g.W)[((long)(b0 + b) * g.nsrc + s) * M + k0 + kk];
            wsh[kk * LDW + b] = v;
        }
        // the tile: ROWS rows x KC columns, 16-byte pieces (M is a multiple of 4)
        for (int c = threadIdx.x; c < ROWS * (KC / 4); c += 256) {
            const int rr = c / (KC / 4), c4 = (c - rr * (KC / 4)) * 4;
            const int r = rw0 + rr, k = k0 + c4;
            float o[4] = {0.f, 0.f, 0.f, 0.f};
            if (r < M && k < M) load_vals<TS, 4>(g, A + (size_t)r * M + k, o);
            *(v4f*)(tile + rr * TP + c4) = v4f{o[0], o[1], o[2], o[3]};
        }
        __syncthreads();
#pragma unroll 2
        for (int kk = 0; kk < KC; kk += 4) {
            T av[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) av[rt] = (T)tile[(row0 + 16 * rt + li) * TP + kk + grp];
            T bf[4];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) bf[ct] = wsh[(kk + grp) * LDW + 16 * ct + li];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    if constexpr (PREC == ERT_FP64)
                        acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rt], bf[ct], acc[rt][ct], 0, 0, 0);
                    else
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rt], bf[ct], acc[rt][ct], 0, 0, 0);
                }
        }
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int b = 16 * ct + li;
        if (b >= nb) continue;
        T* dst = (T*)g.stage + ((long)b * g.nrows + row) * M;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int base = rw0 + row0 + 16 * rt;
            if constexpr (PREC == ERT_FP64) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (base + grp + 4 * i < M) dst[base + grp + 4 * i] = acc[rt][ct][i];
            } else {
                if (base + 4 * grp + 3 < M) *(V*)(dst + base + 4 * grp) = acc[rt][ct];
            }
        }
    }
}

// Split-BF16x3 form of the same products (FP32-stored blocks, FP32 vectors): every
// block value a and source value w is split into BF16 parts (hi = bf16(v), lo =
// bf16(v - hi)) and a w is taken as hi_a hi_w + hi_a lo_w + lo_a hi_w, three
// 16x16x32 BF16 products accumulated in FP32 (the dropped lo_a lo_w is below
// 2^-16 |a w|).  The 64 source vectors of a 32-long reduction chunk are split
// once into LDS, source-major, so that a lane reads its eight reduction indices as
// one 16-byte vector; each lane loads its eight block values along the reduction
// (the backward direction reads them contiguously) and splits them in registers.
template <int RT, bool TRANS>
__global__ __launch_bounds__(256) void k_pair_mfma_bf16x3(PairStream g, int b0, int rblocks)
{
    constexpr int KC = 32;
    constexpr int LDK = KC + 8;                   // padded LDS row (reduction indices)
    __shared__ __bf16 whi[64 * LDK];
    __shared__ __bf16 wlo[64 * LDK];
    const long p = blockIdx.x / rblocks;
    const long row = TRANS ? g.bwd_row[p] : g.fwd_row[p];
    if (row < 0) return;                          // self block: no backward product (uniform)
    const int rblk = (int)(blockIdx.x % rblocks);
    const int nb = (g.B - b0) < 64 ? (g.B - b0) : 64;
    const int s = TRANS ? g.ua[p] : g.ub[p];
    const int M = g.M;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane >> 4, li = lane & 15;
    const int row0 = (rblk * 4 + wave) * 16 * RT;
    const size_t A = (size_t)p * M * M;
    const float* ops = (const float*)g.opsT;
    v4f acc[RT][4];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0, 0, 0, 0};
    for (int k0 = 0; k0 < M; k0 += KC) {
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * KC; i += 256) {
            const int b = i / KC, kk = i - b * KC;
            float v = 0.f;
            if (b < nb && k0 + kk < M) v = ((const float*)g.W)[((long)(b0 + b) * g.nsrc + s) * M + k0 + kk];
            const __bf16 h = (__bf16)v;
            whi[b * LDK + kk] = h;
            wlo[b * LDK + kk] = (__bf16)(v - (float)h);
        }
        __syncthreads();
        v8bf ah[RT], al[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int r = row0 + 16 * rt + li;
            const int kb = k0 + 8 * grp;
            float av[8];
            if (TRANS && r < M && kb + 8 <= M) {
                const v4f x0 = *(const v4f*)(ops + A + (size_t)r * M + kb);
                const v4f x1 = *(const v4f*)(ops + A + (size_t)r * M + kb + 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    av[e] = x0[e];
                    av[4 + e] = x1[e];
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = kb + e;
                    av[e] = (k < M && r < M) ? ops[TRANS ? A + (size_t)r * M + k : A + (size_t)k * M + r] : 0.f;
                }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const __bf16 h = (__bf16)av[e];
                ah[rt][e] = h;
                al[rt][e] = (__bf16)(av[e] - (float)h);
            }
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int b = 16 * ct + li;
            const v8bf bh = *(const v8bf*)(whi + b * LDK + 8 * grp);
            const v8bf bl = *(const v8bf*)(wlo + b * LDK + 8 * grp);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rt], bh, acc[rt][ct], 0, 0, 0);
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rt], bl, acc[rt][ct], 0, 0, 0);
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[rt], bh, acc[rt][ct], 0, 0, 0);
            }
        }
    }
    // rows 4 grp + i of column li
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int b = 16 * ct + li;
        if (b >= nb) continue;
        float* dst = (float*)g.stage + ((long)b * g.nrows + row) * M;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int base = row0 + 16 * rt;
            if (base + 4 * grp + 3 < M) *(v4f*)(dst + base + 4 * grp) = acc[rt][ct];
        }
    }
}

// Per-target sums of the staging rows (rhs b0..b0+nb-1), over the target's
// contiguous directed rows in order, skipping rows of pairs that do not exist.
template <typename T>
__global__ void k_pair_reduce(PairStream g, int b0, int nb)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long per = g.ntarget * g.M;
    if (i >= per * nb) return;
    const int b = (int)(i / per);
    const long rem = i - (long)b * per;
    const long t = rem / g.M;
    const int r = (int)(rem - t * g.M);
    const T* St = (const T*)g.stage + (long)b * g.nrows * g.M + r;
    const long k1 = g.tstart[t + 1];
    T sum = T(0);
    for (long k = g.tstart[t]; k < k1; ++k)
        if (!g.row_src || g.row_src[k] >= 0) sum += St[k * g.M];
    T* d = (T*)g.L + (long)(b0 + b) * per + rem;
    *d = g.accumulate ? *d + sum : sum;
}

template <typename T>
ert_status launch_reduce(hipStream_t s, const PairStream& g, int b0, int nb)
{
    StageTimer t_(g.prof, s, ERT_STAGE_REDUCE);
    const long n = g.ntarget * g.M * nb;
    hipLaunchKernelGGL(k_pair_reduce<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, b0, nb);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

// LDS of the streaming form: forward and backward sources, backward sums, two strips
// of the four waves' forward partials (strip width 64 columns at most).
size_t sym_lds(int M, int rb, size_t tsize)
{
    return tsize * (3 * (size_t)rb * M + 2 * 4 * (size_t)rb * 64);
}

template <typename T, typename TS, int VEC>
void launch_sym(hipStream_t s, const PairStream& g, int b0, int rb, int R, size_t sh)
{
    const dim3 grid((unsigned)g.npairs);
    if (rb == 4) hipLaunchKernelGGL((k_pair_sym<T, TS, 4, VEC>), grid, dim3(256), sh, s, g, b0, R);
    else if (rb == 2) hipLaunchKernelGGL((k_pair_sym<T, TS, 2, VEC>), grid, dim3(256), sh, s, g, b0, R);
    else hipLaunchKernelGGL((k_pair_sym<T, TS, 1, VEC>), grid, dim3(256), sh, s, g, b0, R);
}

constexpr size_t kSymLdsMax = 64 * 1024;

// Streaming form: passes of 4, 2 or 1 right-hand sides (as many as the LDS allows).
template <typename T, typename TS>
ert_status pair_sym_t(hipStream_t s, const PairStream& g)
{
    const int M = g.M;
    if (M < 1 || M > 4096 || sym_lds(M, 1, sizeof(T)) > kSymLdsMax) {
        record_error("pair_stream: unsupported block size");
        return ERT_EINVAL;
    }
    // rows per lane: the fewest chunks of 32 R rows (R <= 8 for FP32 storage, 4 for
    // planes) that cover M, then the smallest R
    const int rmax = std::is_same<TS, float>::value ? 8 : 4;
    const int nchunk = (M + 32 * rmax - 1) / (32 * rmax);
    const int R = std::max(1, std::min(rmax, (M + 32 * nchunk - 1) / (32 * nchunk)));
    for (int b0 = 0; b0 < g.B;) {
        const int left = g.B - b0;
        int rb = left >= 4 ? 4 : (left >= 2 ? 2 : 1);
        while (rb > 1 && sym_lds(M, rb, sizeof(T)) > kSymLdsMax) rb /= 2;
        const size_t sh = sym_lds(M, rb, sizeof(T));
        {
            StageTimer t_(g.prof, s, g.prof_stage);
            if (M % 4 == 0) launch_sym<T, TS, 4>(s, g, b0, rb, R, sh);
            else launch_sym<T, TS, 1>(s, g, b0, rb, R, sh);
            ERT_HIP(hipGetLastError());
        }
        ERT_TRY(launch_reduce<T>(s, g, b0, rb));
        b0 += rb;
    }
    return ERT_OK;
}

// Matrix-core form (FP32 storage, whole or in planes), 64 right-hand sides per pass.
template <int PREC, typename TS>
ert_status pair_mfma_t(hipStream_t s, const PairStream& g)
{
    constexpr int RT = (PREC == ERT_FP64) ? 4 : 8;
    constexpr int RTB = 4;                        // backward: 256 rows per workgroup (LDS tile)
    typedef typename Acc<PREC>::T T;
    const int rblocks = (g.M + 64 * RT - 1) / (64 * RT);
    const int rblocksb = (g.M + 64 * RTB - 1) / (64 * RTB);
    const dim3 grid((unsigned)(g.npairs * rblocks)), gridb((unsigned)(g.npairs * rblocksb));
    for (int b0 = 0; b0 < g.B; b0 += 64) {
        const int nb = std::min(64, g.B - b0);
        {
            StageTimer t_(g.prof, s, g.prof_stage);
            hipLaunchKernelGGL((k_pair_mfma<PREC, RT, TS>), grid, dim3(256), 0, s, g, b0, rblocks);
            ERT_HIP(hipGetLastError());
            hipLaunchKernelGGL((k_pair_mfma_back<PREC, RTB, TS>), gridb, dim3(256), 0, s, g, b0, rblocksb);
            ERT_HIP(hipGetLastError());
        }
        ERT_TRY(launch_reduce<T>(s, g, b0, nb));
    }
    return ERT_OK;
}

// Split-BF16x3 matrix-core form (FP32-stored blocks, FP32 vectors), 64 right-hand
// sides per pass, for any right-hand-side count (it stays HBM-bound with one).
ert_status pair_mfma_bf16x3(hipStream_t s, const PairStream& g)
{
    constexpr int RT = 4;
    if (g.ops_fmt != kOpsF32) {
        record_error("pair_stream: split-BF16x3 products need FP32-stored blocks");
        return ERT_EINVAL;
    }
    const int rblocks = (g.M + 64 * RT - 1) / (64 * RT);
    const dim3 grid((unsigned)(g.npairs * rblocks));
    for (int b0 = 0; b0 < g.B; b0 += 64) {
        const int nb = std::min(64, g.B - b0);
        {
            StageTimer t_(g.prof, s, g.prof_stage);
            hipLaunchKernelGGL((k_pair_mfma_bf16x3<RT, false>), grid, dim3(256), 0, s, g, b0, rblocks);
            ERT_HIP(hipGetLastError());
            hipLaunchKernelGGL((k_pair_mfma_bf16x3<RT, true>), grid, dim3(256), 0, s, g, b0, rblocks);
            ERT_HIP(hipGetLastError());
        }
        ERT_TRY(launch_reduce<float>(s, g, b0, nb));
    }
    return ERT_OK;
}

}  // namespace

ert_status pair_stream(hipStream_t s, int prec, const PairStream& g)
{
    if (g.npairs < 1 || g.B < 1) return ERT_OK;
    if (g.ops_fmt != kOpsF32 && g.ops_fmt != kOpsSplit && g.ops_fmt != kOpsHi) {
        record_error("pair_stream: unknown block storage");
        return ERT_EINVAL;
    }
    const bool f64 = prec == ERT_FP64;
    if (f64 && g.ops_fmt == kOpsHi) {
        record_error("pair_stream: FP64 products do not read the rounded plane alone");
        return ERT_EINVAL;
    }
    if (prec == ERT_BF16X3) {
        if (g.M % 4 != 0) {
            record_error("pair_stream: split-BF16x3 products need blocks of a multiple of 4 rows");
            return ERT_EINVAL;
        }
        return pair_mfma_bf16x3(s, g);
    }
    if (g.B >= kPairMfmaMinRhs && g.M % 4 == 0) {
        switch (g.ops_fmt) {
        case kOpsSplit: return f64 ? pair_mfma_t<ERT_FP64, OpsSplit>(s, g) : pair_mfma_t<ERT_FP32, OpsSplit>(s, g);
        case kOpsHi: return pair_mfma_t<ERT_FP32, OpsHi>(s, g);
        default: return f64 ? pair_mfma_t<ERT_FP64, float>(s, g) : pair_mfma_t<ERT_FP32, float>(s, g);
        }
    }
    switch (g.ops_fmt) {
    case kOpsSplit: return f64 ? pair_sym_t<double, OpsSplit>(s, g) : pair_sym_t<float, OpsSplit>(s, g);
    case kOpsHi: return pair_sym_t<float, OpsHi>(s, g);
    default: return f64 ? pair_sym_t<double, float>(s, g) : pair_sym_t<float, float>(s, g);
    }
}

}  // namespace ertvie
