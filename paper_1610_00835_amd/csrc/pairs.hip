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

// Lane permutations of the DPP butterflies (within rows of 16 lanes).
constexpr int kDppXor1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 8 lanes 8k..8k+7: quad partners, then the other quad of the
// 8-lane group (its mirror image).  IEEE addition commutes, so all 8 lanes end
// with the same bits.
template <typename T>
__device__ __forceinline__ T sum8_lanes(T v)
{
    v += dpp_move<kDppXor1>(v);
    v += dpp_move<kDppXor2>(v);
    v += dpp_move<kDppHalfMirror>(v);
    return v;
}

// Sum over the lanes of a wave that agree in lane % 8 (the 8 row groups of a
// column group): the other half of the 16-lane row, then lanes 16 and 32 away.
template <typename T>
__device__ __forceinline__ T sum_rowgroups(T v)
{
    v += dpp_move<kDppRor8>(v);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

constexpr unsigned kBufOob = 0x80000000u;   // buffer offset past every block: the load returns 0
constexpr int kBufFlags = 0x00020000;       // raw buffer, 32-bit data format

// Streaming form, RB right-hand sides per pass.  Workgroup = one stored block.
// The block is read in strips of SW = CG CPL columns (16 bytes of a row per plane
// and lane); in a strip, lane (rg, cg) holds the CPL columns i = CPL cg + e of rows
// rg R + r of every chunk of CH = RG R rows.  The loads go through a buffer
// resource spanning the block, unconditionally: rows and columns outside the block
// (and steps past the last) take an offset beyond it and read as zero.  Two
// register buffers alternate, so the next chunk is in flight while one is used and
// the wait before each use leaves the newer loads outstanding.  Forward: each lane
// sums its columns over its rows in registers; at the strip end the row groups of
// a wave are combined by a butterfly and the four waves in LDS, in a fixed order,
// into the LDS row of forward sums.  Backward: each row's partial over the lane's
// columns is combined over the CG lanes of the row by a butterfly and added by the
// row's owner lane (cg = 0) to its LDS accumulator, strips in order; with one
// chunk and one right-hand side (NC1) a lane meets the same rows in every strip, so
// their partials stay in registers and the butterfly runs once per row at the end.
// Both LDS rows go to the staging rows once the block is done.  The LDS rows are MP
// long (MP >= rows and columns the chunks and strips cover), zero past M.
template <typename T, typename TS, int RB, int VEC, bool NC1>
__global__ __launch_bounds__(256) void k_pair_sym(PairStream g, int b0, int R, int MP)
{
    static_assert(!NC1 || RB == 1, "register backward partials hold one right-hand side");
    constexpr bool F32 = std::is_same<TS, float>::value;
    constexpr bool SPLIT = std::is_same<TS, OpsSplit>::value;
    constexpr int CPL = F32 ? 4 : 8;                    // columns per lane: 16 bytes per plane
    constexpr int CG = 8;                               // lanes per row
    constexpr int RG = 256 / CG;                        // row groups (8 per wave)
    constexpr int SW = CPL * CG;                        // strip width (columns)
    constexpr int RMAX = CPL == 4 ? 8 : 4;
    // registers per row and lane: VEC 4, the raw 16-byte pieces (4 words per plane);
    // VEC 1, one FP32 value per column
    constexpr int NWD = VEC == 4 ? (SPLIT ? 8 : 4) : CPL;
    constexpr int ESZ = F32 ? 4 : 2;                    // bytes per stored value and plane
    extern __shared__ __align__(16) unsigned char smem[];
    const int M = g.M;
    T* wb = (T*)smem;                                   // [RB][MP] forward sources (box b)
    T* wa = wb + RB * MP;                               // [RB][MP] backward sources (box a)
    T* bacc = wa + RB * MP;                             // [RB][MP] backward sums
    T* facc = bacc + RB * MP;                           // [RB][MP] forward sums
    T* red = facc + RB * MP;                            // [2][4 waves][RB][SW] forward partials of a strip
    const long u = blockIdx.x;
    const int a = g.ua[u], bs = g.ub[u];
    const long frow = g.fwd_row[u], brow = g.bwd_row[u];
    const bool back = brow >= 0;                        // uniform over the workgroup
    const int nb = (g.B - b0) < RB ? (g.B - b0) : RB;
    const int tid = threadIdx.x, cg = tid % CG, rg = tid / CG, wave = tid >> 6;
    const int CH = RG * R;                              // rows per chunk
    const int nchunk = (M + CH - 1) / CH;
    const int nstrip = (M + SW - 1) / SW;
    const int nstep = nchunk * nstrip;
    const size_t base = (size_t)u * M * M;
    const unsigned nbytes = (unsigned)((size_t)M * M * ESZ);
    const __amdgpu_buffer_rsrc_t rs0 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)((const unsigned char*)g.opsT + base * ESZ), 0, (int)nbytes, kBufFlags);
    const __amdgpu_buffer_rsrc_t rs1 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)((const unsigned char*)(SPLIT ? g.opsT_lo : g.opsT) + base * ESZ), 0, (int)nbytes, kBufFlags);

    // step t = (strip t / nchunk, chunk t % nchunk) of the lane: rows c CH + rg R + r,
    // columns s SW + CPL cg + e
    auto load_step = [&](int t, unsigned (&v)[RMAX][NWD]) {
        const int s = t / nchunk, c = t - s * nchunk;
        const int i0 = s * SW + CPL * cg;
        const int j0 = c * CH + rg * R;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const int j = j0 + r;
            const bool ok = t < nstep && r < R && j < M;
            if constexpr (VEC == 4) {
                const unsigned off = ok && i0 < M ? (unsigned)(((size_t)j * M + i0) * ESZ) : kBufOob;
                typedef unsigned v4u __attribute__((ext_vector_type(4)));
                const v4u h = __builtin_amdgcn_raw_buffer_load_b128(rs0, off, 0, 0);
                v[r][0] = h[0]; v[r][1] = h[1]; v[r][2] = h[2]; v[r][3] = h[3];
                if constexpr (SPLIT) {
                    const v4u l = __builtin_amdgcn_raw_buffer_load_b128(rs1, off, 0, 0);
                    v[r][4] = l[0]; v[r][5] = l[1]; v[r][6] = l[2]; v[r][7] = l[3];
                }
            } else {
#pragma unroll
                for (int e = 0; e < CPL; ++e) {
                    const unsigned off = ok && i0 + e < M ? (unsigned)(((size_t)j * M + i0 + e) * ESZ) : kBufOob;
                    if constexpr (F32) {
                        v[r][e] = __builtin_amdgcn_raw_buffer_load_b32(rs0, off, 0, 0);
                    } else {
                        const unsigned hi = __builtin_amdgcn_raw_buffer_load_b16(rs0, off, 0, 0);
                        const int lo = SPLIT ? (int)(short)__builtin_amdgcn_raw_buffer_load_b16(rs1, off, 0, 0) : 0;
                        v[r][e] = (hi << 16) + (unsigned)lo;
                    }
                }
            }
        }
    };
    // row r of a register buffer as FP32 values (planes: (hi << 16) + lo, lo signed)
    auto row_vals = [&](const unsigned (&v)[RMAX][NWD], int r, T (&x)[CPL]) {
        if constexpr (VEC == 4 && !F32) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const unsigned h = v[r][k];
                unsigned e0 = h << 16, e1 = h & 0xffff0000u;
                if constexpr (SPLIT) {
                    const int l = (int)v[r][4 + k];
                    e0 += (unsigned)((l << 16) >> 16);
                    e1 += (unsigned)(l >> 16);
                }
                x[2 * k] = (T)__uint_as_float(e0);
                x[2 * k + 1] = (T)__uint_as_float(e1);
            }
        } else {
#pragma unroll
            for (int e = 0; e < CPL; ++e) x[e] = (T)__uint_as_float(v[r][e]);
        }
    };

    unsigned bufA[RMAX][NWD], bufB[RMAX][NWD];
    load_step(0, bufA);
    const T* W = (const T*)g.W;
    for (int i = tid; i < RB * MP; i += 256) {
        const int b = i / MP, k = i - b * MP;
        const bool in = b < nb && k < M;
        wb[i] = in ? W[((long)(b0 + b) * g.nsrc + bs) * M + k] : T(0);
        wa[i] = (back && in) ? W[((long)(b0 + b) * g.nsrc + a) * M + k] : T(0);
        bacc[i] = T(0);
        facc[i] = T(0);
    }
    T accf[RB][CPL], war[RB][CPL];
    T bpart[NC1 ? RMAX : 1];                            // NC1: backward partials of the lane's rows
#pragma unroll
    for (int r = 0; r < (NC1 ? RMAX : 1); ++r) bpart[r] = T(0);
    __syncthreads();                                    // sources and sums staged

    // step t: strip t / nchunk, chunk t % nchunk
    auto use_step = [&](int t, const unsigned (&v)[RMAX][NWD]) {
        const int s = t / nchunk, c = t - s * nchunk;
        if (c == 0) {
            const int i0 = s * SW + CPL * cg;
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int e = 0; e < CPL; ++e) {
                    accf[b][e] = T(0);
                    war[b][e] = wa[b * MP + i0 + e];
                }
        }
        const int j0 = c * CH + rg * R;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            if (r >= R) break;                          // uniform
            const int j = j0 + r;
            T x[CPL];
            row_vals(v, r, x);
            // forward: the lane's columns
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                const T w = wb[b * MP + j];
#pragma unroll
                for (int e = 0; e < CPL; ++e) accf[b][e] += x[e] * w;
            }
            // backward: row j over the lane's columns of the strip
            if (back) {
                if constexpr (NC1) {
                    T t = bpart[r];
#pragma unroll
                    for (int e = 0; e < CPL; ++e) t += x[e] * war[0][e];
                    bpart[r] = t;
                } else {
#pragma unroll
                    for (int b = 0; b < RB; ++b) {
                        T t = T(0);
#pragma unroll
                        for (int e = 0; e < CPL; ++e) t += x[e] * war[b][e];
                        t = sum8_lanes(t);
                        if (cg == 0) bacc[b * MP + j] += t;
                    }
                }
            }
        }
        if (c == nchunk - 1) {
            // forward sums of the strip: the 8 row groups of a wave, then the four
            // waves in order (two LDS buffers by strip parity: one barrier per strip)
            T* rs = red + (size_t)(s & 1) * 4 * RB * SW;
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int e = 0; e < CPL; ++e) {
                    const T v8 = sum_rowgroups(accf[b][e]);
                    if ((tid & 63) < CG) rs[(wave * RB + b) * SW + CPL * cg + e] = v8;
                }
            __syncthreads();
            for (int idx = tid; idx < RB * SW; idx += 256) {
                const int b = idx / SW, col = idx - b * SW;
                facc[b * MP + s * SW + col] = ((rs[(0 * RB + b) * SW + col] + rs[(1 * RB + b) * SW + col]) +
                                               rs[(2 * RB + b) * SW + col]) + rs[(3 * RB + b) * SW + col];
            }
        }
    };
    for (int t = 0; t < nstep; t += 2) {
        load_step(t + 1, bufB);
        use_step(t, bufA);
        if (t + 1 >= nstep) break;                      // uniform
        load_step(t + 2, bufA);
        use_step(t + 1, bufB);
    }
    if constexpr (NC1) {
        // each row's partials over the CG lanes of its row group (one chunk: row rg R + r)
        if (back) {
#pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                if (r >= R) break;                      // uniform
                const T v = sum8_lanes(bpart[r]);
                if (cg == 0) bacc[rg * R + r] = v;
            }
        }
    }
    __syncthreads();                                    // every forward and backward sum is in LDS
    T* stage = (T*)g.stage;
    for (int idx = tid; idx < RB * M; idx += 256) {
        const int b = idx / M, j = idx - b * M;
        if (b < nb) {
            stage[((long)b * g.nrows + frow) * M + j] = facc[b * MP + j];
            if (back) stage[((long)b * g.nrows + brow) * M + j] = bacc[b * MP + j];
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

// Matrix-core form with both operands staged in LDS and the next chunk in flight:
// per reduction chunk of KC = 32 (FP64: 16) indices the workgroup holds the 64 source
// vectors (wsh, FP32/FP64) and the block's tile (FP32) in LDS; the next chunk's
// values are loaded into registers (through a buffer resource spanning the block:
// rows and columns outside it read as zero) while the MFMAs run on this one, and
// stored to LDS after a barrier.  BACK = false: the forward product (A[r][k] =
// B[k][r], sources of box b, the tile is KC stored rows x the workgroup's 64 RT
// columns); BACK = true: the backward one (A[r][k] = B[r][k], sources of box a,
// the tile is the workgroup's 64 RT stored rows x KC columns).  M is a multiple of 4.
template <int PREC, int RT, typename TS, bool BACK>
__global__ __launch_bounds__(256) void k_pair_mma(PairStream g, int b0, int rblocks)
{
    typedef typename Acc<PREC>::V V;
    typedef typename Acc<PREC>::T T;
    constexpr bool SPLIT = std::is_same<TS, OpsSplit>::value;
    constexpr bool F32 = std::is_same<TS, float>::value;
    constexpr int ESZ = F32 ? 4 : 2;
    constexpr int KC = PREC == ERT_FP64 ? 16 : 32;   // FP64: fewer registers in flight, 2 waves per SIMD
    constexpr int LDW = 80;                       // padded LDS row of the sources (columns)
    constexpr int ROWS = 64 * RT;                 // output rows of the workgroup
    constexpr int TPB = KC + 4;                   // backward tile pitch (rows of KC values)
    constexpr int TPF = ROWS + 4;                 // forward tile pitch (rows of ROWS values)
    constexpr int TILE = BACK ? ROWS * TPB : KC * TPF;
    constexpr int NP = ROWS * KC / 4 / 256;       // 4-value pieces of the tile per thread
    constexpr int NW = 64 * KC / 256;             // source values per thread
    __shared__ T wsh[KC * LDW];
    __shared__ __align__(16) float tile[TILE];
    const long p = blockIdx.x / rblocks;
    const long row = BACK ? g.bwd_row[p] : g.fwd_row[p];
    if (row < 0) return;                          // self block: no backward product (uniform)
    const int rblk = (int)(blockIdx.x % rblocks);
    const int nb = (g.B - b0) < 64 ? (g.B - b0) : 64;
    const int s = BACK ? g.ua[p] : g.ub[p];
    const int M = g.M;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane >> 4, li = lane & 15;
    const int rw0 = rblk * ROWS;                  // first output row of the workgroup
    const int row0 = wave * 16 * RT;              // first output row of the wave (in the tile)
    const size_t base = (size_t)p * M * M;
    const unsigned nbytes = (unsigned)((size_t)M * M * ESZ);
    const __amdgpu_buffer_rsrc_t rs0 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)((const unsigned char*)g.opsT + base * ESZ), 0, (int)nbytes, kBufFlags);
    const __amdgpu_buffer_rsrc_t rs1 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)((const unsigned char*)(SPLIT ? g.opsT_lo : g.opsT) + base * ESZ), 0, (int)nbytes, kBufFlags);
    const T* Ws = (const T*)g.W + ((long)b0 * g.nsrc + s) * M;
    const long wstride = (long)g.nsrc * M;

    // registers of the next chunk: the tile's pieces (raw words) and the source values
    typedef unsigned v2u __attribute__((ext_vector_type(2)));
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    v4u pr[NP];
    v2u pl[SPLIT ? NP : 1];
    T wr[NW];
    // piece q of the thread: tile row tr, first column tc (4 values)
    auto piece = [&](int q, int& tr, int& tc) {
        const int e = threadIdx.x + 256 * q;
        if constexpr (BACK) { tr = e / (KC / 4); tc = 4 * (e - tr * (KC / 4)); }
        else { tr = e / (ROWS / 4); tc = 4 * (e - tr * (ROWS / 4)); }
    };
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            int tr, tc;
            piece(q, tr, tc);
            // stored element (j, i): backward j = rw0 + tr, i = k0 + tc; forward j = k0 + tr, i = rw0 + tc
            const int j = BACK ? rw0 + tr : k0 + tr, i = BACK ? k0 + tc : rw0 + tc;
            const unsigned off = (j < M && i < M) ? (unsigned)(((size_t)j * M + i) * ESZ) : kBufOob;
            if constexpr (F32) {
                pr[q] = __builtin_amdgcn_raw_buffer_load_b128(rs0, off, 0, 0);
            } else {
                const v2u h = __builtin_amdgcn_raw_buffer_load_b64(rs0, off, 0, 0);
                pr[q] = v4u{h[0], h[1], 0u, 0u};
                if constexpr (SPLIT) pl[q] = __builtin_amdgcn_raw_buffer_load_b64(rs1, off, 0, 0);
            }
        }
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int e = threadIdx.x + 256 * q, b = e / KC, kk = e - b * KC;
            wr[q] = (b < nb && k0 + kk < M) ? Ws[(long)b * wstride + k0 + kk] : T(0);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            int tr, tc;
            piece(q, tr, tc);
            v4f v;
            if constexpr (F32) {
                v = v4f{__uint_as_float(pr[q][0]), __uint_as_float(pr[q][1]), __uint_as_float(pr[q][2]),
                        __uint_as_float(pr[q][3])};
            } else {
                const unsigned h0 = pr[q][0], h1 = pr[q][1];
                unsigned e0 = h0 << 16, e1 = h0 & 0xffff0000u, e2 = h1 << 16, e3 = h1 & 0xffff0000u;
                if constexpr (SPLIT) {
                    const int l0 = (int)pl[q][0], l1 = (int)pl[q][1];
                    e0 += (unsigned)((l0 << 16) >> 16);
                    e1 += (unsigned)(l0 >> 16);
                    e2 += (unsigned)((l1 << 16) >> 16);
                    e3 += (unsigned)(l1 >> 16);
                }
                v = v4f{__uint_as_float(e0), __uint_as_float(e1), __uint_as_float(e2), __uint_as_float(e3)};
            }
            *(v4f*)(tile + (BACK ? tr * TPB : tr * TPF) + tc) = v;
        }
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int e = threadIdx.x + 256 * q, b = e / KC, kk = e - b * KC;
            wsh[kk * LDW + b] = wr[q];
        }
    };
    V acc[RT][4];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = V{0, 0, 0, 0};
    fetch(0);
    stash();
    __syncthreads();
    for (int k0 = 0; k0 < M; k0 += KC) {
        const bool more = k0 + KC < M;            // uniform
        if (more) fetch(k0 + KC);
#pragma unroll 2
        for (int kk = 0; kk < KC; kk += 4) {
            T av[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const int r = row0 + 16 * rt + li;
                av[rt] = (T)(BACK ? tile[r * TPB + kk + grp] : tile[(kk + grp) * TPF + r]);
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
        if (!more) break;
        __syncthreads();                          // every wave is done with this chunk
        stash();
        __syncthreads();
    }
    // FP32 tiles: rows 4 grp + i; FP64 tiles: rows grp + 4 i (column li in both)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int b = 16 * ct + li;
        if (b >= nb) continue;
        T* dst = (T*)g.stage + ((long)b * g.nrows + row) * M;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int rb = rw0 + row0 + 16 * rt;
            if constexpr (PREC == ERT_FP64) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (rb + grp + 4 * i < M) dst[rb + grp + 4 * i] = acc[rt][ct][i];
            } else {
                if (rb + 4 * grp + 3 < M) *(V*)(dst + rb + 4 * grp) = acc[rt][ct];
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

// Split-BF16x3 products with both operands staged in LDS and the next reduction
// chunk in flight (the structure of k_pair_mma): the block tile is kept in FP32 and
// split where it is read; the 64 source vectors are split once per chunk into LDS.
template <int RT, bool TRANS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_pair_b3(PairStream g, int b0, int rblocks)
{
    constexpr int KC = 32;
    constexpr int LDK = KC + 8;                   // padded LDS row of the split sources (bf16)
    constexpr int ROWS = 64 * RT;                 // output rows of the workgroup
    constexpr int TPB = KC + 4;                   // backward tile pitch (rows of KC values)
    constexpr int TPF = ROWS + 4;                 // forward tile pitch (rows of ROWS values)
    constexpr int TILE = TRANS ? ROWS * TPB : KC * TPF;
    constexpr int NP = ROWS * KC / 4 / 256;       // 4-value pieces of the tile per thread
    constexpr int NW = 64 * KC / 256;             // source values per thread
    __shared__ __align__(16) __bf16 whi[64 * LDK];
    __shared__ __align__(16) __bf16 wlo[64 * LDK];
    __shared__ __align__(16) float tile[TILE];
    const long p = blockIdx.x / rblocks;
    const long row = TRANS ? g.bwd_row[p] : g.fwd_row[p];
    if (row < 0) return;                          // self block: no backward product (uniform)
    const int rblk = (int)(blockIdx.x % rblocks);
    const int nb = (g.B - b0) < 64 ? (g.B - b0) : 64;
    const int s = TRANS ? g.ua[p] : g.ub[p];
    const int M = g.M;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane >> 4, li = lane & 15;
    const int rw0 = rblk * ROWS;
    const int row0 = wave * 16 * RT;
    const size_t base = (size_t)p * M * M;
    const unsigned nbytes = (unsigned)((size_t)M * M * 4);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)((const float*)g.opsT + base), 0, (int)nbytes, kBufFlags);
    const float* Ws = (const float*)g.W + ((long)b0 * g.nsrc + s) * M;
    const long wstride = (long)g.nsrc * M;
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    v4u pr[NP];
    float wr[NW];
    auto piece = [&](int q, int& tr, int& tc) {
        const int e = threadIdx.x + 256 * q;
        if constexpr (TRANS) { tr = e / (KC / 4); tc = 4 * (e - tr * (KC / 4)); }
        else { tr = e / (ROWS / 4); tc = 4 * (e - tr * (ROWS / 4)); }
    };
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            int tr, tc;
            piece(q, tr, tc);
            const int j = TRANS ? rw0 + tr : k0 + tr, i = TRANS ? k0 + tc : rw0 + tc;
            const unsigned off = (j < M && i < M) ? (unsigned)(((size_t)j * M + i) * 4) : kBufOob;
            pr[q] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int e = threadIdx.x + 256 * q, b = e / KC, kk = e - b * KC;
            wr[q] = (b < nb && k0 + kk < M) ? Ws[(long)b * wstride + k0 + kk] : 0.f;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            int tr, tc;
            piece(q, tr, tc);
            *(v4u*)(tile + (TRANS ? tr * TPB : tr * TPF) + tc) = pr[q];
        }
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int e = threadIdx.x + 256 * q, b = e / KC, kk = e - b * KC;
            const __bf16 h = (__bf16)wr[q];
            whi[b * LDK + kk] = h;
            wlo[b * LDK + kk] = (__bf16)(wr[q] - (float)h);
        }
    };
    v4f acc[RT][4];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0, 0, 0, 0};
    fetch(0);
    stash();
    __syncthreads();
    for (int k0 = 0; k0 < M; k0 += KC) {
        const bool more = k0 + KC < M;            // uniform
        if (more) fetch(k0 + KC);
        v8bf ah[RT], al[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int r = row0 + 16 * rt + li;
            float av[8];
            if constexpr (TRANS) {
                const v4f x0 = *(const v4f*)(tile + r * TPB + 8 * grp);
                const v4f x1 = *(const v4f*)(tile + r * TPB + 8 * grp + 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    av[e] = x0[e];
                    av[4 + e] = x1[e];
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) av[e] = tile[(8 * grp + e) * TPF + r];
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
        if (!more) break;
        __syncthreads();
        stash();
        __syncthreads();
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int b = 16 * ct + li;
        if (b >= nb) continue;
        float* dst = (float*)g.stage + ((long)b * g.nrows + row) * M;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int rb = rw0 + row0 + 16 * rt;
            if (rb + 4 * grp + 3 < M) *(v4f*)(dst + rb + 4 * grp) = acc[rt][ct];
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

// LDS of the streaming form: forward and backward sources, backward and forward
// sums (MP each), two strips of the four waves' forward partials (strip width 64
// columns at most).
size_t sym_lds(int MP, int rb, size_t tsize)
{
    return tsize * (4 * (size_t)rb * MP + 2 * 4 * (size_t)rb * 64);
}

// One right-hand side in one chunk keeps the backward partials in registers when
// they fit without costing occupancy (FP32 sums; the FP64 ones would drop the
// kernel from 4 to 3 waves per SIMD, slower than the per-row LDS sums).
template <typename T, typename TS, int VEC>
void launch_sym(hipStream_t s, const PairStream& g, int b0, int rb, int R, int nchunk, int MP, size_t sh)
{
    const dim3 grid((unsigned)g.npairs);
    if (rb == 4) hipLaunchKernelGGL((k_pair_sym<T, TS, 4, VEC, false>), grid, dim3(256), sh, s, g, b0, R, MP);
    else if (rb == 2) hipLaunchKernelGGL((k_pair_sym<T, TS, 2, VEC, false>), grid, dim3(256), sh, s, g, b0, R, MP);
    else {
        if constexpr (sizeof(T) == 4) {
            if (nchunk == 1) {
                hipLaunchKernelGGL((k_pair_sym<T, TS, 1, VEC, true>), grid, dim3(256), sh, s, g, b0, R, MP);
                return;
            }
        }
        hipLaunchKernelGGL((k_pair_sym<T, TS, 1, VEC, false>), grid, dim3(256), sh, s, g, b0, R, MP);
    }
}

constexpr size_t kSymLdsMax = 64 * 1024;

// Streaming form: passes of 4, 2 or 1 right-hand sides (as many as the LDS allows).
// Runs launch(c) over the stored blocks (c = g), or over the stored prefix and then
// the chunks of on-demand blocks: each chunk filled into the scratch buffer, then
// c = the chunk's pairs.
template <typename F>
ert_status for_each_chunk(hipStream_t s, const PairStream& g, const PairGen* gen, F&& launch)
{
    if (!gen) return launch(g);
    if (gen->chunk < 1 || !gen->scratch || !gen->fill || g.ops_fmt != kOpsF32 || gen->stored < 0 ||
        gen->stored > g.npairs || (gen->stored > 0 && !gen->stored_ops)) {
        record_error("pair_stream: on-demand blocks need a scratch buffer, a fill step and FP32 storage");
        return ERT_EINVAL;
    }
    if (gen->stored > 0) {
        PairStream c = g;
        c.opsT = gen->stored_ops;
        c.opsT_lo = nullptr;
        c.npairs = gen->stored;
        ERT_TRY(launch(c));
    }
    for (long p0 = gen->stored; p0 < g.npairs; p0 += gen->chunk) {
        const long cnt = std::min(gen->chunk, g.npairs - p0);
        ERT_TRY(gen->fill(gen->ctx, s, p0, cnt, gen->scratch));
        PairStream c = g;
        c.opsT = gen->scratch;
        c.opsT_lo = nullptr;
        c.npairs = cnt;
        c.ua = g.ua + p0;
        c.ub = g.ub + p0;
        c.fwd_row = g.fwd_row + p0;
        c.bwd_row = g.bwd_row + p0;
        ERT_TRY(launch(c));
    }
    return ERT_OK;
}

template <typename T, typename TS>
ert_status pair_sym_t(hipStream_t s, const PairStream& g, const PairGen* gen)
{
    constexpr bool F32 = std::is_same<TS, float>::value;
    const int M = g.M;
    // rows per lane: the fewest chunks of 32 R rows (R <= 8 for FP32 storage, 4 for
    // planes) that cover M, then the smallest R; LDS rows cover the chunks and strips
    const int rmax = F32 ? 8 : 4;
    const int cpl = F32 ? 4 : 8, sw = 8 * cpl;
    const int nchunk = M >= 1 ? (M + 32 * rmax - 1) / (32 * rmax) : 1;
    const int R = std::max(1, std::min(rmax, (M + 32 * nchunk - 1) / (32 * nchunk)));
    const int MP = std::max(nchunk * 32 * R, (M + sw - 1) / sw * sw);
    if (M < 1 || M > 4096 || sym_lds(MP, 1, sizeof(T)) > kSymLdsMax) {
        record_error("pair_stream: unsupported block size");
        return ERT_EINVAL;
    }
    for (int b0 = 0; b0 < g.B;) {
        const int left = g.B - b0;
        int rb = left >= 4 ? 4 : (left >= 2 ? 2 : 1);
        while (rb > 1 && sym_lds(MP, rb, sizeof(T)) > kSymLdsMax) rb /= 2;
        const size_t sh = sym_lds(MP, rb, sizeof(T));
        {
            StageTimer t_(g.prof, s, g.prof_stage);
            ERT_TRY(for_each_chunk(s, g, gen, [&](const PairStream& c) -> ert_status {
                // whole 16-byte pieces (CPL values per plane) when rows hold a multiple of CPL
                if (M % cpl == 0) launch_sym<T, TS, 4>(s, c, b0, rb, R, nchunk, MP, sh);
                else launch_sym<T, TS, 1>(s, c, b0, rb, R, nchunk, MP, sh);
                ERT_HIP(hipGetLastError());
                return ERT_OK;
            }));
        }
        ERT_TRY(launch_reduce<T>(s, g, b0, rb));
        b0 += rb;
    }
    return ERT_OK;
}

// Matrix-core form (FP32 storage, whole or in planes), 64 right-hand sides per pass.
template <int PREC, typename TS>
ert_status pair_mfma_t(hipStream_t s, const PairStream& g, const PairGen* gen)
{
    constexpr int RT = (PREC == ERT_FP64) ? 4 : 8;
    constexpr int RTB = 4;                        // backward: 256 rows per workgroup (LDS tile)
    typedef typename Acc<PREC>::T T;
    const int rblocks = (g.M + 64 * RT - 1) / (64 * RT);
    const int rblocksb = (g.M + 64 * RTB - 1) / (64 * RTB);
    for (int b0 = 0; b0 < g.B; b0 += 64) {
        const int nb = std::min(64, g.B - b0);
        StageTimer t_(g.prof, s, g.prof_stage);
        ERT_TRY(for_each_chunk(s, g, gen, [&](const PairStream& c) -> ert_status {
            const dim3 grid((unsigned)(c.npairs * rblocks)), gridb((unsigned)(c.npairs * rblocksb));
            // whole 4-value pieces of the stored rows: both operands staged in LDS, the
            // next chunk in flight (the FP32 forward product over FP32-stored blocks keeps its
            // 512-row tiles, whose operators come straight from memory: it keeps the matrix
            // cores about 60 % busy already)
            const bool piecewise = c.M % 4 == 0;
            bool fwd_done = false;
            if constexpr (PREC == ERT_FP64 || !std::is_same<TS, float>::value) {
                // FP64, or values in 16-bit planes (decoded once into the LDS tile)
                if (piecewise) {
                    hipLaunchKernelGGL((k_pair_mma<PREC, RTB, TS, false>), gridb, dim3(256), 0, s, c, b0, rblocksb);
                    fwd_done = true;
                }
            }
            if (!fwd_done) hipLaunchKernelGGL((k_pair_mfma<PREC, RT, TS>), grid, dim3(256), 0, s, c, b0, rblocks);
            ERT_HIP(hipGetLastError());
            if (piecewise)
                hipLaunchKernelGGL((k_pair_mma<PREC, RTB, TS, true>), gridb, dim3(256), 0, s, c, b0, rblocksb);
            else
                hipLaunchKernelGGL((k_pair_mfma_back<PREC, RTB, TS>), gridb, dim3(256), 0, s, c, b0, rblocksb);
            ERT_HIP(hipGetLastError());
            return ERT_OK;
        }));
        t_.stop();
        ERT_TRY(launch_reduce<T>(s, g, b0, nb));
    }
    return ERT_OK;
}

// Split-BF16x3 matrix-core form (FP32-stored blocks, FP32 vectors), 64 right-hand
// sides per pass, for any right-hand-side count (it stays HBM-bound with one).
ert_status pair_mfma_bf16x3(hipStream_t s, const PairStream& g, const PairGen* gen)
{
    constexpr int RT = 4;
    if (g.ops_fmt != kOpsF32) {
        record_error("pair_stream: split-BF16x3 products need FP32-stored blocks");
        return ERT_EINVAL;
    }
    const int rblocks = (g.M + 64 * RT - 1) / (64 * RT);
    for (int b0 = 0; b0 < g.B; b0 += 64) {
        const int nb = std::min(64, g.B - b0);
        {
            StageTimer t_(g.prof, s, g.prof_stage);
            ERT_TRY(for_each_chunk(s, g, gen, [&](const PairStream& c) -> ert_status {
                const dim3 grid((unsigned)(c.npairs * rblocks));
                if (c.M % 4 == 0) {           // whole 4-value pieces: LDS-staged, next chunk in flight
                    hipLaunchKernelGGL((k_pair_b3<RT, false>), grid, dim3(256), 0, s, c, b0, rblocks);
                    ERT_HIP(hipGetLastError());
                    hipLaunchKernelGGL((k_pair_b3<RT, true>), grid, dim3(256), 0, s, c, b0, rblocks);
                } else {
                    hipLaunchKernelGGL((k_pair_mfma_bf16x3<RT, false>), grid, dim3(256), 0, s, c, b0, rblocks);
                    ERT_HIP(hipGetLastError());
                    hipLaunchKernelGGL((k_pair_mfma_bf16x3<RT, true>), grid, dim3(256), 0, s, c, b0, rblocks);
                }
                ERT_HIP(hipGetLastError());
                return ERT_OK;
            }));
        }
        ERT_TRY(launch_reduce<float>(s, g, b0, nb));
    }
    return ERT_OK;
}

}  // namespace

ert_status pair_stream(hipStream_t s, int prec, const PairStream& g, const PairGen* gen)
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
        return pair_mfma_bf16x3(s, g, gen);
    }
    if (g.B >= kPairMfmaMinRhs && g.M % 4 == 0) {
        switch (g.ops_fmt) {
        case kOpsSplit:
            return f64 ? pair_mfma_t<ERT_FP64, OpsSplit>(s, g, gen) : pair_mfma_t<ERT_FP32, OpsSplit>(s, g, gen);
        case kOpsHi: return pair_mfma_t<ERT_FP32, OpsHi>(s, g, gen);
        default: return f64 ? pair_mfma_t<ERT_FP64, float>(s, g, gen) : pair_mfma_t<ERT_FP32, float>(s, g, gen);
        }
    }
    switch (g.ops_fmt) {
    case kOpsSplit: return f64 ? pair_sym_t<double, OpsSplit>(s, g, gen) : pair_sym_t<float, OpsSplit>(s, g, gen);
    case kOpsHi: return pair_sym_t<float, OpsHi>(s, g, gen);
    default: return f64 ? pair_sym_t<double, float>(s, g, gen) : pair_sym_t<float, float>(s, g, gen);
    }
}

}  // namespace ertvie
