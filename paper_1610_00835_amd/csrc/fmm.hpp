// Internal interface of the fast multipole method (Sec. 3.3): tree geometry
// and the launch descriptions shared by fmm.hip (tree, transfers, operators)
// and m2l.hip (the box-offset GEMMs on the matrix cores).
#pragma once

#include "common.hpp"

namespace ertvie {

constexpr int kMaxLevels = 14;
// Offsets between far boxes lie in [-3,3]^d; far-field operators are indexed
// by the offset's lexicographic position in that cube (x fastest), 7^d slots.
constexpr int kOffSide = 7;

// Uniform 2^d-tree over the leaf lattice: level L holds the leaf boxes
// (leaf^d cells each), level l has ceil(nb / 2^(L-l)) boxes per axis.
struct FmmTree {
    int D = 3;        // dimension
    int nc = 8;       // Chebyshev nodes per axis (the paper's n)
    int K = 512;      // nodes per box, nc^D
    int Kp = 512;     // K padded to a multiple of 32 (zero rows/columns)
    int leaf = 8;     // cells per leaf side
    int S = 512;      // cells per leaf, leaf^D
    int L = 0;        // leaf level; far field exists on levels 2..L
    int nb[3] = {1, 1, 1};
    long nleaf = 1, nslot = 512;
    int nl[kMaxLevels + 1][3] = {};
    long nbox[kMaxLevels + 1] = {};
    double width[kMaxLevels + 1] = {};
};

// One offset of a box-offset GEMM: source box = target box + (o0,o1,o2);
// `op` selects the operator matrix.
struct BoxOffset {
    int o0, o1, o2, op;
};

// Box-offset GEMM on a regular box lattice:
//   L[b][t] (+)= sum_{o in list(class(t))} ops[o.op] * W[b][t + o]
// for every target box t and right-hand side b; sources outside the lattice
// contribute nothing.  With stride 2 the targets are split into the 2^d
// parity classes (each class has its own offset list, as the far-field
// interaction lists do); with stride 1 all targets form one class.
struct BoxGemm {
    int D;
    int nl[3];
    long nbox;
    int B;               // right-hand sides
    int M;               // output rows per box (multiple of 32)
    int Kd;              // reduction length per source box (multiple of 32)
    int stride;          // 2: parity classes, 1: one class
    int nclass;          // 2^d or 1
    int noff;            // offsets per class
    const BoxOffset* offs;   // device, [nclass][noff]
    const void* ops;     // [nops][M][Kd] row-major (FP64/FP32; BF16X3: bf16 high parts)
    const void* ops_lo;  // BF16X3: bf16 low parts
    const void* W;       // [B][nbox][Kd]
    void* L;             // [B][nbox][M]
    int accumulate;      // 1: L += result, 0: L = result
};

ert_status box_gemm(hipStream_t s, int prec, const BoxGemm& g);

// Offset-stationary form of the same product, for lattices with few targets
// per offset: the (target, source) pairs are grouped by offset so every
// operator matrix is streamed once; each pair's product goes to a staging row
// and a second pass sums the rows of each target in a fixed order.
struct PairTiles {
    long npairs = 0;
    int ngroups = 0;
    long ntiles = 0;          // column tiles over all groups, for the rhs capacity they were built for
    int* pt = nullptr;        // [npairs] target box
    int* ps = nullptr;        // [npairs] source box
    int* gstart = nullptr;    // [ngroups + 1] pair range of each offset group
    int* gop = nullptr;       // [ngroups] operator slot of the group
    int* tile_group = nullptr;   // [ntiles]
    int* tile_col0 = nullptr;    // [ntiles] first (pair, rhs) column of the tile
    long ntiles4 = 0;            // the same with 64-column tiles (four column blocks per workgroup)
    int* tile_group4 = nullptr;
    int* tile_col04 = nullptr;
    int* tstart = nullptr;    // [nbox + 1] pairs of each target (CSR, increasing group order)
    int* tpairs = nullptr;    // [npairs]
    // lattices of at most kPadPairs boxes: the same lists padded to kPadPairs entries per
    // target (-1 past the end) and their lengths, so that one round of loads fetches them
    int* tpad = nullptr;      // [nbox][kPadPairs]
    int* tcnt = nullptr;      // [nbox]
};
constexpr int kPadPairs = 64;

// Workgroups are handed to the eight XCDs (each with its own L2) in turn by
// linear id.  For the n workgroups with linear ids s + b, b in [0, n), this
// bijection of [0, n) gives those that share an XCD consecutive positions, so
// work items at consecutive positions share that XCD's L2.
__device__ __forceinline__ long xcd_position(long b, long n, int s = 0)
{
    auto cnt = [](long x, int j) { return (x + 7 - j) >> 3; };   // t in [0, x) with t % 8 == j
    const int k = (int)((b + s) & 7);
    long p = cnt(b + s, k) - cnt(s, k);
    for (int j = 0; j < k; ++j) p += cnt(s + n, j) - cnt(s, j);
    return p;
}

struct OffsetGemm {
    long nbox;
    int B;
    int M, Kd;
    const void* ops;
    const void* ops_lo;
    const void* W;            // [B][nbox][Kd]
    void* L;                  // [B][nbox][M]
    void* stage;              // [B][npairs][M]
    int accumulate;
    int tn;                   // column blocks of 16 per workgroup: 1 or 4
    int tm;                   // row blocks of 16 per wave: 2 or 1 (with tn = 4)
    int lds = 0;              // 1 (FP32, tn = 1): the tile's source columns staged in LDS, each
                              // wave 16 rows over the whole reduction, 64 rows per workgroup;
                              // 2 (FP32): 64-column tiles staged in LDS, each wave every fourth
                              // block of 16 rows, all rows per workgroup
    PairTiles pl;
    // operator from a table over cell offsets instead of ops (the near field of a
    // homogeneous medium; FP32/FP64, leaf a power of two >= 4): four copies of the
    // table, copy r shifted by r entries, each tlen long; tw = 4 leaf - 1 entries
    // per axis; leaf = 2^lshift
    const void* atab = nullptr;
    int tlen = 0, tw = 0, leaf = 0, lshift = 0, dim = 0;
};

ert_status offset_gemm(hipStream_t s, int prec, const OffsetGemm& g);           // products + reduction
ert_status offset_gemm_products(hipStream_t s, int prec, const OffsetGemm& g);  // staged products only
bool offset_lds_ok(int prec, const OffsetGemm& g);     // execution form 4 applies to this product
bool offset_lds64_ok(int prec, const OffsetGemm& g);   // execution form 5 applies to this product
// execution forms: 0 target-tile GEMM, 1 offset-stationary 32x16 tiles, 2 32x64, 3 16x64,
// 4 16-column tiles with the source columns in LDS (FP32), 5 64-column tiles over all rows
// with the source columns in LDS (FP32)
constexpr int kForms = 6;
ert_status offset_gemm_reduce(hipStream_t s, int prec, const OffsetGemm& g);    // per-target sums only
// two independent products (each in its own form, with its own staging rows) in one launch
// (two launches when only one of them is in form 4)
ert_status offset_gemm_pair_products(hipStream_t s, int prec, const OffsetGemm& a, const OffsetGemm& b);

// Storage of the cached blocks read by the pair products.
enum {
    kOpsNative = 0,          // values of the arithmetic type (not used by the heterogeneous caches)
    kOpsF32 = 1,             // FP32 values (FP64 products read FP32 caches)
    kOpsSplit = 2,           // FP32 values as two 16-bit planes: opsT = high halves rounded to
                             // BF16 (bits (X + 0x8000) >> 16), opsT_lo = signed remainders; the
                             // value is rebuilt exactly
    kOpsHi = 3               // the high plane alone: the FP32 values rounded to BF16
};

// Cached-pair products of a heterogeneous medium (pairs.hip).  The kernel is
// symmetric, so one block is stored per unordered pair of boxes {a, b}:
// B[j][i] = G(x_i in a, y_j in b), i fastest (M x M, M = nodes or cells per box).
// It gives the forward product for target a (sources of b) and, unless a = b, the
// backward product for target b (sources of a, through B transposed); each goes
// to the staging row of its directed pair, and a second pass sums the contiguous
// directed rows of every target in a fixed order.
struct PairStream {
    int ops_fmt;             // kOps*
    const void* opsT;        // [npairs][M][M] stored blocks
    const void* opsT_lo;     // kOpsSplit: remainder plane (same layout)
    long npairs;             // stored blocks
    const int* ua;           // [npairs] box a: target of the forward product
    const int* ub;           // [npairs] box b: source of the forward product
    const long* fwd_row;     // [npairs] staging row of the forward product
    const long* bwd_row;     // [npairs] staging row of the backward product, -1 for a self block
    long nrows;              // staging rows: directed pairs
    const int* row_src;      // [nrows] source box of each directed pair, -1: no such pair (skipped);
                             // null: every row exists
    const long* tstart;      // [ntarget + 1] contiguous directed rows of each target
    long ntarget;
    int B;
    int M;
    long nsrc;               // boxes (W is [B][nsrc][M])
    const void* W;
    void* stage;             // [rows per pass][nrows][M]: 4 per streaming pass, 64 on the matrix cores
    void* L;                 // [B][ntarget][M]
    int accumulate;
    // stage timing (ert_vie_profile): the pair products under prof_stage, their
    // per-target sums under ERT_STAGE_REDUCE; null when not profiling
    Profiler* prof = nullptr;
    int prof_stage = 0;
};

// From this many right-hand sides on, cached-pair products run on the matrix cores
// (64 right-hand sides per pass over the blocks; stage then holds min(B, 64) rows).
constexpr int kPairMfmaMinRhs = 16;
// Staging rows per pass of the streaming form.
constexpr int kPairStreamRhs = 4;

// Blocks made on demand (FP32 storage): the products take the pairs in chunks of
// `chunk`, each written into `scratch` by `fill` (kernel launches on the stream only)
// just before its products; the per-target sums follow all chunks, so the results
// are those of the stored blocks.
struct PairGen {
    long stored = 0;                // pairs 0 .. stored - 1 are in stored_ops (no fill)
    const float* stored_ops = nullptr;
    long chunk = 0;                 // pairs per chunk of the others
    float* scratch = nullptr;       // [chunk][M][M]
    ert_status (*fill)(const void* ctx, hipStream_t s, long p0, long cnt, float* dst) = nullptr;
    const void* ctx = nullptr;
};

// prec: ERT_FP64 or ERT_FP32 (streaming below kPairMfmaMinRhs right-hand sides, matrix
// cores from there on), or ERT_BF16X3 (FP32-stored blocks as split-BF16x3 matrix-core
// products with FP32 accumulation, for any right-hand-side count).  gen: null when
// g.opsT holds every block.
ert_status pair_stream(hipStream_t s, int prec, const PairStream& g, const PairGen* gen = nullptr);

// Heterogeneous media: kernel caches shared by the applies of every precision
// of a plan, in FP32 (the FP64 apply reads them and accumulates in FP64; the
// rounding of the stored kernel values, 6e-8 relative, sits far below the
// interpolation error of the far field).  One block per unordered pair of boxes.
struct HetCache {
    int nc = 0, leaf = 0;                   // tree the cache was built for
    bool owns_near = true;                  // false: the near part belongs to another order's cache
    // near field: stored blocks of the self pairs and of the neighbours at offsets
    // after the self in the 3^d order (the other half are their transposes)
    uint16_t* near_hi = nullptr;            // [near_np][S][S] BF16-rounded high halves of the FP32 values
    int16_t* near_lo = nullptr;             // [near_np][S][S] signed remainders
    long near_np = 0;
    int* near_ua = nullptr;                 // [near_np] target leaf of the forward product
    int* near_ub = nullptr;                 // [near_np] source leaf of the forward product
    long* near_fwd = nullptr;               // [near_np] directed row (leaf * 3^d + offset index)
    long* near_bwd = nullptr;               // [near_np] directed row of the transpose, -1 for a self block
    int* near_src = nullptr;                // [leaf * 3^d] source leaf of each directed row, -1 outside the grid
    long* near_tstart = nullptr;            // [nleaf + 1]
    // far field, per level: one block per unordered interaction-list pair
    float* hops[kMaxLevels + 1] = {};       // [pair][Kp][Kp]
    long hnp[kMaxLevels + 1] = {};          // stored blocks
    int* hua[kMaxLevels + 1] = {};
    int* hub[kMaxLevels + 1] = {};
    long* hfwd[kMaxLevels + 1] = {};
    long* hbwd[kMaxLevels + 1] = {};
    long hnd[kMaxLevels + 1] = {};          // directed pairs (staging rows)
    long* pstart[kMaxLevels + 1] = {};      // [nbox + 1] directed pairs of each target
    // levels whose translation matrices exceed the plan's cache budget keep the first
    // hstored[l] pairs in hops[l]; every apply rebuilds the others, `chunk` pairs at a
    // time, into `scratch` from the corner-octet table of sigma_t (kept for this)
    bool rebuilt[kMaxLevels + 1] = {};
    long hstored[kMaxLevels + 1] = {};
    float* scratch = nullptr;               // [chunk][Kp][Kp]
    long chunk = 0;
    double* st8 = nullptr;                  // [N][8] corner octets of sigma_t
    size_t bytes = 0;
    size_t far_bytes = 0;                   // stored translation matrices
    ~HetCache();
};

}  // namespace ertvie
