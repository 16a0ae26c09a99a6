// Internal interface of the fast multipole method (Sec. 3.3): tree geometry
// and the launch descriptions shared by fmm.hip (tree, transfers, near field)
// and m2l.hip (far-field translations on MFMA).
#pragma once

#include "common.hpp"

namespace ertvie {

constexpr int kMaxLevels = 14;
// Offsets between far boxes lie in [-3,3]^d; operators are indexed by the
// offset's lexicographic position in that cube (x fastest), 7^d slots.
constexpr int kOffSide = 7;

// Uniform 2^d-tree over the leaf lattice: level L holds the leaf boxes
// (leaf^d cells each), level l has ceil(nb / 2^(L-l)) boxes per axis.
struct FmmTree {
    int D = 3;        // dimension
    int nc = 6;       // Chebyshev nodes per axis (the paper's n)
    int K = 216;      // nodes per box, nc^D
    int Kp = 224;     // K padded to a multiple of 32 (zero rows/columns)
    int leaf = 4;     // cells per leaf side
    int S = 64;       // cells per leaf, leaf^D
    int L = 0;        // leaf level; far field exists on levels 2..L
    int nb[3] = {1, 1, 1};
    long nleaf = 1, nslot = 64;
    int nl[kMaxLevels + 1][3] = {};
    long nbox[kMaxLevels + 1] = {};
    double width[kMaxLevels + 1] = {};
};

// One level of far-field translations L_t += sum_{s in IL(t)} M(t,s) W_s.
struct M2LArgs {
    int D;
    int nl[3];
    long nbox;
    int Kp;
    int B;               // right-hand sides
    const void* ops;     // homogeneous: [7^d][Kp][Kp] row-major (FP64/FP32; BF16X3: high parts, bf16)
    const void* ops_lo;  // BF16X3: low parts
    const void* W;       // multipoles [B][nbox][Kp]
    void* L;             // locals [B][nbox][Kp], accumulated into
    // heterogeneous media: one operator per (target, source) pair, CSR over targets,
    // stored transposed [pair][Kp (source node)][Kp (target node)]
    const long* pair_start;
    const int* pair_src;
};

ert_status m2l_launch(hipStream_t s, int prec, bool hetero, const M2LArgs& a);

}  // namespace ertvie
