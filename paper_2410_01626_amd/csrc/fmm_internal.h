// fmm_internal.h -- constants and the per-evaluation geometry record shared by
// the kernels and the host side of the library.
#pragma once
#include <cstdint>

namespace fmmk {

constexpr int kDMax = 6;                    // deepest tree: 8^6 leaves
constexpr int kPMax = 15;                   // highest multipole degree
constexpr int kKMax = (kPMax + 1) * (kPMax + 1);  // 256 coefficients
constexpr int kKgMax = kPMax * kPMax;       // gradient coefficients (order p-1)
constexpr int kSortCap = 4096;              // largest leaf sorted in LDS
constexpr int kSiteCap = 1024;              // largest site sorted in LDS
constexpr int kMaxSplit = 4;                // near-field blocks per leaf, at most
constexpr int kScanFuseCap = 4096;          // leaf / site counts scanned inside the scatter kernel
constexpr double kPi = 3.14159265358979323846;
constexpr int kLeafBucketMin = 256;         // leaf bucket capacity, at least (one leaf block's threads)

// Dynamic LDS of the leaf kernel before its site-scan area: the sort buffer
// or the 64 P2M rows, whichever is larger.
constexpr int leaf_lds_base(int K, int tsz) {
    return kSortCap * 4 > 64 * (K + 1) * tsz ? kSortCap * 4 : 64 * (K + 1) * tsz;
}

// status[0]: errors raised in check mode; status[1]: informational bits
constexpr int32_t kStatusNonFinite = 1;
constexpr int32_t kStatusSite = 2;
constexpr int32_t kStatusCoincident = 4;  // two atoms at one position (after the periodic wrap)
constexpr int32_t kInfoBigLeaf = 1;  // a leaf above kSortCap kept its atomic order
constexpr int32_t kInfoBigSite = 2;  // a site above kSiteCap summed in atomic order

// Geometry and sizes of one evaluation, passed by value to every kernel.
struct Geo {
    int32_t depth;     // tree depth d
    int32_t nb;        // 2^d leaf cells per axis
    int32_t p;         // multipole order
    int32_t K;         // (p+1)^2
    int32_t Kp;        // K padded: stride of one box in the expansion arrays
    int32_t Kg;        // p^2
    int32_t nleaf;     // 8^d
    int32_t lmin;      // first level with an interaction list (1 periodic, 2 open)
    int32_t periodic;  // 1 = periodic cubic cell
    int32_t has_far;   // leaves carry a local expansion
    int32_t check;     // device-side input checks
    int32_t pad_;
    double coulomb_k;  // k_e
    int64_t nbox;      // boxes per replica (all levels)
    int64_t lev_off[kDMax + 2];  // first box of level l in the expansion arrays
};

// One replica (independent system) of an evaluation: its atoms occupy
// [a0, a0 + n) and its sites [s0, s0 + S) of the concatenated arrays; box is the
// periodic cell edge (0 for open boundaries).  blockIdx.y selects the replica.
struct RepDesc {
    int64_t a0, n, s0, S;
    double box;
    int64_t pad_;
};

constexpr int kRepsPerSet = 32;  // replica descriptors carried by one k_set_reps launch
struct RepSet {
    int32_t first, count;
    RepDesc d[kRepsPerSet];
};

}  // namespace fmmk

namespace fmmk {

// Matrix-core M2L: work items and tile sizes.
constexpr size_t kLdsBytes = 160 * 1024;  // LDS per compute unit (gfx950)

// Tree-pass kernels (M2M, L2L, root): block size and the split of a K x K
// degree-triangular operator into (segment, row) work items, one per thread.
constexpr int kTreeThreads = 512;
constexpr int kTriCache = 32;  // operator entries a thread keeps in registers
enum TriShape { kTriLower = 0, kTriUpper = 1, kTriFull = 2 };
__host__ __device__ inline int tri_nseg(int K) {
    const int n = kTreeThreads / K;
    return n < 1 ? 1 : (n > 8 ? 8 : n);
}
constexpr int kM2LWaves = 5;                 // wavefronts per matrix-core M2L work-group
constexpr int kM2LTile = 16 * kM2LWaves;     // target columns per work-group
constexpr int kM2LMaxRT = 8;    // row tiles of 16: K <= 128 (p <= 10)
constexpr int kM2LMaxKs = 4;    // bf16 k-steps of 32: K <= 128

// Four-form sites (tautomers): the extra charge forms C, D and the second
// coordinate lambda_t per site; all null for two-form evaluations.
template <typename T>
struct FormArgs {
    const T* qC;
    const T* qD;
    const double* lam_t;
};

// One M2L work item: child class (4 bx + 2 by + bz), tile of that class's
// target columns (the class's boxes of every level, deepest level first) and
// chunk of translation offsets (a range of the global offset set), with the
// chunk's first and end positions in the class's offset list.
struct M2LTask {
    int32_t cls, tile, chunk, o0, o1, pad[3];
};

}  // namespace fmmk
