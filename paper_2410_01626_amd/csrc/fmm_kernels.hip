// fmm_kernels.hip -- gfx950 kernels of the lambda-interpolated FMM Coulomb
// solve.  One evaluation runs, in stream order:
//   bbox (open only) -> charge_key -> scan -> scatter -> leaf_sort_gather ->
//   p2m -> m2m (per level) -> root (periodic lattice, FP64) -> m2l (all levels)
//   -> l2l (per level) -> near_far (P2P + L2P + output) -> reduce
// Box indices are Morton codes at every level; level l occupies
// [lev_off[l], lev_off[l] + 8^l) of the expansion arrays.  Particles are kept
// sorted by leaf with coordinates relative to their leaf centre, so periodic
// images reduce to integer leaf offsets times the leaf edge.
#include <type_traits>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fmm_internal.h"

namespace fmmk {


// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000FF;
    v = (v | (v << 8)) & 0x0300F00F;
    v = (v | (v << 4)) & 0x030C30C3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
}
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
    v &= 0x09249249;
    v = (v ^ (v >> 2)) & 0x030C30C3;
    v = (v ^ (v >> 4)) & 0x0300F00F;
    v = (v ^ (v >> 8)) & 0xFF0000FF;
    v = (v ^ (v >> 16)) & 0x000003FF;
    return v;
}
__device__ __forceinline__ uint32_t morton(uint32_t x, uint32_t y, uint32_t z) {
    return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}
__device__ __forceinline__ void unmorton(uint32_t m, int& x, int& y, int& z) {
    x = (int)compact3(m >> 2);
    y = (int)compact3(m >> 1);
    z = (int)compact3(m);
}

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
template <typename T> using vec4_t = typename Vec4<T>::type;

// Recurrence coefficients of the normalised regular harmonics (see
// operators.h): Rh_m^m = f_m (x + i y) Rh_{m-1}^{m-1}, Rh_{m+1}^m = sqrt(2m+1) z Rh_m^m,
// Rh_l^m = a_lm z Rh_{l-1}^m - b_lm r^2 Rh_{l-2}^m.
struct RhoCoef {
    double f[kPMax + 1];
    double a[(kPMax + 1) * (kPMax + 1)];
    double b[(kPMax + 1) * (kPMax + 1)];
};
__constant__ RhoCoef c_rho;

// The recurrence coefficients in the working type, staged in LDS once per
// block: the recurrences read them at independent addresses, so the reads
// pipeline (scalar constant loads would each wait in turn).
template <typename T>
struct RhoLds {
    T f[kPMax + 1];
    T a[(kPMax + 1) * (kPMax + 1)];
    T b[(kPMax + 1) * (kPMax + 1)];
};
template <typename T, int NT>
__device__ __forceinline__ void load_rho_lds(RhoLds<T>& rc, int p) {
    constexpr int E = ((kPMax + 1) * (kPMax + 1) + NT - 1) / NT;
    const int n = (p + 1) * (kPMax + 1);
    double va[E], vb[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int i = min((int)threadIdx.x + m * NT, n - 1);
        va[m] = c_rho.a[i];
        vb[m] = c_rho.b[i];
    }
    const double vf = c_rho.f[min((int)threadIdx.x, p)];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int i = threadIdx.x + m * NT;
        if (i < n) {
            rc.a[i] = (T)va[m];
            rc.b[i] = (T)vb[m];
        }
    }
    if ((int)threadIdx.x <= p) rc.f[threadIdx.x] = (T)vf;
}

// Visit every coefficient of rho(u) in the order m = 0..p, l = m..p, calling
// fn(kc, has_sin, re, im): kc is the index of the cosine (real) part; the sine
// part, when has_sin (m > 0), sits at kc + 1.
template <typename T, typename Fn>
__device__ __forceinline__ void for_each_rho(int p, const RhoLds<T>& rc, T x, T y, T z, Fn&& fn) {
    const T r2 = x * x + y * y + z * z;
    T cre = T(1), cim = T(0);
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            const T fm = rc.f[m];
            const T nre = fm * (x * cre - y * cim);
            const T nim = fm * (x * cim + y * cre);
            cre = nre;
            cim = nim;
        }
        const int k0 = (m == 0) ? 0 : 2 * m - 1;
        fn(m * m + k0, m > 0, cre, cim);
        if (m + 1 > p) continue;
        T p0re = cre, p0im = cim;
        T p1re = rc.a[(m + 1) * (kPMax + 1) + m] * z * cre;
        T p1im = rc.a[(m + 1) * (kPMax + 1) + m] * z * cim;
        fn((m + 1) * (m + 1) + k0, m > 0, p1re, p1im);
        for (int l = m + 2; l <= p; ++l) {
            const T al = rc.a[l * (kPMax + 1) + m];
            const T bl = rc.b[l * (kPMax + 1) + m];
            const T nre = al * z * p1re - bl * r2 * p0re;
            const T nim = al * z * p1im - bl * r2 * p0im;
            p0re = p1re;
            p0im = p1im;
            p1re = nre;
            p1im = nim;
            fn(l * l + k0, m > 0, p1re, p1im);
        }
    }
}

// Like for_each_rho, but only the orders m = m0, m0 + dm, ... are visited (the
// diagonal Rh_m^m chain is still advanced for every m): lets several
// wavefronts share one expansion evaluation.
template <typename T, typename Fn>
__device__ __forceinline__ void for_rho_orders(int p, const RhoLds<T>& rc, int m0, int dm, T x, T y, T z,
                                               Fn&& fn) {
    const T r2 = x * x + y * y + z * z;
    T cre = T(1), cim = T(0);
    int next = m0;  // next order to visit (no integer division in the loop)
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            const T fm = rc.f[m];
            const T nre = fm * (x * cre - y * cim);
            const T nim = fm * (x * cim + y * cre);
            cre = nre;
            cim = nim;
        }
        if (m != next) continue;
        next += dm;
        const int k0 = (m == 0) ? 0 : 2 * m - 1;
        fn(m * m + k0, m > 0, cre, cim);
        if (m + 1 > p) continue;
        T p0re = cre, p0im = cim;
        T p1re = rc.a[(m + 1) * (kPMax + 1) + m] * z * cre;
        T p1im = rc.a[(m + 1) * (kPMax + 1) + m] * z * cim;
        fn((m + 1) * (m + 1) + k0, m > 0, p1re, p1im);
        for (int l = m + 2; l <= p; ++l) {
            const T al = rc.a[l * (kPMax + 1) + m];
            const T bl = rc.b[l * (kPMax + 1) + m];
            const T nre = al * z * p1re - bl * r2 * p0re;
            const T nim = al * z * p1im - bl * r2 * p0im;
            p0re = p1re;
            p0im = p1im;
            p1re = nre;
            p1im = nim;
            fn(l * l + k0, m > 0, p1re, p1im);
        }
    }
}

// Inclusive scan across the 64 lanes by DPP moves (register to register, no
// LDS crossbar): shifts by 1, 2, 4 and 8 lanes within each row of 16 (a lane
// shifted in from outside the row reads 0), then the last lane of row 0 added
// to row 1 and that of row 2 to row 3, then lane 31 (the first two rows'
// total) added to rows 2 and 3.  Every lane of the wavefront must be active.
template <typename T>
__device__ __forceinline__ T wave_scan(T v) {
    v += __builtin_amdgcn_update_dpp(T(0), v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(T(0), v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(T(0), v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(T(0), v, 0x118, 0xf, 0xf, true);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(T(0), v, 0x142, 0xa, 0xf, true);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(T(0), v, 0x143, 0xc, 0xf, true);  // row_bcast:31
    return v;
}

// Lane l's value as a wavefront-uniform one, bit for bit (the readlane
// builtin returns int: a floating-point argument would be converted)
template <typename T>
__device__ __forceinline__ T lane_value(T v, int l) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    } else {
        static_assert(sizeof(T) == 4, "32- or 64-bit lane values");
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    }
}

// Sum over the 64 lanes in a fixed order (the scan's last lane), returned as
// a wavefront-uniform value.  Every lane must be active.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    return lane_value<T>(wave_scan<T>(v), 63);
}

__device__ __forceinline__ bool finite_d(double v) { return isfinite(v); }

// Split FP32 expansion coefficients into bf16 hi + lo parts (the source
// layout of the bf16x3 M2L): row `box` of the replica's split array.
__device__ __forceinline__ void store_split(uint16_t* __restrict__ msplit_rep, int KP, int64_t box, int k,
                                            float v) {
    const __bf16 h = (__bf16)v;
    const __bf16 l = (__bf16)(v - (float)h);
    uint16_t* row = msplit_rep + (size_t)box * 2 * KP;
    row[k] = __builtin_bit_cast(uint16_t, h);
    row[KP + k] = __builtin_bit_cast(uint16_t, l);
}

// ------------------------------------------------------------------ fills

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_f64(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Copy replica descriptors (carried by value in the launch) to device memory.
__global__ void k_set_reps(RepSet set, RepDesc* __restrict__ reps) {
    const int i = threadIdx.x;
    if (i < set.count) reps[set.first + i] = set.d[i];
}

// The first kernel of an evaluation of at most kRepsPerSet replicas takes the
// descriptors by value (set.count > 0): its blocks read them from the
// argument and block (0, 0) stores them for the later kernels, so no launch
// of its own is needed.  Otherwise (set.count = 0) k_set_reps stored them.
__device__ __forceinline__ RepDesc first_rep(const RepSet& set, const RepDesc* reps, int r) {
    return set.count > 0 ? set.d[r] : reps[r];
}
__device__ __forceinline__ void store_reps(const RepSet& set, RepDesc* reps) {
    if (set.count > 0 && blockIdx.x == 0 && blockIdx.y == 0 && (int)threadIdx.x < set.count)
        reps[set.first + threadIdx.x] = set.d[threadIdx.x];
}

// ------------------------------------------------------------------ domain

// Per-block min/max of the coordinates (open boundaries): part[b] = {min xyz, max xyz}.
template <typename T>
__global__ __launch_bounds__(256) void k_bbox(const T* __restrict__ x, RepSet set,
                                              RepDesc* __restrict__ reps,
                                              double* __restrict__ part) {
    __shared__ double smin[3][256], smax[3][256];
    store_reps(set, reps);
    const RepDesc rd = first_rep(set, reps, blockIdx.y);
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = rd.a0 + blockIdx.x * 256 + threadIdx.x; i < rd.a0 + rd.n;
         i += (int64_t)gridDim.x * 256)
        for (int a = 0; a < 3; ++a) {
            double v = (double)x[3 * i + a];
            mn[a] = fmin(mn[a], v);
            mx[a] = fmax(mx[a], v);
        }
    for (int a = 0; a < 3; ++a) {
        smin[a][threadIdx.x] = mn[a];
        smax[a][threadIdx.x] = mx[a];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int a = 0; a < 3; ++a) {
                smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], smin[a][threadIdx.x + s]);
                smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], smax[a][threadIdx.x + s]);
            }
        __syncthreads();
    }
    const size_t pb = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) {
            part[6 * pb + a] = smin[a][0];
            part[6 * pb + 3 + a] = smax[a][0];
        }
}

// Root cube of an open system: dom = {lo_x, lo_y, lo_z, edge}.  The edge is the
// largest extent, enlarged by a relative 2^-20 so no atom sits on the far face.
// One block per replica; dom + 8 r receives that replica's cube.
__global__ void k_bbox_final(const double* __restrict__ part, int nblk, double* __restrict__ dom_all) {
    if (threadIdx.x != 0) return;
    double* dom = dom_all + 8 * blockIdx.x;
    part += (size_t)6 * nblk * blockIdx.x;
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int b = 0; b < nblk; ++b)
        for (int a = 0; a < 3; ++a) {
            mn[a] = fmin(mn[a], part[6 * b + a]);
            mx[a] = fmax(mx[a], part[6 * b + 3 + a]);
        }
    double e = fmax(mx[0] - mn[0], fmax(mx[1] - mn[1], mx[2] - mn[2]));
    if (!(e > 0) || !(e < 1e300)) {  // no atoms, or all atoms at one point
        e = 1.0;
        if (!(mn[0] < 1e300)) mn[0] = mn[1] = mn[2] = 0.0;
    }
    e *= 1.0 + 0x1p-20;
    for (int a = 0; a < 3; ++a) dom[a] = mn[a] - 0x1p-21 * e;
    dom[3] = e;
}

// ------------------------------------------------------------------ binning

// Wave-aggregated counter increments: the lanes of a wavefront that hold the
// same key share one atomic add on counter[key] and split the returned range
// in lane order, so every lane gets a slot unique per key.  agg_plan finds
// the key groups (leader lane, offset inside the group, group size on the
// leader); the leaders then issue their adds as one instruction (distinct
// addresses, one round trip) and agg_slot spreads the result.  Atoms arrive
// grouped by molecule, so a wavefront touches few distinct leaves.
struct AggPlan {
    int leader, off, count;  // off < 0: lane not taking part
};
__device__ __forceinline__ AggPlan agg_plan(uint32_t key, bool active) {
    const int lane = (int)__lane_id();
    uint64_t todo = __ballot(active);
    AggPlan pl{0, -1, 0};
    while (todo) {
        // the leader is the same for every lane (from a wavefront-wide mask):
        // its key by a scalar lane read, not a cross-lane permute through LDS
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
        const uint64_t peers = __ballot(active && key == lk) & todo;
        if (lane == leader) pl.count = __popcll(peers);
        if ((peers >> lane) & 1) {
            pl.leader = leader;
            pl.off = __popcll(peers & ((1ull << lane) - 1));
        }
        todo &= ~peers;
    }
    return pl;
}
__device__ __forceinline__ int32_t agg_slot(const AggPlan& pl, int32_t got) {
    const int32_t base = __shfl(got, pl.leader, 64);
    return pl.off < 0 ? -1 : base + pl.off;
}

// Leaf buckets of the binning: atom indices filed per (replica, leaf) at
// their rank below cap, the rest appended to one overflow list of ovf_cap
// entries (ovf_n: its length, zeroed by the final reduction; every atom is
// appended at most once per evaluation, so ovf_cap = the atom count holds
// them all).  bucket == null: binning by a global scan and scatter instead.
struct Bins {
    int32_t* bucket;
    int32_t cap;
    int32_t* ovf;
    int32_t* ovf_n;
    int32_t ovf_cap;
};

// What the leaf kernel needs besides the buckets to bin without a scatter
// pass: per-leaf counts (its start), keys and ranks (overflow atoms), and the
// site counts and ranks (it files every site atom in its site's list and
// publishes the site starts).
struct LeafBinArgs {
    const int32_t* leaf_count;
    const int32_t* key;
    const int32_t* rank;
    const int32_t* site_count;
    const int32_t* site_rank;
    int32_t* site_start;
    int32_t* site_members;
    int S_tot;
};

// Leaf key (Morton code of the leaf cell) of every atom, its rank inside the
// leaf and inside its site (atomic counters: ranks are made stable later by
// sorting), and the input checks.  With leaf buckets (Bins.bucket set) the
// atom is also filed under its leaf at its rank (ranks >= Bins.cap go to the
// overflow list), so the leaf kernel finds a leaf's atoms without a global
// scatter pass.  The interpolated charge itself,
// q_i = qA_i + lambda_s (qB_i - qA_i) (eq 1 with interpolated charges), is
// formed in FP64 when the atoms are gathered into leaf order.
template <typename T>
__global__ __launch_bounds__(256) void k_charge_key(
    Geo g, RepSet set, RepDesc* __restrict__ reps, const T* __restrict__ x, const T* __restrict__ qA,
    const T* __restrict__ qB, const int32_t* __restrict__ site,
    const double* __restrict__ lam, FormArgs<T> fa, double* __restrict__ dom_all,
    int32_t* __restrict__ key, int32_t* __restrict__ rank, int32_t* __restrict__ leaf_count_all,
    int32_t* __restrict__ site_count, int32_t* __restrict__ site_rank,
    int32_t* __restrict__ status, Bins bins) {
    const int r = blockIdx.y;
    store_reps(set, reps);
    const RepDesc rd = first_rep(set, reps, r);
    const double box = rd.box;
    double* dom = dom_all + 8 * r;
    int32_t* leaf_count = leaf_count_all + (size_t)r * g.nleaf;
    const int64_t il = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g.periodic && il == 0) {
        dom[0] = dom[1] = dom[2] = 0.0;
        dom[3] = box;
    }
    if (rd.n == 0) return;
    // every input of the lane is loaded up front (idle lanes read the
    // replica's last atom), so the loads are in flight together
    const bool live = il < rd.n;
    const int64_t i = rd.a0 + (live ? il : rd.n - 1);
    const double xv[3] = {(double)x[3 * i], (double)x[3 * i + 1], (double)x[3 * i + 2]};
    const int32_t s_in = site[i];
    const int64_t n_sites = rd.S;
    double lo[3], edge;
    if (g.periodic) {
        lo[0] = lo[1] = lo[2] = 0.0;
        edge = box;
    } else {
        lo[0] = dom[0];
        lo[1] = dom[1];
        lo[2] = dom[2];
        edge = dom[3];
    }
    const double h = edge / g.nb;
    int c[3];
    bool bad = false;
    for (int a = 0; a < 3; ++a) {
        double v = xv[a];
        bad |= live && !finite_d(v);
        if (g.periodic) v -= edge * floor(v / edge);
        int ci = (int)floor((v - lo[a]) / h);
        c[a] = ci < 0 ? 0 : (ci >= g.nb ? g.nb - 1 : ci);
    }
    const uint32_t k = morton(c[0], c[1], c[2]);
    int32_t s = live ? s_in : -1;
    if (s < -1 || s >= n_sites) {
        if (g.check) atomicOr(&status[0], kStatusSite);
        s = -1;
    }
    // every lane of the wavefront takes part in the aggregated increments;
    // both adds are in flight together
    const uint32_t sk = (uint32_t)max(s, 0);
    const AggPlan pl = agg_plan(k, live), ps = agg_plan(sk, live && s >= 0);
    int32_t gl = 0, gs = 0;
    if (pl.count > 0) gl = atomicAdd(&leaf_count[k], pl.count);
    if (ps.count > 0) gs = atomicAdd(&site_count[rd.s0 + sk], ps.count);
    const int32_t lr = agg_slot(pl, gl), sr = agg_slot(ps, gs);
    if (!live) return;
    key[i] = (int32_t)k;
    rank[i] = lr;
    site_rank[i] = sr;
    if (bins.bucket) {
        if (lr < bins.cap) bins.bucket[((size_t)r * g.nleaf + k) * bins.cap + lr] = (int32_t)i;
        else {
            const int32_t o = atomicAdd(bins.ovf_n, 1);
            if (o < bins.ovf_cap) bins.ovf[o] = (int32_t)i;
        }
    }
    if (g.check) {
        bad |= !finite_d((double)qA[i]) || !finite_d((double)qB[i]);
        if (s >= 0) bad |= !finite_d(lam[rd.s0 + s]);
        if (fa.qC) {
            bad |= !finite_d((double)fa.qC[i]) || !finite_d((double)fa.qD[i]);
            if (s >= 0) bad |= !finite_d(fa.lam_t[rd.s0 + s]);
        }
        if (bad) atomicOr(&status[0], kStatusNonFinite);
    }
}

// Exclusive scans, one block per array: blocks 0..R-1 scan the leaf counts of
// replica r into leaf_start[r][0..nleaf] offset by the replica's first atom;
// block R scans the site counts of all replicas (global site order).
__global__ __launch_bounds__(1024) void k_scan2(const RepDesc* __restrict__ reps, int R,
                                                const int32_t* __restrict__ leaf_count,
                                                int32_t* __restrict__ leaf_start, int64_t nleaf,
                                                const int32_t* __restrict__ c1,
                                                int32_t* __restrict__ s1, int64_t n1) {
    const bool leaves = (int)blockIdx.x < R;
    const int32_t* cnt = leaves ? leaf_count + (size_t)blockIdx.x * nleaf : c1;
    int32_t* st = leaves ? leaf_start + (size_t)blockIdx.x * (nleaf + 1) : s1;
    const int64_t n = leaves ? nleaf : n1;
    const int32_t base = leaves ? (int32_t)reps[blockIdx.x].a0 : 0;
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t b = t * chunk, e = (b + chunk < n) ? b + chunk : n;
    int32_t sum = 0;
    for (int64_t i = b; i < e; ++i) sum += cnt[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = base + part[t] - sum;
    for (int64_t i = b; i < e; ++i) {
        st[i] = run;
        run += cnt[i];
    }
    if (t == 1023) st[n] = base + part[1023];
}

__global__ __launch_bounds__(256) void k_scatter(Geo g, const RepDesc* __restrict__ reps,
                                                 const int32_t* __restrict__ key,
                                                 const int32_t* __restrict__ rank,
                                                 const int32_t* __restrict__ leaf_start_all,
                                                 int32_t* __restrict__ perm,
                                                 const int32_t* __restrict__ site,
                                                 const int32_t* __restrict__ site_rank,
                                                 const int32_t* __restrict__ site_start,
                                                 int32_t* __restrict__ site_members) {
    const RepDesc rd = reps[blockIdx.y];
    const int64_t il = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (il >= rd.n) return;
    const int64_t i = rd.a0 + il;
    const int32_t* leaf_start = leaf_start_all + (size_t)blockIdx.y * (g.nleaf + 1);
    perm[leaf_start[key[i]] + rank[i]] = (int32_t)i;
    const int32_t s = site[i];
    if (s >= 0 && s < rd.S) site_members[site_start[rd.s0 + s] + site_rank[i]] = (int32_t)i;
}

// Exclusive scan of n <= kScanFuseCap global counts into LDS (out[0..n],
// offset by base) by a 256-thread block; each thread's 16 counts are loaded
// together.  tmp: 256 ints of LDS.
__device__ void block_scan_256(const int32_t* __restrict__ cnt, int n, int32_t base, int32_t* out,
                               int32_t* tmp) {
    const int t = threadIdx.x;
    constexpr int E = kScanFuseCap / 256;
    const int chunk = (n + 255) / 256;
    const int b = min(n, t * chunk), e = min(n, b + chunk);
    int32_t v[E];
    int32_t sum = 0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
        v[j] = (b + j < e) ? cnt[b + j] : 0;
        sum += v[j];
    }
    tmp[t] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t u = t >= off ? tmp[t - off] : 0;
        __syncthreads();
        tmp[t] += u;
        __syncthreads();
    }
    int32_t run = base + tmp[t] - sum;
#pragma unroll
    for (int j = 0; j < E; ++j)
        if (b + j < e) {
            out[b + j] = run;
            run += v[j];
        }
    if (t == 255) out[n] = base + tmp[255];
    __syncthreads();
}

// Counting-sort placement with the scans fused in (nleaf and the site count
// at most kScanFuseCap): every block scans its replica's leaf counts and all
// site counts in LDS, block 0 of each replica publishes leaf_start (and block
// (0, 0) site_start), then atoms are placed at start + rank.
__global__ __launch_bounds__(256) void k_scan_scatter(
    Geo g, const RepDesc* __restrict__ reps, const int32_t* __restrict__ key,
    const int32_t* __restrict__ rank, const int32_t* __restrict__ leaf_count_all,
    int32_t* __restrict__ leaf_start_all, int32_t* __restrict__ perm, const int32_t* __restrict__ site,
    const int32_t* __restrict__ site_rank, const int32_t* __restrict__ site_count,
    int32_t* __restrict__ site_start, int S_tot, int32_t* __restrict__ site_members) {
    __shared__ int32_t ls[kScanFuseCap + 1], ss[kScanFuseCap + 1], tmp[256];
    const int r = blockIdx.y;
    const RepDesc rd = reps[r];
    block_scan_256(leaf_count_all + (size_t)r * g.nleaf, (int)g.nleaf, (int32_t)rd.a0, ls, tmp);
    if (S_tot > 0) block_scan_256(site_count, S_tot, 0, ss, tmp);
    if (blockIdx.x == 0) {
        int32_t* leaf_start = leaf_start_all + (size_t)r * (g.nleaf + 1);
        for (int i = threadIdx.x; i <= g.nleaf; i += 256) leaf_start[i] = ls[i];
        if (r == 0)
            for (int i = threadIdx.x; i <= S_tot; i += 256) site_start[i] = S_tot > 0 ? ss[i] : 0;
    }
    const int64_t il = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (il >= rd.n) return;
    const int64_t i = rd.a0 + il;
    perm[ls[key[i]] + rank[i]] = (int32_t)i;
    const int32_t s = site[i];
    if (s >= 0 && s < rd.S) site_members[ss[rd.s0 + s] + site_rank[i]] = (int32_t)i;
}

// Bitonic sort of up to kSortCap ints in LDS (ascending), block-wide.
template <int CAP>
__device__ void lds_sort(int32_t* v, int n) {
    int np = 1;
    while (np < n) np <<= 1;
    for (int i = n + threadIdx.x; i < np; i += blockDim.x) v[i] = 0x7fffffff;
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < np; i += blockDim.x) {
                int l = i ^ j;
                if (l > i) {
                    bool up = (i & k) == 0;
                    int32_t a = v[i], b = v[l];
                    if ((a > b) == up) {
                        v[i] = b;
                        v[l] = a;
                    }
                }
            }
            __syncthreads();
        }
}

// ------------------------------------------------------------------ tree operators
//
// The eight child-octant operators of M2M (and of L2L) are one operator seen
// through the reflections of the axes: reflecting x, y or z maps every real
// harmonic onto +-itself, so A_c = S_c A_0 S_c with S_c diagonal +-1 (exactly,
// entry by entry).  The tree kernels (and the leaf kernel's first M2M step)
// load rows of the octant-0 operator once and apply them to signed children.

// Reflection parity of real coefficient k: bit 2 set when the coefficient
// changes sign under x -> -x, bit 1 under y -> -y, bit 0 under z -> -z.  The
// octant index c = 4 bx + 2 by + bz flips the axes whose bit is set, so the
// sign of coefficient k for octant c is (-1)^popcount(c & bits).
__device__ __forceinline__ int refl_bits(int k) {
    const int l = (int)sqrtf((float)k + 0.5f);
    const int rem = k - l * l;
    const int m = (rem + 1) >> 1;
    const int sn = (rem > 0 && !(rem & 1)) ? 1 : 0;  // sine part
    const int xo = sn ? !(m & 1) : (m & 1);
    return (xo << 2) | (sn << 1) | ((l + m) & 1);
}
__device__ __forceinline__ double refl_sign(int c, int bits) {
    return (__popc((unsigned)(c & bits)) & 1) ? -1.0 : 1.0;
}


// One thread's share of a degree-triangular K x K operator A (given
// transposed, At[k K + r]): a row r and a contiguous k range [kb, ke) of it.
// Output degree l takes input degrees <= l (M2M, kTriLower), >= l (L2L,
// kTriUpper) or all (kTriFull).  Each row is cut into nseg = 512 / K
// segments (at most 8), so a block of kTreeThreads holds every (segment,
// row) pair once.  The first kTriCache entries of the range are loaded once
// into registers and reused by every product the block forms.
// The register cache comes from a table packed on the host in the same
// thread order (entry j of thread t at j kTreeThreads + t, zero past the
// range), so its loads are coalesced.
template <typename TO, int kShape, int kCache = kTriCache>
struct TriPart {
    int r, s, kb, ke;
    TO a[kCache];
    __device__ __forceinline__ void load(int K, const TO* __restrict__ packed) {
        load(K, packed, (int)threadIdx.x);
    }
    // the share of (virtual) thread it < kTreeThreads
    __device__ __forceinline__ void load(int K, const TO* __restrict__ packed, int it) {
        const int nseg = tri_nseg(K);
        const int slen = (K + nseg - 1) / nseg;
        r = -1;
        s = kb = ke = 0;
        if (it < nseg * K) {
            s = it / K;
            r = it - s * K;
            const int l = (int)sqrtf((float)r + 0.5f);
            kb = max(s * slen, kShape == kTriUpper ? l * l : 0);
            ke = min(min(K, (s + 1) * slen), kShape == kTriLower ? (l + 1) * (l + 1) : K);
        }
#pragma unroll
        for (int j = 0; j < kCache; ++j) a[j] = packed[j * kTreeThreads + it];
    }
};

// ys[c][r] = sum_k A[r][k] xs[c][k] for the NC right-hand sides in LDS
// (FP64), with the thread's part of A from `tp` and any entries past the
// register cache loaded 16 at a time.  Segment sums are added in a fixed
// order.  part: LDS scratch of kTreeThreads * NC doubles; ys may alias xs.
// The (segment, row) share of one thread: part[(s NC + c) K + r] =
// sum_{k in [kb, ke)} A[r][k] xs[c][k] (FP64, k ascending).
template <typename TO, int NC, int kShape, int kCache>
__device__ __forceinline__ void tri_dot(const TriPart<TO, kShape, kCache>& tp, int K, const TO* __restrict__ At,
                                        const double* xs, double* part) {
    if (tp.r < 0) return;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    const int n = tp.ke - tp.kb;
#pragma unroll
    for (int j = 0; j < kCache; ++j)
        if (j < n)
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] += (double)tp.a[j] * xs[c * K + tp.kb + j];
    for (int k0 = tp.kb + kCache; k0 < tp.ke; k0 += 16) {
        TO a[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) a[j] = At[(size_t)min(k0 + j, tp.ke - 1) * K + tp.r];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int k = min(k0 + j, tp.ke - 1);
            const double aj = (k0 + j < tp.ke) ? (double)a[j] : 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] += aj * xs[c * K + k];
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) part[(tp.s * NC + c) * K + tp.r] = acc[c];
}

template <typename TO, int NC, int kShape>
__device__ void tri_matvec(const TriPart<TO, kShape>& tp, int K, const TO* __restrict__ At, double* xs,
                           double* part, double* ys) {
    const int nseg = tri_nseg(K);
    tri_dot<TO, NC, kShape, kTriCache>(tp, K, At, xs, part);
    __syncthreads();
    for (int it = threadIdx.x; it < NC * K; it += kTreeThreads) {
        double v = 0.0;
        for (int s = 0; s < nseg; ++s) v += part[s * NC * K + it];
        ys[it] = v;
    }
    __syncthreads();
}

// Per leaf, one block of 256 threads: sort the leaf's atoms by caller index
// (stable binning; leaves of up to 256 atoms by counting ranks, larger ones by
// a bitonic sort), gather (x - c_leaf, q) into the sorted particle array with
// the interpolated charge (q = qA + lambda_s (qB - qA); four forms: eq 2)
// formed in FP64, and form
// the leaf multipole mu~_leaf = sum_j q_j rho((x_j - c_leaf) / h) (P2M).
// P2M runs in passes of 64 atoms, the harmonic orders split over the 4
// wavefronts: each writes its part of q rho of every atom into the atom's LDS
// row, and thread k then sums column k in atom order.  The row buffer reuses
// the sort buffer once the sorted indices are in registers.  Periodic: also per-leaf FP64 partial sums
// of q |t/L|^2 and q (t relative to the cell centre).  Dynamic LDS:
// max(kSortCap ints, 64 x (K + 1) elements of T), then with bucket binning
// and sites 256 + S + 1 ints for the site scan.
constexpr int kLeafThreads = 256;
// operator entries a leaf thread keeps per share for the folded M2M step
// (p = 8: segments of 14 entries fit; longer ones load the rest on use)
constexpr int kLeafTriCache = 16;
constexpr int kLeafIdx = kSortCap / kLeafThreads;  // sorted indices per thread
template <typename T, bool FOLD>
__global__ __launch_bounds__(kLeafThreads) void k_leaf_p2m(
    Geo g, const RepDesc* __restrict__ reps, const T* __restrict__ x, const T* __restrict__ qA,
    const T* __restrict__ qB, const int32_t* __restrict__ site, const double* __restrict__ lam,
    FormArgs<T> fa, const double* __restrict__ dom_all, int32_t* __restrict__ leaf_start_all,
    int32_t* __restrict__ perm, vec4_t<T>* __restrict__ pos, int32_t* __restrict__ status,
    T* __restrict__ mult_all, double* __restrict__ leaf_part_all, uint16_t* __restrict__ msplit_all,
    int split_kp, Bins bins, LeafBinArgs lb, const T* __restrict__ m2m0, const T* __restrict__ m2m0_seg,
    double* __restrict__ m2m_part_all) {
    static_assert(2 * kLeafThreads == kTreeThreads, "two tree-operator shares per leaf thread");
    extern __shared__ __align__(16) unsigned char leaf_lds[];
    __shared__ RhoLds<T> rho;
    __shared__ double ps[2][kLeafThreads / 64];
    __shared__ int32_t wpre[kLeafThreads / 64], wsite[kLeafThreads / 64];
    int32_t* sbuf = (int32_t*)leaf_lds;
    T* rows = (T*)leaf_lds;
    const RepDesc rd = reps[blockIdx.y];
    const int64_t n_sites = rd.S;
    lam += rd.s0;
    const double* dom = dom_all + 8 * blockIdx.y;
    int32_t* leaf_start = leaf_start_all + (size_t)blockIdx.y * (g.nleaf + 1);
    T* mult = mult_all + (size_t)blockIdx.y * g.nbox * g.Kp;
    double* leaf_part = leaf_part_all + (size_t)blockIdx.y * g.nleaf * 2;
    const int leaf = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const bool binned = bins.bucket != nullptr;
    // bucket binning: the site starts are scanned into LDS past the sort / P2M
    // rows (the gather files each site atom in its site's list)
    int32_t* sscan = (int32_t*)(leaf_lds + leaf_lds_base(g.K, (int)sizeof(T)));
    int32_t* site_st = sscan + 256;
    // the leaf's atoms in rank order: from its bucket (ranks below bins.cap)
    // and the overflow list, or from the scattered permutation
    const int32_t* bk = binned ? bins.bucket + ((size_t)blockIdx.y * g.nleaf + leaf) * bins.cap : nullptr;
    int32_t mine_b = 0;
    int b, n;
    if (binned) {
        // every load first: the bucket slot of this thread (all slots below
        // bins.cap >= kLeafThreads exist; used where tid < n), the counts of
        // the leaves before this one and its own, and one site count per
        // thread when they fit
        const int32_t* lc = lb.leaf_count + (size_t)blockIdx.y * g.nleaf;
        mine_b = bk[tid];
        const bool one_pass = lb.S_tot <= kLeafThreads;
        const int32_t sc = (one_pass && tid < lb.S_tot) ? lb.site_count[tid] : 0;
        int32_t pre = 0;
        for (int l = tid; l < leaf; l += kLeafThreads) pre += lc[l];
        n = lc[leaf];
        // this leaf's first atom: the replica's first atom plus the counts of
        // the leaves before it (published as leaf_start); the site starts by
        // a scan of the counts, within each wavefront by DPP moves
        pre = wave_sum<int32_t>(pre);
        const int32_t inc = wave_scan<int32_t>(sc);
        if (lane == 0) wpre[wave] = pre;
        if (lane == 63) wsite[wave] = inc;
        __syncthreads();
        b = (int)rd.a0;
        int32_t sbase = 0;
#pragma unroll
        for (int w = 0; w < kLeafThreads / 64; ++w) {
            b += wpre[w];
            sbase += w < wave ? wsite[w] : 0;
        }
        if (tid == 0) {
            leaf_start[leaf] = b;
            if (leaf == g.nleaf - 1) leaf_start[g.nleaf] = b + n;
        }
        if (one_pass) {
            if (tid < lb.S_tot) site_st[tid] = sbase + inc - sc;
            if (tid == lb.S_tot - 1) site_st[lb.S_tot] = sbase + inc;
        } else {
            block_scan_256(lb.site_count, lb.S_tot, 0, site_st, sscan);
        }
        // site_st is read after the barriers below
    } else {
        b = leaf_start[leaf];
        n = leaf_start[leaf + 1] - b;
    }
    auto fill_members = [&](int32_t* dst) {
        for (int r = tid; r < min(n, bins.cap); r += kLeafThreads) dst[r] = bk[r];
        if (n > bins.cap) {
            const int no = min(*bins.ovf_n, bins.ovf_cap);
            for (int o = tid; o < no; o += kLeafThreads) {
                const int32_t i = bins.ovf[o];
                if (i >= rd.a0 && i < rd.a0 + rd.n && lb.key[i] == leaf) dst[lb.rank[i]] = i;
            }
        }
    };
    // folded first M2M step: this thread's two (segment, row) shares of the
    // octant-0 operator, loaded now so that they are in registers at the end
    // (only this instantiation pays the registers)
    TriPart<T, kTriLower, kLeafTriCache> tpa, tpb;
    if constexpr (FOLD) {
        tpa.load(g.K, m2m0_seg, tid);
        tpb.load(g.K, m2m0_seg, tid + kLeafThreads);
    }
    const double edge = dom[3];
    const double dlo[3] = {dom[0], dom[1], dom[2]};
    load_rho_lds<T, kLeafThreads>(rho, g.p);
    const bool sorted = n <= kSortCap;
    if (binned && !sorted) {
        // too large to sort: the permutation in rank order, read back below
        fill_members(perm + b);
        __syncthreads();
    }
    int32_t idx[kLeafIdx];
    if (n <= kLeafThreads) {
        // one atom per thread: its place in caller order is the number of the
        // leaf's (distinct) atom indices below its own
        __shared__ int32_t srt[kLeafThreads];
        const int32_t mine_i = tid < n ? (binned ? mine_b : perm[b + tid]) : 0;
        if (tid < n) sbuf[tid] = mine_i;
        __syncthreads();
        if (tid < n) {
            int r = 0;
            for (int k = 0; k < n; ++k) r += sbuf[k] < mine_i ? 1 : 0;
            srt[r] = mine_i;
        }
        __syncthreads();
        idx[0] = tid < n ? srt[tid] : 0;
#pragma unroll
        for (int m = 1; m < kLeafIdx; ++m) idx[m] = 0;
    } else if (sorted) {
        if (binned) fill_members(sbuf);
        else
            for (int i = tid; i < n; i += kLeafThreads) sbuf[i] = perm[b + i];
        __syncthreads();
        lds_sort<kSortCap>(sbuf, n);
#pragma unroll
        for (int m = 0; m < kLeafIdx; ++m) {
            const int j = tid + m * kLeafThreads;
            idx[m] = j < n ? sbuf[j] : 0;
        }
    } else {
        if (tid == 0) atomicOr(&status[1], kInfoBigLeaf);
#pragma unroll
        for (int m = 0; m < kLeafIdx; ++m) idx[m] = 0;
    }
    __syncthreads();  // sorted indices are in registers: the LDS is free for P2M rows
    if (binned && blockIdx.x == 0 && blockIdx.y == 0)
        for (int i = tid; i <= lb.S_tot; i += kLeafThreads) lb.site_start[i] = lb.S_tot > 0 ? site_st[i] : 0;
    const double h = edge / g.nb;
    const T ih = (T)(1.0 / h);
    int cx, cy, cz;
    unmorton((uint32_t)leaf, cx, cy, cz);
    const double cc[3] = {dlo[0] + (cx + 0.5) * h, dlo[1] + (cy + 0.5) * h, dlo[2] + (cz + 0.5) * h};
    const double off[3] = {(cx + 0.5) * h - 0.5 * edge, (cy + 0.5) * h - 0.5 * edge,
                           (cz + 0.5) * h - 0.5 * edge};
    // gather; this thread's first atom stays in registers for P2M
    vec4_t<T> mine;
    mine.x = mine.y = mine.z = mine.w = T(0);
    double s2 = 0.0, qs = 0.0;
    for (int j = tid, m = 0; j < n; j += kLeafThreads, ++m) {
        const int32_t i = sorted ? (m < kLeafIdx ? idx[m] : 0) : perm[b + j];
        if (sorted) perm[b + j] = i;
        const double xv[3] = {(double)x[3 * i], (double)x[3 * i + 1], (double)x[3 * i + 2]};
        const int32_t st = site[i];
        if (binned && st >= 0 && st < n_sites) lb.site_members[site_st[rd.s0 + st] + lb.site_rank[i]] = i;
        const double a0 = (double)qA[i], b0 = (double)qB[i];
        const bool four = fa.qC != nullptr;
        const double c0 = four ? (double)fa.qC[i] : 0.0, d0 = four ? (double)fa.qD[i] : 0.0;
        double sv[3];
        for (int d = 0; d < 3; ++d) {
            double v = xv[d];
            if (g.periodic) v -= edge * floor(v / edge);
            sv[d] = v - cc[d];
        }
        double q = a0;
        if (st >= 0 && st < n_sites) {
            if (four) {
                // four forms (Methods, eq 2): bilinear in (lambda_p, lambda_t)
                const double lp = lam[st], lt = fa.lam_t[rd.s0 + st];
                q = (1.0 - lp) * ((1.0 - lt) * a0 + lt * b0) + lp * ((1.0 - lt) * c0 + lt * d0);
            } else {
                q += lam[st] * (b0 - a0);
            }
        }
        vec4_t<T> o;
        o.x = (T)sv[0];
        o.y = (T)sv[1];
        o.z = (T)sv[2];
        o.w = (T)q;
        pos[b + j] = o;
        if (m == 0) mine = o;
        if (g.periodic) {
            const double t0 = (double)o.x + off[0], t1 = (double)o.y + off[1], t2 = (double)o.z + off[2];
            s2 += (double)o.w * (t0 * t0 + t1 * t1 + t2 * t2) / (edge * edge);
            qs += (double)o.w;
        }
    }
    if (g.periodic) {
        s2 = wave_sum<double>(s2);
        qs = wave_sum<double>(qs);
        if (lane == 0) {
            ps[0][wave] = s2;
            ps[1][wave] = qs;
        }
    }
    __syncthreads();  // pos of every atom written (later P2M passes read it back)
    // P2M in passes of 64 atoms (lane j of every wavefront takes atom c0 + j):
    // wavefront w writes the orders m = w, w + 4, ... of q rho into the atom's
    // LDS row, then thread k sums column k (one coefficient per thread, K <= 256)
    // in atom order
    constexpr int kWaves = kLeafThreads / 64;
    const int S = g.K + 1;
    T acc = T(0);
    for (int c0 = 0; c0 < n; c0 += 64) {
        const int j = c0 + lane;
        vec4_t<T> a;
        a.x = a.y = a.z = a.w = T(0);
        if (j < n) a = (c0 == 0 && wave == 0) ? mine : pos[b + j];
        const T q = a.w;
        T* row = rows + lane * S;
        for_rho_orders<T>(g.p, rho, wave, kWaves, a.x * ih, a.y * ih, a.z * ih,
                          [&](int kc, bool hs, T re, T im) {
                              row[kc] = q * re;
                              if (hs) row[kc + 1] = q * im;
                          });
        __syncthreads();
        const int nr = min(64, n - c0);
        if (tid < g.K) {
            // four interleaved partial sums keep the LDS reads in flight
            T v0 = T(0), v1 = T(0), v2 = T(0), v3 = T(0);
            int r = 0;
            for (; r + 4 <= nr; r += 4) {
                v0 += rows[r * S + tid];
                v1 += rows[(r + 1) * S + tid];
                v2 += rows[(r + 2) * S + tid];
                v3 += rows[(r + 3) * S + tid];
            }
            for (; r < nr; ++r) v0 += rows[r * S + tid];
            acc += (v0 + v1) + (v2 + v3);
        }
        __syncthreads();
    }
    const int64_t gb = g.lev_off[g.depth] + leaf;
    if (tid < g.K) {
        mult[(size_t)gb * g.Kp + tid] = acc;
        if constexpr (sizeof(T) == 4)
            if (msplit_all)
                store_split(msplit_all + (size_t)blockIdx.y * (g.nbox + 1) * 2 * split_kp, split_kp, gb, tid, acc);
    }
    if (g.periodic && tid == 0) {
        double a2 = 0.0, aq = 0.0;
        for (int w = 0; w < kWaves; ++w) {
            a2 += ps[0][w];
            aq += ps[1][w];
        }
        leaf_part[2 * leaf] = a2;
        leaf_part[2 * leaf + 1] = aq;
    }
    if constexpr (FOLD) {
        // the leaf's term of its parent's multipole, s_c(r) (A_0 S_c mu)[r]
        // for child octant c (FP64, the tree kernels' segment split and sum
        // order); the next M2M launch adds the eight terms of every parent.
        // This thread takes the tree kernels' (segment, row) shares tid and
        // tid + kLeafThreads.
        double* xsm = (double*)leaf_lds;  // K doubles, then nseg K doubles
        double* pm = xsm + g.K;
        const int c = leaf & 7;
        if (tid < g.K) xsm[tid] = refl_sign(c, refl_bits(tid)) * (double)acc;
        __syncthreads();
        tri_dot<T, 1, kTriLower, kLeafTriCache>(tpa, g.K, m2m0, xsm, pm);
        tri_dot<T, 1, kTriLower, kLeafTriCache>(tpb, g.K, m2m0, xsm, pm);
        __syncthreads();
        if (tid < g.K) {
            const int nseg = tri_nseg(g.K);
            double v = 0.0;
            for (int sg = 0; sg < nseg; ++sg) v += pm[sg * g.K + tid];
            m2m_part_all[((size_t)blockIdx.y * g.nleaf + leaf) * g.K + tid] = refl_sign(c, refl_bits(tid)) * v;
        }
    }
}

// ------------------------------------------------------------------ tree passes

// First box of level l in the level-major box order: (8^l - 1) / 7.
__device__ __forceinline__ int64_t lev_offset(int l) { return (((int64_t)1 << (3 * l)) - 1) / 7; }

constexpr int kGatherPer = 8 * kKMax / kTreeThreads;  // child coefficients per thread

// Signed children of one parent into xs[c][k] (FP64) and, for periodic
// systems, their FP64 partials (q |t/L|^2, q) into ps[2 c + w].  All loads are
// issued before any is used.
template <typename T>
__device__ __forceinline__ void gather_children(const Geo& g, int clev, int64_t first, const T* mult,
                                                const double* leaf_part, const double* box_part,
                                                double* xs, double* ps) {
    const int K = g.K;
    const T* src = mult + (size_t)(lev_offset(clev) + first) * g.Kp;
    T v[kGatherPer];
#pragma unroll
    for (int m = 0; m < kGatherPer; ++m) {
        v[m] = T(0);
        if (m * kTreeThreads >= 8 * K) continue;  // a round with no coefficient
        const int i = min((int)threadIdx.x + m * kTreeThreads, 8 * K - 1);
        const int c = i / K, k = i - c * K;
        v[m] = src[(size_t)c * g.Kp + k];
    }
    double pv = 0.0;
    if (g.periodic && threadIdx.x < 16) {
        const int c = threadIdx.x >> 1, w = threadIdx.x & 1;
        pv = clev == g.depth ? leaf_part[2 * (first + c) + w]
                             : box_part[2 * (lev_offset(clev) + first + c) + w];
    }
#pragma unroll
    for (int m = 0; m < kGatherPer; ++m) {
        const int i = threadIdx.x + m * kTreeThreads;
        if (i < 8 * K) {
            const int c = i / K, k = i - c * K;
            xs[i] = refl_sign(c, refl_bits(k)) * (double)v[m];
        }
    }
    if (g.periodic && threadIdx.x < 16) ps[threadIdx.x] = pv;
}

// As gather_children for the children (level d - 1) of level-(d - 2) box
// `box` when the leaf kernel has left each leaf's signed M2M term in part
// (K doubles per leaf): child c = sum over its eight leaves, in octant order,
// stored (T, its bf16 split, periodic partial sums) before it is used.
template <typename T>
__device__ __forceinline__ void gather_children_parts(const Geo& g, int64_t box, const double* part, T* mult,
                                                      const double* leaf_part, double* box_part,
                                                      uint16_t* msplit, int split_kp, double* xs,
                                                      double* ps) {
    const int K = g.K, clev = g.depth - 1;
    const double* src = part + (size_t)64 * box * K;
    double v[kGatherPer];
#pragma unroll
    for (int m = 0; m < kGatherPer; ++m) {
        v[m] = 0.0;
        if (m * kTreeThreads >= 8 * K) continue;  // a round with no coefficient
        const int i = min((int)threadIdx.x + m * kTreeThreads, 8 * K - 1);
        const int c = i / K, k = i - c * K;
        double t[8];
#pragma unroll
        for (int c2 = 0; c2 < 8; ++c2) t[c2] = src[(size_t)(8 * c + c2) * K + k];
        double a = 0.0;
#pragma unroll
        for (int c2 = 0; c2 < 8; ++c2) a += t[c2];
        v[m] = a;
    }
    double pv = 0.0;
    if (g.periodic && threadIdx.x < 16) {
        const int c = threadIdx.x >> 1, w = threadIdx.x & 1;
        for (int c2 = 0; c2 < 8; ++c2) pv += leaf_part[2 * (64 * box + 8 * c + c2) + w];
    }
    const int64_t cb = g.lev_off[clev] + 8 * box;
#pragma unroll
    for (int m = 0; m < kGatherPer; ++m) {
        const int i = threadIdx.x + m * kTreeThreads;
        if (i < 8 * K) {
            const int c = i / K, k = i - c * K;
            const T tv = (T)v[m];
            mult[(size_t)(cb + c) * g.Kp + k] = tv;
            if constexpr (sizeof(T) == 4)
                if (msplit) store_split(msplit, split_kp, cb + c, k, (float)tv);
            xs[i] = refl_sign(c, refl_bits(k)) * (double)tv;
        }
    }
    if (g.periodic && threadIdx.x < 16) {
        ps[threadIdx.x] = pv;
        box_part[2 * (cb + (threadIdx.x >> 1)) + (threadIdx.x & 1)] = pv;
    }
}

// parent[r] = sum_c s_c(r) (A_0 S_c mu_c)[r] from the products in ys.
__device__ __forceinline__ double combine_octants(const double* ys, int K, int r) {
    const int b = refl_bits(r);
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) acc += refl_sign(c, b) * ys[c * K + r];
    return acc;
}

// M2M into the boxes of level lev (>= 2, or >= the coarsest interacting level
// of an open system) from level lev + 1: one block per parent.  Stores the
// parent in T (and its bf16 split when the M2L wants one) and, for periodic
// systems, its FP64 partial sums.
template <typename T>
__global__ __launch_bounds__(kTreeThreads) void k_m2m(Geo g, int lev, T* __restrict__ mult_all,
                                                      const T* __restrict__ op0,
                                                      const T* __restrict__ op0_seg,
                                                      const double* __restrict__ leaf_part_all,
                                                      double* __restrict__ box_part_all,
                                                      uint16_t* __restrict__ msplit_all, int split_kp,
                                                      double* __restrict__ root_part_all,
                                                      const double* __restrict__ m2m_part_all) {
    __shared__ double xs[8 * kKMax], part[8 * kTreeThreads], ps[16];
    TriPart<T, kTriLower> tp;
    tp.load(g.K, op0_seg);
    const int rp = blockIdx.y, K = g.K, box = blockIdx.x;
    T* mult = mult_all + (size_t)rp * g.nbox * g.Kp;
    double* box_part = box_part_all + (size_t)rp * g.nbox * 2;
    if (m2m_part_all)
        // lev = d - 2: the children's multipoles from the leaves' M2M terms
        gather_children_parts<T>(g, box, m2m_part_all + (size_t)rp * g.nleaf * K, mult,
                                 leaf_part_all + (size_t)rp * g.nleaf * 2, box_part,
                                 msplit_all ? msplit_all + (size_t)rp * (g.nbox + 1) * 2 * split_kp : nullptr,
                                 split_kp, xs, ps);
    else
        gather_children<T>(g, lev + 1, 8 * (int64_t)box, mult, leaf_part_all + (size_t)rp * g.nleaf * 2,
                           box_part, xs, ps);
    __syncthreads();
    tri_matvec<T, 8, kTriLower>(tp, K, op0, xs, part, xs);
    const int64_t gb = g.lev_off[lev] + box;
    for (int r = threadIdx.x; r < K; r += kTreeThreads) {
        const double v = combine_octants(xs, K, r);
        mult[(size_t)gb * g.Kp + r] = (T)v;
        // the root share's input S_c mu (octant c = box) over column 0 of xs:
        // this thread alone reads row r of every column above
        if (root_part_all) xs[r] = refl_sign(box, refl_bits(r)) * v;
        if constexpr (sizeof(T) == 4)
            if (msplit_all)
                store_split(msplit_all + (size_t)rp * (g.nbox + 1) * 2 * split_kp, split_kp, gb, r, (float)v);
    }
    if (g.periodic && threadIdx.x < 2) {
        double v = 0.0;
        for (int c = 0; c < 8; ++c) v += ps[2 * c + threadIdx.x];
        box_part[2 * gb + threadIdx.x] = v;
    }
    if (root_part_all) {
        // level 1 of a periodic tree: this box's share of the root multipole,
        // S_c A_0 S_c mu (octant c = box), in FP64 from the unrounded sums;
        // the root is the fixed-order sum of the eight shares
        __syncthreads();
        tri_matvec<T, 1, kTriLower>(tp, K, op0, xs, part, xs);
        double* rpart = root_part_all + ((size_t)rp * 8 + box) * K;
        for (int r = threadIdx.x; r < K; r += kTreeThreads) rpart[r] = refl_sign(box, refl_bits(r)) * xs[r];
    }
}

// Near-field block order: leaves by decreasing atom count, so that the
// largest leaves are dispatched first and the smaller ones fill in behind
// them (longest-processing-time order; with 512 leaves on 256 compute units
// the unordered tail costs ~15% of the near field; ordering by the full work,
// own atoms x neighbourhood atoms, gains < 1% more).  Work-groups go
// round-robin over the 8 XCDs, so slot i runs on XCD i mod 8: when the eight
// level-1 octants hold similar atom counts (none above 9/8 of the mean),
// octant x's leaves take the slots of XCD x (largest first, paired on the
// CUs as described below), and each XCD
// reads one octant's neighbourhoods through its own L2; otherwise all leaves
// go largest first.  Key: octant, count (capped at 2^16 - 1), leaf index
// (ties: lower leaf first); needs nleaf <= kOrderCap.
// buf: kOrderCap ints of LDS.
constexpr int kOrderCap = 4096;
__device__ void leaf_work_order(const Geo& g, const int32_t* __restrict__ leaf_start,
                                int32_t* __restrict__ order, int32_t* key) {
    const int nl = g.nleaf;
    constexpr int kMaxCnt = (1 << 16) - 1;
    __shared__ int32_t oct[8];
    const int shift = g.depth > 0 ? 3 * (g.depth - 1) : 0;
    if (threadIdx.x < 8) oct[threadIdx.x] = 0;
    __syncthreads();
    if (nl >= 8)
        for (int i = threadIdx.x; i < nl; i += blockDim.x)
            atomicAdd(&oct[i >> shift], leaf_start[i + 1] - leaf_start[i]);
    __syncthreads();
    int64_t tot = 0, mx = 0;
    for (int x = 0; x < 8; ++x) {
        tot += oct[x];
        mx = max(mx, (int64_t)oct[x]);
    }
    const bool by_xcd = nl >= 8 && 64 * mx <= 9 * tot;
    for (int i = threadIdx.x; i < nl; i += blockDim.x) {
        const int c = min(leaf_start[i + 1] - leaf_start[i], kMaxCnt);
        key[i] = (by_xcd ? (i >> shift) << 28 : 0) | ((kMaxCnt - c) << 12) | i;
    }
    __syncthreads();
    lds_sort<kOrderCap>(key, nl);
    // an XCD's slots fill its CUs one work-group each, then a second round:
    // its leaves (count descending) take the first round in order and the
    // second in reverse, so each CU pairs a larger leaf with a smaller one
    const int per = nl >> 3;
    for (int i = threadIdx.x; i < nl; i += blockDim.x) {
        const int32_t leaf = key[i] & (kOrderCap - 1);
        if (by_xcd) {
            const int r = i % per, h = per >> 1;
            order[8 * (r < h ? r : h + (per - 1 - r)) + i / per] = leaf;
        } else {
            order[i] = leaf;
        }
    }
}

// Periodic root of replica rp (a block of kTreeThreads threads): mu~_0 by
// M2M from the 8 level-1 multipoles and lambda~_0 = Lat mu~_0 +
// (2 pi / 3) sum q |s/L|^2 e_0, left in v (FP64); with `store` it also writes
// mu~_0, lambda~_0 and dom[4] = Q.  xs: 8 kKMax doubles, part: 8 kTreeThreads
// doubles, ps: 16 doubles of LDS.
// As periodic_root, from the eight level-1 shares of the root multipole
// (k_m2m at level 1) and the level-1 partial sums of q |s/L|^2 and q.
__device__ void periodic_root_from_shares(const Geo& g, int rp, const double* __restrict__ root_part_all,
                                          const double* __restrict__ box_part_all,
                                          const double* __restrict__ latT,
                                          const double* __restrict__ lat_seg,
                                          double* __restrict__ root_m_all, double* __restrict__ root_l_all,
                                          double* __restrict__ dom_all, double* xs, double* part, double* v) {
    const int K = g.K;
    TriPart<double, kTriFull> tl;
    tl.load(K, lat_seg);
    const double* rpart = root_part_all + (size_t)rp * 8 * K;
    const double* bpart = box_part_all + ((size_t)rp * g.nbox + g.lev_off[1]) * 2;
    double sh[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) sh[c] = (int)threadIdx.x < K ? rpart[(size_t)c * K + threadIdx.x] : 0.0;
    double s2 = 0.0, qs = 0.0;
    for (int c = 0; c < 8; ++c) {
        s2 += bpart[2 * c];
        qs += bpart[2 * c + 1];
    }
    if ((int)threadIdx.x < K) {
        double m = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) m += sh[c];
        v[threadIdx.x] = m;
        xs[threadIdx.x] = m;
    }
    __syncthreads();
    tri_matvec<double, 1, kTriFull>(tl, K, latT, xs, part, xs);
    for (int r = threadIdx.x; r < K; r += kTreeThreads) {
        const double lr = xs[r] + (r == 0 ? 2.0 * kPi / 3.0 * s2 : 0.0);
        root_m_all[(size_t)rp * K + r] = v[r];
        root_l_all[(size_t)rp * K + r] = lr;
        v[r] = lr;
    }
    if (threadIdx.x == 0) dom_all[8 * rp + 4] = qs;
}

// periodic_root_from_shares for a work-group of nthr threads (any size): the
// tree kernels' (segment, row) shares of the lattice operator are taken
// kTreeThreads / nthr at a time, so products and sums are the same, bit for
// bit.  xs: K doubles, part: nseg K doubles, v: K doubles of LDS.
template <int kCache>
__device__ void periodic_root_wg(const Geo& g, int rp, const double* __restrict__ root_part_all,
                                 const double* __restrict__ box_part_all, const double* __restrict__ latT,
                                 const double* __restrict__ lat_seg, double* __restrict__ root_m_all,
                                 double* __restrict__ root_l_all, double* __restrict__ dom_all, double* xs,
                                 double* part, double* v, int nthr) {
    const int K = g.K, t = threadIdx.x;
    const double* rpart = root_part_all + (size_t)rp * 8 * K;
    const double* bpart = box_part_all + ((size_t)rp * g.nbox + g.lev_off[1]) * 2;
    for (int r = t; r < K; r += nthr) {
        double m = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) m += rpart[(size_t)c * K + r];
        v[r] = m;
        xs[r] = m;
    }
    __syncthreads();
    for (int it = t; it < kTreeThreads; it += nthr) {
        TriPart<double, kTriFull, kCache> tp;
        tp.load(K, lat_seg, it);
        tri_dot<double, 1, kTriFull, kCache>(tp, K, latT, xs, part);
    }
    __syncthreads();
    double s2 = 0.0, qs = 0.0;
    for (int c = 0; c < 8; ++c) {
        s2 += bpart[2 * c];
        qs += bpart[2 * c + 1];
    }
    const int nseg = tri_nseg(K);
    for (int r = t; r < K; r += nthr) {
        double y = 0.0;
        for (int sg = 0; sg < nseg; ++sg) y += part[sg * K + r];
        const double lr = y + (r == 0 ? 2.0 * kPi / 3.0 * s2 : 0.0);
        root_m_all[(size_t)rp * K + r] = v[r];
        root_l_all[(size_t)rp * K + r] = lr;
    }
    if (t == 0) dom_all[8 * rp + 4] = qs;
}

template <typename T>
__device__ void periodic_root(const Geo& g, int rp, const T* __restrict__ mult_all,
                              const T* __restrict__ m2m0, const T* __restrict__ m2m0_seg,
                              const double* __restrict__ leaf_part_all,
                              const double* __restrict__ box_part_all, const double* __restrict__ latT,
                              const double* __restrict__ lat_seg, double* __restrict__ root_m_all,
                              double* __restrict__ root_l_all, double* __restrict__ dom_all, double* xs,
                              double* part, double* v, double* ps, bool store) {
    const int K = g.K;
    TriPart<T, kTriLower> tm;
    tm.load(K, m2m0_seg);
    TriPart<double, kTriFull> tl;
    tl.load(K, lat_seg);
    gather_children<T>(g, 1, 0, mult_all + (size_t)rp * g.nbox * g.Kp,
                       leaf_part_all + (size_t)rp * g.nleaf * 2, box_part_all + (size_t)rp * g.nbox * 2,
                       xs, ps);
    __syncthreads();
    tri_matvec<T, 8, kTriLower>(tm, K, m2m0, xs, part, xs);
    for (int r = threadIdx.x; r < K; r += kTreeThreads) v[r] = combine_octants(xs, K, r);
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kTreeThreads) xs[k] = v[k];
    __syncthreads();
    tri_matvec<double, 1, kTriFull>(tl, K, latT, xs, part, xs);
    double s2 = 0.0, qs = 0.0;
    for (int c = 0; c < 8; ++c) {
        s2 += ps[2 * c];
        qs += ps[2 * c + 1];
    }
    for (int r = threadIdx.x; r < K; r += kTreeThreads) {
        const double lr = xs[r] + (r == 0 ? 2.0 * kPi / 3.0 * s2 : 0.0);
        if (store) {
            root_m_all[(size_t)rp * K + r] = v[r];
            root_l_all[(size_t)rp * K + r] = lr;
        }
        v[r] = lr;
    }
    if (store && threadIdx.x == 0) dom_all[8 * rp + 4] = qs;
}

// The local-expansion entry e summed over the offset chunks in a fixed order
// (four interleaved partial sums keep 16 loads in flight).
template <typename T>
__device__ __forceinline__ T m2l_chunk_sum(const T* __restrict__ part, int nchunk, int64_t tot, int64_t e) {
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
    int c = 0;
#pragma unroll 4
    for (; c + 4 <= nchunk; c += 4) {
        s0 += part[(size_t)c * tot + e];
        s1 += part[(size_t)(c + 1) * tot + e];
        s2 += part[(size_t)(c + 2) * tot + e];
        s3 += part[(size_t)(c + 3) * tot + e];
    }
    for (; c < nchunk; ++c) s0 += part[(size_t)c * tot + e];
    return (s0 + s1) + (s2 + s3);
}

// One level of the downward pass for deep trees (one block per box of level
// lev): lambda~_box = its M2L sum (in loc) + S_c A_0 S_c lambda~_parent, the
// parent's whole expansion read from loc (the root's from root_l when the
// parent is the periodic root), stored back into loc in T.  The blocks of the
// next level, and the downward pass started below the stored levels, read it.
template <typename T>
__global__ __launch_bounds__(kTreeThreads) void k_l2l_level(Geo g, int lev, int l0, T* __restrict__ loc_all,
                                                          const T* __restrict__ l2l0,
                                                          const T* __restrict__ l2l0_seg,
                                                          const double* __restrict__ root_l_all) {
    __shared__ double xs[kKMax], part[kTreeThreads];
    const int rp = blockIdx.y, K = g.K, box = blockIdx.x, c = box & 7;
    TriPart<T, kTriUpper> tp;
    tp.load(K, l2l0_seg);
    T* loc = loc_all + (size_t)rp * g.nbox * g.Kp;
    const int64_t gb = lev_offset(lev) + box;
    const T own = (int)threadIdx.x < K ? loc[(size_t)gb * g.Kp + threadIdx.x] : T(0);
    for (int k = threadIdx.x; k < K; k += kTreeThreads) {
        const double pv = g.periodic && lev == l0 + 1
                              ? root_l_all[(size_t)rp * K + k]
                              : (double)loc[(size_t)(lev_offset(lev - 1) + (box >> 3)) * g.Kp + k];
        xs[k] = refl_sign(c, refl_bits(k)) * pv;
    }
    __syncthreads();
    tri_matvec<T, 1, kTriUpper>(tp, K, l2l0, xs, part, xs);
    if ((int)threadIdx.x < K)
        loc[(size_t)gb * g.Kp + threadIdx.x] =
            (T)((double)own + refl_sign(c, refl_bits(threadIdx.x)) * xs[threadIdx.x]);
}

// Downward pass in one launch: 8 / NC blocks per box b of level depth - 1,
// each of which forms lambda~ of b and its ancestors from level l0 down (L2L
// of the parent's total plus the box's own M2L sum, in FP64) and adds the L2L
// of lambda~_b into NC of its 8 leaves (fewer leaves per block: more blocks
// share the latency-bound work, each box's chain is formed by each of its
// blocks).  Periodic systems (l0 = 0) start from the root: every block forms
// mu~_0 by M2M from the 8 level-1 multipoles and lambda~_0 = Lat mu~_0 +
// (2 pi / 3) sum q |s/L|^2 e_0 itself (block 0 also stores mu~_0, lambda~_0 and
// dom[4] = Q).  Ancestors shared by several blocks are recomputed by each;
// only the leaf expansions are stored.  Open systems start at level l0 from
// its M2L sum alone.  With root_ready the periodic root was already formed
// (by the M2L reduction launch) and is read from root_l.
template <typename T, int NC>
__global__ __launch_bounds__(kTreeThreads) void k_downward(
    Geo g, int l0, T* __restrict__ loc_all, const T* __restrict__ l2l0, const T* __restrict__ l2l0_seg,
    const T* __restrict__ mult_all, const T* __restrict__ m2m0, const T* __restrict__ m2m0_seg,
    const double* __restrict__ leaf_part_all, const double* __restrict__ box_part_all,
    const double* __restrict__ latT, const double* __restrict__ lat_seg, double* __restrict__ root_m_all,
    double* __restrict__ root_l_all, double* __restrict__ dom_all,
    const int32_t* __restrict__ leaf_start_all, int32_t* __restrict__ leaf_order_all,
    int root_ready, const T* __restrict__ m2l_part_all, int m2l_nchunk, int64_t m2l_nt_all, int l_start) {
    __shared__ double xs[8 * kKMax], part[8 * kTreeThreads];
    if (leaf_order_all && blockIdx.x + 1 == gridDim.x) {
        // the extra last block: the near-field order of this replica's leaves
        leaf_work_order(g, leaf_start_all + (size_t)blockIdx.y * (g.nleaf + 1),
                        leaf_order_all + (size_t)blockIdx.y * g.nleaf, (int32_t*)part);
        return;
    }
    __shared__ double v[kKMax], ps[16];
    __shared__ T anc[kDMax * kKMax];
    TriPart<T, kTriUpper> tp;
    tp.load(g.K, l2l0_seg);
    static_assert(8 % NC == 0, "whole leaf groups per block");
    const int rp = blockIdx.y, K = g.K, D = g.depth;
    T* loc = loc_all + (size_t)rp * g.nbox * g.Kp;
    // box b of level D - 1, its leaves c0 .. c0 + NC - 1
    const int b = blockIdx.x / (8 / NC), c0 = (blockIdx.x - b * (8 / NC)) * NC;
    // prefetch, all loads in flight together: the M2L sums of the ancestors at
    // levels la .. D - 1 and the NC leaves' own expansions
    const int la = g.periodic ? l0 + 1 : l0;
    constexpr int kAncPer = (kDMax * kKMax + kTreeThreads - 1) / kTreeThreads;
    const int nanc = (D - la) * K;
    T av[kAncPer], lv[kGatherPer];
#pragma unroll
    for (int m = 0; m < kAncPer; ++m) {
        const int i = min((int)threadIdx.x + m * kTreeThreads, max(nanc - 1, 0));
        const int li = i / K, k = i - li * K, lev = la + li;
        av[m] = nanc > 0 && !m2l_part_all ? loc[(size_t)(lev_offset(lev) + (b >> (3 * (D - 1 - lev)))) * g.Kp + k]
                                          : T(0);
    }
    T* dst = loc + (size_t)(lev_offset(D) + 8 * (size_t)b + c0) * g.Kp;
#pragma unroll
    for (int m = 0; m < kGatherPer; ++m) {
        const int i = min((int)threadIdx.x + m * kTreeThreads, NC * K - 1);
        const int c = i / K, r = i - c * K;
        lv[m] = m2l_part_all ? T(0) : dst[(size_t)c * g.Kp + r];
    }
#pragma unroll
    for (int m = 0; m < kAncPer; ++m) {
        const int i = threadIdx.x + m * kTreeThreads;
        if (i < nanc && !m2l_part_all) anc[i] = av[m];
    }
    // without a reduction launch: the ancestors' and the NC leaves' M2L sums
    // from the offset-chunk partials, added here in the reduction's order
    __shared__ T lsum[8 * kKMax];
    if (m2l_part_all) {
        const int64_t tot = m2l_nt_all * g.Kp;
        const T* pr = m2l_part_all + (size_t)rp * m2l_nchunk * tot;
        const int64_t lo = lev_offset(g.lmin);
        for (int i = threadIdx.x; i < nanc + NC * K; i += kTreeThreads) {
            int64_t box;
            int k;
            if (i < nanc) {
                const int li = i / K, lev = la + li;
                k = i - li * K;
                box = lev_offset(lev) + (b >> (3 * (D - 1 - lev)));
            } else {
                const int j = i - nanc, c = j / K;
                k = j - c * K;
                box = lev_offset(D) + 8 * (int64_t)b + c0 + c;
            }
            const T sv = m2l_chunk_sum<T>(pr, m2l_nchunk, tot, (box - lo) * g.Kp + k);
            if (i < nanc) anc[i] = sv;
            else lsum[i - nanc] = sv;
        }
    }
    if (l_start > l0) {
        // the ancestor at level l_start already holds its whole local
        // expansion (k_l2l_level launches; no offset-chunk partials here)
        __syncthreads();
        for (int k = threadIdx.x; k < K; k += kTreeThreads) v[k] = (double)anc[(l_start - la) * K + k];
    } else if (g.periodic && root_ready) {
        // formed by the extra block of the M2L reduction launch, or by the
        // resident-source M2L launch's extra work-group
        __syncthreads();
        for (int k = threadIdx.x; k < K; k += kTreeThreads) v[k] = root_l_all[(size_t)rp * K + k];
    } else if (g.periodic) {
        periodic_root<T>(g, rp, mult_all, m2m0, m2m0_seg, leaf_part_all, box_part_all, latT, lat_seg,
                         root_m_all, root_l_all, dom_all, xs, part, v, ps, blockIdx.x == 0);
    } else {
        __syncthreads();
        for (int k = threadIdx.x; k < K; k += kTreeThreads) v[k] = (double)anc[k];
    }
    __syncthreads();
    for (int lev = l_start + 1; lev < D; ++lev) {
        const int a = b >> (3 * (D - 1 - lev)), c = a & 7;
        for (int k = threadIdx.x; k < K; k += kTreeThreads) xs[k] = refl_sign(c, refl_bits(k)) * v[k];
        __syncthreads();
        tri_matvec<T, 1, kTriUpper>(tp, K, l2l0, xs, part, xs);
        for (int r = threadIdx.x; r < K; r += kTreeThreads)
            v[r] = (double)anc[(lev - la) * K + r] + refl_sign(c, refl_bits(r)) * xs[r];
        __syncthreads();
    }
    for (int i = threadIdx.x; i < NC * K; i += kTreeThreads) {
        const int c = i / K, k = i - c * K;
        xs[i] = refl_sign(c0 + c, refl_bits(k)) * v[k];
    }
    __syncthreads();
    tri_matvec<T, NC, kTriUpper>(tp, K, l2l0, xs, part, xs);
#pragma unroll
    for (int m = 0; m < kGatherPer; ++m) {
        const int i = threadIdx.x + m * kTreeThreads;
        if (i < NC * K) {
            const int c = i / K, r = i - c * K;
            const T own = m2l_part_all ? lsum[i] : lv[m];
            dst[(size_t)c * g.Kp + r] = (T)((double)own + refl_sign(c0 + c, refl_bits(r)) * xs[i]);
        }
    }
}

// Root (periodic, FP64): lambda~_root = Lat mu~_root + (2 pi / 3) sum q |s/L|^2 e_0,
// and dom[4] = Q (net charge, used by the background term at the targets).
// For a depth-0 tree the root is the leaf: mu~ is read from the level-0 slot
// of mult and lambda~ is also stored into the level-0 slot of loc.
template <typename T>
__global__ __launch_bounds__(256) void k_root(Geo g, const double* __restrict__ leaf_part_all,
                                              const double* __restrict__ root_m_all,
                                              const T* __restrict__ mult_all,
                                              const double* __restrict__ latT,
                                              double* __restrict__ root_l_all, T* __restrict__ loc_all,
                                              double* __restrict__ dom_all) {
    __shared__ double s2s[256], qss[256], mu[kKMax];
    const int rp = blockIdx.x;
    const double* leaf_part = leaf_part_all + (size_t)rp * g.nleaf * 2;
    const double* root_m = root_m_all + (size_t)rp * g.K;
    const T* mult = mult_all + (size_t)rp * g.nbox * g.Kp;
    double* root_l = root_l_all + (size_t)rp * g.K;
    T* loc = loc_all + (size_t)rp * g.nbox * g.Kp;
    double* dom = dom_all + 8 * rp;
    double s2 = 0.0, qs = 0.0;
    for (int i = threadIdx.x; i < g.nleaf; i += 256) {
        s2 += leaf_part[2 * i];
        qs += leaf_part[2 * i + 1];
    }
    s2s[threadIdx.x] = s2;
    qss[threadIdx.x] = qs;
    for (int k = threadIdx.x; k < g.K; k += 256)
        mu[k] = g.depth == 0 ? (double)mult[k] : root_m[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            s2s[threadIdx.x] += s2s[threadIdx.x + s];
            qss[threadIdx.x] += qss[threadIdx.x + s];
        }
        __syncthreads();
    }
    const int r = threadIdx.x;
    if (r < g.K) {
        double acc = 0.0;
        for (int k = 0; k < g.K; ++k) acc += latT[(size_t)k * g.K + r] * mu[k];
        if (r == 0) acc += 2.0 * kPi / 3.0 * s2s[0];
        root_l[r] = acc;
        if (g.depth == 0) loc[r] = (T)acc;
    }
    if (r == 0) dom[4] = qss[0];
}

// ------------------------------------------------------------------ M2L

// Plain M2L: one block per target box (all levels >= lmin), thread r computes
// lambda~_t[r] = sum over the interaction list of sum_k T(o)[r][k] mu~_s[k].
// Interaction list: children of the parent's 27 neighbours (periodic images
// wrapped) that are not adjacent to the target.  bankT[o][k][r].
template <typename T>
__global__ __launch_bounds__(256) void k_m2l_plain(Geo g, const T* __restrict__ mult_all,
                                                   const T* __restrict__ bankT,
                                                   T* __restrict__ loc_all) {
    __shared__ T src[kKMax];
    const T* mult = mult_all + (size_t)blockIdx.y * g.nbox * g.Kp;
    T* loc = loc_all + (size_t)blockIdx.y * g.nbox * g.Kp;
    // locate (level, box) of this block
    int lev = g.lmin;
    int64_t bidx = blockIdx.x;
    while (lev < g.depth && bidx >= ((int64_t)1 << (3 * lev))) {
        bidx -= (int64_t)1 << (3 * lev);
        ++lev;
    }
    const int n = 1 << lev;
    int tx, ty, tz;
    unmorton((uint32_t)bidx, tx, ty, tz);
    const int px = tx >> 1, py = ty >> 1, pz = tz >> 1;
    const int r = threadIdx.x;
    T acc = T(0);
    for (int nb = 0; nb < 216; ++nb) {
        const int dp = nb >> 3, cb = nb & 7;
        const int sx = 2 * (px + dp / 9 - 1) + ((cb >> 2) & 1);
        const int sy = 2 * (py + (dp / 3) % 3 - 1) + ((cb >> 1) & 1);
        const int sz = 2 * (pz + dp % 3 - 1) + (cb & 1);
        const int ox = tx - sx, oy = ty - sy, oz = tz - sz;
        if (abs(ox) <= 1 && abs(oy) <= 1 && abs(oz) <= 1) continue;
        int wx = sx, wy = sy, wz = sz;
        if (g.periodic) {
            wx = (sx % n + n) % n;
            wy = (sy % n + n) % n;
            wz = (sz % n + n) % n;
        } else if (sx < 0 || sy < 0 || sz < 0 || sx >= n || sy >= n || sz >= n) {
            continue;
        }
        const T* ms = mult + (size_t)(g.lev_off[lev] + morton(wx, wy, wz)) * g.Kp;
        __syncthreads();
        for (int k = threadIdx.x; k < g.K; k += blockDim.x) src[k] = ms[k];
        __syncthreads();
        if (r < g.K) {
            const T* op = bankT + (size_t)(((ox + 3) * 7 + (oy + 3)) * 7 + (oz + 3)) * g.K * g.K;
            for (int k = 0; k < g.K; ++k) acc += op[(size_t)k * g.K + r] * src[k];
        }
    }
    if (r < g.K) loc[(size_t)(g.lev_off[lev] + bidx) * g.Kp + r] = acc;
}

// ------------------------------------------------------------------ M2L on matrix cores
//
// For one tree level, the targets that share a child class (position inside
// their parent) share the same 189 translation offsets, so for every offset o
// the class does lambda~[:, T] += T(o) mu~[:, T - o]: a dense (K x K) x (K x 64)
// product.  A work-group takes one (level, class, 64-target tile, offset
// chunk); per offset it stages T(o) and the 64 gathered source expansions in
// LDS (k contiguous) and each wavefront multiplies one 16-target column tile
// on the matrix cores, all row tiles, accumulating in registers across the
// chunk.  Chunks write partial sums that k_m2l_reduce adds in a fixed order.
//
// Policies:
//   F32    v_mfma_f32_16x16x4_f32   A lane l: A[l%16][l/16], B: B[l/16][l%16]
//   F64    v_mfma_f64_16x16x4_f64   same inputs, output D[4v + l/16][l%16]
//   BF16X3 v_mfma_f32_16x16x32_bf16 A lane l: A[l%16][8(l/16)+e], B: B[8(l/16)+e][l%16];
//          T = Th + Tl, mu = mh + ml (bf16 parts), product Th mh + Th ml + Tl mh
// FP32 and BF16 outputs: lane l holds D[4(l/16) + v][l%16].

typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));
typedef __bf16 mbf8 __attribute__((ext_vector_type(8)));

struct M2LGeom {
    int32_t RP;      // output rows padded to 16
    int32_t KP;      // contraction length padded (4 for f32/f64, 32 for bf16)
    int32_t SA;      // LDS row stride of the operator (elements)
    int32_t SB;      // LDS row stride of the sources (elements)
    int32_t nchunk;  // offset chunks
    int32_t csize;   // nominal offsets per chunk
    int32_t ncol;    // target columns per class (all levels)
    int32_t pad_;
    int64_t nt_all;  // boxes at levels >= lmin (partial-buffer stride)
};

// Decode target column j of a work item: the class's boxes of every level,
// deepest level first.  Returns false past the class's last column.
__device__ __forceinline__ bool m2l_column(const Geo& g, int cls, int tile, int j, int& lev, int& tx,
                                           int& ty, int& tz) {
    int u = tile * kM2LTile + j;
    for (lev = g.depth; lev >= g.lmin; --lev) {
        const int sh = lev - 1, half = 1 << sh;  // half = 2^(lev - 1): shifts, not divisions
        const int ntc = 1 << (3 * sh);
        if (u < ntc) {
            const int ux = u >> (2 * sh), uy = (u >> sh) & (half - 1), uz = u & (half - 1);
            tx = 2 * ux + ((cls >> 2) & 1);
            ty = 2 * uy + ((cls >> 1) & 1);
            tz = 2 * uz + (cls & 1);
            return true;
        }
        u -= ntc;
    }
    return false;
}

// Per offset, the target columns of a work item read their sources from
// these boxes (row of the expansion arrays, or -1: no source).
__device__ __forceinline__ void m2l_source_boxes(const Geo& g, int cls, int tile, int oi,
                                                 int* __restrict__ sbox) {
    const int j = threadIdx.x;
    if (j >= kM2LTile) return;
    const int ox = oi / 49 - 3, oy = (oi / 7) % 7 - 3, oz = oi % 7 - 3;
    int lev, tx, ty, tz, b = -1;
    if (m2l_column(g, cls, tile, j, lev, tx, ty, tz)) {
        const int n = 1 << lev;
        int sx = tx - ox, sy = ty - oy, sz = tz - oz;
        bool ok = true;
        if (g.periodic) {
            sx = (sx % n + n) % n;
            sy = (sy % n + n) % n;
            sz = (sz % n + n) % n;
        } else {
            ok = sx >= 0 && sy >= 0 && sz >= 0 && sx < n && sy < n && sz < n;
        }
        if (ok) b = (int)(g.lev_off[lev] + morton(sx, sy, sz));
    }
    sbox[j] = b;
}

// Index split c -> (c / d, c % d) for small non-negative c by a float
// reciprocal (exact for c < 2^20: the fraction (c mod d + 1/2) / d stays
// inside (0, 1)).
__device__ __forceinline__ void divmod_small(int c, int d, float inv_d, int& q, int& r) {
    q = (int)(((float)c + 0.5f) * inv_d);
    r = c - q * d;
}

constexpr int kStageGroup = 8;  // loads in flight per thread while staging

// Copy operator block oi (RP x KP, row-major) into LDS rows of stride SA in
// vector chunks of type V (KP and SA are multiples of the chunk).  Loads are
// issued in groups of kStageGroup per thread before their LDS stores.
template <typename TE, typename V>
__device__ __forceinline__ void m2l_stage_op(const M2LGeom& mg, const TE* __restrict__ bank, int oi,
                                             TE* __restrict__ A) {
    constexpr int E = sizeof(V) / sizeof(TE);
    const V* src = (const V*)(bank + (size_t)oi * mg.RP * mg.KP);
    const int cpr = mg.KP / E;  // chunks per row
    const float inv = 1.0f / (float)cpr;
    const int tot = mg.RP * cpr;
    const int nt = blockDim.x;
    for (int c0 = threadIdx.x; c0 < tot; c0 += kStageGroup * nt) {
        V v[kStageGroup];
#pragma unroll
        for (int m = 0; m < kStageGroup; ++m) v[m] = src[min(c0 + m * nt, tot - 1)];
#pragma unroll
        for (int m = 0; m < kStageGroup; ++m) {
            const int c = c0 + m * nt;
            if (c < tot) {
                int r, k;
                divmod_small(c, cpr, inv, r, k);
                *(V*)(A + r * mg.SA + k * E) = v[m];
            }
        }
    }
}

// Gather the target columns' source expansions (16-byte chunks of the
// expansion rows, masked past K) into LDS as B[j][k]; bf16: split into hi and
// lo parts.  Loads are issued in groups of kStageGroup per thread.
template <typename TS, typename TL>
__device__ __forceinline__ void m2l_stage_src(const Geo& g, const M2LGeom& mg, const int* __restrict__ sbox,
                                              const TS* __restrict__ mult, TL* __restrict__ Bh,
                                              TL* __restrict__ Bl) {
    constexpr int E = 16 / sizeof(TS);
    const int cpr = mg.KP / E;
    const float inv = 1.0f / (float)cpr;
    const int tot = kM2LTile * cpr;
    const int nt = blockDim.x;
    for (int c0 = threadIdx.x; c0 < tot; c0 += kStageGroup * nt) {
        uint4 v[kStageGroup];
#pragma unroll
        for (int m = 0; m < kStageGroup; ++m) {
            const int c = min(c0 + m * nt, tot - 1);
            int j, kc;
            divmod_small(c, cpr, inv, j, kc);
            const int k = kc * E;
            const int b = sbox[j];
            // rows past the class's columns or without a source read row 0 and
            // are zeroed below; k < KP <= Kp keeps the read inside the row
            v[m] = *(const uint4*)(mult + (size_t)(b >= 0 ? b : 0) * g.Kp + (k < g.Kp ? k : 0));
        }
#pragma unroll
        for (int m = 0; m < kStageGroup; ++m) {
            const int c = c0 + m * nt;
            if (c >= tot) continue;
            int j, kc;
            divmod_small(c, cpr, inv, j, kc);
            const int k = kc * E;
            uint4 w = v[m];
            const int valid = sbox[j] >= 0 ? g.K - k : 0;  // the row padding [K, Kp) is never written
            if (E == 4) {
                if (valid < 1) w.x = 0u;
                if (valid < 2) w.y = 0u;
                if (valid < 3) w.z = 0u;
                if (valid < 4) w.w = 0u;
            } else {
                if (valid < 1) { w.x = 0u; w.y = 0u; }
                if (valid < 2) { w.z = 0u; w.w = 0u; }
            }
            if constexpr (sizeof(TL) == 2) {
                const float f0 = __uint_as_float(w.x), f1 = __uint_as_float(w.y);
                const float f2 = __uint_as_float(w.z), f3 = __uint_as_float(w.w);
                const __bf16 h0 = (__bf16)f0, h1 = (__bf16)f1, h2 = (__bf16)f2, h3 = (__bf16)f3;
                const __bf16 l0 = (__bf16)(f0 - (float)h0), l1 = (__bf16)(f1 - (float)h1);
                const __bf16 l2 = (__bf16)(f2 - (float)h2), l3 = (__bf16)(f3 - (float)h3);
                auto pk = [](__bf16 a, __bf16 c2) {
                    return (uint32_t)__builtin_bit_cast(uint16_t, a) |
                           ((uint32_t)__builtin_bit_cast(uint16_t, c2) << 16);
                };
                *(uint2*)(Bh + j * mg.SB + k) = make_uint2(pk(h0, h1), pk(h2, h3));
                *(uint2*)(Bl + j * mg.SB + k) = make_uint2(pk(l0, l1), pk(l2, l3));
            } else if constexpr (sizeof(TL) == 4) {
                *(uint2*)(Bh + j * mg.SB + k) = make_uint2(w.x, w.y);
                *(uint2*)(Bh + j * mg.SB + k + 2) = make_uint2(w.z, w.w);
            } else {
                *(uint4*)(Bh + j * mg.SB + k) = w;
            }
        }
    }
}

// Write the accumulator of row tile rt, lane layout given by `f64layout`.
template <typename TA, typename TO>
__device__ __forceinline__ void m2l_store(const Geo& g, const M2LGeom& mg, int cls, int tile,
                                          int chunk, int wave, int lane, int rt, const TA& acc,
                                          bool f64layout, TO* __restrict__ loc,
                                          TO* __restrict__ part) {
    const int j = 16 * wave + (lane & 15);
    int lev, tx, ty, tz;
    if (!m2l_column(g, cls, tile, j, lev, tx, ty, tz)) return;
    const int64_t box = lev_offset(lev) + morton(tx, ty, tz);
    TO* dst;
    if (mg.nchunk == 1) dst = loc + (size_t)box * g.Kp;
    else dst = part + ((size_t)chunk * mg.nt_all + (box - lev_offset(g.lmin))) * g.Kp;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = 16 * rt + (f64layout ? 4 * v + (lane >> 4) : 4 * (lane >> 4) + v);
        if (r < g.K) dst[r] = (TO)acc[v];
    }
}

template <int RT>
__global__ __launch_bounds__(64 * kM2LWaves) void k_m2l_f32(Geo g, M2LGeom mg, const M2LTask* __restrict__ tasks,
                                                 const int16_t* __restrict__ olist,
                                                 const int16_t* __restrict__ cstart,
                                                 const float* __restrict__ mult,
                                                 const float* __restrict__ bank,
                                                 float* __restrict__ loc, float* __restrict__ part) {
    extern __shared__ __align__(16) float lds_f32[];
    float* A = lds_f32;
    float* B = lds_f32 + mg.RP * mg.SA;
    __shared__ int sbox[kM2LTile];
    const M2LTask tk = tasks[blockIdx.x];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    mult += (size_t)blockIdx.y * g.nbox * g.Kp;
    loc += (size_t)blockIdx.y * g.nbox * g.Kp;
    if (part) part += (size_t)blockIdx.y * mg.nchunk * mg.nt_all * g.Kp;
    const bool active = tk.tile * kM2LTile + 16 * wave < mg.ncol;
    mf4 acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r] = mf4{0.f, 0.f, 0.f, 0.f};
    const int o0 = cstart[tk.cls * (mg.nchunk + 1) + tk.chunk];
    const int o1 = cstart[tk.cls * (mg.nchunk + 1) + tk.chunk + 1];
    for (int oc = o0; oc < o1; ++oc) {
        const int oi = olist[tk.cls * 189 + oc];
        __syncthreads();
        m2l_source_boxes(g, tk.cls, tk.tile, oi, sbox);
        m2l_stage_op<float, uint2>(mg, bank, oi, A);
        __syncthreads();
        m2l_stage_src<float, float>(g, mg, sbox, mult, B, nullptr);
        __syncthreads();
        if (!active) continue;
        const float* Bw = B + (16 * wave + (lane & 15)) * mg.SB + (lane >> 4);
        const float* Aw = A + (lane & 15) * mg.SA + (lane >> 4);
        for (int ks = 0; ks < mg.KP; ks += 4) {
            const float b = Bw[ks];
#pragma unroll
            for (int r = 0; r < RT; ++r)
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(Aw[16 * r * mg.SA + ks], b, acc[r], 0, 0, 0);
        }
    }
    if (!active) return;
#pragma unroll
    for (int r = 0; r < RT; ++r)
        m2l_store<mf4, float>(g, mg, tk.cls, tk.tile, tk.chunk, wave, lane, r, acc[r], false,
                              loc, part);
}

template <int RT>
__global__ __launch_bounds__(64 * kM2LWaves) void k_m2l_f64(Geo g, M2LGeom mg, const M2LTask* __restrict__ tasks,
                                                 const int16_t* __restrict__ olist,
                                                 const int16_t* __restrict__ cstart,
                                                 const double* __restrict__ mult,
                                                 const double* __restrict__ bank,
                                                 double* __restrict__ loc, double* __restrict__ part) {
    extern __shared__ __align__(16) double lds_f64[];
    double* A = lds_f64;
    double* B = lds_f64 + mg.RP * mg.SA;
    __shared__ int sbox[kM2LTile];
    const M2LTask tk = tasks[blockIdx.x];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    mult += (size_t)blockIdx.y * g.nbox * g.Kp;
    loc += (size_t)blockIdx.y * g.nbox * g.Kp;
    if (part) part += (size_t)blockIdx.y * mg.nchunk * mg.nt_all * g.Kp;
    const bool active = tk.tile * kM2LTile + 16 * wave < mg.ncol;
    md4 acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r] = md4{0.0, 0.0, 0.0, 0.0};
    const int o0 = cstart[tk.cls * (mg.nchunk + 1) + tk.chunk];
    const int o1 = cstart[tk.cls * (mg.nchunk + 1) + tk.chunk + 1];
    for (int oc = o0; oc < o1; ++oc) {
        const int oi = olist[tk.cls * 189 + oc];
        __syncthreads();
        m2l_source_boxes(g, tk.cls, tk.tile, oi, sbox);
        m2l_stage_op<double, uint4>(mg, bank, oi, A);
        __syncthreads();
        m2l_stage_src<double, double>(g, mg, sbox, mult, B, nullptr);
        __syncthreads();
        if (!active) continue;
        const double* Bw = B + (16 * wave + (lane & 15)) * mg.SB + (lane >> 4);
        const double* Aw = A + (lane & 15) * mg.SA + (lane >> 4);
        for (int ks = 0; ks < mg.KP; ks += 4) {
            const double b = Bw[ks];
#pragma unroll
            for (int r = 0; r < RT; ++r)
                acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(Aw[16 * r * mg.SA + ks], b, acc[r], 0, 0, 0);
        }
    }
    if (!active) return;
#pragma unroll
    for (int r = 0; r < RT; ++r)
        m2l_store<md4, double>(g, mg, tk.cls, tk.tile, tk.chunk, wave, lane, r, acc[r], true,
                               loc, part);
}

// bf16x3 matrix-core M2L with direct global-to-LDS staging (gfx950
// global_load_lds_dwordx4: each lane's 16 bytes land at the wavefront's LDS
// base + 16 lane).  The operator bank and the source expansions are stored
// pre-split into bf16 hi/lo parts in layouts that are their own LDS images:
//   operator o: [part][KC][RP] chunks of 8 bf16 (chunk kc of row r holds
//               k = 8 kc .. 8 kc + 7), 2 KC RP chunks, zero padded;
//   box b:      [part][KC] chunks, row nbox of each replica all zero.
// A step (one offset) copies the operator contiguously and, per target
// column, the source box's 2 KC chunks plus one pad chunk, consecutive lanes
// on consecutive chunks of one source row (a few cache lines per copy
// instruction instead of one per lane); the source box of every column for
// the offset two steps ahead is tabulated in LDS by the column's thread.  The
// odd row stride 2 KC + 1 puts the 16 columns of a fragment read in distinct
// LDS banks, and the operator fragments are 16 consecutive 16-byte chunks per
// quarter wavefront.  With two buffers the copy of offset
// i + 1 is in flight while offset i is multiplied: one wait and one barrier
// per offset.  Products Th mh + Th ml + Tl mh accumulate in FP32.
//
// Every class works from the 189 operators of class 0 (the bank holds those
// only, in list order): reflecting the axes whose bit is set in the class
// maps class 0's offsets onto the class's own, and T(P o) = S T(o) S with S
// the diagonal +-1 reflection signs.  So a column of class c applies T(o') of
// the canonical offset o' to S mu of the source at offset P o' (signs flipped
// on the B fragments) and its result is S times the accumulator (at the
// store).  Offset chunks are then equal for all classes.
constexpr int kM2LThreads = 64 * kM2LWaves;
// source copy slots per lane: kM2LTile columns of up to 2 KC + 1 = 33 chunks
constexpr int kM2LSlots = (kM2LTile * (8 * kM2LMaxKs + 1) + kM2LThreads - 1) / kM2LThreads;

__device__ __forceinline__ void lds_dma16(const uint4* gsrc, uint4* lds_wave_base) {
    __builtin_amdgcn_global_load_lds((const void*)gsrc,
                                     (__attribute__((address_space(3))) void*)lds_wave_base, 16, 0, 0);
}

template <int RT>
__global__ __launch_bounds__(kM2LThreads) void k_m2l_bf16x3(Geo g, M2LGeom mg,
                                                           const M2LTask* __restrict__ tasks,
                                                           const int16_t* __restrict__ olist,
                                                           const int16_t* __restrict__ cstart,
                                                           const uint4* __restrict__ msplit,
                                                           const uint4* __restrict__ bank, int nbuf,
                                                           const uint4* __restrict__ sign_tab,
                                                           float* __restrict__ loc, float* __restrict__ part) {
    extern __shared__ __align__(16) uint4 lds_q[];
    __shared__ int col_box[kM2LTile];
    __shared__ int src_box[2][kM2LTile];  // source box per column, two offsets ahead
    const int KC = mg.KP / 8;
    // sources: per target column its 2 KC chunks and one pad chunk (odd row
    // stride: the 16 columns of a fragment read fall in distinct LDS banks)
    const int SBc = 2 * KC + 1;
    const int a_chunks = 2 * KC * mg.RP, b_chunks = SBc * kM2LTile;
    const M2LTask tk = tasks[blockIdx.x];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    msplit += (size_t)blockIdx.y * (g.nbox + 1) * 2 * KC;
    loc += (size_t)blockIdx.y * g.nbox * g.Kp;
    if (part) part += (size_t)blockIdx.y * mg.nchunk * mg.nt_all * g.Kp;
    const bool active = tk.tile * kM2LTile + 16 * wave < mg.ncol;
    // threads < kM2LTile: their target column and its place in the tree
    int clev = 0, ctx = 0, cty = 0, ctz = 0;
    const bool col_ok = tid < kM2LTile && m2l_column(g, tk.cls, tk.tile, tid, clev, ctx, cty, ctz);
    const int cn = 1 << clev;
    const int64_t clo = lev_offset(clev);
    if (tid < kM2LTile) col_box[tid] = col_ok ? (int)(clo + morton(ctx, cty, ctz)) : -1;
    const int o0 = tk.o0, o1 = tk.o1;
    // the chunk's offsets, 64 at a time in a register (lane i: offset o0 + i)
    const int16_t* ol = olist + tk.cls * 189;
    int ol_reg = lane < o1 - o0 ? ol[o0 + lane] : 0;
    const int fx = (tk.cls & 4) ? -1 : 1, fy = (tk.cls & 2) ? -1 : 1, fz = (tk.cls & 1) ? -1 : 1;
    // source copy: buffer chunk e = t kM2LThreads + tid is chunk sc[t] of column
    // sj[t], so consecutive lanes read consecutive chunks of one source row
    int sj[kM2LSlots], sc[kM2LSlots];
#pragma unroll
    for (int t = 0; t < kM2LSlots; ++t) {
        const int e = t * kM2LThreads + tid;
        sj[t] = min(e / SBc, kM2LTile - 1);
        const int c = e - (e / SBc) * SBc;
        sc[t] = e < b_chunks ? (c == 2 * KC ? 0 : c) : -1;  // pad chunk: any in-bounds source
    }
    // the source boxes of offset slot oc for the block's columns (threads < kM2LTile)
    auto sources = [&](int oc, int* dst) {
        const int st = oc - o0;
        if (st > 0 && (st & 63) == 0) ol_reg = ol[min(oc + lane, o1 - 1)];
        const int oi = __builtin_amdgcn_readlane(ol_reg, st & 63);  // canonical offset
        if (tid < kM2LTile) {
            const int ox = fx * (oi / 49 - 3), oy = fy * ((oi / 7) % 7 - 3), oz = fz * (oi % 7 - 3);
            int sx = ctx - ox, sy = cty - oy, sz = ctz - oz;
            bool ok = col_ok;
            if (g.periodic) {
                sx &= cn - 1;
                sy &= cn - 1;
                sz &= cn - 1;
            } else {
                ok = ok && sx >= 0 && sy >= 0 && sz >= 0 && sx < cn && sy < cn && sz < cn;
            }
            dst[tid] = ok ? (int)(clo + morton(sx, sy, sz)) : (int)g.nbox;
        }
    };
    auto issue = [&](int oc, uint4* dst) {
        const uint4* src = bank + (size_t)oc * a_chunks;
        for (int c0 = 0; c0 < a_chunks; c0 += kM2LThreads)
            if (c0 + tid < a_chunks) lds_dma16(src + c0 + tid, dst + c0 + 64 * wave);
        const int* sb = src_box[(oc - o0) & 1];
        uint4* d = dst + a_chunks;
#pragma unroll
        for (int t = 0; t < kM2LSlots; ++t)
            if (sc[t] >= 0) lds_dma16(msplit + (size_t)sb[sj[t]] * 2 * KC + sc[t], d + t * kM2LThreads + 64 * wave);
    };

    mf4 acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r] = mf4{0.f, 0.f, 0.f, 0.f};
    const int col = 16 * wave + (lane & 15), kq = lane >> 4, row = lane & 15;
    // sign bits of S for the lane's B fragments (k = 8 kc + e, kc = 4 si + kq),
    // from the table sign_tab[class][kc] (bf16 sign-bit masks of 8 entries)
    uint4 bsg[kM2LMaxKs];
#pragma unroll
    for (int si = 0; si < kM2LMaxKs; ++si) bsg[si] = sign_tab[tk.cls * 4 * kM2LMaxKs + 4 * si + kq];
    if (o0 < o1) sources(o0, src_box[0]);
    if (o0 + 1 < o1) sources(o0 + 1, src_box[1]);
    __syncthreads();
    if (o0 < o1) issue(o0, lds_q);
    for (int oc = o0; oc < o1; ++oc) {
        const int st = oc - o0;
        uint4* cur = lds_q + (size_t)(st & (nbuf - 1)) * (a_chunks + b_chunks);
        __builtin_amdgcn_s_waitcnt(0);  // this lane's copies of offset oc have landed
        __syncthreads();                // everyone's have; the other buffer is free
        if (nbuf == 2 && oc + 1 < o1) issue(oc + 1, lds_q + (size_t)((st + 1) & 1) * (a_chunks + b_chunks));
        // the table slot of offset oc was last read by issue(oc) (before the
        // barrier): it now takes offset oc + 2
        if (oc + 2 < o1) sources(oc + 2, src_box[st & 1]);
        if (active) {
            const uint4* A = cur;
            const uint4* B = cur + a_chunks;
#pragma unroll
            for (int si = 0; si < kM2LMaxKs; ++si) {
                if (4 * si >= KC) break;
                const int kc = 4 * si + kq;
                uint4 uh = B[col * SBc + kc], ul = B[col * SBc + KC + kc];
                uh.x ^= bsg[si].x;
                uh.y ^= bsg[si].y;
                uh.z ^= bsg[si].z;
                uh.w ^= bsg[si].w;
                ul.x ^= bsg[si].x;
                ul.y ^= bsg[si].y;
                ul.z ^= bsg[si].z;
                ul.w ^= bsg[si].w;
                const mbf8 bh = __builtin_bit_cast(mbf8, uh);
                const mbf8 bl = __builtin_bit_cast(mbf8, ul);
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    const mbf8 ah = __builtin_bit_cast(mbf8, A[kc * mg.RP + 16 * r + row]);
                    const mbf8 al = __builtin_bit_cast(mbf8, A[(KC + kc) * mg.RP + 16 * r + row]);
                    acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[r], 0, 0, 0);
                    acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[r], 0, 0, 0);
                    acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[r], 0, 0, 0);
                }
            }
        }
        if (nbuf == 1 && oc + 1 < o1) {
            __syncthreads();
            issue(oc + 1, lds_q);
        }
    }
    // Output rows get the class's signs S; the block's results are transposed
    // through LDS (the staging buffers are free now) so that each box row is
    // written as contiguous 16-byte chunks, padding rows (zero) included.
    __syncthreads();
    float* tt = (float*)lds_q;
    const int ts = mg.RP + 4;
    if (active) {
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            // row 16 r + 4 kq + v is entry 4 (kq & 1) + v of sign chunk 2 r + kq / 2
            const uint4 m = sign_tab[tk.cls * 4 * kM2LMaxKs + 2 * r + (kq >> 1)];
            const uint32_t lo = (kq & 1) ? m.z : m.x, hi = (kq & 1) ? m.w : m.y;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t wd = v < 2 ? lo : hi;
                const bool neg = (wd >> ((v & 1) ? 31 : 15)) & 1u;
                tt[col * ts + 16 * r + 4 * kq + v] = neg ? -acc[r][v] : acc[r][v];
            }
        }
    }
    __syncthreads();
    const int cpb = g.Kp / 4;
    for (int c = tid; c < kM2LTile * cpb; c += kM2LThreads) {
        const int j = c / cpb, q4 = c - j * cpb;
        const int box = col_box[j];
        if (box < 0) continue;
        float* dst = mg.nchunk == 1
                         ? loc + (size_t)box * g.Kp
                         : part + ((size_t)tk.chunk * mg.nt_all + (box - lev_offset(g.lmin))) * g.Kp;
        *(float4*)(dst + 4 * q4) = *(const float4*)(tt + j * ts + 4 * q4);
    }
}

// bf16x3 M2L with resident sources, for trees whose classes have at most
// kM2LTile target columns (depth <= 3: one tile per class).  The target
// columns of class c sit at coordinates 2u + c (per axis, at every level), so
// the source of every column for a canonical offset o' is a box of parity
// q = c XOR (o' mod 2) at the column's level, and over all columns the
// sources are exactly that parity class of every level: one box per column.
// Chunks of offsets are cut within parity groups, so a work-group copies its
// class's source rows once (2 KC chunks each, the rows in column order, plus
// the zero row for open-boundary sources outside the domain) and per offset
// only the operator; a column reads its source at the row of the source's
// own column index (the rows are a permutation of the columns).  Staging,
// fragments and signs are those of k_m2l_bf16x3; results go to memory
// straight from the accumulators.
constexpr int kM2LRsMaxRT = 7;  // row tiles whose resident-source staging fits the LDS

// What the periodic root needs (root_l == null: no root work-group): the
// level-1 shares of the root multipole, the level-1 partial sums of q |t/L|^2
// and q, the lattice operator and where the root goes.
struct RootArgs {
    const double* root_part;
    const double* box_part;
    const double* latT;
    const double* lat_seg;
    double* root_m;
    double* root_l;
    double* dom;
};

// Largest staging sizes (16-byte chunks) of a row-tile count: the operator
// (2 KC RP) and the resident source rows (kM2LTile + 1 rows of 2 KC + 1).
__host__ __device__ constexpr int m2l_rs_kc(int rt) { return ((16 * rt + 31) / 32) * 4; }
__host__ __device__ constexpr int m2l_rs_op_chunks(int rt) { return 2 * m2l_rs_kc(rt) * 16 * rt; }
__host__ __device__ constexpr int m2l_rs_src_chunks(int rt) { return (kM2LTile + 1) * (2 * m2l_rs_kc(rt) + 1); }

template <int RT>
__global__ __launch_bounds__(kM2LThreads) void k_m2l_bf16x3_rs(Geo g, M2LGeom mg,
                                                              const M2LTask* __restrict__ tasks,
                                                              const int16_t* __restrict__ olist,
                                                              const uint4* __restrict__ msplit,
                                                              const uint4* __restrict__ bank,
                                                              const uint4* __restrict__ sign_tab,
                                                              float* __restrict__ loc, float* __restrict__ part,
                                                              RootArgs ra) {
    // three distinct LDS objects: the copy into one operator buffer provably
    // does not touch the other buffer or the source rows, so fragment reads
    // need not wait for it (one buffer in a single array made the compiler
    // wait for every copy before any LDS read)
    __shared__ uint4 opb0[m2l_rs_op_chunks(RT)], opb1[m2l_rs_op_chunks(RT)];
    __shared__ uint4 res[m2l_rs_src_chunks(RT)];
    __shared__ int col_box[kM2LTile], row_box[kM2LTile + 1];
    if (ra.root_l && blockIdx.x + 1 == gridDim.x) {
        // the extra last work-group of a periodic tree: the root's local
        // expansion from the level-1 shares, on a CU the M2L leaves free
        double* xs = (double*)opb0;
        periodic_root_wg<16>(g, blockIdx.y, ra.root_part, ra.box_part, ra.latT, ra.lat_seg, ra.root_m, ra.root_l,
                             ra.dom, xs, xs + g.K, (double*)opb1, kM2LThreads);
        return;
    }
    // KC = KP / 8 follows from the row-tile count (KP = K rounded up to 32)
    constexpr int KC = m2l_rs_kc(RT);
    constexpr int SBc = 2 * KC + 1;  // odd row stride: a fragment read's 16 rows fall in distinct banks
    constexpr int RP = 16 * RT;      // operator rows (K padded to the row tiles)
    constexpr int NKS = KC / 4;      // k-steps of 32
    constexpr int a_chunks = 2 * KC * RP;
    const int nres = mg.ncol + 1;  // source rows: one per column, then the zero row
    const M2LTask tk = tasks[blockIdx.x];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    msplit += (size_t)blockIdx.y * (g.nbox + 1) * 2 * KC;
    loc += (size_t)blockIdx.y * g.nbox * g.Kp;
    if (part) part += (size_t)blockIdx.y * mg.nchunk * mg.nt_all * g.Kp;
    const bool active = 16 * wave < mg.ncol;
    const int o0 = tk.o0, o1 = tk.o1;
    const int16_t* ol = olist + tk.cls * 189;
    int ol_reg = lane < o1 - o0 ? ol[o0 + lane] : 0;
    // parity class of the chunk's sources (every offset of the chunk has the
    // same parity)
    const int oi0 = __builtin_amdgcn_readlane(ol_reg, 0);
    const int q = tk.cls ^ ((((oi0 / 49 - 3) & 1) << 2) | ((((oi0 / 7) % 7 - 3) & 1) << 1) | ((oi0 % 7 - 3) & 1));
    auto issue = [&](int oc, uint4* dst) {
        const uint4* src = bank + (size_t)oc * a_chunks;
        for (int c0 = 0; c0 < a_chunks; c0 += kM2LThreads)
            if (c0 + tid < a_chunks) lds_dma16(src + c0 + tid, dst + c0 + 64 * wave);
    };
    // the first operator's copy, then the boxes of the target columns and of
    // the source rows (one per thread), then the source rows' copy
    if (o0 < o1) issue(o0, opb0);
    if (tid < kM2LTile) {
        int l, x, y, z;
        col_box[tid] = m2l_column(g, tk.cls, 0, tid, l, x, y, z) ? (int)(lev_offset(l) + morton(x, y, z)) : -1;
    } else if (tid < kM2LTile + nres) {
        const int j = tid - kM2LTile;
        int l, x, y, z;
        row_box[j] = (j < mg.ncol && m2l_column(g, q, 0, j, l, x, y, z)) ? (int)(lev_offset(l) + morton(x, y, z))
                                                                       : (int)g.nbox;
    }
    __syncthreads();
    // chunk e = t kM2LThreads + tid is chunk e % SBc of row e / SBc (the pad
    // chunk copies chunk 0 again)
    for (int e0 = 0; e0 < nres * SBc; e0 += kM2LThreads) {
        const int e = e0 + tid;
        if (e < nres * SBc) {
            const int j = e / SBc, c = e - j * SBc;
            lds_dma16(msplit + (size_t)row_box[j] * 2 * KC + (c == 2 * KC ? 0 : c), res + e0 + 64 * wave);
        }
    }
    // this lane's column and its place: source row = column index - u(t) + u(s)
    const int col = 16 * wave + (lane & 15), kq = lane >> 4, row = lane & 15;
    int clev = 0, ctx = 0, cty = 0, ctz = 0;
    const bool cok = m2l_column(g, tk.cls, 0, col, clev, ctx, cty, ctz);
    const int chalf = 1 << max(clev - 1, 0), cn = 1 << clev;
    const int cu = ((ctx >> 1) * chalf + (cty >> 1)) * chalf + (ctz >> 1);
    const int fx = (tk.cls & 4) ? -1 : 1, fy = (tk.cls & 2) ? -1 : 1, fz = (tk.cls & 1) ? -1 : 1;
    mf4 acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r] = mf4{0.f, 0.f, 0.f, 0.f};
    uint4 bsg[kM2LMaxKs];
#pragma unroll
    for (int si = 0; si < kM2LMaxKs; ++si) bsg[si] = sign_tab[tk.cls * 4 * kM2LMaxKs + 4 * si + kq];
    // one offset: wait for its operator (and, first, the source rows), start
    // the next operator's copy into the other buffer, multiply
    auto step = [&](int oc, const uint4* A, uint4* nxt) {
        const int st = oc - o0;
        if (st > 0 && (st & 63) == 0) ol_reg = ol[min(oc + lane, o1 - 1)];
        const int oi = __builtin_amdgcn_readlane(ol_reg, st & 63);
        __builtin_amdgcn_s_waitcnt(0);  // this lane's copies have landed
        __syncthreads();                // everyone's have; the other buffer is free
        if (oc + 1 < o1) issue(oc + 1, nxt);
        if (!active) return;
        int srow = mg.ncol;  // zero row
        if (cok) {
            int sx = ctx - fx * (oi / 49 - 3), sy = cty - fy * ((oi / 7) % 7 - 3), sz = ctz - fz * (oi % 7 - 3);
            bool ok = true;
            if (g.periodic) {
                sx &= cn - 1;
                sy &= cn - 1;
                sz &= cn - 1;
            } else {
                ok = sx >= 0 && sy >= 0 && sz >= 0 && sx < cn && sy < cn && sz < cn;
            }
            if (ok) srow = col - cu + ((sx >> 1) * chalf + (sy >> 1)) * chalf + (sz >> 1);
        }
        const uint4* B = res + (size_t)srow * SBc;
        // fragments of k-step si into registers: B (signed by the class's S)
        // and every row tile's A; the next k-step's are loaded while this
        // one's products run, which are issued by product over independent
        // accumulators (per accumulator still al bh, ah bl, ah bh in order)
        struct Frags {
            mbf8 bh, bl, ah[RT], al[RT];
        };
        auto load = [&](int si, Frags& f) {
            const int kc = 4 * si + kq;
            uint4 uh = B[kc], ul = B[KC + kc];
            uh.x ^= bsg[si].x;
            uh.y ^= bsg[si].y;
            uh.z ^= bsg[si].z;
            uh.w ^= bsg[si].w;
            ul.x ^= bsg[si].x;
            ul.y ^= bsg[si].y;
            ul.z ^= bsg[si].z;
            ul.w ^= bsg[si].w;
            f.bh = __builtin_bit_cast(mbf8, uh);
            f.bl = __builtin_bit_cast(mbf8, ul);
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                f.ah[r] = __builtin_bit_cast(mbf8, A[kc * RP + 16 * r + row]);
                f.al[r] = __builtin_bit_cast(mbf8, A[(KC + kc) * RP + 16 * r + row]);
            }
        };
        Frags fr[2];
        load(0, fr[0]);
#pragma unroll
        for (int si = 0; si < NKS; ++si) {
            if (si + 1 < NKS) load(si + 1, fr[(si + 1) & 1]);
            // keep the next k-step's reads ahead of this k-step's products
            __builtin_amdgcn_sched_barrier(0);
            const Frags& f = fr[si & 1];
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.al[r], f.bh, acc[r], 0, 0, 0);
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ah[r], f.bl, acc[r], 0, 0, 0);
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ah[r], f.bh, acc[r], 0, 0, 0);
        }
    };
    for (int oc = o0; oc < o1; oc += 2) {
        step(oc, opb0, opb1);
        if (oc + 1 < o1) step(oc + 1, opb1, opb0);
    }
    // signs S on the output rows, stored straight from the accumulators: lane
    // (col, kq) holds rows 16 r + 4 kq .. + 3 of its column, one 16-byte chunk
    // of the box row per row tile (four lanes of a column: 64 bytes in a row)
    const int box = cok ? col_box[col] : -1;
    if (active && box >= 0) {
        float* dst = mg.nchunk == 1
                         ? loc + (size_t)box * g.Kp
                         : part + ((size_t)tk.chunk * mg.nt_all + (box - lev_offset(g.lmin))) * g.Kp;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            if (16 * r + 4 * kq >= g.Kp) break;  // padding rows past the stored row length
            const uint4 m = sign_tab[tk.cls * 4 * kM2LMaxKs + 2 * r + (kq >> 1)];
            const uint32_t lo = (kq & 1) ? m.z : m.x, hi = (kq & 1) ? m.w : m.y;
            float4 o;
            o.x = ((lo >> 15) & 1u) ? -acc[r][0] : acc[r][0];
            o.y = ((lo >> 31) & 1u) ? -acc[r][1] : acc[r][1];
            o.z = ((hi >> 15) & 1u) ? -acc[r][2] : acc[r][2];
            o.w = ((hi >> 31) & 1u) ? -acc[r][3] : acc[r][3];
            *(float4*)(dst + 16 * r + 4 * kq) = o;
        }
    }
}

// Sum the offset-chunk partials into the local expansions (fixed chunk order).
// For periodic systems the launch carries one extra block per replica (the
// last, blockDim = kTreeThreads) that forms the root expansion (periodic_root),
// which then stays off the downward pass's critical path.
template <typename T>
__global__ __launch_bounds__(kTreeThreads) void k_m2l_reduce(
    Geo g, M2LGeom mg, const T* __restrict__ part_all, T* __restrict__ loc_all, int root_block,
    const T* __restrict__ mult_all, const T* __restrict__ m2m0, const T* __restrict__ m2m0_seg,
    const double* __restrict__ leaf_part_all, const double* __restrict__ box_part_all,
    const double* __restrict__ latT, const double* __restrict__ lat_seg, double* __restrict__ root_m_all,
    double* __restrict__ root_l_all, double* __restrict__ dom_all, const double* __restrict__ root_part_all) {
    const int nred = (int)gridDim.x - (root_block ? 1 : 0);
    if ((int)blockIdx.x >= nred) {
        __shared__ double xs[8 * kKMax], tp[8 * kTreeThreads], v[kKMax], ps[16];
        if (root_part_all)
            periodic_root_from_shares(g, blockIdx.y, root_part_all, box_part_all, latT, lat_seg, root_m_all,
                                      root_l_all, dom_all, xs, tp, v);
        else
            periodic_root<T>(g, blockIdx.y, mult_all, m2m0, m2m0_seg, leaf_part_all, box_part_all, latT,
                             lat_seg, root_m_all, root_l_all, dom_all, xs, tp, v, ps, true);
        return;
    }
    const int64_t tot = mg.nt_all * g.Kp;
    const T* part = part_all + (size_t)blockIdx.y * mg.nchunk * tot;
    T* loc = loc_all + (size_t)blockIdx.y * g.nbox * g.Kp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)nred * blockDim.x) {
        if ((int)(e % g.Kp) >= g.K) continue;
        loc[(size_t)g.lev_off[g.lmin] * g.Kp + e] = m2l_chunk_sum<T>(part, mg.nchunk, tot, e);
    }
}

// ------------------------------------------------------------------ downward pass

// ------------------------------------------------------------------ near + far field

template <typename T> __device__ __forceinline__ T inv_sqrt(T v);
// hardware reciprocal square root (about 1 ulp); pair distances squared are
// far from the denormal range, so no range scaling is needed
template <> __device__ __forceinline__ float inv_sqrt<float>(float v) { return __builtin_amdgcn_rsqf(v); }
template <> __device__ __forceinline__ double inv_sqrt<double>(double v) { return rsqrt(v); }


// Per target leaf (kNW wavefronts, one lane per target): the sources of the 27
// neighbour leaves (periodic images through integer leaf offsets) are staged
// through LDS in tiles of 64 kNW and split between the wavefronts.  The far
// field from the leaf's local expansion (L2P with its gradient) is split
// between the wavefronts by order m.  Wavefront 0 adds the per-wave partials in
// a fixed order, applies the periodic background term and writes potential,
// force, the per-leaf energy partial and (qB - qA) phi for the site sums.
template <typename T, int kNW>
__global__ __launch_bounds__(64 * kNW) void k_near_far(
    Geo g, int nsplit, const RepDesc* __restrict__ reps, const vec4_t<T>* __restrict__ pos,
    const int32_t* __restrict__ leaf_start_all, const int32_t* __restrict__ perm,
    const double* __restrict__ dom_all, const T* __restrict__ loc_all,
    const int32_t* __restrict__ gidx, const T* __restrict__ gcoef,
    const T* __restrict__ qA, const T* __restrict__ qB, const int32_t* __restrict__ site,
    T* __restrict__ phi_out, T* __restrict__ F_out,
    double* __restrict__ leaf_energy_all, double* __restrict__ cphi, int unit_dq,
    const int32_t* __restrict__ leaf_order_all, int32_t* __restrict__ status) {
    constexpr int NT = 64 * kNW;
    // sources staged per pass: the whole 27-leaf neighbourhood of a typical leaf
    constexpr int CAP = sizeof(T) == 4 ? 2048 : 1024;
    const int64_t n_sites = reps[blockIdx.y].S;
    const int32_t* leaf_start = leaf_start_all + (size_t)blockIdx.y * (g.nleaf + 1);
    const double* dom = dom_all + 8 * blockIdx.y;
    const T* loc = loc_all + (size_t)blockIdx.y * g.nbox * g.Kp;
    double* leaf_energy = leaf_energy_all + (size_t)blockIdx.y * g.nleaf * nsplit;
    __shared__ vec4_t<T> tile[CAP];
    __shared__ int nb_start[28], nb_cnt[28], nb_pre[29];
    __shared__ T nb_off[27][3];
    __shared__ T lam[kKMax];
    __shared__ T gr[3][kKgMax];
    __shared__ RhoLds<T> rho;
    load_rho_lds<T, 64 * kNW>(rho, g.p);
    __shared__ T part[kNW][4][64];
    __shared__ double esum_part[kNW][64];
    __shared__ int32_t t_idx[NT], t_site[NT];
    __shared__ double t_dq[NT];
    // block `sub` of the leaf takes targets 32 sub .. 32 sub + 31 (the last
    // block of the leaf all the rest); one block per leaf takes them all
    // leaves in the order given by leaf_work_order (largest first), if any
    const int lslot = blockIdx.x / nsplit, sub = blockIdx.x - lslot * nsplit;
    const int leaf = leaf_order_all ? leaf_order_all[(size_t)blockIdx.y * g.nleaf + lslot] : lslot;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lb = leaf_start[leaf], ln = leaf_start[leaf + 1] - lb;
    const int ta = 32 * sub;
    const int tb = lb + ta, tn = sub + 1 == nsplit ? ln - ta : min(32, ln - ta);
    if (tn <= 0) {
        if (tid == 0) leaf_energy[blockIdx.x] = 0.0;
        return;
    }
    const bool far = g.has_far;
    // loads issued up front, in flight with the neighbour set-up: the gradient
    // table entries of this thread and, for the first NT targets, the caller
    // index (their site and charges are loaded after the pair loop, which
    // hides that latency)
    const bool ge = far && tid < 3 * g.Kg;
    int32_t gi4[4];
    T gc4[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        gi4[t] = ge ? gidx[(size_t)tid * 4 + t] : -1;
        gc4[t] = ge ? gcoef[(size_t)tid * 4 + t] : T(0);
    }
    const bool tpre = tid < tn;
    const int32_t pre_i = tpre ? perm[tb + tid] : 0;
    const double edge = dom[3];
    const double h = edge / g.nb;
    int cx, cy, cz;
    unmorton((uint32_t)leaf, cx, cy, cz);
    int my_cnt = 0;
    if (tid < 27) {
        const int dx = tid / 9 - 1, dy = (tid / 3) % 3 - 1, dz = tid % 3 - 1;
        int nx = cx + dx, ny = cy + dy, nz = cz + dz;
        bool ok = true;
        if (g.periodic) {
            nx = (nx % g.nb + g.nb) % g.nb;
            ny = (ny % g.nb + g.nb) % g.nb;
            nz = (nz % g.nb + g.nb) % g.nb;
        } else {
            ok = nx >= 0 && ny >= 0 && nz >= 0 && nx < g.nb && ny < g.nb && nz < g.nb;
        }
        int s = 0, c = 0;
        if (ok) {
            const uint32_t m = morton(nx, ny, nz);
            s = leaf_start[m];
            c = leaf_start[m + 1] - s;
        }
        nb_start[tid] = s;
        nb_cnt[tid] = c;
        my_cnt = c;
        nb_off[tid][0] = (T)(dx * h);
        nb_off[tid][1] = (T)(dy * h);
        nb_off[tid][2] = (T)(dz * h);
    }
    if (wave == 0) {
        // inclusive scan of the 27 counts across lanes (in registers)
        const int v = wave_scan<int>(my_cnt);
        if (lane < 27) nb_pre[lane + 1] = v;
        if (lane == 0) {
            nb_pre[0] = 0;
            nb_pre[28] = 0x7fffffff;
        }
    }
    if (far) {
        const T* lsrc = loc + (size_t)(g.lev_off[g.depth] + leaf) * g.Kp;
        for (int k = tid; k < g.K; k += NT) lam[k] = lsrc[k];
    }
    __syncthreads();
    if (far) {
        if (ge) {
            T v = T(0);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (gi4[t] >= 0) v += gc4[t] * lam[gi4[t]];
            gr[tid / g.Kg][tid % g.Kg] = v;
        }
        for (int e = tid + NT; e < 3 * g.Kg; e += NT) {  // orders p > 13 only
            const int a = e / g.Kg, r = e % g.Kg;
            T v = T(0);
            for (int t = 0; t < 4; ++t) {
                const int kk = gidx[(size_t)e * 4 + t];
                if (kk >= 0) v += gcoef[(size_t)e * 4 + t] * lam[kk];
            }
            gr[a][r] = v;
        }
    }
    __syncthreads();
    const int total = nb_pre[27];
    const T ih = (T)(1.0 / h);
    double esum = 0.0;
    // Targets are processed in rounds of up to kNW chunks of 64.  A chunk of
    // tc targets runs on lane groups of gsz = pow2ceil(tc) lanes: the 64 / gsz
    // groups of a wavefront take interleaved sources and are added by
    // shuffles at the end, so a short chunk does not leave lanes idle.  The
    // kNW wavefronts are shared between the chunks in proportion to their
    // work (sources x gsz); each wavefront of a chunk takes a contiguous slice
    // of every source tile.
    __shared__ int w_first[kNW + 1];
    for (int t0 = 0; t0 < tn; t0 += 64 * kNW) {
        const int nch = min(kNW, (tn - t0 + 63) / 64);
        // every thread derives the same split (no barrier): w[c] wavefronts
        // for chunk c, each extra one to the largest gs / w (ties: lower c);
        // all indices are compile-time, so the arrays stay in registers
        int w[kNW], gs[kNW], wf[kNW + 1];
#pragma unroll
        for (int c = 0; c < kNW; ++c) {
            const int tc = min(64, tn - t0 - 64 * c);
            int gz = 1;
            while (gz < tc) gz <<= 1;
            gs[c] = gz;
            w[c] = c < nch ? 1 : 0;
        }
        for (int e = nch; e < kNW; ++e) {
            int best = 0, wb = w[0], gb = gs[0];
#pragma unroll
            for (int c = 1; c < kNW; ++c)
                if (c < nch && gs[c] * wb > gb * w[c]) {
                    best = c;
                    wb = w[c];
                    gb = gs[c];
                }
#pragma unroll
            for (int c = 0; c < kNW; ++c) w[c] += c == best ? 1 : 0;
        }
        wf[0] = 0;
#pragma unroll
        for (int c = 0; c < kNW; ++c) wf[c + 1] = wf[c] + w[c];
        int chunk = 0, wc0 = 0, wc1 = wf[1];
#pragma unroll
        for (int c = 1; c < kNW; ++c)
            if (c < nch && wf[c] <= wave) {
                chunk = c;
                wc0 = wf[c];
                wc1 = wf[c + 1];
            }
        const int wpc = wc1 - wc0, slice = wave - wc0;
        // kept for the energy sum at the end of the round (read after barriers)
        if (tid <= kNW) {
#pragma unroll
            for (int c = 0; c <= kNW; ++c)
                if (c == tid) w_first[c] = wf[c];
        }
        const int tc = min(64, tn - t0 - 64 * chunk);
        int gsz = 1;
        while (gsz < tc) gsz <<= 1;
        const int ngrp = 64 / gsz, grp = lane / gsz, tl = lane & (gsz - 1);
        const int tj = t0 + 64 * chunk + tl;
        const bool tv = tl < tc;
        vec4_t<T> me;
        if (tv) me = pos[tb + tj];
        else { me.x = me.y = me.z = me.w = T(0); }
        T ph = T(0), fx = T(0), fy = T(0), fz = T(0);
        for (int s0 = 0; s0 < total; s0 += CAP) {
            const int cnt = min(CAP, total - s0);
            if (t0 > 0 || s0 > 0) __syncthreads();  // the tile's previous readers are done
            if (total <= CAP) {
                // the whole neighbourhood in one pass: wavefront w copies
                // neighbours w, w + kNW, ..., lane j their atom j (all loads
                // in flight together), larger neighbours in extra rounds
                constexpr int J = (27 + kNW - 1) / kNW;
                vec4_t<T> a[J];
#pragma unroll
                for (int m = 0; m < J; ++m) {
                    const int nbk = min(wave + kNW * m, 26);
                    // an empty neighbour reads entry 0 (never stored)
                    const int c = nb_cnt[nbk];
                    a[m] = pos[c > 0 ? nb_start[nbk] + min(lane, c - 1) : 0];
                }
#pragma unroll
                for (int m = 0; m < J; ++m) {
                    const int nbk = wave + kNW * m;
                    if (nbk < 27 && lane < nb_cnt[nbk]) {
                        vec4_t<T> v = a[m];
                        v.x += nb_off[nbk][0];
                        v.y += nb_off[nbk][1];
                        v.z += nb_off[nbk][2];
                        tile[nb_pre[nbk] + lane] = v;
                    }
                }
                for (int nbk = wave; nbk < 27; nbk += kNW)
                    for (int j = 64 + lane; j < nb_cnt[nbk]; j += 64) {
                        vec4_t<T> v = pos[nb_start[nbk] + j];
                        v.x += nb_off[nbk][0];
                        v.y += nb_off[nbk][1];
                        v.z += nb_off[nbk][2];
                        tile[nb_pre[nbk] + j] = v;
                    }
            } else {
                // stage the pass's sources, CAP / NT loads in flight per thread
                constexpr int G = CAP / NT;
                vec4_t<T> a[G];
                int lo_[G];
#pragma unroll
                for (int m = 0; m < G; ++m) {
                    const int gsrc = s0 + min(tid + m * NT, cnt - 1);
                    // neighbour holding source gsrc: largest i with nb_pre[i] <= gsrc
                    int lo = 0, hi = 27;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (nb_pre[mid] <= gsrc) lo = mid;
                        else hi = mid;
                    }
                    lo_[m] = lo;
                    a[m] = pos[nb_start[lo] + (gsrc - nb_pre[lo])];
                }
#pragma unroll
                for (int m = 0; m < G; ++m) {
                    if (tid + m * NT < cnt) {
                        vec4_t<T> v = a[m];
                        v.x += nb_off[lo_[m]][0];
                        v.y += nb_off[lo_[m]][1];
                        v.z += nb_off[lo_[m]][2];
                        tile[tid + m * NT] = v;
                    }
                }
            }
            __syncthreads();
            const int sl = (cnt + wpc - 1) / wpc;
            const int jb = slice * sl;
            const int je = min(jb + sl, cnt);
            // Only the target's own leaf (neighbour 13, zero offset) can hold a
            // source at distance 0 (the target itself, or a duplicate position):
            // the r > 0 guard runs on that range alone.  Lane group grp takes
            // the sources jb + grp, jb + grp + ngrp, ...
            const int own_b = nb_pre[13] - s0, own_e = nb_pre[14] - s0;
            auto sweep = [&](int j0, int j1, auto guard) {
                const int first = j0 + ((grp - (j0 - jb)) & (ngrp - 1));
#pragma unroll 4
                for (int j = first; j < j1; j += ngrp) {
                    const vec4_t<T> s = tile[j];
                    const T dx = me.x - s.x, dy = me.y - s.y, dz = me.z - s.z;
                    const T r2 = dx * dx + dy * dy + dz * dz;
                    T ri;
                    if constexpr (decltype(guard)::value) ri = r2 > T(0) ? inv_sqrt<T>(r2) : T(0);
                    else ri = inv_sqrt<T>(r2);
                    const T qr = s.w * ri;
                    const T qr3 = qr * (ri * ri);
                    ph += qr;
                    fx += qr3 * dx;
                    fy += qr3 * dy;
                    fz += qr3 * dz;
                }
            };
            sweep(jb, min(je, own_b), std::false_type{});
            sweep(max(jb, own_b), min(je, own_e), std::true_type{});
            sweep(max(jb, own_e), je, std::false_type{});
            if (g.check && tv) {
                // check mode: a zero distance to any source of the own leaf
                // other than the target itself is a coincident pair
                const int self_j = nb_pre[13] + ta + tj - s0;
                const int j0 = max(jb, own_b), j1 = min(je, own_e);
                bool bad = false;
                for (int j = j0 + ((grp - (j0 - jb)) & (ngrp - 1)); j < j1; j += ngrp) {
                    const vec4_t<T> s = tile[j];
                    const T dx = me.x - s.x, dy = me.y - s.y, dz = me.z - s.z;
                    bad |= j != self_j && !(dx * dx + dy * dy + dz * dz > T(0));
                }
                if (bad) atomicOr(&status[0], kStatusCoincident);
            }
        }
        // sites and charges of the first NT targets (for the outputs), in
        // flight during the far-field evaluation
        int32_t pre_s = -1;
        double pre_dq = 0.0;
        if (t0 == 0 && tpre) {
            pre_s = site[pre_i];
            // site weight of phi: qB - qA (two forms), or 1 (four forms: the
            // site sums weight phi by the form coordinates themselves)
            pre_dq = unit_dq ? 1.0 : (double)qB[pre_i] - (double)qA[pre_i];
        }
        if (far && tv) {
            // far field, orders m = slice + wpc grp, stepping by wpc ngrp
            T fp = T(0), gx = T(0), gy = T(0), gz = T(0);
            const int Kg = g.Kg;
            for_rho_orders<T>(g.p, rho, slice + wpc * grp, wpc * ngrp, me.x * ih, me.y * ih, me.z * ih,
                              [&](int kc, bool has_s, T re, T im) {
                                  fp += lam[kc] * re;
                                  if (has_s) fp += lam[kc + 1] * im;
                                  if (kc < Kg) {
                                      gx += gr[0][kc] * re;
                                      gy += gr[1][kc] * re;
                                      gz += gr[2][kc] * re;
                                      if (has_s) {
                                          gx += gr[0][kc + 1] * im;
                                          gy += gr[1][kc + 1] * im;
                                          gz += gr[2][kc + 1] * im;
                                      }
                                  }
                              });
            ph += fp * ih;
            fx -= gx * ih * ih;
            fy -= gy * ih * ih;
            fz -= gz * ih * ih;
        }
        // add the lane groups (fixed butterfly order)
        for (int off = gsz; off < 64; off <<= 1) {
            ph += __shfl_xor(ph, off, 64);
            fx += __shfl_xor(fx, off, 64);
            fy += __shfl_xor(fy, off, 64);
            fz += __shfl_xor(fz, off, 64);
        }
        if (grp == 0) {
            part[wave][0][tl] = ph;
            part[wave][1][tl] = fx;
            part[wave][2][tl] = fy;
            part[wave][3][tl] = fz;
        }
        if (t0 == 0 && tpre) {
            t_idx[tid] = pre_i;
            t_site[tid] = pre_s;
            t_dq[tid] = pre_dq;
        }
        __syncthreads();
        // the first wavefront of each chunk adds the chunk's slices in order
        if (slice == 0 && grp == 0 && tv) {
            T p = T(0), ex = T(0), ey = T(0), ez = T(0);
            for (int w = wave; w < wave + wpc; ++w) {
                p += part[w][0][tl];
                ex += part[w][1][tl];
                ey += part[w][2][tl];
                ez += part[w][3][tl];
            }
            if (g.periodic) {
                // background: phi += (2 pi / 3) Q |t|^2 / V, field -= (4 pi / 3) Q t / V
                const double Q = dom[4];
                const double V = edge * edge * edge;
                const double t0v = (double)me.x + (cx + 0.5) * h - 0.5 * edge;
                const double t1v = (double)me.y + (cy + 0.5) * h - 0.5 * edge;
                const double t2v = (double)me.z + (cz + 0.5) * h - 0.5 * edge;
                p += (T)(2.0 * kPi / 3.0 * Q * (t0v * t0v + t1v * t1v + t2v * t2v) / V);
                ex -= (T)(4.0 * kPi / 3.0 * Q * t0v / V);
                ey -= (T)(4.0 * kPi / 3.0 * Q * t1v / V);
                ez -= (T)(4.0 * kPi / 3.0 * Q * t2v / V);
            }
            const bool pre = tj < NT;  // prefetched at the start
            const int32_t i = pre ? t_idx[tj] : perm[tb + tj];
            const T q = me.w;
            const T ke = (T)g.coulomb_k;
            if (phi_out) phi_out[i] = ke * p;
            if (F_out) {
                F_out[3 * (size_t)i] = ke * q * ex;
                F_out[3 * (size_t)i + 1] = ke * q * ey;
                F_out[3 * (size_t)i + 2] = ke * q * ez;
            }
            const double qp = (double)q * (double)p;
            esum_part[wave][lane] = qp;
            const int32_t st = pre ? t_site[tj] : site[i];
            if (st >= 0 && st < n_sites) {
                const double dq = pre ? t_dq[tj] : (unit_dq ? 1.0 : (double)qB[i] - (double)qA[i]);
                cphi[i] = g.coulomb_k * dq * (double)p;
            }
        } else if (slice == 0) {
            esum_part[wave][lane] = 0.0;
        }
        __syncthreads();
        // energy partial of this round, in target order
        if (wave == 0) {
            double v = 0.0;
            for (int c = 0; c < nch; ++c) v += esum_part[w_first[c]][lane];
            esum += v;
        }
    }
    if (wave == 0) {
        esum = wave_sum<double>(esum);
        if (lane == 0) leaf_energy[blockIdx.x] = esum;
    }
}

// Hamiltonian interpolation (Methods, eq 1) against the charge-interpolated
// energy, one block per site s (global index): eq 1 mixes each site's two end
// Hamiltonians linearly, and the Coulomb energy is a quadratic form in the
// charges, so the two interpolations differ by
//   dE_s = k_e lambda (1 - lambda) 1/2 sum_{i,j in s} d_i d_j psi(r_ij),  d = qA - qB,
// psi = 1/r (open; i != j) or the periodic Green's function of the cell
// (psi(0) = its self-image limit).  Writes dE_s and d(dE_s)/dlambda_s (hc_e,
// hc_dl; added by k_reduce) and adds -d(dE_s)/dr_i to F_i (each atom belongs
// to one site: no two blocks touch the same force).  Periodic psi of a cell of
// edge L at r: u = minimum image of r / L,
//   psi = (1/L) [sum_{n in {-1,0,1}^3} 1/|u + n| + (2 pi / 3)|u|^2 + h(u)],
// with h from its degree-kPMax harmonic coefficients (green) and grad h from
// the gradient coefficients that follow them.  All arithmetic is FP64.
constexpr int kHcorrThreads = 1024;  // threads of a correction block
template <typename T>
__global__ __launch_bounds__(kHcorrThreads) void k_hcorr(Geo g, int R, const RepDesc* __restrict__ reps,
                                               const int32_t* __restrict__ site_start,
                                               const int32_t* __restrict__ site_members,
                                               const T* __restrict__ x, const T* __restrict__ qA,
                                               const T* __restrict__ qB, const double* __restrict__ lam,
                                               const double* __restrict__ green, T* __restrict__ F,
                                               double* __restrict__ hc_e, double* __restrict__ hc_dl,
                                               int32_t* __restrict__ status) {
    constexpr int kH = kSiteCap / 4;  // atoms of a site staged in LDS
    constexpr int kHPair = 8;         // sites up to this size: pair tables (n^2 <= 64)
    constexpr int kHW = kHcorrThreads / 64;     // wavefronts: one harmonic order each
    __shared__ double pp[kHW][kHPair * kHPair][4];
    __shared__ int32_t mem[kSiteCap];
    __shared__ double sp[kH][4];  // x, y, z, d
    __shared__ double gc[kKMax + 3 * kKgMax];
    __shared__ RhoLds<double> rho;
    __shared__ double red[kHcorrThreads];
    const int s = blockIdx.x, t = threadIdx.x;
    int r = 0;
    while (r + 1 < R && s >= reps[r].s0 + reps[r].S) ++r;
    const double L = reps[r].box;
    const int m0 = site_start[s], n = site_start[s + 1] - m0;
    const double lm = lam[s], w = lm * (1.0 - lm);
    if (n > kH) {
        // sites are a few atoms; a site this large is reported and left alone
        if (t == 0) {
            atomicOr(&status[1], kInfoBigSite);
            hc_e[s] = 0.0;
            hc_dl[s] = 0.0;
        }
        return;
    }
    for (int i = t; i < n; i += kHcorrThreads) mem[i] = site_members[m0 + i];
    if (g.periodic) {
        for (int k = t; k < kKMax + 3 * kKgMax; k += kHcorrThreads) gc[k] = green[k];
        load_rho_lds<double, kHcorrThreads>(rho, kPMax);
    }
    __syncthreads();
    lds_sort<kSiteCap>(mem, n);  // caller order: a fixed summation order
    for (int i = t; i < n; i += kHcorrThreads) {
        const int32_t a = mem[i];
        sp[i][0] = (double)x[3 * (size_t)a];
        sp[i][1] = (double)x[3 * (size_t)a + 1];
        sp[i][2] = (double)x[3 * (size_t)a + 2];
        sp[i][3] = (double)qA[a] - (double)qB[a];
    }
    __syncthreads();
    // self-image limit of the unit cube: sum over the 26 neighbour images + h(0)
    const double psi0 = 6.0 + 12.0 / sqrt(2.0) + 8.0 / sqrt(3.0) + gc[0];
    double v = 0.0;
    if (n <= kHPair) {
        // sites of up to 8 atoms: lane q of every wavefront takes ordered
        // pair q (up to 64 pairs); wavefront w takes harmonic order w of h
        // and every 16th of the 27 direct images, so every lane of a
        // wavefront runs the same recurrence steps; the partial tables are
        // added in wavefront order
        const int np = n * n, wv = t >> 6, q = t & 63;
        const int i = q < np ? q / n : 0, j = q < np ? q - i * n : 0;
        double ps = 0.0, qx = 0.0, qy = 0.0, qz = 0.0;
        if (q < np && i != j) {
            const double rx = sp[i][0] - sp[j][0], ry = sp[i][1] - sp[j][1], rz = sp[i][2] - sp[j][2];
            if (!g.periodic) {
                if (wv == 0) {
                    const double r2 = rx * rx + ry * ry + rz * rz, ir = 1.0 / sqrt(r2);
                    const double ir3 = ir * ir * ir;
                    ps = ir;
                    qx = -rx * ir3;
                    qy = -ry * ir3;
                    qz = -rz * ir3;
                }
            } else {
                double u[3] = {rx / L, ry / L, rz / L};
                for (int c = 0; c < 3; ++c) u[c] -= rint(u[c]);
                if (wv == 0) {
                    ps = 2.0 * kPi / 3.0 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                    qx = 4.0 * kPi / 3.0 * u[0];
                    qy = 4.0 * kPi / 3.0 * u[1];
                    qz = 4.0 * kPi / 3.0 * u[2];
                }
                for (int im = wv; im < 27; im += kHW) {
                    const double vx = u[0] + (im / 9 - 1), vy = u[1] + ((im / 3) % 3 - 1),
                                 vz = u[2] + (im % 3 - 1);
                    const double r2 = vx * vx + vy * vy + vz * vz, ir = 1.0 / sqrt(r2);
                    const double ir3 = ir * ir * ir;
                    ps += ir;
                    qx -= vx * ir3;
                    qy -= vy * ir3;
                    qz -= vz * ir3;
                }
                const double* gh = gc + kKMax;
                for_rho_orders<double>(kPMax, rho, wv, kHW, u[0], u[1], u[2],
                                       [&](int kc, bool has_s, double re, double im_) {
                                           ps += gc[kc] * re;
                                           if (has_s) ps += gc[kc + 1] * im_;
                                           if (kc < kKgMax) {
                                               qx += gh[kc] * re;
                                               qy += gh[kKgMax + kc] * re;
                                               qz += gh[2 * kKgMax + kc] * re;
                                               if (has_s) {
                                                   qx += gh[kc + 1] * im_;
                                                   qy += gh[kKgMax + kc + 1] * im_;
                                                   qz += gh[2 * kKgMax + kc + 1] * im_;
                                               }
                                           }
                                       });
                ps /= L;
                qx /= L * L;
                qy /= L * L;
                qz /= L * L;
            }
        }
        if (q < np) {
            pp[wv][q][0] = ps;
            pp[wv][q][1] = qx;
            pp[wv][q][2] = qy;
            pp[wv][q][3] = qz;
        }
        __syncthreads();
        // table sums in wavefront order, one thread per (pair, component)
        double acc = 0.0;
        const int qc = t >> 2, cc = t & 3;
        if (qc < np)
            for (int w = 0; w < kHW; ++w) acc += pp[w][qc][cc];
        __syncthreads();
        if (qc < np) pp[0][qc][cc] = acc;
        __syncthreads();
    }
    for (int i = t; i < n; i += kHcorrThreads) {
        double e = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        for (int j = 0; j < n; ++j) {
            const double dj = sp[j][3];
            if (j == i) {
                if (g.periodic) e += dj * psi0 / L;
                continue;
            }
            if (n <= kHPair) {  // psi and its gradient from the pair tables
                const int q = i * n + j;
                e += dj * pp[0][q][0];
                gx += dj * pp[0][q][1];
                gy += dj * pp[0][q][2];
                gz += dj * pp[0][q][3];
                continue;
            }
            double rx = sp[i][0] - sp[j][0], ry = sp[i][1] - sp[j][1], rz = sp[i][2] - sp[j][2];
            double psi, px, py, pz;  // psi and its gradient with respect to r_i
            if (!g.periodic) {
                const double r2 = rx * rx + ry * ry + rz * rz, ir = 1.0 / sqrt(r2), ir3 = ir * ir * ir;
                psi = ir;
                px = -rx * ir3;
                py = -ry * ir3;
                pz = -rz * ir3;
            } else {
                double u[3] = {rx / L, ry / L, rz / L};
                for (int c = 0; c < 3; ++c) u[c] -= rint(u[c]);
                double ps = 2.0 * kPi / 3.0 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                double qx = 4.0 * kPi / 3.0 * u[0], qy = 4.0 * kPi / 3.0 * u[1], qz = 4.0 * kPi / 3.0 * u[2];
                for (int a = -1; a <= 1; ++a)
                    for (int b = -1; b <= 1; ++b)
                        for (int c = -1; c <= 1; ++c) {
                            const double vx = u[0] + a, vy = u[1] + b, vz = u[2] + c;
                            const double r2 = vx * vx + vy * vy + vz * vz, ir = 1.0 / sqrt(r2);
                            const double ir3 = ir * ir * ir;
                            ps += ir;
                            qx -= vx * ir3;
                            qy -= vy * ir3;
                            qz -= vz * ir3;
                        }
                const double* gh = gc + kKMax;
                for_each_rho<double>(kPMax, rho, u[0], u[1], u[2], [&](int kc, bool has_s, double re, double im) {
                    ps += gc[kc] * re;
                    if (has_s) ps += gc[kc + 1] * im;
                    if (kc < kKgMax) {
                        qx += gh[kc] * re;
                        qy += gh[kKgMax + kc] * re;
                        qz += gh[2 * kKgMax + kc] * re;
                        if (has_s) {
                            qx += gh[kc + 1] * im;
                            qy += gh[kKgMax + kc + 1] * im;
                            qz += gh[2 * kKgMax + kc + 1] * im;
                        }
                    }
                });
                psi = ps / L;
                px = qx / (L * L);
                py = qy / (L * L);
                pz = qz / (L * L);
            }
            e += dj * psi;
            gx += dj * px;
            gy += dj * py;
            gz += dj * pz;
        }
        const double di = sp[i][3];
        v += di * e;
        if (F) {
            const int32_t a = mem[i];
            const double f = -g.coulomb_k * w * di;
            F[3 * (size_t)a] += (T)(f * gx);
            F[3 * (size_t)a + 1] += (T)(f * gy);
            F[3 * (size_t)a + 2] += (T)(f * gz);
        }
    }
    red[t] = v;
    __syncthreads();
    for (int st = kHcorrThreads / 2; st > 0; st >>= 1) {
        if (t < st) red[t] += red[t + st];
        __syncthreads();
    }
    if (t == 0) {
        hc_e[s] = 0.5 * g.coulomb_k * w * red[0];
        hc_dl[s] = 0.5 * g.coulomb_k * (1.0 - 2.0 * lm) * red[0];
    }
}

// Final reductions: block r < R -> E_r = k_e / 2 sum of replica r's leaf
// partials (fixed order); block R + s -> dVdl_s = sum over global site s's
// atoms in caller order (four forms: dV/dlambda_p and dV/dlambda_t of site s;
// with cphi2, the adjoint's glam_s = sum of cphi2 over the same atoms).
// Also clears the evaluation's leaf and site counters.
template <typename T>
__global__ __launch_bounds__(256) void k_reduce(Geo g, int R, int64_t nparts,
                                                const double* __restrict__ leaf_energy,
                                                const int32_t* __restrict__ site_start,
                                                const int32_t* __restrict__ site_members,
                                                const double* __restrict__ cphi,
                                                double* __restrict__ E, double* __restrict__ dVdl,
                                                int32_t* __restrict__ status, const T* __restrict__ qA,
                                                const T* __restrict__ qB, const double* __restrict__ lam,
                                                FormArgs<T> fa, double* __restrict__ dVdl_t,
                                                const RepDesc* __restrict__ reps,
                                                const double* __restrict__ hc_e,
                                                const double* __restrict__ hc_dl,
                                                int32_t* __restrict__ leaf_count,
                                                int32_t* __restrict__ site_count,
                                                const double* __restrict__ excl_e, int excl_parts,
                                                const double* __restrict__ cphi2,
                                                double* __restrict__ glam, int32_t* __restrict__ ovf_n) {
    __shared__ double red[4], red_t[4];
    __shared__ int32_t mem[kSiteCap];
    const int t = threadIdx.x;
    const int b = blockIdx.x;
    // the leaf and site counters of this evaluation are spent: leave them
    // zero for the next one (the plan clears them once at creation)
    if (b < R) {
        for (int i = t; i < g.nleaf; i += 256) leaf_count[(size_t)b * g.nleaf + i] = 0;
        if (b == 0 && t == 0 && ovf_n) *ovf_n = 0;
    } else if (t == 0) {
        site_count[b - R] = 0;
    }
    const bool four = fa.qC != nullptr && b >= R;
    double v = 0.0, vt = 0.0;
    // four forms: cphi = k_e phi, and the two site derivatives (Methods, eq 2)
    // weight it by
    // dq/dlambda_p = lt~ (qC - qA) + lt (qD - qB), dq/dlambda_t = lp~ (qB - qA) + lp (qD - qC)
    auto add = [&](int32_t i) {
        if (!four) {
            v += cphi[i];
            if (cphi2) vt += cphi2[i];
            return;
        }
        const double lp = lam[b - R], lt = fa.lam_t[b - R];
        const double a0 = (double)qA[i], b0 = (double)qB[i], c0 = (double)fa.qC[i], d0 = (double)fa.qD[i];
        v += cphi[i] * ((1.0 - lt) * (c0 - a0) + lt * (d0 - b0));
        vt += cphi[i] * ((1.0 - lp) * (b0 - a0) + lp * (d0 - c0));
    };
    if (b < R) {
        for (int64_t i = t; i < nparts; i += 256) v += leaf_energy[(size_t)b * nparts + i];
        // bonded exclusions: the removed pair energies, same units
        if (excl_e)
            for (int i = t; i < excl_parts; i += 256) v += excl_e[(size_t)b * excl_parts + i];
    } else {
        const int s = b - R;
        const int m0 = site_start[s], n = site_start[s + 1] - m0;
        if (n <= kSiteCap) {
            for (int i = t; i < n; i += 256) mem[i] = site_members[m0 + i];
            __syncthreads();
            lds_sort<kSiteCap>(mem, n);
            for (int i = t; i < n; i += 256) add(mem[i]);
        } else {
            if (t == 0) atomicOr(&status[1], kInfoBigSite);
            for (int i = t; i < n; i += 256) add(site_members[m0 + i]);
        }
    }
    // fixed order: a DPP scan within each wavefront, then the four
    // wavefronts' sums in order (one barrier)
    v = wave_sum<double>(v);
    vt = wave_sum<double>(vt);
    if ((t & 63) == 0) {
        red[t >> 6] = v;
        red_t[t >> 6] = vt;
    }
    __syncthreads();
    if (t == 0) {
        red[0] = ((red[0] + red[1]) + red[2]) + red[3];
        red_t[0] = ((red_t[0] + red_t[1]) + red_t[2]) + red_t[3];
        if (b < R) {
            double e = 0.5 * g.coulomb_k * red[0];
            if (hc_e) {  // Hamiltonian interpolation: the replica's site corrections, in order
                const RepDesc rd = reps[b];
                for (int64_t q = 0; q < rd.S; ++q) e += hc_e[rd.s0 + q];
            }
            if (E) E[b] = e;
        } else {
            if (dVdl) dVdl[b - R] = red[0] + (hc_dl ? hc_dl[b - R] : 0.0);
            if (four && dVdl_t) dVdl_t[b - R] = red_t[0];
            if (glam) glam[b - R] = red_t[0];
        }
    }
}

// Adjoint of E for the upstream weights gE[r] (see fmm_eval_adjoint).
template <typename T>
__global__ __launch_bounds__(256) void k_adjoint(const RepDesc* __restrict__ reps,
                                                 const int32_t* __restrict__ site,
                                                 const double* __restrict__ lam,
                                                 const double* __restrict__ gE,
                                                 const T* __restrict__ F, const T* __restrict__ phi,
                                                 const double* __restrict__ dVdl,
                                                 T* __restrict__ gx, T* __restrict__ gqA,
                                                 T* __restrict__ gqB, double* __restrict__ glam) {
    const RepDesc rd = reps[blockIdx.y];
    const int64_t il = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const double w = gE[blockIdx.y];
    if (glam && il < rd.S) glam[rd.s0 + il] = w * dVdl[rd.s0 + il];
    if (il >= rd.n) return;
    const int64_t i = rd.a0 + il;
    if (gx) {
        gx[3 * i] = (T)(-w * (double)F[3 * i]);
        gx[3 * i + 1] = (T)(-w * (double)F[3 * i + 1]);
        gx[3 * i + 2] = (T)(-w * (double)F[3 * i + 2]);
    }
    const int32_t s = site[i];
    const double l = (s >= 0 && s < rd.S) ? lam[rd.s0 + s] : 0.0;
    const double p = (double)phi[i];
    if (gqA) gqA[i] = (T)(w * (1.0 - l) * p);
    if (gqB) gqB[i] = (T)(w * l * p);
}

}  // namespace fmmk
