// fmm_api.hip -- host side of the C ABI declared in include/fmmcph.h: plan
// creation (operator tables, workspace), argument validation and the ordered
// launch sequence of one evaluation on the plan's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "fmm_kernels.hip"
#include "exclusions.hip"
#include "adjoint.hip"
#include "fmmcph.h"
#include "operators.h"

using fmmk::Geo;

// Per-evaluation scratch of a plan: the buffers every evaluation rewrites
// (sorted particles, keys, counters, expansions, partial sums).  They live in
// one arena: the plan's own allocation, or (fmm_eval_noalloc) the library's
// static scratch array.
struct Workspace {
    void* pos = nullptr;
    int32_t *perm = nullptr, *key = nullptr, *rank = nullptr;
    int32_t *leaf_count = nullptr, *leaf_start = nullptr, *leaf_order = nullptr;
    int32_t *site_count = nullptr, *site_start = nullptr, *site_rank = nullptr,
            *site_members = nullptr;
    // leaf buckets of the binning (trees of at most kScanFuseCap leaves):
    // replicas x leaves x leaf_cap atom indices, the overflow list and its length
    int32_t *bucket = nullptr, *ovf = nullptr, *ovf_n = nullptr;
    int32_t ovf_cap = 0;  // entries of ovf
    // the leaves' M2M terms into their parents (FP64, K per leaf), when the
    // leaf kernel takes the first M2M step
    double* m2m_part = nullptr;
    void *mult = nullptr, *loc = nullptr;
    double *root_m = nullptr, *root_l = nullptr;
    double* root_part = nullptr;  // periodic: the 8 level-1 shares of the root multipole
    double* box_part = nullptr;   // per-box FP64 sums of q |t/L|^2 and q (upward pass)
    double *dom = nullptr, *bbox_part = nullptr, *leaf_part = nullptr, *leaf_energy = nullptr,
           *cphi = nullptr;
    fmmk::RepDesc* reps = nullptr;  // device replica descriptors
    void *F_tmp = nullptr, *phi_tmp = nullptr;
    double *dVdl_tmp = nullptr, *E_tmp = nullptr;
    // adjoint with weights on E, phi and F: the second sources (w, g) in leaf
    // order, the per-atom (phi, E, A, B) of the leaf pass, the site terms of
    // dL/dq and the energy partials of the combine kernel
    void *adj_src2 = nullptr, *adj_acc = nullptr;
    double *adj_cphi2 = nullptr, *adj_part = nullptr;
    // Hamiltonian interpolation: per-site energy and lambda-derivative corrections
    double *hc_e = nullptr, *hc_dl = nullptr;
    void* msplit = nullptr;    // bf16x3: source expansions split into hi/lo (replicas x (nbox + 1) rows)
    void* m2l_part = nullptr;  // matrix-core M2L: partial sums of the offset chunks
};

struct fmm_plan_s {
    fmm_params prm{};
    hipStream_t stream = nullptr;
    int device = 0;
    bool fp64 = true;
    size_t tsz = 8;  // bytes of the working real type
    int K = 0, Kp = 0, Kg = 0, nleaf = 0;
    int64_t nbox = 0;
    int64_t lev_off[fmmk::kDMax + 2] = {};
    Workspace ws;
    void* ws_arena = nullptr;  // the plan's own workspace allocation
    // operator tables (device)
    void *bankT = nullptr, *m2mT = nullptr, *l2lT = nullptr, *gcoef = nullptr;
    void *m2m_seg = nullptr, *l2l_seg = nullptr;  // tree-pass register caches (thread order)
    double* lat_seg = nullptr;
    double* latT = nullptr;
    int32_t* gidx = nullptr;
    int32_t* status = nullptr;
    // Hamiltonian interpolation (periodic): the Green's function coefficients of
    // the unit cube (degree kPMax) followed by those of its gradient (3 x kPMax^2)
    double* green = nullptr;
    // bonded exclusions (fmm_set_exclusions): per-atom partner lists for
    // excl_n atoms and the per-block energy partials of their removal
    int64_t excl_n = 0;
    int32_t *excl_start = nullptr, *excl_idx = nullptr;
    double* excl_e = nullptr;
    // graph replay (params.graph): the last captured evaluation and its argument key
    bool graph_valid = false;
    std::vector<unsigned char> graph_key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int R_max = 1;
    int leaf_cap = 0;  // leaf bucket capacity (0: binning by scan and scatter)
    // matrix-core M2L
    int p2p_waves = 8;  // wavefronts per near-field block (4, 8 or 16)
    int p2p_split = 1;  // near-field blocks per leaf (1 to 4)
    int m2l_mode = 0;  // 0 plain, 1 f32, 2 f64, 3 bf16x3
    fmmk::M2LGeom mg{};
    int m2l_rt = 0;
    size_t m2l_lds = 0;
    int64_t n_tasks = 0;
    fmmk::M2LTask* tasks = nullptr;
    int16_t* olist = nullptr;
    int16_t* cstart = nullptr;
    void *bank_mma = nullptr;
    void* sign_tab = nullptr;  // bf16x3: reflection sign-bit masks [class][k chunk of 8]
    int m2l_nbuf = 1;        // bf16x3: LDS staging buffers (2: copy of the next offset overlaps)
    bool m2l_rs = false;     // bf16x3 with resident sources (one tile per class, parity-group chunks)
    std::vector<void*> allocs;
    size_t ws_bytes = 0;
    std::string err;
    // per-phase timing (fmm_profile): events recorded at phase boundaries
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;
    std::vector<int> prof_phase;  // phase that starts at the event with the same index
    size_t prof_used = 0;
    uint32_t prof_mask = 0xffffffffu;  // phases whose boundaries get events
    int prof_every = 1;                // events on every prof_every-th evaluation
    int64_t prof_evals = 0;
    bool prof_sample = false, prof_open = false;
};

// Static scratch of fmm_eval_noalloc, for callers that cannot allocate
// device memory: the per-evaluation workspace is laid out in this array
// instead of the plan's own.  Every GPU the library runs on holds one copy
// until the process ends; calls that overlap on one GPU share it and race.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kBboxBlocks = 256;

// Device address of each GPU's copy of `scratch`, looked up once per device
// with that device current (plan creation); host code uses only these
// addresses, never the array's name.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

bool scratch_lookup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return false;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return true;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return false;
    g_scratch_ptr[dev] = ptr;
    return true;
}

void* scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[dev];
}

fmm_status fail(fmm_plan_t p, fmm_status st, const std::string& msg) {
    if (p) p->err = msg;
    return st;
}

// A view of the host replica descriptors of one call (a vector or an array on
// the stack).
struct RepSpan {
    const fmmk::RepDesc* p;
    size_t n;
    RepSpan(const std::vector<fmmk::RepDesc>& v) : p(v.data()), n(v.size()) {}
    RepSpan(const fmmk::RepDesc* q, size_t m) : p(q), n(m) {}
    size_t size() const { return n; }
    const fmmk::RepDesc& operator[](size_t i) const { return p[i]; }
    const fmmk::RepDesc* begin() const { return p; }
    const fmmk::RepDesc* end() const { return p + n; }
};

// Bytes of the bf16x3 split source rows: (nbox + 1) rows of 2 KP bf16 per slot.
size_t msplit_bytes(const fmm_plan_s* P, size_t RM) {
    return RM * ((size_t)P->nbox + 1) * 2 * P->mg.KP * 2;
}

bool dev_alloc(fmm_plan_t p, void** ptr, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (hipMalloc(ptr, bytes) != hipSuccess) return false;
    p->allocs.push_back(*ptr);
    p->ws_bytes += bytes;
    return true;
}

// Reflection parity bits of real coefficient k (bit 2: x -> -x, bit 1:
// y -> -y, bit 0: z -> -z), as the kernels' refl_bits.
// Lay out a plan's per-evaluation buffers for up to N atoms, S sites and RM
// expansion slots (adjoint: with the adjoint's buffers) from base, each
// buffer aligned to 256 bytes; returns the arena size.  base = NULL only
// sizes it.  The matrix-core M2L geometry (mg, m2l_mode) must be set.
size_t ws_layout(const fmm_plan_s* P, int64_t N, int64_t S, size_t RM, bool adjoint, char* base,
                 Workspace* w) {
    N = std::max<int64_t>(N, 1);
    S = std::max<int64_t>(S, 1);
    Workspace tmp;
    if (!w) w = &tmp;
    size_t off = 0;
    auto take = [&](auto*& ptr, size_t bytes) {
        using PT = std::remove_reference_t<decltype(ptr)>;
        ptr = base ? reinterpret_cast<PT>(base + off) : nullptr;
        off += (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
    };
    const size_t ts = P->tsz, K = P->K, nl = P->nleaf, nb = P->nbox, Kp = P->Kp;
    take(w->pos, N * 4 * ts);
    take(w->perm, N * 4);
    take(w->key, N * 4);
    take(w->rank, N * 4);
    take(w->leaf_count, RM * nl * 4);
    take(w->leaf_start, RM * (nl + 1) * 4);
    take(w->leaf_order, RM * nl * 4);
    take(w->site_count, S * 4);
    take(w->site_start, (S + 1) * 4);
    take(w->site_rank, N * 4);
    take(w->site_members, N * 4);
    if (P->leaf_cap > 0) {
        take(w->bucket, RM * nl * (size_t)P->leaf_cap * 4);
        take(w->ovf, N * 4);
        take(w->ovf_n, 4);
        w->ovf_cap = (int32_t)N;
    } else {
        w->bucket = w->ovf = w->ovf_n = nullptr;
    }
    take(w->mult, RM * nb * Kp * ts);
    if (P->prm.depth - 2 >= (P->prm.boundary == FMM_PERIODIC ? 1 : 2) && nl <= (size_t)fmmk::kScanFuseCap)
        take(w->m2m_part, RM * nl * K * 8);
    else w->m2m_part = nullptr;
    take(w->loc, RM * nb * Kp * ts);
    take(w->root_m, RM * K * 8);
    take(w->root_l, RM * K * 8);
    take(w->root_part, RM * 8 * K * 8);
    take(w->dom, RM * 8 * 8);
    take(w->bbox_part, RM * kBboxBlocks * 6 * 8);
    take(w->leaf_part, RM * nl * 2 * 8);
    take(w->box_part, RM * nb * 2 * 8);
    take(w->leaf_energy, RM * nl * fmmk::kMaxSplit * 8);
    take(w->reps, RM * sizeof(fmmk::RepDesc));
    take(w->cphi, N * 8);
    take(w->F_tmp, N * 3 * ts);
    take(w->phi_tmp, N * ts);
    take(w->dVdl_tmp, S * 8);
    take(w->E_tmp, RM * 8);
    if (adjoint) {
        take(w->adj_src2, N * 4 * ts);
        take(w->adj_acc, N * 8 * ts);
        take(w->adj_cphi2, N * 8);
        take(w->adj_part, ((N + 255) / 256) * 8);
    } else {
        w->adj_src2 = w->adj_acc = nullptr;
        w->adj_cphi2 = w->adj_part = nullptr;
    }
    if (P->prm.hamiltonian) {
        take(w->hc_e, S * 8);
        take(w->hc_dl, S * 8);
    } else {
        w->hc_e = w->hc_dl = nullptr;
    }
    if (P->m2l_mode == 3) take(w->msplit, msplit_bytes(P, RM));
    else w->msplit = nullptr;
    if (P->m2l_mode != 0 && P->mg.nchunk > 1)
        take(w->m2l_part, RM * P->mg.nchunk * P->mg.nt_all * Kp * ts);
    else w->m2l_part = nullptr;
    return off;
}

int refl_bits_host(int k) {
    const int l = (int)std::floor(std::sqrt((double)k + 0.5));
    const int rem = k - l * l;
    const int m = (rem + 1) >> 1;
    const int sn = (rem > 0 && !(rem & 1)) ? 1 : 0;
    const int xo = sn ? !(m & 1) : (m & 1);
    return (xo << 2) | (sn << 1) | ((l + m) & 1);
}

// Pack a K x K row-major operator in the tree kernels' thread order: entry j
// of thread t (row r, k range [kb, ke) of its segment, as the kernels derive
// it) at j kTreeThreads + t, zero past the range.
template <typename T>
std::vector<T> pack_tri(const double* A, int K, int shape) {
    using namespace fmmk;
    std::vector<T> out((size_t)kTriCache * kTreeThreads, T(0));
    const int nseg = tri_nseg(K), slen = (K + nseg - 1) / nseg;
    for (int it = 0; it < nseg * K && it < kTreeThreads; ++it) {
        const int s = it / K, r = it % K;
        const int l = (int)std::floor(std::sqrt((double)r + 0.5));
        const int kb = std::max(s * slen, shape == kTriUpper ? l * l : 0);
        const int ke = std::min(std::min(K, (s + 1) * slen), shape == kTriLower ? (l + 1) * (l + 1) : K);
        for (int j = 0; j < kTriCache && kb + j < ke; ++j)
            out[(size_t)j * kTreeThreads + it] = (T)A[(size_t)r * K + kb + j];
    }
    return out;
}

template <typename T>
std::vector<T> transpose_blocks(const std::vector<double>& src, int nblk, int K) {
    std::vector<T> out(src.size());
    for (int b = 0; b < nblk; ++b)
        for (int r = 0; r < K; ++r)
            for (int k = 0; k < K; ++k)
                out[(size_t)b * K * K + (size_t)k * K + r] = (T)src[(size_t)b * K * K + (size_t)r * K + k];
    return out;
}

void init_rho_coef() {
    fmmk::RhoCoef rc{};
    const int P = fmmk::kPMax;
    rc.f[0] = 1.0;
    for (int m = 1; m <= P; ++m) rc.f[m] = -std::sqrt((2.0 * m - 1) / (2.0 * m));
    for (int m = 0; m <= P; ++m) {
        if (m + 1 <= P) rc.a[(m + 1) * (P + 1) + m] = std::sqrt(2.0 * m + 1);
        for (int l = m + 2; l <= P; ++l) {
            rc.a[l * (P + 1) + m] = (2.0 * l - 1) / std::sqrt(double((l + m) * (l - m)));
            rc.b[l * (P + 1) + m] =
                std::sqrt(double((l + m - 1) * (l - m - 1)) / double((l + m) * (l - m)));
        }
    }
    (void)hipMemcpyToSymbol(HIP_SYMBOL(fmmk::c_rho), &rc, sizeof(rc));
}

// Offset list of every child class: o = t - s for the children s of the
// parent's 27 neighbours that are not adjacent to t, in a fixed order.
std::vector<int16_t> class_offsets() {
    std::vector<int16_t> out;
    for (int c = 0; c < 8; ++c) {
        const int tb[3] = {(c >> 2) & 1, (c >> 1) & 1, c & 1};
        int cnt = 0;
        for (int nb = 0; nb < 216; ++nb) {
            const int dp[3] = {nb / 72 - 1, (nb / 24) % 3 - 1, (nb / 8) % 3 - 1};
            const int cb[3] = {(nb >> 2) & 1, (nb >> 1) & 1, nb & 1};
            int o[3];
            for (int a = 0; a < 3; ++a) o[a] = tb[a] - 2 * dp[a] - cb[a];
            if (std::abs(o[0]) <= 1 && std::abs(o[1]) <= 1 && std::abs(o[2]) <= 1) continue;
            out.push_back((int16_t)(((o[0] + 3) * 7 + (o[1] + 3)) * 7 + (o[2] + 3)));
            ++cnt;
        }
        if (cnt != 189) return {};
    }
    return out;
}

uint16_t to_bf16(float f) {  // round to nearest even
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float from_bf16(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// LDS row stride (elements) of a matrix-core operand: f32 rows are padded to
// 2 mod 32 words (16-lane groups reading 4 consecutive k hit distinct banks),
// f64 rows to an odd number of elements, bf16 rows to 8 mod 64 elements.
int lds_stride(int mode, int kp) {
    if (mode == 1) { int s = kp; while (s % 32 != 2) ++s; return s; }
    if (mode == 2) return kp + 2;  // even: 16-byte aligned rows
    int s = kp; while (s % 64 != 40 && s % 64 != 8) s += 8; return s;
}

Geo make_geo(const fmm_plan_s* p) {
    Geo g{};
    g.depth = p->prm.depth;
    g.nb = 1 << g.depth;
    g.p = p->prm.order_p;
    g.K = p->K;
    g.Kp = p->Kp;
    g.Kg = p->Kg;
    g.nleaf = p->nleaf;
    g.periodic = p->prm.boundary == FMM_PERIODIC;
    g.lmin = g.periodic ? 1 : 2;
    g.has_far = g.periodic ? 1 : (g.depth >= 2 ? 1 : 0);
    g.check = p->prm.check;
    g.coulomb_k = p->prm.coulomb_k;
    g.nbox = p->nbox;
    for (int l = 0; l <= fmmk::kDMax + 1; ++l) g.lev_off[l] = p->lev_off[l];
    return g;
}

// Record a phase boundary: the event marks the start of `phase` (and the end of
// the previous one); phase -1 closes the evaluation.
// Only the boundaries of the selected phases are recorded (an event opens a
// selected phase; the next mark closes it), on every prof_every-th evaluation.
void mark(fmm_plan_t P, int phase) {
    if (!P->prof_on) return;
    if (phase == 0) {
        P->prof_sample = (P->prof_evals++ % P->prof_every) == 0;
        P->prof_open = false;
    }
    if (!P->prof_sample) return;
    const bool sel = phase >= 0 && ((P->prof_mask >> phase) & 1u);
    if (!sel && !P->prof_open) return;
    if (P->prof_used >= P->prof_ev.size()) return;
    (void)hipEventRecord(P->prof_ev[P->prof_used], P->stream);
    P->prof_phase[P->prof_used] = sel ? phase : -1;
    ++P->prof_used;
    P->prof_open = sel;
}

// Dynamic LDS of the leaf kernel: the sort buffer, later the P2M rows.
template <typename T>
size_t leaf_lds_bytes(int K) {
    return (size_t)fmmk::leaf_lds_base(K, (int)sizeof(T));
}
// ... and its largest form: bucket binning with kScanFuseCap sites
template <typename T>
size_t leaf_lds_bytes_max(int K) {
    return leaf_lds_bytes<T>(K) + (size_t)(256 + fmmk::kScanFuseCap + 1) * 4;
}

// Dynamic LDS of the second-source leaf kernel of the adjoint: the P2M rows.
template <typename T>
size_t src2_lds_bytes(int K) {
    return (size_t)64 * (K + 1) * sizeof(T);
}

inline unsigned nblocks(int64_t n, int b) { return (unsigned)std::max<int64_t>(1, (n + b - 1) / b); }

// The resident-source bf16x3 M2L for a row-tile count whose static staging
// fits the LDS (up to 7 row tiles: p <= 9).
template <int RTV>
void launch_m2l_rs(fmm_plan_t P, const Geo& g, const fmmk::M2LGeom& mg, dim3 nt, float* loc, float* part,
                   bool root) {
    if constexpr (RTV <= fmmk::kM2LRsMaxRT) {
        // with root: one extra work-group per replica forms the periodic root
        const fmmk::RootArgs ra{P->ws.root_part, P->ws.box_part, P->latT, P->lat_seg,
                                P->ws.root_m, root ? P->ws.root_l : nullptr, P->ws.dom};
        const dim3 grid(nt.x + (root ? 1u : 0u), nt.y);
        fmmk::k_m2l_bf16x3_rs<RTV><<<grid, fmmk::kM2LThreads, 0, P->stream>>>(
            g, mg, P->tasks, P->olist, (const uint4*)P->ws.msplit, (const uint4*)P->bank_mma,
            (const uint4*)P->sign_tab, loc, part, ra);
    }
}

// Matrix-core M2L launch: the kernel instance for the plan's precision and row
// tile count, then the fixed-order chunk reduction.  Returns whether the
// periodic root was formed (by the reduction launch or, with resident sources,
// by the M2L launch itself); *fused is set when no reduction launch ran and
// the downward pass adds the offset-chunk partials itself.
template <typename T>
bool launch_m2l_mma(fmm_plan_t P, const Geo& g, int R, bool want_root, bool* fused) {
    *fused = false;
    using namespace fmmk;
    hipStream_t st = P->stream;
    const M2LGeom mg = P->mg;
    const dim3 nt((unsigned)P->n_tasks, (unsigned)R);
    const size_t lds = P->m2l_lds;
    T* loc = (T*)P->ws.loc;
    T* part = (T*)P->ws.m2l_part;
    const T* mult = (const T*)P->ws.mult;
    // resident sources with offset chunks: the root (periodic trees of depth >= 2,
    // whose level-1 M2M leaves the root shares) in an extra M2L work-group and
    // the chunk sums in the downward pass, so no reduction launch
    // (only where a downward launch follows: it forms every leaf's expansion)
    const bool rs_fused = P->m2l_rs && mg.nchunk > 1 && (!g.periodic || (want_root && g.depth >= 2)) &&
                          g.depth - 1 >= (g.periodic ? 0 : g.lmin);
    switch (P->m2l_mode * 16 + P->m2l_rt) {
#define FMM_M2L_F32(RTV)                                                                    \
    case 16 + RTV:                                                                          \
        k_m2l_f32<RTV><<<nt, 64 * kM2LWaves, lds, st>>>(g, mg, P->tasks, P->olist, P->cstart, (const float*)mult, \
                                             (const float*)P->bank_mma, (float*)loc,         \
                                             (float*)part);                                  \
        break;
#define FMM_M2L_F64(RTV)                                                                      \
    case 32 + RTV:                                                                            \
        k_m2l_f64<RTV><<<nt, 64 * kM2LWaves, lds, st>>>(g, mg, P->tasks, P->olist, P->cstart, (const double*)mult, \
                                             (const double*)P->bank_mma, (double*)loc,         \
                                             (double*)part);                                   \
        break;
#define FMM_M2L_BF(RTV)                                                                         \
    case 48 + RTV:                                                                              \
        if (P->m2l_rs)                                                                          \
            launch_m2l_rs<RTV>(P, g, mg, nt, (float*)loc, (float*)part, rs_fused && want_root);  \
        else                                                                                    \
            k_m2l_bf16x3<RTV><<<nt, kM2LThreads, lds, st>>>(g, mg, P->tasks, P->olist, P->cstart, \
                                                (const uint4*)P->ws.msplit,                        \
                                                (const uint4*)P->bank_mma, P->m2l_nbuf,         \
                                                (const uint4*)P->sign_tab, (float*)loc,         \
                                                (float*)part);                                  \
        break;
        FMM_M2L_F32(1) FMM_M2L_F32(2) FMM_M2L_F32(3) FMM_M2L_F32(4)
        FMM_M2L_F32(5) FMM_M2L_F32(6) FMM_M2L_F32(7) FMM_M2L_F32(8)
        FMM_M2L_F64(1) FMM_M2L_F64(2) FMM_M2L_F64(3) FMM_M2L_F64(4)
        FMM_M2L_F64(5) FMM_M2L_F64(6)
        FMM_M2L_BF(1) FMM_M2L_BF(2) FMM_M2L_BF(3) FMM_M2L_BF(4)
        FMM_M2L_BF(5) FMM_M2L_BF(6) FMM_M2L_BF(7) FMM_M2L_BF(8)
        default: break;
    }
    if (rs_fused) {
        *fused = true;
        return g.periodic;
    }
    if (mg.nchunk > 1) {
        const int64_t tot = mg.nt_all * g.Kp;
        const unsigned nb = (unsigned)std::min<int64_t>(4096, (tot + 255) / 256);
        // periodic trees with a downward pass: the extra block forms the root
        k_m2l_reduce<T><<<dim3(nb + (want_root ? 1u : 0u), (unsigned)R), kTreeThreads, 0, st>>>(
            g, mg, part, loc, want_root ? 1 : 0, mult, (const T*)P->m2mT, (const T*)P->m2m_seg,
            P->ws.leaf_part, P->ws.box_part, P->latT, P->lat_seg, P->ws.root_m, P->ws.root_l, P->ws.dom,
            g.depth >= 2 ? P->ws.root_part : nullptr);
        return want_root;
    }
    return false;
}

// Binning and leaf multipoles of R replicas (grid y = replica): replica
// descriptors, the open bounding cube, leaf keys, the counting sort and the
// leaf kernel (sort in leaf, gather with the interpolated charges, P2M).
// nstore replica descriptors are stored (nstore >= R: extra slots describe
// the same systems for kernels run on more expansion slots later).
template <typename T>
void enqueue_bin_p2m(fmm_plan_t P, const fmmk::Geo& g, RepSpan rd, int R,
                     const T* x, const T* qA, const T* qB, const int32_t* site, const double* lam,
                     const fmmk::FormArgs<T>& fa, int64_t maxn, int64_t S_tot, bool fold) {
    using namespace fmmk;
    hipStream_t st = P->stream;
    const int nstore = (int)rd.size();
    // replica descriptors: by value to the first kernel (which stores them)
    // when they fit one set, else stored by k_set_reps launches first.  The
    // leaf and site counters are already zero (plan creation, then the final
    // reduction of every evaluation).
    RepSet set0{};
    if (nstore <= kRepsPerSet) {
        set0.first = 0;
        set0.count = nstore;
        for (int i = 0; i < nstore; ++i) set0.d[i] = rd[i];
    } else {
        for (int f = 0; f < nstore; f += kRepsPerSet) {
            RepSet set{};
            set.first = f;
            set.count = std::min(kRepsPerSet, nstore - f);
            for (int i = 0; i < set.count; ++i) set.d[i] = rd[f + i];
            k_set_reps<<<1, kRepsPerSet, 0, st>>>(set, P->ws.reps);
        }
    }
    const RepDesc* reps = P->ws.reps;
    const unsigned ab = nblocks(maxn, 256);
    if (!g.periodic) {
        const int nb = (int)std::min<int64_t>(kBboxBlocks, ab);
        k_bbox<T><<<dim3(nb, R), 256, 0, st>>>(x, set0, P->ws.reps, P->ws.bbox_part);
        k_bbox_final<<<R, 64, 0, st>>>(P->ws.bbox_part, nb, P->ws.dom);
        set0.count = 0;  // stored by k_bbox
    }
    // bucket binning: the leaf kernel finds each leaf's atoms in its bucket and
    // forms the leaf and site starts itself (no scan or scatter launch)
    const bool binned = P->ws.bucket && g.nleaf <= kScanFuseCap && S_tot <= kScanFuseCap;
    const Bins bins{binned ? P->ws.bucket : nullptr, P->leaf_cap, P->ws.ovf, P->ws.ovf_n, P->ws.ovf_cap};
    k_charge_key<T><<<dim3(ab, R), 256, 0, st>>>(g, set0, P->ws.reps, x, qA, qB, site, lam, fa, P->ws.dom, P->ws.key,
                                                 P->ws.rank, P->ws.leaf_count, P->ws.site_count,
                                                 P->ws.site_rank, P->status, bins);
    if (binned) {
        // nothing between the key and leaf launches
    } else if (g.nleaf <= kScanFuseCap && S_tot <= kScanFuseCap) {
        k_scan_scatter<<<dim3(ab, R), 256, 0, st>>>(g, reps, P->ws.key, P->ws.rank, P->ws.leaf_count,
                                                    P->ws.leaf_start, P->ws.perm, site, P->ws.site_rank,
                                                    P->ws.site_count, P->ws.site_start, (int)S_tot,
                                                    P->ws.site_members);
    } else {
        k_scan2<<<R + 1, 1024, 0, st>>>(reps, R, P->ws.leaf_count, P->ws.leaf_start, g.nleaf,
                                        P->ws.site_count, P->ws.site_start, S_tot);
        k_scatter<<<dim3(ab, R), 256, 0, st>>>(g, reps, P->ws.key, P->ws.rank, P->ws.leaf_start, P->ws.perm,
                                               site, P->ws.site_rank, P->ws.site_start, P->ws.site_members);
    }
    using V4 = vec4_t<T>;
    mark(P, 1);
    const LeafBinArgs lb{P->ws.leaf_count, P->ws.key,          P->ws.rank,         P->ws.site_count,
                         P->ws.site_rank,  P->ws.site_start,   P->ws.site_members, (int)S_tot};
    const size_t lds = leaf_lds_bytes<T>(g.K) + (binned && S_tot > 0 ? (size_t)(256 + S_tot + 1) * 4 : 0);
    // the folded first M2M step is its own instantiation (it needs more
    // registers, which would lower every other launch's occupancy)
    auto leaf = fold ? k_leaf_p2m<T, true> : k_leaf_p2m<T, false>;
    leaf<<<dim3(g.nleaf, R), kLeafThreads, lds, st>>>(
        g, reps, x, qA, qB, site, lam, fa, P->ws.dom, P->ws.leaf_start, P->ws.perm, (V4*)P->ws.pos, P->status,
        (T*)P->ws.mult, P->ws.leaf_part, (uint16_t*)P->ws.msplit, P->mg.KP, bins, lb, (const T*)P->m2mT,
        (const T*)P->m2m_seg, fold ? P->ws.m2m_part : nullptr);
}

// The tree passes of R expansion slots (grid y = slot): M2M per level, the
// periodic root with its lattice operator, M2L at every level and the
// downward pass into the leaves.  With want_order the downward launch's extra
// block orders the leaves for the near field; returns that order (or null).
template <typename T>
int32_t* enqueue_tree(fmm_plan_t P, const fmmk::Geo& g, int R, bool want_order, bool folded) {
    using namespace fmmk;
    hipStream_t st = P->stream;
    T* mult = (T*)P->ws.mult;
    T* loc = (T*)P->ws.loc;
    // upward pass: one launch per level down to the coarsest interacting
    // level (1 periodic, 2 open); the periodic root and its lattice operator
    // are formed by the M2L reduction launch (or else at the start of the
    // downward pass)
    mark(P, 2);
    // periodic trees whose M2L ends in a reduction launch form the root there;
    // the level-1 M2M blocks then also leave their shares of the root multipole
    const bool root_in_reduce = g.periodic && g.depth >= 1 && P->m2l_mode != 0 && P->mg.nchunk > 1;
    // folded: the leaf kernel left each leaf's term of level d - 1, and the
    // first launch (level d - 2) forms level d - 1 from them first
    const int top = folded ? g.depth - 2 : g.depth - 1;
    for (int lev = top; lev >= g.lmin; --lev)
        k_m2m<T><<<dim3(1u << (3 * lev), R), kTreeThreads, 0, st>>>(
            g, lev, mult, (const T*)P->m2mT, (const T*)P->m2m_seg, P->ws.leaf_part, P->ws.box_part,
            (uint16_t*)P->ws.msplit, P->mg.KP, root_in_reduce && lev == 1 ? P->ws.root_part : nullptr,
            folded && lev == top ? P->ws.m2m_part : nullptr);
    mark(P, 3);
    if (g.periodic && g.depth == 0)
        k_root<T><<<R, 256, 0, st>>>(g, P->ws.leaf_part, P->ws.root_m, mult, P->latT, P->ws.root_l, loc,
                                     P->ws.dom);
    mark(P, 4);
    bool root_ready = false;  // the periodic root formed by the M2L launches
    bool fused = false;       // the downward pass adds the M2L chunk partials
    if (g.depth >= g.lmin) {
        if (P->m2l_mode == 0) {
            int64_t nt = 0;
            for (int l = g.lmin; l <= g.depth; ++l) nt += (int64_t)1 << (3 * l);
            k_m2l_plain<T><<<dim3((unsigned)nt, R), 256, 0, st>>>(g, mult, (const T*)P->bankT, loc);
        } else {
            root_ready = launch_m2l_mma<T>(P, g, R, root_in_reduce, &fused);
        }
    }
    // deep periodic trees whose M2L launches did not form the root (no
    // offset chunks): the root once (a single root block of the reduction
    // kernel), instead of in every block of a downward pass of several rounds
    if (g.periodic && !root_ready && !fused && g.depth >= 1 && (1u << (3 * (g.depth - 1))) > 256) {
        k_m2l_reduce<T><<<dim3(1, R), kTreeThreads, 0, st>>>(
            g, P->mg, (const T*)P->ws.m2l_part, loc, 1, mult, (const T*)P->m2mT, (const T*)P->m2m_seg,
            P->ws.leaf_part, P->ws.box_part, P->latT, P->lat_seg, P->ws.root_m, P->ws.root_l, P->ws.dom, nullptr);
        root_ready = true;
    }
    // downward pass: ancestors' local expansions and the L2L into the leaves
    mark(P, 5);
    const int l0 = g.periodic ? 0 : g.lmin;
    // the downward launch carries one extra block per replica that orders the
    // leaves for the near field by decreasing work
    int32_t* order = nullptr;
    if (g.depth >= 1 && g.depth - 1 >= l0) {
        if (want_order && g.nleaf <= kOrderCap) order = P->ws.leaf_order;
        // up to 64 boxes above the leaves: two blocks per box (four leaves
        // each), so that the latency-bound chain runs on twice the CUs (one
        // block of 512 threads fits a CU; four blocks per box would leave the
        // order block without one)
        const unsigned nbox1 = 1u << (3 * (g.depth - 1));
        const bool half = nbox1 <= 64;
        // deep trees whose M2L sums are all in loc and whose root is formed:
        // the levels from l0 + 1 to d - 2 one launch each (every box once),
        // the downward launch from there (its blocks would otherwise each
        // redo the whole ancestor chain)
        int l_start = l0;
        if (!fused && (root_ready || !g.periodic) && g.depth - 1 - l0 >= 4) {
            for (int lev = l0 + 1; lev <= g.depth - 2; ++lev)
                k_l2l_level<T><<<dim3(1u << (3 * lev), R), kTreeThreads, 0, st>>>(
                    g, lev, l0, loc, (const T*)P->l2lT, (const T*)P->l2l_seg, P->ws.root_l);
            l_start = g.depth - 2;
        }
        const unsigned nbx = nbox1 * (half ? 2u : 1u) + (order ? 1u : 0u);
        auto down = half ? k_downward<T, 4> : k_downward<T, 8>;
        down<<<dim3(nbx, R), kTreeThreads, 0, st>>>(
            g, l0, loc, (const T*)P->l2lT, (const T*)P->l2l_seg, mult, (const T*)P->m2mT,
            (const T*)P->m2m_seg, P->ws.leaf_part, P->ws.box_part, P->latT, P->lat_seg, P->ws.root_m, P->ws.root_l,
            P->ws.dom, P->ws.leaf_start, order, root_ready ? 1 : 0, fused ? (const T*)P->ws.m2l_part : nullptr,
            P->mg.nchunk, P->mg.nt_all, l_start);
    }
    return order;
}

// Enqueue one evaluation of R replicas (arguments already validated; rd holds
// the host copy of the replica descriptors).  Every phase is one launch over
// all replicas (grid y = replica).
template <typename T>
fmm_status enqueue_eval(fmm_plan_t P, RepSpan rd, const T* x,
                        const T* qA, const T* qB, const int32_t* site, const double* lam,
                        double* E, T* F, T* phi, double* dVdl,
                        const fmmk::FormArgs<T> fa = {nullptr, nullptr, nullptr},
                        double* dVdl_t = nullptr) {
    using namespace fmmk;
    hipStream_t st = P->stream;
    const Geo g = make_geo(P);
    const int R = (int)rd.size();
    int64_t maxn = 0, S_tot = 0;
    int64_t n_tot = 0;
    for (const RepDesc& d : rd) {
        maxn = std::max(maxn, d.n);
        S_tot += d.S;
        n_tot += d.n;
    }
    if (P->excl_n > 0 && n_tot != P->excl_n)
        return fail(P, FMM_E_INVALID, "the exclusion lists were set for a different atom count");
    mark(P, 0);
    // the leaf kernel takes the first M2M step when a later M2M launch is
    // left to add its terms (depth - 2 >= the coarsest interacting level) and
    // the tree is small enough for launch latency to matter (deeper trees
    // keep the separate launch, which then costs little next to the work)
    const bool fold = P->ws.m2m_part != nullptr && g.depth - 2 >= g.lmin && g.nleaf <= kScanFuseCap;
    enqueue_bin_p2m<T>(P, g, rd, R, x, qA, qB, site, lam, fa, maxn, S_tot, fold);
    int32_t* order = enqueue_tree<T>(P, g, R, true, fold);
    const RepDesc* reps = P->ws.reps;
    const unsigned ab = nblocks(maxn, 256);
    using V4 = vec4_t<T>;
    const V4* pos = (const V4*)P->ws.pos;
    const T* loc = (const T*)P->ws.loc;
    mark(P, 6);
    switch (P->p2p_waves) {
#define FMM_NEAR(NWV)                                                                            \
    case NWV:                                                                                    \
        k_near_far<T, NWV><<<dim3(g.nleaf * P->p2p_split, R), 64 * NWV, 0, st>>>(               \
            g, P->p2p_split, reps, pos, P->ws.leaf_start, P->ws.perm, P->ws.dom, loc, P->gidx,              \
            (const T*)P->gcoef, qA, qB, site, phi, F, P->ws.leaf_energy, P->ws.cphi, fa.qC != nullptr,   \
            order, P->status);                                                                     \
        break;
        FMM_NEAR(4)
        FMM_NEAR(8)
        FMM_NEAR(16)
        default: break;
    }
    if (P->excl_n > 0)
        k_excl<T><<<dim3(ab, R), 256, 0, st>>>(g, reps, x, qA, qB, site, lam, fa, P->ws.dom, P->excl_start,
                                               P->excl_idx, phi, F, P->ws.cphi, fa.qC != nullptr,
                                               P->excl_e);
    mark(P, 7);
    const bool ham = P->prm.hamiltonian != 0;
    if (ham && S_tot > 0)
        k_hcorr<T><<<(unsigned)S_tot, kHcorrThreads, 0, st>>>(g, R, reps, P->ws.site_start, P->ws.site_members, x, qA,
                                                    qB, lam, P->green, F, P->ws.hc_e, P->ws.hc_dl,
                                                    P->status);
    k_reduce<T><<<(unsigned)(R + S_tot), 256, 0, st>>>(g, R, g.nleaf * P->p2p_split, P->ws.leaf_energy,
                                                       P->ws.site_start, P->ws.site_members, P->ws.cphi, E,
                                                       dVdl, P->status, qA, qB, lam, fa, dVdl_t, reps,
                                                       ham && S_tot > 0 ? P->ws.hc_e : nullptr,
                                                       ham && S_tot > 0 ? P->ws.hc_dl : nullptr,
                                                       P->ws.leaf_count, P->ws.site_count,
                                                       P->excl_n > 0 ? P->excl_e : nullptr, (int)ab,
                                                       nullptr, nullptr, P->ws.ovf_n);
    mark(P, -1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(P, FMM_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return FMM_OK;
}

template <typename T>
fmm_status enqueue_adjoint(fmm_plan_t P, RepSpan rd, const T* x,
                           const T* qA, const T* qB, const int32_t* site, const double* lam,
                           const double* gE, T* gx, T* gqA, T* gqB, double* glam, double* E, T* F,
                           T* phi, double* dVdl) {
    T* Fw = F ? F : (T*)P->ws.F_tmp;
    T* pw = phi ? phi : (T*)P->ws.phi_tmp;
    double* dw = dVdl ? dVdl : P->ws.dVdl_tmp;
    fmm_status s = enqueue_eval<T>(P, rd, x, qA, qB, site, lam, E ? E : P->ws.E_tmp, Fw, pw, dw);
    if (s != FMM_OK) return s;
    int64_t m = 0;
    for (const fmmk::RepDesc& d : rd) m = std::max(m, std::max(d.n, d.S));
    fmmk::k_adjoint<T><<<dim3(nblocks(m, 256), (unsigned)rd.size()), 256, 0, P->stream>>>(
        P->ws.reps, site, lam, gE, Fw, pw, dw, gx, gqA, gqB, glam);
    return hipGetLastError() == hipSuccess ? FMM_OK : fail(P, FMM_E_HIP, "adjoint launch failed");
}

// Gradients of gE E + gphi . phi + gF . F for one system in one tree pass:
// the charges q in expansion slot 0 and the second sources (charges gphi,
// dipoles -q gF) in slot 1, then the leaf pass of both, the combine kernel
// (exclusions, outputs) and the fixed-order reductions (E, dV/dlambda and the
// lambda gradient).  gE is read from device memory when gE_dev is set.
template <typename T>
fmm_status enqueue_adjoint_full(fmm_plan_t P, const fmmk::RepDesc& r0, const T* x, const T* qA,
                                const T* qB, const int32_t* site, const double* lam,
                                const double* gE_dev, double gE, const T* gphi, const T* gF, T* gx,
                                T* gqA, T* gqB, double* glam, double* E, T* F, T* phi,
                                double* dVdl) {
    using namespace fmmk;
    hipStream_t st = P->stream;
    const Geo g = make_geo(P);
    const int64_t n = r0.n, S = r0.S;
    if (P->excl_n > 0 && n != P->excl_n)
        return fail(P, FMM_E_INVALID, "the exclusion lists were set for a different atom count");
    const RepDesc rd2[2] = {r0, r0};  // slot 1: the second sources of the same system
    const RepSpan rd(rd2, 2);
    const FormArgs<T> fa{nullptr, nullptr, nullptr};
    mark(P, 0);
    enqueue_bin_p2m<T>(P, g, rd, 1, x, qA, qB, site, lam, fa, n, S, false);
    using V4 = vec4_t<T>;
    k_leaf_src2<T><<<g.nleaf, kLeafThreads, src2_lds_bytes<T>(g.K), st>>>(
        g, (const V4*)P->ws.pos, P->ws.perm, P->ws.leaf_start, gphi, gF, P->ws.dom, (V4*)P->ws.adj_src2, (T*)P->ws.mult,
        P->ws.leaf_part, (uint16_t*)P->ws.msplit, P->mg.KP);
    enqueue_tree<T>(P, g, 2, false, false);
    mark(P, 6);
    k_near_adj<T, kAdjWaves><<<g.nleaf, 64 * kAdjWaves, 0, st>>>(g, (const V4*)P->ws.pos, (const V4*)P->ws.adj_src2,
                                                   P->ws.leaf_start, P->ws.perm, P->ws.dom, (const T*)P->ws.loc,
                                                   P->gidx, (const T*)P->gcoef, (T*)P->ws.adj_acc);
    const unsigned nb = nblocks(n, 256);
    k_adj_combine<T><<<nb, 256, 0, st>>>(g, n, S, x, qA, qB, site, lam, gphi, gF, gE_dev, gE, P->ws.dom,
                                         P->excl_n > 0 ? P->excl_start : nullptr, P->excl_idx,
                                         (const T*)P->ws.adj_acc, phi, F, gx, gqA, gqB, P->ws.cphi,
                                         P->ws.adj_cphi2, P->ws.adj_part);
    mark(P, 7);
    k_reduce<T><<<(unsigned)(1 + S), 256, 0, st>>>(g, 1, (int64_t)nb, P->ws.adj_part, P->ws.site_start,
                                                    P->ws.site_members, P->ws.cphi, E ? E : P->ws.E_tmp, dVdl,
                                                    P->status, qA, qB, lam, fa, nullptr, P->ws.reps, nullptr,
                                                    nullptr, P->ws.leaf_count, P->ws.site_count, nullptr, 0,
                                                    P->ws.adj_cphi2, glam, P->ws.ovf_n);
    mark(P, -1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(P, FMM_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return FMM_OK;
}

// Run `enqueue` eagerly, or (params.graph) replay the cached graph when the
// argument key matches, else capture a new graph and replay it.
template <class Fn>
fmm_status run_maybe_graph(fmm_plan_t P, const std::vector<unsigned char>& key, Fn&& enqueue) {
    if (!P->prm.graph || P->prof_on) return enqueue();
    if (!P->stream) return fail(P, FMM_E_INVALID, "graph replay needs a non-default stream");
    if (P->graph_valid && P->graph_key == key) {
        if (hipGraphLaunch(P->graph_exec, P->stream) != hipSuccess)
            return fail(P, FMM_E_HIP, "hipGraphLaunch failed");
        return FMM_OK;
    }
    if (P->graph_exec) (void)hipGraphExecDestroy(P->graph_exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    P->graph_exec = nullptr;
    P->graph = nullptr;
    P->graph_valid = false;
    if (hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(P, FMM_E_HIP, "hipStreamBeginCapture failed");
    fmm_status s = enqueue();
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(P->stream, &gr);
    if (s != FMM_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return s;
    }
    if (e != hipSuccess || !gr) return fail(P, FMM_E_HIP, "hipStreamEndCapture failed");
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return fail(P, FMM_E_HIP, "hipGraphInstantiate failed");
    }
    P->graph = gr;
    P->graph_exec = ex;
    P->graph_key = key;
    P->graph_valid = true;
    if (hipGraphLaunch(ex, P->stream) != hipSuccess) return fail(P, FMM_E_HIP, "hipGraphLaunch failed");
    return FMM_OK;
}

struct KeyBuf {
    std::vector<unsigned char> b;
    template <typename V>
    KeyBuf& add(const V& v) {
        const unsigned char* p = (const unsigned char*)&v;
        b.insert(b.end(), p, p + sizeof(V));
        return *this;
    }
};

fmm_status check_box(fmm_plan_t P, const double* box, double* L) {
    if (P->prm.boundary == FMM_PERIODIC) {
        if (!box) return fail(P, FMM_E_INVALID, "periodic plan needs a box");
        if (!(box[0] > 0) || !std::isfinite(box[0]))
            return fail(P, FMM_E_INVALID, "box edges must be positive and finite");
        if (box[1] != box[0] || box[2] != box[0])
            return fail(P, FMM_E_UNSUPPORTED, "only cubic periodic cells are supported");
        *L = box[0];
    } else {
        if (box) return fail(P, FMM_E_INVALID, "open plan: box must be NULL");
        *L = 0.0;
    }
    return FMM_OK;
}

fmm_status check_common(fmm_plan_t P, int64_t n, const void* x, const void* qA, const void* qB,
                        const int32_t* site, int64_t S, const double* lam) {
    if (!P) return FMM_E_INVALID;
    if (n < 0 || n > P->prm.max_atoms) return fail(P, FMM_E_INVALID, "n outside [0, max_atoms]");
    if (n > INT32_MAX) return fail(P, FMM_E_UNSUPPORTED, "n above 2^31 - 1");
    if (S < 0 || S > P->prm.max_sites) return fail(P, FMM_E_INVALID, "n_sites outside [0, max_sites]");
    if (n > 0 && (!x || !qA || !qB || !site))
        return fail(P, FMM_E_INVALID, "null input pointer");
    if (S > 0 && !lam) return fail(P, FMM_E_INVALID, "null lambda pointer");
    return FMM_OK;
}

}  // namespace

extern "C" {

fmm_status fmm_plan_create(const fmm_params* prm, void* hip_stream, fmm_plan_t* out) {
    if (!prm || !out) return FMM_E_INVALID;
    *out = nullptr;
    if (prm->depth < 0 || prm->depth > fmmk::kDMax || prm->order_p < 1 ||
        prm->order_p > fmmk::kPMax || prm->max_atoms < 0 || prm->max_sites < 0 ||
        prm->max_replicas < 1 || (prm->boundary != FMM_OPEN && prm->boundary != FMM_PERIODIC) ||
        (prm->precision != FMM_FP64 && prm->precision != FMM_MIXED_F32 &&
         prm->precision != FMM_MIXED_BF16X3) ||
        !std::isfinite(prm->coulomb_k) || prm->max_atoms > INT32_MAX ||
        prm->m2l_kernel < 0 || prm->m2l_kernel > 3 || prm->m2l_chunk < 0 || prm->m2l_chunk > 189 ||
        (prm->p2p_waves != 0 && prm->p2p_waves != 4 && prm->p2p_waves != 8 &&
         prm->p2p_waves != 16) || prm->graph < 0 || prm->graph > 1 || prm->p2p_split < 0 ||
        prm->p2p_split > fmmk::kMaxSplit || prm->hamiltonian < 0 || prm->hamiltonian > 1)
        return FMM_E_INVALID;
    {
        const int K = (prm->order_p + 1) * (prm->order_p + 1);
        const bool mma_ok = K <= 16 * fmmk::kM2LMaxRT && (prm->precision != FMM_FP64 || K <= 96);
        if (prm->m2l_kernel >= 2 && !mma_ok) return FMM_E_INVALID;
    }
    fmm_plan_s* P = new fmm_plan_s();
    P->prm = *prm;
    P->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&P->device) != hipSuccess || !scratch_lookup(P->device)) {
        delete P;
        return FMM_E_HIP;
    }
    P->fp64 = prm->precision == FMM_FP64;
    // near-field block shape: 8 wavefronts per leaf, 4 when the leaves hold
    // at most 32 atoms on average (a deep tree: smaller blocks, more of them
    // per CU; 500,000 atoms at depth 5: 634 against 863 us)
    if (prm->p2p_waves) {
        P->p2p_waves = prm->p2p_waves;
    } else {
        const double per_leaf = (double)prm->max_atoms /
                                ((double)std::max(prm->max_replicas, 1) * std::ldexp(1.0, 3 * prm->depth));
        P->p2p_waves = per_leaf <= 32.0 ? 4 : 8;
    }
    P->p2p_split = prm->p2p_split ? prm->p2p_split : 1;
    P->tsz = P->fp64 ? 8 : 4;
    const int p = prm->order_p, d = prm->depth;
    P->K = (p + 1) * (p + 1);
    P->Kp = (P->K + 3) & ~3;
    P->Kg = p * p;
    P->nleaf = 1 << (3 * d);
    int64_t off = 0;
    for (int l = 0; l <= fmmk::kDMax + 1; ++l) {
        P->lev_off[l] = off;
        if (l <= d) off += (int64_t)1 << (3 * l);
    }
    P->nbox = off;
    init_rho_coef();
    const int64_t N = std::max<int64_t>(prm->max_atoms, 1), S = std::max<int64_t>(prm->max_sites, 1);
    const size_t ts = P->tsz, K = P->K;
    // replica slots of the tree workspace: at least two (the adjoint runs its
    // second sources through slot 1); the M2L tiling still follows max_replicas
    const size_t RM = (size_t)std::max(prm->max_replicas, 2);
    const size_t RT = (size_t)prm->max_replicas;
    P->R_max = prm->max_replicas;
    // leaf buckets hold about three times a replica's mean leaf population
    // (at least one leaf block's threads, at most the in-LDS sort size);
    // fuller leaves spill into the overflow list
    if (P->nleaf <= fmmk::kScanFuseCap) {
        const int64_t mean = (N + (int64_t)P->R_max * P->nleaf - 1) / ((int64_t)P->R_max * P->nleaf);
        int cap = fmmk::kLeafBucketMin;
        while (cap < 3 * mean && cap < fmmk::kSortCap) cap <<= 1;
        P->leaf_cap = cap;
    }
    bool ok = true;
    ok &= dev_alloc(P, &P->bankT, 343 * K * K * ts);
    ok &= dev_alloc(P, &P->m2mT, K * K * ts);  // octant 0; the others are its reflections
    ok &= dev_alloc(P, &P->l2lT, K * K * ts);
    ok &= dev_alloc(P, (void**)&P->latT, K * K * 8);
    const size_t seg = (size_t)fmmk::kTriCache * fmmk::kTreeThreads;
    ok &= dev_alloc(P, &P->m2m_seg, seg * ts);
    ok &= dev_alloc(P, &P->l2l_seg, seg * ts);
    ok &= dev_alloc(P, (void**)&P->lat_seg, seg * 8);
    ok &= dev_alloc(P, (void**)&P->gidx, 3 * (size_t)P->Kg * 4 * 4);
    ok &= dev_alloc(P, &P->gcoef, 3 * (size_t)P->Kg * 4 * ts);
    ok &= dev_alloc(P, (void**)&P->status, 4 * 4);
    if (prm->hamiltonian) ok &= dev_alloc(P, (void**)&P->green, (fmmk::kKMax + 3 * fmmk::kKgMax) * 8);
    if (!ok) {
        fmm_plan_destroy(P);
        return FMM_E_OOM;
    }
    // operator tables (FP64 on the host, converted to the working type)
    std::vector<double> bank(343 * K * K), m2m(8 * K * K), l2l(8 * K * K), lat(K * K);
    fmmops::build_m2l_bank(p, bank.data());
    fmmops::build_m2m(p, m2m.data());
    fmmops::build_l2l(p, l2l.data());
    std::vector<int32_t> gi(3 * (size_t)P->Kg * 4);
    std::vector<double> gc(3 * (size_t)P->Kg * 4);
    fmmops::build_grad_table(p, gi.data(), gc.data());
    if (prm->boundary == FMM_PERIODIC) fmmops::build_lattice(p, lat.data());
    hipError_t e = hipSuccess;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    if (P->fp64) {
        auto b = transpose_blocks<double>(bank, 343, K);
        auto a = transpose_blocks<double>(m2m, 1, K);
        auto c = transpose_blocks<double>(l2l, 1, K);
        up(P->bankT, b.data(), b.size() * 8);
        up(P->m2mT, a.data(), K * K * 8);
        up(P->l2lT, c.data(), K * K * 8);
        up(P->gcoef, gc.data(), gc.size() * 8);
    } else {
        auto b = transpose_blocks<float>(bank, 343, K);
        auto a = transpose_blocks<float>(m2m, 1, K);
        auto c = transpose_blocks<float>(l2l, 1, K);
        std::vector<float> gf(gc.begin(), gc.end());
        up(P->bankT, b.data(), b.size() * 4);
        up(P->m2mT, a.data(), K * K * 4);
        up(P->l2lT, c.data(), K * K * 4);
        up(P->gcoef, gf.data(), gf.size() * 4);
    }
    auto lt = transpose_blocks<double>(lat, 1, K);
    up(P->latT, lt.data(), lt.size() * 8);
    {
        auto ls = pack_tri<double>(lat.data(), (int)K, fmmk::kTriFull);
        up(P->lat_seg, ls.data(), ls.size() * 8);
        if (P->fp64) {
            auto a = pack_tri<double>(m2m.data(), (int)K, fmmk::kTriLower);
            auto c = pack_tri<double>(l2l.data(), (int)K, fmmk::kTriUpper);
            up(P->m2m_seg, a.data(), a.size() * 8);
            up(P->l2l_seg, c.data(), c.size() * 8);
        } else {
            auto a = pack_tri<float>(m2m.data(), (int)K, fmmk::kTriLower);
            auto c = pack_tri<float>(l2l.data(), (int)K, fmmk::kTriUpper);
            up(P->m2m_seg, a.data(), a.size() * 4);
            up(P->l2l_seg, c.data(), c.size() * 4);
        }
    }
    up(P->gidx, gi.data(), gi.size() * 4);
    // matrix-core M2L: mode, tile geometry, offset lists, task list, banks
    {
        const int lmin = prm->boundary == FMM_PERIODIC ? 1 : 2;
        const bool mma_ok = (int)K <= 16 * fmmk::kM2LMaxRT && (!P->fp64 || K <= 96);
        if (d >= lmin && mma_ok && prm->m2l_kernel != 1)
            P->m2l_mode = P->fp64 ? 2 : (prm->precision == FMM_MIXED_BF16X3 ? 3 : 1);
    }
    if (P->m2l_mode && e == hipSuccess) {
        fmmk::M2LGeom& mg = P->mg;
        const int lmin = prm->boundary == FMM_PERIODIC ? 1 : 2;
        mg.RP = round_up((int)K, 16);
        mg.KP = round_up((int)K, P->m2l_mode == 3 ? 32 : 4);
        mg.SA = lds_stride(P->m2l_mode, mg.KP);
        mg.SB = mg.SA;
        P->m2l_rt = mg.RP / 16;
        // target columns of one class: its boxes at every level >= lmin
        int64_t ncol = 0, nt_all = 0;
        for (int l = lmin; l <= d; ++l) {
            ncol += (int64_t)1 << (3 * (l - 1));
            nt_all += (int64_t)1 << (3 * l);
        }
        mg.ncol = (int)ncol;
        mg.nt_all = nt_all;
        const int ntile = (int)((ncol + fmmk::kM2LTile - 1) / fmmk::kM2LTile);
        const int64_t items = 8 * (int64_t)ntile * (int64_t)RT;
        // bf16x3 with one tile per class: resident sources, chunks within the
        // canonical offsets' parity groups
        P->m2l_rs = P->m2l_mode == 3 && ntile == 1 && prm->m2l_kernel != 3 && P->m2l_rt <= fmmk::kM2LRsMaxRT &&
                    mg.KP / 8 == fmmk::m2l_rs_kc(P->m2l_rt);
        // chunks of the parity groups (sizes of class 0's list: 26, 3 x 25,
        // 3 x 23, 19) for a chunk size
        auto rs_chunks = [](int cs) {
            const int gs[8] = {26, 25, 25, 25, 23, 23, 23, 19};
            int n = 0;
            for (int gz : gs) n += (gz + cs - 1) / cs;
            return n;
        };
        int csize = prm->m2l_chunk;
        if (csize == 0 && P->m2l_rs) {
            // about one work-group per CU over all replicas: the smallest chunk
            // size with at most 256 work-groups (7 for one replica: 31 chunks
            // per class, 248 work-groups), at least one chunk per group
            csize = 1;
            while (csize < 26 && 8 * (int64_t)RT * rs_chunks(csize) > 256) ++csize;
        } else if (csize == 0) {
            // bf16x3 runs one double-buffered work-group per CU: about one task per CU;
            // the others overlap two single-buffered work-groups per CU
            const int64_t target = P->m2l_mode == 3 ? 256 : 2048, cap = P->m2l_mode == 3 ? 63 : 27;
            const int64_t want = std::max<int64_t>(1, std::min<int64_t>(cap, (target + items - 1) / items));
            csize = (int)((189 + want - 1) / want);
        }
        mg.csize = csize;
        mg.nchunk = (189 + csize - 1) / csize;
        // resident sources: the canonical offsets ordered by parity group
        // (x, y, z parities of o' = (oi / 49 - 3, (oi / 7) % 7 - 3, oi % 7 - 3)),
        // each group cut into near-equal chunks of at most csize
        std::vector<int> rs_bound;  // chunk boundaries in list positions
        auto parity = [](int oi) {
            return (((oi / 49 - 3) & 1) << 2) | ((((oi / 7) % 7 - 3) & 1) << 1) | ((oi % 7 - 3) & 1);
        };
        // Offset chunks are contiguous ranges of the global (bank-index sorted)
        // offset set, so a chunk's operators are the same for every class; each
        // class takes the part of its 189 offsets that falls in the range.
        std::vector<int16_t> cls_off = class_offsets();
        std::vector<int> used;
        {
            std::vector<char> seen(343, 0);
            for (int16_t o : cls_off) seen[o] = 1;
            for (int o = 0; o < 343; ++o)
                if (seen[o]) used.push_back(o);
        }
        std::vector<int16_t> cstart(8 * (mg.nchunk + 1));
        if (P->m2l_mode == 3 && P->m2l_rs) {
            std::sort(cls_off.begin(), cls_off.begin() + 189, [&](int16_t a, int16_t b) {
                const int pa = parity(a), pb = parity(b);
                return pa != pb ? pa < pb : a < b;
            });
            for (int c = 1; c < 8; ++c)
                std::copy(cls_off.begin(), cls_off.begin() + 189, cls_off.begin() + 189 * c);
            rs_bound.push_back(0);
            for (int g0 = 0; g0 < 189;) {
                int g1 = g0;
                while (g1 < 189 && parity(cls_off[g1]) == parity(cls_off[g0])) ++g1;
                const int sz = g1 - g0, nch = (sz + csize - 1) / csize;
                for (int k = 1; k <= nch; ++k) rs_bound.push_back(g0 + k * sz / nch);
                g0 = g1;
            }
            mg.nchunk = (int)rs_bound.size() - 1;
            cstart.assign(8 * (mg.nchunk + 1), 0);
            for (int c = 0; c < 8; ++c)
                for (int k = 0; k <= mg.nchunk; ++k) cstart[c * (mg.nchunk + 1) + k] = (int16_t)rs_bound[k];
        } else if (P->m2l_mode == 3) {
            // every class runs on class 0's (canonical) offsets, mirrored by
            // the class's reflection; chunks are equal slices of that list
            std::sort(cls_off.begin(), cls_off.begin() + 189);
            for (int c = 1; c < 8; ++c)
                std::copy(cls_off.begin(), cls_off.begin() + 189, cls_off.begin() + 189 * c);
            for (int c = 0; c < 8; ++c)
                for (int k = 0; k <= mg.nchunk; ++k)
                    cstart[c * (mg.nchunk + 1) + k] = (int16_t)(k * 189 / mg.nchunk);
        } else {
            std::vector<int> bound(mg.nchunk + 1);
            for (int k = 0; k <= mg.nchunk; ++k) {
                const size_t u = (size_t)k * used.size() / mg.nchunk;
                bound[k] = u < used.size() ? used[u] : 343;
            }
            for (int c = 0; c < 8; ++c) {
                std::sort(cls_off.begin() + 189 * c, cls_off.begin() + 189 * (c + 1));
                int pos = 0;
                for (int k = 0; k <= mg.nchunk; ++k) {
                    while (pos < 189 && cls_off[189 * c + pos] < bound[k]) ++pos;
                    cstart[c * (mg.nchunk + 1) + k] = (int16_t)pos;
                }
            }
        }
        // Work-groups are dispatched round-robin over the 8 XCDs (group i on XCD
        // i mod 8), each with its own L2.  Tasks are ordered so that slot i holds
        // a task of an offset chunk assigned to XCD i mod 8: every XCD then reads
        // only its share of the operator bank, which stays in its L2.
        const int kXcd = 8;
        std::vector<std::vector<fmmk::M2LTask>> byx(kXcd);
        for (int ch = 0; ch < mg.nchunk; ++ch)
            for (int c = 0; c < 8; ++c)
                for (int t = 0; t < ntile; ++t) {
                    int x;
                    if (mg.nchunk >= kXcd) x = ch % kXcd;
                    else x = ch + mg.nchunk * ((c * ntile + t) % (kXcd / mg.nchunk));
                    const int o0 = cstart[c * (mg.nchunk + 1) + ch], o1 = cstart[c * (mg.nchunk + 1) + ch + 1];
                    byx[x].push_back({c, t, ch, o0, o1, {0, 0, 0}});
                }
        std::vector<fmmk::M2LTask> tl;
        size_t longest = 0;
        for (auto& v : byx) longest = std::max(longest, v.size());
        for (size_t j = 0; j < longest; ++j)
            for (int x = 0; x < kXcd; ++x)
                if (j < byx[x].size()) tl.push_back(byx[x][j]);
        P->n_tasks = (int64_t)tl.size();
        const size_t esz = P->m2l_mode == 2 ? 8 : (P->m2l_mode == 1 ? 4 : 2);
        P->m2l_lds = esz * ((size_t)mg.RP * mg.SA + (size_t)fmmk::kM2LTile * mg.SB);
        const int KC = mg.KP / 8;
        if (P->m2l_mode == 3 && P->m2l_rs) {
            // resident source rows and two operator buffers: static LDS
            P->m2l_nbuf = 2;
            P->m2l_lds = 0;
        } else if (P->m2l_mode == 3) {
            // one staging buffer: operator (2 KC RP chunks) + sources ((2 KC + 1) 80 chunks)
            const size_t one = (size_t)16 * (2 * KC * mg.RP + (2 * KC + 1) * fmmk::kM2LTile);
            P->m2l_nbuf = 2 * one <= fmmk::kLdsBytes ? 2 : 1;
            P->m2l_lds = P->m2l_nbuf * one;
        }
        const std::vector<int16_t>& ol = cls_off;
        bool ok2 = !ol.empty();
        ok2 &= dev_alloc(P, (void**)&P->tasks, tl.size() * sizeof(fmmk::M2LTask));
        ok2 &= dev_alloc(P, (void**)&P->olist, ol.size() * sizeof(int16_t));
        ok2 &= dev_alloc(P, (void**)&P->cstart, cstart.size() * sizeof(int16_t));
        const size_t nb = (size_t)343 * mg.RP * mg.KP;
        ok2 &= dev_alloc(P, &P->bank_mma, nb * esz * (P->m2l_mode == 3 ? 2 : 1));
        if (P->m2l_mode == 3) ok2 &= dev_alloc(P, &P->sign_tab, 8 * 4 * fmmk::kM2LMaxKs * 16);
        if (!ok2) {
            fmm_plan_destroy(P);
            return FMM_E_OOM;
        }
        up(P->tasks, tl.data(), tl.size() * sizeof(fmmk::M2LTask));
        up(P->olist, ol.data(), ol.size() * sizeof(int16_t));
        up(P->cstart, cstart.data(), cstart.size() * sizeof(int16_t));
        if (P->m2l_mode == 2) {
            std::vector<double> bm(nb, 0.0);
            for (int o = 0; o < 343; ++o)
                for (size_t r = 0; r < K; ++r)
                    for (size_t k = 0; k < K; ++k)
                        bm[((size_t)o * mg.RP + r) * mg.KP + k] = bank[((size_t)o * K + r) * K + k];
            up(P->bank_mma, bm.data(), nb * 8);
        } else if (P->m2l_mode == 1) {
            std::vector<float> bm(nb, 0.f);
            for (int o = 0; o < 343; ++o)
                for (size_t r = 0; r < K; ++r)
                    for (size_t k = 0; k < K; ++k)
                        bm[((size_t)o * mg.RP + r) * mg.KP + k] = (float)bank[((size_t)o * K + r) * K + k];
            up(P->bank_mma, bm.data(), nb * 4);
        } else {
            // slot j = canonical offset j: [part hi/lo][KC][RP][8], the LDS image
            // of the operator
            std::vector<uint16_t> bm(2 * nb, 0);
            for (int o = 0; o < 189; ++o)
                for (size_t r = 0; r < K; ++r)
                    for (size_t k = 0; k < K; ++k) {
                        const double v = bank[((size_t)ol[o] * K + r) * K + k];
                        const uint16_t h = to_bf16((float)v);
                        const uint16_t l = to_bf16((float)(v - (double)from_bf16(h)));
                        const size_t kc = k / 8, e8 = k % 8;
                        const size_t base = (size_t)o * 2 * mg.RP * mg.KP;
                        bm[base + ((0 * KC + kc) * mg.RP + r) * 8 + e8] = h;
                        bm[base + (((size_t)KC + kc) * mg.RP + r) * 8 + e8] = l;
                    }
            up(P->bank_mma, bm.data(), 2 * nb * 2);
            // sign-bit masks of S for class c: chunk kc covers k = 8 kc .. 8 kc + 7
            // (bf16 entry e at bit 16 (e % 2) + 15 of dword e / 2)
            std::vector<uint32_t> sg(8 * 4 * fmmk::kM2LMaxKs * 4, 0u);
            for (int c = 0; c < 8; ++c)
                for (int k = 0; k < (int)K; ++k)
                    if (__builtin_popcount((unsigned)(c & refl_bits_host(k))) & 1)
                        sg[((size_t)c * 4 * fmmk::kM2LMaxKs + k / 8) * 4 + (k % 8) / 2] |=
                            (k & 1) ? 0x80000000u : 0x8000u;
            up(P->sign_tab, sg.data(), sg.size() * 4);
        }
        hipError_t ea = hipSuccess;
        auto setlds = [&](const void* fn) {
            if (ea == hipSuccess)
                ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)P->m2l_lds);
        };
        switch (P->m2l_mode * 16 + P->m2l_rt) {
#define FMM_LDS_CASE(MODE, RTV, KER) \
    case MODE * 16 + RTV: setlds((const void*)&KER<RTV>); break;
#define FMM_LDS_ALL(MODE, KER) \
    FMM_LDS_CASE(MODE, 1, KER) FMM_LDS_CASE(MODE, 2, KER) FMM_LDS_CASE(MODE, 3, KER) \
    FMM_LDS_CASE(MODE, 4, KER) FMM_LDS_CASE(MODE, 5, KER) FMM_LDS_CASE(MODE, 6, KER) \
    FMM_LDS_CASE(MODE, 7, KER) FMM_LDS_CASE(MODE, 8, KER)
            FMM_LDS_ALL(1, fmmk::k_m2l_f32)
            FMM_LDS_ALL(2, fmmk::k_m2l_f64)
            FMM_LDS_ALL(3, fmmk::k_m2l_bf16x3)
            default: break;
        }

        if (ea != hipSuccess) e = ea;
    }
    for (int fold = 0; fold < 2 && e == hipSuccess; ++fold) {
        const void* f = P->fp64 ? (fold ? (const void*)&fmmk::k_leaf_p2m<double, true>
                                        : (const void*)&fmmk::k_leaf_p2m<double, false>)
                                : (fold ? (const void*)&fmmk::k_leaf_p2m<float, true>
                                        : (const void*)&fmmk::k_leaf_p2m<float, false>);
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                P->fp64 ? (int)leaf_lds_bytes_max<double>((int)K)
                                        : (int)leaf_lds_bytes_max<float>((int)K));
    }
    if (e == hipSuccess) {
        e = P->fp64 ? hipFuncSetAttribute((const void*)&fmmk::k_leaf_src2<double>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)src2_lds_bytes<double>((int)K))
                    : hipFuncSetAttribute((const void*)&fmmk::k_leaf_src2<float>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)src2_lds_bytes<float>((int)K));
    }
    // the workspace: one arena for every per-evaluation buffer, cleared once
    // (counters start at zero, and every evaluation's final reduction
    // re-zeroes the ones it used; the bf16 split rows' zero row and padding
    // past K are never written)
    if (e == hipSuccess) {
        const size_t bytes = ws_layout(P, N, S, RM, true, nullptr, nullptr);
        if (!dev_alloc(P, &P->ws_arena, bytes)) {
            fmm_plan_destroy(P);
            return FMM_E_OOM;
        }
        ws_layout(P, N, S, RM, true, (char*)P->ws_arena, &P->ws);
        e = hipMemset(P->ws_arena, 0, bytes);
    }
    if (prm->hamiltonian) {
        // periodic pair potential: h of the unit cube to degree kPMax and the
        // coefficients of its gradient (degree kPMax - 1); zero for open cells
        const int PH = fmmk::kPMax, KH = fmmk::kKMax, KG = fmmk::kKgMax;
        std::vector<double> gv((size_t)KH + 3 * KG, 0.0);
        if (prm->boundary == FMM_PERIODIC) {
            fmmops::build_periodic_green(PH, gv.data());
            std::vector<int32_t> hi((size_t)3 * KG * 4);
            std::vector<double> hcf((size_t)3 * KG * 4);
            fmmops::build_grad_table(PH, hi.data(), hcf.data());
            for (int q = 0; q < 3 * KG; ++q) {
                double v = 0.0;
                for (int t = 0; t < 4; ++t)
                    if (hi[(size_t)q * 4 + t] >= 0) v += hcf[(size_t)q * 4 + t] * gv[hi[(size_t)q * 4 + t]];
                gv[(size_t)KH + q] = v;
            }
        }
        up(P->green, gv.data(), gv.size() * 8);
    }
    int32_t z[4] = {0, 0, 0, 0};
    up(P->status, z, sizeof(z));
    if (e != hipSuccess) {
        fmm_plan_destroy(P);
        return FMM_E_HIP;
    }
    *out = P;
    return FMM_OK;
}

void fmm_plan_destroy(fmm_plan_t P) {
    if (!P) return;
    if (P->graph_exec) (void)hipGraphExecDestroy(P->graph_exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    for (hipEvent_t ev : P->prof_ev) (void)hipEventDestroy(ev);
    for (void* a : {(void*)P->excl_start, (void*)P->excl_idx, (void*)P->excl_e})
        if (a) (void)hipFree(a);
    for (void* a : P->allocs) (void)hipFree(a);
    delete P;
}

fmm_status fmm_set_exclusions(fmm_plan_t P, int64_t n, const int32_t* start, const int32_t* idx) {
    if (!P) return FMM_E_INVALID;
    if (n < 0 || n > P->prm.max_atoms) return fail(P, FMM_E_INVALID, "exclusion atom count outside [0, max_atoms]");
    if (n > 0 && P->prm.hamiltonian)
        return fail(P, FMM_E_UNSUPPORTED, "exclusions with Hamiltonian interpolation");
    if (n > 0 && (!start || (start[n] > 0 && !idx))) return fail(P, FMM_E_INVALID, "null exclusion list");
    if (n > 0) {
        if (start[0] != 0) return fail(P, FMM_E_INVALID, "exclusion offsets must start at 0");
        for (int64_t i = 0; i < n; ++i)
            if (start[i + 1] < start[i]) return fail(P, FMM_E_INVALID, "exclusion offsets must not decrease");
        // partners in range, not the atom itself, each list ascending without
        // repeats, and every pair listed from both sides
        for (int64_t i = 0; i < n; ++i)
            for (int32_t k = start[i]; k < start[i + 1]; ++k) {
                const int32_t j = idx[k];
                if (j < 0 || j >= n || j == i) return fail(P, FMM_E_INVALID, "exclusion partner out of range");
                if (k > start[i] && idx[k - 1] >= j)
                    return fail(P, FMM_E_INVALID, "exclusion lists must ascend without repeats");
                if (!std::binary_search(idx + start[j], idx + start[j + 1], (int32_t)i))
                    return fail(P, FMM_E_INVALID, "exclusion lists must be symmetric");
            }
    }
    // evaluations already enqueued may still read the old lists
    if (P->excl_n > 0 && hipStreamSynchronize(P->stream) != hipSuccess)
        return fail(P, FMM_E_HIP, "stream sync failed");
    for (int32_t** a : {&P->excl_start, &P->excl_idx}) {
        if (*a) (void)hipFree(*a);
        *a = nullptr;
    }
    if (P->excl_e) (void)hipFree(P->excl_e);
    P->excl_e = nullptr;
    P->excl_n = 0;
    P->graph_valid = false;  // the launch sequence changes
    if (n == 0) return FMM_OK;
    const size_t ne = (size_t)start[n];
    const size_t parts = (size_t)P->R_max * std::max<int64_t>(1, (P->prm.max_atoms + 255) / 256);
    if (hipMalloc((void**)&P->excl_start, (n + 1) * 4) != hipSuccess ||
        hipMalloc((void**)&P->excl_idx, std::max<size_t>(ne, 1) * 4) != hipSuccess ||
        hipMalloc((void**)&P->excl_e, parts * 8) != hipSuccess)
        return fail(P, FMM_E_OOM, "exclusion lists do not fit");
    if (hipMemcpy(P->excl_start, start, (n + 1) * 4, hipMemcpyHostToDevice) != hipSuccess ||
        (ne && hipMemcpy(P->excl_idx, idx, ne * 4, hipMemcpyHostToDevice) != hipSuccess))
        return fail(P, FMM_E_HIP, "exclusion upload failed");
    P->excl_n = n;
    return FMM_OK;
}

const char* fmm_last_error(fmm_plan_t P) {
    if (!P) return "null plan";
    return P->err.c_str();
}

fmm_status fmm_eval(fmm_plan_t P, int64_t n, const void* x, const void* qA, const void* qB,
                    const int32_t* site, int64_t S, const double* lam, const double* box,
                    double* E, void* F, void* phi, double* dVdl) {
    fmm_status s = check_common(P, n, x, qA, qB, site, S, lam);
    if (s != FMM_OK) return s;
    double L = 0;
    if ((s = check_box(P, box, &L)) != FMM_OK) return s;
    P->err.clear();
    std::vector<fmmk::RepDesc> rd(1);
    rd[0] = {0, n, 0, S, L, 0};
    KeyBuf key;
    key.add(1).add(rd[0]).add(x).add(qA).add(qB).add(site).add(lam).add(E).add(F).add(phi).add(dVdl);
    return run_maybe_graph(P, key.b, [&]() {
        if (P->fp64)
            return enqueue_eval<double>(P, rd, (const double*)x, (const double*)qA,
                                        (const double*)qB, site, lam, E, (double*)F, (double*)phi,
                                        dVdl);
        return enqueue_eval<float>(P, rd, (const float*)x, (const float*)qA, (const float*)qB, site,
                                   lam, E, (float*)F, (float*)phi, dVdl);
    });
}

fmm_status fmm_eval_noalloc(fmm_plan_t P, int64_t n, const void* x, const void* qA, const void* qB,
                            const int32_t* site, int64_t S, const double* lam, const double* box,
                            double* E, void* F, void* phi, double* dVdl) {
    fmm_status s = check_common(P, n, x, qA, qB, site, S, lam);
    if (s != FMM_OK) return s;
    double L = 0;
    if ((s = check_box(P, box, &L)) != FMM_OK) return s;
    void* base = scratch_address(P->device);
    if (!base) return fail(P, FMM_E_HIP, "no static scratch address for this device");
    const size_t need = ws_layout(P, n, S, 1, false, nullptr, nullptr);
    if (need > kScratchBytes) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "fmm_eval_noalloc: %zu bytes of scratch needed, the static "
                      "scratch holds %zu (fewer atoms or a shallower tree)", need, kScratchBytes);
        return fail(P, FMM_E_INVALID, msg);
    }
    P->err.clear();
    Workspace sw;
    ws_layout(P, n, S, 1, false, (char*)base, &sw);
    const fmmk::RepDesc rd{0, n, 0, S, L, 0};
    // what must start at zero: the leaf and site counters, the cube record
    // and the bf16 split rows (the zero row and the padding past K); fill
    // kernels, no memset nodes
    hipStream_t st = P->stream;
    fmmk::k_fill_i32<<<nblocks(P->nleaf, 256), 256, 0, st>>>(sw.leaf_count, P->nleaf, 0);
    fmmk::k_fill_i32<<<nblocks(std::max<int64_t>(S, 1), 256), 256, 0, st>>>(sw.site_count,
                                                                            std::max<int64_t>(S, 1), 0);
    fmmk::k_fill_f64<<<1, 64, 0, st>>>(sw.dom, 8, 0.0);
    if (sw.ovf_n) fmmk::k_fill_i32<<<1, 64, 0, st>>>(sw.ovf_n, 1, 0);
    if (sw.msplit) {
        const int64_t words = (int64_t)(msplit_bytes(P, 1) / 4);
        fmmk::k_fill_i32<<<(unsigned)std::min<int64_t>(1024, (words + 255) / 256), 256, 0, st>>>(
            (int32_t*)sw.msplit, words, 0);
    }
    const Workspace own = P->ws;
    P->ws = sw;
    const RepSpan rs(&rd, 1);
    if (P->fp64)
        s = enqueue_eval<double>(P, rs, (const double*)x, (const double*)qA, (const double*)qB, site, lam,
                                 E, (double*)F, (double*)phi, dVdl);
    else
        s = enqueue_eval<float>(P, rs, (const float*)x, (const float*)qA, (const float*)qB, site, lam, E,
                                (float*)F, (float*)phi, dVdl);
    P->ws = own;
    return s;
}

fmm_status fmm_eval_adjoint(fmm_plan_t P, int64_t n, const void* x, const void* qA,
                            const void* qB, const int32_t* site, int64_t S, const double* lam,
                            const double* box, const double* gE, void* grad_x, void* grad_qA,
                            void* grad_qB, double* grad_lambda, double* E, void* F, void* phi,
                            double* dVdl) {
    fmm_status s = check_common(P, n, x, qA, qB, site, S, lam);
    if (s != FMM_OK) return s;
    if (!gE) return fail(P, FMM_E_INVALID, "null upstream weight");
    if (P->prm.hamiltonian)
        return fail(P, FMM_E_UNSUPPORTED, "the adjoint covers charge interpolation only");
    double L = 0;
    if ((s = check_box(P, box, &L)) != FMM_OK) return s;
    P->err.clear();
    std::vector<fmmk::RepDesc> rd(1);
    rd[0] = {0, n, 0, S, L, 0};
    KeyBuf key;
    key.add(2).add(rd[0]).add(x).add(qA).add(qB).add(site).add(lam).add(gE).add(grad_x)
        .add(grad_qA).add(grad_qB).add(grad_lambda).add(E).add(F).add(phi).add(dVdl);
    return run_maybe_graph(P, key.b, [&]() {
        if (P->fp64)
            return enqueue_adjoint<double>(P, rd, (const double*)x, (const double*)qA,
                                           (const double*)qB, site, lam, gE, (double*)grad_x,
                                           (double*)grad_qA, (double*)grad_qB, grad_lambda, E,
                                           (double*)F, (double*)phi, dVdl);
        return enqueue_adjoint<float>(P, rd, (const float*)x, (const float*)qA, (const float*)qB,
                                      site, lam, gE, (float*)grad_x, (float*)grad_qA,
                                      (float*)grad_qB, grad_lambda, E, (float*)F, (float*)phi, dVdl);
    });
}

// Shared validation and launch of the one-pass adjoint (weights on E, phi, F).
static fmm_status adjoint_full_entry(fmm_plan_t P, int key_tag, int64_t n, const void* x, const void* qA,
                                     const void* qB, const int32_t* site, int64_t S, const double* lam,
                                     const double* box, const double* gE_dev, double gE, const void* gphi,
                                     const void* gF, void* grad_x, void* grad_qA, void* grad_qB,
                                     double* grad_lambda, double* E, void* F, void* phi, double* dVdl) {
    fmm_status s = check_common(P, n, x, qA, qB, site, S, lam);
    if (s != FMM_OK) return s;
    if (!std::isfinite(gE)) return fail(P, FMM_E_INVALID, "non-finite upstream weight");
    if (P->prm.hamiltonian)
        return fail(P, FMM_E_UNSUPPORTED, "the adjoint covers charge interpolation only");
    double L = 0;
    if ((s = check_box(P, box, &L)) != FMM_OK) return s;
    P->err.clear();
    const fmmk::RepDesc r0{0, n, 0, S, L, 0};
    KeyBuf key;
    key.add(key_tag).add(r0).add(x).add(qA).add(qB).add(site).add(lam).add(gE_dev).add(gE).add(gphi)
        .add(gF).add(grad_x).add(grad_qA).add(grad_qB).add(grad_lambda).add(E).add(F).add(phi).add(dVdl);
    return run_maybe_graph(P, key.b, [&]() {
        if (P->fp64)
            return enqueue_adjoint_full<double>(P, r0, (const double*)x, (const double*)qA,
                                                (const double*)qB, site, lam, gE_dev, gE,
                                                (const double*)gphi, (const double*)gF, (double*)grad_x,
                                                (double*)grad_qA, (double*)grad_qB, grad_lambda, E,
                                                (double*)F, (double*)phi, dVdl);
        return enqueue_adjoint_full<float>(P, r0, (const float*)x, (const float*)qA, (const float*)qB,
                                           site, lam, gE_dev, gE, (const float*)gphi, (const float*)gF,
                                           (float*)grad_x, (float*)grad_qA, (float*)grad_qB, grad_lambda,
                                           E, (float*)F, (float*)phi, dVdl);
    });
}

fmm_status fmm_eval_adjoint_phi(fmm_plan_t P, int64_t n, const void* x, const void* qA,
                                const void* qB, const int32_t* site, int64_t S, const double* lam,
                                const double* box, double gE, const void* gphi, void* grad_x,
                                void* grad_qA, void* grad_qB, double* grad_lambda, double* E, void* F,
                                void* phi, double* dVdl) {
    if (P && !gphi) return fail(P, FMM_E_INVALID, "null potential weights");
    return adjoint_full_entry(P, 5, n, x, qA, qB, site, S, lam, box, nullptr, gE, gphi, nullptr, grad_x,
                              grad_qA, grad_qB, grad_lambda, E, F, phi, dVdl);
}

fmm_status fmm_eval_adjoint_full(fmm_plan_t P, int64_t n, const void* x, const void* qA,
                                 const void* qB, const int32_t* site, int64_t S, const double* lam,
                                 const double* box, const double* gE, const void* gphi, const void* gF,
                                 void* grad_x, void* grad_qA, void* grad_qB, double* grad_lambda,
                                 double* E, void* F, void* phi, double* dVdl) {
    return adjoint_full_entry(P, 6, n, x, qA, qB, site, S, lam, box, gE, 0.0, gphi, gF, grad_x, grad_qA,
                              grad_qB, grad_lambda, E, F, phi, dVdl);
}

fmm_status fmm_eval_batched(fmm_plan_t P, int32_t R, const int64_t* atom_off,
                            const int64_t* site_off, const void* x, const void* qA,
                            const void* qB, const int32_t* site_local, const double* lam,
                            const double* boxes, double* E, void* F, void* phi, double* dVdl) {
    if (!P) return FMM_E_INVALID;
    if (R < 1 || R > P->prm.max_replicas || !atom_off || !site_off)
        return fail(P, FMM_E_INVALID, "bad replica count or offsets");
    if (atom_off[0] != 0 || site_off[0] != 0)
        return fail(P, FMM_E_INVALID, "offsets must start at 0");
    std::vector<fmmk::RepDesc> rd((size_t)R);
    for (int r = 0; r < R; ++r) {
        const int64_t n = atom_off[r + 1] - atom_off[r], S = site_off[r + 1] - site_off[r];
        if (n < 0 || S < 0) return fail(P, FMM_E_INVALID, "offsets must be non-decreasing");
        fmm_status s = check_common(P, n, x, qA, qB, site_local, S, lam);
        if (s != FMM_OK) return s;
        double L = 0;
        if (P->prm.boundary == FMM_PERIODIC && !boxes)
            return fail(P, FMM_E_INVALID, "periodic plan needs boxes");
        if ((s = check_box(P, boxes ? boxes + 3 * r : nullptr, &L)) != FMM_OK) return s;
        rd[r] = {atom_off[r], n, site_off[r], S, L, 0};
    }
    if (atom_off[R] > P->prm.max_atoms || site_off[R] > P->prm.max_sites)
        return fail(P, FMM_E_INVALID, "total atoms or sites above the plan maxima");
    P->err.clear();
    KeyBuf key;
    key.add(3).add(R);
    for (const fmmk::RepDesc& d : rd) key.add(d);
    key.add(x).add(qA).add(qB).add(site_local).add(lam).add(E).add(F).add(phi).add(dVdl);
    return run_maybe_graph(P, key.b, [&]() {
        if (P->fp64)
            return enqueue_eval<double>(P, rd, (const double*)x, (const double*)qA,
                                        (const double*)qB, site_local, lam, E, (double*)F,
                                        (double*)phi, dVdl);
        return enqueue_eval<float>(P, rd, (const float*)x, (const float*)qA, (const float*)qB,
                                   site_local, lam, E, (float*)F, (float*)phi, dVdl);
    });
}

fmm_status fmm_eval_tautomer_batched(fmm_plan_t P, int32_t R, const int64_t* atom_off,
                                     const int64_t* site_off, const void* x, const void* qA,
                                     const void* qB, const void* qC, const void* qD,
                                     const int32_t* site_local, const double* lam_p,
                                     const double* lam_t, const double* boxes, double* E, void* F,
                                     void* phi, double* dVdl_p, double* dVdl_t) {
    if (!P) return FMM_E_INVALID;
    if (P->prm.hamiltonian)
        return fail(P, FMM_E_UNSUPPORTED, "four-form sites use charge interpolation");
    if (R < 1 || R > P->prm.max_replicas || !atom_off || !site_off)
        return fail(P, FMM_E_INVALID, "bad replica count or offsets");
    if (atom_off[0] != 0 || site_off[0] != 0)
        return fail(P, FMM_E_INVALID, "offsets must start at 0");
    std::vector<fmmk::RepDesc> rd((size_t)R);
    for (int r = 0; r < R; ++r) {
        const int64_t n = atom_off[r + 1] - atom_off[r], S = site_off[r + 1] - site_off[r];
        if (n < 0 || S < 0) return fail(P, FMM_E_INVALID, "offsets must be non-decreasing");
        fmm_status s = check_common(P, n, x, qA, qB, site_local, S, lam_p);
        if (s != FMM_OK) return s;
        if (n > 0 && (!qC || !qD)) return fail(P, FMM_E_INVALID, "null input pointer");
        if (S > 0 && !lam_t) return fail(P, FMM_E_INVALID, "null lambda pointer");
        double L = 0;
        if (P->prm.boundary == FMM_PERIODIC && !boxes)
            return fail(P, FMM_E_INVALID, "periodic plan needs boxes");
        if ((s = check_box(P, boxes ? boxes + 3 * r : nullptr, &L)) != FMM_OK) return s;
        rd[r] = {atom_off[r], n, site_off[r], S, L, 0};
    }
    if (atom_off[R] > P->prm.max_atoms || site_off[R] > P->prm.max_sites)
        return fail(P, FMM_E_INVALID, "total atoms or sites above the plan maxima");
    P->err.clear();
    KeyBuf key;
    key.add(4).add(R);
    for (const fmmk::RepDesc& d : rd) key.add(d);
    key.add(x).add(qA).add(qB).add(qC).add(qD).add(site_local).add(lam_p).add(lam_t).add(E).add(F)
        .add(phi).add(dVdl_p).add(dVdl_t);
    return run_maybe_graph(P, key.b, [&]() {
        if (P->fp64)
            return enqueue_eval<double>(P, rd, (const double*)x, (const double*)qA,
                                        (const double*)qB, site_local, lam_p, E, (double*)F,
                                        (double*)phi, dVdl_p,
                                        {(const double*)qC, (const double*)qD, lam_t}, dVdl_t);
        return enqueue_eval<float>(P, rd, (const float*)x, (const float*)qA, (const float*)qB,
                                   site_local, lam_p, E, (float*)F, (float*)phi, dVdl_p,
                                   {(const float*)qC, (const float*)qD, lam_t}, dVdl_t);
    });
}

fmm_status fmm_eval_tautomer(fmm_plan_t P, int64_t n, const void* x, const void* qA,
                             const void* qB, const void* qC, const void* qD, const int32_t* site,
                             int64_t S, const double* lam_p, const double* lam_t,
                             const double* box, double* E, void* F, void* phi, double* dVdl_p,
                             double* dVdl_t) {
    if (!P) return FMM_E_INVALID;
    if (n < 0 || S < 0) return fail(P, FMM_E_INVALID, "negative size");
    const int64_t ao[2] = {0, n}, so[2] = {0, S};
    return fmm_eval_tautomer_batched(P, 1, ao, so, x, qA, qB, qC, qD, site, lam_p, lam_t, box, E,
                                     F, phi, dVdl_p, dVdl_t);
}

fmm_status fmm_sync_check(fmm_plan_t P) {
    if (!P) return FMM_E_INVALID;
    if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(P, FMM_E_HIP, "stream sync failed");
    int32_t st[4];
    if (hipMemcpy(st, P->status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(P, FMM_E_HIP, "status read failed");
    int32_t z[4] = {0, 0, 0, 0};
    if (hipMemcpy(P->status, z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess)
        return fail(P, FMM_E_HIP, "status reset failed");
    if (st[0] & fmmk::kStatusSite) return fail(P, FMM_E_SITE, "site index outside [-1, n_sites)");
    if (st[0] & fmmk::kStatusNonFinite) return fail(P, FMM_E_NONFINITE, "non-finite input");
    if (st[0] & fmmk::kStatusCoincident)
        return fail(P, FMM_E_COINCIDENT, "two atoms at the same position (after the periodic wrap)");
    return FMM_OK;
}

fmm_status fmm_profile(fmm_plan_t P, int32_t mode, int32_t capacity, double* out) {
    if (!P) return FMM_E_INVALID;
    if (mode == 1) {
        if (capacity < 1) return fail(P, FMM_E_INVALID, "profile capacity must be >= 1");
        const size_t want = (size_t)capacity * (FMM_NPHASES + 1);
        while (P->prof_ev.size() < want) {
            hipEvent_t ev;
            if (hipEventCreate(&ev) != hipSuccess) return fail(P, FMM_E_HIP, "hipEventCreate failed");
            P->prof_ev.push_back(ev);
        }
        P->prof_phase.assign(P->prof_ev.size(), -1);
        P->prof_used = 0;
        P->prof_evals = 0;
        P->prof_on = true;
        return FMM_OK;
    }
    if (mode == 0) {
        P->prof_on = false;
        return FMM_OK;
    }
    if (mode == 2) {
        if (!out) return fail(P, FMM_E_INVALID, "null output");
        if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(P, FMM_E_HIP, "sync failed");
        for (int i = 0; i < 2 * FMM_NPHASES; ++i) out[i] = 0.0;
        for (size_t i = 0; i + 1 < P->prof_used; ++i) {
            const int ph = P->prof_phase[i];
            if (ph < 0) continue;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, P->prof_ev[i], P->prof_ev[i + 1]) != hipSuccess)
                return fail(P, FMM_E_HIP, "hipEventElapsedTime failed");
            out[ph] += ms;
            out[FMM_NPHASES + ph] += 1.0;
        }
        return FMM_OK;
    }
    return fail(P, FMM_E_INVALID, "profile mode must be 0, 1 or 2");
}

fmm_status fmm_profile_select(fmm_plan_t P, uint32_t phase_mask, int32_t every) {
    if (!P) return FMM_E_INVALID;
    if (every < 1) return fail(P, FMM_E_INVALID, "profile sampling interval must be >= 1");
    if (P->prof_on) return fail(P, FMM_E_INVALID, "select phases before fmm_profile mode 1");
    P->prof_mask = phase_mask;
    P->prof_every = every;
    return FMM_OK;
}

fmm_status fmm_plan_info(fmm_plan_t P, int64_t out[10]) {
    if (!P || !out) return FMM_E_INVALID;
    out[0] = P->m2l_mode;
    out[1] = P->m2l_mode ? P->mg.csize : 0;
    out[2] = P->m2l_mode ? P->mg.nchunk : 0;
    out[3] = P->n_tasks;
    out[4] = P->p2p_waves;
    out[5] = (int64_t)P->m2l_lds;
    out[6] = (int64_t)P->ws_bytes;
    out[7] = P->prm.graph;
    out[8] = P->p2p_split;
    out[9] = 0;
    return FMM_OK;
}

int64_t fmm_host_operator(int32_t p, int32_t which, double* out) {
    if (p < 1 || p > fmmk::kPMax || !out) return -1;
    const int64_t K = (int64_t)(p + 1) * (p + 1);
    switch (which) {
        case 0: fmmops::build_m2l_bank(p, out); return 343 * K * K;
        case 1: fmmops::build_m2m(p, out); return 8 * K * K;
        case 2: fmmops::build_l2l(p, out); return 8 * K * K;
        case 3: fmmops::build_lattice(p, out); return K * K;
        case 4: {
            double r[3] = {out[0], out[1], out[2]};
            fmmops::eval_rho(p, r, out);
            return K;
        }
        case 5: fmmops::build_periodic_green(p, out); return K;
        default: return -1;
    }
}

}  // extern "C"
