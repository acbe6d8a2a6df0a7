/*
 * fmmcph.h -- C ABI of the lambda-interpolated fast-multipole Coulomb solver
 * for gfx950 (AMD Instinct MI355X).
 *
 * What it computes (Kohnke et al., constant-pH lambda-dynamics with FMM
 * electrostatics).  Methods, eq 1: the lambda-dependent Hamiltonian
 * interpolates between the forms A and B of each titratable site, and the
 * forms differ only in their partial charges (Methods, end of the
 * lambda-dynamics subsection, and "Calibration of Protonation Dynamics", where
 * the lambda-derivative of the Hamiltonian reduces to the Coulomb term).  The
 * electrostatics are solved with the fast multipole method ("Constant pH
 * Simulations with FMM Electrostatics"), whose parameters are the multipole
 * order p and the tree depth d (section "Practical Aspects", the minimal .mdp
 * example).  For N atoms, S sites, per-atom site index s(i) (-1 = no site) and
 * per-site lambda_s this library evaluates, with charge interpolation
 *
 *   q_i       = qA_i + lambda_{s(i)} (qB_i - qA_i)        (q_i = qA_i if s(i) = -1)
 *   phi_i     = k_e sum_j' q_j psi(r_i - r_j)               potential at atom i
 *   E         = 1/2 sum_i q_i phi_i                         total Coulomb energy
 *   F_i       = -dE/dr_i                                    force on atom i
 *   dVdl_s    = sum_{i in s} (qB_i - qA_i) phi_i            = dE/dlambda_s
 *
 * psi = 1/r for open boundaries.  For periodic boundaries psi is the periodic
 * Coulomb potential with conducting (tin-foil) surroundings, a uniform
 * neutralising background for a net charge and zero mean over the cell (the
 * Ewald convention); self images are included and the i = j term removed.
 * phi is returned including k_e.  lambda is never clamped (the paper's
 * calibration grid runs from -0.1 to 1.1).
 *
 * Precision.  FMM_FP64: every array below is double and all arithmetic is
 * FP64.  FMM_MIXED_F32 / FMM_MIXED_BF16X3: x, qA, qB, F and phi are float; the
 * near field, the expansions below the root and the M2L translations run in
 * FP32 (BF16X3: M2L on bf16 matrix cores with a three-product split and FP32
 * accumulation), while the root expansions, the periodic lattice operator, the
 * energy and the dV/dlambda reductions stay in FP64.  E, lambda and dVdl are
 * always double.
 *
 * Memory and streams.  Every array argument is a DEVICE pointer owned by the
 * caller unless stated otherwise; arrays are in the caller's atom order and
 * row-major (x, F: N x 3).  The plan owns its workspace, sized at creation
 * from the fmm_params maxima; fmm_eval* allocate nothing.  Work is enqueued on
 * the plan's HIP stream and the call returns before it completes; results are
 * valid once that stream has been synchronised.  A plan is not thread-safe.
 *
 * Errors.  No exception crosses this boundary.  Arguments are validated on the
 * host before anything is enqueued; on error the call returns a non-zero
 * status, enqueues nothing and leaves the outputs untouched, and
 * fmm_last_error() describes the problem.  With params.check = 1 the kernels
 * also flag non-finite inputs, site indices outside [-1, S) and coincident
 * atoms (two atoms at one position, periodic images included: their pair term
 * is infinite); such flags are reported by fmm_sync_check().  Without check
 * the result for such inputs is undefined (a coincident pair is skipped).
 */
#ifndef FMMCPH_H
#define FMMCPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_plan_s* fmm_plan_t;

typedef enum {
    FMM_OK = 0,
    FMM_E_INVALID = 1,      /* bad argument (null pointer, size, box, parameter) */
    FMM_E_OOM = 2,          /* device allocation failed at plan creation */
    FMM_E_HIP = 3,          /* a HIP runtime call failed */
    FMM_E_UNSUPPORTED = 4,  /* valid but unsupported (non-cubic periodic box, ...) */
    FMM_E_NONFINITE = 5,    /* check mode: non-finite input seen by a kernel */
    FMM_E_SITE = 6,         /* check mode: site index outside [-1, S) */
    FMM_E_COINCIDENT = 7    /* check mode: two atoms at the same position */
} fmm_status;

typedef enum { FMM_OPEN = 0, FMM_PERIODIC = 1 } fmm_boundary;

typedef enum { FMM_FP64 = 0, FMM_MIXED_F32 = 1, FMM_MIXED_BF16X3 = 2 } fmm_precision;

/* Plan parameters.
 *   depth       tree depth d: 8^d leaf boxes (0 <= d <= 6)
 *   order_p     maximum multipole degree p: (p+1)^2 coefficients (1 <= p <= 15)
 *   boundary    fmm_boundary
 *   precision   fmm_precision
 *   coulomb_k   k_e; 1.0 for reduced units, 138.935458 for kJ mol^-1 nm e^-2
 *   max_atoms   largest N (per call, summed over replicas for the batched call)
 *   max_sites   largest S (same)
 *   max_replicas largest replica count of fmm_eval_batched (>= 1)
 *   check       1 = run the device-side input checks described above
 *   m2l_kernel  0 = automatic, 1 = plain (vector ALU) M2L, 2 = matrix-core M2L
 *               (available for p <= 10; FP64 needs p <= 8), 3 = matrix-core M2L
 *               that copies every column's source per offset even where the
 *               bf16x3 kernel could keep a class's sources resident (depth <= 3)
 *   m2l_chunk   offsets per matrix-core M2L work-group (0 = automatic, else 1..189)
 *   p2p_waves   wavefronts per near-field block: 4, 8 or 16 (0 = automatic: 4
 *               when max_atoms / (max_replicas 8^d) <= 32, else 8)
 *   p2p_split   near-field blocks per leaf, 1 to 4 (0 = 1): with more than one,
 *               block s of a leaf takes its targets 32 s .. 32 s + 31 (the last
 *               block all the rest), so the hardware can balance uneven leaves
 *   graph       1 = record the launch sequence of an evaluation in a HIP graph on
 *               first use and replay the graph while every argument (pointers,
 *               sizes, boxes, replica offsets) is unchanged; needs a non-NULL
 *               stream.  Per-phase profiling (fmm_profile) runs eagerly.
 *   hamiltonian 0 = charge interpolation (q = qA + lambda (qB - qA) in one
 *               Coulomb energy); 1 = Hamiltonian interpolation (Methods, eq 1:
 *               H = (1 - lambda) H_A + lambda H_B per site, multilinear over
 *               sites).  The two differ only inside each site: with
 *               d_i = qA_i - qB_i and psi the pair potential (1/r, or the periodic
 *               Green's function with psi(0) its self-image limit), eq 1 adds
 *                 dE_s = k_e lambda_s (1 - lambda_s) 1/2 sum_{i,j in s} d_i d_j psi(r_ij)
 *               (i = j only for periodic cells), and fmm_eval / fmm_eval_batched
 *               add dE to E, its lambda-derivative (1 - 2 lambda_s)/(lambda_s
 *               (1 - lambda_s)) dE_s to dVdl and its position derivative to F; phi
 *               stays the potential of the interpolated charges.  fmm_eval_adjoint
 *               and the four-form calls return FMM_E_UNSUPPORTED on such a plan. */
typedef struct {
    int32_t depth;
    int32_t order_p;
    int32_t boundary;
    int32_t precision;
    double coulomb_k;
    int64_t max_atoms;
    int64_t max_sites;
    int32_t max_replicas;
    int32_t check;
    int32_t m2l_kernel;
    int32_t m2l_chunk;
    int32_t p2p_waves;
    int32_t graph;
    int32_t p2p_split;
    int32_t hamiltonian;
} fmm_params;

/* Create a plan on the current HIP device.  hip_stream is a hipStream_t (NULL =
 * the default stream).  Builds the FP64 translation operators for order_p (and
 * the periodic lattice operator) on the host, uploads them, and allocates the
 * workspace.  *out receives the plan on FMM_OK. */
fmm_status fmm_plan_create(const fmm_params* params, void* hip_stream, fmm_plan_t* out);

/* One evaluation (one system).
 *   n        number of atoms (0 <= n <= max_atoms)
 *   x        n x 3 positions (nm)                       [float | double per precision]
 *   qA, qB   n charges of forms A and B (e)             [float | double]
 *   site     n site indices in [-1, n_sites)            [int32]
 *   n_sites  S (0 <= S <= max_sites)
 *   lambda   S lambda values                            [double]
 *   box      HOST pointer to 3 doubles: the periodic cell edges (must be equal:
 *            cubic cells only; positions are wrapped into [0, L)).  Must be
 *            NULL for open boundaries: the octree root is then the bounding
 *            cube of the atoms, found on the device.
 * Outputs (any of F, phi, dVdl may be NULL to skip it):
 *   E        1 double: total energy
 *   F        n x 3 forces                               [float | double]
 *   phi      n potentials (including k_e)               [float | double]
 *   dVdl     S values dE/dlambda_s                      [double] */
fmm_status fmm_eval(fmm_plan_t plan, int64_t n, const void* x, const void* qA,
                    const void* qB, const int32_t* site, int64_t n_sites,
                    const double* lambda, const double* box, double* E, void* F,
                    void* phi, double* dVdl);

/* fmm_eval for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same evaluation, arguments and results as fmm_eval, but the per-evaluation
 * workspace (sorted particles, counters, expansions, partial sums) is laid
 * out in a static device array of the library (32 MiB per GPU, held until the
 * process ends) instead of the plan's own workspace.  The call allocates
 * nothing.  It clears the counters it needs at its start (fill kernels);
 * every call on one GPU shares the array, so calls that overlap on one GPU
 * (other streams, other threads) race.  FMM_E_INVALID, with nothing
 * enqueued, when n atoms and n_sites sites on this plan need more than the
 * array holds (about 60 bytes per atom in mixed precision plus the tree's
 * expansions and partial sums, some 7 MB at depth 3, p = 8: about 400,000
 * atoms there); fmm_last_error() gives the sizes.  Never replayed from a
 * graph. */
fmm_status fmm_eval_noalloc(fmm_plan_t plan, int64_t n, const void* x, const void* qA,
                            const void* qB, const int32_t* site, int64_t n_sites,
                            const double* lambda, const double* box, double* E, void* F,
                            void* phi, double* dVdl);

/* Adjoint of E (reverse mode for an upstream weight gE on the energy).  The
 * tree and every expansion are recomputed from the inputs (nothing is kept
 * from a previous forward call).  With w = *gE (a DEVICE double):
 *   grad_x      = -w F                       n x 3   [float | double]
 *   grad_qA_i   = w (1 - lambda_s(i)) phi_i  (w phi_i if s(i) = -1)
 *   grad_qB_i   = w lambda_s(i) phi_i        (0 if s(i) = -1)
 *   grad_lambda = w dVdl                     S       [double]
 * Any gradient pointer may be NULL.  E, F, phi, dVdl are as in fmm_eval and may
 * each be NULL. */
fmm_status fmm_eval_adjoint(fmm_plan_t plan, int64_t n, const void* x, const void* qA,
                            const void* qB, const int32_t* site, int64_t n_sites,
                            const double* lambda, const double* box, const double* gE,
                            void* grad_x, void* grad_qA, void* grad_qB,
                            double* grad_lambda, double* E, void* F, void* phi,
                            double* dVdl);

/* Adjoint with upstream weights on the energy, the potentials and the forces
 * (reverse mode of the whole solve; "Coulomb interactions and their
 * derivatives" are what the paper's lambda-dynamics consumes, Methods):
 *   L = gE E + sum_i gphi_i phi_i + sum_i gF_i . F_i.
 * With phi = k_e Psi q (Psi the symmetric pair matrix of psi), F_i = k_e q_i
 * E_i(q) (E_i(c) the field of charges c at atom i), the dipoles p_j = q_j gF_j
 * and w = gF:
 *   dL/dq_i   = gE phi_i + k_e [phi_i(gphi) - phi_i(p) + w_i . E_i(q)]
 *   dL/dx_i   = -gE F_i - k_e gphi_i E_i(q)
 *               - k_e q_i [E_i(gphi) - E_i(p) - (grad E(q))_i w_i]
 *   grad_qA_i = (1 - lambda_s(i)) dL/dq_i   (dL/dq_i if s(i) = -1)
 *   grad_qB_i = lambda_s(i) dL/dq_i         (0 if s(i) = -1)
 *   grad_lambda_s = sum_{i in s} (qB_i - qA_i) dL/dq_i          [double]
 * (phi(p), E(p): potential and field of the dipoles).  One tree pass: the
 * charges and the second sources (charges gphi, dipoles -p) share the octree
 * and every translation; nothing is kept from a previous call.
 *   gE       DEVICE pointer to 1 double (NULL = 0)
 *   gphi     n weights on phi, or NULL                 [float | double, device]
 *   gF       n x 3 weights on F, or NULL               [float | double, device]
 * Any gradient pointer, and each of E, F, phi, dVdl (the forward outputs, as
 * in fmm_eval), may be NULL.  One system per call; bonded exclusions set on
 * the plan apply.  FMM_E_UNSUPPORTED on a Hamiltonian plan. */
fmm_status fmm_eval_adjoint_full(fmm_plan_t plan, int64_t n, const void* x, const void* qA,
                                 const void* qB, const int32_t* site, int64_t n_sites,
                                 const double* lambda, const double* box, const double* gE,
                                 const void* gphi, const void* gF, void* grad_x, void* grad_qA,
                                 void* grad_qB, double* grad_lambda, double* E, void* F, void* phi,
                                 double* dVdl);

/* fmm_eval_adjoint_full with gF = NULL and the energy weight gE given as a
 * HOST double; gphi must be non-NULL. */
fmm_status fmm_eval_adjoint_phi(fmm_plan_t plan, int64_t n, const void* x, const void* qA,
                                const void* qB, const int32_t* site, int64_t n_sites,
                                const double* lambda, const double* box, double gE,
                                const void* gphi, void* grad_x, void* grad_qA, void* grad_qB,
                                double* grad_lambda, double* E, void* F, void* phi, double* dVdl);

/* R independent systems (replicas) in one call.  Atoms and sites of replica r
 * occupy [atom_off[r], atom_off[r+1]) and [site_off[r], site_off[r+1]) of the
 * concatenated arrays; atom_off and site_off are HOST arrays of R+1 int64
 * (atom_off[0] = site_off[0] = 0).  site_local holds site indices local to the
 * atom's replica.  boxes is a HOST array of R x 3 doubles for periodic plans
 * and must be NULL for open ones.  E receives R doubles; F, phi, dVdl are the
 * concatenated per-replica outputs.  Each replica equals what fmm_eval returns
 * for it alone. */
fmm_status fmm_eval_batched(fmm_plan_t plan, int32_t R, const int64_t* atom_off,
                            const int64_t* site_off, const void* x, const void* qA,
                            const void* qB, const int32_t* site_local,
                            const double* lambda, const double* boxes, double* E,
                            void* F, void* phi, double* dVdl);

/* Four-form sites (protonation tautomers; Methods, eq 2, in charge-
 * interpolated form).  Every site s carries two coordinates, lambda_p[s]
 * (protonation) and lambda_t[s] (tautomer), and its atoms carry four charge
 * forms A, B, C, D; with u~ := 1 - u,
 *   q_i = lp~ (lt~ qA_i + lt qB_i) + lp (lt~ qC_i + lt qD_i)   (s(i) >= 0)
 *   q_i = qA_i                                                 (s(i) = -1)
 * and the two site derivatives of V = E are
 *   dVdl_p[s] = sum_{i in s} phi_i (lt~ (qC_i - qA_i) + lt (qD_i - qB_i))
 *   dVdl_t[s] = sum_{i in s} phi_i (lp~ (qB_i - qA_i) + lp (qD_i - qC_i))
 * (phi including k_e).  A site without tautomers is qB = qA and qD = qC: then
 * q and dVdl_p are those of fmm_eval with forms (qA, qC) and lambda_p, and
 * dVdl_t = 0.  qC and qD have the type of qA; lambda_t has S doubles; dVdl_t
 * receives S doubles (either derivative pointer may be NULL).  Everything else
 * (arguments, ownership, errors, asynchrony) is as in fmm_eval and
 * fmm_eval_batched. */
fmm_status fmm_eval_tautomer(fmm_plan_t plan, int64_t n, const void* x, const void* qA,
                             const void* qB, const void* qC, const void* qD,
                             const int32_t* site, int64_t n_sites, const double* lambda_p,
                             const double* lambda_t, const double* box, double* E, void* F,
                             void* phi, double* dVdl_p, double* dVdl_t);
fmm_status fmm_eval_tautomer_batched(fmm_plan_t plan, int32_t R, const int64_t* atom_off,
                                     const int64_t* site_off, const void* x, const void* qA,
                                     const void* qB, const void* qC, const void* qD,
                                     const int32_t* site_local, const double* lambda_p,
                                     const double* lambda_t, const double* boxes, double* E,
                                     void* F, void* phi, double* dVdl_p, double* dVdl_t);

/* Wait for the plan's stream and report device-side check flags raised since
 * the previous call (FMM_E_NONFINITE, FMM_E_SITE, FMM_E_COINCIDENT), or FMM_E_HIP. */
fmm_status fmm_sync_check(fmm_plan_t plan);

/* Human-readable description of the last error on this plan (never NULL). */
const char* fmm_last_error(fmm_plan_t plan);

/* Bonded exclusions (not in the paper: MD topologies exclude the Coulomb
 * terms of bonded neighbours).  start[0..n] (ascending, start[0] = 0) and
 * idx[start[i] .. start[i+1]) list the excluded partners of atom i: host
 * arrays, copied to the device now (this call allocates, and waits for the
 * plan's stream before replacing lists already set; evaluations allocate
 * nothing).  Every list ascends without repeats, never names i itself, and each
 * pair appears from both sides.  From then on every evaluation of this plan
 * (single, batched with n = the total atom count, four-form, adjoint) removes
 * the listed pairs' terms: k_e q_j / r from phi_i, their force from F_i and
 * energy from E, and the matching site terms from dV/dlambda, with r the
 * minimum-image distance for a periodic cell (the pair's other images stay);
 * partners in another replica are skipped.  An evaluation whose total atom
 * count differs from n returns FMM_E_INVALID.  n = 0 removes the lists.
 * FMM_E_UNSUPPORTED on a Hamiltonian plan; FMM_E_INVALID for a malformed
 * list (nothing changes); FMM_E_OOM / FMM_E_HIP if the upload fails (the
 * plan is left without exclusions). */
fmm_status fmm_set_exclusions(fmm_plan_t plan, int64_t n, const int32_t* start, const int32_t* idx);

/* Release the plan and its device workspace (NULL is ignored). */
void fmm_plan_destroy(fmm_plan_t plan);

/* Per-phase timing with HIP events recorded on the plan's stream (a
 * measurement aid; it changes no result).  The phases of one evaluation are
 *   0 binning (leaf keys, counting sort), 1 leaf sort + gather (interpolated
 *   charges) + P2M,
 *   2 M2M with the periodic root and lattice operator (one launch),
 *   3 root of a depth-0 periodic tree (empty otherwise), 4 M2L, 5 L2L,
 *   6 near field + far-field evaluation + outputs (P2P, L2P), 7 reductions.
 * mode 1: start recording for up to `capacity` evaluations (creates the events
 *         now, never inside an evaluation; resets the record),
 * mode 0: stop recording,
 * mode 2: wait for the stream and write out[0..7] = total milliseconds per
 *         phase and out[8..15] = number of timed instances of each phase. */
#define FMM_NPHASES 8
fmm_status fmm_profile(fmm_plan_t plan, int32_t mode, int32_t capacity, double* out);

/* Restrict the events fmm_profile records (each event is a marker in the
 * stream and costs a few microseconds of GPU time): only the boundaries of
 * the phases whose bit is set in phase_mask, and only on every `every`-th
 * evaluation (1 = all), counted from fmm_profile mode 1.  Call before mode 1;
 * the default is all phases on every evaluation.  Returns FMM_E_INVALID for
 * every < 1 or while recording. */
fmm_status fmm_profile_select(fmm_plan_t plan, uint32_t phase_mask, int32_t every);

/* Resolved launch configuration of a plan (host only, no GPU work):
 *   out[0] M2L kernel (0 plain, 1 FP32, 2 FP64, 3 bf16x3 matrix cores)
 *   out[1] offsets per M2L work-group   out[2] offset chunks
 *   out[3] M2L work-groups per replica  out[4] wavefronts per near-field block
 *   out[5] M2L LDS bytes per work-group out[6] device workspace bytes
 *   out[7] graph replay enabled         out[8] near-field blocks per leaf
 *   out[9] zero (reserved) */
fmm_status fmm_plan_info(fmm_plan_t plan, int64_t out[10]);

/* Host-only access to the FP64 operator tables a plan of order p uploads; no
 * GPU is touched.  which: 0 = M2L bank (343 x K x K), 1 = M2M (8 x K x K),
 * 2 = L2L (8 x K x K), 3 = periodic lattice operator (K x K), 4 = regular
 * harmonics rho(r) at the point out[0..2] (K values, written over out).
 * 5 = real local coefficients of the smooth part h of the unit cube's periodic
 * Green's function, psi(u) = sum_{n in {-1,0,1}^3} 1/|u+n| + (2 pi/3)|u|^2 + h(u)
 * (K values; degree p).
 * Layouts as documented in the library's operators.h; K = (p+1)^2.  Returns
 * the number of doubles written, or -1 for a bad argument. */
int64_t fmm_host_operator(int32_t order_p, int32_t which, double* out);

/* ---- lambda dynamics around the solve ------------------------------------
 * The lambda coordinates of R replicas are one FP64 array of C entries;
 * replica r owns [coord_off[r], coord_off[r+1]) (device int32 array of R + 1
 * ascending offsets in [0, C]; entries outside are clamped into it).  Units:
 * energies kJ/mol (run the solve with coulomb_k = 138.935458 so that its
 * dV/dlambda is in kJ/mol), mass u, time ps, temperature K.  All pointers are
 * device pointers owned by the caller; nothing is allocated.  The calls
 * validate their arguments on the host (FMM_E_INVALID, nothing enqueued),
 * enqueue one launch on hip_stream and return FMM_E_HIP if the launch fails.
 * The bias of coordinate c (Methods, eq 3) is V_MM + V_pH + V_dw:
 *   V_MM: dV_MM/dlambda = -G(lambda_c, lambda_partner), the negated fit of the
 *         reference compound's mean dH/dlambda ("Calibration of Protonation
 *         Dynamics"), G = sum_{i,j=0..5} mm[36 c + 6 i + j] lambda_c^i
 *         lambda_partner^j (lambda_partner = 0 when partner[c] < 0 or partner
 *         is NULL; mm NULL = no V_MM);
 *   V_pH = lambda ln(10) k_B T (pKa[c] - pH[r]) (eq 4 with a linear profile;
 *         pKa NaN or pka NULL = none, as for tautomer coordinates);
 *   V_dw: cubic Hermite spline through the knots (p0 - 0.3, 30), (p0, 0),
 *         ((p0 + p1)/2, B), (p1, y1), (p1 + 0.3, y1 + 30) with slopes -300, 0,
 *         0, 0, 300 per unit lambda, continued linearly beyond the end knots
 *         plus a confining 10^4 d^2 (d the distance past the end knot), from
 *         dwp[4 c ..] = (B, p0, p1, y1) (dwp NULL = none).
 * Tautomer coordinates (pKa NaN and a partner, the site's protonation
 * coordinate) may carry a second barrier: with dwp2 (C x 2, NULL = none),
 * V_dw takes (B, y1) = (dwp2[2 c], dwp2[2 c + 1]) instead while the site is
 * deprotonated, lambda_partner >= 1/2 (lambda = 0 is protonated; "Dynamic
 * Barrier and Well Optimization": the tautomeric force nearly vanishes in one
 * protonation state, so its barrier is tuned separately); the wells p0, p1
 * are shared.  The switch is a step in lambda_partner: it adds no force on
 * the partner. */
typedef struct {
    double mass;         /* lambda-particle mass, u (the paper uses 60) */
    double dt;           /* time step, ps */
    double temperature;  /* K */
    double tau;          /* Bussi coupling time, ps; <= 0 = no thermostat */
    double near0;        /* DBO statistics: lambda < near0 is near well 0 (0.2) */
    double near1;        /* lambda > near1 is near well 1 (0.8) */
} fmm_lambda_params;

/* One velocity-Verlet step of the lambda particles ("Constant pH
 * Parameters"), with the forces -dH/dlambda at lambda (eq 1: dvdl[c] is the
 * solve's dV_Coul/dlambda for coordinate c, plus the bias above):
 *   v_n = v + dt/2 F/m (omitted when first = 1: v is then the full-step v_n);
 *   v_n *= alpha per replica, the Bussi-Donadio-Parrinello rescaling of the
 *        replica's lambda kinetic energy K (N_f = its coordinate count) with
 *        c = exp(-dt/tau), K' = K + (1-c)(K_bar (R1^2 + X)/N_f - K)
 *        + 2 R1 sqrt(c (1-c) K K_bar / N_f), K_bar = N_f k_B T / 2,
 *        alpha = sqrt(K'/K) (skipped for tau <= 0, N_f = 0 or K = 0); R1 =
 *        noise[2 r] is a standard normal and X = noise[2 r + 1] a chi-square
 *        sample with N_f - 1 degrees of freedom, drawn by the caller;
 *   v = v_n + dt/2 F/m (written back, the half-step velocity) and
 *   lam_new = lam + dt v (lam_new must not alias lam).
 * kin[r] (optional) receives K before the rescaling, e_bias[r] (optional)
 * the sum of V_pH + V_dw at lam.  stats_w (C x 5: steps, steps near 0, sum of
 * lambda near 0, steps near 1, sum near 1) and stats_b (C x 2: steps, steps
 * with near0 <= lambda <= near1), both optional, accumulate the DBO block
 * statistics of lam; with stats_b2 (C x 2, needs dwp2 and stats_b) the
 * barrier statistics of tautomer coordinates in their second state go there
 * instead.  dwp2 needs dwp and partner. */
fmm_status fmm_lambda_step(void* hip_stream, int32_t R, const int32_t* coord_off, int64_t C,
                           const fmm_lambda_params* prm, int32_t first, const double* lam,
                           double* lam_new, double* v, const double* dvdl, const int32_t* partner,
                           const double* pka, const double* ph, const double* mm, const double* dwp,
                           const double* noise, double* stats_w, double* stats_b, double* kin,
                           double* e_bias, const double* dwp2, double* stats_b2);

/* Dynamic Barrier and Well Optimization ("Dynamic Barrier and Well
 * Optimization"); NULL = the paper's values {0.2, 0.8, 0.7, 0.03, 0.5, 0.08,
 * 0.25, 0.05, 1.0, 1.0, 20.0} in field order. */
typedef struct {
    double near0, near1;   /* thresholds of the well statistics (the step's) */
    double occupancy;      /* fraction of a block near a well before it moves */
    double well_tol;       /* |mean - ideal| that moves a well */
    double well_gain;      /* the well moves by -well_gain (mean - ideal) */
    double max_shift;      /* |well - ideal end point| <= max_shift */
    double target;         /* in-transition fraction aimed for */
    double target_tol;     /* dead band around it */
    double barrier_step;   /* kJ/mol per adjustment */
    double barrier_min, barrier_max;
} fmm_dbo_params;

/* At the end of a DBO block: mode bit 0 applies the well rule from stats_w,
 * bit 1 the barrier rule from stats_b, to dwp (in place), and clears the
 * statistics it used.  With pfc = 1 every coordinate whose well or barrier
 * moved gets the partition function correction below.  adjusted[c]
 * (optional) is set to 1 for a moved coordinate, else 0 (for censoring the
 * trajectory after a change).  With dwp2 (then partner, and stats_b2 for
 * mode bit 1, are required) a tautomer coordinate's second barrier moves by
 * the same rule from stats_b2, and the correction also gives the second
 * state its own y1 (dwp2[2 c + 1]). */
fmm_status fmm_lambda_dbo(void* hip_stream, int32_t R, const int32_t* coord_off, int64_t C,
                          int32_t mode, int32_t pfc, const fmm_dbo_params* prm, double temperature,
                          const double* pka, const double* ph, double* dwp, double* stats_w,
                          double* stats_b, int32_t* adjusted, const int32_t* partner, double* dwp2,
                          double* stats_b2);

/* Partition function correction ("Partition Function Correction") of every
 * coordinate: sets y1 = dwp[4 c + 3] so that the free energy of
 * deprotonation -k_B T ln(Z_1 / Z_0) of V_pH + V_dw, Z_0 and Z_1 the integrals
 * of exp(-(V_pH + V_dw)/k_B T) over [0, 1/2] and [1/2, 1], equals
 * ln(10) k_B T (pKa - pH) (0 without pKa); Gauss-Legendre quadrature on the
 * spline pieces and a safeguarded regula falsi on y1 in [-200, 200] kJ/mol.  The free energy
 * grows with y1 but is bounded (the barrier-top part of [1/2, 1] does not
 * move with y1): a target out of reach leaves y1 at the nearer end.  With
 * dwp2 (and partner) tautomer coordinates also get y1 of their second state,
 * from (dwp2[2 c], p0, p1). */
fmm_status fmm_lambda_pfc(void* hip_stream, int32_t R, const int32_t* coord_off, int64_t C,
                          double temperature, const double* pka, const double* ph, double* dwp,
                          const int32_t* partner, double* dwp2);

#ifdef __cplusplus
}
#endif

#endif /* FMMCPH_H */
