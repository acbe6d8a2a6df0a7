// Lambda-dynamics step around the Coulomb solve: the bias potentials of the
// lambda coordinates, velocity Verlet with the Bussi-Donadio-Parrinello
// thermostat, the DBO block statistics and rules, and the partition function
// correction (constant-pH paper, Methods: eq 1, eq 3, eq 4, "Partition
// Function Correction", "Dynamic Barrier and Well Optimization", "Constant pH
// Parameters").  All arithmetic is FP64.  The step runs one work-group per
// replica (its lambda coordinates are a contiguous range), DBO and the
// correction one wavefront per coordinate.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fmmcph.h"

namespace fmml {

constexpr double kKB = 8.314462618e-3;  // kJ mol^-1 K^-1
constexpr double kLn10 = 2.302585092994045684;
// synthetic double-well shape: wall knots 0.3 from each well, 30 kJ/mol above
// it, slope 300 kJ/mol per unit lambda; past them the linear continuation
// gains a confining (kWallK / 2) d^2, d the distance past the end knot
constexpr double kWallDx = 0.3, kWallDy = 30.0, kWallSlope = 300.0, kWallK = 2.0e4;
constexpr int kThreads = 256;
constexpr int kGL = 16;     // Gauss-Legendre points per panel
constexpr int kPanels = 4;  // panels per smooth piece of the PFC integrands

struct GaussLegendre {
    double x[kGL], w[kGL];  // nodes and weights on [-1, 1]
};

// Five knots (x, value, slope): wall, well 0 at p0 (height 0), barrier top B
// midway between the wells, well 1 at p1 (height y1), wall.
struct Knots {
    double x[5], y[5], s[5];
};

__device__ Knots dw_knots(double B, double p0, double p1, double y1) {
    Knots k;
    k.x[0] = p0 - kWallDx; k.y[0] = kWallDy;       k.s[0] = -kWallSlope;
    k.x[1] = p0;           k.y[1] = 0.0;           k.s[1] = 0.0;
    k.x[2] = 0.5 * (p0 + p1); k.y[2] = B;          k.s[2] = 0.0;
    k.x[3] = p1;           k.y[3] = y1;            k.s[3] = 0.0;
    k.x[4] = p1 + kWallDx; k.y[4] = y1 + kWallDy;  k.s[4] = kWallSlope;
    return k;
}

// Cubic Hermite interpolation through the knots, linear with the end slopes
// outside them: value and derivative at t.
__device__ void hermite(const Knots& k, double t, double& V, double& dV) {
    if (t < k.x[0]) {
        V = k.y[0] + k.s[0] * (t - k.x[0]);
        dV = k.s[0];
        return;
    }
    if (t > k.x[4]) {
        V = k.y[4] + k.s[4] * (t - k.x[4]);
        dV = k.s[4];
        return;
    }
    int i = 0;
    while (i < 3 && t >= k.x[i + 1]) ++i;
    const double h = k.x[i + 1] - k.x[i];
    const double u = (t - k.x[i]) / h, u2 = u * u, u3 = u2 * u;
    const double y0 = k.y[i], y1 = k.y[i + 1], m0 = h * k.s[i], m1 = h * k.s[i + 1];
    V = (2 * u3 - 3 * u2 + 1) * y0 + (u3 - 2 * u2 + u) * m0 + (-2 * u3 + 3 * u2) * y1 + (u3 - u2) * m1;
    dV = ((6 * u2 - 6 * u) * y0 + (3 * u2 - 4 * u + 1) * m0 + (-6 * u2 + 6 * u) * y1 + (3 * u2 - 2 * u) * m1) / h;
}

// V_dw and its derivative: the spline plus the confining walls.
__device__ void double_well(const Knots& k, double t, double& V, double& dV) {
    hermite(k, t, V, dV);
    const double past = fmin(t - k.x[0], 0.0) + fmax(t - k.x[4], 0.0);
    V += 0.5 * kWallK * past * past;
    dV += kWallK * past;
}

struct StepArgs {
    const int32_t* coord_off;
    int64_t C;
    fmm_lambda_params prm;
    int first;
    const double* lam;
    double* lam_new;
    double* v;
    const double* dvdl;
    const int32_t* partner;
    const double* pka;
    const double* ph;
    const double* mm;
    const double* dwp;
    const double* noise;
    double* stats_w;
    double* stats_b;
    double* kin;
    double* e_bias;
    const double* dwp2;  // tautomer coordinates: (B2, y1_2) of the deprotonated state, or null
    double* stats_b2;    // their barrier statistics in that state, or null
};

// A tautomer coordinate (no pKa, a partner: the site's protonation
// coordinate) uses its second barrier set while the site is deprotonated
// (partner lambda >= 1/2; lambda = 0 is protonated).
// Evaluated without per-lane early exits: every load is in bounds (an
// invalid partner reads the coordinate's own lambda) and the answer is one
// predicate.
__device__ __forceinline__ bool second_state(const StepArgs& A, int64_t c) {
    if (!A.dwp2 || !A.partner) return false;
    const int32_t pc = A.partner[c];
    const bool paired = pc >= 0 && pc < A.C;
    const bool no_pka = !A.pka || isnan(A.pka[c]);
    const double lp = A.lam[paired ? (int64_t)pc : c];
    return paired && no_pka && lp >= 0.5;
}

__device__ __forceinline__ void replica_range(const int32_t* off, int64_t C, int r, int64_t& a, int64_t& b) {
    a = min<int64_t>(max<int64_t>(off[r], 0), C);
    b = min<int64_t>(max<int64_t>(off[r + 1], a), C);
}

// Force -dH/dlambda on coordinate c (eq 1, eq 3): the Coulomb derivative from
// the solve, V_MM (minus the fitted mean dH_ref/dlambda, a degree-5 polynomial
// in the coordinate and its partner), V_pH (linear, eq 4) and V_dw; eb gets
// V_pH + V_dw.
__device__ double lambda_force(const StepArgs& A, int64_t c, double ph_r, double& eb) {
    const double l = A.lam[c];
    double dH = A.dvdl[c];
    if (A.mm) {
        const int32_t pc = A.partner ? A.partner[c] : -1;
        const double y = (pc >= 0 && pc < A.C) ? A.lam[pc] : 0.0;
        const double* g = A.mm + 36 * c;
        double G = 0.0, li = 1.0;
        for (int i = 0; i < 6; ++i) {
            double row = 0.0, yj = 1.0;
            for (int j = 0; j < 6; ++j) {
                row += g[6 * i + j] * yj;
                yj *= y;
            }
            G += row * li;
            li *= l;
        }
        dH -= G;
    }
    eb = 0.0;
    if (A.pka) {
        const double pk = A.pka[c];
        if (!isnan(pk)) {
            const double s = kLn10 * kKB * A.prm.temperature * (pk - ph_r);
            dH += s;
            eb += s * l;
        }
    }
    if (A.dwp) {
        const double* d = A.dwp + 4 * c;
        const bool sec = second_state(A, c);
        const double B = sec ? A.dwp2[2 * c] : d[0], y1 = sec ? A.dwp2[2 * c + 1] : d[3];
        double V, dV;
        double_well(dw_knots(B, d[1], d[2], y1), l, V, dV);
        dH += dV;
        eb += V;
    }
    return -dH;
}

// Fixed-order block sum of two values (result in thread 0): a shuffle tree
// per wavefront, then the wavefront sums in order.
__device__ void block_sum2(double& a, double& b) {
    __shared__ double sa[kThreads / 64], sb[kThreads / 64];
    const int t = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    if ((t & 63) == 0) {
        sa[t >> 6] = a;
        sb[t >> 6] = b;
    }
    __syncthreads();
    if (t == 0) {
        a = sa[0];
        b = sb[0];
        for (int w = 1; w < kThreads / 64; ++w) {
            a += sa[w];
            b += sb[w];
        }
    }
}

// One velocity-Verlet step of replica blockIdx.x with the forces at lambda_n:
// closing half kick (unless first), Bussi rescaling of the full-step
// velocities, half kick, drift into lam_new.  A thread keeps the force and
// full-step velocity of its first kKeep coordinates in registers; further
// coordinates evaluate the force again after the kinetic-energy sum (from the
// unmodified inputs, so both evaluations agree).
constexpr int kKeep = 4;
__global__ __launch_bounds__(kThreads) void k_lambda_step(StepArgs A) {
    const int r = blockIdx.x, t = threadIdx.x;
    int64_t a, b;
    replica_range(A.coord_off, A.C, r, a, b);
    const double ph_r = A.ph[r];
    const double hm = 0.5 * A.prm.dt / A.prm.mass;
    double K = 0.0, E = 0.0;
    double keepF[kKeep], keepV[kKeep];
    int m = 0;
    for (int64_t c = a + t; c < b; c += kThreads, ++m) {
        double eb;
        const double F = lambda_force(A, c, ph_r, eb);
        double v = A.v[c];
        if (!A.first) v += hm * F;
#pragma unroll
        for (int k = 0; k < kKeep; ++k)
            if (k == m) {
                keepF[k] = F;
                keepV[k] = v;
            }
        K += 0.5 * A.prm.mass * v * v;
        E += eb;
        const double l = A.lam[c];
        if (A.stats_w) {
            double* s = A.stats_w + 5 * c;
            const bool n0 = l < A.prm.near0, n1 = l > A.prm.near1;
            s[0] += 1.0;
            if (n0) {
                s[1] += 1.0;
                s[2] += l;
            }
            if (n1) {
                s[3] += 1.0;
                s[4] += l;
            }
        }
        if (A.stats_b) {
            // tautomer coordinates in their second state count into stats_b2.
            // Both arrays take a masked increment (adding 0 is exact) instead
            // of one update through a per-lane choice of array: hipcc
            // (ROCm 7.2, -O3) lost the choice of array in that form, sending
            // every paired coordinate to stats_b2.
            const double tr = (!(l < A.prm.near0) && !(l > A.prm.near1)) ? 1.0 : 0.0;
            const double u = (A.stats_b2 && second_state(A, c)) ? 1.0 : 0.0;
            A.stats_b[2 * c] += 1.0 - u;
            A.stats_b[2 * c + 1] += (1.0 - u) * tr;
            if (A.stats_b2) {
                A.stats_b2[2 * c] += u;
                A.stats_b2[2 * c + 1] += u * tr;
            }
        }
    }
    block_sum2(K, E);
    __shared__ double alpha_s;
    if (t == 0) {
        double alpha = 1.0;
        const int64_t nf = b - a;
        if (A.prm.tau > 0.0 && nf > 0 && K > 0.0) {
            const double kbar = 0.5 * (double)nf * kKB * A.prm.temperature;
            const double cc = exp(-A.prm.dt / A.prm.tau);
            const double R1 = A.noise[2 * r], chi2 = A.noise[2 * r + 1];
            const double Kn = K + (1.0 - cc) * (kbar * (R1 * R1 + chi2) / (double)nf - K) +
                              2.0 * R1 * sqrt(K * kbar / (double)nf * (1.0 - cc) * cc);
            alpha = sqrt(fmax(Kn, 0.0) / K);
        }
        alpha_s = alpha;
        if (A.kin) A.kin[r] = K;
        if (A.e_bias) A.e_bias[r] = E;
    }
    __syncthreads();
    const double alpha = alpha_s;
    m = 0;
    for (int64_t c = a + t; c < b; c += kThreads, ++m) {
        double F = 0.0, v = 0.0;
        bool kept = false;
#pragma unroll
        for (int k = 0; k < kKeep; ++k)
            if (k == m) {
                F = keepF[k];
                v = keepV[k];
                kept = true;
            }
        if (!kept) {
            double eb;
            F = lambda_force(A, c, ph_r, eb);
            v = A.v[c];
            if (!A.first) v += hm * F;
        }
        v = v * alpha + hm * F;
        A.v[c] = v;
        A.lam_new[c] = A.lam[c] + A.prm.dt * v;
    }
}

// Free energy of deprotonation -k_B T ln(Z_deprot / Z_prot) of V_pH + V_dw,
// Z over [0, 1/2] and [1/2, 1]: Gauss-Legendre on kPanels panels of every
// piece between the knots that fall inside.  One wavefront: lane l takes the
// quadrature points l, l + 64, ...; the lane sums are added in a fixed tree
// and lane 0's total is broadcast, so every lane returns the same value.
__device__ double pfc_dg(const Knots& k, double slope, double beta, const GaussLegendre& gl) {
    const int lane = threadIdx.x & 63;
    double z[2];
    for (int h = 0; h < 2; ++h) {
        const double lo = 0.5 * h, hi = lo + 0.5;
        double cuts[7];
        int n = 0;
        cuts[n++] = lo;
        for (int i = 0; i < 5; ++i)
            if (k.x[i] > lo && k.x[i] < hi) cuts[n++] = k.x[i];  // knots ascend
        cuts[n++] = hi;
        const int per_piece = kPanels * kGL, npts = (n - 1) * per_piece;
        double sum = 0.0;
        for (int j = lane; j < npts; j += 64) {
            const int p = j / per_piece, q = (j % per_piece) / kGL, g = j % kGL;
            const double w = (cuts[p + 1] - cuts[p]) / kPanels, hw = 0.5 * w;
            const double x = cuts[p] + q * w + hw + hw * gl.x[g];
            double V, dV;
            double_well(k, x, V, dV);
            sum += hw * gl.w[g] * exp(-beta * (V + slope * x));
        }
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
        z[h] = __shfl(sum, 0, 64);
    }
    return -log(z[1] / z[0]) / beta;
}

// y1 for which the free energy of deprotonation of V_pH + V_dw equals
// ln(10) k_B T (pKa - pH) (0 without pKa), searched in [-200, 200] kJ/mol
// (the free energy increases with y1; a target out of reach leaves y1 at the
// nearer end).  Safeguarded regula falsi: Illinois steps (the retained end's
// residual halved when the same end is kept twice) alternate with bisection
// steps, so every two steps at least halve the bracket; it stops on the
// bracket width alone (below 1e-11 kJ/mol; a residual test would not bound the
// error in y1 where the free energy saturates and its slope in y1 is small),
// or on an exact zero; wave-uniform (every lane holds the same residuals).
__device__ double pfc_solve(double B, double p0, double p1, double pk, double ph_r, double T,
                            const GaussLegendre& gl) {
    const double beta = 1.0 / (kKB * T);
    const double slope = isnan(pk) ? 0.0 : kLn10 * kKB * T * (pk - ph_r);
    const double target = slope;  // V_pH(1) - V_pH(0)
    auto resid = [&](double y1) { return pfc_dg(dw_knots(B, p0, p1, y1), slope, beta, gl) - target; };
    double lo = -200.0, hi = 200.0;
    double glo = resid(lo), ghi = resid(hi);
    if (glo >= 0.0) return lo;
    if (ghi <= 0.0) return hi;
    int side = 0;  // end kept by the last step: -1 lo, +1 hi
    for (int it = 0; it < 200 && hi - lo > 1e-11; ++it) {
        double x = (it & 1) ? 0.5 * (lo + hi) : (lo * ghi - hi * glo) / (ghi - glo);
        if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
        if (x <= lo || x >= hi) break;  // no representable point inside
        const double gx = resid(x);
        if (gx == 0.0) return x;
        if (gx < 0.0) {
            lo = x;
            glo = gx;
            if (side == 1) ghi *= 0.5;
            side = 1;
        } else {
            hi = x;
            ghi = gx;
            if (side == -1) glo *= 0.5;
            side = -1;
        }
    }
    return (lo * ghi - hi * glo) / (ghi - glo);
}

struct DboArgs {
    const int32_t* coord_off;
    int R;
    int64_t C;
    int mode, pfc, all;  // all: correct every coordinate (no rules)
    fmm_dbo_params prm;
    double T;
    const double* pka;
    const double* ph;
    double* dwp;
    double* stats_w;
    double* stats_b;
    int32_t* adjusted;
    const int32_t* partner;  // with dwp2: the protonation partner of each coordinate
    double* dwp2;            // tautomer coordinates: (B2, y1_2), or null
    double* stats_b2;
};

constexpr int kDboWaves = 4;

// DBO rules at the end of a block (mode bit 0: wells from stats_w, bit 1:
// barrier from stats_b), then the partition function correction of every
// adjusted coordinate; the used statistics are cleared.  One wavefront per
// coordinate: every lane evaluates the rules on the same values (uniform
// branches), lane 0 writes, all lanes share the quadrature.
__global__ __launch_bounds__(64 * kDboWaves) void k_lambda_dbo(DboArgs A, GaussLegendre gl) {
    const int64_t c = (int64_t)blockIdx.x * kDboWaves + (threadIdx.x >> 6);
    const bool w0 = (threadIdx.x & 63) == 0;
    if (c >= A.C) return;  // whole wavefront
    // replica of c: the last r with (clamped) coord_off[r] <= c
    int lo = 0, hi = A.R;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (min<int64_t>(max<int64_t>(A.coord_off[mid], 0), A.C) <= c) lo = mid;
        else hi = mid;
    }
    int64_t a, b;
    replica_range(A.coord_off, A.C, lo, a, b);
    if (c < a || c >= b) return;  // outside every replica's range
    const double ph_r = A.ph[lo];
    const fmm_dbo_params& P = A.prm;
    double d[4] = {A.dwp[4 * c], A.dwp[4 * c + 1], A.dwp[4 * c + 2], A.dwp[4 * c + 3]};
    bool adj = false;
    if (A.mode & 1) {
        double* s = A.stats_w + 5 * c;
        const double s0 = s[0], cnt[2] = {s[1], s[3]}, tot[2] = {s[2], s[4]};
        if (s0 > 0.0) {
            for (int w = 0; w < 2; ++w) {
                if (cnt[w] > P.occupancy * s0) {
                    const double dev = tot[w] / cnt[w] - (double)w;
                    if (fabs(dev) > P.well_tol) {
                        const double pos = d[1 + w] - P.well_gain * dev;
                        const double nw = fmin(fmax(pos, (double)w - P.max_shift), (double)w + P.max_shift);
                        if (nw != d[1 + w]) {
                            d[1 + w] = nw;
                            adj = true;
                        }
                    }
                }
            }
        }
        if (w0)
            for (int k = 0; k < 5; ++k) s[k] = 0.0;
    }
    if (A.mode & 2) {
        double* s = A.stats_b + 2 * c;
        const double s0 = s[0], s1 = s[1];
        if (s0 > 0.0) {
            const double frac = s1 / s0;
            double B = d[0];
            if (frac < P.target - P.target_tol) B -= P.barrier_step;
            else if (frac > P.target + P.target_tol) B += P.barrier_step;
            B = fmin(fmax(B, P.barrier_min), P.barrier_max);
            if (B != d[0]) {
                d[0] = B;
                adj = true;
            }
        }
        if (w0) {
            s[0] = 0.0;
            s[1] = 0.0;
        }
    }
    // tautomer coordinate with a second barrier (the deprotonated state's)
    const double pk = A.pka ? A.pka[c] : NAN;
    const bool taut = A.dwp2 && A.partner && A.partner[c] >= 0 && A.partner[c] < A.C && isnan(pk);
    double d2[2] = {taut ? A.dwp2[2 * c] : 0.0, taut ? A.dwp2[2 * c + 1] : 0.0};
    if (taut && (A.mode & 2) && A.stats_b2) {
        double* s = A.stats_b2 + 2 * c;
        const double s0 = s[0], s1 = s[1];
        if (s0 > 0.0) {
            const double frac = s1 / s0;
            double B = d2[0];
            if (frac < P.target - P.target_tol) B -= P.barrier_step;
            else if (frac > P.target + P.target_tol) B += P.barrier_step;
            B = fmin(fmax(B, P.barrier_min), P.barrier_max);
            if (B != d2[0]) {
                d2[0] = B;
                adj = true;
            }
        }
        if (w0) {
            s[0] = 0.0;
            s[1] = 0.0;
        }
    }
    if ((adj && A.pfc) || A.all) {
        d[3] = pfc_solve(d[0], d[1], d[2], pk, ph_r, A.T, gl);
        if (taut) d2[1] = pfc_solve(d2[0], d[1], d[2], pk, ph_r, A.T, gl);
    }
    if (w0) {
        for (int k = 0; k < 4; ++k) A.dwp[4 * c + k] = d[k];
        if (taut) {
            A.dwp2[2 * c] = d2[0];
            A.dwp2[2 * c + 1] = d2[1];
        }
        if (A.adjusted) A.adjusted[c] = adj ? 1 : 0;
    }
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on the
// Legendre polynomial P_n (three-term recurrence) from the Chebyshev-like
// starting guesses cos(pi (i + 3/4) / (n + 1/2)).
GaussLegendre make_gl() {
    GaussLegendre g{};
    const int n = kGL;
    for (int i = 0; i < n; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        g.x[i] = x;
        g.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return g;
}

const GaussLegendre& gl_table() {
    static const GaussLegendre g = make_gl();
    return g;
}

bool valid_params(const fmm_lambda_params* p) {
    return p && std::isfinite(p->mass) && p->mass > 0 && std::isfinite(p->dt) && p->dt > 0 &&
           std::isfinite(p->temperature) && p->temperature >= 0 && std::isfinite(p->tau) &&
           std::isfinite(p->near0) && std::isfinite(p->near1) && p->near0 <= p->near1;
}

}  // namespace fmml

extern "C" {

fmm_status fmm_lambda_step(void* hip_stream, int32_t R, const int32_t* coord_off, int64_t C,
                           const fmm_lambda_params* prm, int32_t first, const double* lam,
                           double* lam_new, double* v, const double* dvdl, const int32_t* partner,
                           const double* pka, const double* ph, const double* mm, const double* dwp,
                           const double* noise, double* stats_w, double* stats_b, double* kin,
                           double* e_bias, const double* dwp2, double* stats_b2) {
    using namespace fmml;
    if (R < 1 || C < 0 || !coord_off || !fmml::valid_params(prm) || !ph || (first != 0 && first != 1))
        return FMM_E_INVALID;
    if (C > 0 && (!lam || !lam_new || !v || !dvdl || lam == lam_new)) return FMM_E_INVALID;
    if (prm->tau > 0 && (!noise || !(prm->temperature > 0))) return FMM_E_INVALID;
    if (C > 0 && dwp2 && (!dwp || !partner)) return FMM_E_INVALID;
    if (C > 0 && stats_b2 && (!dwp2 || !stats_b)) return FMM_E_INVALID;
    StepArgs A{coord_off, C, *prm, first, lam, lam_new, v, dvdl, partner, pka, ph, mm, dwp,
               noise, stats_w, stats_b, kin, e_bias, dwp2, stats_b2};
    k_lambda_step<<<R, kThreads, 0, (hipStream_t)hip_stream>>>(A);
    return hipGetLastError() == hipSuccess ? FMM_OK : FMM_E_HIP;
}

fmm_status fmm_lambda_dbo(void* hip_stream, int32_t R, const int32_t* coord_off, int64_t C,
                          int32_t mode, int32_t pfc, const fmm_dbo_params* prm, double temperature,
                          const double* pka, const double* ph, double* dwp, double* stats_w,
                          double* stats_b, int32_t* adjusted, const int32_t* partner, double* dwp2,
                          double* stats_b2) {
    using namespace fmml;
    if (R < 1 || C < 0 || !coord_off || !ph || mode < 0 || mode > 3 || (pfc != 0 && pfc != 1) ||
        !(temperature > 0) || !std::isfinite(temperature))
        return FMM_E_INVALID;
    if (C > 0 && (!dwp || ((mode & 1) && !stats_w) || ((mode & 2) && !stats_b))) return FMM_E_INVALID;
    if (C > 0 && dwp2 && (!partner || ((mode & 2) && !stats_b2))) return FMM_E_INVALID;
    fmm_dbo_params P = prm ? *prm : fmm_dbo_params{0.2, 0.8, 0.7, 0.03, 0.5, 0.08, 0.25, 0.05, 1.0, 1.0, 20.0};
    if (C == 0) return FMM_OK;
    DboArgs A{coord_off, R, C, mode, pfc, 0, P, temperature, pka, ph, dwp, stats_w, stats_b, adjusted,
              partner, dwp2, stats_b2};
    const unsigned nb = (unsigned)((C + kDboWaves - 1) / kDboWaves);
    k_lambda_dbo<<<nb, 64 * kDboWaves, 0, (hipStream_t)hip_stream>>>(A, gl_table());
    return hipGetLastError() == hipSuccess ? FMM_OK : FMM_E_HIP;
}

fmm_status fmm_lambda_pfc(void* hip_stream, int32_t R, const int32_t* coord_off, int64_t C,
                          double temperature, const double* pka, const double* ph, double* dwp,
                          const int32_t* partner, double* dwp2) {
    using namespace fmml;
    if (R < 1 || C < 0 || !coord_off || !ph || !(temperature > 0) || !std::isfinite(temperature))
        return FMM_E_INVALID;
    if (C > 0 && (!dwp || (dwp2 && !partner))) return FMM_E_INVALID;
    if (C == 0) return FMM_OK;
    DboArgs A{coord_off, R, C, 0, 1, 1, fmm_dbo_params{}, temperature, pka, ph, dwp, nullptr, nullptr,
              nullptr, partner, dwp2, nullptr};
    const unsigned nb = (unsigned)((C + kDboWaves - 1) / kDboWaves);
    k_lambda_dbo<<<nb, 64 * kDboWaves, 0, (hipStream_t)hip_stream>>>(A, gl_table());
    return hipGetLastError() == hipSuccess ? FMM_OK : FMM_E_HIP;
}

}  // extern "C"
