/*
 * coulomb_oracle.c -- plain, slow, FP64 CPU oracle for the lambda-interpolated
 * Coulomb solve (energy, forces, potentials and per-site lambda-forces).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP library.
 *
 * What it computes (Kohnke et al., constant-pH lambda-dynamics with FMM
 * electrostatics; Methods, "Constant pH Simulations Based on lambda-dynamics",
 * eq 1 and the text that follows it, and "Calibration of Protonation
 * Dynamics", where the derivative of the Hamiltonian with respect to lambda is
 * stated to be purely Coulombic because forms differ only in their charges):
 *
 *   q_i       = qA_i + lambda_{s(i)} (qB_i - qA_i)      (q_i = qA_i if s(i) = -1)
 *   phi_i     = k_e * sum_{j != i} q_j / r_ij           (open boundaries)
 *   E         = 1/2 sum_i q_i phi_i
 *   F_i       = q_i * field_i = -dE/dr_i
 *   dV/dl_s   = sum_{i in s} (qB_i - qA_i) phi_i        (= dE/dlambda_s)
 *
 * Periodic boundaries (the paper's simulations are periodic and lattice-summed,
 * Introduction, and it requires the box to stay neutral, "Sites Acting as
 * Charge Buffers"): phi is the periodic solution of Poisson's equation with a
 * uniform neutralising background, conducting ("tin-foil") surroundings and
 * zero cell mean, with the self term removed.  It is evaluated by a plain
 * Ewald sum: real-space erfc sum over images, reciprocal-space sum over k != 0,
 * self term -2 beta q_i / sqrt(pi), background term -pi Q / (V beta^2).
 *
 * All arithmetic is FP64.  Loops are the textbook double loops, parallel over
 * target atoms with OpenMP; no blocking, sorting or tree of any kind.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* Neumaier compensated accumulator. */
typedef struct { double s, c; } acc_t;
static inline void acc_add(acc_t* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static inline double acc_get(const acc_t* a) { return a->s + a->c; }

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Charge interpolation of eq 1 written per atom: q = qA + lambda_s (qB - qA).
 * Returns 0, or -1 if a site index lies outside [-1, nsites). */
int orc_lambda_charges(int64_t n, const double* qA, const double* qB,
                       const int32_t* site, int64_t nsites,
                       const double* lam, double* q) {
    for (int64_t i = 0; i < n; ++i) {
        int32_t s = site ? site[i] : -1;
        if (s < -1 || s >= nsites) return -1;
        q[i] = (s < 0) ? qA[i] : qA[i] + lam[s] * (qB[i] - qA[i]);
    }
    return 0;
}

/* Open-boundary direct sum (the plain definition of the Coulomb potential).
 * targets: ntarget indices into [0,n) (NULL means all n atoms, ntarget = n).
 * phi[t] = sum_{j != i} q_j / |r_i - r_j|,
 * field[3t..3t+2] = sum_{j != i} q_j (r_i - r_j) / |r_i - r_j|^3, with i = targets[t].
 * x is n x 3 row-major.  k_e is applied by orc_outputs, not here. */
void orc_direct(int64_t n, const double* x, const double* q,
                int64_t ntarget, const int64_t* targets,
                double* phi, double* field) {
    if (!targets) ntarget = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ntarget; ++t) {
        int64_t i = targets ? targets[t] : t;
        acc_t p = {0, 0}, fx = {0, 0}, fy = {0, 0}, fz = {0, 0};
        double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = xi - x[3 * j], dy = yi - x[3 * j + 1], dz = zi - x[3 * j + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            double r = sqrt(r2);
            double qr = q[j] / r;
            double qr3 = qr / r2;
            acc_add(&p, qr);
            acc_add(&fx, qr3 * dx);
            acc_add(&fy, qr3 * dy);
            acc_add(&fz, qr3 * dz);
        }
        phi[t] = acc_get(&p);
        field[3 * t] = acc_get(&fx);
        field[3 * t + 1] = acc_get(&fy);
        field[3 * t + 2] = acc_get(&fz);
    }
}

/* Ewald sum for an orthorhombic box with edges box[0..2] (tin-foil surroundings,
 * uniform background for a net charge, zero-mean potential).
 *   beta  : splitting parameter (1/length)
 *   rcut  : real-space cutoff; every image n with |r_ij + n L| < rcut is summed,
 *           including self images (j = i, n != 0)
 *   kmax  : |m_a| <= kmax[a] for k = 2 pi (m_x/Lx, m_y/Ly, m_z/Lz), k != 0
 * Outputs as for orc_direct (potential excludes only the i = j, n = 0 term).
 * Returns 0, or -1 on bad arguments / allocation failure. */
int orc_ewald(int64_t n, const double* x, const double* q, const double* box,
              double beta, double rcut, const int32_t* kmax,
              int64_t ntarget, const int64_t* targets,
              double* phi, double* field) {
    if (!targets) ntarget = n;
    if (box[0] <= 0 || box[1] <= 0 || box[2] <= 0 || beta <= 0 || rcut <= 0) return -1;
    if (kmax[0] < 0 || kmax[1] < 0 || kmax[2] < 0) return -1;
    const double L[3] = {box[0], box[1], box[2]};
    const double V = L[0] * L[1] * L[2];
    const double rc2 = rcut * rcut;
    const double two_b_sqrtpi = 2.0 * beta / sqrt(ORC_PI);

    double Q = 0.0;
    for (int64_t j = 0; j < n; ++j) Q += q[j];

    /* k-vectors on a half space: (mx > 0) or (mx = 0, my > 0) or (mx = my = 0, mz > 0);
     * each carries the factor 2 of its -k partner. */
    const int kx = kmax[0], ky = kmax[1], kz = kmax[2];
    int64_t nk_max = (int64_t)(2 * kx + 1) * (2 * ky + 1) * (2 * kz + 1);
    int32_t* km = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)nk_max);
    double* kc = (double*)malloc(sizeof(double) * (size_t)nk_max);
    if (!km || !kc) { free(km); free(kc); return -1; }
    int64_t nk = 0;
    for (int mx = 0; mx <= kx; ++mx)
        for (int my = -ky; my <= ky; ++my)
            for (int mz = -kz; mz <= kz; ++mz) {
                if (mx == 0 && (my < 0 || (my == 0 && mz <= 0))) continue;
                double gx = 2 * ORC_PI * mx / L[0], gy = 2 * ORC_PI * my / L[1],
                       gz = 2 * ORC_PI * mz / L[2];
                double k2 = gx * gx + gy * gy + gz * gz;
                km[3 * nk] = mx; km[3 * nk + 1] = my; km[3 * nk + 2] = mz;
                kc[nk] = 2.0 * (4.0 * ORC_PI / V) * exp(-k2 / (4 * beta * beta)) / k2;
                ++nk;
            }

    /* Per-atom tables cos/sin(2 pi m x_a / L_a) for |m| <= kmax_a, each entry
     * from one direct libm call, so exp(i k.r) = product of three table entries. */
    const int wx = 2 * kx + 1, wy = 2 * ky + 1, wz = 2 * kz + 1, w = wx + wy + wz;
    double* tc = (double*)malloc(sizeof(double) * (size_t)n * w);
    double* ts = (double*)malloc(sizeof(double) * (size_t)n * w);
    double* Sre = (double*)calloc((size_t)(nk ? nk : 1), sizeof(double));
    double* Sim = (double*)calloc((size_t)(nk ? nk : 1), sizeof(double));
    if (!tc || !ts || !Sre || !Sim) {
        free(km); free(kc); free(tc); free(ts); free(Sre); free(Sim); return -1;
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        double* c = tc + (size_t)j * w;
        double* s = ts + (size_t)j * w;
        for (int m = -kx; m <= kx; ++m) {
            double a = 2 * ORC_PI * m * x[3 * j] / L[0];
            c[m + kx] = cos(a); s[m + kx] = sin(a);
        }
        for (int m = -ky; m <= ky; ++m) {
            double a = 2 * ORC_PI * m * x[3 * j + 1] / L[1];
            c[wx + m + ky] = cos(a); s[wx + m + ky] = sin(a);
        }
        for (int m = -kz; m <= kz; ++m) {
            double a = 2 * ORC_PI * m * x[3 * j + 2] / L[2];
            c[wx + wy + m + kz] = cos(a); s[wx + wy + m + kz] = sin(a);
        }
    }
#define ORC_EIKR(j, k, RE, IM) do {                                              \
        const double* c_ = tc + (size_t)(j) * w; const double* s_ = ts + (size_t)(j) * w; \
        int ix_ = km[3 * (k)] + kx, iy_ = wx + km[3 * (k) + 1] + ky,              \
            iz_ = wx + wy + km[3 * (k) + 2] + kz;                                 \
        double ar_ = c_[ix_] * c_[iy_] - s_[ix_] * s_[iy_];                        \
        double ai_ = c_[ix_] * s_[iy_] + s_[ix_] * c_[iy_];                        \
        RE = ar_ * c_[iz_] - ai_ * s_[iz_];                                       \
        IM = ar_ * s_[iz_] + ai_ * c_[iz_];                                       \
    } while (0)

    /* Structure factor S(k) = sum_j q_j exp(i k.r_j). */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nk; ++k) {
        acc_t re = {0, 0}, im = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            double er, ei;
            ORC_EIKR(j, k, er, ei);
            acc_add(&re, q[j] * er);
            acc_add(&im, q[j] * ei);
        }
        Sre[k] = acc_get(&re);
        Sim[k] = acc_get(&im);
    }

#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t t = 0; t < ntarget; ++t) {
        int64_t i = targets ? targets[t] : t;
        acc_t p = {0, 0}, fx = {0, 0}, fy = {0, 0}, fz = {0, 0};
        /* real space: every image n with |r_i - r_j + n L| < rcut */
        for (int64_t j = 0; j < n; ++j) {
            double d0[3];
            int lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                d0[a] = x[3 * i + a] - x[3 * j + a];
                lo[a] = (int)ceil((-rcut - d0[a]) / L[a]);
                hi[a] = (int)floor((rcut - d0[a]) / L[a]);
            }
            for (int a = lo[0]; a <= hi[0]; ++a)
                for (int b = lo[1]; b <= hi[1]; ++b)
                    for (int c = lo[2]; c <= hi[2]; ++c) {
                        if (j == i && a == 0 && b == 0 && c == 0) continue;
                        double dx = d0[0] + a * L[0], dy = d0[1] + b * L[1], dz = d0[2] + c * L[2];
                        double r2 = dx * dx + dy * dy + dz * dz;
                        if (r2 >= rc2) continue;
                        double r = sqrt(r2);
                        double e = erfc(beta * r) / r;
                        double g = (e + two_b_sqrtpi * exp(-beta * beta * r2)) / r2;
                        acc_add(&p, q[j] * e);
                        acc_add(&fx, q[j] * g * dx);
                        acc_add(&fy, q[j] * g * dy);
                        acc_add(&fz, q[j] * g * dz);
                    }
        }
        /* reciprocal space: phi += sum_k c Re[S e^{-ik.r}], field -= sum_k c k Im[S e^{-ik.r}] */
        for (int64_t k = 0; k < nk; ++k) {
            double er, ei;
            ORC_EIKR(i, k, er, ei);
            double re = Sre[k] * er + Sim[k] * ei;   /* Re[S e^{-ik.r}] */
            double im = Sim[k] * er - Sre[k] * ei;   /* Im[S e^{-ik.r}] */
            double c = kc[k];
            acc_add(&p, c * re);
            acc_add(&fx, -c * (2 * ORC_PI * km[3 * k] / L[0]) * im);
            acc_add(&fy, -c * (2 * ORC_PI * km[3 * k + 1] / L[1]) * im);
            acc_add(&fz, -c * (2 * ORC_PI * km[3 * k + 2] / L[2]) * im);
        }
        /* self and background */
        acc_add(&p, -two_b_sqrtpi * q[i]);
        acc_add(&p, -ORC_PI * Q / (V * beta * beta));
        phi[t] = acc_get(&p);
        field[3 * t] = acc_get(&fx);
        field[3 * t + 1] = acc_get(&fy);
        field[3 * t + 2] = acc_get(&fz);
    }
#undef ORC_EIKR
    free(km); free(kc); free(tc); free(ts); free(Sre); free(Sim);
    return 0;
}

/* Assemble the method's outputs from per-atom potentials and fields (all n atoms):
 *   E = 1/2 k_e sum q_i phi_i ;  F_i = k_e q_i field_i ;
 *   dVdl_s = k_e sum_{i in s} (qB_i - qA_i) phi_i   (dV/dlambda_s, eq 1 with
 *   charge interpolation; atoms with site -1 contribute nothing).
 * Returns 0, or -1 on a site index outside [-1, nsites). */
int orc_outputs(int64_t n, const double* q, const double* qA, const double* qB,
                const int32_t* site, int64_t nsites, const double* phi,
                const double* field, double k_e, double* E, double* F, double* dVdl) {
    acc_t e = {0, 0};
    acc_t* d = (acc_t*)calloc((size_t)(nsites > 0 ? nsites : 1), sizeof(acc_t));
    if (!d) return -1;
    for (int64_t i = 0; i < n; ++i) {
        acc_add(&e, q[i] * phi[i]);
        if (F) {
            F[3 * i] = k_e * q[i] * field[3 * i];
            F[3 * i + 1] = k_e * q[i] * field[3 * i + 1];
            F[3 * i + 2] = k_e * q[i] * field[3 * i + 2];
        }
        int32_t s = site ? site[i] : -1;
        if (s < -1 || s >= nsites) { free(d); return -1; }
        if (s >= 0) acc_add(&d[s], (qB[i] - qA[i]) * phi[i]);
    }
    *E = 0.5 * k_e * acc_get(&e);
    if (dVdl)
        for (int64_t s = 0; s < nsites; ++s) dVdl[s] = k_e * acc_get(&d[s]);
    free(d);
    return 0;
}

/* Four charge forms per site (protonation tautomers; Methods, eq 2, where the
 * Hamiltonian is interpolated bilinearly between forms A, B, C, D by the
 * protonation coordinate lambda_p and the tautomer coordinate lambda_t; here
 * in charge-interpolated form, as eq 1 above).  With u~ = 1 - u:
 *   q_i = lp~ (lt~ qA_i + lt qB_i) + lp (lt~ qC_i + lt qD_i)    (q_i = qA_i if s(i) = -1)
 * Returns 0, or -1 if a site index lies outside [-1, nsites). */
int orc_tautomer_charges(int64_t n, const double* qA, const double* qB, const double* qC,
                         const double* qD, const int32_t* site, int64_t nsites,
                         const double* lp, const double* lt, double* q) {
    for (int64_t i = 0; i < n; ++i) {
        int32_t s = site ? site[i] : -1;
        if (s < -1 || s >= nsites) return -1;
        if (s < 0) {
            q[i] = qA[i];
        } else {
            const double p = lp[s], t = lt[s];
            q[i] = (1.0 - p) * ((1.0 - t) * qA[i] + t * qB[i]) + p * ((1.0 - t) * qC[i] + t * qD[i]);
        }
    }
    return 0;
}

/* The two site derivatives of the four-form energy: q_i is bilinear in
 * (lambda_p, lambda_t), so with phi including k_e
 *   dV/dlambda_p[s] = k_e sum_{i in s} phi_i (dq_i/dlambda_p)
 *                   = k_e sum_{i in s} phi_i (lt~ (qC_i - qA_i) + lt (qD_i - qB_i))
 *   dV/dlambda_t[s] = k_e sum_{i in s} phi_i (lp~ (qB_i - qA_i) + lp (qD_i - qC_i))
 * (phi here without k_e, as orc_outputs).  Returns 0, or -1 on a bad site. */
int orc_tautomer_dvdl(int64_t n, const double* qA, const double* qB, const double* qC,
                      const double* qD, const int32_t* site, int64_t nsites, const double* lp,
                      const double* lt, const double* phi, double k_e, double* dVdlp,
                      double* dVdlt) {
    acc_t* d = (acc_t*)calloc((size_t)(2 * (nsites > 0 ? nsites : 1)), sizeof(acc_t));
    if (!d) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int32_t s = site ? site[i] : -1;
        if (s < -1 || s >= nsites) { free(d); return -1; }
        if (s < 0) continue;
        const double p = lp[s], t = lt[s];
        acc_add(&d[2 * s], phi[i] * ((1.0 - t) * (qC[i] - qA[i]) + t * (qD[i] - qB[i])));
        acc_add(&d[2 * s + 1], phi[i] * ((1.0 - p) * (qB[i] - qA[i]) + p * (qD[i] - qC[i])));
    }
    for (int64_t s = 0; s < nsites; ++s) {
        dVdlp[s] = k_e * acc_get(&d[2 * s]);
        dVdlt[s] = k_e * acc_get(&d[2 * s + 1]);
    }
    free(d);
    return 0;
}

/* ---- upstream weights on the forces (second-order adjoint) ----------------
 * For L_F = sum_m w_m . F_m (w: one 3-vector weight per atom) the gradient
 * needs, per target atom m, two pair sums over all other atoms j (and, for a
 * periodic cell, every image of every atom, self images included):
 *
 *   hw_m = sum_j q_j [grad grad psi](r_m - r_j) (w_m - w_j)        (3-vector)
 *   ew_m = sum_j q_j e(r_m - r_j) . (w_m - w_j),   e = -grad psi   (scalar)
 *
 * because F_m = k_e q_m sum_j q_j e(r_m - r_j) gives
 *   dL_F / dx_m = -k_e q_m hw_m   and   dL_F / dq_m = k_e ew_m
 * (the j = m terms of both sums vanish: w_m - w_m = 0).  psi = 1/r for open
 * boundaries: grad grad (1/r) = (3 r r^T - r^2 I) / r^5, e = r / r^3.
 * w is n x 3 row-major; outputs per target t (atom i = targets[t]). */
void orc_direct_wpair(int64_t n, const double* x, const double* q, const double* w,
                      int64_t ntarget, const int64_t* targets, double* hw, double* ew) {
    if (!targets) ntarget = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ntarget; ++t) {
        int64_t i = targets ? targets[t] : t;
        acc_t h0 = {0, 0}, h1 = {0, 0}, h2 = {0, 0}, e = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r[3], dw[3];
            for (int a = 0; a < 3; ++a) {
                r[a] = x[3 * i + a] - x[3 * j + a];
                dw[a] = w[3 * i + a] - w[3 * j + a];
            }
            double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            double rr = sqrt(r2);
            double r3 = r2 * rr, r5 = r3 * r2;
            double rdw = r[0] * dw[0] + r[1] * dw[1] + r[2] * dw[2];
            /* (3 r r^T / r^5 - I / r^3) dw */
            acc_add(&h0, q[j] * (3.0 * r[0] * rdw / r5 - dw[0] / r3));
            acc_add(&h1, q[j] * (3.0 * r[1] * rdw / r5 - dw[1] / r3));
            acc_add(&h2, q[j] * (3.0 * r[2] * rdw / r5 - dw[2] / r3));
            acc_add(&e, q[j] * rdw / r3);
        }
        hw[3 * t] = acc_get(&h0);
        hw[3 * t + 1] = acc_get(&h1);
        hw[3 * t + 2] = acc_get(&h2);
        ew[t] = acc_get(&e);
    }
}

/* The same pair sums for the Ewald potential of an orthorhombic box (the
 * conventions of orc_ewald).  Real space, every image within rcut:
 *   grad grad [erfc(b r)/r] = C r r^T - B I,  e = B r,
 *   B = [erfc(b r) + c r exp(-b^2 r^2)] / r^3,
 *   C = [3 erfc(b r) + c r (3 + 2 b^2 r^2) exp(-b^2 r^2)] / r^5,  c = 2 b / sqrt(pi).
 * Reciprocal space, psi_rec(r) = sum_k c_k cos(k.r) over the half space k
 * (c_k = 2 (4 pi / V) exp(-k^2 / 4 b^2) / k^2): grad grad psi_rec =
 * -sum c_k k k^T cos(k.r) and e_rec = sum c_k k sin(k.r); with
 * S(k) = sum_j q_j exp(i k.r_j) and P(k) = sum_j q_j w_j exp(i k.r_j),
 *   sum_j q_j (w_m - w_j) cos(k.r_mj) = w_m Re[S e^{-ik.r_m}] - Re[P e^{-ik.r_m}],
 *   sum_j q_j (w_m - w_j) sin(k.r_mj) = -(w_m Im[S e^{-ik.r_m}] - Im[P e^{-ik.r_m}]).
 * The self and background terms of the potential are constants or cancel in
 * w_m - w_j, so they add nothing.  Returns 0, or -1 on bad arguments. */
int orc_ewald_wpair(int64_t n, const double* x, const double* q, const double* w,
                    const double* box, double beta, double rcut, const int32_t* kmax,
                    int64_t ntarget, const int64_t* targets, double* hw, double* ew) {
    if (!targets) ntarget = n;
    if (box[0] <= 0 || box[1] <= 0 || box[2] <= 0 || beta <= 0 || rcut <= 0) return -1;
    if (kmax[0] < 0 || kmax[1] < 0 || kmax[2] < 0) return -1;
    const double L[3] = {box[0], box[1], box[2]};
    const double V = L[0] * L[1] * L[2];
    const double rc2 = rcut * rcut;
    const double cb = 2.0 * beta / sqrt(ORC_PI);
    const int kx = kmax[0], ky = kmax[1], kz = kmax[2];
    int64_t nk_max = (int64_t)(2 * kx + 1) * (2 * ky + 1) * (2 * kz + 1);
    double* kv = (double*)malloc(sizeof(double) * 3 * (size_t)nk_max);
    double* kc = (double*)malloc(sizeof(double) * (size_t)nk_max);
    /* per k: S re, S im, then P re/im for x, y, z */
    double* sf = (double*)calloc((size_t)(nk_max ? nk_max : 1) * 8, sizeof(double));
    if (!kv || !kc || !sf) { free(kv); free(kc); free(sf); return -1; }
    int64_t nk = 0;
    for (int mx = 0; mx <= kx; ++mx)
        for (int my = -ky; my <= ky; ++my)
            for (int mz = -kz; mz <= kz; ++mz) {
                if (mx == 0 && (my < 0 || (my == 0 && mz <= 0))) continue;
                double g0 = 2 * ORC_PI * mx / L[0], g1 = 2 * ORC_PI * my / L[1],
                       g2 = 2 * ORC_PI * mz / L[2];
                double k2 = g0 * g0 + g1 * g1 + g2 * g2;
                kv[3 * nk] = g0; kv[3 * nk + 1] = g1; kv[3 * nk + 2] = g2;
                kc[nk] = 2.0 * (4.0 * ORC_PI / V) * exp(-k2 / (4 * beta * beta)) / k2;
                ++nk;
            }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nk; ++k) {
        acc_t a[8];
        for (int c = 0; c < 8; ++c) { a[c].s = 0; a[c].c = 0; }
        for (int64_t j = 0; j < n; ++j) {
            double ph = kv[3 * k] * x[3 * j] + kv[3 * k + 1] * x[3 * j + 1] +
                        kv[3 * k + 2] * x[3 * j + 2];
            double cr = cos(ph), si = sin(ph);
            acc_add(&a[0], q[j] * cr);
            acc_add(&a[1], q[j] * si);
            for (int d = 0; d < 3; ++d) {
                acc_add(&a[2 + 2 * d], q[j] * w[3 * j + d] * cr);
                acc_add(&a[3 + 2 * d], q[j] * w[3 * j + d] * si);
            }
        }
        for (int c = 0; c < 8; ++c) sf[8 * k + c] = acc_get(&a[c]);
    }
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t t = 0; t < ntarget; ++t) {
        int64_t i = targets ? targets[t] : t;
        acc_t h0 = {0, 0}, h1 = {0, 0}, h2 = {0, 0}, e = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            double d0[3], dw[3];
            int lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                d0[a] = x[3 * i + a] - x[3 * j + a];
                dw[a] = w[3 * i + a] - w[3 * j + a];
                lo[a] = (int)ceil((-rcut - d0[a]) / L[a]);
                hi[a] = (int)floor((rcut - d0[a]) / L[a]);
            }
            for (int a = lo[0]; a <= hi[0]; ++a)
                for (int b = lo[1]; b <= hi[1]; ++b)
                    for (int c = lo[2]; c <= hi[2]; ++c) {
                        if (j == i && a == 0 && b == 0 && c == 0) continue;
                        double r[3] = {d0[0] + a * L[0], d0[1] + b * L[1], d0[2] + c * L[2]};
                        double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                        if (r2 >= rc2) continue;
                        double rr = sqrt(r2);
                        double ex = exp(-beta * beta * r2), ec = erfc(beta * rr);
                        double B = (ec + cb * rr * ex) / (r2 * rr);
                        double C = (3.0 * ec + cb * rr * (3.0 + 2.0 * beta * beta * r2) * ex) /
                                   (r2 * r2 * rr);
                        double rdw = r[0] * dw[0] + r[1] * dw[1] + r[2] * dw[2];
                        acc_add(&h0, q[j] * (C * r[0] * rdw - B * dw[0]));
                        acc_add(&h1, q[j] * (C * r[1] * rdw - B * dw[1]));
                        acc_add(&h2, q[j] * (C * r[2] * rdw - B * dw[2]));
                        acc_add(&e, q[j] * B * rdw);
                    }
        }
        for (int64_t k = 0; k < nk; ++k) {
            const double* kk = kv + 3 * k;
            const double* s = sf + 8 * k;
            double ph = kk[0] * x[3 * i] + kk[1] * x[3 * i + 1] + kk[2] * x[3 * i + 2];
            double er = cos(ph), ei = -sin(ph); /* e^{-ik.r_i} */
            double sre = s[0] * er - s[1] * ei, sim = s[0] * ei + s[1] * er;
            double cosv[3], sinv[3];  /* sum_j q_j (w_i - w_j) cos / sin (k.r_ij) */
            for (int d = 0; d < 3; ++d) {
                double pre = s[2 + 2 * d] * er - s[3 + 2 * d] * ei;
                double pim = s[2 + 2 * d] * ei + s[3 + 2 * d] * er;
                cosv[d] = w[3 * i + d] * sre - pre;
                sinv[d] = -(w[3 * i + d] * sim - pim);
            }
            double kc_ = kc[k];
            double kcos = kk[0] * cosv[0] + kk[1] * cosv[1] + kk[2] * cosv[2];
            double ksin = kk[0] * sinv[0] + kk[1] * sinv[1] + kk[2] * sinv[2];
            acc_add(&h0, -kc_ * kk[0] * kcos);
            acc_add(&h1, -kc_ * kk[1] * kcos);
            acc_add(&h2, -kc_ * kk[2] * kcos);
            acc_add(&e, kc_ * ksin);
        }
        hw[3 * t] = acc_get(&h0);
        hw[3 * t + 1] = acc_get(&h1);
        hw[3 * t + 2] = acc_get(&h2);
        ew[t] = acc_get(&e);
    }
    free(kv); free(kc); free(sf);
    return 0;
}
