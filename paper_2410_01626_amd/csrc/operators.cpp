// operators.cpp -- host-side FP64 construction of the multipole translation
// operators (see operators.h for the basis and scaling conventions).
//
// Every operator is first written as a complex linear map on unnormalised
// complex coefficients
//   R_l^m(r) = r^l P_l^m(cos th) e^{i m ph} / (l+m)!      (regular)
//   I_l^m(r) = (l-m)! P_l^m(cos th) e^{i m ph} / r^(l+1)  (irregular)
// for which 1/|r - a| = sum_{l,m} conj(R_l^m(a)) I_l^m(r) (|a| < |r|), the
// regular addition theorem R_l^m(a+b) = sum_{j,k} R_j^k(a) R_{l-j}^{m-k}(b)
// holds, and I_k^n(d+u) = sum_{j,m} (-1)^j conj(R_j^m(u)) I_{k+j}^{n+m}(d)
// for |u| < |d|.  With M_l^m = sum q conj(R_l^m(x - c)) and a local expansion
// phi(t) = sum L_l^m R_l^m(t - c'):
//   M2M   M'_l^m = sum_{k,n} M_k^n conj(R_{l-k}^{m-n}(c_child - c_parent))
//   M2L   L_j^m  = (-1)^(j+m) sum_{k,n} M_k^n I_{k+j}^{n-m}(c_t - c_s)
//   L2L   L'_j^k = sum_{l,m} L_l^m R_{l-j}^{m-k}(c_child - c_parent)
// The complex maps are then converted column by column to the real
// normalised scaled basis that the kernels use.
#include "operators.h"

#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace fmmops {
namespace {

using cplx = std::complex<double>;
constexpr double kPi = 3.14159265358979323846;

inline int cidx(int l, int m) { return l * l + l + m; }  // complex index, |m| <= l

double fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}
inline double nrm(int l, int m) { return std::sqrt(fact(l + m) * fact(l - std::abs(m))); }

// Complex regular harmonics R_l^m, all |m| <= l <= P.
void regular(int P, const double r[3], std::vector<cplx>& out) {
    out.assign((size_t)(P + 1) * (P + 1), cplx(0, 0));
    const double x = r[0], y = r[1], z = r[2], r2 = x * x + y * y + z * z;
    const cplx xp(x, y);
    cplx rmm(1.0, 0.0);
    for (int m = 0; m <= P; ++m) {
        if (m > 0) rmm = -xp / (2.0 * m) * rmm;
        out[cidx(m, m)] = rmm;
        if (m + 1 <= P) out[cidx(m + 1, m)] = z * rmm;
        for (int l = m + 2; l <= P; ++l)
            out[cidx(l, m)] = ((2.0 * l - 1) * z * out[cidx(l - 1, m)] - r2 * out[cidx(l - 2, m)]) /
                              double((l + m) * (l - m));
    }
    for (int l = 0; l <= P; ++l)
        for (int m = 1; m <= l; ++m)
            out[cidx(l, -m)] = ((m & 1) ? -1.0 : 1.0) * std::conj(out[cidx(l, m)]);
}

// Complex irregular harmonics I_l^m, all |m| <= l <= P.
void irregular(int P, const double r[3], std::vector<cplx>& out) {
    out.assign((size_t)(P + 1) * (P + 1), cplx(0, 0));
    const double x = r[0], y = r[1], z = r[2], r2 = x * x + y * y + z * z, ir2 = 1.0 / r2;
    const cplx xp(x, y);
    cplx imm(1.0 / std::sqrt(r2), 0.0);
    for (int m = 0; m <= P; ++m) {
        if (m > 0) imm = -(2.0 * m - 1) * xp * ir2 * imm;
        out[cidx(m, m)] = imm;
        if (m + 1 <= P) out[cidx(m + 1, m)] = (2.0 * m + 1) * z * ir2 * imm;
        for (int l = m + 2; l <= P; ++l)
            out[cidx(l, m)] = ((2.0 * l - 1) * z * out[cidx(l - 1, m)] -
                               double((l - 1) * (l - 1) - m * m) * out[cidx(l - 2, m)]) * ir2;
    }
    for (int l = 0; l <= P; ++l)
        for (int m = 1; m <= l; ++m)
            out[cidx(l, -m)] = ((m & 1) ? -1.0 : 1.0) * std::conj(out[cidx(l, m)]);
}

enum class Kind { Multipole, Local };

// Complex coefficient vector that a single real basis vector e_k (order p,
// of the given kind) stands for: entries (index, value) -- at most 2.
int basis_to_complex(int p, Kind kind, int k, int ci[2], cplx cv[2]) {
    (void)p;
    int l = (int)std::floor(std::sqrt((double)k) + 1e-9);
    while ((l + 1) * (l + 1) <= k) ++l;
    while (l * l > k) --l;
    int off = k - l * l;
    int m = (off + 1) / 2, part = (off == 0) ? 0 : (off - 1) % 2;
    double f = nrm(l, m);
    double sg = (m & 1) ? -1.0 : 1.0;
    if (m == 0) {
        ci[0] = cidx(l, 0);
        cv[0] = (kind == Kind::Multipole) ? cplx(1.0 / f, 0) : cplx(f, 0);
        return 1;
    }
    // multipole: M = (mu_c - i mu_s)/f ; local: L = (lam_c - i lam_s) f / 2
    cplx a = (kind == Kind::Multipole) ? cplx(1.0 / f, 0) : cplx(0.5 * f, 0);
    cplx v = part == 0 ? a : cplx(0, -1) * a;
    ci[0] = cidx(l, m);
    cv[0] = v;
    ci[1] = cidx(l, -m);
    cv[1] = sg * std::conj(v);
    return 2;
}

// Real coefficients (order p, kind) of a complex vector (only m >= 0 read).
void complex_to_real(int p, Kind kind, const std::vector<cplx>& c, double* out) {
    for (int l = 0; l <= p; ++l)
        for (int m = 0; m <= l; ++m) {
            double f = nrm(l, m);
            cplx v = c[cidx(l, m)];
            if (kind == Kind::Multipole) {  // mu = (Re M f, -Im M f)
                out[ridx(l, m, 0)] = v.real() * f;
                if (m > 0) out[ridx(l, m, 1)] = -v.imag() * f;
            } else {  // lam = (Re L / f, 2 Re L / f, -2 Im L / f)
                if (m == 0) out[ridx(l, 0, 0)] = v.real() / f;
                else {
                    out[ridx(l, m, 0)] = 2.0 * v.real() / f;
                    out[ridx(l, m, 1)] = -2.0 * v.imag() / f;
                }
            }
        }
}

// Build a real K_out x K_in matrix (row-major) from a complex column function
// col(ci, out): out = image of the unit complex input at complex index ci.
template <class ColFn>
void build_real(int p_in, Kind kin, int p_out, Kind kout, ColFn col, double* mat) {
    const int Kin = ncoef(p_in), Kout = ncoef(p_out);
    std::vector<cplx> acc((size_t)Kout), tmp((size_t)Kout);
    std::vector<double> rcol((size_t)Kout);
    for (int k = 0; k < Kin; ++k) {
        int ci[2];
        cplx cv[2];
        int nnz = basis_to_complex(p_in, kin, k, ci, cv);
        std::fill(acc.begin(), acc.end(), cplx(0, 0));
        for (int t = 0; t < nnz; ++t) {
            std::fill(tmp.begin(), tmp.end(), cplx(0, 0));
            col(ci[t], tmp);
            for (int i = 0; i < Kout; ++i) acc[i] += cv[t] * tmp[i];
        }
        complex_to_real(p_out, kout, acc, rcol.data());
        for (int i = 0; i < Kout; ++i) mat[(size_t)i * Kin + k] = rcol[i];
    }
}

void decode(int ci, int& l, int& m) {
    l = (int)std::floor(std::sqrt((double)ci) + 1e-9);
    while ((l + 1) * (l + 1) <= ci) ++l;
    while (l * l > ci) --l;
    m = ci - l * l - l;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Smooth part of the periodic Green's function of the unit cube near the
// origin: h(u) = psi(u) - sum_{n in {-1,0,1}^3} 1/|u+n| - (2 pi / 3)|u|^2,
// where psi is the tin-foil, background-neutralised, zero-mean periodic
// potential of a unit charge.  h is harmonic for |u| < 2.  Evaluated by an
// Ewald split with beta = 3 (real-space images |n_a| <= 3, |k_a| <= 2 pi 7).
double lattice_h(const double u[3]) {
    const double beta = 3.0;
    double s = 0.0;
    for (int a = -3; a <= 3; ++a)
        for (int b = -3; b <= 3; ++b)
            for (int c = -3; c <= 3; ++c) {
                double dx = u[0] + a, dy = u[1] + b, dz = u[2] + c;
                double r = std::sqrt(dx * dx + dy * dy + dz * dz);
                bool near = std::abs(a) <= 1 && std::abs(b) <= 1 && std::abs(c) <= 1;
                if (!near) s += std::erfc(beta * r) / r;
                else if (r > 1e-12) s -= std::erf(beta * r) / r;
                else s -= 2.0 * beta / std::sqrt(kPi);
            }
    const int km = 7;
    for (int a = 0; a <= km; ++a)
        for (int b = -km; b <= km; ++b)
            for (int c = -km; c <= km; ++c) {
                if (a == 0 && (b < 0 || (b == 0 && c <= 0))) continue;
                double kx = 2 * kPi * a, ky = 2 * kPi * b, kz = 2 * kPi * c;
                double k2 = kx * kx + ky * ky + kz * kz;
                s += 2.0 * 4.0 * kPi * std::exp(-k2 / (4 * beta * beta)) / k2 *
                     std::cos(kx * u[0] + ky * u[1] + kz * u[2]);
            }
    s -= kPi / (beta * beta);
    s -= 2.0 * kPi / 3.0 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    return s;
}

// Coefficients c_L^M (L <= P) of h(u) = sum c_L^M R_L^M(u), by projecting h
// sampled on a sphere of radius 0.8 onto spherical harmonics (Gauss-Legendre
// in cos(theta) x trapezoid in phi, exact for the degrees that matter).
void lattice_coeffs(int P, std::vector<cplx>& c) {
    const double rho = 0.8;
    const int nth = 2 * P + 24, nph = 4 * P + 48;
    std::vector<double> xg, wg;
    gauss_legendre(nth, xg, wg);
    c.assign((size_t)(P + 1) * (P + 1), cplx(0, 0));
    std::vector<cplx> R;
    for (int i = 0; i < nth; ++i) {
        double ct = xg[i], st = std::sqrt(std::max(0.0, 1 - ct * ct));
        for (int j = 0; j < nph; ++j) {
            double ph = 2 * kPi * j / nph;
            double u[3] = {rho * st * std::cos(ph), rho * st * std::sin(ph), rho * ct};
            double h = lattice_h(u);
            double w = wg[i] * 2 * kPi / nph;
            regular(P, u, R);
            for (int L = 0; L <= P; ++L)
                for (int M = 0; M <= L; ++M) c[cidx(L, M)] += w * h * std::conj(R[cidx(L, M)]);
        }
    }
    for (int L = 0; L <= P; ++L)
        for (int M = 0; M <= L; ++M) {
            // integral of |R_L^M|^2 over the sphere of radius rho
            double nr = std::pow(rho, 2 * L) * 4 * kPi / ((2 * L + 1) * fact(L + M) * fact(L - M));
            c[cidx(L, M)] /= nr;
            if (M > 0) c[cidx(L, -M)] = ((M & 1) ? -1.0 : 1.0) * std::conj(c[cidx(L, M)]);
        }
}

}  // namespace

void eval_rho(int p, const double r[3], double* out) {
    std::vector<cplx> R;
    regular(p, r, R);
    std::vector<cplx> cj(R.size());
    for (size_t i = 0; i < R.size(); ++i) cj[i] = std::conj(R[i]);
    complex_to_real(p, Kind::Multipole, cj, out);
}

void build_m2l_bank(int p, double* out) {
    const int K = ncoef(p);
    std::memset(out, 0, sizeof(double) * 343 * (size_t)K * K);
    std::vector<cplx> I;
    for (int ox = -3; ox <= 3; ++ox)
        for (int oy = -3; oy <= 3; ++oy)
            for (int oz = -3; oz <= 3; ++oz) {
                if (std::abs(ox) <= 1 && std::abs(oy) <= 1 && std::abs(oz) <= 1) continue;
                double d[3] = {(double)ox, (double)oy, (double)oz};
                irregular(2 * p, d, I);
                double* blk = out + (size_t)(((ox + 3) * 7 + (oy + 3)) * 7 + (oz + 3)) * K * K;
                build_real(p, Kind::Multipole, p, Kind::Local,
                           [&](int ci, std::vector<cplx>& o) {
                               int k, n;
                               decode(ci, k, n);
                               for (int j = 0; j <= p; ++j)
                                   for (int m = 0; m <= j; ++m) {
                                       if (std::abs(n - m) > k + j) continue;
                                       double sg = ((j + m) & 1) ? -1.0 : 1.0;
                                       o[cidx(j, m)] = sg * I[cidx(k + j, n - m)];
                                   }
                           },
                           blk);
            }
}

void build_m2m(int p, double* out) {
    const int K = ncoef(p);
    std::vector<cplx> R;
    for (int c = 0; c < 8; ++c) {
        double dd[3] = {((c >> 2) & 1) - 0.5, ((c >> 1) & 1) - 0.5, (c & 1) - 0.5};
        regular(p, dd, R);
        double* blk = out + (size_t)c * K * K;
        build_real(p, Kind::Multipole, p, Kind::Multipole,
                   [&](int ci, std::vector<cplx>& o) {
                       int k, n;
                       decode(ci, k, n);
                       for (int l = k; l <= p; ++l)
                           for (int m = 0; m <= l; ++m)
                               if (std::abs(m - n) <= l - k)
                                   o[cidx(l, m)] = std::conj(R[cidx(l - k, m - n)]);
                   },
                   blk);
        for (int l = 0; l <= p; ++l) {
            double s = std::ldexp(1.0, -l);
            for (int r = l * l; r < (l + 1) * (l + 1); ++r)
                for (int k = 0; k < K; ++k) blk[(size_t)r * K + k] *= s;
        }
    }
}

void build_l2l(int p, double* out) {
    const int K = ncoef(p);
    std::vector<cplx> R;
    for (int c = 0; c < 8; ++c) {
        // child centre relative to parent centre, in units of the parent edge
        double dd[3] = {0.5 * (((c >> 2) & 1) - 0.5), 0.5 * (((c >> 1) & 1) - 0.5),
                        0.5 * ((c & 1) - 0.5)};
        regular(p, dd, R);
        double* blk = out + (size_t)c * K * K;
        build_real(p, Kind::Local, p, Kind::Local,
                   [&](int ci, std::vector<cplx>& o) {
                       int l, m;
                       decode(ci, l, m);
                       for (int j = 0; j <= l; ++j)
                           for (int k = 0; k <= j; ++k)
                               if (std::abs(m - k) <= l - j) o[cidx(j, k)] = R[cidx(l - j, m - k)];
                   },
                   blk);
        for (int j = 0; j <= p; ++j) {
            double s = std::ldexp(1.0, -(j + 1));
            for (int r = j * j; r < (j + 1) * (j + 1); ++r)
                for (int k = 0; k < K; ++k) blk[(size_t)r * K + k] *= s;
        }
    }
}

void build_grad_table(int p, int32_t* out_idx, double* out_coef) {
    const int K = ncoef(p), Kg = p * p;
    std::vector<double> G((size_t)Kg * K);
    for (int a = 0; a < 3; ++a) {
        build_real(p, Kind::Local, p - 1, Kind::Local,
                   [&](int ci, std::vector<cplx>& o) {
                       int l, m;
                       decode(ci, l, m);
                       if (l == 0) return;
                       // d/dz R_l^m = R_{l-1}^m ; (d/dx + i d/dy) R_l^m = R_{l-1}^{m+1} ;
                       // (d/dx - i d/dy) R_l^m = -R_{l-1}^{m-1}
                       const int lo = l - 1;
                       auto put = [&](int mm, cplx v) {
                           if (std::abs(mm) <= lo && mm >= 0) o[cidx(lo, mm)] += v;
                       };
                       if (a == 2) put(m, 1.0);
                       else if (a == 0) {
                           put(m + 1, 0.5);
                           put(m - 1, -0.5);
                       } else {
                           put(m + 1, cplx(0, -0.5));
                           put(m - 1, cplx(0, -0.5));
                       }
                   },
                   G.data());
        for (int r = 0; r < Kg; ++r) {
            int nn = 0;
            for (int k = 0; k < 4; ++k) {
                out_idx[((size_t)a * Kg + r) * 4 + k] = -1;
                out_coef[((size_t)a * Kg + r) * 4 + k] = 0.0;
            }
            for (int k = 0; k < K; ++k) {
                double v = G[(size_t)r * K + k];
                if (std::fabs(v) > 1e-300) {
                    if (nn < 4) {
                        out_idx[((size_t)a * Kg + r) * 4 + nn] = k;
                        out_coef[((size_t)a * Kg + r) * 4 + nn] = v;
                    }
                    ++nn;
                }
            }
        }
    }
}

void build_lattice(int p, double* out) {
    // the lattice sum is the costly table (a sphere quadrature of an Ewald
    // sum): keep it per order for the life of the process
    static std::mutex mu;
    static std::map<int, std::vector<double>> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(p);
        if (it != cache.end()) {
            std::memcpy(out, it->second.data(), it->second.size() * sizeof(double));
            return;
        }
    }
    std::vector<cplx> c;
    lattice_coeffs(2 * p, c);
    build_real(p, Kind::Multipole, p, Kind::Local,
               [&](int ci, std::vector<cplx>& o) {
                   int n, mp;
                   decode(ci, n, mp);
                   for (int j = 0; j <= p; ++j)
                       for (int k = 0; k <= j; ++k) {
                           if (std::abs(k - mp) > j + n) continue;
                           double sg = ((n + mp) & 1) ? -1.0 : 1.0;
                           o[cidx(j, k)] += sg * c[cidx(j + n, k - mp)];
                       }
                   // dipole part of the background quadratic: -(4 pi / 3) t . D
                   if (n == 1) {
                       const double a = -4.0 * kPi / 3.0;
                       if (mp == 0) o[cidx(1, 0)] += a;
                       else if (mp == 1) o[cidx(1, 1)] += 2.0 * a;
                   }
               },
               out);
    std::lock_guard<std::mutex> lk(mu);
    cache[p].assign(out, out + (size_t)ncoef(p) * ncoef(p));
}

void build_periodic_green(int P, double* out) {
    static std::mutex mu;
    static std::map<int, std::vector<double>> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(P);
        if (it != cache.end()) {
            std::memcpy(out, it->second.data(), it->second.size() * sizeof(double));
            return;
        }
    }
    std::vector<cplx> c;
    lattice_coeffs(P, c);
    // h(u) = sum_L sum_M c_L^M R_L^M(u) is a potential: its real local
    // coefficients follow the local-expansion convention of the translations
    complex_to_real(P, Kind::Local, c, out);
    std::lock_guard<std::mutex> lk(mu);
    cache[P].assign(out, out + (size_t)ncoef(P));
}

}  // namespace fmmops
