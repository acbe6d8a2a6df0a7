// operators.h -- FP64 translation-operator tables of the fast multipole method,
// built once per (order p) on the host when a plan is created.
//
// Basis.  Expansions use real, "fully normalised" regular solid harmonics
//   Rh_l^m(r) = sqrt((l-m)!/(l+m)!) r^l P_l^m(cos th) e^{i m ph}
// (P_l^m with the Condon-Shortley phase), stored per degree l as
//   [Re Rh_l^0, Re Rh_l^1, Im Rh_l^1, ..., Re Rh_l^l, Im Rh_l^l]
// at offset l*l, so an order-p expansion has K = (p+1)^2 real coefficients.
// A multipole about centre c is mu = sum_j q_j rho(x_j - c) and the far
// potential it produces is phi(t) = sum_k lambda_k rho_k(t - c') for the local
// expansion lambda about c'.  Coefficients are stored scaled by the box edge h
// of their tree level: mu~_l = mu_l / h^l and lambda~_l = lambda_l h^(l+1), so
// every operator below depends only on integer box offsets and is shared by
// all levels and all box sizes.
//
// The mathematics is the textbook multipole method of Greengard and Rokhlin,
// which the paper adopts as its Coulomb solver; the translation identities
// (regular-harmonic addition theorem, irregular-harmonic translation) are
// standard results for these harmonics.
#pragma once
#include <cstdint>

namespace fmmops {

constexpr int kMaxOrder = 16;
inline int ncoef(int p) { return (p + 1) * (p + 1); }
inline int ridx(int l, int m, int part) { return l * l + (m == 0 ? 0 : 2 * m - 1 + part); }

// M2L: lambda~_t += T(o) mu~_s for o = (t - s) in box units, o in [-3,3]^3.
// out: 343 blocks of K*K row-major (row = output coefficient), block index
// ((ox+3)*7 + (oy+3))*7 + (oz+3); blocks with max|o_a| <= 1 are zero.
void build_m2l_bank(int p, double* out);

// M2M: mu~_parent += A_c mu~_child for child octant c = 4*bx + 2*by + bz where
// the child centre is parent centre + (b - 1/2) * h_child.  out: 8 blocks K*K.
void build_m2m(int p, double* out);

// L2L: lambda~_child += B_c lambda~_parent, same octant numbering.  8 blocks K*K.
void build_l2l(int p, double* out);

// Gradient table: for a local expansion lambda (order p) the derivative of
// sum_k lambda_k rho_k(t) along axis a equals sum_k g_a,k rho_k(t) with
// g_a = G_a lambda (order p-1, p*p coefficients).  Each row of G_a has at most
// 4 non-zeros; out_idx/out_coef hold [3][p*p][4] entries (index -1 = unused).
void build_grad_table(int p, int32_t* out_idx, double* out_coef);

// Periodic lattice operator for a cubic unit cell (scale-free):
// lambda~_root += Lat mu~_root accounts for all periodic images outside the
// 3x3x3 block of cells around the root, under conducting (tin-foil)
// surroundings, a uniform neutralising background and the zero-mean gauge.
// The non-harmonic remainder of the background term is applied separately:
// lambda~_0 += (2 pi / 3) sum_j q_j |s_j / L|^2 and, at every target,
// phi += (2 pi / 3) Q |t / L|^2 / L (s, t relative to the cell centre).
// out: K*K row-major.
void build_lattice(int p, double* out);

// Periodic Green's function of the unit cube (tin-foil, neutralising
// background, zero mean) near the origin:
//   psi(u) = sum_{n in {-1,0,1}^3} 1/|u + n| + (2 pi / 3)|u|^2 + h(u),
// with h harmonic for |u| < 2.  out: the K = (P+1)^2 real local coefficients
// of h (h(u) = sum_k out[k] rho_k(u)); psi of a cell of edge L at r is
// psi(r / L) / L.
void build_periodic_green(int P, double* out);

// Evaluate the real normalised regular harmonics rho(r) (K values) -- the same
// recurrence the kernels use, exposed for host-side checks.
void eval_rho(int p, const double r[3], double* out);

}  // namespace fmmops
