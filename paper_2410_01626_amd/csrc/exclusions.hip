// Bonded exclusions: the pair terms of listed partners removed from the
// solve's potential, forces, site derivatives and energy.  A pair (i, j) is
// excluded through its minimum image (for a periodic cell the other images
// of the pair stay), the usual convention for bonded neighbours.  Included
// by fmm_api.hip after fmm_kernels.hip.
#pragma once

namespace fmmk {

// Interpolated charge of atom i (two forms, or four forms: Methods, eq 1 / 2),
// as the leaf kernel forms it, in FP64.
template <typename T>
__device__ __forceinline__ double excl_charge(const RepDesc& rd, int64_t i, const T* __restrict__ qA,
                                             const T* __restrict__ qB, const int32_t* __restrict__ site,
                                             const double* __restrict__ lam, const FormArgs<T>& fa) {
    const double a0 = (double)qA[i], b0 = (double)qB[i];
    const int32_t s = site[i];
    if (s < 0 || s >= rd.S) return a0;
    const double lp = lam[rd.s0 + s];
    if (fa.qC) {
        const double lt = fa.lam_t[rd.s0 + s], c0 = (double)fa.qC[i], d0 = (double)fa.qD[i];
        return (1.0 - lp) * ((1.0 - lt) * a0 + lt * b0) + lp * ((1.0 - lt) * c0 + lt * d0);
    }
    return a0 + lp * (b0 - a0);
}

// One thread per atom of replica blockIdx.y (caller order): removes
// k_e q_j / r from phi_i, k_e q_i q_j r / r^3 from F_i and the matching site
// term from cphi_i for every listed partner j of i, and leaves the block's
// share of the energy change (sum of -q_i dphi_i / k_e, in the units of the
// leaf energy partials, which the final reduction adds) in excl_e.  Partners
// outside the atom's replica are skipped.
template <typename T>
__global__ __launch_bounds__(256) void k_excl(Geo g, const RepDesc* __restrict__ reps,
                                              const T* __restrict__ x, const T* __restrict__ qA,
                                              const T* __restrict__ qB, const int32_t* __restrict__ site,
                                              const double* __restrict__ lam, FormArgs<T> fa,
                                              const double* __restrict__ dom_all,
                                              const int32_t* __restrict__ estart,
                                              const int32_t* __restrict__ eidx, T* __restrict__ phi,
                                              T* __restrict__ F, double* __restrict__ cphi, int unit_dq,
                                              double* __restrict__ excl_e) {
    __shared__ double red[256];
    const int r = blockIdx.y, t = threadIdx.x;
    const RepDesc rd = reps[r];
    const int64_t il = (int64_t)blockIdx.x * 256 + t;
    const double L = g.periodic ? dom_all[8 * r + 3] : 0.0;
    double e = 0.0;
    if (il < rd.n) {
        const int64_t i = rd.a0 + il;
        const double qi = excl_charge(rd, i, qA, qB, site, lam, fa);
        const double xi[3] = {(double)x[3 * i], (double)x[3 * i + 1], (double)x[3 * i + 2]};
        double dphi = 0.0, f[3] = {0.0, 0.0, 0.0};
        for (int32_t k = estart[i]; k < estart[i + 1]; ++k) {
            const int64_t j = eidx[k];
            if (j < rd.a0 || j >= rd.a0 + rd.n || j == i) continue;
            const double qj = excl_charge(rd, j, qA, qB, site, lam, fa);
            double d[3], r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double v = xi[a] - (double)x[3 * j + a];
                if (g.periodic) v -= L * rint(v / L);
                d[a] = v;
                r2 += v * v;
            }
            if (!(r2 > 0.0)) continue;
            const double ri = 1.0 / sqrt(r2), qr3 = qj * ri * ri * ri;
            dphi += qj * ri;
            for (int a = 0; a < 3; ++a) f[a] += qr3 * d[a];
        }
        const double ke = g.coulomb_k;
        if (phi) phi[i] = (T)((double)phi[i] - ke * dphi);
        if (F)
            for (int a = 0; a < 3; ++a) F[3 * i + a] = (T)((double)F[3 * i + a] - ke * qi * f[a]);
        const int32_t s = site[i];
        if (s >= 0 && s < rd.S) {
            const double dq = unit_dq ? 1.0 : (double)qB[i] - (double)qA[i];
            cphi[i] -= ke * dq * dphi;
        }
        e = -qi * dphi;
    }
    red[t] = e;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    if (t == 0) excl_e[(size_t)r * gridDim.x + blockIdx.x] = red[0];
}

}  // namespace fmmk
