// adjoint.hip -- reverse mode of the solve for upstream weights on the
// energy, the potentials and the forces,
//     L = gE E + sum_m gphi_m . phi_m + sum_m gF_m . F_m,
// in one tree pass.  Included by fmm_api.hip after fmm_kernels.hip.
//
// With phi = k_e Psi q (Psi the symmetric pair matrix of the Coulomb kernel
// psi, periodic images included), E = 1/2 q . phi and F_m = k_e q_m E_m(q),
// E_m(c) the field of charges c at atom m (self term removed),
//   dL/dq_m = gE phi_m + k_e [phi_m(g) - phi_m(p) + w_m . E_m(q)]
//   dL/dx_m = -gE F_m - k_e g_m E_m(q) - k_e q_m [E_m(g) - E_m(p) - (grad E(q))_m w_m]
// with g = gphi, w = gF and the dipoles p_j = q_j w_j; phi(p) and E(p) are
// the potential and field of those dipoles.  So a second set of sources,
// charges g with dipoles -p, runs through the same tree as the charges q
// (replica slot 1 of the plan's expansion arrays; every tree operator is
// linear in the sources), and the leaf pass forms, per target m,
//   A_m = phi_m(g, -p) + w_m . E_m(q)
//   B_m = E_m(g, -p) - (grad E(q))_m w_m
// from which dL/dq_m = gE phi_m + k_e A_m and
// dL/dx_m = -gE F_m - k_e g_m E_m(q) - k_e q_m B_m.  Per near pair (r = x_m -
// x_j, v = q_j (w_j - w_m)) the two are
//   A += g_j / r - (v . r) / r^3,   B += [(g_j - 3 (v . r) / r^2) r + v] / r^3,
// and in the far field the harmonics are evaluated as dual numbers along w_m
// (rho(u + e w) to first order in e), which gives the field gradient of the
// charges' local expansion applied to w_m.  No sum of large terms is
// differenced, so the result keeps the precision of a forward solve for any
// scale of the weights.
#pragma once

namespace fmmk {

// Like for_rho_orders, with the derivative of every harmonic along (dx, dy, dz):
// fn(kc, has_sin, re, im, dre, dim), d/de rho(u + e du) at e = 0.
template <typename T, typename Fn>
__device__ __forceinline__ void for_rho_orders_dual(int p, const RhoLds<T>& rc, int m0, int dm, T x, T y,
                                                    T z, T dx, T dy, T dz, Fn&& fn) {
    const T r2 = x * x + y * y + z * z;
    const T dr2 = T(2) * (x * dx + y * dy + z * dz);
    T cre = T(1), cim = T(0), dcre = T(0), dcim = T(0);
    int next = m0;
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            const T fm = rc.f[m];
            const T nre = fm * (x * cre - y * cim);
            const T nim = fm * (x * cim + y * cre);
            const T dnre = fm * (dx * cre + x * dcre - dy * cim - y * dcim);
            const T dnim = fm * (dx * cim + x * dcim + dy * cre + y * dcre);
            cre = nre;
            cim = nim;
            dcre = dnre;
            dcim = dnim;
        }
        if (m != next) continue;
        next += dm;
        const int k0 = (m == 0) ? 0 : 2 * m - 1;
        fn(m * m + k0, m > 0, cre, cim, dcre, dcim);
        if (m + 1 > p) continue;
        T p0re = cre, p0im = cim, d0re = dcre, d0im = dcim;
        const T a1 = rc.a[(m + 1) * (kPMax + 1) + m];
        T p1re = a1 * z * cre, p1im = a1 * z * cim;
        T d1re = a1 * (dz * cre + z * dcre), d1im = a1 * (dz * cim + z * dcim);
        fn((m + 1) * (m + 1) + k0, m > 0, p1re, p1im, d1re, d1im);
        for (int l = m + 2; l <= p; ++l) {
            const T al = rc.a[l * (kPMax + 1) + m];
            const T bl = rc.b[l * (kPMax + 1) + m];
            const T nre = al * z * p1re - bl * r2 * p0re;
            const T nim = al * z * p1im - bl * r2 * p0im;
            const T dnre = al * (dz * p1re + z * d1re) - bl * (dr2 * p0re + r2 * d0re);
            const T dnim = al * (dz * p1im + z * d1im) - bl * (dr2 * p0im + r2 * d0im);
            p0re = p1re;
            p0im = p1im;
            d0re = d1re;
            d0im = d1im;
            p1re = nre;
            p1im = nim;
            d1re = dnre;
            d1im = dnim;
            fn(l * l + k0, m > 0, p1re, p1im, d1re, d1im);
        }
    }
}

// Second sources of the adjoint, per leaf (one block of kLeafThreads, after
// the leaf kernel of the charges has sorted them): gathers (w, g) of every
// atom into leaf order (src2) and forms the leaf multipole of charges g and
// dipoles -q w, mu~_k = sum_j [g_j rho_k(u_j) - q_j (w~_j . grad) rho_k(u_j)]
// (u = t / h, w~ = w / h), into replica slot 1.  Periodic: the slot's FP64
// partial sums, sum [g |t|^2 - 2 q t . w] / L^2 (the dipoles' share of the
// second moment) and sum g.  Also copies the leaf offsets and the cube of
// slot 0 into slot 1, which the tree kernels of slot 1 read.
// Dynamic LDS: 64 x (K + 1) elements of T.
template <typename T>
__global__ __launch_bounds__(kLeafThreads) void k_leaf_src2(
    Geo g, const vec4_t<T>* __restrict__ pos, const int32_t* __restrict__ perm,
    int32_t* __restrict__ leaf_start_all, const T* __restrict__ gphi, const T* __restrict__ gF,
    double* __restrict__ dom_all, vec4_t<T>* __restrict__ src2, T* __restrict__ mult_all,
    double* __restrict__ leaf_part_all, uint16_t* __restrict__ msplit_all, int split_kp) {
    extern __shared__ __align__(16) unsigned char src2_lds[];
    __shared__ RhoLds<T> rho;
    __shared__ double ps[2][kLeafThreads / 64];
    T* rows = (T*)src2_lds;
    const int leaf = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int32_t* ls0 = leaf_start_all;
    int32_t* ls1 = leaf_start_all + (g.nleaf + 1);
    const int b = ls0[leaf], n = ls0[leaf + 1] - b;
    if (tid == 0) {
        ls1[leaf] = b;
        if (leaf + 1 == g.nleaf) ls1[g.nleaf] = ls0[g.nleaf];
    }
    if (leaf == 0 && tid < 4) dom_all[8 + tid] = dom_all[tid];
    load_rho_lds<T, kLeafThreads>(rho, g.p);
    const double edge = dom_all[3];
    const double h = edge / g.nb;
    const T ih = (T)(1.0 / h);
    int cx, cy, cz;
    unmorton((uint32_t)leaf, cx, cy, cz);
    const double off[3] = {(cx + 0.5) * h - 0.5 * edge, (cy + 0.5) * h - 0.5 * edge,
                           (cz + 0.5) * h - 0.5 * edge};
    double s2 = 0.0, qs = 0.0;
    for (int j = tid; j < n; j += kLeafThreads) {
        const int32_t i = perm[b + j];
        vec4_t<T> o;
        o.x = gF ? gF[3 * (size_t)i] : T(0);
        o.y = gF ? gF[3 * (size_t)i + 1] : T(0);
        o.z = gF ? gF[3 * (size_t)i + 2] : T(0);
        o.w = gphi ? gphi[i] : T(0);
        src2[b + j] = o;
        if (g.periodic) {
            const vec4_t<T> a = pos[b + j];
            const double t0 = (double)a.x + off[0], t1 = (double)a.y + off[1], t2 = (double)a.z + off[2];
            const double tw = t0 * (double)o.x + t1 * (double)o.y + t2 * (double)o.z;
            s2 += ((double)o.w * (t0 * t0 + t1 * t1 + t2 * t2) - 2.0 * (double)a.w * tw) / (edge * edge);
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
    __syncthreads();  // src2 of the leaf written (the passes below read it back)
    constexpr int kWaves = kLeafThreads / 64;
    const int S = g.K + 1;
    T acc = T(0);
    for (int c0 = 0; c0 < n; c0 += 64) {
        const int j = c0 + lane;
        vec4_t<T> a, w;
        a.x = a.y = a.z = a.w = T(0);
        w.x = w.y = w.z = w.w = T(0);
        if (j < n) {
            a = pos[b + j];
            w = src2[b + j];
        }
        const T q = a.w, gq = w.w;
        T* row = rows + lane * S;
        for_rho_orders_dual<T>(g.p, rho, wave, kWaves, a.x * ih, a.y * ih, a.z * ih, w.x * ih, w.y * ih,
                               w.z * ih, [&](int kc, bool hs, T re, T im, T dre, T dim) {
                                   row[kc] = gq * re - q * dre;
                                   if (hs) row[kc + 1] = gq * im - q * dim;
                               });
        __syncthreads();
        const int nr = min(64, n - c0);
        if (tid < g.K) {
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
        mult_all[((size_t)g.nbox + gb) * g.Kp + tid] = acc;
        if constexpr (sizeof(T) == 4)
            if (msplit_all)
                store_split(msplit_all + ((size_t)g.nbox + 1) * 2 * split_kp, split_kp, gb, tid, acc);
    }
    if (g.periodic && tid == 0) {
        double a2 = 0.0, aq = 0.0;
        for (int w = 0; w < kWaves; ++w) {
            a2 += ps[0][w];
            aq += ps[1][w];
        }
        double* lp1 = leaf_part_all + (size_t)g.nleaf * 2;
        lp1[2 * leaf] = a2;
        lp1[2 * leaf + 1] = aq;
    }
}

// Per target leaf (one block of kAdjWaves wavefronts): the near field of the
// 27 neighbour leaves from LDS tiles of (x - c, q) and (w, g) and the far
// field of both local expansions (slot 0: charges q; slot 1: charges g with
// dipoles -q w), giving per target m, in caller order, acc[8 m ..] = (phi(q),
// E(q), A, B) without k_e (the periodic background terms included).  A target
// chunk of tc atoms runs on lane groups of pow2ceil(tc) threads that take
// interleaved sources and orders; the groups' partials are added in a fixed
// order.  The neighbourhood is staged as in the forward near field (whole
// neighbours per wavefront when it fits one tile, else a binary search of
// the neighbour prefix sums with every thread's loads in flight), and only
// the target's own leaf needs the zero-distance guard.
constexpr int kAdjWaves = 8;
template <typename T, int kNW>
__global__ __launch_bounds__(64 * kNW, sizeof(T) == 4 ? 4 : 1) void k_near_adj(
    Geo g, const vec4_t<T>* __restrict__ pos, const vec4_t<T>* __restrict__ src2,
    const int32_t* __restrict__ leaf_start, const int32_t* __restrict__ perm,
    const double* __restrict__ dom_all, const T* __restrict__ loc_all, const int32_t* __restrict__ gidx,
    const T* __restrict__ gcoef, T* __restrict__ acc_out) {
    constexpr int NT = 64 * kNW;
    // sources staged per pass: a typical neighbourhood in one, two blocks per CU
    constexpr int CAP = sizeof(T) == 4 ? 2048 : 1024;
    static_assert(CAP % NT == 0, "whole staging rounds");
    static_assert(8 * NT * sizeof(T) <= CAP * sizeof(vec4_t<T>), "partials fit the source tile");
    __shared__ vec4_t<T> tile[CAP], tilew[CAP];
    __shared__ int nb_start[27], nb_cnt[27], nb_pre[29];
    __shared__ T nb_off[27][3];
    __shared__ T lam0[kKMax], lam1[kKMax];
    __shared__ T gr0[3][kKgMax], gr1[3][kKgMax];
    __shared__ RhoLds<T> rho;
    // the groups' partials (8 NT values) reuse the source tile after the sweep
    T* red = reinterpret_cast<T*>(tile);
    load_rho_lds<T, NT>(rho, g.p);
    const int leaf = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lb = leaf_start[leaf], ln = leaf_start[leaf + 1] - lb;
    if (ln == 0) return;
    const double edge = dom_all[3];
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
    const bool far = g.has_far;
    if (far) {
        const size_t lo = (size_t)(g.lev_off[g.depth] + leaf) * g.Kp;
        for (int k = tid; k < g.K; k += NT) {
            lam0[k] = loc_all[lo + k];
            lam1[k] = loc_all[(size_t)g.nbox * g.Kp + lo + k];
        }
    }
    __syncthreads();
    if (far) {
        for (int e = tid; e < 3 * g.Kg; e += NT) {
            const int a = e / g.Kg, r = e - a * g.Kg;
            T v0 = T(0), v1 = T(0);
            for (int t = 0; t < 4; ++t) {
                const int kk = gidx[(size_t)e * 4 + t];
                if (kk >= 0) {
                    const T c = gcoef[(size_t)e * 4 + t];
                    v0 += c * lam0[kk];
                    v1 += c * lam1[kk];
                }
            }
            gr0[a][r] = v0;
            gr1[a][r] = v1;
        }
    }
    __syncthreads();
    const int total = nb_pre[27];
    const T ih = (T)(1.0 / h);
    const double Q0 = g.periodic ? dom_all[4] : 0.0, G1 = g.periodic ? dom_all[8 + 4] : 0.0;
    for (int t0 = 0; t0 < ln; t0 += NT) {
        const int tc = min(NT, ln - t0);
        int gsz = 1;
        while (gsz < tc) gsz <<= 1;
        const int ngrp = NT / gsz, grp = tid / gsz, tl = tid & (gsz - 1);
        const bool tv = tl < tc;
        vec4_t<T> me, mw;
        me.x = me.y = me.z = me.w = T(0);
        mw.x = mw.y = mw.z = mw.w = T(0);
        if (tv) {
            me = pos[lb + t0 + tl];
            mw = src2[lb + t0 + tl];
        }
        T ph = T(0), ex = T(0), ey = T(0), ez = T(0), A = T(0), bx = T(0), by = T(0), bz = T(0);
        for (int s0 = 0; s0 < total; s0 += CAP) {
            const int cnt = min(CAP, total - s0);
            __syncthreads();  // the tiles' previous readers are done
            if (total <= CAP) {
                // the whole neighbourhood in one pass: wavefront w copies
                // neighbours w, w + kNW, ..., lane j their atom j (all loads
                // in flight together), larger neighbours in extra rounds
                constexpr int J = (27 + kNW - 1) / kNW;
                vec4_t<T> a[J], aw[J];
#pragma unroll
                for (int m = 0; m < J; ++m) {
                    const int nbk = min(wave + kNW * m, 26);
                    // an empty neighbour reads entry 0 (never stored)
                    const int c = nb_cnt[nbk];
                    const int src = c > 0 ? nb_start[nbk] + min(lane, c - 1) : 0;
                    a[m] = pos[src];
                    aw[m] = src2[src];
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
                        tilew[nb_pre[nbk] + lane] = aw[m];
                    }
                }
                for (int nbk = wave; nbk < 27; nbk += kNW)
                    for (int j = 64 + lane; j < nb_cnt[nbk]; j += 64) {
                        vec4_t<T> v = pos[nb_start[nbk] + j];
                        v.x += nb_off[nbk][0];
                        v.y += nb_off[nbk][1];
                        v.z += nb_off[nbk][2];
                        tile[nb_pre[nbk] + j] = v;
                        tilew[nb_pre[nbk] + j] = src2[nb_start[nbk] + j];
                    }
            } else {
                // stage the pass's sources, CAP / NT of each kind in flight per thread
                constexpr int G = CAP / NT;
                vec4_t<T> a[G], aw[G];
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
                    const int src = nb_start[lo] + (gsrc - nb_pre[lo]);
                    a[m] = pos[src];
                    aw[m] = src2[src];
                }
#pragma unroll
                for (int m = 0; m < G; ++m) {
                    if (tid + m * NT < cnt) {
                        vec4_t<T> v = a[m];
                        v.x += nb_off[lo_[m]][0];
                        v.y += nb_off[lo_[m]][1];
                        v.z += nb_off[lo_[m]][2];
                        tile[tid + m * NT] = v;
                        tilew[tid + m * NT] = aw[m];
                    }
                }
            }
            __syncthreads();
            if (tv) {
                // Only the own leaf (neighbour 13) can hold the target itself
                // or another atom at distance 0: the guard (zero weight at
                // r = 0, which zeroes every term) runs on that range alone.
                // Lane group grp takes the sources grp, grp + ngrp, ...
                const int own_b = nb_pre[13] - s0, own_e = nb_pre[14] - s0;
                auto sweep = [&](int j0, int j1, auto guard) {
                    const int first = j0 + ((grp - j0) & (ngrp - 1));
#pragma unroll 4
                    for (int j = first; j < j1; j += ngrp) {
                        const vec4_t<T> s = tile[j];
                        const vec4_t<T> sw = tilew[j];
                        const T dx = me.x - s.x, dy = me.y - s.y, dz = me.z - s.z;
                        const T r2 = dx * dx + dy * dy + dz * dz;
                        T ri;
                        if constexpr (decltype(guard)::value) ri = r2 > T(0) ? inv_sqrt<T>(r2) : T(0);
                        else ri = inv_sqrt<T>(r2);
                        const T ri2 = ri * ri;
                        const T ri3 = ri * ri2;
                        const T qr = s.w * ri;
                        const T qr3 = s.w * ri3;
                        ph += qr;
                        ex += qr3 * dx;
                        ey += qr3 * dy;
                        ez += qr3 * dz;
                        const T vx = s.w * (sw.x - mw.x), vy = s.w * (sw.y - mw.y), vz = s.w * (sw.z - mw.z);
                        const T vr = vx * dx + vy * dy + vz * dz;
                        A += sw.w * ri - vr * ri3;
                        const T c = sw.w - T(3) * vr * ri2;
                        bx += ri3 * (c * dx + vx);
                        by += ri3 * (c * dy + vy);
                        bz += ri3 * (c * dz + vz);
                    }
                };
                sweep(0, min(cnt, max(own_b, 0)), std::false_type{});
                sweep(max(own_b, 0), min(cnt, own_e), std::true_type{});
                sweep(max(own_e, 0), cnt, std::false_type{});
            }
        }
        if (far && tv) {
            T f0 = T(0), f1 = T(0), g0[3] = {T(0), T(0), T(0)}, d0[3] = {T(0), T(0), T(0)},
              g1[3] = {T(0), T(0), T(0)};
            const int Kg = g.Kg;
            for_rho_orders_dual<T>(g.p, rho, grp, ngrp, me.x * ih, me.y * ih, me.z * ih, mw.x * ih,
                                   mw.y * ih, mw.z * ih,
                                   [&](int kc, bool hs, T re, T im, T dre, T dim) {
                                       f0 += lam0[kc] * re;
                                       f1 += lam1[kc] * re;
                                       if (hs) {
                                           f0 += lam0[kc + 1] * im;
                                           f1 += lam1[kc + 1] * im;
                                       }
                                       if (kc < Kg) {
#pragma unroll
                                           for (int a = 0; a < 3; ++a) {
                                               g0[a] += gr0[a][kc] * re;
                                               d0[a] += gr0[a][kc] * dre;
                                               g1[a] += gr1[a][kc] * re;
                                               if (hs) {
                                                   g0[a] += gr0[a][kc + 1] * im;
                                                   d0[a] += gr0[a][kc + 1] * dim;
                                                   g1[a] += gr1[a][kc + 1] * im;
                                               }
                                           }
                                       }
                                   });
            const T ih2 = ih * ih;
            ph += f0 * ih;
            ex -= g0[0] * ih2;
            ey -= g0[1] * ih2;
            ez -= g0[2] * ih2;
            // A: potential of slot 1 plus w . (far field of the charges)
            A += f1 * ih - (mw.x * g0[0] + mw.y * g0[1] + mw.z * g0[2]) * ih2;
            // B: field of slot 1 minus the charges' field gradient along w
            bx += (d0[0] - g1[0]) * ih2;
            by += (d0[1] - g1[1]) * ih2;
            bz += (d0[2] - g1[2]) * ih2;
        }
        __syncthreads();  // every sweep is done with the tile
        red[0 * NT + tid] = ph;
        red[1 * NT + tid] = ex;
        red[2 * NT + tid] = ey;
        red[3 * NT + tid] = ez;
        red[4 * NT + tid] = A;
        red[5 * NT + tid] = bx;
        red[6 * NT + tid] = by;
        red[7 * NT + tid] = bz;
        __syncthreads();
        if (grp == 0 && tv) {
            double v[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                T s = T(0);
                for (int q = 0; q < ngrp; ++q) s += red[c * NT + q * gsz + tl];
                v[c] = (double)s;
            }
            if (g.periodic) {
                // background of a net charge (Q0 for q, G1 for g; dipoles carry none):
                // phi += (2 pi / 3) Q |t|^2 / V, field -= (4 pi / 3) Q t / V,
                // field gradient -= (4 pi / 3) Q / V
                const double V = edge * edge * edge;
                const double t[3] = {(double)me.x + (cx + 0.5) * h - 0.5 * edge,
                                     (double)me.y + (cy + 0.5) * h - 0.5 * edge,
                                     (double)me.z + (cz + 0.5) * h - 0.5 * edge};
                const double w[3] = {(double)mw.x, (double)mw.y, (double)mw.z};
                const double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
                const double tw = t[0] * w[0] + t[1] * w[1] + t[2] * w[2];
                const double c2 = 2.0 * kPi / 3.0 / V, c4 = 4.0 * kPi / 3.0 / V;
                v[0] += c2 * Q0 * t2;
                v[4] += c2 * G1 * t2 - c4 * Q0 * tw;
                for (int a = 0; a < 3; ++a) {
                    v[1 + a] -= c4 * Q0 * t[a];
                    v[5 + a] += c4 * (Q0 * w[a] - G1 * t[a]);
                }
            }
            const int32_t i = perm[lb + t0 + tl];
#pragma unroll
            for (int c = 0; c < 8; ++c) acc_out[8 * (size_t)i + c] = (T)v[c];
        }
    }
}

// Per atom m (caller order, one thread each): removes the pair terms of the
// listed exclusion partners (minimum image, FP64; same convention as k_excl)
// from (phi(q), E(q), A, B) and forms the outputs
//   phi_m = k_e phi(q), F_m = k_e q_m E(q),
//   dL/dq_m = gE phi_m + k_e A_m,
//   dL/dx_m = -gE F_m - k_e g_m E(q) - k_e q_m B_m,
//   dL/dqA_m = (1 - l) dL/dq_m, dL/dqB_m = l dL/dq_m (l = lambda of m's site,
//   0 without one), the site terms cphi = k_e (qB - qA) phi(q) and
//   cphi2 = (qB - qA) dL/dq, and the block's partial of sum q phi(q).
// gE is *gE_dev when that is set, else gE_val.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_combine(
    Geo g, int64_t n, int64_t S, const T* __restrict__ x, const T* __restrict__ qA,
    const T* __restrict__ qB, const int32_t* __restrict__ site, const double* __restrict__ lam,
    const T* __restrict__ gphi, const T* __restrict__ gF, const double* __restrict__ gE_dev, double gE_val,
    const double* __restrict__ dom_all,
    const int32_t* __restrict__ estart, const int32_t* __restrict__ eidx,
    const T* __restrict__ acc, T* __restrict__ phi_out, T* __restrict__ F_out, T* __restrict__ gx,
    T* __restrict__ gqA, T* __restrict__ gqB, double* __restrict__ cphi, double* __restrict__ cphi2,
    double* __restrict__ part) {
    __shared__ double red[4];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 256 + t;
    const RepDesc rd{0, n, 0, S, 0.0, 0};
    const FormArgs<T> fa{nullptr, nullptr, nullptr};
    const double gE = gE_dev ? *gE_dev : gE_val;
    double e = 0.0;
    if (i < n) {
        double v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = (double)acc[8 * i + c];
        const double qi = excl_charge(rd, i, qA, qB, site, lam, fa);
        const double gi = gphi ? (double)gphi[i] : 0.0;
        const double wi[3] = {gF ? (double)gF[3 * i] : 0.0, gF ? (double)gF[3 * i + 1] : 0.0,
                              gF ? (double)gF[3 * i + 2] : 0.0};
        if (estart) {
            const double L = g.periodic ? dom_all[3] : 0.0;
            const double xi[3] = {(double)x[3 * i], (double)x[3 * i + 1], (double)x[3 * i + 2]};
            for (int32_t k = estart[i]; k < estart[i + 1]; ++k) {
                const int64_t j = eidx[k];
                if (j < 0 || j >= n || j == i) continue;
                const double qj = excl_charge(rd, j, qA, qB, site, lam, fa);
                const double gj = gphi ? (double)gphi[j] : 0.0;
                double d[3], r2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double u = xi[a] - (double)x[3 * j + a];
                    if (g.periodic) u -= L * rint(u / L);
                    d[a] = u;
                    r2 += u * u;
                }
                if (!(r2 > 0.0)) continue;
                const double ri = 1.0 / sqrt(r2), ri2 = ri * ri, ri3 = ri * ri2;
                double vv[3], vr = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double wj = gF ? (double)gF[3 * j + a] : 0.0;
                    vv[a] = qj * (wj - wi[a]);
                    vr += vv[a] * d[a];
                }
                const double c = gj - 3.0 * vr * ri2;
                v[0] -= qj * ri;
                v[4] -= gj * ri - vr * ri3;
                for (int a = 0; a < 3; ++a) {
                    v[1 + a] -= qj * ri3 * d[a];
                    v[5 + a] -= ri3 * (c * d[a] + vv[a]);
                }
            }
        }
        const double ke = g.coulomb_k;
        const double ph = ke * v[0];
        const double gq = gE * ph + ke * v[4];
        if (phi_out) phi_out[i] = (T)ph;
        for (int a = 0; a < 3; ++a) {
            const double F = ke * qi * v[1 + a];
            if (F_out) F_out[3 * i + a] = (T)F;
            if (gx) gx[3 * i + a] = (T)(-gE * F - ke * gi * v[1 + a] - ke * qi * v[5 + a]);
        }
        const int32_t s = site[i];
        const bool sited = s >= 0 && s < S;
        const double l = sited ? lam[s] : 0.0;
        if (gqA) gqA[i] = (T)((1.0 - l) * gq);
        if (gqB) gqB[i] = (T)(l * gq);
        if (sited) {
            const double dq = (double)qB[i] - (double)qA[i];
            cphi[i] = ke * dq * v[0];
            cphi2[i] = dq * gq;
        }
        e = qi * v[0];
    }
    // fixed order: a DPP scan within each wavefront, then the four sums in order
    e = wave_sum<double>(e);
    if ((t & 63) == 0) red[t >> 6] = e;
    __syncthreads();
    if (t == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

}  // namespace fmmk
