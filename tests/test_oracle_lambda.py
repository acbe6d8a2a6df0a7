"""Pins of the lambda-dynamics oracle (bias potentials, velocity Verlet, Bussi
thermostat, partition function correction, DBO) against closed forms,
textbook values, a library evaluation of the same definition and the paper's
stated constants."""
import math

import numpy as np
import pytest

from oracle import lambda_dynamics as L


def test_hermite_reproduces_a_cubic_and_is_c1():
    # a cubic Hermite spline fed a cubic's values and slopes is that cubic
    a, b, c, d = 0.3, -1.7, 2.2, 0.9
    f = lambda t: a + b * t + c * t ** 2 + d * t ** 3
    fp = lambda t: b + 2 * c * t + 3 * d * t ** 2
    x = np.array([-0.4, 0.1, 0.35, 0.9, 1.3])
    t = np.linspace(-0.4, 1.3, 301)
    V, dV = L.hermite(x, f(x), fp(x), t)
    assert np.allclose(V, f(t), atol=1e-13) and np.allclose(dV, fp(t), atol=1e-12)
    # linear continuation with the end slopes outside the knots
    V, dV = L.hermite(x, f(x), fp(x), np.array([-1.0, 2.0]))
    assert np.allclose(V, [f(x[0]) + fp(x[0]) * (-0.6), f(x[-1]) + fp(x[-1]) * 0.7])
    # value and slope continuous across every knot of the double well
    kx, ky, ks = L.dw_knots(6.0, 0.02, 0.97, -1.3)
    eps = 1e-9
    lo, dlo = L.hermite(kx, ky, ks, kx - eps)
    hi, dhi = L.hermite(kx, ky, ks, kx + eps)
    assert np.allclose(lo, hi, atol=1e-6) and np.allclose(dlo, dhi, atol=1e-5)


def test_double_well_template_shape():
    B, p0, p1, y1 = 6.0, -0.03, 1.05, 0.7
    V, dV = L.v_dw(np.tile([B, p0, p1, y1], (3, 1)), np.array([p0, 0.5 * (p0 + p1), p1]))
    assert np.allclose(V, [0.0, B, y1]) and np.allclose(dV, 0.0)
    # derivative agrees with central differences of the value
    # (off the knots, where the second derivative jumps; past the end knots
    # the confining quadratic wall)
    t = np.linspace(-0.5, 1.5, 41) + 0.0123
    dwp = np.tile([B, p0, p1, y1], (t.size, 1))
    h = 1e-6
    Vp, _ = L.v_dw(dwp, t + h)
    Vm, _ = L.v_dw(dwp, t - h)
    _, dV = L.v_dw(dwp, t)
    assert np.allclose((Vp - Vm) / (2 * h), dV, atol=1e-4)
    # the walls: linear continuation of the end slope plus (k / 2) d^2
    V, dV = L.v_dw(np.tile([B, p0, p1, y1], (2, 1)), np.array([p0 - 0.4, p1 + 0.5]))
    assert V[0] == pytest.approx(30.0 + 300.0 * 0.1 + 0.5 * L.WALL_K * 0.1 ** 2)
    assert dV[1] == pytest.approx(300.0 + L.WALL_K * 0.2)


def test_mm_bias_flattens_the_reference_landscape():
    # V_MM cancels the reference compound's mean dH/dlambda: G(own, partner)
    # from numpy's own 2-D polynomial evaluation plus dV_MM/dlambda is zero
    rng = np.random.default_rng(5)
    C = 6
    mm = rng.normal(0, 10, (C, 36))
    lam = rng.uniform(-0.1, 1.1, C)
    partner = np.array([1, 0, -1, 4, 3, -1], dtype=np.int32)
    got = L.mm_slope(mm, lam, partner)
    for c in range(C):
        y = lam[partner[c]] if partner[c] >= 0 else 0.0
        G = np.polynomial.polynomial.polyval2d(lam[c], y, mm[c].reshape(6, 6))
        assert got[c] + G == pytest.approx(0.0, abs=1e-9 * max(1.0, abs(G)))


def test_ph_term_matches_eq4_and_the_textbook_value():
    # eq 4: V_pH(1) - V_pH(0) = ln(10) R T (pKa_ref - pH); one pH unit at
    # 298.15 K is 5.708 kJ/mol (2.303 RT)
    s = L.ph_slope(np.array([5.0, np.nan]), np.array([4.0, 4.0]), 298.15)
    assert s[0] == pytest.approx(5.708, abs=5e-4)
    assert s[1] == 0.0
    # the step's bias energy difference between lambda = 1 and 0
    _, e1 = L.lambda_forces(np.array([1.0]), np.zeros(1), np.array([-1]), np.array([7.0]),
                            np.array([3.5]), None, None, 300.0)
    _, e0 = L.lambda_forces(np.array([0.0]), np.zeros(1), np.array([-1]), np.array([7.0]),
                            np.array([3.5]), None, None, 300.0)
    assert e1[0] - e0[0] == pytest.approx(math.log(10) * 8.314462618e-3 * 300.0 * 3.5, rel=1e-14)


def _harmonic_run(dt, t_end, k=50.0, m=60.0, lam0=0.4, v0=0.0):
    """Velocity Verlet on V_MM = k lambda^2 / 2 (G = -k lambda) alone."""
    mm = np.zeros((1, 36))
    mm[0, 6] = -k  # g_10: G = -k lambda
    lam, v = np.array([lam0]), np.array([v0])
    off = np.array([0, 1])
    n = int(round(t_end / dt))
    energies = []
    for i in range(n + 1):
        lam_n = lam.copy()
        lam, v, kin, _ = L.lambda_step(off, lam, v, np.zeros(1), np.array([-1]), np.array([np.nan]),
                                       np.array([7.0]), mm, None, np.zeros((1, 2)), m, dt, 300.0,
                                       0.0, i == 0)
        energies.append(kin[0] + 0.5 * k * lam_n[0] ** 2)
        if i == n:
            return lam_n[0], np.array(energies)


def test_velocity_verlet_converges_at_second_order_and_keeps_energy():
    k, m, lam0 = 50.0, 60.0, 0.4
    w = math.sqrt(k / m)
    t_end = 2.0
    exact = lam0 * math.cos(w * t_end)
    e1 = abs(_harmonic_run(0.02, t_end)[0] - exact)
    e2 = abs(_harmonic_run(0.01, t_end)[0] - exact)
    assert 3.6 < e1 / e2 < 4.4  # second order
    _, en = _harmonic_run(0.01, 20.0)
    E0 = 0.5 * k * lam0 ** 2
    assert np.max(np.abs(en - E0)) < 1e-4 * E0  # bounded, O(dt^2) fluctuation


def test_bussi_rescaling_keeps_the_canonical_kinetic_distribution():
    # K ~ Gamma(N_f / 2, k_B T) is stationary under the rescaling for any
    # coupling: compare the first three moments after one update
    rng = np.random.default_rng(11)
    nf, T, c = 5, 300.0, 0.8
    kT = L.KB * T
    kbar = 0.5 * nf * kT
    n = 400_000
    K = rng.gamma(nf / 2, kT, n)
    R1 = rng.standard_normal(n)
    chi2 = rng.chisquare(nf - 1, n)
    Kn = (K + (1 - c) * (kbar * (R1 ** 2 + chi2) / nf - K)
          + 2 * R1 * np.sqrt(K * kbar / nf * (1 - c) * c))
    got = np.array([L.bussi_kinetic(K[i], nf, kbar, c, R1[i], chi2[i]) for i in range(0, n, 4000)])
    assert np.allclose(got, Kn[::4000], rtol=1e-14)
    mean, var = nf / 2 * kT, nf / 2 * kT ** 2
    skew = 2 / math.sqrt(nf / 2)
    assert abs(Kn.mean() - mean) < 5 * math.sqrt(var / n)
    assert abs(Kn.var() / var - 1) < 0.02
    sk = np.mean((Kn - Kn.mean()) ** 3) / Kn.std() ** 3
    assert abs(sk - skew) < 0.05
    # limits: no coupling keeps K; instant coupling draws K from the target
    assert L.bussi_kinetic(3.0, nf, kbar, 1.0, 0.7, 2.0) == 3.0
    assert L.bussi_kinetic(3.0, nf, kbar, 0.0, 0.7, 2.0) == pytest.approx(kbar * (0.49 + 2.0) / nf)


def test_thermostat_scales_each_replica_separately():
    rng = np.random.default_rng(3)
    off = np.array([0, 3, 7])
    C = 7
    lam = rng.uniform(0, 1, C)
    v = rng.normal(0, 1, C)
    noise = np.array([[0.4, 1.3], [-0.8, 2.5]])
    m, dt, T, tau = 60.0, 0.002, 300.0, 0.5
    lam1, v1, kin, _ = L.lambda_step(off, lam, v, np.zeros(C), np.full(C, -1), np.full(C, np.nan),
                                     np.array([7.0, 7.0]), None, None, noise, m, dt, T, tau, True)
    # no forces: v1 is the rescaled v; the ratio is one alpha per replica
    for r in range(2):
        a, b = off[r], off[r + 1]
        ratio = v1[a:b] / v[a:b]
        assert np.allclose(ratio, ratio[0])
        K = 0.5 * m * np.sum(v[a:b] ** 2)
        assert kin[r] == pytest.approx(K)
        kbar = 0.5 * (b - a) * L.KB * T
        Kn = L.bussi_kinetic(K, b - a, kbar, math.exp(-dt / tau), *noise[r])
        assert ratio[0] == pytest.approx(math.sqrt(Kn / K), rel=1e-13)
    assert np.allclose(lam1, lam + dt * v1)


def test_pfc_free_energy_closed_forms():
    T = 300.0
    kT = L.KB * T
    assert L.pfc_dg(lambda x: 0.0, T) == pytest.approx(0.0, abs=1e-12)
    # V = a lambda: Z_deprot / Z_prot = exp(-a / (2 kT)), so dG = a / 2
    for a in (-7.0, 3.0, 11.0):
        assert L.pfc_dg(lambda x, a=a: a * x, T) == pytest.approx(a / 2, rel=1e-10)
    # a landscape symmetric about 1/2 has dG = 0
    assert L.pfc_dg(lambda x: 5 * (x - 0.5) ** 2 + math.cos(9 * (x - 0.5)), T) == pytest.approx(0.0, abs=1e-10)
    # V = b (x - 1/2)^2 + a x: closed form through the error function
    a, b = 2.0, 20.0
    beta = 1 / kT
    # integral of exp(-beta (b u^2 + a u)) over u in [0, 1/2] and [-1/2, 0]
    # (u = x - 1/2; the constant a/2 cancels in the ratio)
    def gauss_int(lo, hi):
        s = math.sqrt(beta * b)
        shift = a / (2 * b)
        pre = math.exp(beta * a * a / (4 * b)) * math.sqrt(math.pi) / (2 * s)
        return pre * (math.erf(s * (hi + shift)) - math.erf(s * (lo + shift)))
    dg = -kT * math.log(gauss_int(0.0, 0.5) / gauss_int(-0.5, 0.0))
    assert L.pfc_dg(lambda x: b * (x - 0.5) ** 2 + a * x, T) == pytest.approx(dg, rel=1e-10)


def test_pfc_solve_hits_the_target():
    T = 300.0
    # symmetric wells and no pH term: the correction is zero
    assert L.pfc_solve(6.0, 0.0, 1.0, float("nan"), 7.0, T) == pytest.approx(0.0, abs=1e-9)
    for B, p0, p1, pka, ph in ((6.0, 0.02, 0.97, 4.0, 5.5), (12.0, -0.05, 1.06, 6.5, 4.0)):
        y1 = L.pfc_solve(B, p0, p1, pka, ph, T)
        slope = math.log(10) * L.KB * T * (pka - ph)
        dg = L.pfc_dg(L.pfc_landscape(B, p0, p1, y1, slope), T)
        assert dg == pytest.approx(math.log(10) * L.KB * T * (pka - ph), abs=1e-9)


def test_pfc_out_of_reach_stays_at_the_bound():
    # low barrier, pKa - pH = 8: the barrier-top half of [1/2, 1] alone keeps
    # the free energy below the 46 kJ/mol target whatever y1 is
    T = 300.0
    y1 = L.pfc_solve(1.0, 0.0, 1.0, 12.0, 4.0, T)
    assert y1 == 200.0
    dg = L.pfc_dg(L.pfc_landscape(1.0, 0.0, 1.0, 200.0, math.log(10) * L.KB * T * 8.0), T)
    assert dg < math.log(10) * L.KB * T * 8.0
    assert L.pfc_solve(1.0, 0.0, 1.0, 4.0, 12.0, T) > -200.0  # the other side is reachable


def test_dbo_rules_follow_the_paper_constants():
    dwp = np.array([[6.0, 0.0, 1.0, 0.0]] * 6)
    n = 100.0
    sw = np.zeros((6, 5))
    # 0: 80% near 0 with mean 0.05 -> well 0 moves by -0.025
    sw[0] = [n, 80, 80 * 0.05, 10, 10 * 0.9]
    # 1: 60% near 0 (below the 70% occupancy) -> no move
    sw[1] = [n, 60, 60 * 0.05, 30, 30 * 0.95]
    # 2: 90% near 1 with mean 0.98 (inside the 0.03 tolerance) -> no move
    sw[2] = [n, 5, 5 * 0.1, 90, 90 * 0.98]
    # 3: 90% near 1 with mean 0.90 -> well 1 moves by +0.05
    sw[3] = [n, 5, 5 * 0.1, 90, 90 * 0.90]
    # 4: 75% near 0 with mean 0.4 -> clamped at +0.08
    sw[4] = [n, 75, 75 * 0.19, 10, 10 * 0.9]
    sb = np.zeros((6, 2))
    sb[:, 0] = n
    sb[:, 1] = [10, 40, 25, 21, 29, 50]  # transition fractions
    nan = np.full(6, np.nan)
    out, adj, sw2, sb2 = L.dbo_update(sw, sb, dwp, 3, nan, np.full(6, 7.0), 300.0, pfc=False)
    assert out[0, 1] == pytest.approx(-0.025) and out[0, 2] == 1.0
    assert out[1, 1] == 0.0 and out[2, 2] == 1.0
    assert out[3, 2] == pytest.approx(1.05)
    assert out[4, 1] == pytest.approx(-0.08)  # mean 0.19: -0.095, clamped
    # barrier: 10% -> down one step, 40% -> up, 25/21/29% -> inside 25 +- 5
    assert list(out[:, 0]) == [5.0, 7.0, 6.0, 6.0, 6.0, 7.0]
    assert list(adj) == [1, 1, 0, 1, 1, 1]
    assert not sw2.any() and not sb2.any()
    # clamps of the barrier range [1, 20]
    lo = np.array([[1.0, 0.0, 1.0, 0.0], [20.0, 0.0, 1.0, 0.0]])
    out, adj, _, _ = L.dbo_update(np.zeros((2, 5)), np.array([[n, 0.0], [n, 90.0]]), lo, 2,
                                  np.full(2, np.nan), np.full(2, 7.0), 300.0, pfc=False)
    assert list(out[:, 0]) == [1.0, 20.0] and list(adj) == [0, 0]
    # with the correction, adjusted coordinates get the matching well height
    out, adj, _, _ = L.dbo_update(sw[:1], sb[:1], dwp[:1], 3, np.array([5.0]), np.array([6.0]),
                                  300.0, pfc=True)
    assert out[0, 3] == pytest.approx(L.pfc_solve(out[0, 0], out[0, 1], out[0, 2], 5.0, 6.0, 300.0))


def test_block_statistics():
    lam = np.array([0.1, 0.5, 0.9, -0.05, 0.2, 0.8])
    sw, sb = L.accumulate_stats(lam, np.zeros((6, 5)), np.zeros((6, 2)))
    assert list(sw[:, 1]) == [1, 0, 0, 1, 0, 0]
    assert list(sw[:, 3]) == [0, 0, 1, 0, 0, 0]
    assert sw[3, 2] == -0.05 and sw[2, 4] == 0.9
    assert list(sb[:, 1]) == [0, 1, 0, 0, 1, 1]


def _tautomer_site():
    # coordinates 0 (protonation, pKa 5) and 1 (its tautomer, no pKa) form one
    # site; coordinate 2 is a plain protonation coordinate without a partner
    partner = np.array([1, 0, -1])
    pka = np.array([5.0, np.nan, 6.0])
    dwp = np.array([[6.0, 0.0, 1.0, 0.4], [6.0, 0.02, 0.98, 0.0], [5.0, 0.0, 1.0, -0.3]])
    dwp2 = np.array([[9.0, 1.0], [2.0, 0.3], [11.0, 2.0]])
    return partner, pka, dwp, dwp2


def test_tautomer_second_barrier_switches_with_the_protonation_state():
    """The tautomer coordinate takes its second barrier only while its site is
    deprotonated (partner lambda >= 1/2, lambda = 0 protonated); protonation
    coordinates ignore dwp2; with B2 = B the forces are the one-barrier ones."""
    partner, pka, dwp, dwp2 = _tautomer_site()
    for lp, expect in ((0.1, False), (0.49, False), (0.5, True), (0.93, True)):
        lam = np.array([lp, 0.37, 0.8])
        sec = L.second_state(lam, partner, pka, dwp2)
        assert list(sec) == [False, expect, False]
        F, eb = L.lambda_forces(lam, np.zeros(3), partner, pka, np.full(3, 7.0), None, dwp, 300.0,
                                dwp2)
        used = dwp.copy()
        if expect:
            used[1, 0], used[1, 3] = dwp2[1]
        Fr, ebr = L.lambda_forces(lam, np.zeros(3), partner, pka, np.full(3, 7.0), None, used, 300.0)
        assert np.array_equal(F, Fr) and np.array_equal(eb, ebr)
        # the tautomer coordinate's barrier top value is the barrier in force
        m = 0.5 * (dwp[1, 1] + dwp[1, 2])
        V, _ = L.v_dw(L.dw_params(dwp, dwp2, sec), np.array([0.0, m, 0.0]))
        assert V[1] == pytest.approx(dwp2[1, 0] if expect else dwp[1, 0])
    same = dwp2.copy()
    same[1] = [dwp[1, 0], dwp[1, 3]]
    lam = np.array([0.8, 0.37, 0.8])
    a = L.lambda_forces(lam, np.zeros(3), partner, pka, np.full(3, 7.0), None, dwp, 300.0, same)
    b = L.lambda_forces(lam, np.zeros(3), partner, pka, np.full(3, 7.0), None, dwp, 300.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_tautomer_barrier_statistics_and_dbo_per_state():
    """In-transition statistics of the deprotonated state go to stats_b2 and
    move only the second barrier (down when the tautomer rarely crosses in
    that state, the paper's reason for a lower barrier there); the correction
    gives each state its own y1: for symmetric wells without pKa the free
    energy of either state is zero at y1 = 0, whatever the barrier."""
    partner, pka, dwp, dwp2 = _tautomer_site()
    dwp[1] = [6.0, 0.0, 1.0, 0.4]
    sw, sb, sb2 = np.zeros((3, 5)), np.zeros((3, 2)), np.zeros((3, 2))
    # 100 steps protonated with the tautomer half in transition, then 100
    # deprotonated with it never in transition
    for k in range(200):
        lp = 0.1 if k < 100 else 0.9
        lt = 0.5 if (k < 100 and k % 2) else 0.05
        lam = np.array([lp, lt, 0.5])
        sec = L.second_state(lam, partner, pka, dwp2)
        sw, sb, sb2 = L.accumulate_stats(lam, sw, sb, stats_b2=sb2, second=sec)
    assert np.array_equal(sb[1], [100, 50]) and np.array_equal(sb2[1], [100, 0])
    assert np.array_equal(sb[0], [200, 0]) and np.array_equal(sb2[0], [0, 0])
    d, adj, _, sbc, d2, sb2c = L.dbo_update(sw, sb, dwp, 2, pka, np.full(3, 7.0), 300.0,
                                            dwp2=dwp2, stats_b2=sb2, partner=partner)
    assert d[1, 0] == 7.0          # 50% in transition: above target + tol, up one step
    assert d2[1, 0] == 1.0         # 0% in the deprotonated state: down, clamped at 1
    assert d2[0, 0] == dwp2[0, 0]  # protonation coordinates keep their dwp2 untouched
    assert adj[1] == 1
    assert d[1, 3] == pytest.approx(0.0, abs=1e-9) and d2[1, 1] == pytest.approx(0.0, abs=1e-9)
    assert not sbc.any() and not sb2c.any()
