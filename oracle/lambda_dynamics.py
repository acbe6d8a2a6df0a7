"""FP64 CPU oracle for the lambda-dynamics step around the Coulomb solve.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the product library never does, and
this module never imports the product package.  Plain numpy in float64, with
scipy's adaptive quadrature and root finder as library steps.

What is computed (constant-pH paper, Methods: the extended Hamiltonian of
lambda-dynamics, eq 1; "Calibration of Protonation Dynamics": the split of the
bias V = V_MM + V_pH + V_dw, eq 3, and the pH term, eq 4; "Partition Function
Correction"; "Dynamic Barrier and Well Optimization"; "Constant pH Parameters":
velocity Verlet for the lambda particles and the Bussi-Donadio-Parrinello
thermostat on the lambda subsystem).

Units: lambda is dimensionless, energies kJ/mol, mass u (g/mol), time ps, so
that a force of 1 kJ/mol per unit lambda on a mass of 1 u accelerates by
1 ps^-2.

Readings of the paper taken here (each also listed in the design notes):
  * V_MM: the fitted polynomial G(l_own, l_partner) = sum_{i,j<=5} g_ij
    l_own^i l_partner^j approximates the reference compound's mean
    dH_ref/dlambda; V_MM is minus the integrated TI profile, so dV_MM/dlambda
    = -G and the reference landscape is flat.  A coordinate without a partner
    evaluates G at l_partner = 0.
  * V_pH is linear in lambda, V_pH = lambda ln(10) k_B T (pKa_ref - pH), the
    simplest form with the end-point difference of eq 4; coordinates with no
    pKa (tautomer coordinates) have no pH term.
  * V_dw is the cubic Hermite spline of five knots built from (B, p0, p1, y1)
    by dw_knots below (synthetic shape: the calibrated splines are not
    available), extended linearly beyond its end knots plus a confining
    quadratic wall there.
  * Thermostat: one Bussi thermostat per replica over all its lambda
    coordinates (N_f = their number), applied to the full-step velocities,
    positive square root of the kinetic-energy ratio; the random numbers
    (one standard normal R1 and one chi-square sample with N_f - 1 degrees of
    freedom per replica and step) are inputs.
  * PFC: the free energy of deprotonation -k_B T ln(Z_deprot / Z_prot), with
    the integrals over [0, 1/2] and [1/2, 1] as the paper writes them, of
    exp(-(V_pH + V_dw) / k_B T), matched to ln(10) k_B T (pKa_ref - pH)
    (0 for a coordinate without pKa) by moving the height y1 of well 1 within
    [-200, 200] kJ/mol; a target out of reach there (large pKa_ref - pH over a
    low barrier) leaves y1 at the nearer end.
  * DBO: a well moves by -gain (mean - ideal) when the coordinate spent more
    than the occupancy threshold of the block near it and |mean - ideal|
    exceeds the tolerance, its total offset from the ideal end point clamped
    to +-max_shift; the barrier moves one step down (up) when the in-transition
    fraction is below (above) target -+ tolerance, clamped to [B_min, B_max].
  * Tautomer coordinates (no pKa, a partner: the site's protonation
    coordinate) may carry a second barrier (dwp2 = (B2, y1_2) per coordinate):
    V_dw uses (B, y1) while the site is protonated (partner lambda < 1/2,
    lambda = 0 being protonated) and (B2, y1_2) while it is deprotonated; the
    in-transition statistics of the two states go to stats_b and stats_b2,
    and DBO adjusts each barrier from its own statistics; the correction
    gives each state its own y1.  The wells are shared.
"""
from __future__ import annotations

import math

import numpy as np

KB = 8.314462618e-3  # Boltzmann constant, kJ mol^-1 K^-1 (molar gas constant)
LN10 = math.log(10.0)

# synthetic double-well template: wall knots 0.3 from each well, 30 kJ/mol
# above it, with slope 300 kJ/mol per unit lambda; beyond them the linear
# continuation gains a confining (WALL_K / 2) d^2, d the distance past the knot
WALL_DX, WALL_DY, WALL_SLOPE, WALL_K = 0.3, 30.0, 300.0, 2.0e4

# DBO constants as the paper states them ("Dynamic Barrier and Well Optimization")
DBO_DEFAULTS = dict(near0=0.2, near1=0.8, occupancy=0.7, well_tol=0.03, well_gain=0.5,
                    max_shift=0.08, target=0.25, target_tol=0.05, barrier_step=1.0,
                    barrier_min=1.0, barrier_max=20.0)


def dw_knots(B, p0, p1, y1):
    """Knots (x, y, slope) of the double well: walls, well 0 (height 0), the
    barrier top B midway between the wells, well 1 (height y1), wall."""
    m = 0.5 * (p0 + p1)
    x = np.array([p0 - WALL_DX, p0, m, p1, p1 + WALL_DX])
    y = np.array([WALL_DY, 0.0, B, y1, y1 + WALL_DY])
    s = np.array([-WALL_SLOPE, 0.0, 0.0, 0.0, WALL_SLOPE])
    return x, y, s


def hermite(x, y, s, t):
    """Cubic Hermite spline through (x_k, y_k) with slopes s_k at the points t
    (value, derivative); linear with the end slope outside [x_0, x_n]."""
    t = np.asarray(t, dtype=np.float64)
    V = np.empty_like(t)
    dV = np.empty_like(t)
    lo, hi = t < x[0], t > x[-1]
    V[lo] = y[0] + s[0] * (t[lo] - x[0])
    dV[lo] = s[0]
    V[hi] = y[-1] + s[-1] * (t[hi] - x[-1])
    dV[hi] = s[-1]
    mid = ~(lo | hi)
    k = np.clip(np.searchsorted(x, t[mid], side="right") - 1, 0, len(x) - 2)
    h = x[k + 1] - x[k]
    u = (t[mid] - x[k]) / h
    h00, h10 = 2 * u ** 3 - 3 * u ** 2 + 1, u ** 3 - 2 * u ** 2 + u
    h01, h11 = -2 * u ** 3 + 3 * u ** 2, u ** 3 - u ** 2
    V[mid] = h00 * y[k] + h10 * h * s[k] + h01 * y[k + 1] + h11 * h * s[k + 1]
    d00, d10 = 6 * u ** 2 - 6 * u, 3 * u ** 2 - 4 * u + 1
    d01, d11 = -6 * u ** 2 + 6 * u, 3 * u ** 2 - 2 * u
    dV[mid] = (d00 * y[k] + d10 * h * s[k] + d01 * y[k + 1] + d11 * h * s[k + 1]) / h
    return V, dV


def second_state(lam, partner, pka, dwp2):
    """Per coordinate: True where the second barrier applies (a tautomer
    coordinate, i.e. no pKa and a partner, whose partner is deprotonated,
    lambda_partner >= 1/2); all False without dwp2."""
    lam = np.asarray(lam, dtype=np.float64)
    if dwp2 is None or partner is None:
        return np.zeros(lam.size, dtype=bool)
    partner = np.asarray(partner)
    taut = (partner >= 0) & np.isnan(np.asarray(pka, dtype=np.float64))
    return taut & (lam[np.maximum(partner, 0)] >= 0.5)


def dw_params(dwp, dwp2, second):
    """C x 4 (B, p0, p1, y1) in force: the second set (B2, p0, p1, y1_2) where
    `second`."""
    d = np.array(dwp, dtype=np.float64)
    if dwp2 is not None:
        d[second, 0] = np.asarray(dwp2)[second, 0]
        d[second, 3] = np.asarray(dwp2)[second, 1]
    return d


def v_dw(dwp, lam):
    """V_dw and dV_dw/dlambda per coordinate; dwp is C x 4 (B, p0, p1, y1)."""
    lam = np.asarray(lam, dtype=np.float64)
    V, dV = np.empty_like(lam), np.empty_like(lam)
    for c in range(lam.size):
        x, y, s = dw_knots(*dwp[c])
        v, d = hermite(x, y, s, lam[c:c + 1])
        past = min(lam[c] - x[0], 0.0) + max(lam[c] - x[-1], 0.0)
        V[c] = v[0] + 0.5 * WALL_K * past * past
        dV[c] = d[0] + WALL_K * past
    return V, dV


def ph_slope(pka, ph_c, T):
    """dV_pH/dlambda = ln(10) k_B T (pKa_ref - pH) (eq 4 with linear V_pH);
    zero where pKa is NaN."""
    pka = np.asarray(pka, dtype=np.float64)
    out = LN10 * KB * T * (pka - ph_c)
    return np.where(np.isnan(pka), 0.0, out)


def mm_slope(mm, lam, partner):
    """dV_MM/dlambda = -G(l_own, l_partner), G = sum_ij g_ij l_own^i l_partner^j."""
    lam = np.asarray(lam, dtype=np.float64)
    y = np.where(partner >= 0, lam[np.maximum(partner, 0)], 0.0)
    G = np.zeros_like(lam)
    for i in range(6):
        for j in range(6):
            G += mm[:, 6 * i + j] * lam ** i * y ** j
    return -G


def lambda_forces(lam, dvdl, partner, pka, ph_c, mm, dwp, T, dwp2=None):
    """Force -dH/dlambda on every coordinate (eq 1 and eq 3) and the per-
    coordinate bias energy V_pH + V_dw; dwp None: no double well; mm None:
    no V_MM; dwp2: second barriers of tautomer coordinates (second_state)."""
    lam = np.asarray(lam, dtype=np.float64)
    if dwp is None:
        Vdw, dVdw = np.zeros_like(lam), np.zeros_like(lam)
    else:
        sec = second_state(lam, partner, pka, dwp2)
        Vdw, dVdw = v_dw(dw_params(dwp, dwp2, sec), lam)
    if mm is None:
        mm = np.zeros((lam.size, 36))
    sph = ph_slope(pka, ph_c, T)
    F = -(dvdl + mm_slope(mm, lam, partner) + sph + dVdw)
    return F, sph * lam + Vdw


def bussi_kinetic(K, nf, kbar, c, R1, chi2):
    """New kinetic energy of the Bussi-Donadio-Parrinello stochastic velocity
    rescaling over one step (their appendix), c = exp(-dt / tau)."""
    return (K + (1.0 - c) * (kbar * (R1 * R1 + chi2) / nf - K)
            + 2.0 * R1 * math.sqrt(K * kbar / nf * (1.0 - c) * c))


def lambda_step(coord_off, lam, v, dvdl, partner, pka, ph, mm, dwp, noise, mass, dt, T, tau,
                first, dwp2=None):
    """One velocity-Verlet step of the lambda particles with the forces at the
    current lambda (from the solve that just ran):
      v_n = v_{n-1/2} + dt/2 F_n / m        (skipped when first: v is v_n)
      v_n *= alpha                           (Bussi, tau > 0, per replica)
      v_{n+1/2} = v_n + dt/2 F_n / m,  lambda_{n+1} = lambda_n + dt v_{n+1/2}.
    Returns (lambda_{n+1}, v_{n+1/2}, K_n before the thermostat per replica,
    bias energy sum of V_pH + V_dw at lambda_n per replica)."""
    lam = np.array(lam, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    R = len(coord_off) - 1
    ph_c = np.empty_like(lam)
    for r in range(R):
        ph_c[coord_off[r]:coord_off[r + 1]] = ph[r]
    F, eb = lambda_forces(lam, dvdl, partner, pka, ph_c, mm, dwp, T, dwp2)
    if not first:
        v = v + 0.5 * dt * F / mass
    kin = np.zeros(R)
    ebias = np.zeros(R)
    for r in range(R):
        a, b = coord_off[r], coord_off[r + 1]
        K = 0.5 * mass * np.sum(v[a:b] ** 2)
        kin[r] = K
        ebias[r] = np.sum(eb[a:b])
        nf = b - a
        if tau > 0 and nf > 0 and K > 0:
            kbar = 0.5 * nf * KB * T
            Kn = bussi_kinetic(K, nf, kbar, math.exp(-dt / tau), noise[r, 0], noise[r, 1])
            v[a:b] *= math.sqrt(max(Kn, 0.0) / K)
    v = v + 0.5 * dt * F / mass
    return lam + dt * v, v, kin, ebias


def accumulate_stats(lam, stats_w, stats_b, near0=0.2, near1=0.8, stats_b2=None, second=None):
    """DBO block statistics of the full-step lambda: stats_w per coordinate
    (steps, steps near 0, sum of lambda near 0, steps near 1, sum near 1),
    stats_b (steps, steps in transition near0 < lambda < near1); with
    stats_b2, the barrier statistics of coordinates in their second state
    (`second`, see second_state) go there instead.  Returns (stats_w,
    stats_b) or, with stats_b2, (stats_w, stats_b, stats_b2)."""
    lam = np.asarray(lam, dtype=np.float64)
    n0, n1 = lam < near0, lam > near1
    stats_w = stats_w + np.stack([np.ones_like(lam), n0, np.where(n0, lam, 0.0), n1,
                                  np.where(n1, lam, 0.0)], axis=1)
    inc = np.stack([np.ones_like(lam), ~n0 & ~n1], axis=1).astype(np.float64)
    if stats_b2 is None:
        return stats_w, stats_b + inc
    sec = np.zeros(lam.size, dtype=bool) if second is None else np.asarray(second)
    return stats_w, stats_b + inc * ~sec[:, None], stats_b2 + inc * sec[:, None]


def pfc_dg(V, T):
    """Free energy of deprotonation -k_B T ln(Z_deprot / Z_prot) of the
    landscape V (a callable of lambda), Z over [0, 1/2] and [1/2, 1]."""
    from scipy.integrate import quad
    beta = 1.0 / (KB * T)
    f = lambda x: math.exp(-beta * V(x))
    zp = quad(f, 0.0, 0.5, epsabs=0.0, epsrel=1e-13, limit=400)[0]
    zd = quad(f, 0.5, 1.0, epsabs=0.0, epsrel=1e-13, limit=400)[0]
    return -KB * T * math.log(zd / zp)


def pfc_landscape(B, p0, p1, y1, slope_ph):
    dwp = np.array([[B, p0, p1, y1]])
    return lambda t: slope_ph * t + v_dw(dwp, np.array([t]))[0][0]


def pfc_target(pka, ph_c, T):
    return 0.0 if math.isnan(pka) else LN10 * KB * T * (pka - ph_c)


def pfc_solve(B, p0, p1, pka, ph_c, T):
    """Height y1 of well 1 for which the landscape V_pH + V_dw has the target
    free energy of deprotonation (partition function correction)."""
    from scipy.optimize import brentq
    slope = 0.0 if math.isnan(pka) else LN10 * KB * T * (pka - ph_c)
    target = pfc_target(pka, ph_c, T)
    g = lambda y1: pfc_dg(pfc_landscape(B, p0, p1, y1, slope), T) - target
    # the free energy grows with y1 but is bounded above (the part of
    # [1/2, 1] left of the barrier top does not move with y1): a target out
    # of reach leaves y1 at the end of the search range nearest to it
    if g(-200.0) >= 0.0:
        return -200.0
    if g(200.0) <= 0.0:
        return 200.0
    return brentq(g, -200.0, 200.0, xtol=1e-13, rtol=1e-15, maxiter=500)


def _barrier_rule(B, sb_c, p):
    """The barrier after one block with statistics sb_c = (steps, steps in
    transition)."""
    frac = sb_c[1] / sb_c[0]
    if frac < p["target"] - p["target_tol"]:
        B -= p["barrier_step"]
    elif frac > p["target"] + p["target_tol"]:
        B += p["barrier_step"]
    return min(max(B, p["barrier_min"]), p["barrier_max"])


def dbo_update(stats_w, stats_b, dwp, mode, pka, ph_c, T, pfc=True, dwp2=None, stats_b2=None,
               partner=None, **kw):
    """Apply the DBO rules at the end of a block: mode bit 0 = well block
    (stats_w), bit 1 = barrier block (stats_b).  Returns (new dwp, adjusted
    flags, cleared stats_w, cleared stats_b); adjusted coordinates get a new
    y1 from the partition function correction when pfc.  With dwp2 (and
    stats_b2, partner), tautomer coordinates also move their second barrier
    from stats_b2 and get a new y1_2; then returns (dwp, adj, sw, sb, dwp2,
    sb2)."""
    p = dict(DBO_DEFAULTS)
    p.update(kw)
    dwp = np.array(dwp, dtype=np.float64)
    sw, sb = np.array(stats_w, dtype=np.float64), np.array(stats_b, dtype=np.float64)
    adj = np.zeros(dwp.shape[0], dtype=np.int32)
    two = dwp2 is not None
    if two:
        dwp2 = np.array(dwp2, dtype=np.float64)
        sb2 = np.array(stats_b2, dtype=np.float64)
        taut = (np.asarray(partner) >= 0) & np.isnan(np.asarray(pka, dtype=np.float64))
    for c in range(dwp.shape[0]):
        if mode & 1 and sw[c, 0] > 0:
            for w, (cnt, tot) in enumerate(((sw[c, 1], sw[c, 2]), (sw[c, 3], sw[c, 4]))):
                if cnt > p["occupancy"] * sw[c, 0]:
                    dev = tot / cnt - float(w)
                    if abs(dev) > p["well_tol"]:
                        pos = dwp[c, 1 + w] - p["well_gain"] * dev
                        lo, hi = w - p["max_shift"], w + p["max_shift"]
                        new = min(max(pos, lo), hi)
                        if new != dwp[c, 1 + w]:
                            dwp[c, 1 + w] = new
                            adj[c] = 1
        if mode & 2 and sb[c, 0] > 0:
            B = _barrier_rule(dwp[c, 0], sb[c], p)
            if B != dwp[c, 0]:
                dwp[c, 0] = B
                adj[c] = 1
        if two and taut[c] and mode & 2 and sb2[c, 0] > 0:
            B2 = _barrier_rule(dwp2[c, 0], sb2[c], p)
            if B2 != dwp2[c, 0]:
                dwp2[c, 0] = B2
                adj[c] = 1
        if adj[c] and pfc:
            dwp[c, 3] = pfc_solve(dwp[c, 0], dwp[c, 1], dwp[c, 2], pka[c], ph_c[c], T)
            if two and taut[c]:
                dwp2[c, 1] = pfc_solve(dwp2[c, 0], dwp[c, 1], dwp[c, 2], pka[c], ph_c[c], T)
    if mode & 1:
        sw[:] = 0.0
    if mode & 2:
        sb[:] = 0.0
        if two:
            sb2[:] = 0.0
    if two:
        return dwp, adj, sw, sb, dwp2, sb2
    return dwp, adj, sw, sb
