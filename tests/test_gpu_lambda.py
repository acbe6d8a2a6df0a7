"""Lambda-dynamics kernels (step, DBO, partition function correction) through
the C ABI against the FP64 oracle on the same seeded inputs, and the driver
around a Coulomb solve."""
import math

import numpy as np
import pytest

from oracle import lambda_dynamics as L

pytestmark = pytest.mark.gpu

REL = 1e-12


def _case(seed, sizes, with_partner=True):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    C, R = int(off[-1]), len(sizes)
    lam = rng.uniform(-0.2, 1.2, C)
    v = rng.normal(0, 2.0, C)
    dvdl = rng.normal(0, 40.0, C)
    partner = np.full(C, -1, dtype=np.int32)
    if with_partner:
        for r in range(R):  # pair neighbouring coordinates of a replica
            for c in range(off[r], off[r + 1] - 1, 3):
                partner[c], partner[c + 1] = c + 1, c
    pka = rng.uniform(3.0, 10.0, C)
    pka[rng.uniform(size=C) < 0.3] = np.nan
    ph = rng.uniform(2.0, 9.0, R)
    mm = rng.normal(0, 5.0, (C, 36)) / (1 + np.arange(36) % 6)[None, :]
    dwp = np.stack([rng.uniform(2, 12, C), rng.uniform(-0.06, 0.06, C),
                    rng.uniform(0.94, 1.06, C), rng.uniform(-3, 3, C)], axis=1)
    noise = np.stack([rng.normal(size=R), rng.chisquare(np.maximum(np.array(sizes) - 1, 1))], axis=1)
    return dict(off=off, lam=lam, v=v, dvdl=dvdl, partner=partner, pka=pka, ph=ph, mm=mm,
                dwp=dwp, noise=noise)


def _t(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a)
    dt = dtype or (torch.int32 if a.dtype.kind == "i" else torch.float64)
    return torch.tensor(a, dtype=dt, device="cuda:0")


def _close(got, ref, rel=REL):
    got, ref = np.asarray(got), np.asarray(ref)
    scale = max(1.0, np.abs(ref).max()) if ref.size else 1.0
    assert np.abs(got - ref).max() <= rel * scale if ref.size else True


@pytest.mark.parametrize("first", [False, True])
@pytest.mark.parametrize("tau", [0.5, 0.0])
def test_step_matches_oracle(first, tau):
    import torch
    from paper_2410_01626_amd import lambda_dynamics as LD
    d = _case(7, [5, 0, 600, 33])
    C, R = d["lam"].size, d["ph"].size
    m, dt, T = 60.0, 0.002, 300.0
    lam, lam_new, v = _t(d["lam"]), torch.empty(C, dtype=torch.float64, device="cuda:0"), _t(d["v"])
    sw = torch.zeros(5 * C, dtype=torch.float64, device="cuda:0")
    sb = torch.zeros(2 * C, dtype=torch.float64, device="cuda:0")
    kin = torch.zeros(R, dtype=torch.float64, device="cuda:0")
    eb = torch.zeros(R, dtype=torch.float64, device="cuda:0")
    prm = LD.LambdaParams(m, dt, T, tau, 0.2, 0.8)
    LD.lambda_step(_t(d["off"], torch.int32), lam, lam_new, v, _t(d["dvdl"]), _t(d["ph"]), prm,
                   first=first, partner=_t(d["partner"]), pka=_t(d["pka"]), mm=_t(d["mm"].ravel()),
                   dwp=_t(d["dwp"].ravel()), noise=_t(d["noise"].ravel()), stats_w=sw, stats_b=sb,
                   kin=kin, e_bias=eb)
    torch.cuda.synchronize()
    rl, rv, rk, re = L.lambda_step(d["off"], d["lam"], d["v"], d["dvdl"], d["partner"], d["pka"],
                                   d["ph"], d["mm"], d["dwp"], d["noise"], m, dt, T, tau, first)
    rsw, rsb = L.accumulate_stats(d["lam"], np.zeros((C, 5)), np.zeros((C, 2)))
    _close(lam_new.cpu().numpy(), rl)
    _close(v.cpu().numpy(), rv)
    _close(kin.cpu().numpy(), rk)
    _close(eb.cpu().numpy(), re)
    assert np.array_equal(sw.cpu().numpy().reshape(C, 5), rsw)
    assert np.array_equal(sb.cpu().numpy().reshape(C, 2), rsb)
    assert np.array_equal(lam.cpu().numpy(), d["lam"])  # the input is untouched


def test_step_with_tautomer_second_barriers():
    """Tautomer coordinates (no pKa, a partner) switch to their second barrier
    set while the partner is deprotonated, and their barrier statistics go to
    stats_b2 in that state; both match the oracle."""
    import torch
    from paper_2410_01626_amd import lambda_dynamics as LD
    d = _case(9, [40, 90])
    C, R = d["lam"].size, d["ph"].size
    rng = np.random.default_rng(4)
    dwp2 = np.stack([rng.uniform(1, 12, C), rng.uniform(-3, 3, C)], axis=1)
    sec = L.second_state(d["lam"], d["partner"], d["pka"], dwp2)
    assert sec.sum() >= 5 and (~sec & np.isnan(d["pka"]) & (d["partner"] >= 0)).sum() >= 5
    m, dt, T, tau = 60.0, 0.002, 300.0, 0.5
    lam, lam_new, v = _t(d["lam"]), torch.empty(C, dtype=torch.float64, device="cuda:0"), _t(d["v"])
    z = lambda k: torch.zeros(k, dtype=torch.float64, device="cuda:0")
    sw, sb, sb2, kin, eb = z(5 * C), z(2 * C), z(2 * C), z(R), z(R)
    prm = LD.LambdaParams(m, dt, T, tau, 0.2, 0.8)
    LD.lambda_step(_t(d["off"], torch.int32), lam, lam_new, v, _t(d["dvdl"]), _t(d["ph"]), prm,
                   partner=_t(d["partner"]), pka=_t(d["pka"]), mm=_t(d["mm"].ravel()),
                   dwp=_t(d["dwp"].ravel()), noise=_t(d["noise"].ravel()), stats_w=sw, stats_b=sb,
                   kin=kin, e_bias=eb, dwp2=_t(dwp2.ravel()), stats_b2=sb2)
    torch.cuda.synchronize()
    rl, rv, rk, re = L.lambda_step(d["off"], d["lam"], d["v"], d["dvdl"], d["partner"], d["pka"],
                                   d["ph"], d["mm"], d["dwp"], d["noise"], m, dt, T, tau, False,
                                   dwp2=dwp2)
    rsw, rsb, rsb2 = L.accumulate_stats(d["lam"], np.zeros((C, 5)), np.zeros((C, 2)),
                                        stats_b2=np.zeros((C, 2)), second=sec)
    _close(lam_new.cpu().numpy(), rl)
    _close(v.cpu().numpy(), rv)
    _close(eb.cpu().numpy(), re)
    assert np.array_equal(sb.cpu().numpy().reshape(C, 2), rsb)
    assert np.array_equal(sb2.cpu().numpy().reshape(C, 2), rsb2)
    # the second barrier matters: the one-barrier step differs
    rl1, _, _, _ = L.lambda_step(d["off"], d["lam"], d["v"], d["dvdl"], d["partner"], d["pka"],
                                 d["ph"], d["mm"], d["dwp"], d["noise"], m, dt, T, tau, False)
    assert np.abs(rl1 - rl).max() > 1e-9
    # DBO of both barriers and the correction of both states
    nst = np.zeros((C, 2))
    nst[:, 0] = 100.0
    nst[:, 1] = rng.integers(0, 60, C)
    nst2 = nst.copy()
    nst2[:, 1] = rng.integers(0, 60, C)
    swn = np.zeros((C, 5))
    g_dwp, g_dwp2, g_sb, g_sb2 = _t(d["dwp"].ravel()), _t(dwp2.ravel()), _t(nst.ravel()), _t(nst2.ravel())
    adj = torch.zeros(C, dtype=torch.int32, device="cuda:0")
    LD.lambda_dbo(_t(d["off"], torch.int32), g_dwp, _t(d["ph"]), T, mode=2, pfc=True,
                  pka=_t(d["pka"]), stats_w=_t(swn.ravel()), stats_b=g_sb, adjusted=adj,
                  partner=_t(d["partner"]), dwp2=g_dwp2, stats_b2=g_sb2)
    torch.cuda.synchronize()
    ph_c = np.repeat(d["ph"], np.diff(d["off"]))
    rd, radj, _, _, rd2, _ = L.dbo_update(swn, nst, d["dwp"], 2, d["pka"], ph_c, T, pfc=True,
                                          dwp2=dwp2, stats_b2=nst2, partner=d["partner"])
    assert np.array_equal(adj.cpu().numpy(), radj)
    got, got2 = g_dwp.cpu().numpy().reshape(C, 4), g_dwp2.cpu().numpy().reshape(C, 2)
    taut = np.isnan(d["pka"]) & (d["partner"] >= 0)
    assert np.array_equal(got[:, 0], rd[:, 0]) and np.array_equal(got2[taut, 0], rd2[taut, 0])
    assert np.allclose(got[:, 3], rd[:, 3], atol=1e-8, rtol=0)
    assert np.allclose(got2[taut, 1], rd2[taut, 1], atol=1e-8, rtol=0)
    assert np.array_equal(got2[~taut], dwp2[~taut])  # other coordinates keep dwp2
    assert not g_sb.any() and not g_sb2[torch.tensor(np.repeat(taut, 2), device="cuda:0")].any()


def test_step_without_optional_terms():
    # no partner, pKa, V_MM, double well, statistics or outputs: only the
    # Coulomb derivative moves lambda
    import torch
    from paper_2410_01626_amd import lambda_dynamics as LD
    d = _case(8, [17, 4], with_partner=False)
    C = d["lam"].size
    lam, lam_new, v = _t(d["lam"]), torch.empty(C, dtype=torch.float64, device="cuda:0"), _t(d["v"])
    prm = LD.LambdaParams(60.0, 0.002, 300.0, 0.0, 0.2, 0.8)
    LD.lambda_step(_t(d["off"], torch.int32), lam, lam_new, v, _t(d["dvdl"]), _t(d["ph"]), prm)
    torch.cuda.synchronize()
    rl, rv, _, _ = L.lambda_step(d["off"], d["lam"], d["v"], d["dvdl"], np.full(C, -1),
                                 np.full(C, np.nan), d["ph"], None, None, None, 60.0, 0.002, 300.0,
                                 0.0, False)
    _close(lam_new.cpu().numpy(), rl)
    _close(v.cpu().numpy(), rv)


def test_dbo_and_pfc_match_oracle():
    import torch
    from paper_2410_01626_amd import lambda_dynamics as LD
    rng = np.random.default_rng(21)
    sizes = [9, 70]
    off = np.concatenate([[0], np.cumsum(sizes)])
    C, R = int(off[-1]), len(sizes)
    T = 300.0
    pka = rng.uniform(3.0, 10.0, C)
    pka[::4] = np.nan
    ph = rng.uniform(2.0, 9.0, R)
    ph_c = np.repeat(ph, sizes)
    dwp = np.stack([rng.integers(1, 21, C).astype(float), rng.uniform(-0.08, 0.08, C),
                    rng.uniform(0.92, 1.08, C), np.zeros(C)], axis=1)
    n = rng.integers(50, 200, C).astype(float)
    f0, f1 = rng.uniform(0, 1, C), rng.uniform(0, 1, C)
    n0 = np.floor(n * f0 * 0.95)
    n1 = np.floor((n - n0) * f1)
    sw = np.stack([n, n0, n0 * rng.uniform(-0.1, 0.19, C), n1, n1 * rng.uniform(0.81, 1.1, C)], axis=1)
    sb = np.stack([n, np.floor(n * rng.uniform(0, 0.6, C))], axis=1)
    # partition function correction of every coordinate
    g_dwp = _t(dwp.ravel())
    LD.lambda_pfc(_t(off, torch.int32), g_dwp, _t(ph), T, pka=_t(pka))
    torch.cuda.synchronize()
    got = g_dwp.cpu().numpy().reshape(C, 4)
    for c in range(C):
        y1 = L.pfc_solve(dwp[c, 0], dwp[c, 1], dwp[c, 2], pka[c], ph_c[c], T)
        assert got[c, 3] == pytest.approx(y1, abs=1e-8), c
    assert np.array_equal(got[:, :3], dwp[:, :3])
    dwp[:, 3] = got[:, 3]
    # DBO rules, both blocks at once, then the correction of moved coordinates
    g_dwp, g_sw, g_sb = _t(dwp.ravel()), _t(sw.ravel()), _t(sb.ravel())
    adj = torch.zeros(C, dtype=torch.int32, device="cuda:0")
    LD.lambda_dbo(_t(off, torch.int32), g_dwp, _t(ph), T, mode=3, pfc=True, pka=_t(pka),
                  stats_w=g_sw, stats_b=g_sb, adjusted=adj)
    torch.cuda.synchronize()
    rd, radj, rsw, rsb = L.dbo_update(sw, sb, dwp, 3, pka, ph_c, T, pfc=True)
    got = g_dwp.cpu().numpy().reshape(C, 4)
    assert np.array_equal(adj.cpu().numpy(), radj)
    assert radj.sum() > C // 4  # the case moves a good share of the coordinates
    assert np.array_equal(got[:, 0], rd[:, 0])
    # well moves: the kernel may fuse the multiply-add (one rounding less)
    assert np.allclose(got[:, 1:3], rd[:, 1:3], atol=1e-15, rtol=0)
    assert np.allclose(got[:, 3], rd[:, 3], atol=1e-8, rtol=0)
    assert not g_sw.any() and not g_sb.any()
    # the well rule alone leaves the barrier statistics
    g_sb2 = _t(sb.ravel())
    g_sw2 = _t(sw.ravel())
    LD.lambda_dbo(_t(off, torch.int32), _t(dwp.ravel()), _t(ph), T, mode=1, pfc=False,
                  stats_w=g_sw2, stats_b=g_sb2)
    torch.cuda.synchronize()
    assert not g_sw2.any() and np.array_equal(g_sb2.cpu().numpy(), sb.ravel())


def test_pfc_near_the_unreachable_target():
    """Targets just inside and just past the largest free energy a low barrier
    allows (1 kJ/mol, wells at 0 and 1, pH 7): the free energy saturates in y1
    there (slope ~0.006), so the root finder must stop on the bracket, not on
    the residual.  y1 equals the oracle's to 1e-8 and solves the oracle's
    equation; past the edge y1 stays at the bound."""
    import torch
    from paper_2410_01626_amd import lambda_dynamics as LD
    from scipy.optimize import brentq
    T, ph = 300.0, 7.0

    def g(pk, y1):
        slope = L.LN10 * L.KB * T * (pk - ph)
        return L.pfc_dg(L.pfc_landscape(1.0, 0.0, 1.0, y1, slope), T) - L.pfc_target(pk, ph, T)

    edge = brentq(lambda pk: g(pk, 200.0), 8.0, 10.0, xtol=1e-12)
    pka = edge + np.array([-0.5, -0.1, -0.02, -0.005, -0.001, 0.01, 0.2])
    C = pka.size
    dwp = np.stack([np.ones(C), np.zeros(C), np.ones(C), np.zeros(C)], axis=1)
    g_dwp = _t(dwp.ravel())
    LD.lambda_pfc(_t(np.array([0, C]), torch.int32), g_dwp, _t(np.array([ph])), T, pka=_t(pka))
    torch.cuda.synchronize()
    got = g_dwp.cpu().numpy().reshape(C, 4)[:, 3]
    for c in range(C):
        y1 = L.pfc_solve(1.0, 0.0, 1.0, pka[c], ph, T)
        assert got[c] == pytest.approx(y1, abs=1e-8), (c, got[c], y1)
        if pka[c] < edge:
            assert abs(g(pka[c], got[c])) < 1e-10, c
        else:
            assert got[c] == 200.0


def test_thermostat_samples_the_canonical_kinetic_energy():
    # free lambda particles under the Bussi thermostat: <K> = N_f k_B T / 2
    import torch
    from paper_2410_01626_amd import lambda_dynamics as LD
    C = 400
    dyn = LD.LambdaDynamics([0, C], np.full(C, 0.5), [7.0], np.full(C, np.nan), tau=0.05,
                            barrier=6.0, seed=3, well_block=10 ** 9, barrier_block=10 ** 9)
    dyn.dwp = None  # no double well: free particles
    zero = torch.zeros(C, dtype=torch.float64, device="cuda:0")
    ks = []
    for i in range(600):
        dyn.step(zero)
        if i >= 100:
            ks.append(dyn.kin[0].item())
    kbar = 0.5 * C * L.KB * 300.0
    # K is Gamma(C/2, kT): relative sd sqrt(2/C) = 7% per sample, ~0.5% over
    # 500 correlated samples (tau = 25 steps)
    assert abs(np.mean(ks) / kbar - 1) < 0.03
    assert np.isfinite(dyn.lam.cpu().numpy()).all()


def test_driver_around_the_solve():
    # lambda moves under the Coulomb derivative of the solve plus the bias:
    # one driver step equals the oracle step with the same noise
    import torch
    from paper_2410_01626_amd import fmm
    from paper_2410_01626_amd import lambda_dynamics as LD
    from paper_2410_01626_amd import workloads as W
    d = W.tiny_periodic(41, n=1500, edge=2.0, n_sites=6, depth=2, order=6)
    S = d["lam"].size
    plan = fmm.Plan(2, 6, periodic=True, precision="f32", coulomb_k=138.935458, max_atoms=1500,
                    max_sites=S, device="cuda:0")
    dt = torch.float32
    x, qA, qB = (torch.tensor(d[k], dtype=dt, device="cuda:0") for k in ("x", "qA", "qB"))
    site = torch.tensor(d["site"], dtype=torch.int32, device="cuda:0")
    pka = np.linspace(4.0, 7.0, S)
    dyn = LD.LambdaDynamics([0, S], d["lam"], [5.5], pka, tau=0.5, seed=5)
    for it in range(3):
        lam = dyn.lam.clone()
        v = dyn.v.clone()
        dwp = dyn.dwp.clone()
        out = plan.eval(x, qA, qB, site, lam, box=d["box"])
        dyn.step(out["dVdl"])
        torch.cuda.synchronize()
        noise = dyn.noise.cpu().numpy().reshape(1, 2)  # the step's own row of the bank
        rl, rv, _, _ = L.lambda_step(np.array([0, S]), lam.cpu().numpy(), v.cpu().numpy(),
                                     out["dVdl"].cpu().numpy(), np.full(S, -1), pka, np.array([5.5]),
                                     None, dwp.cpu().numpy().reshape(S, 4), noise, 60.0, 0.002,
                                     300.0, 0.5, it == 0)
        _close(dyn.lam.cpu().numpy(), rl)
        _close(dyn.v.cpu().numpy(), rv)
    plan.close()


def test_mm_calibration_flattens_an_isolated_site():
    # the reference compound of a site is the site alone: its dV/dlambda is
    # linear in lambda, so G from two solves (lambda = 0, 1) cancels the
    # solve's derivative at every lambda (the step then feels no force)
    import torch
    from paper_2410_01626_amd import fmm
    from paper_2410_01626_amd import lambda_dynamics as LD
    rng = np.random.default_rng(17)
    S = 5
    x = np.concatenate([rng.normal(0, 0.15, (4, 3)) + rng.uniform(0, 3, 3) for _ in range(S)])
    qA = rng.uniform(-1, 1, 4 * S)
    qB = qA + rng.uniform(-0.5, 0.5, 4 * S)
    ao, so = np.arange(0, 4 * S + 1, 4), np.arange(S + 1)
    plan = fmm.Plan(1, 8, periodic=False, precision="fp64", coulomb_k=138.935458, max_atoms=4 * S,
                    max_sites=S, max_replicas=S, device="cuda:0")
    t = [_t(a) for a in (x, qA, qB)]
    site = torch.zeros(4 * S, dtype=torch.int32, device="cuda:0")
    dv = lambda lam: plan.eval_batched(ao, so, *t, site, _t(lam))["dVdl"]
    g0, g1 = dv(np.zeros(S)).cpu().numpy(), dv(np.ones(S)).cpu().numpy()
    mm = np.zeros((S, 36))
    mm[:, 0], mm[:, 6] = g0, g1 - g0
    lam = rng.uniform(-0.1, 1.1, S)
    dvdl = dv(lam)
    v = torch.zeros(S, dtype=torch.float64, device="cuda:0")
    lam_new = torch.empty(S, dtype=torch.float64, device="cuda:0")
    prm = LD.LambdaParams(60.0, 0.002, 300.0, 0.0, 0.2, 0.8)
    LD.lambda_step(_t(np.array([0, S]), torch.int32), _t(lam), lam_new, v, dvdl,
                   _t(np.array([7.0])), prm, first=True, mm=_t(mm.ravel()))
    torch.cuda.synchronize()
    scale = np.abs(dvdl.cpu().numpy()).max()
    # v = dt/2 F/m: F vanishes up to rounding of the solve
    F = v.cpu().numpy() * 60.0 / 0.001
    assert np.abs(F).max() <= 1e-9 * scale
    plan.close()
