"""Pins of the four-form (tautomer) oracle (Methods, eq 2, charge-interpolated):
each check is fixed by the mathematics, not by retyping the oracle's formula.

* corners: at (lambda_p, lambda_t) in {0, 1}^2 every site carries exactly one
  form, so the solve equals a plain single-form solve with those charges (pins
  which form sits at which corner);
* no tautomers (B = A, D = C): the four-form solve is the two-form solve of
  eq 1 with forms (A, C) and lambda_p, and dV/dlambda_t vanishes;
* derivatives: E is quadratic in each coordinate separately, so a central
  difference with any step equals dV/dlambda_p and dV/dlambda_t to rounding;
* relabelling symmetry: swapping A <-> B and C <-> D while lambda_t -> 1 -
  lambda_t leaves E and dV/dlambda_p unchanged and flips dV/dlambda_t.
"""
import numpy as np
import pytest

import oracle
from paper_2410_01626_amd import workloads as W


def _open():
    return W.with_tautomers(W.random_open(31, n=160, edge=1.5, n_sites=4, depth=1, order=4))


def _periodic():
    return W.with_tautomers(W.tiny_periodic(32, n=96, edge=1.3, n_sites=3, depth=1, order=4))


CASES = {"open": _open, "periodic": _periodic}
EWALD = 1e-12


def _solve4(d, lp=None, lt=None, **kw):
    lp = d["lam_p"] if lp is None else lp
    lt = d["lam_t"] if lt is None else lt
    return oracle.solve_tautomer(d["x"], kw.get("qA", d["qA"]), kw.get("qB", d["qB"]),
                                 kw.get("qC", d["qC"]), kw.get("qD", d["qD"]), d["site"], lp, lt,
                                 box=d["box"], periodic=d["periodic"], eps=EWALD)


def _solve2(d, qA, qB, lam):
    return oracle.solve(d["x"], qA, qB, d["site"], lam, box=d["box"], periodic=d["periodic"],
                        eps=EWALD)


@pytest.mark.parametrize("case", sorted(CASES))
def test_workload_has_real_tautomers(case):
    d = CASES[case]()
    assert np.any(d["qB"] != d["qA"]) and np.any(d["qD"] != d["qC"])
    # tautomers move charge inside a site: per-site sums of B - A vanish
    for s in range(d["lam_p"].size):
        m = d["site"] == s
        assert abs(float(np.sum(d["qB"][m].astype(np.float64) - d["qA"][m]))) < 1e-6


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("corner", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_corners_are_single_forms(case, corner):
    d = CASES[case]()
    S = d["lam_p"].size
    lp, lt = np.full(S, float(corner[0])), np.full(S, float(corner[1]))
    form = {(0, 0): "qA", (0, 1): "qB", (1, 0): "qC", (1, 1): "qD"}[corner]
    q = d[form].astype(np.float64).copy()
    q[d["site"] < 0] = d["qA"][d["site"] < 0]
    r4 = _solve4(d, lp, lt)
    r1 = _solve2(d, q, q, np.zeros(S))
    np.testing.assert_array_equal(r4["q"], q)
    assert r4["E"] == pytest.approx(r1["E"], rel=1e-13, abs=1e-13)
    np.testing.assert_allclose(r4["F"], r1["F"], rtol=0, atol=1e-12 * np.abs(r1["F"]).max())


@pytest.mark.parametrize("case", sorted(CASES))
def test_no_tautomers_reduces_to_two_forms(case):
    d = CASES[case]()
    r4 = _solve4(d, qB=d["qA"], qD=d["qC"])
    r2 = _solve2(d, d["qA"], d["qC"], d["lam_p"])
    assert r4["E"] == pytest.approx(r2["E"], rel=1e-12)
    np.testing.assert_allclose(r4["F"], r2["F"], rtol=0, atol=1e-11 * np.abs(r2["F"]).max())
    np.testing.assert_allclose(r4["dVdl_p"], r2["dVdl"], rtol=1e-11, atol=1e-12)
    assert np.all(r4["dVdl_t"] == 0.0)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("which", ["p", "t"])
def test_site_derivatives_are_energy_differences(case, which):
    d = CASES[case]()
    base = _solve4(d)
    h = 0.25  # any step: E is quadratic in each coordinate
    key = "lam_" + which
    for s in range(d[key].size):
        lp_, lm_ = d[key].copy(), d[key].copy()
        lp_[s] += h
        lm_[s] -= h
        kw_p = {"lp": lp_} if which == "p" else {"lt": lp_}
        kw_m = {"lp": lm_} if which == "p" else {"lt": lm_}
        fd = (_solve4(d, **kw_p)["E"] - _solve4(d, **kw_m)["E"]) / (2 * h)
        got = base["dVdl_" + which][s]
        assert fd == pytest.approx(got, rel=1e-9, abs=1e-10 * max(1.0, abs(base["E"]))), (s, fd, got)


@pytest.mark.parametrize("case", sorted(CASES))
def test_relabelling_tautomers(case):
    d = CASES[case]()
    a = _solve4(d)
    b = _solve4(d, lt=1.0 - d["lam_t"], qA=d["qB"], qB=d["qA"], qC=d["qD"], qD=d["qC"])
    assert b["E"] == pytest.approx(a["E"], rel=1e-12)
    np.testing.assert_allclose(b["dVdl_p"], a["dVdl_p"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(b["dVdl_t"], -a["dVdl_t"], rtol=1e-10, atol=1e-12)
