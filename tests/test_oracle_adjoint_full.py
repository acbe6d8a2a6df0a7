"""Pins of the oracle's gradient of L = gE E + sum gphi phi + sum gF . F
(upstream weights on the energy, the potentials and the forces): central
differences of L from the oracle's own solve, open and periodic; the
two-charge closed form; beta-independence and translation invariance of the
periodic pair sums."""
import math

import numpy as np
import pytest

import oracle
from paper_2410_01626_amd import workloads as W


def _system(periodic, seed=12, n=40):
    d = W.tiny_periodic(seed, n=n, edge=1.2, n_sites=3, depth=1) if periodic else \
        W.random_open(seed, n=n, edge=1.2, n_sites=3, depth=1)
    x, qA, qB, lam = (np.array(d[k], dtype=np.float64) for k in ("x", "qA", "qB", "lam"))
    return d, x, qA, qB, d["site"].astype(np.int32), lam


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("with_phi", [False, True])
def test_force_weight_gradient_matches_finite_differences(periodic, with_phi):
    d, x, qA, qB, site, lam = _system(periodic)
    rng = np.random.default_rng(5)
    n = x.shape[0]
    gF = rng.normal(0, 1, (n, 3))
    gphi = rng.normal(0, 1, n) if with_phi else None
    gE, k_e = 0.7, 1.3
    kw = dict(box=d["box"], periodic=periodic, k_e=k_e)

    def L(x_, qA_, qB_, lam_):
        r = oracle.solve(x_, qA_, qB_, site, lam_, **kw)
        v = gE * r["E"] + np.sum(gF * r["F"])
        if gphi is not None:
            v += np.dot(gphi, r["phi"])
        return v

    gx, gqA, gqB, glam = oracle.adjoint_full(x, qA, qB, site, lam, gE, gphi, gF, **kw)
    h = 1e-5
    scale = np.abs(gx).max()
    for i, a in ((0, 0), (7, 1), (23, 2), (39, 0), (12, 1)):
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        fd = (L(xp, qA, qB, lam) - L(xm, qA, qB, lam)) / (2 * h)
        assert gx[i, a] == pytest.approx(fd, rel=1e-6, abs=1e-7 * scale), (i, a)
    # L is quadratic in the charges and in lambda: central differences are exact
    for i in (0, 5, site.tolist().index(1), site.tolist().index(2)):
        for g, which in ((gqA, 0), (gqB, 1)):
            a_, b_ = qA.copy(), qB.copy()
            (a_ if which == 0 else b_)[i] += h
            ap, bp = a_, b_
            a_, b_ = qA.copy(), qB.copy()
            (a_ if which == 0 else b_)[i] -= h
            fd = (L(x, ap, bp, lam) - L(x, a_, b_, lam)) / (2 * h)
            assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-8), (which, i)
    for s in range(lam.size):
        lp, lm = lam.copy(), lam.copy()
        lp[s] += h
        lm[s] -= h
        fd = (L(x, qA, qB, lp) - L(x, qA, qB, lm)) / (2 * h)
        assert glam[s] == pytest.approx(fd, rel=1e-6, abs=1e-8), s


def test_two_charges_closed_form():
    """L = w1 . F1 + w2 . F2 with F1 = -F2 = k q1 q2 r / |r|^3, r = r1 - r2:
    L = k q1 q2 (w1 - w2) . r / |r|^3, so
    dL/dr1 = -dL/dr2 = k q1 q2 [(w1 - w2) / |r|^3 - 3 ((w1 - w2) . r) r / |r|^5],
    dL/dq1 = k q2 (w1 - w2) . r / |r|^3 and dL/dq2 = k q1 (w1 - w2) . r / |r|^3."""
    x = np.array([[0.1, -0.2, 0.35], [0.6, 0.15, -0.1]])
    q = np.array([0.8, -1.3])
    w = np.array([[0.3, -1.1, 0.5], [-0.7, 0.2, 0.9]])
    k = 2.5
    site = np.array([-1, -1], dtype=np.int32)
    gx, gqA, gqB, _ = oracle.adjoint_full(x, q, q, site, np.zeros(0), 0.0, None, w, k_e=k)
    r = x[0] - x[1]
    dw = w[0] - w[1]
    rn = math.sqrt(r @ r)
    g1 = k * q[0] * q[1] * (dw / rn ** 3 - 3 * (dw @ r) * r / rn ** 5)
    np.testing.assert_allclose(gx[0], g1, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(gx[1], -g1, rtol=1e-13, atol=1e-14)
    s = (dw @ r) / rn ** 3
    np.testing.assert_allclose(gqA, [k * q[1] * s, k * q[0] * s], rtol=1e-13)
    assert np.all(gqB == 0)


def test_periodic_pair_sums_independent_of_beta_and_translation():
    """The Ewald splitting parameter and a rigid shift of every atom change
    nothing (the real- and reciprocal-space parts trade off exactly)."""
    d, x, qA, qB, site, lam = _system(True, seed=13, n=30)
    q = oracle.lambda_charges(qA, qB, site, lam)
    w = np.random.default_rng(8).normal(0, 1, x.shape)
    box = d["box"]
    L = float(box[0])
    a = oracle.force_weight_sums(x, q, w, box, True, beta=2.2 / (0.5 * L) * 2.8, rcut=0.5 * L,
                                 eps=1e-14)
    b = oracle.force_weight_sums(x, q, w, box, True, rcut=0.45 * L, eps=1e-14)
    c = oracle.force_weight_sums(x + np.array([0.31, -0.57, 0.12]), q, w, box, True, eps=1e-14)
    for u, v in ((a, b), (a, c)):
        np.testing.assert_allclose(u[0], v[0], rtol=1e-9, atol=1e-9 * np.abs(a[0]).max())
        np.testing.assert_allclose(u[1], v[1], rtol=1e-9, atol=1e-9 * np.abs(a[1]).max())


def test_force_weights_in_a_large_cell_approach_the_direct_sum():
    """A cluster in the middle of a large periodic cell: the periodic pair
    sums tend to the open ones as the images move away (the difference from
    the image field falls off with the cell edge)."""
    d, x, qA, qB, site, lam = _system(False, seed=14, n=25)
    q = oracle.lambda_charges(qA, qB, site, lam)
    q = q - q.mean()  # neutral, so the images contribute from the dipole order on
    w = np.random.default_rng(9).normal(0, 1, x.shape)
    h0, e0 = oracle.force_weight_sums(x, q, w)
    errs = []
    for L in (12.0, 24.0):
        xs = x + L / 2 - 0.6
        h, e = oracle.force_weight_sums(xs, q, w, [L] * 3, True, eps=1e-12)
        errs.append(np.abs(h - h0).max() / np.abs(h0).max())
    assert errs[1] < errs[0] < 2e-3, errs


@pytest.mark.parametrize("periodic", [False, True])
def test_targets_subset_equals_full_gradient(periodic):
    """The per-target form (the sums still over every atom) returns the rows
    of the full gradient, and glam once every site atom is a target."""
    d, x, qA, qB, site, lam = _system(periodic, seed=15, n=28)
    rng = np.random.default_rng(10)
    gphi = rng.normal(0, 1, x.shape[0])
    gF = rng.normal(0, 1, x.shape)
    kw = dict(box=d["box"], periodic=True) if periodic else {}
    full = oracle.adjoint_full(x, qA, qB, site, lam, 0.4, gphi, gF, **kw)
    t = np.union1d(rng.choice(x.shape[0], 7, replace=False), np.flatnonzero(site >= 0))
    part = oracle.adjoint_full(x, qA, qB, site, lam, 0.4, gphi, gF, targets=t, **kw)
    for a, b in zip(full[:3], part[:3]):
        np.testing.assert_allclose(b, a[t], rtol=1e-12, atol=1e-12 * np.abs(a).max())
    np.testing.assert_allclose(part[3], full[3], rtol=1e-12, atol=1e-12)
    t2 = np.setdiff1d(t, np.flatnonzero(site >= 0)[:1])
    assert oracle.adjoint_full(x, qA, qB, site, lam, 0.4, gphi, gF, targets=t2, **kw)[3] is None
