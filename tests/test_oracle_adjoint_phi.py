"""Pin of the oracle's gradient of L = gE E + sum gphi phi (upstream weights
on the energy and on the potential) by central differences of L from the
oracle's own solve, open and periodic."""
import numpy as np
import pytest

import oracle
from paper_2410_01626_amd import workloads as W


@pytest.mark.parametrize("periodic", [False, True])
def test_potential_weight_gradient_matches_finite_differences(periodic):
    d = W.tiny_periodic(12, n=40, edge=1.2, n_sites=3, depth=1) if periodic else \
        W.random_open(12, n=40, edge=1.2, n_sites=3, depth=1)
    x, qA, qB, site, lam = (np.array(d[k], dtype=np.float64) for k in ("x", "qA", "qB", "site", "lam"))
    site = site.astype(np.int32)
    rng = np.random.default_rng(4)
    gphi = rng.normal(0, 1, x.shape[0])
    gE, k_e = 0.7, 1.3
    kw = dict(box=d["box"], periodic=periodic, k_e=k_e)

    def L(x_, qA_, qB_, lam_):
        r = oracle.solve(x_, qA_, qB_, site, lam_, **kw)
        return gE * r["E"] + np.dot(gphi, r["phi"])

    gx, gqA, gqB, glam = oracle.adjoint_phi(x, qA, qB, site, lam, gE, gphi, **kw)
    h = 1e-5
    for i, a in ((0, 0), (7, 1), (23, 2), (39, 0)):
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        assert gx[i, a] == pytest.approx((L(xp, qA, qB, lam) - L(xm, qA, qB, lam)) / (2 * h),
                                         rel=1e-6, abs=1e-7)
    for i in (0, 5, site.tolist().index(1)):
        for g, which in ((gqA, 0), (gqB, 1)):
            a_, b_ = qA.copy(), qB.copy()
            (a_ if which == 0 else b_)[i] += h
            ap, bp = a_, b_
            a_, b_ = qA.copy(), qB.copy()
            (a_ if which == 0 else b_)[i] -= h
            fd = (L(x, ap, bp, lam) - L(x, a_, b_, lam)) / (2 * h)
            assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    for s in range(lam.size):
        lp, lm = lam.copy(), lam.copy()
        lp[s] += h
        lm[s] -= h
        assert glam[s] == pytest.approx((L(x, qA, qB, lp) - L(x, qA, qB, lm)) / (2 * h), rel=1e-6, abs=1e-8)
