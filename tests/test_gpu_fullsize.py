"""Full-size configurations, checked on outputs the oracle computes atom by
atom: sampled potentials and forces, and every site's dV/dlambda (which needs
the potential only at site atoms)."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL_F
from paper_2410_01626_amd import workloads as W

pytestmark = pytest.mark.gpu


def _oracle_sample(d, targets, periodic):
    q = oracle.lambda_charges(d["qA"], d["qB"], d["site"], d["lam"])
    if periodic:
        phi, field = oracle.ewald(d["x"], q, d["box"], eps=1e-11, targets=targets)
    else:
        phi, field = oracle.direct(d["x"], q, targets=targets)
    return q, phi, q[targets, None] * field


def _site_dvdl(d, phi_sites, site_atoms):
    dv = np.zeros(d["lam"].size)
    np.add.at(dv, d["site"][site_atoms], (d["qB"] - d["qA"])[site_atoms] * phi_sites)
    return dv


def _check(d, phi_gpu, F_gpu, dvdl_gpu, periodic, p, n_sample=600, seed=0):
    rng = np.random.default_rng(seed)
    n = d["x"].shape[0]
    samp = np.sort(rng.choice(n, min(n_sample, n), replace=False))
    site_atoms = np.flatnonzero(d["site"] >= 0)
    targets = np.concatenate([samp, site_atoms])
    q, phi, F = _oracle_sample(d, targets, periodic)
    ns = samp.size
    eF = np.sqrt(np.sum((F_gpu[samp] - F[:ns]) ** 2) / np.sum(F[:ns] ** 2))
    ephi = np.sqrt(np.sum((phi_gpu[samp] - phi[:ns]) ** 2) / np.sum(phi[:ns] ** 2))
    dv = _site_dvdl(d, phi[ns:], site_atoms)
    edv = np.abs(dvdl_gpu - dv).max() / np.sqrt(np.mean(dv ** 2))
    tol = TOL_F[p]
    assert eF <= tol and ephi <= tol and edv <= tol, (eF, ephi, edv)
    return eF, ephi, edv


@pytest.mark.parametrize("prec", ["bf16x3", "f32"])
def test_large_box_sampled(prec):
    """500,000 atoms, periodic 17 nm, depth 5, p = 10; forward and adjoint."""
    import torch
    from paper_2410_01626_amd import fmm
    from paper_2410_01626_amd.autograd import fmm_coulomb
    dev = torch.device("cuda:0")
    d = W.large_box()
    n, S = d["x"].shape[0], d["lam"].size
    plan = fmm.Plan(d["depth"], d["order"], periodic=True, precision=prec, max_atoms=n,
                    max_sites=S, device=dev)
    x = torch.tensor(d["x"], dtype=torch.float32, device=dev, requires_grad=True)
    qA = torch.tensor(d["qA"], dtype=torch.float32, device=dev, requires_grad=True)
    qB = torch.tensor(d["qB"], dtype=torch.float32, device=dev, requires_grad=True)
    site = torch.tensor(d["site"], device=dev)
    lam = torch.tensor(d["lam"], device=dev, requires_grad=True)
    E, F, phi, dVdl = fmm_coulomb(plan, x, qA, qB, site, lam, d["box"])
    gx, gqA, gqB, gl = torch.autograd.grad(E, [x, qA, qB, lam])
    torch.cuda.synchronize()
    Fn, pn, dn = F.detach().double().cpu().numpy(), phi.detach().double().cpu().numpy(), dVdl.cpu().numpy()
    _check(d, pn, Fn, dn, True, d["order"])
    # the adjoint of a unit weight is (-F, (1-l) phi, l phi, dV/dl) of the same solve
    np.testing.assert_array_equal(gx.cpu().numpy(), -F.detach().cpu().numpy())
    np.testing.assert_allclose(gl.cpu().numpy(), dn, rtol=0, atol=0)
    assert np.isfinite(E.item())
    # and the gradients themselves against the oracle's on 600 sampled atoms
    # and every site atom: dE/dx = -F, dE/dqA = (1 - l) phi, dE/dqB = l phi
    rng = np.random.default_rng(11)
    samp = np.union1d(rng.choice(n, 600, replace=False), np.flatnonzero(d["site"] >= 0))
    q, phi_o, F_o = _oracle_sample(d, samp, True)
    lam_s = np.where(d["site"] >= 0, d["lam"][np.maximum(d["site"], 0)], 0.0)[samp]
    tol = TOL_F[d["order"]]
    for got, exp in ((gx.double().cpu().numpy()[samp], -F_o),
                     (gqA.double().cpu().numpy()[samp], (1 - lam_s) * phi_o),
                     (gqB.double().cpu().numpy()[samp], lam_s * phi_o)):
        nz = np.sum(exp ** 2)
        if nz == 0:
            assert np.all(got == 0)
            continue
        err = np.sqrt(np.sum((got - exp) ** 2) / nz)
        assert err <= tol, err


def test_replicas_full_size_sampled():
    """16 open replicas of 10k-60k atoms (~560k atoms) in one batched call."""
    import torch
    from paper_2410_01626_amd import fmm
    dev = torch.device("cuda:0")
    reps = W.replicas()
    ao = np.cumsum([0] + [r["x"].shape[0] for r in reps])
    so = np.cumsum([0] + [r["lam"].size for r in reps])
    cat = {k: np.concatenate([r[k] for r in reps]) for k in ("x", "qA", "qB", "site", "lam")}
    plan = fmm.Plan(3, 8, periodic=False, precision="bf16x3", max_atoms=int(ao[-1]),
                    max_sites=int(so[-1]), max_replicas=len(reps), device=dev)
    t = [torch.tensor(cat[k], dtype=torch.float32, device=dev) for k in ("x", "qA", "qB")]
    out = plan.eval_batched(ao, so, t[0], t[1], t[2], torch.tensor(cat["site"], device=dev),
                            torch.tensor(cat["lam"], device=dev))
    torch.cuda.synchronize()
    F = out["F"].double().cpu().numpy()
    phi = out["phi"].double().cpu().numpy()
    dv = out["dVdl"].cpu().numpy()
    for r in (0, 7, 15):
        d = reps[r]
        _check(d, phi[ao[r]:ao[r + 1]], F[ao[r]:ao[r + 1]], dv[so[r]:so[r + 1]], False, 8,
               n_sample=300, seed=r)
