"""Adjoint with upstream weights on the energy and on the potential
(fmm_eval_adjoint_phi) against the oracle's analytic gradient."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL_F
from paper_2410_01626_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2))


def _run(d, prec, gE, gphi, **kw):
    import torch
    from paper_2410_01626_amd import fmm
    n, S = d["x"].shape[0], d["lam"].size
    plan = fmm.Plan(d["depth"], d["order"], periodic=d["periodic"], precision=prec, max_atoms=n,
                    max_sites=S, device="cuda:0", **kw)
    dt = plan.dtype
    t = [torch.tensor(d[k], dtype=dt, device="cuda:0") for k in ("x", "qA", "qB")]
    site = torch.tensor(d["site"], dtype=torch.int32, device="cuda:0")
    lam = torch.tensor(d["lam"], dtype=torch.float64, device="cuda:0")
    g = torch.tensor(gphi, dtype=dt, device="cuda:0")
    out = plan.eval_adjoint_phi(*t, site, lam, gE, g, box=d["box"] if d["periodic"] else None)
    torch.cuda.synchronize()
    res = {k: v.double().cpu().numpy() for k, v in out.items()}
    plan.close()
    return res


@pytest.mark.parametrize("prec", ["fp64", "f32"])
def test_periodic_potential_weights_match_oracle(prec):
    d = W.tiny_periodic(71, n=2500, edge=2.2, n_sites=4, depth=3, order=6)
    gphi = np.random.default_rng(5).normal(0, 1, d["x"].shape[0])
    gE = 0.6
    got = _run(d, prec, gE, gphi)
    gx, gqA, gqB, glam = oracle.adjoint_phi(d["x"], d["qA"], d["qB"], d["site"], d["lam"], gE, gphi,
                                            box=d["box"], periodic=True)
    tol = 3 * TOL_F[6] * (1 if prec == "fp64" else 2)
    assert _rel(got["grad_x"], gx) <= tol
    assert _rel(got["grad_qA"], gqA) <= tol
    assert _rel(got["grad_qB"], gqB) <= tol
    assert np.abs(got["grad_lambda"] - glam).max() <= tol * np.sqrt(np.mean(glam ** 2))


def test_open_potential_weights_exact_without_far_field():
    d = W.random_open(72, n=500, edge=1.4, n_sites=3, depth=1, order=4)
    gphi = np.random.default_rng(6).normal(0, 1, d["x"].shape[0])
    got = _run(d, "fp64", -1.3, gphi)
    gx, gqA, gqB, glam = oracle.adjoint_phi(d["x"], d["qA"], d["qB"], d["site"], d["lam"], -1.3, gphi)
    assert _rel(got["grad_x"], gx) <= 1e-10
    assert _rel(got["grad_qA"], gqA) <= 1e-11 and _rel(got["grad_qB"], gqB) <= 1e-11
    assert np.allclose(got["grad_lambda"], glam, rtol=1e-9, atol=1e-9 * np.abs(glam).max())
    # the forward outputs are those of the plain solve
    ref = oracle.solve(d["x"], d["qA"], d["qB"], d["site"], d["lam"])
    assert got["E"][0] == pytest.approx(ref["E"], rel=1e-11)


def test_potential_weights_rejected_on_hamiltonian_plans():
    from paper_2410_01626_amd import fmm
    d = W.random_open(73, n=100, edge=1.0, n_sites=2, depth=1, order=4)
    with pytest.raises(fmm.FmmError) as e:
        _run(d, "f32", 1.0, np.ones(100), hamiltonian=True)
    assert e.value.status == fmm.FMM_E_UNSUPPORTED


def test_graph_replay_of_the_three_solves():
    # a graph plan captures the three solves and the combine kernel once and
    # replays them; every replay equals the eager plan bitwise
    import torch
    from paper_2410_01626_amd import fmm
    d = W.tiny_periodic(74, n=1800, edge=2.0, n_sites=3, depth=3, order=6)
    n, S = d["x"].shape[0], d["lam"].size
    stream = torch.cuda.Stream("cuda:0")
    kw = dict(periodic=True, precision="f32", max_atoms=n, max_sites=S, device="cuda:0")
    eager = fmm.Plan(3, 6, **kw)
    gplan = fmm.Plan(3, 6, stream=stream, graph=True, **kw)
    t = [torch.tensor(d[k], dtype=torch.float32, device="cuda:0") for k in ("x", "qA", "qB")]
    site = torch.tensor(d["site"], dtype=torch.int32, device="cuda:0")
    lam = torch.tensor(d["lam"], dtype=torch.float64, device="cuda:0")
    g = torch.tensor(np.random.default_rng(8).normal(0, 1, n), dtype=torch.float32, device="cuda:0")
    ref = eager.eval_adjoint_phi(*t, site, lam, 0.5, g, box=d["box"])
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(stream):
            got = gplan.eval_adjoint_phi(*t, site, lam, 0.5, g, box=d["box"])
        stream.synchronize()
        junk = torch.randn(1000, device="cuda:0").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert junk.isfinite()
        for k in ("grad_x", "grad_qA", "grad_qB", "grad_lambda", "E", "F", "phi"):
            assert torch.equal(got[k], ref[k]), k
    eager.close()
    gplan.close()
