"""Hamiltonian interpolation (Methods, eq 1; plan parameter hamiltonian = 1):
the HIP path through the C ABI against the FP64 oracle, and the correction
alone against the oracle's correction."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_within, errors, run
from paper_2410_01626_amd import workloads as W

pytestmark = pytest.mark.gpu


def ref_h(d, lam=None):
    lam = d["lam"] if lam is None else lam
    return oracle.solve(d["x"], d["qA"], d["qB"], d["site"], lam, box=d["box"],
                        periodic=d["periodic"], hamiltonian=True)


@pytest.mark.parametrize("prec", ["fp64", "f32", "bf16x3"])
def test_open_cube_hamiltonian(prec):
    d = W.open_cube()
    err = errors(run(d, prec, hamiltonian=True), ref_h(d))
    assert_within(err, d["order"], label="open_cube hamiltonian " + prec)


@pytest.mark.parametrize("depth", [0, 2, 3])
@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_periodic_hamiltonian(depth, prec):
    d = W.tiny_periodic(81, n=400, edge=1.6, n_sites=6, depth=depth, order=8)
    err = errors(run(d, prec, hamiltonian=True), ref_h(d))
    assert_within(err, 8, label="periodic hamiltonian depth %d %s" % (depth, prec))


def test_water_box_hamiltonian_full_size():
    from gpu_util import cached_reference
    d, ref = cached_reference("water_box")
    dE, dF, dD = oracle.hamiltonian_correction(d["x"], d["qA"], d["qB"], d["site"], d["lam"],
                                               d["box"], True)
    refh = dict(ref, E=ref["E"] + dE, F=ref["F"] + dF, dVdl=ref["dVdl"] + dD)
    err = errors(run(d, "bf16x3", hamiltonian=True), refh)
    assert_within(err, 8, label="water_box hamiltonian")


@pytest.mark.parametrize("periodic", [False, True])
def test_correction_alone_matches_oracle(periodic):
    """Same inputs, same FMM: the difference between the two interpolations is
    the site correction only, which is computed exactly (FP64, no truncation
    beyond the degree-15 smooth part of the periodic Green's function)."""
    if periodic:
        d = W.tiny_periodic(82, n=300, edge=1.5, n_sites=5, depth=2, order=6)
    else:
        d = W.random_open(83, n=300, edge=2.0, n_sites=5, depth=2, order=6)
    a = run(d, "fp64", hamiltonian=True)
    b = run(d, "fp64")
    dE, dF, dD = oracle.hamiltonian_correction(d["x"], d["qA"], d["qB"], d["site"], d["lam"],
                                               d["box"], periodic)
    assert a["E"] - b["E"] == pytest.approx(dE, rel=1e-8, abs=1e-12)
    np.testing.assert_allclose(a["F"] - b["F"], dF, rtol=0, atol=1e-8 * np.abs(dF).max())
    np.testing.assert_allclose(a["dVdl"] - b["dVdl"], dD, rtol=1e-8, atol=1e-12)
    np.testing.assert_array_equal(a["phi"], b["phi"])


def test_end_states_match_charge_interpolation():
    d = W.tiny_periodic(84, n=200, edge=1.2, n_sites=4, depth=2, order=6)
    lam = np.array([0.0, 1.0, 0.0, 1.0])
    a = run(d, "f32", lam=lam, hamiltonian=True)
    b = run(d, "f32", lam=lam)
    assert a["E"] == b["E"]
    np.testing.assert_array_equal(a["F"], b["F"])


def test_lambda_derivative_is_derivative_of_energy():
    d = W.tiny_periodic(85, n=200, edge=1.2, n_sites=3, depth=2, order=6)
    base = run(d, "fp64", hamiltonian=True)
    h = 1e-3
    for s in range(d["lam"].size):
        lp, lm = d["lam"].copy(), d["lam"].copy()
        lp[s] += h
        lm[s] -= h
        fd = (run(d, "fp64", lam=lp, hamiltonian=True)["E"] -
              run(d, "fp64", lam=lm, hamiltonian=True)["E"]) / (2 * h)
        assert abs(fd - base["dVdl"][s]) <= 1e-9 * max(1.0, abs(base["E"])), (s, fd, base["dVdl"][s])


def test_adjoint_and_four_forms_are_unsupported():
    import torch
    from paper_2410_01626_amd import fmm
    dev = torch.device("cuda:0")
    d = W.with_tautomers(W.open_cube())
    plan = fmm.Plan(2, 4, precision="f32", max_atoms=1000, max_sites=10, device=dev,
                    hamiltonian=True)
    t = lambda v, ty=torch.float32: torch.tensor(v, dtype=ty, device=dev)
    x, qA, qB, qC, qD = (t(d[k]) for k in ("x", "qA", "qB", "qC", "qD"))
    site, lp, lt = t(d["site"], torch.int32), t(d["lam_p"], torch.float64), t(d["lam_t"], torch.float64)
    with pytest.raises(fmm.FmmError) as e:
        plan.eval_adjoint(x, qA, qB, site, lp, t([1.0], torch.float64))
    assert e.value.status == fmm.FMM_E_UNSUPPORTED
    with pytest.raises(fmm.FmmError) as e:
        plan.eval_tautomer(x, qA, qB, qC, qD, site, lp, lt)
    assert e.value.status == fmm.FMM_E_UNSUPPORTED
    plan.close()
