"""Pins of the Hamiltonian-interpolation oracle (Methods, eq 1 taken literally:
each site's Hamiltonian is the lambda-weighted mix of its two end states, and
several sites mix multilinearly).  The pin is the definition itself, evaluated
the long way: the energy and forces of every one of the 2^S end-state
combinations, weighted by prod_s (1 - lambda_s or lambda_s).  Since that
mixture is linear in each lambda_s, dV/dlambda_s is also the difference of the
two mixtures with lambda_s set to 1 and to 0.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2410_01626_amd import workloads as W

EW = 1e-12


def _cases():
    return {"open": W.random_open(71, n=120, edge=1.4, n_sites=3, depth=1, order=4),
            "periodic": W.tiny_periodic(72, n=80, edge=1.2, n_sites=3, depth=1, order=4)}


def _mixture(d, lam):
    """Hamiltonian interpolation by enumeration of the end-state combinations."""
    S = lam.size
    E, F = 0.0, np.zeros((d["x"].shape[0], 3))
    for combo in itertools.product((0, 1), repeat=S):
        w = np.prod([lam[s] if c else 1.0 - lam[s] for s, c in enumerate(combo)])
        lc = np.array(combo, dtype=np.float64)
        r = oracle.solve(d["x"], d["qA"], d["qB"], d["site"], lc, box=d["box"],
                         periodic=d["periodic"], eps=EW)
        E += w * r["E"]
        F += w * r["F"]
    return E, F


@pytest.mark.parametrize("case", ["open", "periodic"])
def test_hamiltonian_interpolation_is_the_mixture_of_end_states(case):
    d = _cases()[case]
    lam = d["lam"]
    r = oracle.solve(d["x"], d["qA"], d["qB"], d["site"], lam, box=d["box"],
                     periodic=d["periodic"], eps=EW, hamiltonian=True)
    E, F = _mixture(d, lam)
    assert r["E"] == pytest.approx(E, rel=1e-11, abs=1e-11)
    np.testing.assert_allclose(r["F"], F, rtol=0, atol=1e-10 * np.abs(F).max())
    for s in range(lam.size):
        hi, lo = lam.copy(), lam.copy()
        hi[s], lo[s] = 1.0, 0.0
        exact = _mixture(d, hi)[0] - _mixture(d, lo)[0]
        assert r["dVdl"][s] == pytest.approx(exact, rel=1e-10, abs=1e-10), s


@pytest.mark.parametrize("case", ["open", "periodic"])
def test_end_states_need_no_correction(case):
    """At lambda in {0, 1} the two interpolations coincide."""
    d = _cases()[case]
    lam = np.array([0.0, 1.0, 1.0])
    dE, dF, _ = oracle.hamiltonian_correction(d["x"], d["qA"], d["qB"], d["site"], lam,
                                              d["box"], d["periodic"])
    assert dE == 0.0 and not np.any(dF)
