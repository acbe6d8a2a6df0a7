"""Pins of the oracle's bonded exclusions: the solve with a molecule's internal
pairs excluded against an independent pair-by-pair sum over atoms of
different molecules, the all-pairs-excluded limit, finite differences, and
invariance of the periodic result under shifting molecules across the cell
boundary (which breaks if the minimum image is wrong)."""
import numpy as np
import pytest

import oracle


def _molecules(seed, n_mol=6, edge=2.0):
    rng = np.random.default_rng(seed)
    x, q, mol = [], [], []
    for m in range(n_mol):
        c = rng.uniform(0.2, edge - 0.2, 3)
        for a in range(3):
            x.append(c + rng.normal(0, 0.08, 3))
            q.append([-0.8, 0.4, 0.4][a] * (1 + 0.1 * m))
            mol.append(m)
    return np.array(x), np.array(q), np.array(mol)


def _intramolecular(mol):
    start, idx = [0], []
    for i in range(mol.size):
        idx += [j for j in range(mol.size) if j != i and mol[j] == mol[i]]
        start.append(len(idx))
    return np.array(start), np.array(idx)


def test_open_exclusions_equal_the_intermolecular_sum():
    x, q, mol = _molecules(1)
    ex = _intramolecular(mol)
    site = np.full(q.size, -1, dtype=np.int32)
    r = oracle.solve(x, q, q, site, np.zeros(0), exclusions=ex)
    E = 0.0
    phi = np.zeros(q.size)
    for i in range(q.size):
        for j in range(q.size):
            if mol[i] != mol[j]:
                d = np.linalg.norm(x[i] - x[j])
                phi[i] += q[j] / d
                if i < j:
                    E += q[i] * q[j] / d
    assert r["E"] == pytest.approx(E, rel=1e-12)
    assert np.allclose(r["phi"], phi, rtol=1e-12, atol=1e-12)


def test_excluding_every_pair_leaves_nothing():
    x, q, _ = _molecules(2, n_mol=3)
    n = q.size
    start = np.arange(0, n * (n - 1) + 1, n - 1)
    idx = np.array([j for i in range(n) for j in range(n) if j != i])
    r = oracle.solve(x, q, q, np.full(n, -1, dtype=np.int32), np.zeros(0), exclusions=(start, idx))
    assert abs(r["E"]) < 1e-12 and np.abs(r["F"]).max() < 1e-11 and np.abs(r["phi"]).max() < 1e-12


@pytest.mark.parametrize("periodic", [False, True])
def test_exclusion_forces_and_lambda_derivative_by_finite_differences(periodic):
    x, q, mol = _molecules(3, n_mol=5)
    ex = _intramolecular(mol)
    n = q.size
    qB = q + np.where(np.arange(n) < 3, [0.3, -0.1, -0.2][0], 0.0)
    qB[:3] = q[:3] + np.array([0.3, -0.1, -0.2])
    site = np.where(np.arange(n) < 3, 0, -1).astype(np.int32)
    box = np.array([2.0, 2.0, 2.0]) if periodic else None
    kw = dict(box=box, periodic=periodic, exclusions=ex)
    lam = np.array([0.37])
    r = oracle.solve(x, q, qB, site, lam, **kw)
    h = 1e-5
    for i, a in ((0, 0), (4, 2), (11, 1)):
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        fd = -(oracle.solve(xp, q, qB, site, lam, **kw)["E"] - oracle.solve(xm, q, qB, site, lam, **kw)["E"]) / (2 * h)
        assert r["F"][i, a] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    fd = (oracle.solve(x, q, qB, site, lam + h, **kw)["E"] - oracle.solve(x, q, qB, site, lam - h, **kw)["E"]) / (2 * h)
    assert r["dVdl"][0] == pytest.approx(fd, rel=1e-7)


def test_periodic_exclusions_follow_the_minimum_image():
    # shifting every atom by a vector (molecules then straddle the faces)
    # changes nothing in a periodic cell, also with exclusions
    x, q, mol = _molecules(4, n_mol=5)
    q = q - q.mean()
    ex = _intramolecular(mol)
    site = np.full(q.size, -1, dtype=np.int32)
    box = np.array([2.0, 2.0, 2.0])
    a = oracle.solve(x, q, q, site, np.zeros(0), box=box, periodic=True, exclusions=ex)
    xs = np.mod(x + np.array([0.93, 1.41, 0.27]), 2.0)
    b = oracle.solve(xs, q, q, site, np.zeros(0), box=box, periodic=True, exclusions=ex)
    assert b["E"] == pytest.approx(a["E"], rel=1e-10)
    assert np.allclose(b["F"], a["F"], rtol=1e-8, atol=1e-9)
    # and removing the exclusions changes the energy by the molecules' own pairs
    full = oracle.solve(x, q, q, site, np.zeros(0), box=box, periodic=True)
    own = sum(q[i] * q[j] / np.linalg.norm(x[i] - x[j])
              for i in range(q.size) for j in range(i + 1, q.size) if mol[i] == mol[j])
    assert full["E"] - a["E"] == pytest.approx(own, rel=1e-10)
