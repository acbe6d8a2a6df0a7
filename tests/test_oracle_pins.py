"""Pins of the FP64 oracle against closed forms, invariants and brute force.

None of these compares the oracle with another implementation of the same
formula: each check is fixed by mathematics (closed forms, exact symmetries,
finite differences of the oracle's own energy, or an independent brute-force
image sum), so a dropped term, a wrong sign or a transposed operand in the
oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
from conftest import golden
from paper_2410_01626_amd import workloads as W

G = golden("lattice_constants.txt")


def _rng(k):
    return np.random.default_rng(1000 + k)


# ---------------------------------------------------------------- open boundaries

def test_two_charges_closed_form():
    x = np.array([[0.1, -0.2, 0.3], [0.7, 0.4, -0.5]])
    q = np.array([1.5, -0.75])
    phi, field = oracle.direct(x, q)
    d = x[0] - x[1]
    r = np.linalg.norm(d)
    assert phi[0] == pytest.approx(q[1] / r, rel=1e-15)
    assert phi[1] == pytest.approx(q[0] / r, rel=1e-15)
    E, F, _ = oracle.outputs(q, q, q, np.full(2, -1), 0, phi, field, k_e=2.0)
    assert E == pytest.approx(2.0 * q[0] * q[1] / r, rel=1e-15)
    # Coulomb's law: F_0 = k q0 q1 d / r^3
    np.testing.assert_allclose(F[0], 2.0 * q[0] * q[1] * d / r ** 3, rtol=1e-14)
    np.testing.assert_allclose(F[1], -F[0], rtol=1e-14)


def test_three_charges_brute_force():
    # an equilateral triangle of equal charges: every potential is 2q/a
    a = 0.37
    x = np.array([[0, 0, 0], [a, 0, 0], [a / 2, a * math.sqrt(3) / 2, 0]])
    q = np.full(3, 0.6)
    phi, field = oracle.direct(x, q)
    np.testing.assert_allclose(phi, 2 * 0.6 / a, rtol=1e-15)
    # field at each vertex points away from the centroid with magnitude sqrt(3) q / a^2
    c = x.mean(0)
    for i in range(3):
        u = (x[i] - c) / np.linalg.norm(x[i] - c)
        np.testing.assert_allclose(field[i], math.sqrt(3) * 0.6 / a ** 2 * u, rtol=1e-13,
                                   atol=1e-13)


def _fd_force(fun, x, i, a, h):
    xp = x.copy(); xp[i, a] += h
    xm = x.copy(); xm[i, a] -= h
    return -(fun(xp) - fun(xm)) / (2 * h)


@pytest.mark.parametrize("periodic", [False, True])
def test_force_is_minus_energy_gradient(periodic):
    rng = _rng(1)
    n = 24
    L = 1.3
    x = rng.uniform(0, L, (n, 3))
    q = rng.uniform(-1, 1, n)
    if periodic:
        q -= q.mean() * 0.5  # non-neutral on purpose: the background term has no force

    def energy(xx):
        if periodic:
            phi, _ = oracle.ewald(xx, q, [L] * 3)
        else:
            phi, _ = oracle.direct(xx, q)
        return 0.5 * np.sum(q * phi)

    if periodic:
        phi, field = oracle.ewald(x, q, [L] * 3)
    else:
        phi, field = oracle.direct(x, q)
    F = q[:, None] * field
    for i in (0, 5, 17):
        for a in range(3):
            fd = _fd_force(energy, x, i, a, 1e-5)
            assert F[i, a] == pytest.approx(fd, rel=2e-7, abs=2e-7 * np.abs(F).max())


@pytest.mark.parametrize("periodic", [False, True])
def test_net_force_zero(periodic):
    rng = _rng(2)
    n = 60
    x = rng.uniform(0, 2.0, (n, 3))
    q = rng.uniform(-1, 1, n)
    if periodic:
        phi, field = oracle.ewald(x, q, [2.0] * 3)
    else:
        phi, field = oracle.direct(x, q)
    F = q[:, None] * field
    assert np.abs(F.sum(0)).max() <= 1e-12 * n * np.sqrt(np.mean(F ** 2))


@pytest.mark.parametrize("periodic", [False, True])
def test_dvdl_is_lambda_derivative_of_energy(periodic):
    """E is exactly quadratic in lambda, so a central difference is exact up to
    rounding; dV/dlambda_s = sum_{i in s} (qB - qA) phi_i must equal it."""
    d = W.tiny_periodic(7, n=48, edge=1.4, n_sites=3, neutral=True)
    box = d["box"] if periodic else None

    def E_of(lam):
        r = oracle.solve(d["x"], d["qA"], d["qB"], d["site"], lam, box=box,
                         periodic=periodic, k_e=1.7)
        return r["E"], r["dVdl"]

    E0, dV = E_of(d["lam"])
    h = 1e-3
    for s in range(d["lam"].size):
        lp = d["lam"].copy(); lp[s] += h
        lm = d["lam"].copy(); lm[s] -= h
        fd = (E_of(lp)[0] - E_of(lm)[0]) / (2 * h)
        assert dV[s] == pytest.approx(fd, rel=1e-9, abs=1e-9 * abs(E0))


def test_lambda_charges_no_clamp_and_unsited_atoms():
    qA = np.array([0.5, -0.2, 1.0])
    qB = np.array([-0.5, 0.8, 7.0])
    site = np.array([0, 0, -1], dtype=np.int32)
    q = oracle.lambda_charges(qA, qB, site, np.array([1.1]))
    np.testing.assert_allclose(q, [0.5 + 1.1 * -1.0, -0.2 + 1.1 * 1.0, 1.0], rtol=1e-15)
    q = oracle.lambda_charges(qA, qB, site, np.array([-0.1]))
    np.testing.assert_allclose(q, [0.5 + 0.1, -0.2 - 0.1, 1.0], rtol=1e-15)
    with pytest.raises(ValueError):
        oracle.lambda_charges(qA, qB, np.array([0, 1, -1], dtype=np.int32), np.array([0.3]))


@pytest.mark.parametrize("periodic", [False, True])
def test_linearity_in_charges(periodic):
    rng = _rng(3)
    n = 40
    x = rng.uniform(0, 1.5, (n, 3))
    q1 = rng.uniform(-1, 1, n)
    q2 = rng.uniform(-1, 1, n)
    f = (lambda q: oracle.ewald(x, q, [1.5] * 3)) if periodic else (lambda q: oracle.direct(x, q))
    p1, e1 = f(q1)
    p2, e2 = f(q2)
    p3, e3 = f(q1 + 2.5 * q2)
    np.testing.assert_allclose(p3, p1 + 2.5 * p2, rtol=1e-12, atol=1e-12 * np.abs(p3).max())
    np.testing.assert_allclose(e3, e1 + 2.5 * e2, rtol=1e-12, atol=1e-12 * np.abs(e3).max())


# ---------------------------------------------------------------- periodic boundaries

def _nacl(a):
    pos, q = [], []
    for i in range(2):
        for j in range(2):
            for k in range(2):
                pos.append([i * a / 2, j * a / 2, k * a / 2])
                q.append(1.0 if (i + j + k) % 2 == 0 else -1.0)
    return np.array(pos), np.array(q)


@pytest.mark.parametrize("a", [1.0, 0.5627])
def test_madelung_nacl(a):
    x, q = _nacl(a)
    x = x + 0.1234 * a  # arbitrary origin
    phi, field = oracle.ewald(x, q, [a] * 3)
    E = 0.5 * np.sum(q * phi)
    M = -E * (a / 2) / 4
    assert M == pytest.approx(G["madelung_nacl"], rel=1e-12)
    assert np.abs(field).max() < 1e-11 / a ** 2  # every ion sits at a centre of symmetry


def test_madelung_cscl():
    a = 0.8
    x = np.array([[0, 0, 0], [a / 2, a / 2, a / 2]]) + 0.05
    q = np.array([1.0, -1.0])
    phi, _ = oracle.ewald(x, q, [a] * 3)
    E = 0.5 * np.sum(q * phi)
    r0 = math.sqrt(3) * a / 2
    assert -E * r0 == pytest.approx(G["madelung_cscl"], rel=1e-12)


def test_madelung_zincblende():
    a = 1.1
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]]) * a
    x = np.concatenate([fcc, fcc + a / 4])
    q = np.array([1.0] * 4 + [-1.0] * 4)
    phi, _ = oracle.ewald(x, q, [a] * 3)
    E = 0.5 * np.sum(q * phi)
    r0 = math.sqrt(3) * a / 4
    assert -E * r0 / 4 == pytest.approx(G["madelung_zns"], rel=1e-12)


@pytest.mark.parametrize("L", [1.0, 3.7])
def test_single_charge_wigner_constant(L):
    """One charge with a uniform neutralising background: E = xi q^2 / (2 L).
    Pins the background and the zero-mean gauge together with the self term."""
    x = np.array([[0.3, 0.7, 0.11]]) * L
    q = np.array([-1.3])
    phi, field = oracle.ewald(x, q, [L] * 3)
    E = 0.5 * q[0] * phi[0]
    assert E == pytest.approx(G["wigner_sc"] * q[0] ** 2 / (2 * L), rel=1e-12)
    assert np.abs(field).max() < 1e-12


def test_ewald_beta_independence():
    rng = _rng(4)
    n = 50
    box = [2.0, 2.2, 1.9]
    x = rng.uniform(0, 2, (n, 3))
    q = rng.normal(size=n)  # non-neutral on purpose
    p1, f1 = oracle.ewald(x, q, box, rcut=0.95)
    p2, f2 = oracle.ewald(x, q, box, rcut=0.6)
    p3, f3 = oracle.ewald(x, q, box, rcut=1.7)  # several images inside the cutoff
    for p, f in ((p2, f2), (p3, f3)):
        np.testing.assert_allclose(p, p1, rtol=0, atol=1e-12 * np.abs(p1).max())
        np.testing.assert_allclose(f, f1, rtol=0, atol=1e-11 * np.abs(f1).max())


def test_ewald_translation_invariance():
    rng = _rng(5)
    n = 40
    L = 1.6
    x = rng.uniform(0, L, (n, 3))
    q = rng.uniform(-1, 1, n)
    p1, f1 = oracle.ewald(x, q, [L] * 3)
    p2, f2 = oracle.ewald(np.mod(x + np.array([0.37, -1.1, 2.9]), L), q, [L] * 3)
    np.testing.assert_allclose(p2, p1, atol=1e-12 * np.abs(p1).max())
    np.testing.assert_allclose(f2, f1, atol=1e-11 * np.abs(f1).max())


def test_spherical_image_sum_brute_force():
    """Summing whole neutral cells inside growing spheres converges to the
    tin-foil Ewald energy plus the vacuum surface term 2 pi |D|^2 / (3 V)
    (de Leeuw, Perram & Smith 1980).  Brute force over ~ 10^5 images, with a
    Richardson step in 1/R^2 on the shell-cut sequence."""
    rng = _rng(6)
    L = 1.0
    n = 6
    x = rng.uniform(0, L, (n, 3))
    q = rng.uniform(-1, 1, n)
    q -= q.mean()
    D = (q[:, None] * x).sum(0)
    phi, _ = oracle.ewald(x, q, [L] * 3)
    E_ew = 0.5 * np.sum(q * phi)
    E_vac = E_ew + 2 * math.pi * (D @ D) / (3 * L ** 3)

    def shell_energy(R):
        m = int(R) + 1
        g = np.arange(-m, m + 1)
        nv = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(float)
        nv = nv[np.sum(nv ** 2, 1) <= R * R]
        d = x[:, None, :] - x[None, :, :]                      # (n, n, 3)
        r = np.linalg.norm(d[:, :, None, :] + nv[None, None] * L, axis=-1)
        iszero = np.all(nv == 0, axis=1)
        w = np.where(r > 0, 1.0 / np.where(r > 0, r, 1.0), 0.0)
        w[:, :, iszero] *= (1 - np.eye(n))[:, :, None]
        return 0.5 * np.einsum("i,j,ijk->", q, q, w)

    R1, R2 = 24.0, 34.0
    e1, e2 = shell_energy(R1), shell_energy(R2)
    extrap = (e2 * R2 ** 2 - e1 * R1 ** 2) / (R2 ** 2 - R1 ** 2)
    assert abs(e2 - E_vac) < 3e-4 * abs(E_vac)
    assert abs(extrap - E_vac) < 3e-5 * abs(E_vac)
    # and tin-foil without the surface term is clearly different when D != 0
    assert abs(E_ew - E_vac) > 1e-2 * abs(E_vac)


def test_large_box_tends_to_open_boundaries():
    """A small neutral cluster in an ever larger periodic box: image,
    background and gauge terms all vanish like 1/L^3."""
    rng = _rng(7)
    n = 30
    xc = rng.uniform(0, 0.6, (n, 3))
    q = rng.uniform(-1, 1, n)
    q -= q.mean()
    p0, f0 = oracle.direct(xc, q)
    errs = []
    for L in (10.0, 20.0):
        x = xc + L / 2
        p, f = oracle.ewald(x, q, [L] * 3, rcut=3.0)
        errs.append(np.abs(p - p0).max() / np.abs(p0).max())
        np.testing.assert_allclose(f, f0, atol=1e-3 / L ** 2 * np.abs(f0).max())
    assert errs[1] < 1e-4
    assert errs[1] < errs[0] / 4  # ~ 1/L^3 decay


def test_ewald_subset_targets_match_full():
    rng = _rng(8)
    n = 70
    x = rng.uniform(0, 1.7, (n, 3))
    q = rng.uniform(-1, 1, n)
    p, f = oracle.ewald(x, q, [1.7] * 3)
    t = np.array([3, 0, 69, 12])
    ps, fs = oracle.ewald(x, q, [1.7] * 3, targets=t)
    np.testing.assert_array_equal(ps, p[t])
    np.testing.assert_array_equal(fs, f[t])
    pd, fd = oracle.direct(x, q)
    pds, fds = oracle.direct(x, q, targets=t)
    np.testing.assert_array_equal(pds, pd[t])
    np.testing.assert_array_equal(fds, fd[t])


def test_energy_is_euler_sum_and_k_e_scaling():
    d = W.open_cube()
    r1 = oracle.solve(d["x"], d["qA"], d["qB"], d["site"], d["lam"], k_e=1.0)
    r2 = oracle.solve(d["x"], d["qA"], d["qB"], d["site"], d["lam"], k_e=138.935458)
    assert r2["E"] == pytest.approx(138.935458 * r1["E"], rel=1e-14)
    np.testing.assert_allclose(r2["dVdl"], 138.935458 * r1["dVdl"], rtol=1e-13)
    assert r1["E"] == pytest.approx(0.5 * np.sum(r1["q"] * r1["phi"]), rel=1e-14)
