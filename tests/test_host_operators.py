"""Host-side (CPU) checks of the library: exported symbols and the FP64
operator tables it builds at plan creation.

The operator tables are checked against mathematics, not against another copy
of themselves: the regular harmonics against scipy's spherical harmonics,
translations against direct Coulomb sums (exact where the translation is
exact, within the expected truncation error where it is not), and the
periodic lattice operator against the FP64 Ewald oracle.
"""
import ctypes
import math
import re

import numpy as np
import pytest
import scipy.special as sp

import oracle
from paper_2410_01626_amd import fmm

HEADER = open(__file__.rsplit("/tests/", 1)[0] + "/include/fmmcph.h").read()


def test_library_exports_every_declared_symbol():
    lib = fmm.load_library()
    declared = set(re.findall(r"\b(fmm_[a-z_]+)\s*\(", HEADER)) - {"fmm_plan_t"}
    assert declared == set(fmm.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_params_struct_layout():
    # int32 x4, double, int64 x2, int32 x8 -> 72 bytes with natural alignment
    assert ctypes.sizeof(fmm.fmm_params) == 72
    assert fmm.fmm_params.coulomb_k.offset == 16
    assert fmm.fmm_params.max_atoms.offset == 24


def test_plan_create_rejects_bad_params_without_gpu():
    lib = fmm.load_library()
    out = ctypes.c_void_p()
    for bad in (dict(depth=-1), dict(depth=7), dict(order_p=0), dict(order_p=16),
                dict(boundary=2), dict(precision=3), dict(max_replicas=0),
                dict(max_atoms=-5), dict(coulomb_k=float("nan")), dict(m2l_kernel=4),
                dict(m2l_chunk=190), dict(graph=2), dict(p2p_waves=5), dict(p2p_split=5),
                dict(p2p_split=-1), dict(hamiltonian=2), dict(hamiltonian=-1), dict(order_p=11, m2l_kernel=2),
                dict(order_p=11, m2l_kernel=3), dict(order_p=9, precision=0, m2l_kernel=2)):
        kw = dict(depth=2, order_p=4, boundary=0, precision=0, coulomb_k=1.0,
                  max_atoms=10, max_sites=1, max_replicas=1, check=0, m2l_kernel=0,
                  m2l_chunk=0, p2p_waves=0, graph=0)
        kw.update(bad)
        prm = fmm.fmm_params(**kw)
        assert lib.fmm_plan_create(ctypes.byref(prm), None, ctypes.byref(out)) == fmm.FMM_E_INVALID


def _sph(p, pts):
    """Real normalised regular harmonics from scipy: Rh_l^m = r^l sqrt(4pi/(2l+1)) Y_l^m."""
    pts = np.atleast_2d(pts)
    r = np.linalg.norm(pts, axis=1)
    th = np.arccos(np.clip(pts[:, 2] / np.where(r > 0, r, 1), -1, 1))
    ph = np.arctan2(pts[:, 1], pts[:, 0])
    K = (p + 1) ** 2
    out = np.zeros((pts.shape[0], K))
    for l in range(p + 1):
        for m in range(l + 1):
            y = sp.sph_harm_y(l, m, th, ph) * np.sqrt(4 * np.pi / (2 * l + 1)) * r ** l
            if m == 0:
                out[:, l * l] = y.real
            else:
                out[:, l * l + 2 * m - 1] = y.real
                out[:, l * l + 2 * m] = y.imag
    return out


def _rho(p, pts):
    return np.array([fmm.fmm_host_operator(p, 4, q) for q in np.atleast_2d(pts)])


@pytest.mark.parametrize("p", [3, 10])
def test_regular_harmonics_match_scipy(p):
    rng = np.random.default_rng(0)
    pts = rng.normal(size=(5, 3)) * 0.6
    np.testing.assert_allclose(_rho(p, pts), _sph(p, pts), rtol=1e-12, atol=1e-13)


def test_m2l_translation_reproduces_coulomb_sum():
    p = 8
    bank = fmm.fmm_host_operator(p, 0)
    rng = np.random.default_rng(1)
    q = rng.uniform(-1, 1, 25)
    xs = rng.uniform(-0.5, 0.5, (25, 3))
    mu = q @ _rho(p, xs)
    for o, tol in (((3, -2, 1), 2e-5), ((2, 0, 0), 5e-3), ((-2, 3, 3), 5e-6)):
        T = bank[o[0] + 3, o[1] + 3, o[2] + 3]
        xt = rng.uniform(-0.5, 0.5, (9, 3))
        lam = T @ mu
        phi = _rho(p, xt) @ lam
        exact = (q[None] / np.linalg.norm(xt[:, None] + np.array(o) - xs[None], axis=2)).sum(1)
        assert np.abs(phi - exact).max() <= tol * np.abs(exact).max(), o
    # near offsets are not translated
    assert np.all(bank[2:5, 2:5, 2:5] == 0)


def test_m2l_symmetric_truncation():
    """T(-o) = T(o)^T: the FMM energy is then an exactly symmetric quadratic form,
    so dE/dq_i equals the returned potential."""
    p = 6
    bank = fmm.fmm_host_operator(p, 0)
    for o in ((2, 1, -3), (3, 3, 3), (0, -2, 0)):
        a = bank[o[0] + 3, o[1] + 3, o[2] + 3]
        b = bank[-o[0] + 3, -o[1] + 3, -o[2] + 3]
        np.testing.assert_allclose(b, a.T, rtol=0, atol=1e-14 * np.abs(a).max())


def test_m2m_is_exact():
    p = 7
    A = fmm.fmm_host_operator(p, 1)
    rng = np.random.default_rng(2)
    mu_parent = np.zeros((p + 1) ** 2)
    direct = np.zeros((p + 1) ** 2)
    for c in range(8):
        b = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1]) - 0.5   # child centre, child units
        q = rng.uniform(-1, 1, 6)
        xs = rng.uniform(-0.5, 0.5, (6, 3)) + b                  # child units, parent centre 0
        mu_parent += A[c] @ (q @ _rho(p, xs - b))
        direct += q @ _rho(p, xs / 2)                            # parent edge = 2
    np.testing.assert_allclose(mu_parent, direct, rtol=1e-12, atol=1e-13)


def test_l2l_is_exact():
    p = 7
    B = fmm.fmm_host_operator(p, 2)
    rng = np.random.default_rng(3)
    lam_p = rng.normal(size=(p + 1) ** 2)
    for c in range(8):
        b = (np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1]) - 0.5) / 2  # parent units
        t = rng.uniform(-0.25, 0.25, (5, 3)) + b
        # phi = (1/h) lam~ . rho(t/h): parent h = 1, child h = 1/2
        phi_p = _rho(p, t) @ lam_p
        phi_c = 2.0 * _rho(p, (t - b) * 2) @ (B[c] @ lam_p)
        np.testing.assert_allclose(phi_c, phi_p, rtol=1e-12, atol=1e-12)


def _reflection_bits(p):
    """Per real coefficient: bit 2 if it flips sign under x -> -x, bit 1 under
    y -> -y, bit 0 under z -> -z (cos m phi, sin m phi and P_l^m parities)."""
    out = []
    for l in range(p + 1):
        for m in range(l + 1):
            zo = (l + m) & 1
            out.append(((m & 1) << 2) | zo)                 # cos part
            if m:
                out.append(((1 - (m & 1)) << 2) | 2 | zo)   # sin part
    return np.array(out)


@pytest.mark.parametrize("which", [1, 2])
def test_octant_operators_are_reflections_of_octant_0(which):
    """The device tree passes keep only octant 0 of M2M and L2L and form the
    other seven as S_c A_0 S_c; that must hold entry by entry."""
    p = 9
    A = fmm.fmm_host_operator(p, which)
    bits = _reflection_bits(p)
    for c in range(8):
        s = np.where(np.array([bin(c & b).count("1") & 1 for b in bits]) == 1, -1.0, 1.0)
        np.testing.assert_array_equal(A[c], s[:, None] * A[0] * s[None, :])


def test_m2l_operators_of_mirrored_offsets():
    """The bf16x3 M2L keeps one class's 189 operators and applies the others as
    T(P o) = S T(o) S (P a reflection of axes, S its diagonal signs)."""
    p = 7
    bank = fmm.fmm_host_operator(p, 0)
    bits = _reflection_bits(p)
    import itertools
    for c in range(1, 8):
        f = np.array([-1 if (c >> 2) & 1 else 1, -1 if (c >> 1) & 1 else 1, -1 if c & 1 else 1])
        s = np.where(np.array([bin(c & b).count("1") & 1 for b in bits]) == 1, -1.0, 1.0)
        for o in itertools.product(range(-3, 4), repeat=3):
            po = np.array(o) * f + 3
            np.testing.assert_array_equal(bank[po[0], po[1], po[2]],
                                          s[:, None] * bank[o[0] + 3, o[1] + 3, o[2] + 3] * s[None, :])


@pytest.mark.parametrize("neutral", [True, False])
def test_lattice_operator_matches_ewald(neutral):
    """Depth-0 periodic FMM assembled from the host lattice operator: near field
    over the 27 cells around the root, far field Lat mu, plus the background
    terms; compared with the FP64 Ewald oracle.  Pins the lattice sum, the
    tin-foil convention and the zero-mean gauge (a constant offset in phi
    would show up directly)."""
    p = 10
    L = 1.0
    rng = np.random.default_rng(4)
    n = 40
    x = rng.uniform(0, L, (n, 3))
    q = rng.uniform(-1, 1, n)
    if neutral:
        q -= q.mean()
    Lat = fmm.fmm_host_operator(p, 3)
    c = np.full(3, L / 2)
    s = (x - c) / L
    mu = q @ _rho(p, s)
    lam = Lat @ mu
    lam[0] += 2 * math.pi / 3 * np.sum(q * np.sum(s * s, 1))
    Q = q.sum()
    phi = _rho(p, s) @ lam / L + 2 * math.pi / 3 * Q * np.sum(s * s, 1) / L
    imgs = np.array([[a, b, cc] for a in (-1, 0, 1) for b in (-1, 0, 1) for cc in (-1, 0, 1)])
    d = x[:, None, None, :] - x[None, :, None, :] + imgs[None, None] * L
    r = np.linalg.norm(d, axis=-1)
    with np.errstate(divide="ignore"):
        w = np.where(r > 0, 1.0 / r, 0.0)
    phi += np.einsum("j,ijk->i", q, w)
    ref, _ = oracle.ewald(x, q, [L] * 3)
    err = np.abs(phi - ref).max() / np.abs(ref).max()
    assert err < 2e-5, err
    assert abs(np.mean(phi - ref)) < 2e-5 * np.abs(ref).max()


def test_periodic_green_function_matches_ewald():
    """The pair potential of the Hamiltonian-interpolation correction: the unit
    cube's periodic Green's function rebuilt from the host coefficients of its
    smooth part, sum_{27 images} 1/|u+n| + (2 pi/3)|u|^2 + h(u), against the
    FP64 Ewald potential of one unit charge (tin-foil, background, zero mean),
    and its self-image limit against the Ewald self term."""
    P = 15
    c = fmm.fmm_host_operator(P, 5)
    imgs = np.array([[a, b, cc] for a in (-1, 0, 1) for b in (-1, 0, 1) for cc in (-1, 0, 1)],
                    dtype=np.float64)
    rng = np.random.default_rng(9)
    for u in list(rng.uniform(-0.3, 0.3, (6, 3))) + [np.array([0.5, -0.2, 0.1])]:
        psi = np.sum(1.0 / np.linalg.norm(u + imgs, axis=1))
        psi += 2 * math.pi / 3 * float(u @ u) + float(c @ _rho(P, u)[0])
        ref, _ = oracle.ewald(np.array([u, [0.0, 0.0, 0.0]]), np.array([0.0, 1.0]), [1.0] * 3,
                              eps=1e-14)
        assert psi == pytest.approx(ref[0], rel=1e-9, abs=1e-9), (u, psi, ref[0])
    near = np.sum([1.0 / np.linalg.norm(n) for n in imgs if np.any(n)])
    ref0, _ = oracle.ewald(np.zeros((1, 3)), np.ones(1), [1.0] * 3, eps=1e-14)
    assert near + c[0] == pytest.approx(ref0[0], rel=1e-10, abs=1e-10)
