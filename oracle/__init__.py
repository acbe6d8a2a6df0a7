"""FP64 CPU oracle for the lambda-interpolated Coulomb solve.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library never does, and
this package never imports the product package.  The arithmetic lives in
``coulomb_oracle.c`` (plain C, FP64, OpenMP over target atoms); this file only
marshals numpy arrays and chooses Ewald parameters.

What is computed (constant-pH lambda-dynamics paper, Methods, eq 1 with the
charge-interpolated form, and "Calibration of Protonation Dynamics", where the
lambda-derivative of the Hamiltonian is the Coulomb term alone):

    q_i     = qA_i + lambda_{s(i)} (qB_i - qA_i)         (site -1: q_i = qA_i)
    phi_i   = k_e sum_j' q_j psi(r_i - r_j)              (potential at atom i)
    E       = 1/2 sum_i q_i phi_i
    F_i     = -dE/dr_i
    dVdl_s  = sum_{i in s} (qB_i - qA_i) phi_i           (= dE/dlambda_s)

with psi = 1/r for open boundaries (direct sum) and psi the tin-foil,
neutralising-background, zero-mean periodic Green's function for periodic ones
(Ewald sum).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "coulomb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if (not os.path.exists(_LIB_PATH)
            or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_lambda_charges.restype = ctypes.c_int
    lib.orc_lambda_charges.argtypes = [ctypes.c_int64, _f64p, _f64p, _i32p,
                                       ctypes.c_int64, _f64p, _f64p]
    lib.orc_direct.restype = None
    lib.orc_direct.argtypes = [ctypes.c_int64, _f64p, _f64p, ctypes.c_int64,
                               ctypes.c_void_p, _f64p, _f64p]
    lib.orc_ewald.restype = ctypes.c_int
    lib.orc_ewald.argtypes = [ctypes.c_int64, _f64p, _f64p, _f64p, ctypes.c_double,
                              ctypes.c_double, _i32p, ctypes.c_int64,
                              ctypes.c_void_p, _f64p, _f64p]
    lib.orc_outputs.restype = ctypes.c_int
    lib.orc_outputs.argtypes = [ctypes.c_int64, _f64p, _f64p, _f64p, _i32p,
                                ctypes.c_int64, _f64p, _f64p, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                ctypes.c_void_p]
    lib.orc_tautomer_charges.restype = ctypes.c_int
    lib.orc_tautomer_charges.argtypes = [ctypes.c_int64, _f64p, _f64p, _f64p, _f64p, _i32p,
                                         ctypes.c_int64, _f64p, _f64p, _f64p]
    lib.orc_tautomer_dvdl.restype = ctypes.c_int
    lib.orc_tautomer_dvdl.argtypes = [ctypes.c_int64, _f64p, _f64p, _f64p, _f64p, _i32p,
                                      ctypes.c_int64, _f64p, _f64p, _f64p, ctypes.c_double,
                                      _f64p, _f64p]
    lib.orc_direct_wpair.restype = None
    lib.orc_direct_wpair.argtypes = [ctypes.c_int64, _f64p, _f64p, _f64p, ctypes.c_int64,
                                     ctypes.c_void_p, _f64p, _f64p]
    lib.orc_ewald_wpair.restype = ctypes.c_int
    lib.orc_ewald_wpair.argtypes = [ctypes.c_int64, _f64p, _f64p, _f64p, _f64p, ctypes.c_double,
                                    ctypes.c_double, _i32p, ctypes.c_int64, ctypes.c_void_p,
                                    _f64p, _f64p]
    _lib = lib
    return lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def lambda_charges(qA, qB, site, lam):
    """eq 1, charge-interpolated: q = qA + lambda_s (qB - qA); site -1 keeps qA."""
    qA, qB, lam = _f64(qA), _f64(qB), _f64(np.atleast_1d(lam))
    site = np.ascontiguousarray(site, dtype=np.int32)
    q = np.empty_like(qA)
    rc = _load().orc_lambda_charges(qA.size, qA, qB, site, lam.size, lam, q)
    if rc != 0:
        raise ValueError("site index outside [-1, n_sites)")
    return q


def _targets(targets, n):
    if targets is None:
        return None, n, None
    t = np.ascontiguousarray(targets, dtype=np.int64)
    if t.size and (t.min() < 0 or t.max() >= n):
        raise ValueError("target index out of range")
    return t, t.size, t.ctypes.data


def direct(x, q, targets=None):
    """Open-boundary direct sum: phi_i = sum_{j!=i} q_j/r_ij and the field at i."""
    x, q = _f64(x).reshape(-1, 3), _f64(q)
    t, nt, tp = _targets(targets, q.size)
    phi = np.empty(nt)
    field = np.empty((nt, 3))
    _load().orc_direct(q.size, x, q, nt, tp, phi, field)
    return phi, field


def ewald_params(box, eps: float = 1e-13, rcut: float | None = None):
    """Ewald parameters for a relative accuracy of about eps.

    rcut defaults to half the shortest edge; beta = s / rcut with
    erfc(s) ~ eps; kmax_a = ceil(2 beta s L_a / (2 pi)) so that
    exp(-k^2 / 4 beta^2) < eps beyond it.
    """
    box = np.asarray(box, dtype=np.float64).reshape(3)
    if rcut is None:
        rcut = 0.5 * float(box.min())
    s = math.sqrt(-math.log(eps))
    while math.erfc(s) > eps:
        s += 0.05
    beta = s / rcut
    kmax = np.array([int(math.ceil(2 * beta * s * L / (2 * math.pi))) for L in box],
                    dtype=np.int32)
    return float(beta), float(rcut), kmax


def ewald(x, q, box, beta=None, rcut=None, kmax=None, eps=1e-13, targets=None):
    """Periodic Ewald potential and field (tin-foil, background, zero mean)."""
    x, q = _f64(x).reshape(-1, 3), _f64(q)
    box = _f64(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
    b0, r0, k0 = ewald_params(box, eps, rcut)
    beta = b0 if beta is None else float(beta)
    rcut = r0 if rcut is None else float(rcut)
    if kmax is None:
        s = beta * rcut
        kmax = np.array([int(math.ceil(2 * beta * s * L / (2 * math.pi))) for L in box],
                        dtype=np.int32)
    kmax = np.ascontiguousarray(np.broadcast_to(np.asarray(kmax), (3,)), dtype=np.int32)
    t, nt, tp = _targets(targets, q.size)
    phi = np.empty(nt)
    field = np.empty((nt, 3))
    rc = _load().orc_ewald(q.size, x, q, box, beta, rcut, kmax, nt, tp, phi, field)
    if rc != 0:
        raise ValueError("orc_ewald: bad arguments or out of memory")
    return phi, field


def outputs(q, qA, qB, site, n_sites, phi, field, k_e=1.0):
    """E = 1/2 k_e sum q phi ; F = k_e q field ; dVdl_s = k_e sum_{i in s} dq_i phi_i."""
    q, qA, qB, phi = _f64(q), _f64(qA), _f64(qB), _f64(phi)
    field = _f64(field).reshape(-1, 3)
    site = np.ascontiguousarray(site, dtype=np.int32)
    F = np.empty((q.size, 3))
    dVdl = np.empty(max(int(n_sites), 0))
    E = ctypes.c_double(0.0)
    rc = _load().orc_outputs(q.size, q, qA, qB, site, int(n_sites), phi, field,
                             float(k_e), ctypes.byref(E), F.ctypes.data,
                             dVdl.ctypes.data if dVdl.size else None)
    if rc != 0:
        raise ValueError("site index outside [-1, n_sites)")
    return E.value, F, dVdl


def exclusion_terms(x, q, excl_start, excl_idx, box=None, periodic=False):
    """Potential and field at every atom from its excluded partners alone:
    phi_i = sum_{j in excl(i)} q_j / r_ij, field_i = sum q_j r_ij / r_ij^3,
    r_ij = x_i - x_j (periodic: the minimum image, each component wrapped
    into [-L/2, L/2]).  Plain numpy loops over the listed pairs."""
    x = _f64(x).reshape(-1, 3)
    q = _f64(q)
    phi, field = np.zeros(q.size), np.zeros((q.size, 3))
    for i in range(len(excl_start) - 1):
        for e in range(excl_start[i], excl_start[i + 1]):
            j = int(excl_idx[e])
            d = x[i] - x[j]
            if periodic:
                L = float(np.atleast_1d(box)[0])
                d = d - L * np.round(d / L)
            r = math.sqrt(float(d @ d))
            phi[i] += q[j] / r
            field[i] += q[j] * d / r ** 3
    return phi, field


def solve(x, qA, qB, site, lam, box=None, periodic=False, k_e=1.0, eps=1e-13,
          ewald_kw=None, hamiltonian=False, exclusions=None):
    """Full oracle solve.  Returns dict(E, F, phi, dVdl, q), all FP64.

    phi is returned already multiplied by k_e.  With hamiltonian=True the
    energy is that of eq 1 taken literally (each site's two end Hamiltonians
    mixed linearly): see hamiltonian_correction; phi stays the potential of the
    interpolated charges.  exclusions = (start, idx), a symmetric per-atom
    list of excluded partners: their pair terms (the minimum image for a
    periodic cell; the other images stay) are removed from phi and the field
    before the outputs are formed.
    """
    lam = _f64(np.atleast_1d(lam))
    q = lambda_charges(qA, qB, site, lam)
    if periodic:
        phi, field = ewald(x, q, box, eps=eps, **(ewald_kw or {}))
    else:
        phi, field = direct(x, q)
    if exclusions is not None:
        ephi, efield = exclusion_terms(x, q, exclusions[0], exclusions[1], box, periodic)
        phi, field = phi - ephi, field - efield
    E, F, dVdl = outputs(q, qA, qB, site, lam.size, phi, field, k_e)
    if hamiltonian:
        dE, dF, dD = hamiltonian_correction(x, qA, qB, site, lam, box, periodic, k_e, eps)
        E, F, dVdl = E + dE, F + dF, dVdl + dD
    return {"E": E, "F": F, "phi": k_e * phi, "dVdl": dVdl, "q": q}


def adjoint_phi(x, qA, qB, site, lam, gE, gphi, box=None, periodic=False, k_e=1.0, eps=1e-13):
    """Gradients of L = gE E + sum_i gphi_i phi_i (phi as solve returns it,
    with k_e) with respect to x, qA, qB and lambda.  phi = k_e Psi q is
    linear in q with the symmetric pair matrix Psi, so dL/dq = gE phi +
    k_e Psi gphi (the potential of charges gphi), and
    dL/dx_k = -gE F_k - k_e (gphi_k field_k(q) + q_k field_k(gphi)),
    field(c) the field of charges c at the atoms.  Returns (gx, gqA, gqB, glam)."""
    x = _f64(x).reshape(-1, 3)
    qA, qB, gphi = _f64(qA), _f64(qB), _f64(gphi)
    lam = _f64(np.atleast_1d(lam))
    site = np.ascontiguousarray(site, dtype=np.int32)
    q = lambda_charges(qA, qB, site, lam)
    if periodic:
        pq, fq = ewald(x, q, box, eps=eps)
        pg, fg = ewald(x, gphi, box, eps=eps)
    else:
        pq, fq = direct(x, q)
        pg, fg = direct(x, gphi)
    gq = k_e * (gE * pq + pg)
    gx = -k_e * (gE * q[:, None] * fq + gphi[:, None] * fq + q[:, None] * fg)
    insite = (site >= 0)
    lam_i = np.where(insite, lam[np.maximum(site, 0)], 0.0)
    gqA = (1.0 - lam_i) * gq
    gqB = lam_i * gq
    glam = np.zeros(lam.size)
    for s in range(lam.size):
        m = site == s
        glam[s] = np.sum((qB[m] - qA[m]) * gq[m])
    return gx, gqA, gqB, glam


def _ewald_setup(box, beta, rcut, kmax, eps):
    box = _f64(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
    b0, r0, k0 = ewald_params(box, eps, rcut)
    beta = b0 if beta is None else float(beta)
    rcut = r0 if rcut is None else float(rcut)
    if kmax is None:
        s = beta * rcut
        kmax = np.array([int(math.ceil(2 * beta * s * L / (2 * math.pi))) for L in box],
                        dtype=np.int32)
    kmax = np.ascontiguousarray(np.broadcast_to(np.asarray(kmax), (3,)), dtype=np.int32)
    return box, beta, rcut, kmax


def force_weight_sums(x, q, w, box=None, periodic=False, beta=None, rcut=None, kmax=None,
                      eps=1e-13, targets=None):
    """Pair sums of the force-weight adjoint at every target m (w: n x 3
    weights, one per atom's force):
        hw_m = sum_j q_j [grad grad psi](r_m - r_j) (w_m - w_j)
        ew_m = sum_j q_j e(r_m - r_j) . (w_m - w_j),  e = -grad psi,
    psi = 1/r (open, j != m) or the Ewald potential (periodic, all images).
    Returns (hw, ew)."""
    x, q = _f64(x).reshape(-1, 3), _f64(q)
    w = _f64(w).reshape(-1, 3)
    t, nt, tp = _targets(targets, q.size)
    hw = np.empty((nt, 3))
    ew = np.empty(nt)
    if periodic:
        box, beta, rcut, kmax = _ewald_setup(box, beta, rcut, kmax, eps)
        rc = _load().orc_ewald_wpair(q.size, x, q, w, box, beta, rcut, kmax, nt, tp, hw, ew)
        if rc != 0:
            raise ValueError("orc_ewald_wpair: bad arguments or out of memory")
    else:
        _load().orc_direct_wpair(q.size, x, q, w, nt, tp, hw, ew)
    return hw, ew


def adjoint_full(x, qA, qB, site, lam, gE=0.0, gphi=None, gF=None, box=None, periodic=False,
                 k_e=1.0, eps=1e-13, targets=None):
    """Gradients of L = gE E + sum_i gphi_i phi_i + sum_i gF_i . F_i (phi and F
    as solve returns them, with k_e) with respect to x, qA, qB and lambda.

    E = 1/2 k_e q^T Psi q, phi = k_e Psi q and F_m = k_e q_m sum_j q_j e(r_mj)
    (Psi the symmetric pair matrix of psi, e = -grad psi).  Differentiating
    each term:
        dL/dq_m = gE phi_m + k_e (Psi gphi)_m + k_e ew_m
        dL/dx_m = -gE F_m - k_e (gphi_m field_m(q) + q_m field_m(gphi)) - k_e q_m hw_m
    with hw, ew the force-weight pair sums (force_weight_sums); then
    dL/dqA = (1 - lambda_s) dL/dq, dL/dqB = lambda_s dL/dq (site -1: qB gets 0)
    and dL/dlambda_s = sum_{m in s} (qB_m - qA_m) dL/dq_m.
    With targets (atom indices), the per-atom gradients are returned for those
    atoms only (the sums still run over every atom), and glam only when every
    site atom is among them (else None).
    Returns (gx, gqA, gqB, glam)."""
    x = _f64(x).reshape(-1, 3)
    qA, qB = _f64(qA), _f64(qB)
    lam = _f64(np.atleast_1d(lam))
    site = np.ascontiguousarray(site, dtype=np.int32)
    n = qA.size
    q = lambda_charges(qA, qB, site, lam)
    t = np.arange(n) if targets is None else np.asarray(targets, dtype=np.int64)

    def field_of(c):
        return (ewald(x, c, box, eps=eps, targets=t) if periodic else direct(x, c, targets=t))

    pq, fq = field_of(q)
    qt = q[t]
    gq = k_e * gE * pq
    gx = -k_e * gE * qt[:, None] * fq
    if gphi is not None:
        gphi = _f64(gphi)
        pg, fg = field_of(gphi)
        gq = gq + k_e * pg
        gx = gx - k_e * (gphi[t][:, None] * fq + qt[:, None] * fg)
    if gF is not None:
        hw, ew = force_weight_sums(x, q, _f64(gF).reshape(n, 3), box, periodic, eps=eps,
                                   targets=t)
        gq = gq + k_e * ew
        gx = gx - k_e * qt[:, None] * hw
    st = site[t]
    insite = st >= 0
    lam_i = np.where(insite, np.append(lam, 0.0)[np.where(insite, st, lam.size)], 0.0)
    gqA = (1.0 - lam_i) * gq
    gqB = lam_i * gq
    if np.count_nonzero(insite) != np.count_nonzero(site >= 0):
        return gx, gqA, gqB, None
    glam = np.zeros(lam.size)
    for s in range(lam.size):
        m = st == s
        glam[s] = np.sum((qB[t][m] - qA[t][m]) * gq[m])
    return gx, gqA, gqB, glam


def hamiltonian_correction(x, qA, qB, site, lam, box=None, periodic=False, k_e=1.0, eps=1e-13):
    """Hamiltonian minus charge interpolation (Methods, eq 1).

    The Coulomb energy is a quadratic form E(q) = 1/2 q^T Psi q (Psi: the pair
    potential, with the self-image term on the diagonal for periodic cells).
    Mixing a site's two end states linearly, (1 - l) E(a) + l E(b), exceeds
    E((1 - l) a + l b) by l (1 - l) 1/2 (a - b)^T Psi (a - b) for the site's
    own block of Psi; every cross-site term is bilinear and agrees.  Per site
    this is the energy of the charges d = qA - qB placed on the site's atoms
    alone, which the direct or Ewald sum gives.  Returns (dE, dF, d dE/dlambda)."""
    x = _f64(x).reshape(-1, 3)
    qA, qB, lam = _f64(qA), _f64(qB), _f64(np.atleast_1d(lam))
    site = np.asarray(site)
    dE, dF, dD = 0.0, np.zeros_like(x), np.zeros(lam.size)
    for s in range(lam.size):
        idx = np.nonzero(site == s)[0]
        if idx.size == 0:
            continue
        d = qA[idx] - qB[idx]
        if periodic:
            ph, fd = ewald(x[idx], d, box, eps=eps)
        else:
            ph, fd = direct(x[idx], d)
        e = 0.5 * float(np.dot(d, ph))
        w = lam[s] * (1.0 - lam[s])
        dE += k_e * w * e
        dD[s] = k_e * (1.0 - 2.0 * lam[s]) * e
        dF[idx] += k_e * w * d[:, None] * fd
    return dE, dF, dD


def tautomer_charges(qA, qB, qC, qD, site, lam_p, lam_t):
    """eq 2 in charge-interpolated form: q = lp~ (lt~ qA + lt qB) + lp (lt~ qC + lt qD)."""
    qA, qB, qC, qD = _f64(qA), _f64(qB), _f64(qC), _f64(qD)
    lam_p, lam_t = _f64(np.atleast_1d(lam_p)), _f64(np.atleast_1d(lam_t))
    if lam_p.size != lam_t.size:
        raise ValueError("lambda_p and lambda_t must have one value per site")
    site = np.ascontiguousarray(site, dtype=np.int32)
    q = np.empty_like(qA)
    rc = _load().orc_tautomer_charges(qA.size, qA, qB, qC, qD, site, lam_p.size, lam_p, lam_t, q)
    if rc != 0:
        raise ValueError("site index outside [-1, n_sites)")
    return q


def solve_tautomer(x, qA, qB, qC, qD, site, lam_p, lam_t, box=None, periodic=False, k_e=1.0,
                   eps=1e-13, ewald_kw=None):
    """Full four-form oracle solve (Methods, eq 2).  Returns dict(E, F, phi,
    dVdl_p, dVdl_t, q), all FP64; phi includes k_e."""
    lam_p, lam_t = _f64(np.atleast_1d(lam_p)), _f64(np.atleast_1d(lam_t))
    q = tautomer_charges(qA, qB, qC, qD, site, lam_p, lam_t)
    if periodic:
        phi, field = ewald(x, q, box, eps=eps, **(ewald_kw or {}))
    else:
        phi, field = direct(x, q)
    site = np.ascontiguousarray(site, dtype=np.int32)
    # E and F from the generic outputs (their site sums are not used here)
    E, F, _ = outputs(q, q, q, site, lam_p.size, phi, field, k_e)
    dp = np.empty(lam_p.size)
    dt = np.empty(lam_p.size)
    rc = _load().orc_tautomer_dvdl(q.size, _f64(qA), _f64(qB), _f64(qC), _f64(qD), site,
                                   lam_p.size, lam_p, lam_t, _f64(phi), float(k_e), dp, dt)
    if rc != 0:
        raise ValueError("site index outside [-1, n_sites)")
    return {"E": E, "F": F, "phi": k_e * phi, "dVdl_p": dp, "dVdl_t": dt, "q": q}
