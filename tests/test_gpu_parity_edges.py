"""Edge cases of the periodic wrap and the mixed-precision error budget, each
compared with the FP64 oracle element by element."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL_F, assert_within, cached_reference, errors, reference, run
from paper_2410_01626_amd import workloads as W

pytestmark = pytest.mark.gpu


def _on_grid(d, q=2.0 ** -12, face=2.0 ** -7):
    """The periodic workload with every coordinate rounded to a multiple of q
    (so that adding whole cells stays exact in FP32 and the library's FP64
    wrap gives the coordinate back exactly), and coordinates within `face` of
    the lower face put on it (0.0).  Returns the copy and the (atom, axis)
    pairs put on the face."""
    L = float(d["box"][0])
    assert np.float32(L) == L and (L / q) == int(L / q), "the cell edge must sit on the grid"
    x = np.round(d["x"] / q) * q
    x[x >= L] -= L
    near = np.argwhere(x < face)
    x[x < face] = 0.0
    d2 = dict(d)
    d2["x"] = x
    return d2, near


def _shifted(d, near, seed):
    """Every atom moved by whole cells per axis (-2, -1, 0, +1 or +2 edges:
    negative coordinates and values past L and 2L); half of the face atoms go
    to exactly x = L, the others stay at 0."""
    L = float(d["box"][0])
    rng = np.random.default_rng(seed)
    n = d["x"].shape[0]
    shift = rng.choice([-2, -1, 0, 0, 0, 1, 2], size=(n, 3)).astype(np.float64)
    for k, (i, a) in enumerate(near):
        shift[i, a] = 1.0 if k % 2 == 0 else 0.0
    x = d["x"] + L * shift
    assert np.array_equal(x.astype(np.float32).astype(np.float64), x), "shifts must be exact"
    d2 = dict(d)
    d2["x"] = x
    return d2


def _check_wrap(d, near, seed, prec):
    d2 = _shifted(d, near, seed)
    x = d2["x"]
    L = float(d["box"][0])
    assert (x < 0).any() and (x >= 2 * L).any()
    if len(near):
        assert (x == L).any() and (x == 0.0).any()
    a = run(d, prec)
    b = run(d2, prec)
    # the FP64 wrap returns every coordinate exactly: the same evaluation bit for bit
    for k in ("F", "phi", "dVdl"):
        np.testing.assert_array_equal(b[k], a[k])
    assert b["E"] == a["E"]
    ref = reference(d2)
    err_a, err_b = errors(a, reference(d)), errors(b, ref)
    print("wrap %s: shifted %s, unshifted %s" % (prec, err_b, err_a))
    assert_within(err_b, 8, label="shifted " + prec)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_periodic_positions_outside_cell_tiny(prec):
    """Periodic inputs are wrapped into [0, L) in FP64: negative coordinates,
    coordinates exactly L, and shifts by +-L and +-2L give the same evaluation
    as the coordinates inside the cell (bit for bit) and the oracle's answer
    for the shifted positions."""
    d, near = _on_grid(W.tiny_periodic(21, n=400, edge=1.5, n_sites=4, depth=2, order=8))
    assert len(near) >= 4, "the case needs atoms on the faces"
    _check_wrap(d, near, 1, prec)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_periodic_positions_outside_cell_water_box(prec):
    """The 30,000-atom water box in a 6.75 nm cell (6.7 is not on the FP32
    grid; no atom lies within the face band) with its atoms moved by whole
    cells (|shift| <= 2 L per axis) and wrapped back by the library."""
    d, _ = cached_reference("water_box")
    d = dict(d)
    d["box"] = np.full(3, 6.75)
    d, near = _on_grid(d)
    _check_wrap(d, near, 2, prec)


# ---------------------------------------------------------------- error budget

_WATER = {}


def _water_errors():
    """Errors of the three plans on the 30,000-atom water box against the full
    Ewald oracle (computed once)."""
    if not _WATER:
        d, ref = cached_reference("water_box")
        for prec in ("fp64", "f32", "bf16x3"):
            _WATER[prec] = errors(run(d, prec), ref)
    return _WATER


@pytest.mark.parametrize("prec", ["fp64", "f32", "bf16x3"])
def test_water_box_full_size(prec):
    """30,000-atom periodic water box at depth 3, p = 8: every output element
    against the full Ewald oracle."""
    err = _water_errors()[prec]
    print("water_box %s errors %s" % (prec, err))
    assert_within(err, 8, label="water_box " + prec)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_mixed_precision_within_twice_fp64_error(prec):
    """The mixed-precision plans stay within twice the FP64 FMM's own error at
    p = 8 in every output (forces, potentials, energy, dV/dlambda).  The FP64
    plan's error is the truncation error of the expansions; the mixed plans
    add rounding of FP32 pair sums and of the bf16 three-product split."""
    e = _water_errors()
    em, e64 = e[prec], e["fp64"]
    print("%s / fp64 error ratios: %s" % (prec, {k: em[k] / e64[k] for k in em}))
    for k in ("F", "phi", "E", "dVdl"):
        assert em[k] <= 2.0 * e64[k], (k, em[k], e64[k])


def test_fp64_error_decays_with_order_on_water_box_sample():
    """The FP64 FMM's error on the water box falls geometrically with p (a
    floor would mean a convention mismatch), measured on 400 sampled atoms."""
    d, _ = cached_reference("water_box")
    rng = np.random.default_rng(3)
    samp = np.sort(rng.choice(d["x"].shape[0], 400, replace=False))
    q = oracle.lambda_charges(d["qA"], d["qB"], d["site"], d["lam"])
    phi, field = oracle.ewald(d["x"], q, d["box"], eps=1e-12, targets=samp)
    F = q[samp, None] * field
    errs = []
    for p in (4, 6, 8, 10):
        out = run(d, "fp64", order=p)
        eF = np.sqrt(np.sum((out["F"][samp] - F) ** 2) / np.sum(F ** 2))
        errs.append(eF)
        assert eF <= TOL_F[p], (p, eF)
    print("water box FP64 force error vs p (4, 6, 8, 10): %s" % errs)
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:])), errs
