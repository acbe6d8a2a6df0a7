"""GPU parity of the HIP path against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest

from gpu_util import TOL_F, assert_within, errors, reference, run
from paper_2410_01626_amd import workloads as W

pytestmark = pytest.mark.gpu


# ---------------------------------------------------------------- exact limits

@pytest.mark.parametrize("depth", [0, 1])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("f32", 2e-6)])
def test_open_shallow_tree_is_direct_sum(depth, prec, tol):
    """Open boundaries with depth 0 or 1 have no interaction lists: the FMM is
    the direct sum (every pair is near), up to rounding."""
    d = W.open_cube()
    out = run(d, prec, depth=depth)
    err = errors(out, reference(d))
    assert max(err.values()) <= tol, err


# ---------------------------------------------------------------- open boundaries

@pytest.mark.parametrize("prec", ["fp64", "f32", "bf16x3"])
def test_open_cube(prec):
    d = W.open_cube()
    out = run(d, prec)
    err = errors(out, reference(d))
    assert_within(err, d["order"], label="open_cube " + prec)


def test_open_error_decays_with_order():
    d = W.open_cube()
    ref = reference(d)
    errs = []
    for p in (2, 4, 6, 8, 10, 12):
        e = errors(run(d, "fp64", order=p), ref)
        assert_within(e, p, label="open p")
        errs.append(e["F"])
    # geometric decay, no floor above 1e-7 (a floor would mean a convention mismatch)
    assert errs[-1] < 1e-5 and all(b < a for a, b in zip(errs, errs[1:])), errs


@pytest.mark.parametrize("depth", [2, 3, 4])
def test_open_depths(depth):
    d = W.random_open(11, n=1500, edge=2.5, depth=depth, order=8)
    err = errors(run(d, "fp64"), reference(d))
    assert_within(err, 8, label="open depth %d" % depth)


# ---------------------------------------------------------------- periodic

@pytest.mark.parametrize("depth", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", ["fp64", "f32", "bf16x3"])
def test_periodic_small(depth, prec):
    d = W.tiny_periodic(21, n=400, edge=1.6, n_sites=4, depth=depth, order=8)
    err = errors(run(d, prec), reference(d))
    assert_within(err, 8, label="periodic depth %d %s" % (depth, prec))


@pytest.mark.parametrize("prec", ["fp64", "f32"])
def test_periodic_non_neutral_gauge(prec):
    """Net charge: background and zero-mean gauge must match Ewald; a constant
    offset in phi would move dV/dlambda by offset * sum(Delta)."""
    d = W.tiny_periodic(22, n=300, edge=1.3, n_sites=3, neutral=False, depth=2, order=8)
    assert abs(d["qA"].sum()) > 0.5
    ref = reference(d)
    out = run(d, prec)
    err = errors(out, ref)
    assert_within(err, 8, label="non-neutral " + prec)
    assert abs(np.mean(out["phi"] - ref["phi"])) < TOL_F[8] * np.sqrt(np.mean(ref["phi"] ** 2))


def test_periodic_error_decays_with_order():
    d = W.tiny_periodic(23, n=300, edge=1.0, n_sites=2, depth=1, order=4)
    ref = reference(d)
    errs = []
    for p in (4, 6, 8, 10, 12, 14):
        e = errors(run(d, "fp64", order=p), ref)
        assert_within(e, p, label="periodic p")
        errs.append(e["F"])
    assert errs[-1] < 2e-6 and all(b < a for a, b in zip(errs, errs[1:])), errs


# ---------------------------------------------------------------- invariants and edge cases

def test_lambda_derivative_is_derivative_of_fmm_energy():
    """E_fmm is exactly quadratic in lambda; with symmetric translation operators
    its central difference equals the returned dV/dlambda to rounding."""
    d = W.tiny_periodic(24, n=200, edge=1.2, n_sites=3, depth=2, order=6)
    base = run(d, "fp64")
    h = 1e-3
    for s in range(d["lam"].size):
        lp = d["lam"].copy(); lp[s] += h
        lm = d["lam"].copy(); lm[s] -= h
        fd = (run(d, "fp64", lam=lp)["E"] - run(d, "fp64", lam=lm)["E"]) / (2 * h)
        assert abs(fd - base["dVdl"][s]) <= 1e-9 * max(1.0, abs(base["E"])), (s, fd, base["dVdl"][s])


@pytest.mark.parametrize("prec", ["fp64", "f32"])
def test_deterministic(prec):
    d = W.random_open(12, n=2000, edge=3.0, depth=3, order=6)
    a, b = run(d, prec), run(d, prec)
    assert a["E"] == b["E"]
    np.testing.assert_array_equal(a["F"], b["F"])
    np.testing.assert_array_equal(a["phi"], b["phi"])
    np.testing.assert_array_equal(a["dVdl"], b["dVdl"])


def test_lambda_outside_unit_interval_not_clamped():
    d = W.open_cube()
    lam = np.linspace(-0.1, 1.1, d["lam"].size)
    err = errors(run(d, "fp64", lam=lam), reference(d, lam=lam))
    assert_within(err, d["order"], label="lambda range")


def test_coulomb_constant_scaling():
    d = W.open_cube()
    a = run(d, "fp64")
    b = run(d, "fp64", k_e=138.935458)
    assert b["E"] == pytest.approx(138.935458 * a["E"], rel=1e-13)
    np.testing.assert_allclose(b["F"], 138.935458 * a["F"], rtol=1e-12, atol=1e-12 * np.abs(b["F"]).max())


@pytest.mark.parametrize("depth", [1, 2])
def test_no_sites_and_tiny_systems(depth):
    """One, two and seven atoms without sites.  Depth 1 is the direct sum; at
    depth 2 far pairs go through the expansions (order 12 here)."""
    for n in (1, 2, 7):
        d = W.random_open(13, n=n, edge=1.0, n_sites=0, depth=depth, order=12)
        out = run(d, "fp64")
        ref = reference(d)
        tol = 1e-12 if depth == 1 else 3e-5
        assert out["E"] == pytest.approx(ref["E"], rel=tol, abs=1e-14)
        np.testing.assert_allclose(out["F"], ref["F"], rtol=tol, atol=tol * np.abs(ref["F"]).max())
        assert out["dVdl"].size == 0


def test_all_atoms_in_one_leaf_region():
    """A dense clump: most leaves empty, one leaf crowded (ragged binning)."""
    rng = np.random.default_rng(5)
    d = W.random_open(14, n=600, edge=2.0, depth=3, order=8)
    x = d["x"].copy()
    x[:500] = 0.05 + rng.uniform(0, 0.1, (500, 3))
    d["x"] = x.astype(np.float32).astype(np.float64)
    err = errors(run(d, "fp64"), reference(d))
    assert_within(err, 8, label="clump")


def test_axis_permutation_symmetry():
    d = W.tiny_periodic(25, n=250, edge=1.1, n_sites=2, depth=2, order=6)
    a = run(d, "fp64")
    d2 = dict(d)
    d2["x"] = d["x"][:, [1, 2, 0]].copy()
    b = run(d2, "fp64")
    assert b["E"] == pytest.approx(a["E"], rel=1e-12)
    np.testing.assert_allclose(b["F"], a["F"][:, [1, 2, 0]], rtol=1e-9, atol=1e-9 * np.abs(a["F"]).max())


def test_check_mode_reports_bad_input():
    from paper_2410_01626_amd import fmm
    d = W.random_open(15, n=100, edge=1.0, n_sites=2, depth=2, order=4)
    d["site"] = d["site"].copy()
    d["site"][3] = 7
    with pytest.raises(fmm.FmmError) as e:
        run(d, "fp64", check=True)
    assert e.value.status == fmm.FMM_E_SITE
    d = W.random_open(15, n=100, edge=1.0, n_sites=2, depth=2, order=4)
    d["qA"] = d["qA"].copy()
    d["qA"][5] = np.nan
    with pytest.raises(fmm.FmmError) as e:
        run(d, "fp64", check=True)
    assert e.value.status == fmm.FMM_E_NONFINITE


@pytest.mark.parametrize("periodic", [False, True])
def test_check_mode_reports_coincident_atoms(periodic):
    """Two atoms at one position (periodic: an atom and another one whole cell
    away, which the wrap puts on the same point) are flagged in check mode;
    valid inputs, with one or several near-field blocks per leaf, are not."""
    from paper_2410_01626_amd import fmm
    if periodic:
        d = W.tiny_periodic(16, n=300, edge=1.5, n_sites=2, depth=2, order=4)
    else:
        d = W.random_open(16, n=300, edge=1.5, n_sites=2, depth=2, order=4)
    for split in (1, 3):
        run(d, "fp64", check=True, p2p_split=split)  # no flag
        run(d, "f32", check=True, p2p_split=split)
    x = d["x"].copy()
    x[123] = np.round(x[123] * 4096) / 4096  # on a grid where +-L stays exact in FP32
    x[7] = x[123] + (np.array([1.5, 0.0, -1.5]) if periodic else 0.0)
    d2 = dict(d)
    d2["x"] = x
    for prec in ("fp64", "f32"):
        with pytest.raises(fmm.FmmError) as e:
            run(d2, prec, check=True, p2p_split=2)
        assert e.value.status == fmm.FMM_E_COINCIDENT


# ---------------------------------------------------------------- matrix-core M2L

@pytest.mark.parametrize("prec", ["fp64", "f32", "bf16x3"])
@pytest.mark.parametrize("periodic", [False, True])
def test_matrix_core_m2l_matches_plain(prec, periodic):
    """The matrix-core M2L (FP64 / FP32 / bf16 three-product) and the plain
    vector-ALU M2L compute the same translations; compare complete outputs.
    FP64: equal to 1e-12.  FP32: both paths carry the rounding of sums of 189 K
    products per local coefficient (in different orders), so each is measured
    against the FP64 plain solve: the matrix-core path may differ from it by at
    most 1.5 times what the FP32 plain path does.  bf16x3: the split keeps
    Th mh + Th ml + Tl mh and drops Tl ml; with 8-bit hi parts and bf16-rounded
    lo parts each product is off by at most about 2^-16 of |T| |mu|.  Summed,
    that is 2^-16 of the potential the charges' magnitudes |q| would give
    without sign cancellation; relative to the actual potential it is 2^-16
    kappa, kappa = RMS phi(|q|) / RMS phi (phi(|q|): the open-boundary FP64
    solve of the same positions with |q|, an upper estimate of the terms'
    size).  The bound is the FP32 plain path's error plus that (forces: plus
    2^-16 times the same ratio for the field)."""
    if periodic:
        d = W.tiny_periodic(31, n=3000, edge=2.4, n_sites=4, depth=3, order=8)
    else:
        d = W.random_open(32, n=3000, edge=2.4, n_sites=4, depth=3, order=8)

    def rel(u, v, k):
        return np.sqrt(np.sum((u[k] - v[k]) ** 2) / np.sum(v[k] ** 2))
    if prec == "fp64":
        a = run(d, "fp64", m2l_kernel=1)
        b = run(d, "fp64", m2l_kernel=2)
        assert rel(b, a, "F") <= 1e-12 and rel(b, a, "phi") <= 1e-12
        return
    r = run(d, "fp64", m2l_kernel=1)
    a = run(d, "f32", m2l_kernel=1)
    b = run(d, prec, m2l_kernel=2)
    ea = {k: rel(a, r, k) for k in ("F", "phi")}
    eb = {k: rel(b, r, k) for k in ("F", "phi")}
    print("%s periodic=%s: plain-FP32 vs FP64 %s, matrix-core vs FP64 %s"
          % (prec, periodic, ea, eb))
    kappa = {"F": 1.0, "phi": 1.0}
    if prec == "bf16x3":
        da = dict(d)
        da["periodic"] = False
        da["qA"], da["qB"] = np.abs(d["qA"]), np.abs(d["qA"])
        ab = run(da, "fp64", depth=1)
        kappa = {k: np.sqrt(np.mean(ab[k] ** 2) / np.mean(r[k] ** 2)) for k in ("F", "phi")}
        print("cancellation ratios", kappa)
    for k in ("F", "phi"):
        bound = 1.5 * ea[k] + 1e-7 if prec == "f32" else ea[k] + 2.0 ** -16 * kappa[k]
        assert eb[k] <= bound, (k, eb[k], ea[k], bound)


@pytest.mark.parametrize("order", [2, 4, 6, 10])
def test_matrix_core_m2l_orders(order):
    d = W.tiny_periodic(33, n=1500, edge=2.0, n_sites=3, depth=2, order=order)
    ref = reference(d)
    for prec in ("f32", "bf16x3"):
        assert_within(errors(run(d, prec, m2l_kernel=2), ref), order, label=prec)


@pytest.mark.parametrize("chunk", [1, 7, 50, 189])
def test_m2l_offset_chunking_invariant(chunk):
    """Splitting the 189 offsets over work-groups only regroups a fixed-order sum."""
    d = W.tiny_periodic(34, n=2000, edge=2.0, n_sites=3, depth=3, order=6)
    a = run(d, "fp64", m2l_kernel=2, m2l_chunk=189)
    b = run(d, "fp64", m2l_kernel=2, m2l_chunk=chunk)
    np.testing.assert_allclose(b["phi"], a["phi"], rtol=1e-12, atol=1e-12 * np.abs(a["phi"]).max())
    np.testing.assert_allclose(b["F"], a["F"], rtol=1e-11, atol=1e-11 * np.abs(a["F"]).max())


@pytest.mark.parametrize("periodic", [False, True])
def test_bf16x3_resident_source_chunking(periodic):
    """Trees of at most 73 target columns per class run the bf16x3 M2L with
    the class's sources resident and chunks cut within parity groups.  Every
    chunk size (1 to 26 offsets: 189 to 8 partial sums per coefficient) keeps
    the bound of the matrix-core test above against the FP64 plain solve: the
    FP32 plain path's error plus 2^-16 kappa (kappa: the cancellation ratio
    RMS phi(|q|) / RMS phi); against the oracle, the default chunking stays
    within twice the FP64 FMM's own error on the same input."""
    mk = W.tiny_periodic if periodic else W.random_open
    d = mk(38, n=2500, edge=2.2, n_sites=3, depth=3, order=8)

    def rel(u, v, k):
        return np.sqrt(np.sum((u[k] - v[k]) ** 2) / np.sum(v[k] ** 2))
    r = run(d, "fp64", m2l_kernel=1)
    a = run(d, "f32", m2l_kernel=1)
    da = dict(d)
    da["periodic"] = False
    da["qA"], da["qB"] = np.abs(d["qA"]), np.abs(d["qA"])
    ab = run(da, "fp64", depth=1)
    kappa = {k: np.sqrt(np.mean(ab[k] ** 2) / np.mean(r[k] ** 2)) for k in ("F", "phi")}
    for chunk in (1, 7, 13, 26):
        b = run(d, "bf16x3", m2l_chunk=chunk)
        for k in ("F", "phi"):
            bound = rel(a, r, k) + 2.0 ** -16 * kappa[k]
            assert rel(b, r, k) <= bound, (chunk, k, rel(b, r, k), bound)
    ref = reference(d)
    e64, eb = errors(r, ref), errors(run(d, "bf16x3"), ref)
    for k in ("F", "phi", "E", "dVdl"):
        assert eb[k] <= 2.0 * e64[k] + 1e-9, (k, eb[k], e64[k])


@pytest.mark.parametrize("periodic", [False, True])
def test_bf16x3_deep_tree(periodic):
    """Depth 4 (512 leaf columns per class): the bf16x3 M2L that stages
    every column's source per offset."""
    mk = W.tiny_periodic if periodic else W.random_open
    d = mk(39, n=6000, edge=2.6, n_sites=4, depth=4, order=8)
    assert_within(errors(run(d, "bf16x3"), reference(d)), 8, label="bf16x3 depth 4")


@pytest.mark.parametrize("waves", [4, 16])
def test_near_field_wave_count_invariant(waves):
    """4, 8 or 16 wavefronts per leaf only regroup the near-field sums."""
    d = W.tiny_periodic(35, n=2500, edge=2.0, n_sites=3, depth=3, order=6)
    a = run(d, "fp64", p2p_waves=8)
    b = run(d, "fp64", p2p_waves=waves)
    np.testing.assert_allclose(b["phi"], a["phi"], rtol=1e-12, atol=1e-12 * np.abs(a["phi"]).max())
    np.testing.assert_allclose(b["F"], a["F"], rtol=1e-11, atol=1e-11 * np.abs(a["F"]).max())


@pytest.mark.parametrize("waves,split", [(4, 2), (4, 4), (8, 3), (16, 4)])
def test_near_field_split_invariant(waves, split):
    """Several near-field blocks per leaf (targets in windows of 32) only regroup
    the near-field sums; leaves here hold 60-92 atoms, so windows of every kind
    (full, remainder, empty) occur."""
    d = W.tiny_periodic(37, n=5000, edge=2.0, n_sites=3, depth=2, order=6)
    a = run(d, "fp64", p2p_waves=8, p2p_split=1)
    b = run(d, "fp64", p2p_waves=waves, p2p_split=split)
    np.testing.assert_allclose(b["phi"], a["phi"], rtol=1e-12, atol=1e-12 * np.abs(a["phi"]).max())
    np.testing.assert_allclose(b["F"], a["F"], rtol=1e-11, atol=1e-11 * np.abs(a["F"]).max())
    assert abs(b["E"] - a["E"]) <= 1e-12 * abs(a["E"])
    np.testing.assert_allclose(b["dVdl"], a["dVdl"], rtol=1e-12, atol=1e-12 * np.abs(a["dVdl"]).max())


def test_autotuner_picks_valid_shapes(tmp_path):
    import torch
    from paper_2410_01626_amd import autotune, fmm
    dev = torch.device("cuda:0")
    d = W.tiny_periodic(36, n=4000, edge=2.2, n_sites=3, depth=3, order=6)
    t = [torch.tensor(d[k], dtype=torch.float32, device=dev) for k in ("x", "qA", "qB")]
    site = torch.tensor(d["site"], device=dev)
    lam = torch.tensor(d["lam"], device=dev)

    def make_run(plan):
        return lambda: plan.eval(t[0], t[1], t[2], site, lam, box=d["box"])
    make_run.max_sites = 3
    cache = str(tmp_path / "tune.json")
    res = autotune.tune(make_run, 3, 6, True, "bf16x3", 4000, cache=cache, steps=2)
    assert res["m2l_chunk"] in autotune.CHUNKS and res["p2p_waves"] in autotune.WAVES
    assert autotune.tune(make_run, 3, 6, True, "bf16x3", 4000, cache=cache) == res  # cached
    plan = fmm.Plan(3, 6, periodic=True, precision="bf16x3", max_atoms=4000, max_sites=3,
                    device=dev, m2l_chunk=res["m2l_chunk"], p2p_waves=res["p2p_waves"])
    info = plan.info()
    assert info["m2l_chunk"] == res["m2l_chunk"] and info["p2p_waves"] == res["p2p_waves"]
