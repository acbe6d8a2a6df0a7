"""Input generators: determinism, shapes and the stated recipe invariants."""
import numpy as np

from paper_2410_01626_amd import workloads as W


def _check(d, n, n_sites):
    assert d["x"].shape == (n, 3)
    for k in ("x", "qA", "qB"):
        assert d[k].dtype == np.float64
        assert np.array_equal(d[k], d[k].astype(np.float32).astype(np.float64))
    assert d["site"].dtype == np.int32
    assert d["site"].min() >= -1 and d["site"].max() == n_sites - 1
    assert d["lam"].shape == (n_sites,)
    # atoms outside sites have identical forms
    free = d["site"] < 0
    assert np.array_equal(d["qA"][free], d["qB"][free])
    # each site changes its net charge by exactly one unit (up to FP32 rounding)
    for s in range(n_sites):
        dq = (d["qB"] - d["qA"])[d["site"] == s].sum()
        assert abs(abs(dq) - 1.0) < 1e-6 or d.get("buffers")


def test_open_cube_recipe():
    d = W.open_cube()
    _check(d, 1000, 10)
    assert np.all(np.bincount(d["site"][d["site"] >= 0]) == 4)
    assert d["x"].min() >= 0 and d["x"].max() < 3.0
    diff = d["x"][:, None] - d["x"][None]
    r = np.sqrt((diff ** 2).sum(-1)) + np.eye(1000) * 9
    assert r.min() >= 0.1 - 1e-6
    rest = d["qA"][d["site"] < 0]
    assert rest.sum() == 0 and set(rest) == {1.0, -1.0}
    assert np.array_equal(W.open_cube()["x"], d["x"])  # seeded


def test_water_box_recipe():
    d = W.water_box()
    _check(d, 30000, 20)
    assert d["periodic"] and np.all(d["box"] == 6.7)
    assert d["x"].min() >= 0 and d["x"].max() < 6.7
    qw = d["qA"][:27000].reshape(-1, 3)
    assert np.allclose(qw, [-0.834, 0.417, 0.417], atol=1e-7)
    oh = np.linalg.norm(d["x"][1:27000:3] - d["x"][0:27000:3], axis=1)
    oh = np.minimum(oh, np.linalg.norm(((d["x"][1:27000:3] - d["x"][0:27000:3] + 3.35) % 6.7) - 3.35, axis=1))
    assert np.allclose(oh, 0.096, atol=1e-6)
    assert abs(d["qA"].sum()) < 1e-4  # neutral at lambda = 0 (FP32 rounding only)


def test_replicas_recipe():
    reps = W.replicas(sizes=[2000, 3000])
    assert len(reps) == 2
    for d in reps:
        n = d["x"].shape[0]
        _check(d, n, n // 100)
        assert np.all((d["lam"] < 0.1) | (d["lam"] > 0.9))


def test_buffers_keep_total_charge():
    d = W.water_box(buffers=True)
    for s in range(20):
        m = d["site"] == s
        assert m.sum() == 5
        assert abs((d["qB"] - d["qA"])[m].sum()) < 1e-6


def test_site_count_sweep_boxes():
    """with_sites keeps positions and qA and draws the requested number of
    sites: four-atom cluster sites first, then whole waters, each changing
    its charge by +-1 in total."""
    d = W.water_box()
    for S in (0, 20, 200, 2000):
        e = W.with_sites(d, S)
        assert e["lam"].size == S
        np.testing.assert_array_equal(e["x"], d["x"])
        np.testing.assert_array_equal(e["qA"], d["qA"])
        assert set(np.unique(e["site"])) <= set(range(-1, S))
        for s in range(S):
            m = e["site"] == s
            assert m.sum() in (3, 4)
            assert abs(abs(float(np.sum(e["qB"][m].astype(np.float64) - e["qA"][m]))) - 1.0) < 1e-6
        assert np.all(e["qB"][e["site"] < 0] == e["qA"][e["site"] < 0])
