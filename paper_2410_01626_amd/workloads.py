"""Seeded synthetic inputs for the lambda-interpolated Coulomb solve.

This module only draws inputs (positions, the two charge forms, site
membership, lambda values, box).  It holds none of the method's arithmetic:
both the oracle and the HIP path consume what it returns, and it imports
neither of them.

Every floating-point value it returns is representable in FP32, so the FP64
and the mixed-precision paths see bit-identical inputs.

Recipes (the paper's own systems are proteins in water; none of their
structures ship here, so these stand in for them with the same shapes,
densities, charge scales and site structure):

* ``open_cube`` (1,000 atoms, open):  uniform in a 3 nm cube, minimum distance
  0.1 nm; 10 sites of 4 spatially nearest atoms with qA ~ U(-1, 1) and
  qB = qA + Delta, Delta = sigma * w, w ~ Dirichlet(1,1,1,1), sigma = +-1 (each
  site changes its net charge by one unit, as titratable residues do); every
  other atom +-1 alternating in index order (net zero); lambda ~ U(0, 1).
* ``water_box`` (30,000 atoms, periodic 6.7 nm): 9,000 three-site waters
  (O -0.834 e, H +0.417 e, O-H 0.096 nm, H-O-H 104.52 deg, random orientation)
  on a jittered 22^3 lattice outside a 3,000-atom compact cluster (uniform in
  a sphere of radius 1.93 nm, minimum distance 0.1 nm, q ~ N(0, 0.3) shifted to
  zero mean); 20 sites, each a cluster atom and its 3 nearest cluster
  neighbours, qA = their cluster charges, qB = qA + Delta as above.
* ``replicas`` (16 open systems, 10k-60k atoms): atoms on a jittered cubic
  lattice at 100 atoms/nm^3 (minimum distance 0.1 nm), +-1 alternating; one
  4-atom site per 100 atoms; replica r at pH 2 + 7 r / 15 draws lambda near 1
  (deprotonated) with probability 1 / (10^(pKa - pH) + 1), pKa = 4.0, else near
  0, |lambda - end| ~ U(0, 0.1).
* ``large_box`` (500,000 atoms, periodic 17 nm): 160,000 waters around a
  20,000-atom cluster (radius 3.63 nm), 200 sites.

``with_tautomers(d)`` adds four-form sites (protonation tautomers) to any of
these: forms A = qA and C = qB of the workload (the two protonation states),
B = A + tau and D = C + tau' with tau, tau' moving charge between the site's
atoms without changing its net charge (tau = 0.5 (w - 1/size), w ~
Dirichlet(1,...,1)), on every other site; the remaining sites have no
tautomers (B = A, D = C).  lambda_t ~ U(0, 1) per site.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 2410016260
WATER_Q_O = -0.834
WATER_Q_H = 0.417
WATER_OH = 0.096
WATER_HOH_DEG = 104.52

__all__ = [
    "open_cube", "water_box", "replicas", "large_box", "tiny_periodic",
    "random_open", "by_name", "CONFIGS", "with_tautomers",
]


def _f32(a):
    """Round to FP32-representable values, returned as FP64."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _rsa(n, draw, dmin, rng, lo, hi, existing=None, max_tries=200):
    """Random sequential addition with a minimum distance (cell-hash check).

    draw(rng, k) -> k candidate points; points must lie in [lo, hi)^3.
    """
    cell = dmin
    grid = {}
    pts = []

    def key(p):
        return tuple(((p - lo) // cell).astype(np.int64))

    def ok(p):
        k = key(p)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for q in grid.get((k[0] + dx, k[1] + dy, k[2] + dz), ()):
                        d = p - q
                        if d @ d < dmin * dmin:
                            return False
        return True

    if existing is not None:
        for p in existing:
            grid.setdefault(key(p), []).append(p)
    tries = 0
    while len(pts) < n:
        cand = draw(rng, max(64, 2 * (n - len(pts))))
        for p in cand:
            if ok(p):
                grid.setdefault(key(p), []).append(p)
                pts.append(p)
                if len(pts) == n:
                    break
        tries += 1
        if tries > max_tries:
            raise RuntimeError("rsa: density too high for the minimum distance")
    return np.array(pts)


def _site_deltas(rng, n_sites, size=4):
    """Delta = sigma * w with w ~ Dirichlet(1,...,1) and sigma = +-1 per site."""
    w = rng.dirichlet(np.ones(size), size=n_sites)
    sigma = rng.choice([-1.0, 1.0], size=n_sites)
    return w * sigma[:, None], sigma


def _pick_sites(rng, pos, pool, n_sites, size=4):
    """Each site: a random atom of `pool` plus its size-1 nearest pool atoms
    not already taken.  Returns an (n_sites, size) array of atom indices."""
    pool = np.asarray(pool)
    taken = np.zeros(pos.shape[0], dtype=bool)
    order = rng.permutation(pool)
    sites = []
    it = iter(order)
    while len(sites) < n_sites:
        c = next(it)
        if taken[c]:
            continue
        cand = pool[~taken[pool]]
        d = np.sum((pos[cand] - pos[c]) ** 2, axis=1)
        sel = cand[np.argsort(d, kind="stable")[:size]]
        if sel.size < size:
            continue
        taken[sel] = True
        sites.append(sel)
    return np.array(sites, dtype=np.int64)


def _water(rng, centres):
    """Three-site waters with O at `centres`, random orientation."""
    m = centres.shape[0]
    half = math.radians(WATER_HOH_DEG) / 2
    # random rotation per molecule from a random unit quaternion
    qv = rng.normal(size=(m, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    R = np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], 1)
    h1 = np.array([math.sin(half), 0.0, math.cos(half)]) * WATER_OH
    h2 = np.array([-math.sin(half), 0.0, math.cos(half)]) * WATER_OH
    H1 = centres + R @ h1
    H2 = centres + R @ h2
    pos = np.stack([centres, H1, H2], 1).reshape(-1, 3)
    q = np.tile([WATER_Q_O, WATER_Q_H, WATER_Q_H], m)
    return pos, q


def _finish(name, x, qA, qB, site, lam, box, periodic, depth, order, **extra):
    d = {
        "name": name,
        "x": _f32(x),
        "qA": _f32(qA),
        "qB": _f32(qB),
        "site": np.ascontiguousarray(site, dtype=np.int32),
        "lam": np.ascontiguousarray(lam, dtype=np.float64),
        "box": None if box is None else np.array(box, dtype=np.float64),
        "periodic": bool(periodic),
        "depth": int(depth),
        "order": int(order),
    }
    d.update(extra)
    return d


def open_cube(seed=SEED_BASE + 1, n=1000, n_sites=10, edge=3.0, depth=2, order=6):
    """1,000 atoms uniform in a 3 nm cube, open boundaries, 10 four-atom sites."""
    rng = np.random.default_rng(seed)
    x = _rsa(n, lambda r, k: r.uniform(0, edge, (k, 3)), 0.1, rng, 0.0, edge)
    sites = _pick_sites(rng, x, np.arange(n), n_sites)
    site = np.full(n, -1, dtype=np.int32)
    qA = np.empty(n)
    qB = np.empty(n)
    delta, _ = _site_deltas(rng, n_sites)
    for s, idx in enumerate(sites):
        site[idx] = s
        qA[idx] = rng.uniform(-1, 1, size=idx.size)
        qB[idx] = qA[idx] + delta[s]
    rest = np.flatnonzero(site < 0)
    qA[rest] = np.where(np.arange(rest.size) % 2 == 0, 1.0, -1.0)
    qB[rest] = qA[rest]
    lam = rng.uniform(0, 1, n_sites)
    return _finish("open_cube", x, qA, qB, site, lam, None, False, depth, order,
                   edge=edge)


def _solvated(seed, edge, n_water, n_cluster, r_cluster, n_sites, lattice_n,
              depth, order, name, buffers=False):
    rng = np.random.default_rng(seed)
    c = np.full(3, edge / 2)

    def in_sphere(r, k):
        v = r.normal(size=(k, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        rad = r_cluster * r.uniform(0, 1, k) ** (1 / 3)
        return c + v * rad[:, None]

    cl = _rsa(n_cluster, in_sphere, 0.1, rng, 0.0, edge)
    qc = rng.normal(0, 0.3, n_cluster)
    qc -= qc.mean()
    h = edge / lattice_n
    g = (np.arange(lattice_n) + 0.5) * h
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    jit = 0.15 * (h - 0.25) if h > 0.25 else 0.0
    lat = lat + rng.uniform(-jit, jit, lat.shape)
    outside = np.linalg.norm(lat - c, axis=1) > r_cluster + 0.15
    lat = lat[outside]
    if lat.shape[0] < n_water:
        raise RuntimeError("not enough lattice sites for the waters")
    lat = lat[np.sort(rng.choice(lat.shape[0], n_water, replace=False))]
    xw, qw = _water(rng, lat)
    x = np.concatenate([xw, cl])
    x = np.mod(x, edge)
    qA = np.concatenate([qw, qc])
    n = x.shape[0]
    off = xw.shape[0]
    sites = _pick_sites(rng, cl, np.arange(n_cluster), n_sites) + off
    site = np.full(n, -1, dtype=np.int32)
    qB = qA.copy()
    delta, sigma = _site_deltas(rng, n_sites)
    for s, idx in enumerate(sites):
        site[idx] = s
        qB[idx] = qA[idx] + delta[s]
    if buffers:
        # one water oxygen per site takes the opposite charge change
        # (a charge-buffer site keeps the pair's total charge constant)
        oxy = rng.choice(n_water, n_sites, replace=False) * 3
        for s in range(n_sites):
            site[oxy[s]] = s
            qB[oxy[s]] = qA[oxy[s]] - sigma[s]
    lam = rng.uniform(0, 1, n_sites)
    return _finish(name, x, qA, qB, site, lam, [edge] * 3, True, depth, order,
                   n_water=n_water, n_cluster=n_cluster)


def water_box(seed=SEED_BASE + 2, buffers=False, depth=3, order=8):
    """30,000 atoms: 9,000 waters + a 3,000-atom cluster, periodic 6.7 nm cube."""
    return _solvated(seed, 6.7, 9000, 3000, 1.93, 20, 22, depth, order,
                     "water_box", buffers)


def small_water_box(seed=SEED_BASE + 7, depth=2, order=6):
    """2,300 atoms: 700 waters + a 200-atom cluster, periodic 3 nm cube, 4 sites
    (the water box recipe at a size the oracle finishes in seconds)."""
    return _solvated(seed, 3.0, 700, 200, 0.9, 4, 10, depth, order, "small_water_box")


def with_sites(d, n_sites, seed=SEED_BASE + 8, max_cluster_sites=500):
    """The same solvated box with its titratable sites redrawn: n_sites sites,
    the first min(n_sites, max_cluster_sites) of four nearest cluster atoms
    (as in the water box recipe), the rest whole water molecules (three-atom
    sites, in molecule order); qB = qA + sigma w per site (w ~ Dirichlet,
    sigma = +-1), lambda ~ U(0, 1).  Positions and qA are unchanged, so only
    the site bookkeeping differs between the boxes of a site-count sweep."""
    rng = np.random.default_rng(seed)
    x, qA = d["x"], d["qA"]
    n = x.shape[0]
    n_water, n_cluster = d["n_water"], d["n_cluster"]
    off = 3 * n_water
    site = np.full(n, -1, dtype=np.int32)
    qB = qA.astype(np.float64).copy()
    n_cl = min(n_sites, max_cluster_sites)
    n_w = n_sites - n_cl
    if n_w > n_water:
        raise ValueError("more sites than the box can hold")
    groups = []
    if n_cl:
        groups += list(_pick_sites(rng, x[off:off + n_cluster], np.arange(n_cluster), n_cl) + off)
    for k in range(n_w):
        groups.append(np.arange(3 * k, 3 * k + 3))
    for s, idx in enumerate(groups):
        w = rng.dirichlet(np.ones(idx.size))
        site[idx] = s
        qB[idx] = qA[idx] + rng.choice([-1.0, 1.0]) * w
    lam = rng.uniform(0, 1, n_sites)
    return _finish(d["name"] + "_S%d" % n_sites, x, qA, qB, site, lam, d["box"], d["periodic"],
                   d["depth"], d["order"], n_water=n_water, n_cluster=n_cluster)


def water_exclusions(n_water, n_atoms):
    """Per-atom excluded partners of the first n_water three-atom waters (each
    atom excludes the other two atoms of its molecule); the other atoms have
    none.  Returns (start, idx) as int32 arrays."""
    start = np.zeros(n_atoms + 1, dtype=np.int32)
    idx = []
    for i in range(n_atoms):
        if i < 3 * n_water:
            m = 3 * (i // 3)
            idx += [j for j in (m, m + 1, m + 2) if j != i]
        start[i + 1] = len(idx)
    return start, np.array(idx, dtype=np.int32)


def large_box(seed=SEED_BASE + 5, depth=5, order=10):
    """500,000 atoms: 160,000 waters + a 20,000-atom cluster, periodic 17 nm."""
    return _solvated(seed, 17.0, 160000, 20000, 3.63, 200, 56, depth, order,
                     "large_box")


def _lattice_open(rng, n, density=100.0):
    edge = (n / density) ** (1 / 3)
    m = int(math.ceil(n ** (1 / 3)))
    a = edge / m
    g = (np.arange(m) + 0.5) * a
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    lat = lat[np.sort(rng.choice(lat.shape[0], n, replace=False))]
    jit = max(0.0, (a - 0.1) / 2) * 0.999
    return lat + rng.uniform(-jit, jit, lat.shape), edge


def replicas(seed=SEED_BASE + 4, n_rep=16, pka=4.0, depth=3, order=8,
             sizes=None):
    """16 open systems of 10k-60k atoms, each at its own pH and lambda vector."""
    rng = np.random.default_rng(seed)
    out = []
    if sizes is None:
        sizes = [10000 + (50000 * r) // max(n_rep - 1, 1) for r in range(n_rep)]
    for r, n in enumerate(sizes):
        x, edge = _lattice_open(rng, n)
        n_sites = max(1, n // 100)
        sites = _pick_sites(rng, x, np.arange(n), n_sites) if n_sites * 4 <= n else None
        site = np.full(n, -1, dtype=np.int32)
        qA = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
        qB = qA.copy()
        delta, _ = _site_deltas(rng, n_sites)
        for s, idx in enumerate(sites):
            site[idx] = s
            qA[idx] = rng.uniform(-1, 1, size=idx.size)
            qB[idx] = qA[idx] + delta[s]
        ph = 2.0 + 7.0 * r / max(n_rep - 1, 1)
        frac = 1.0 / (10.0 ** (pka - ph) + 1.0)
        near_one = rng.uniform(0, 1, n_sites) < frac
        dev = rng.uniform(0, 0.1, n_sites)
        lam = np.where(near_one, 1.0 - dev, dev)
        out.append(_finish("replica%d" % r, x, qA, qB, site, lam, None, False,
                           depth, order, pH=ph, edge=edge))
    return out


def tiny_periodic(seed, n=64, edge=1.0, n_sites=2, neutral=True, depth=1, order=8):
    """Small periodic box for quick parity: uniform atoms, 4-atom sites."""
    rng = np.random.default_rng(seed)
    dmin = min(0.1, 0.5 * edge / max(n, 1) ** (1 / 3))
    x = _rsa(n, lambda r, k: r.uniform(0, edge, (k, 3)), dmin, rng, 0.0, edge)
    qA = rng.uniform(-1, 1, n)
    if neutral:
        qA -= qA.mean()
    site = np.full(n, -1, dtype=np.int32)
    qB = qA.copy()
    if n_sites:
        sites = _pick_sites(rng, x, np.arange(n), n_sites)
        delta, _ = _site_deltas(rng, n_sites)
        for s, idx in enumerate(sites):
            site[idx] = s
            qB[idx] = qA[idx] + delta[s]
    lam = rng.uniform(0, 1, n_sites)
    return _finish("tiny_periodic", x, qA, qB, site, lam, [edge] * 3, True, depth,
                   order)


def random_open(seed, n=200, edge=2.0, n_sites=3, depth=2, order=6):
    """Small open system for quick parity: uniform atoms, 4-atom sites."""
    d = tiny_periodic(seed, n=n, edge=edge, n_sites=n_sites, neutral=False,
                      depth=depth, order=order)
    d.update(name="random_open", box=None, periodic=False, edge=edge)
    return d


CONFIGS = {
    "open_cube": open_cube,
    "water_box": water_box,
    "replicas": replicas,
    "large_box": large_box,
}


def by_name(name, **kw):
    return CONFIGS[name](**kw)


def with_tautomers(d, seed=SEED_BASE + 7):
    """A copy of workload `d` with four charge forms per site (qA, qB, qC, qD)
    and a second coordinate lam_t per site; the workload's lam becomes lam_p."""
    rng = np.random.default_rng(seed)
    qA = d["qA"].astype(np.float64)
    qC = d["qB"].astype(np.float64)
    qB = qA.copy()
    qD = qC.copy()
    site = d["site"]
    S = int(d["lam"].size)
    for s in range(0, S, 2):  # every other site has tautomers
        idx = np.nonzero(site == s)[0]
        if idx.size < 2:
            continue
        w1 = rng.dirichlet(np.ones(idx.size))
        w2 = rng.dirichlet(np.ones(idx.size))
        qB[idx] = qA[idx] + 0.5 * (w1 - 1.0 / idx.size)
        qD[idx] = qC[idx] + 0.5 * (w2 - 1.0 / idx.size)
    out = dict(d)
    out.update(name=d["name"] + "_tautomers", qA=_f32(qA), qB=_f32(qB), qC=_f32(qC), qD=_f32(qD),
               lam_p=np.ascontiguousarray(d["lam"], dtype=np.float64),
               lam_t=np.ascontiguousarray(rng.uniform(0.0, 1.0, S), dtype=np.float64))
    return out
