"""Autotuner for the tree depth and the two launch-shape knobs of a plan.

* ``m2l_chunk``: translation offsets handled per matrix-core M2L work-group
  (fewer offsets per group = more groups in flight, more partial sums).
* ``p2p_waves``: wavefronts per leaf in the near-field kernel (4, 8 or 16).

The two knobs act on different phases, so each is tuned on its own phase time,
measured with HIP events on the plan's stream (fmm_profile).  ``tune_depth``
first picks the depth from candidate depths by whole-evaluation time, then
tunes the two knobs at that depth.  Results are cached in a JSON file keyed by
GPU architecture and problem shape.
"""
from __future__ import annotations

import json
import os

CHUNKS = [1, 3, 7, 14, 27, 63, 189]
WAVES = [4, 8, 16]
DEFAULT_CACHE = os.environ.get(
    "FMMCPH_TUNE_CACHE",
    os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json"))


def _key(arch, n, depth, order, periodic, precision, replicas):
    nb = 1 << max(0, int(n - 1).bit_length())  # atoms rounded up to a power of two
    return "%s|n%d|d%d|p%d|%s|%s|R%d" % (arch, nb, depth, order,
                                         "pbc" if periodic else "open", precision, replicas)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _phase_mean(plan, run, steps):
    run()
    import torch
    torch.cuda.synchronize(plan.device)
    plan.profile_start(steps)
    for _ in range(steps):
        run()
    plan.profile_stop()
    prof = plan.profile_read()
    return {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()}


def tune(make_run, depth, order, periodic, precision, n_atoms, replicas=1, steps=5,
         cache=DEFAULT_CACHE, device=None, verbose=False):
    """Pick (m2l_chunk, p2p_waves).

    make_run(plan) -> a zero-argument callable that enqueues one evaluation
    (or one batched evaluation) on `plan`.  Returns a dict with the choice and
    the measured phase times; the choice is cached.
    """
    import torch

    from . import fmm
    dev = torch.device(device) if device is not None else torch.device("cuda", 0)
    arch = torch.cuda.get_device_properties(dev).gcnArchName.split(":")[0]
    key = _key(arch, n_atoms, depth, order, periodic, precision, replicas)
    db = _load(cache)
    if key in db:
        return db[key]
    base = dict(periodic=periodic, precision=precision, max_atoms=n_atoms,
                max_sites=make_run.max_sites, max_replicas=replicas, device=dev)
    chunk_t = {}
    for c in CHUNKS:
        plan = fmm.Plan(depth, order, m2l_chunk=c, **base)
        if plan.m2l_kernel_mode() == 0:
            break  # plain M2L: the chunk knob does not apply
        chunk_t[c] = _phase_mean(plan, make_run(plan), steps)["m2l"]
        plan.close()
        if verbose:
            print("m2l_chunk %3d: %.1f us" % (c, 1e3 * chunk_t[c]), flush=True)
    wave_t = {}
    for w in WAVES:
        plan = fmm.Plan(depth, order, p2p_waves=w, **base)
        wave_t[w] = _phase_mean(plan, make_run(plan), steps)["near_far"]
        plan.close()
        if verbose:
            print("p2p_waves %2d: %.1f us" % (w, 1e3 * wave_t[w]), flush=True)
    res = {"m2l_chunk": min(chunk_t, key=chunk_t.get) if chunk_t else 0,
           "p2p_waves": min(wave_t, key=wave_t.get),
           "m2l_ms": {str(k): v for k, v in chunk_t.items()},
           "near_far_ms": {str(k): v for k, v in wave_t.items()}}
    db = _load(cache)
    db[key] = res
    try:
        with open(cache + ".tmp", "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(cache + ".tmp", cache)
    except OSError:
        pass
    return res


def _eval_time(plan, run, steps):
    """Seconds per evaluation (wall clock, stream synchronised) after a warm-up."""
    import time

    import torch
    run()
    torch.cuda.synchronize(plan.device)
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize(plan.device)
    return (time.perf_counter() - t0) / steps


def tune_depth(make_run, depths, order, periodic, precision, n_atoms, replicas=1, steps=5,
               cache=DEFAULT_CACHE, device=None, verbose=False):
    """Pick the tree depth among `depths` by whole-evaluation time (default
    launch shapes), then the launch shapes at that depth (tune).  The depth
    trades near-field pairs (fewer at a deeper tree) against translations and
    tree passes (more).  Returns tune()'s dict with "depth" and the measured
    "depth_ms" added; cached like tune()."""
    import torch

    from . import fmm
    dev = torch.device(device) if device is not None else torch.device("cuda", 0)
    arch = torch.cuda.get_device_properties(dev).gcnArchName.split(":")[0]
    key = _key(arch, n_atoms, -1, order, periodic, precision, replicas) + "|depths" + ",".join(
        str(d) for d in depths)
    db = _load(cache)
    if key in db:
        return db[key]
    base = dict(periodic=periodic, precision=precision, max_atoms=n_atoms,
                max_sites=make_run.max_sites, max_replicas=replicas, device=dev)
    depth_t = {}
    for d in depths:
        plan = fmm.Plan(d, order, **base)
        depth_t[d] = _eval_time(plan, make_run(plan), steps)
        plan.close()
        if verbose:
            print("depth %d: %.1f us" % (d, 1e6 * depth_t[d]), flush=True)
    best = min(depth_t, key=depth_t.get)
    res = dict(tune(make_run, best, order, periodic, precision, n_atoms, replicas, steps, cache,
                    device, verbose))
    res["depth"] = best
    res["depth_ms"] = {str(k): 1e3 * v for k, v in depth_t.items()}
    db = _load(cache)
    db[key] = res
    try:
        with open(cache + ".tmp", "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(cache + ".tmp", cache)
    except OSError:
        pass
    return res
