#!/usr/bin/env python
"""Throughput of the lambda-interpolated FMM Coulomb solve on one MI355X.

One step = one evaluation of E, F, phi and dV/dlambda (every kernel of the hot
path: binning, P2M, M2M, lattice operator, M2L, L2L, P2P + L2P, reductions) for
the 30,000-atom periodic water box (6.7 nm cube, depth 3, p = 8), with inputs
already resident in device memory.  The mixed-precision plan is the measured
value; the FP64 plan is timed beside it.  The FP64 CPU oracle (Ewald) is timed
on the host for one full evaluation of the same system.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks
    "fp32_vector": 157.3e12, "fp64_vector": 78.6e12, "fp32_mfma": 157.3e12,
    "fp64_mfma": 78.6e12, "bf16_mfma": 2.5e15, "hbm": 8.0e12,
}


def leaf_counts(x, box, depth):
    """Atoms per leaf cell, binned exactly as the library bins them."""
    nb = 1 << depth
    h = box / nb
    w = x - box * np.floor(x / box)
    c = np.clip(np.floor(w / h).astype(np.int64), 0, nb - 1)
    cnt = np.zeros((nb, nb, nb), dtype=np.int64)
    np.add.at(cnt, (c[:, 0], c[:, 1], c[:, 2]), 1)
    return cnt


def p2p_pairs(cnt, periodic=True):
    """Directed near-field pairs: every target with every source of the 27
    neighbour leaves (periodic images included), minus the i = j terms."""
    tot = np.zeros_like(cnt)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                tot += np.roll(cnt, shift=(dx, dy, dz), axis=(0, 1, 2))
    return int(np.sum(cnt * tot) - cnt.sum())


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_water_box_30k_p8.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2410_01626_amd", "csrc", "fmm_kernels.hip")
PHASE_KERNEL = {"near_far": "k_near_far<float, 8>", "m2l": "k_m2l_bf16x3_rs<6>"}


def measured_traffic(phase):
    """HBM bytes per launch of the phase's kernel from the committed FETCH_SIZE /
    WRITE_SIZE summary, or None when there is none or the kernel source has
    changed since the counters were taken (hash recorded in the summary)."""
    import hashlib
    import re
    name = PHASE_KERNEL.get(phase)
    if name is None or not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m = re.search(r"^source_sha256 = ([0-9a-f]{64})$", text, re.M)
    if not m or m.group(1) != hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest():
        return None
    m = re.search(r"^traffic\[%s\] = (\d+)$" % re.escape(name), text, re.M)
    return int(m.group(1)) if m else None


def eval_bytes(n, S, depth, order, ts=4):
    """Algorithmic HBM bytes of one evaluation outside the near-field and M2L
    arithmetic: inputs read once (x, qA, qB, site: 24 B per atom), outputs
    written once (F, phi: 16 B), the sorted particle array written and read
    (2 x 16 B) with its permutation (2 x 4 B) and leaf keys (2 x 4 B), every
    box's multipole and local expansion written and read (4 x Kp x 4 B) with
    its bf16 hi/lo split (2 x 2 Kp x 2 B), the bf16 hi/lo operators of the 189
    canonical translations read once (189 x 2 Kp' x K x 2 B, Kp' = K rounded to
    32), and the sites' lambda and dV/dlambda."""
    K = (order + 1) ** 2
    Kp = (K + 3) // 4 * 4
    Kb = (K + 31) // 32 * 32
    nbox = sum(8 ** l for l in range(depth + 1))
    per_atom = 24 + 16 + 32 + 8 + 8
    boxes = nbox * (4 * Kp * ts + 2 * 2 * Kp * 2)
    bank = 189 * 2 * Kb * K * 2
    return n * per_atom + boxes + bank + 16 * S


def m2l_translations(depth, periodic=True):
    lmin = 1 if periodic else 2
    return sum(189 * 8 ** l for l in range(lmin, depth + 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--fp64-steps", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the replica-batch leg")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--no-large", action="store_true", help="skip the 500,000-atom leg")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy (3 times): the reference for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(64 * 1024 * 1024, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * a.numel(), "copies": 3}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver runs on a single device and this "
              "build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2410_01626_amd import fmm, workloads

    dev = torch.device("cuda", 0)
    d = workloads.water_box()
    n, S = d["x"].shape[0], d["lam"].size
    box = float(d["box"][0])
    depth, order = d["depth"], d["order"]
    K = (order + 1) ** 2

    def make(prec):
        plan = fmm.Plan(depth, order, periodic=True, precision=prec, max_atoms=n,
                        max_sites=S, device=dev)
        dt = plan.dtype
        inp = (torch.tensor(d["x"], dtype=dt, device=dev),
               torch.tensor(d["qA"], dtype=dt, device=dev),
               torch.tensor(d["qB"], dtype=dt, device=dev),
               torch.tensor(d["site"], dtype=torch.int32, device=dev),
               torch.tensor(d["lam"], dtype=torch.float64, device=dev))
        return plan, inp

    def breakdown(plan, inp, n=20):
        """Per-phase mean ms from an untimed pass with events at every phase
        boundary (each event costs GPU time, so this pass is not the timed one)."""
        plan.profile_select(None, 1)
        plan.profile_start(n)
        for _ in range(n):
            plan.eval(*inp, box=d["box"])
        plan.profile_stop()
        prof = plan.profile_read()
        return {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()}

    def timed(plan, inp, steps, warmup, roof_phase=None, every=20):
        """Seconds per evaluation over `steps` timed evaluations; with roof_phase,
        HIP events on the plan's stream around that phase on every `every`-th
        timed evaluation give its mean duration (ms) inside the timed region."""
        for _ in range(warmup):
            plan.eval(*inp, box=d["box"])
        torch.cuda.synchronize(dev)
        if roof_phase:
            plan.profile_select([roof_phase], every)
            plan.profile_start(steps)
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.eval(*inp, box=d["box"])
        torch.cuda.synchronize(dev)
        t1 = time.perf_counter()
        dur = None
        if roof_phase:
            plan.profile_stop()
            tot, cnt = plan.profile_read()[roof_phase]
            dur = tot / cnt if cnt else None
        return (t1 - t0) / steps, dur

    plan, inp = make("bf16x3")
    for _ in range(args.warmup):
        plan.eval(*inp, box=d["box"])
    phase_ms = breakdown(plan, inp)
    dom = max(phase_ms, key=phase_ms.get)
    sec, dom_ms = timed(plan, inp, args.steps, args.warmup, roof_phase=dom)
    # four more timed runs of the same K steps (no events): spread and median of five
    rep = [sec] + [timed(plan, inp, args.steps, 0)[0] for _ in range(4)]
    plan32, inp32 = make("f32")
    sec32, _ = timed(plan32, inp32, args.fp64_steps, max(2, args.warmup // 4))
    phase_ms32 = breakdown(plan32, inp32)
    plan64, inp64 = make("fp64")
    sec64, _ = timed(plan64, inp64, args.fp64_steps, max(2, args.warmup // 4))
    phase_ms64 = breakdown(plan64, inp64)

    # graph replay of the same evaluation (dedicated stream, fixed output buffers)
    gstream = torch.cuda.Stream(dev)
    gplan = fmm.Plan(depth, order, periodic=True, precision="bf16x3", max_atoms=n, max_sites=S,
                     device=dev, stream=gstream, graph=True)
    gout = {"E": torch.empty(1, dtype=torch.float64, device=dev),
            "F": torch.empty((n, 3), dtype=torch.float32, device=dev),
            "phi": torch.empty(n, dtype=torch.float32, device=dev),
            "dVdl": torch.empty(S, dtype=torch.float64, device=dev)}
    torch.cuda.synchronize(dev)
    with torch.cuda.stream(gstream):
        for _ in range(args.warmup):
            gplan.eval(*inp, box=d["box"], out=gout)
        gstream.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            gplan.eval(*inp, box=d["box"], out=gout)
        gstream.synchronize()
        t1 = time.perf_counter()
    sec_graph = (t1 - t0) / args.steps

    # the same box with four charge forms on every site (protonation tautomers,
    # two lambda coordinates per site): fmm_eval_tautomer
    dt4 = workloads.with_tautomers(d)
    tplan = fmm.Plan(depth, order, periodic=True, precision="bf16x3", max_atoms=n, max_sites=S,
                     device=dev)
    t4 = (torch.tensor(dt4["x"], dtype=torch.float32, device=dev),
          *(torch.tensor(dt4[k], dtype=torch.float32, device=dev) for k in ("qA", "qB", "qC", "qD")),
          torch.tensor(dt4["site"], dtype=torch.int32, device=dev),
          torch.tensor(dt4["lam_p"], dtype=torch.float64, device=dev),
          torch.tensor(dt4["lam_t"], dtype=torch.float64, device=dev))
    for _ in range(args.warmup):
        tplan.eval_tautomer(*t4, box=d["box"])
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tplan.eval_tautomer(*t4, box=d["box"])
    torch.cuda.synchronize(dev)
    t1 = time.perf_counter()
    sec_taut = (t1 - t0) / args.steps

    # the same box under Hamiltonian interpolation (eq 1 taken literally: the
    # intra-site correction is added to E, F and dV/dlambda)
    hplan = fmm.Plan(depth, order, periodic=True, precision="bf16x3", max_atoms=n, max_sites=S,
                     device=dev, hamiltonian=True)
    sec_ham, _ = timed(hplan, inp, args.steps, args.warmup)

    # the same box with the intramolecular pairs of its 9,000 waters excluded
    xplan = fmm.Plan(depth, order, periodic=True, precision="bf16x3", max_atoms=n, max_sites=S,
                     device=dev)
    xplan.set_exclusions(*workloads.water_exclusions(9000, n))
    sec_excl, _ = timed(xplan, inp, args.steps, args.warmup)

    # constant-pH dynamics of the same box: every step one solve (kJ/mol) and
    # one velocity-Verlet step of the 20 lambda particles (bias V_pH + V_dw,
    # Bussi thermostat; pKa_ref 4.0 at pH 4.0)
    from paper_2410_01626_amd import lambda_dynamics as LD
    lplan = fmm.Plan(depth, order, periodic=True, precision="bf16x3", coulomb_k=138.935458,
                     max_atoms=n, max_sites=S, device=dev)
    # V_MM from a synthetic calibration: each site alone in vacuum is its
    # reference compound, whose dV/dlambda is linear in lambda (the Coulomb
    # energy is quadratic in the charges), so two solves at lambda = 0 and 1
    # (all sites as replicas of one batched call) give G = g_00 + g_10 lambda
    mm = np.zeros((S, 36))
    members = [np.nonzero(d["site"] == s_)[0] for s_ in range(S)]
    cao = np.cumsum([0] + [m_.size for m_ in members])
    cso = np.arange(S + 1)
    idx = np.concatenate(members)
    cplan = fmm.Plan(1, 8, periodic=False, precision="fp64", coulomb_k=138.935458,
                     max_atoms=int(cao[-1]), max_sites=S, max_replicas=S, device=dev)
    cin = [torch.tensor(d[k][idx], dtype=torch.float64, device=dev) for k in ("x", "qA", "qB")]
    csite = torch.zeros(int(cao[-1]), dtype=torch.int32, device=dev)
    g_end = [cplan.eval_batched(cao, cso, *cin, csite, torch.full((S,), float(e), dtype=torch.float64,
                                                                   device=dev))["dVdl"].cpu().numpy()
             for e in (0.0, 1.0)]
    mm[:, 0], mm[:, 6] = g_end[0], g_end[1] - g_end[0]
    dyn = LD.LambdaDynamics([0, S], d["lam"], [4.0], np.full(S, 4.0), mm=mm, seed=1, device=dev)
    lout = lplan.eval(inp[0], inp[1], inp[2], inp[3], dyn.lam, box=d["box"])

    def md_steps(k):
        for _ in range(k):
            lplan.eval(inp[0], inp[1], inp[2], inp[3], dyn.lam, box=d["box"], out=lout)
            dyn.step(lout["dVdl"])

    md_steps(args.warmup)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    md_steps(args.steps)
    torch.cuda.synchronize(dev)
    sec_md = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dyn.step(lout["dVdl"])
    torch.cuda.synchronize(dev)
    sec_lstep = (time.perf_counter() - t0) / args.steps
    lam_dyn = {"workload": "same box, 20 lambda particles (m = 60 u, dt = 2 fs, 300 K, Bussi "
                           "tau = 1 ps, barrier 6 kJ/mol, V_MM from each isolated site), k_e in "
                           "kJ/mol",
               "md_steps_per_s": 1.0 / sec_md, "ms_per_step": sec_md * 1e3,
               "lambda_step_us": sec_lstep * 1e6,
               "lambda_range": [float(dyn.lam.min().item()), float(dyn.lam.max().item())],
               "end_state_fraction": float(((dyn.lam < 0.2) | (dyn.lam > 0.8)).double().mean().item())}

    # 16 open replicas of 10k-60k atoms at pH 2-9 in one batched call per step
    batched = None
    if not args.no_batched:
        reps = workloads.replicas()
        ao = np.cumsum([0] + [r["x"].shape[0] for r in reps])
        so = np.cumsum([0] + [r["lam"].size for r in reps])
        cat = {k: np.concatenate([r[k] for r in reps]) for k in ("x", "qA", "qB", "site", "lam")}
        bplan = fmm.Plan(3, 8, periodic=False, precision="bf16x3", max_atoms=int(ao[-1]),
                         max_sites=int(so[-1]), max_replicas=len(reps), device=dev)
        bin_ = (torch.tensor(cat["x"], dtype=torch.float32, device=dev),
                torch.tensor(cat["qA"], dtype=torch.float32, device=dev),
                torch.tensor(cat["qB"], dtype=torch.float32, device=dev),
                torch.tensor(cat["site"], dtype=torch.int32, device=dev),
                torch.tensor(cat["lam"], dtype=torch.float64, device=dev))
        for _ in range(2):
            bplan.eval_batched(ao, so, *bin_)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(args.batched_steps):
            bplan.eval_batched(ao, so, *bin_)
        torch.cuda.synchronize(dev)
        t1 = time.perf_counter()
        bsec = (t1 - t0) / args.batched_steps
        # phase breakdown from a separate pass (events at every phase boundary)
        bplan.profile_start(3)
        for _ in range(3):
            bplan.eval_batched(ao, so, *bin_)
        bplan.profile_stop()
        bprof = bplan.profile_read()
        # the same batch with the depth and launch shapes picked by the
        # autotuner (depth 3 or 4), replayed from a HIP graph
        from paper_2410_01626_amd import autotune

        def make_run(pl):
            return lambda: pl.eval_batched(ao, so, *bin_)
        make_run.max_sites = int(so[-1])
        tune_res = autotune.tune_depth(make_run, (3, 4), 8, False, "bf16x3", int(ao[-1]),
                                       replicas=len(reps), steps=3, device=dev)
        gs_ = torch.cuda.Stream(dev)
        tplan = fmm.Plan(tune_res["depth"], 8, periodic=False, precision="bf16x3",
                         max_atoms=int(ao[-1]), max_sites=int(so[-1]), max_replicas=len(reps),
                         device=dev, stream=gs_, graph=True, m2l_chunk=tune_res["m2l_chunk"],
                         p2p_waves=tune_res["p2p_waves"])
        nb_ = int(ao[-1])
        tout = {"E": torch.empty(len(reps), dtype=torch.float64, device=dev),
                "F": torch.empty((nb_, 3), dtype=torch.float32, device=dev),
                "phi": torch.empty(nb_, dtype=torch.float32, device=dev),
                "dVdl": torch.empty(int(so[-1]), dtype=torch.float64, device=dev)}
        torch.cuda.synchronize(dev)
        with torch.cuda.stream(gs_):
            for _ in range(2):
                tplan.eval_batched(ao, so, *bin_, out=tout)
            gs_.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.batched_steps):
                tplan.eval_batched(ao, so, *bin_, out=tout)
            gs_.synchronize()
            tsec = (time.perf_counter() - t0) / args.batched_steps
        tuned = {"depth": tune_res["depth"], "m2l_chunk": tune_res["m2l_chunk"],
                 "p2p_waves": tune_res["p2p_waves"], "depth_ms": tune_res.get("depth_ms"),
                 "graph_replay": True, "batch_evals_per_s": 1.0 / tsec,
                 "replica_evals_per_s": len(reps) / tsec, "ms_per_batch": tsec * 1e3}
        tplan.close()
        batched = {"workload": "16 open replicas, 10,000-60,000 atoms (%d total), depth 3, p = 8, "
                               "pH 2-9" % int(ao[-1]),
                   "tuned": tuned,
                   "batch_evals_per_s": 1.0 / bsec, "replica_evals_per_s": len(reps) / bsec,
                   "ms_per_batch": bsec * 1e3, "atoms_per_s": float(ao[-1]) / bsec,
                   "phase_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in bprof.items()}}
        # constant-pH dynamics of the replicas: one batched solve (kJ/mol) and
        # one lambda step of all replicas' sites per step, each replica at its pH
        bplan_k = fmm.Plan(3, 8, periodic=False, precision="bf16x3", coulomb_k=138.935458,
                           max_atoms=int(ao[-1]), max_sites=int(so[-1]), max_replicas=len(reps),
                           device=dev)
        bdyn = LD.LambdaDynamics(so, cat["lam"], [r["pH"] for r in reps], np.full(int(so[-1]), 4.0),
                                 seed=2, device=dev)
        for _ in range(2):
            bout = bplan_k.eval_batched(ao, so, bin_[0], bin_[1], bin_[2], bin_[3], bdyn.lam)
            bdyn.step(bout["dVdl"])
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(args.batched_steps):
            bout = bplan_k.eval_batched(ao, so, bin_[0], bin_[1], bin_[2], bin_[3], bdyn.lam)
            bdyn.step(bout["dVdl"])
        torch.cuda.synchronize(dev)
        bmd = (time.perf_counter() - t0) / args.batched_steps
        batched["lambda_dynamics"] = {"md_steps_per_s": 1.0 / bmd, "ms_per_step": bmd * 1e3,
                                      "lambda_particles": int(so[-1])}

    def wall(fn, steps, warm=3):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize(dev)
        return (time.perf_counter() - t0) / steps

    # site-count sweep on the same box (the paper: the cost of the charge
    # interpolation does not grow with the number of titratable sites)
    sweep = {}
    for S_ in (0, 20, 200, 2000):
        ds = workloads.with_sites(d, S_)
        splan = fmm.Plan(depth, order, periodic=True, precision="bf16x3", max_atoms=n,
                         max_sites=max(S_, 1), device=dev)
        sin = (inp[0], inp[1], torch.tensor(ds["qB"], dtype=torch.float32, device=dev),
               torch.tensor(ds["site"], dtype=torch.int32, device=dev),
               torch.tensor(ds["lam"], dtype=torch.float64, device=dev))
        tS = wall(lambda: splan.eval(*sin, box=d["box"]), args.steps, args.warmup)
        sweep[str(S_)] = {"evals_per_s": 1.0 / tS, "ms_per_step": tS * 1e3,
                          "site_atoms": int((ds["site"] >= 0).sum())}
        splan.close()

    # forward + backward at the 30k shape (FP32 positions and charges, upstream
    # weight on E): fmm_eval then fmm_eval_adjoint (tree rebuilt in backward);
    # and the one-pass adjoint with weights on E, phi and F
    gE1 = torch.ones(1, dtype=torch.float64, device=dev)
    rng_ = np.random.default_rng(5)
    gphi_ = torch.tensor(rng_.normal(0, 1, n), dtype=torch.float32, device=dev)
    gF_ = torch.tensor(rng_.normal(0, 1, (n, 3)), dtype=torch.float32, device=dev)

    def fwd_bwd():
        plan.eval(*inp, box=d["box"])
        plan.eval_adjoint(*inp, gE1, box=d["box"])

    t_fb = wall(fwd_bwd, args.steps // 2)
    t_full = wall(lambda: plan.eval_adjoint_full(*inp, gE=gE1, gphi=gphi_, gF=gF_, box=d["box"]),
                  args.steps // 2)
    diff = {"workload": "same box, forward (fmm_eval) + backward (fmm_eval_adjoint, weight on E)",
            "fwd_bwd_per_s": 1.0 / t_fb, "ms_per_fwd_bwd": t_fb * 1e3,
            "adjoint_full_per_s": 1.0 / t_full, "ms_per_adjoint_full": t_full * 1e3,
            "adjoint_full": "fmm_eval_adjoint_full, weights on E, phi and F (one tree pass, "
                            "second sources in expansion slot 1)"}

    # the 500,000-atom periodic box (17 nm, depth 5, p = 10): forward and
    # forward + adjoint
    large = None
    if not args.no_large:
        dl = workloads.large_box()
        nl_, Sl_ = dl["x"].shape[0], dl["lam"].size
        lplan5 = fmm.Plan(dl["depth"], dl["order"], periodic=True, precision="bf16x3",
                          max_atoms=nl_, max_sites=Sl_, device=dev)
        lin = (torch.tensor(dl["x"], dtype=torch.float32, device=dev),
               torch.tensor(dl["qA"], dtype=torch.float32, device=dev),
               torch.tensor(dl["qB"], dtype=torch.float32, device=dev),
               torch.tensor(dl["site"], dtype=torch.int32, device=dev),
               torch.tensor(dl["lam"], dtype=torch.float64, device=dev))
        t_l = wall(lambda: lplan5.eval(*lin, box=dl["box"]), 10)
        t_la = wall(lambda: lplan5.eval_adjoint(*lin, gE1, box=dl["box"]), 10)
        lplan5.profile_start(3)
        for _ in range(3):
            lplan5.eval(*lin, box=dl["box"])
        lplan5.profile_stop()
        lprof = lplan5.profile_read()
        large = {"workload": "large_box: 500,000 atoms (160,000 waters + 20,000-atom cluster), "
                             "periodic 17 nm, 200 sites, depth 5, p = 10, bf16x3 M2L",
                 "evals_per_s": 1.0 / t_l, "ms_per_eval": t_l * 1e3,
                 "fwd_adjoint_per_s": 1.0 / t_la, "ms_per_fwd_adjoint": t_la * 1e3,
                 "atoms_per_s": nl_ / t_l,
                 "phase_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in lprof.items()}}
        lplan5.close()

    # the dominant kernel's work over its duration measured inside the timed region
    pairs = p2p_pairs(leaf_counts(d["x"], box, depth))
    n_m2l = m2l_translations(depth)
    # the headline plan runs M2L as bf16 matrix-core products (three per
    # translation); the algorithmic work is the dense FP32 product 2 K^2
    work = {"near_far": (20.0 * pairs, "alu", PEAK["fp32_vector"], "TFLOP/s"),
            "m2l": (2.0 * K * K * n_m2l, "mfma", PEAK["bf16_mfma"], "TFLOP/s")}
    if dom in work:
        flops, bound, peak, unit = work[dom]
        achieved = flops / (dom_ms * 1e-3)
        roof = {"kernel": dom, "bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": unit, "frac": achieved / peak, "traffic": measured_traffic(dom),
                "duration_ms": dom_ms,
                "work": {"flops_per_launch": flops, "near_field_pairs": pairs,
                         "m2l_translations": n_m2l}}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": PEAK["hbm"] / 1e9,
                "unit": "GB/s", "frac": None, "traffic": None}

    cpu = None
    errors = None
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        ref = oracle.solve(d["x"], d["qA"], d["qB"], d["site"], d["lam"], box=d["box"],
                           periodic=True)
        t1 = time.perf_counter()
        cpu = {"value": 1.0 / (t1 - t0), "unit": "evals/s", "cores": oracle.num_threads(),
               "nproc": len(os.sched_getaffinity(0)), "kind": "oracle",
               "sample": "one full FP64 Ewald evaluation of the 30,000-atom box (all atoms)"}
        # each plan's error against that oracle result (relative RMS of F and
        # phi, energy error over 1/2 sum |q phi|, max dV/dlambda error over
        # the RMS of dV/dlambda)
        errors = {}
        for name_, (pl_, in_) in (("bf16x3", (plan, inp)), ("f32", (plan32, inp32)),
                                  ("fp64", (plan64, inp64))):
            o = pl_.eval(*in_, box=d["box"])
            torch.cuda.synchronize(dev)
            F_ = o["F"].double().cpu().numpy()
            p_ = o["phi"].double().cpu().numpy()
            dv = ref["dVdl"]
            errors[name_] = {
                "F": float(np.sqrt(np.sum((F_ - ref["F"]) ** 2) / np.sum(ref["F"] ** 2))),
                "phi": float(np.sqrt(np.sum((p_ - ref["phi"]) ** 2) / np.sum(ref["phi"] ** 2))),
                "E": float(abs(o["E"].item() - ref["E"]) / (0.5 * np.sum(np.abs(ref["q"] * ref["phi"])))),
                "dVdl": float(np.abs(o["dVdl"].cpu().numpy() - dv).max() / np.sqrt(np.mean(dv ** 2)))}

    # whole evaluation against its ideal time: each phase at its own ceiling
    # (near field: FP32 vector; M2L: bf16 matrix cores, three products per
    # translation; every other byte once at the HBM rate)
    tree_bytes = eval_bytes(n, S, depth, order)
    t_ideal = {"near_field_us": 1e6 * 20.0 * pairs / PEAK["fp32_vector"],
               "m2l_us": 1e6 * 3 * 2.0 * K * K * n_m2l / PEAK["bf16_mfma"],
               "tree_and_io_us": 1e6 * tree_bytes / PEAK["hbm"]}
    t_ideal_us = sum(t_ideal.values())
    eval_roof = {"t_ideal_us": t_ideal_us, "t_measured_us": sec * 1e6, "frac": t_ideal_us / (sec * 1e6),
                 "parts": t_ideal, "tree_and_io_bytes": tree_bytes}

    res = {
        "metric": "E+F+dV/dlambda evals/s at 30k atoms p=8 (mixed vs FP64 FMM), roofline %",
        "value": 1.0 / sec,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 + bf16x3 M2L (FP64 root, lattice operator and reductions)",
        "data": "synthetic",
        "config": {"workload": "water_box: 30,000 atoms (9,000 TIP3P-like waters + 3,000-atom "
                               "charged cluster), periodic 6.7 nm cube, 20 four-atom sites",
                   "depth": depth, "order_p": order, "n_atoms": n, "n_sites": S,
                   "parallelism": "single GPU"},
        "fp64": {"value": 1.0 / sec64, "ms_per_step": sec64 * 1e3, "steps": args.fp64_steps},
        "f32": {"value": 1.0 / sec32, "ms_per_step": sec32 * 1e3, "steps": args.fp64_steps},
        "speedup_mixed_vs_fp64": sec64 / sec,
        "graph_replay": {"value": 1.0 / sec_graph, "ms_per_step": sec_graph * 1e3},
        "hamiltonian": {"value": 1.0 / sec_ham, "ms_per_step": sec_ham * 1e3,
                        "workload": "same box, Hamiltonian interpolation (intra-site "
                                    "correction on E, F, dV/dlambda)"},
        "tautomers": {"value": 1.0 / sec_taut, "ms_per_step": sec_taut * 1e3,
                      "workload": "same box, four charge forms per site (half the sites with "
                                  "tautomers), E+F+dV/dlambda_p+dV/dlambda_t"},
        "exclusions": {"value": 1.0 / sec_excl, "ms_per_step": sec_excl * 1e3,
                       "workload": "same box, the 3 intramolecular pairs of each of the 9,000 "
                                   "waters excluded (54,000 partner entries)"},
        "lambda_dynamics": lam_dyn,
        "batched": batched,
        "repeats": {"values": [1.0 / t for t in rep], "median": 1.0 / float(np.median(rep)),
                    "steps_each": args.steps},
        "errors": errors,
        "eval_roofline": eval_roof,
        "site_sweep": sweep,
        "differentiation": diff,
        "large": large,
        "phase_ms": phase_ms,
        "phase_ms_fp64": phase_ms64,
        "phase_ms_f32": phase_ms32,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
