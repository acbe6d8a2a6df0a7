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
PHASE_KERNEL = {"near_far": "k_near_far<float, 8>", "m2l": "k_m2l_bf16x3<6>"}


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

    def timed(plan, inp, steps, warmup, roof_phase=None, every=4):
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
        batched = {"workload": "16 open replicas, 10,000-60,000 atoms (%d total), depth 3, p = 8, "
                               "pH 2-9" % int(ao[-1]),
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
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        oracle.solve(d["x"], d["qA"], d["qB"], d["site"], d["lam"], box=d["box"], periodic=True)
        t1 = time.perf_counter()
        cpu = {"value": 1.0 / (t1 - t0), "unit": "evals/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "one full FP64 Ewald evaluation of the 30,000-atom box (all atoms)"}

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
        "phase_ms": phase_ms,
        "phase_ms_fp64": phase_ms64,
        "phase_ms_f32": phase_ms32,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
