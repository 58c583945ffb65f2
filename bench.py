"""Benchmark: grid cell-updates/s of the KDK split step on one MI355X.

Workload: the coupled halo -- 256^3 complex64 wave field (GRF with power
exp(-k^2/k0^2), k0 = 16 * 2 pi / L, plus a soliton core) and 1e6 CIC-coupled
Plummer baryon particles, dt = 0.2 dx^2 -- resident in HBM before timing.
A step is one full kick-drift-kick step (all eight grid passes plus the
particle kick/drift/deposit; periodic particle re-sorts included).

Prints one JSON line with the metric, a per-kernel roofline entry for the
largest grid pass that does not share the chip with the particle kernel
(algorithmic bytes / HIP-event duration on the stream it runs on),
the whole-step roofline fraction, and the FP64 CPU oracle timed on a bounded
sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--particles 1000000]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per cell (grid passes) and per particle
BYTES_PER_CELL = {
    "z_potential_kick": 24, "y_fft_psi_fwd": 16, "x_kinetic": 16, "y_fft_psi_inv": 16,
    "z_density_r2c": 28, "y_fft_spec_fwd": 8, "x_green": 8, "y_fft_spec_inv": 8,
    "z_potential_close_kick": 24,
}
BYTES_PER_PARTICLE = {"particles_kick_drift_deposit": 48, "particles_close_kick": 36}
# tuning-table slot of each grid pass (P1, P2/P4, P3, P5, P6/P8, P7)
PASS_SLOT = {"z_potential_kick": 0, "z_potential_close_kick": 0, "y_fft_psi_fwd": 1,
             "y_fft_psi_inv": 1, "x_kinetic": 2, "z_density_r2c": 3, "y_fft_spec_fwd": 4,
             "y_fft_spec_inv": 4, "x_green": 5}


def pass_variant(name, tuning):
    # the closing kick always runs the default plan
    if name == "z_potential_close_kick":
        return 0
    return int(tuning[PASS_SLOT[name]])


# grid passes that run while the particle kernel is in flight on its own stream
OVERLAPS_PARTICLES = {"y_fft_psi_fwd", "x_kinetic", "y_fft_psi_inv"}
STEP_BYTES_PER_CELL = 124
STEP_BYTES_PER_PARTICLE = 48


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted((ROOT / "paper_2606_25026_amd" / "csrc").glob("*")):
        h.update(f.read_bytes())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str, variant: int = 0):
    """HBM bytes per launch of `kernel` with FFT plan `variant` from committed
    rocprofv3 counter summaries, or None."""
    f = ROOT / "profiles" / "traffic_counters.json"
    if not f.exists():
        return None
    try:
        d = json.loads(f.read_text())
    except Exception:
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None  # the kernels changed since the counters were taken
    k = d.get("kernels", {}).get(kernel, {}).get(str(variant))
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def cpu_baseline(wl, budget_s: float = 20.0):
    """The FP64 oracle on the host cores over a bounded sample of the workload:
    unmerged KDK steps with every core the process may use, then with one."""
    import oracle

    cores = len(os.sched_getaffinity(0))
    cfg = oracle.make_config((wl.n,) * 3, n_particles=wl.n_particles,
                             particle_mass=wl.particle_mass)
    pos = wl.pos.astype(np.float64)
    vel = wl.vel.astype(np.float64)

    def per_step(threads, budget):
        oracle.set_threads(threads)
        t = time.perf_counter()
        oracle.kdk(cfg, wl.psi, pos, vel, nsteps=0, dt=wl.dt)   # initial potential only
        setup = time.perf_counter() - t
        t = time.perf_counter()
        oracle.kdk(cfg, wl.psi, pos, vel, nsteps=1, dt=wl.dt)
        one = time.perf_counter() - t - setup
        steps = max(1, min(10, int(budget / max(one, 1e-3))))
        if steps == 1:
            return one, 1
        t = time.perf_counter()
        oracle.kdk(cfg, wl.psi, pos, vel, nsteps=steps, dt=wl.dt)
        return (time.perf_counter() - t - setup) / steps, steps

    per, steps = per_step(cores, budget_s)
    per1, steps1 = per_step(1, budget_s)
    return {"value": wl.n ** 3 / per, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} unmerged FP64 KDK steps of the same {wl.n}^3 + "
                      f"{wl.n_particles}-particle halo (initial Poisson solve subtracted)",
            "s_per_step": per,
            "single_thread": {"value": wl.n ** 3 / per1, "unit": "cell-updates/s", "cores": 1,
                              "s_per_step": per1,
                              "sample": f"{steps1} unmerged FP64 KDK steps, one thread"}}


def learned_cost(h, wl, args, dev, ms_per_step, every=8, blocks=16):
    """Seconds per simulated time unit of the plain fine solve (this run's step
    time over dt) and of the 2x-coarser solve with the learned corrector
    attached (a correction every `every` coarse steps, inside the captured
    block), from the same state restricted to the coarse grid.  The cost does
    not depend on the weights' values: the network is randomly initialised."""
    import torch

    from paper_2606_25026_amd import wdm

    nc = args.n // 2
    coarse = wdm.Plan(wdm.make_config(nc, n_particles=wl.n_particles,
                                      particle_mass=wl.particle_mass), device=dev)
    net = wdm.Net(nc, device=dev)
    rng = np.random.default_rng(0)
    wdm.wdm_net_set_params(net.handle, (rng.standard_normal(wdm.wdm_net_param_count())
                                        * 0.05).astype(np.float32))
    wdm.wdm_net_set_scales(net.handle, 1.0, 1.0, 1e-3)
    buf = torch.empty((nc,) * 3, dtype=torch.complex64, device=dev)
    wdm.wdm_restrict(h, 0, coarse.handle, 0, buf)
    p = v = None
    if wl.n_particles:
        p = torch.empty((wl.n_particles, 3), dtype=torch.float32, device=dev)
        v = torch.empty_like(p)
        wdm.wdm_particles(h, 0, p, v)
    wdm.wdm_set_state(coarse.handle, 0, buf, p, v)
    wdm.wdm_set_sort_interval(coarse.handle, args.sort_interval)
    wdm.wdm_plan_attach_corrector(coarse.handle, net.handle, 0, every)
    dt_c = 0.2 / nc ** 2
    wdm.wdm_step(coarse.handle, every, dt_c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wdm.wdm_step(coarse.handle, every * blocks, dt_c)
    torch.cuda.synchronize()
    t_c = time.perf_counter() - t0
    wdm.wdm_plan_attach_corrector(coarse.handle, None, 0, 0)
    # the same blocks without the corrector: the difference is what a
    # correction costs inside the captured block
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(blocks):
        wdm.wdm_step(coarse.handle, every, dt_c)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    # the corrector alone: one correction (inputs, three convolutions, update,
    # potential rebuilt) and the network's forward pass, HIP events on the
    # stream they run on
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    reps = 20
    wdm.wdm_net_apply(net.handle, coarse.handle, 0)
    ev[0].record()
    for _ in range(reps):
        wdm.wdm_net_apply(net.handle, coarse.handle, 0)
    ev[1].record()
    x = torch.randn((nc ** 3, 3), dtype=torch.float32, device=dev)
    wdm.wdm_net_forward(net.handle, x)
    ev[2].record()
    for _ in range(reps):
        wdm.wdm_net_forward(net.handle, x)
    ev[3].record()
    torch.cuda.synchronize()
    apply_us = ev[0].elapsed_time(ev[1]) * 1e3 / reps
    fwd_us = ev[2].elapsed_time(ev[3]) * 1e3 / reps
    net.close()
    coarse.close()
    cells = nc ** 3
    # forward pass: bf16 activations in and out of the three 3x3x3 layers
    # (3 -> 16 -> 16 -> 2 channels, inputs packed from f32): 12 + 8 (pack) +
    # 32 + 32 + 32 + 32 + 8 = 156 B and 2 * 27 * (3*16 + 16*16 + 16*2) flop per cell
    fwd_bytes = 156 * cells
    fwd_flop = 2 * 27 * (3 * 16 + 16 * 16 + 16 * 2) * cells
    s_fine = ms_per_step * 1e-3 / wl.dt
    s_learned = t_c / (every * blocks * dt_c)
    return {"s_per_unit_fine": s_fine, "s_per_unit_learned": s_learned,
            "ratio": s_fine / s_learned,
            "apply_us": apply_us,
            "apply_in_block_us": (t_c - t_plain) / blocks * 1e6,
            "corrector_roofline": {
                "kernel": "k_conv x3 + input pack (network forward pass)", "bound": "hbm",
                "achieved": fwd_bytes / (fwd_us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": fwd_bytes / (fwd_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                "avg_launch_us": fwd_us, "alg_bytes_per_launch": fwd_bytes,
                "mfma_tflops": fwd_flop / (fwd_us * 1e-6) / 1e12,
                "mfma_peak_tflops_bf16": 2500.0},
            "sample": f"{blocks} blocks of {every} coarse {nc}^3 steps + correction (BF16 MFMA "
                      f"3-layer conv) vs this run's {args.n}^3 step; weights random (cost does "
                      "not depend on them)"}


def bench_ensemble(args):
    """48 independent halos on mixed grids (16 x 64^3, 16 x 96^3, 16 x 128^3), 1e4
    Plummer particles each, advanced together by one captured step with per-member
    dt = 0.2 dx_i^2."""
    import torch

    from paper_2606_25026_amd import inputs, wdm

    members = [inputs.ensemble_member(seed=s, n=n, n_particles=10_000)
               for s, n in enumerate(inputs.ENSEMBLE_SIZES)]
    cfgs = [wdm.make_config(m.n, n_particles=m.n_particles, particle_mass=m.particle_mass)
            for m in members]
    plan = wdm.Plan(cfgs)
    h = plan.handle
    tuning = wdm.autotune(h, cfgs, reps=20) if not args.no_tune else wdm.wdm_get_tuning(h)
    keep = []
    for i, m in enumerate(members):
        psi = torch.from_numpy(m.psi.astype(np.complex64)).cuda()
        pos = torch.from_numpy(m.pos).cuda()
        vel = torch.from_numpy(m.vel).cuda()
        keep.append((psi, pos, vel))
        wdm.wdm_set_state(h, i, psi, pos, vel)
        wdm.wdm_set_member_dt(h, i, m.dt)
    cells = sum(m.n ** 3 for m in members)
    parts = sum(m.n_particles for m in members)
    wdm.wdm_step(h, args.warmup, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wdm.wdm_step(h, args.steps, 0.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el * 1e3 / args.steps
    step_bytes = STEP_BYTES_PER_CELL * cells + STEP_BYTES_PER_PARTICLE * parts
    gbs = step_bytes / (ms * 1e-3) / 1e9
    out = {"metric": "aggregate grid cell-updates/s, 48-member mixed-size ensemble",
           "value": cells * args.steps / el, "unit": "cell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
           "data": "synthetic",
           "config": {"workload": "ensemble 16x64^3 + 16x96^3 + 16x128^3, 1e4 particles each",
                      "members": len(members), "cells": cells, "particles": parts,
                      "fft_plan_variants": tuning},
           "step_roofline": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": gbs / HBM_PEAK_GBS}}
    print(json.dumps(out))
    plan.close()


def bench_precision(args):
    """Precision study: complex64 with FP64 arguments vs complex128 at 512^3, and
    both against the FP64 oracle on the 128^3 sub-box (sampled reference)."""
    import math

    import torch

    from paper_2606_25026_amd import inputs, wdm

    res = {}

    def log(msg):
        print(f"# {msg}", file=sys.stderr, flush=True)

    # --- sub-box vs oracle
    g = np.load(ROOT / "tests" / "golden" / "subbox_128_steps2000.npz")
    n, L, steps = int(g["n"]), float(g["L"]), int(g["steps"])
    psi0 = inputs.grf_soliton(n, L=L, k0=16.0 * 2 * math.pi, rc=0.03, rho_c=50.0, seed=int(g["seed"]))
    for prec, dt_ in ((0, torch.complex64), (1, torch.complex128)):
        plan = wdm.Plan(wdm.make_config(n, L=L, precision=prec))
        x = torch.from_numpy(psi0).to(dt_).cuda()
        wdm.wdm_set_state(plan.handle, 0, x)
        e0 = wdm.wdm_energy(plan.handle, 0)
        wdm.wdm_step(plan.handle, steps, float(g["dt"]))
        out = torch.empty_like(x)
        wdm.wdm_get_psi(plan.handle, 0, out)
        e1 = wdm.wdm_energy(plan.handle, 0)
        got = out.cpu().numpy().ravel()[g["cells"]].astype(np.complex128)
        res[f"subbox128_{'c64' if prec == 0 else 'c128'}"] = {
            "rel_l2_vs_oracle": float(np.linalg.norm(got - g["psi"]) / np.linalg.norm(g["psi"])),
            "mass_drift": e1["mass"] / e0["mass"] - 1,
            "energy_drift": e1["e_total"] / e0["e_total"] - 1,
            "oracle_mass_drift": float(g["mass1"] / g["mass0"] - 1),
            "oracle_energy_drift": float(g["etot1"] / g["etot0"] - 1)}
        plan.close()
        del x, out
        log(f"sub-box {n}^3 {'c64' if prec == 0 else 'c128'} done: {res[f'subbox128_' + ('c64' if prec == 0 else 'c128')]}")
    # --- 512^3: complex64 vs complex128
    n = args.n if args.n != 256 else 512
    log(f"generating the {n}^3 field")
    psi0 = inputs.grf_soliton(n, L=1.0, k0=16.0 * 2 * math.pi, rc=0.03, rho_c=50.0, seed=0)
    dt = 0.2 / n ** 2
    outs = {}
    for prec, dt_ in ((0, torch.complex64), (1, torch.complex128)):
        cfg = wdm.make_config(n, precision=prec)
        plan = wdm.Plan(cfg)
        tuning = wdm.autotune(plan.handle, cfg, reps=5) if not args.no_tune else [0] * 6
        x = torch.from_numpy(psi0).to(dt_).cuda()
        wdm.wdm_set_state(plan.handle, 0, x)
        e0 = wdm.wdm_energy(plan.handle, 0)
        wdm.wdm_step(plan.handle, 5, dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wdm.wdm_step(plan.handle, args.precision_steps, dt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        e1 = wdm.wdm_energy(plan.handle, 0)
        wdm.wdm_get_psi(plan.handle, 0, x)
        outs[prec] = x
        res[f"grid{n}_{'c64' if prec == 0 else 'c128'}"] = {
            "ms_per_step": el * 1e3 / args.precision_steps,
            "cell_updates_per_s": n ** 3 * args.precision_steps / el,
            "mass_drift": e1["mass"] / e0["mass"] - 1,
            "energy_drift": e1["e_total"] / e0["e_total"] - 1,
            "fft_plan_variants": tuning}
        plan.close()
        log(f"{n}^3 {'c64' if prec == 0 else 'c128'} done: {res[f'grid{n}_' + ('c64' if prec == 0 else 'c128')]}")
    d = outs[0].to(torch.complex128) - outs[1]
    res[f"grid{n}_c64_vs_c128_rel_l2"] = float(torch.linalg.vector_norm(d) /
                                               torch.linalg.vector_norm(outs[1]))
    v = res[f"grid{n}_c64"]["cell_updates_per_s"]
    print(json.dumps({"metric": f"precision study: complex64 (FP64 arguments) vs complex128 "
                                f"after {steps} steps", "value": v, "unit": "cell-updates/s",
                      "n_gpus": 1, "steps": args.precision_steps, "dtype": "c64",
                      "data": "synthetic", "higher_is_better": True, "results": res}))


def bench_learned(args):
    """Learned coarse corrector: 128^3 coarse + corrector vs the 256^3 plain solve."""
    from paper_2606_25026_amd import learned

    cfg = learned.LearnedConfig(horizon_checkpoints=(64, 256, 1024, 4096))
    if args.learned_small:
        cfg = learned.LearnedConfig(n_fine=64, n_coarse=32, n_particles=2000,
                                    train_seeds=tuple(range(6)), windows=6, pair_stride=16,
                                    heldout_seeds=(100, 101), epochs=30, judge_steps=48,
                                    lr=2e-3, k0_modes=4.0, rc=0.1,
                                    horizon_checkpoints=(48, 256, 1024))
    res = learned.run(cfg, log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps({
        "metric": "seconds per simulated time unit: plain fine solve / (coarse + corrector)",
        "value": res["effective_speedup"], "unit": "x", "n_gpus": 1,
        "higher_is_better": True, "dtype": "c64 solver, bf16 corrector", "data": "synthetic",
        "config": {"workload": f"learned corrector {cfg.n_coarse}^3 coarse vs {cfg.n_fine}^3 fine, "
                               f"{cfg.n_particles} particles, {res['pairs']} training pairs",
                   "every": cfg.every, "judge_steps": cfg.judge_steps},
        "results": {k: v for k, v in res.items() if k != "train_losses"},
        "train_loss_first_last": [res["train_losses"][0], res["train_losses"][-1]]}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--particles", type=int, default=1_000_000)
    ap.add_argument("--sort-interval", type=int, default=128,
                    help="steps between particle re-sorts (the halo's fastest particles cross "
                         "about 0.1 cell in 128 steps at its dt)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the coarse + corrector timing of the learned path")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without per-kernel HIP events")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default FFT plan of every pass (no autotuning)")
    ap.add_argument("--plans", choices=["tune", "default", "second", "exchange"], default="tune",
                    help="step FFT plans: chosen by timing, or all default / all second plans / "
                         "the complex-exchange plan wherever it exists")
    ap.add_argument("--workload", choices=["halo", "ensemble", "precision", "learned"],
                    default="halo")
    ap.add_argument("--learned-small", action="store_true")
    ap.add_argument("--precision-steps", type=int, default=2000)
    ap.add_argument("--kappa", type=float, default=0.0,
                    help="halo workload: local self-interaction strength (0 = none)")
    ap.add_argument("--absorb-alpha", type=float, default=0.0,
                    help="halo workload: absorbing boundary strength (0 = periodic box)")
    ap.add_argument("--absorb-nb", type=float, default=50.0,
                    help="halo workload: absorbing layer width parameter N_b")
    ap.add_argument("--baryons", choices=["dynamic", "static"], default="dynamic",
                    help="halo workload: particles move (dynamic) or only source the potential")
    ap.add_argument("--substeps", type=int, default=1,
                    help="halo workload: particle leapfrog sub-steps per wave step")
    ap.add_argument("--boundary", choices=["periodic", "vacuum"], default="periodic",
                    help="halo workload: gravity boundary (vacuum = zero-padded isolated solve)")
    ap.add_argument("--tidal", type=float, default=0.0,
                    help="halo workload: strength of an external tidal potential "
                         "T (x^2 + y^2 - 2 z^2) / 2 about the box centre (0 = none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design note, not a built path", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2606_25026_amd import inputs, wdm

    wdm.load()
    if args.workload == "ensemble":
        return bench_ensemble(args)
    if args.workload == "precision":
        return bench_precision(args)
    if args.workload == "learned":
        return bench_learned(args)
    dev = torch.device("cuda:0")
    wl = inputs.coupled_halo(n=args.n, n_particles=args.particles, seed=0)
    n3 = args.n ** 3
    extended = dict(kappa=args.kappa, absorb_alpha=args.absorb_alpha, absorb_nb=args.absorb_nb,
                    baryon_mode=1 if args.baryons == "static" else 0,
                    nbody_substeps=args.substeps,
                    boundary=1 if args.boundary == "vacuum" else 0,
                    external_potential=1 if args.tidal != 0.0 else 0)
    cfg = wdm.make_config(args.n, n_particles=wl.n_particles, particle_mass=wl.particle_mass,
                          **extended)
    plan = wdm.Plan(cfg, device=dev)
    h = plan.handle
    # choose each step pass's FFT plan by timing (before the state is set)
    if args.no_tune or args.plans == "default":
        tuning = wdm.wdm_get_tuning(h)
    elif args.plans == "second":
        wdm.wdm_set_tuning(h, [1] * wdm.wdm_tuning_entries(h))
        tuning = wdm.wdm_get_tuning(h)
    elif args.plans == "exchange":
        # the complex-exchange plan on every pass that has one (the library
        # rejects a table naming it where it does not exist)
        ne = wdm.wdm_tuning_entries(h)
        table = [0] * ne
        for j in range(ne):
            try:
                wdm.wdm_set_tuning(h, [3 if k == j else 0 for k in range(ne)])
                table[j] = 3
            except wdm.WdmError:
                pass
        wdm.wdm_set_tuning(h, table)
        tuning = wdm.wdm_get_tuning(h)
    else:
        tuning = wdm.autotune(h, cfg, reps=20)
    if args.tidal != 0.0:
        x = torch.arange(args.n, dtype=torch.float32, device=dev) / args.n - 0.5
        X, Y, Z = torch.meshgrid(x, x, x, indexing="ij")
        ext = (0.5 * args.tidal * (X * X + Y * Y - 2 * Z * Z)).contiguous()
        wdm.wdm_set_external_potential(h, 0, ext)
        del X, Y, Z, ext
    psi = torch.from_numpy(wl.psi.astype(np.complex64)).to(dev)
    pos = torch.from_numpy(wl.pos).to(dev) if wl.n_particles else None
    vel = torch.from_numpy(wl.vel).to(dev) if wl.n_particles else None
    wdm.wdm_set_state(h, 0, psi, pos, vel)
    wdm.wdm_set_sort_interval(h, args.sort_interval)
    e0 = wdm.wdm_energy(h, 0)
    print(f"# workload ready: {args.n}^3 + {wl.n_particles} particles, dt={wl.dt:.4e}, "
          f"dt_auto={e0['dt_auto']:.4e}", file=sys.stderr, flush=True)

    # achievable-bandwidth reference (plain copy of one psi-sized buffer)
    src = torch.empty(n3 * 8, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    copy_ms = wdm.wdm_copy_bandwidth(dst, src, n3 * 8, reps=20)
    copy_gbs = 2 * n3 * 8 / (copy_ms * 1e-3) / 1e9
    del src, dst

    wdm.wdm_step(h, args.warmup, wl.dt)
    torch.cuda.synchronize()
    # timed region: K steps, captured-graph replay, synchronised on both sides
    t0 = time.perf_counter()
    wdm.wdm_step(h, args.steps, wl.dt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # per-kernel durations: the same K steps again, every launch bracketed by
    # HIP events on the stream it runs on (direct launches; the particle kernel
    # still runs on its own stream, overlapping the y/x/y passes)
    stats = []
    elapsed_prof = None
    if not args.no_profile:
        wdm.wdm_profile_read(h)          # clear
        wdm.wdm_profile(h, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wdm.wdm_step(h, args.steps, wl.dt)
        torch.cuda.synchronize()
        elapsed_prof = time.perf_counter() - t0
        wdm.wdm_profile(h, False)
        stats = wdm.wdm_profile_read(h)
    e1 = wdm.wdm_energy(h, 0)
    ms_per_step = elapsed * 1e3 / args.steps
    value = n3 * args.steps / elapsed

    roofline = None
    per_kernel = {}
    for s in stats:
        nm = s["name"]
        avg_ms = s["total_ms"] / max(1, s["launches"])
        if nm in BYTES_PER_CELL:
            alg = BYTES_PER_CELL[nm] * n3
        elif nm in BYTES_PER_PARTICLE:
            alg = BYTES_PER_PARTICLE[nm] * wl.n_particles
        else:
            alg = None
        per_kernel[nm] = {"launches": s["launches"], "avg_us": avg_ms * 1e3,
                          "share": s["total_ms"] / (elapsed_prof * 1e3),
                          "gbs": (alg / (avg_ms * 1e-3) / 1e9) if alg else None}
    # the roofline kernel is the largest grid pass that runs alone: the passes
    # inside the particle branch's window share the chip with it, so their
    # event durations are not theirs alone
    grid_kernels = [s for s in stats if s["name"] in BYTES_PER_CELL
                    and s["name"] not in OVERLAPS_PARTICLES]
    if grid_kernels:
        dom = max(grid_kernels, key=lambda s: s["total_ms"])
        avg_s = dom["total_ms"] / dom["launches"] * 1e-3
        alg = BYTES_PER_CELL[dom["name"]] * n3
        ach = alg / avg_s / 1e9
        roofline = {"bound": "hbm", "kernel": dom["name"], "achieved": ach,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                    "traffic": traffic_from_profiles(dom["name"], pass_variant(dom["name"], tuning)),
                    "fft_plan_variant": pass_variant(dom["name"], tuning),
                    "alg_bytes_per_launch": alg, "avg_launch_us": avg_s * 1e6}
    # what a wdm_step call of K steps carries besides its K steps: the closing
    # half kick (P1's kick-only pass and the particles' closing kick) once per
    # call, and a particle re-sort every sort_interval steps
    amortised = None
    if per_kernel:
        close_us = sum(per_kernel[k]["avg_us"] for k in ("z_potential_close_kick",
                                                          "particles_close_kick")
                       if k in per_kernel)
        sort = per_kernel.get("particle_sort")
        amortised = {"closing_kick_us_per_call": close_us,
                     "closing_kick_us_per_step": close_us / args.steps,
                     "sorts_in_profiled_region": sort["launches"] if sort else 0,
                     "sort_us": sort["avg_us"] if sort else None,
                     "sort_us_per_step": (sort["launches"] * sort["avg_us"] / args.steps
                                          if sort else 0.0)}
    step_bytes = STEP_BYTES_PER_CELL * n3 + STEP_BYTES_PER_PARTICLE * wl.n_particles
    step_gbs = step_bytes / (ms_per_step * 1e-3) / 1e9

    learned_line = None
    if args.boundary == "periodic" and not args.no_learned:
        learned_line = learned_cost(h, wl, args, dev, ms_per_step)

    cpu = None
    if not args.no_cpu_baseline:
        print("# timing the FP64 CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl)

    base_workload = (f"coupled halo {args.n}^3 complex64 + {wl.n_particles} CIC "
                     "Plummer particles (GRF k0=16*2pi + soliton rc=0.05)")
    out = {
        "metric": "grid cell-updates/s (KDK) at 256^3 c64 + % HBM roofline; learned vs plain s/unit-time",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": base_workload,
                   "grid": args.n, "particles": wl.n_particles, "dt": wl.dt,
                   "phase_args": "fp64", "sort_interval": args.sort_interval,
                   "fft_plan_variants": dict(zip(["P1", "P2/P4", "P3", "P5", "P6/P8", "P7"], tuning)),
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "step_roofline": {"bytes_per_cell_update": step_bytes / n3, "achieved": step_gbs,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": step_gbs / HBM_PEAK_GBS,
                          "copy_kernel_gbs": copy_gbs},
        "per_kernel": per_kernel,
        "per_call_amortised": amortised,
        "timing": "value: captured-graph replay, no per-kernel events; per_kernel and "
                  "roofline: HIP events around every launch over an equal profiled region",
        "profiled_region_ms_per_step": (elapsed_prof * 1e3 / args.steps) if elapsed_prof else None,
        "mass_drift": e1["mass"] / e0["mass"] - 1.0,
        "learned": learned_line,
        "cpu_baseline": cpu,
    }
    if args.kappa != 0.0 or args.absorb_alpha != 0.0:
        out["config"]["workload"] += (f", self-interaction kappa={args.kappa:g}, absorbing "
                                      f"boundary alpha={args.absorb_alpha:g} N_b={args.absorb_nb:g}")
    if args.baryons != "dynamic" or args.substeps > 1:
        out["config"]["workload"] += (f", {args.baryons} baryons, {args.substeps} particle "
                                      "sub-steps per step")
    if args.boundary != "periodic":
        out["config"]["workload"] += ", vacuum gravity boundary (zero-padded isolated solve)"
    if args.tidal != 0.0:
        out["config"]["workload"] += f", external tidal potential T={args.tidal:g}"

    if out["config"]["workload"] != base_workload:
        out["config"].update(extended)
    print(json.dumps(out))
    plan.close()


if __name__ == "__main__":
    main()
