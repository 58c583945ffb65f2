"""Learned coarse-grid corrector workload: data generation, training and the
P(k) judge with fallback, sequenced over libwdm entry points.

Every computation runs in the library's kernels (fine and coarse KDK steps,
spectral restriction, network forward/backward/Adam, correction, shell power
spectra); this module only orders the calls and keeps tensors alive.

Workload (the defaults): fine 256^3 and coarse 128^3 periodic boxes of the
coupled-halo generator (GRF k0 = 16 * 2 pi + soliton, Plummer baryons carrying
0.1 of the wave mass, particles in both runs), dt_f = 0.2 dx_f^2 and
dt_c = 0.2 dx_c^2 = 4 dt_f.  A training pair is (restricted fine state at t0,
advanced 8 coarse steps) -> (restricted fine state at t0 + 8 dt_c); the
network learns the residual.  The judge runs 64 coarse steps (8 corrections)
and compares the shell power spectrum of the density contrast with the plain
fine solve over shells 1..nc/2-1.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs, wdm


@dataclass
class LearnedConfig:
    n_fine: int = 256
    n_coarse: int = 128
    n_particles: int = 1_000_000
    train_seeds: tuple = tuple(range(20))
    windows: int = 10
    heldout_seeds: tuple = tuple(range(100, 110))
    every: int = 8                # coarse steps between corrections
    judge_steps: int = 64         # coarse steps in the judged run
    epochs: int = 20
    lr: float = 1e-3
    threshold: float = 0.02       # P(k) error above which the fine solve is used
    init_scale: float = 0.05
    seed: int = 0
    extra: dict = field(default_factory=dict)


def _torch():
    import torch

    return torch


def _state(wl, device):
    torch = _torch()
    psi = torch.from_numpy(wl.psi.astype(np.complex64)).to(device)
    pos = torch.from_numpy(wl.pos).to(device) if wl.n_particles else None
    vel = torch.from_numpy(wl.vel).to(device) if wl.n_particles else None
    return psi, pos, vel


class Pipeline:
    """A fine and a coarse single-member plan on one stream, plus buffers."""

    def __init__(self, cfg: LearnedConfig, particle_mass: float, device="cuda"):
        torch = _torch()
        self.cfg = cfg
        self.device = device
        nf, nc, npart = cfg.n_fine, cfg.n_coarse, cfg.n_particles
        self.fine = wdm.Plan(wdm.make_config(nf, n_particles=npart, particle_mass=particle_mass),
                             device=device)
        self.coarse = wdm.Plan(wdm.make_config(nc, n_particles=npart,
                                               particle_mass=particle_mass), device=device)
        self.dt_f = 0.2 / nf ** 2
        self.dt_c = 0.2 / nc ** 2
        self.ratio = int(round(self.dt_c / self.dt_f))
        self.buf_c = torch.empty((nc,) * 3, dtype=torch.complex64, device=device)
        self.phi_c = torch.empty((nc,) * 3, dtype=torch.float32, device=device)
        self.pos = torch.empty((max(npart, 1), 3), dtype=torch.float32, device=device)
        self.vel = torch.empty_like(self.pos)

    def particles_of(self, plan):
        if self.cfg.n_particles:
            wdm.wdm_particles(plan.handle, 0, self.pos, self.vel)
            return self.pos, self.vel
        return None, None

    def coarse_from_fine(self):
        """Restrict the fine state (psi, particles) onto the coarse plan."""
        wdm.wdm_restrict(self.fine.handle, 0, self.coarse.handle, 0, self.buf_c)
        p, v = self.particles_of(self.fine)
        wdm.wdm_set_state(self.coarse.handle, 0, self.buf_c, p, v)

    def coarse_psi_phi(self):
        torch = _torch()
        psi = torch.empty_like(self.buf_c)
        wdm.wdm_get_psi(self.coarse.handle, 0, psi)
        phi = torch.empty_like(self.phi_c)
        wdm.wdm_potential(self.coarse.handle, 0, phi)
        return psi, phi

    def close(self):
        self.fine.close()
        self.coarse.close()


def make_pairs(cfg: LearnedConfig, seeds, device="cuda", log=print):
    """(input psi/phi after 8 coarse steps, restricted fine target) per window."""
    torch = _torch()
    pipe = None
    xs, ys = [], []
    for s in seeds:
        wl = inputs.coupled_halo(n=cfg.n_fine, n_particles=cfg.n_particles, seed=s)
        if pipe is None:
            pipe = Pipeline(cfg, wl.particle_mass, device)
        psi, pos, vel = _state(wl, device)
        wdm.wdm_set_state(pipe.fine.handle, 0, psi, pos, vel)
        for w in range(cfg.windows):
            pipe.coarse_from_fine()
            wdm.wdm_step(pipe.coarse.handle, cfg.every, pipe.dt_c)
            cpsi, cphi = pipe.coarse_psi_phi()
            wdm.wdm_step(pipe.fine.handle, cfg.every * pipe.ratio, pipe.dt_f)
            tgt = torch.empty_like(pipe.buf_c)
            wdm.wdm_restrict(pipe.fine.handle, 0, pipe.coarse.handle, 0, tgt)
            xs.append(torch.stack([cpsi.real, cpsi.imag, cphi], dim=-1).reshape(-1, 3).contiguous())
            ys.append(torch.stack([(tgt - cpsi).real, (tgt - cpsi).imag], dim=-1)
                      .reshape(-1, 2).contiguous())
        log(f"# pairs: seed {s} done ({len(xs)} pairs)")
    return xs, ys, pipe


def normalisation(xs, ys):
    """Input and output scales from the training set (host scalars)."""
    torch = _torch()
    x = torch.stack(xs)
    y = torch.stack(ys)
    s_psi = 1.0 / float(torch.sqrt(torch.mean(x[..., 0] ** 2 + x[..., 1] ** 2)))
    s_phi = 1.0 / float(torch.std(x[..., 2]))
    s_out = float(torch.std(y))
    return s_psi, s_phi, max(s_out, 1e-30)


def train(cfg: LearnedConfig, net, xs, ys, scales, log=print):
    torch = _torch()
    s_psi, s_phi, s_out = scales
    sc_in = torch.tensor([s_psi, s_psi, s_phi], device=xs[0].device)
    xin = [x * sc_in for x in xs]
    tgt = [y / s_out for y in ys]
    rng = np.random.default_rng(cfg.seed)
    losses = []
    for ep in range(cfg.epochs):
        order = rng.permutation(len(xin))
        tot = 0.0
        for i in order:
            wdm.wdm_net_forward(net.handle, xin[i])
            tot += wdm.wdm_net_mse_backward(net.handle, tgt[i])
            wdm.wdm_net_adam(net.handle, cfg.lr)
        losses.append(tot / len(order))
        log(f"# epoch {ep}: mean loss {losses[-1]:.4e}")
    return losses


def pk_error(pk_c, pk_f, nbins):
    b = slice(1, nbins)
    d = pk_c[b] - pk_f[b]
    return float(math.sqrt(np.sum(d * d) / np.sum(pk_f[b] ** 2)))


def judge(cfg: LearnedConfig, pipe: Pipeline, net, scales, seed, device="cuda"):
    """P(k) error of coarse runs with and without the corrector vs the fine run."""
    wl = inputs.coupled_halo(n=cfg.n_fine, n_particles=cfg.n_particles, seed=seed)
    psi, pos, vel = _state(wl, device)
    nb = cfg.n_coarse // 2
    s_psi, s_phi, s_out = scales
    res = {}
    for use_net in (False, True):
        wdm.wdm_set_state(pipe.fine.handle, 0, psi, pos, vel)
        pipe.coarse_from_fine()
        for _ in range(cfg.judge_steps // cfg.every):
            wdm.wdm_step(pipe.coarse.handle, cfg.every, pipe.dt_c)
            if use_net:
                wdm.wdm_net_apply(net.handle, pipe.coarse.handle, 0, s_psi, s_phi, s_out)
        pk_c, _ = wdm.wdm_power_spectrum(pipe.coarse.handle, 0, nb)
        res["with_net" if use_net else "without_net"] = pk_c
    wdm.wdm_set_state(pipe.fine.handle, 0, psi, pos, vel)
    wdm.wdm_step(pipe.fine.handle, cfg.judge_steps * pipe.ratio, pipe.dt_f)
    pk_f, _ = wdm.wdm_power_spectrum(pipe.fine.handle, 0, nb)
    return {"err_without_net": pk_error(res["without_net"], pk_f, nb),
            "err_with_net": pk_error(res["with_net"], pk_f, nb)}


def seconds_per_unit_time(cfg: LearnedConfig, pipe: Pipeline, net, scales, reps=3):
    """Wall time per simulated time unit: fine plain solve vs coarse + corrector."""
    torch = _torch()
    s_psi, s_phi, s_out = scales

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    def fine_block():
        wdm.wdm_step(pipe.fine.handle, cfg.every * pipe.ratio, pipe.dt_f)

    def coarse_block():
        wdm.wdm_step(pipe.coarse.handle, cfg.every, pipe.dt_c)
        wdm.wdm_net_apply(net.handle, pipe.coarse.handle, 0, s_psi, s_phi, s_out)

    t_f = timed(fine_block) / (cfg.every * pipe.ratio * pipe.dt_f)
    t_c = timed(coarse_block) / (cfg.every * pipe.dt_c)
    return t_f, t_c


def run(cfg: LearnedConfig, device="cuda", log=print) -> dict:
    """Generate pairs, train, judge on held-out seeds, time both paths."""
    torch = _torch()
    t0 = time.perf_counter()
    xs, ys, pipe = make_pairs(cfg, [s for s in cfg.train_seeds], device, log)
    t_pairs = time.perf_counter() - t0
    scales = normalisation(xs, ys)
    net = wdm.Net(cfg.n_coarse, device=device)
    rng = np.random.default_rng(cfg.seed)
    wdm.wdm_net_set_params(net.handle, (rng.standard_normal(wdm.wdm_net_param_count())
                                        * cfg.init_scale).astype(np.float32))
    # untrained baseline loss (identity residual = 0 target scale)
    t1 = time.perf_counter()
    losses = train(cfg, net, xs, ys, scales, log)
    t_train = time.perf_counter() - t1
    del xs, ys
    torch.cuda.empty_cache()
    judged = []
    for s in cfg.heldout_seeds:
        judged.append(judge(cfg, pipe, net, scales, s, device))
        log(f"# judge: seed {s}: {judged[-1]}")
    err_with = float(np.mean([j["err_with_net"] for j in judged]))
    err_without = float(np.mean([j["err_without_net"] for j in judged]))
    t_f, t_c = seconds_per_unit_time(cfg, pipe, net, scales)
    fallback = err_with > cfg.threshold
    out = {"pk_err_with_net": err_with, "pk_err_without_net": err_without,
           "gain": err_without - err_with, "per_seed": judged,
           "s_per_unit_time_fine": t_f, "s_per_unit_time_learned": t_c,
           "speedup": t_f / t_c, "fallback_to_fine": fallback,
           "effective_speedup": 1.0 if fallback else t_f / t_c,
           "train_losses": losses, "scales": scales, "pairs": len(cfg.train_seeds) * cfg.windows,
           "seconds_pairs": t_pairs, "seconds_train": t_train}
    net.close()
    pipe.close()
    return out
