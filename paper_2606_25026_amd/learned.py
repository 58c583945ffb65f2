"""Learned coarse-grid corrector workload: training-pair generation, training,
the P(k) judge and the fine-solve fallback, sequenced over libwdm entry points.

Every computation runs in the library's kernels (fine and coarse KDK steps,
spectral restriction, training pairs and their normalisation, network
forward/backward/Adam, the correction inside the coarse plan's captured step,
shell power spectra); this module orders the calls, keeps tensors alive and
compares scalars.

Workload (the defaults): fine 256^3 and coarse 128^3 periodic boxes of the
coupled-halo generator (GRF k0 = 16 * 2 pi + soliton, Plummer baryons carrying
0.1 of the wave mass, particles in both runs), dt_f = 0.2 dx_f^2 and
dt_c = 0.2 dx_c^2 = 4 dt_f.  A training pair is (restricted fine state at t0,
advanced `every` coarse steps) -> (restricted fine state at t0 + every dt_c);
the network learns the residual.  Window starts are spread along the judged
horizon.  The judge runs `judge_steps` coarse steps (a correction every
`every` steps) and compares the shell power spectrum of the density contrast
with the plain fine solve over shells 1..nc/2-1; above `threshold` the fine
solve is used instead (fallback).
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
    pair_stride: int = 8          # coarse steps between training-window starts
    heldout_seeds: tuple = tuple(range(100, 110))
    every: int = 8                # coarse steps between corrections
    judge_steps: int = 64         # coarse steps in the judged run
    epochs: int = 20
    lr: float = 1e-3
    threshold: float = 0.02       # P(k) error above which the fine solve is used
    init_scale: float = 0.05
    horizon_checkpoints: tuple = ()   # coarse steps at which to report the no-net error
    k0_modes: float = 16.0        # generator: GRF scale k0 = k0_modes * 2 pi / L
    rc: float = 0.05              # generator: soliton core radius
    seed: int = 0
    extra: dict = field(default_factory=dict)


def _torch():
    import torch

    return torch


def halo(cfg, seed):
    """The coupled-halo field and particles of one seed on the fine grid."""
    return inputs.coupled_halo(n=cfg.n_fine, n_particles=cfg.n_particles, seed=seed, rc=cfg.rc,
                               k0_modes=cfg.k0_modes)


def _state(wl, device):
    torch = _torch()
    psi = torch.from_numpy(wl.psi.astype(np.complex64)).to(device)
    pos = torch.from_numpy(wl.pos).to(device) if wl.n_particles else None
    vel = torch.from_numpy(wl.vel).to(device) if wl.n_particles else None
    return psi, pos, vel


def pk_error(pk_c, pk_f, nbins):
    """Relative L2 distance of two shell spectra over shells 1 .. nbins-1."""
    b = slice(1, nbins)
    d = pk_c[b] - pk_f[b]
    return float(math.sqrt(np.sum(d * d) / np.sum(pk_f[b] ** 2)))


class Pipeline:
    """A fine and a coarse single-member plan and the corrector network, on
    one stream, plus buffers."""

    def __init__(self, cfg: LearnedConfig, particle_mass: float, device="cuda"):
        torch = _torch()
        self.cfg = cfg
        self.device = device
        nf, nc, npart = cfg.n_fine, cfg.n_coarse, cfg.n_particles
        self.fine = wdm.Plan(wdm.make_config(nf, n_particles=npart, particle_mass=particle_mass),
                             device=device)
        self.coarse = wdm.Plan(wdm.make_config(nc, n_particles=npart,
                                               particle_mass=particle_mass), device=device)
        self.net = wdm.Net(nc, device=device)
        self.dt_f = 0.2 / nf ** 2
        self.dt_c = 0.2 / nc ** 2
        self.ratio = int(round(self.dt_c / self.dt_f))
        self.buf_c = torch.empty((nc,) * 3, dtype=torch.complex64, device=device)
        self.pos = torch.empty((max(npart, 1), 3), dtype=torch.float32, device=device)
        self.vel = torch.empty_like(self.pos)
        self.fallback = False

    # -- state hand-over --------------------------------------------------
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

    def attach(self, on: bool):
        wdm.wdm_plan_attach_corrector(self.coarse.handle, self.net.handle if on else None, 0,
                                      self.cfg.every if on else 0)

    def coarse_pk(self):
        return wdm.wdm_power_spectrum(self.coarse.handle, 0, self.cfg.n_coarse // 2)[0]

    def fine_pk(self):
        return wdm.wdm_power_spectrum(self.fine.handle, 0, self.cfg.n_coarse // 2)[0]

    # -- training ------------------------------------------------------------
    def make_pairs(self, seeds, log=print):
        """Training pairs (x, y) as device tensors: x = (Re psi, Im psi, Phi)
        of the coarse state after `every` steps from the restricted fine state,
        y = restricted fine state at the same time minus the coarse psi."""
        torch = _torch()
        cfg, nc = self.cfg, self.cfg.n_coarse
        xs, ys = [], []
        for s in seeds:
            wl = halo(cfg, s)
            psi, pos, vel = _state(wl, self.device)
            wdm.wdm_set_state(self.fine.handle, 0, psi, pos, vel)
            self.attach(False)
            for w in range(cfg.windows):
                if w:
                    gap = cfg.pair_stride - cfg.every
                    if gap > 0:
                        wdm.wdm_step(self.fine.handle, gap * self.ratio, self.dt_f)
                self.coarse_from_fine()
                wdm.wdm_step(self.coarse.handle, cfg.every, self.dt_c)
                wdm.wdm_step(self.fine.handle, cfg.every * self.ratio, self.dt_f)
                tgt = torch.empty_like(self.buf_c)
                wdm.wdm_restrict(self.fine.handle, 0, self.coarse.handle, 0, tgt)
                x = torch.empty((nc ** 3, 3), dtype=torch.float32, device=self.device)
                y = torch.empty((nc ** 3, 2), dtype=torch.float32, device=self.device)
                wdm.wdm_net_pair(self.coarse.handle, 0, tgt, x, y)
                xs.append(x)
                ys.append(y)
            log(f"# pairs: seed {s} done ({len(xs)} pairs)")
        return xs, ys

    def train(self, xs, ys, log=print):
        cfg = self.cfg
        wdm.wdm_net_fit_scales(self.net.handle, xs, ys)
        rng = np.random.default_rng(cfg.seed)
        wdm.wdm_net_set_params(self.net.handle,
                               (rng.standard_normal(wdm.wdm_net_param_count())
                                * cfg.init_scale).astype(np.float32))
        losses = []
        for ep in range(cfg.epochs):
            order = rng.permutation(len(xs))
            tot = 0.0
            for i in order:
                wdm.wdm_net_forward(self.net.handle, xs[i])
                tot += wdm.wdm_net_mse_backward(self.net.handle, ys[i])
                wdm.wdm_net_adam(self.net.handle, cfg.lr)
            losses.append(tot / len(order))
            log(f"# epoch {ep}: mean loss {losses[-1]:.4e}")
        return losses

    # -- judge and fallback ----------------------------------------------------
    def judge_seed(self, seed):
        """P(k) errors after judge_steps coarse steps, with and without the
        corrector, against the plain fine solve over the same time."""
        cfg = self.cfg
        wl = halo(cfg, seed)
        psi, pos, vel = _state(wl, self.device)
        torch = _torch()
        res, fields = {}, {}
        for use_net in (False, True):
            wdm.wdm_set_state(self.fine.handle, 0, psi, pos, vel)
            self.coarse_from_fine()
            self.attach(use_net)
            wdm.wdm_step(self.coarse.handle, cfg.judge_steps, self.dt_c)
            res[use_net] = self.coarse_pk()
            fields[use_net] = torch.empty_like(self.buf_c)
            wdm.wdm_get_psi(self.coarse.handle, 0, fields[use_net])
        self.attach(False)
        wdm.wdm_set_state(self.fine.handle, 0, psi, pos, vel)
        wdm.wdm_step(self.fine.handle, cfg.judge_steps * self.ratio, self.dt_f)
        pk_f = self.fine_pk()
        nb = cfg.n_coarse // 2
        # field error: the coarse field against the restricted fine field
        target = torch.empty_like(self.buf_c)
        wdm.wdm_restrict(self.fine.handle, 0, self.coarse.handle, 0, target)
        ferr = {}
        for use_net in (False, True):
            wdm.wdm_set_state(self.coarse.handle, 0, fields[use_net], *self.particles_of(self.fine))
            d, o = wdm.wdm_distance(self.coarse.handle, 0, target)
            ferr[use_net] = math.sqrt(d / o)
        return {"err_without_net": pk_error(res[False], pk_f, nb),
                "err_with_net": pk_error(res[True], pk_f, nb),
                "field_err_without_net": ferr[False], "field_err_with_net": ferr[True]}

    def judge(self, seeds, log=print):
        """Judge on held-out seeds; the fallback is taken when the mean error
        with the corrector exceeds the threshold."""
        judged = []
        for s in seeds:
            judged.append(self.judge_seed(s))
            log(f"# judge: seed {s}: {judged[-1]}")
        mean = {k: float(np.mean([j[k] for j in judged])) for k in judged[0]}
        self.fallback = mean["err_with_net"] > self.cfg.threshold
        return {"pk_err_with_net": mean["err_with_net"],
                "pk_err_without_net": mean["err_without_net"],
                "gain": mean["err_without_net"] - mean["err_with_net"],
                "field_err_with_net": mean["field_err_with_net"],
                "field_err_without_net": mean["field_err_without_net"],
                "per_seed": judged, "fallback_to_fine": self.fallback}

    def advance(self, psi, pos, vel, coarse_steps):
        """Advance an initial state by coarse_steps * dt_c of simulated time on
        the path the judge chose: the coarse plan with the corrector attached
        (restricted state), or, after a fallback, the plain fine plan.  Returns
        (plan name, field as a device tensor)."""
        torch = _torch()
        wdm.wdm_set_state(self.fine.handle, 0, psi, pos, vel)
        if self.fallback:
            wdm.wdm_step(self.fine.handle, coarse_steps * self.ratio, self.dt_f)
            out = torch.empty_like(psi)
            wdm.wdm_get_psi(self.fine.handle, 0, out)
            return "fine", out
        self.coarse_from_fine()
        self.attach(True)
        wdm.wdm_step(self.coarse.handle, coarse_steps, self.dt_c)
        self.attach(False)
        out = torch.empty_like(self.buf_c)
        wdm.wdm_get_psi(self.coarse.handle, 0, out)
        return "coarse", out

    # -- cost ------------------------------------------------------------------
    def seconds_per_unit_time(self, reps=3, blocks=4):
        """Wall time per simulated time unit of the plain fine solve and of the
        coarse solve with the corrector attached (its correction inside the
        captured block), each over `blocks` correction intervals."""
        torch = _torch()
        cfg = self.cfg

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

        nfine = blocks * cfg.every * self.ratio
        ncoarse = blocks * cfg.every
        t_f = timed(lambda: wdm.wdm_step(self.fine.handle, nfine, self.dt_f)) / (nfine * self.dt_f)
        self.attach(True)
        t_c = timed(lambda: wdm.wdm_step(self.coarse.handle, ncoarse, self.dt_c)) / (
            ncoarse * self.dt_c)
        self.attach(False)
        return t_f, t_c

    def error_horizon(self, seed, checkpoints):
        """P(k) error of the coarse solve without the corrector against the
        fine solve at each checkpoint (coarse steps, increasing)."""
        cfg = self.cfg
        wl = halo(cfg, seed)
        psi, pos, vel = _state(wl, self.device)
        wdm.wdm_set_state(self.fine.handle, 0, psi, pos, vel)
        self.coarse_from_fine()
        self.attach(False)
        out, done = [], 0
        for c in checkpoints:
            wdm.wdm_step(self.coarse.handle, c - done, self.dt_c)
            wdm.wdm_step(self.fine.handle, (c - done) * self.ratio, self.dt_f)
            done = c
            out.append((c, pk_error(self.coarse_pk(), self.fine_pk(), cfg.n_coarse // 2)))
        return out

    def close(self):
        self.net.close()
        self.fine.close()
        self.coarse.close()


def run(cfg: LearnedConfig, device="cuda", log=print) -> dict:
    """Generate pairs, train, judge on held-out seeds, time both paths."""
    torch = _torch()
    wl0 = halo(cfg, cfg.train_seeds[0])
    pipe = Pipeline(cfg, wl0.particle_mass, device)
    del wl0
    t0 = time.perf_counter()
    xs, ys = pipe.make_pairs(cfg.train_seeds, log)
    t_pairs = time.perf_counter() - t0
    t1 = time.perf_counter()
    losses = pipe.train(xs, ys, log)
    t_train = time.perf_counter() - t1
    scales = wdm.wdm_net_get_scales(pipe.net.handle)
    del xs, ys
    torch.cuda.empty_cache()
    res = pipe.judge(cfg.heldout_seeds, log)
    if cfg.horizon_checkpoints:
        res["horizon_without_net"] = pipe.error_horizon(cfg.heldout_seeds[0],
                                                        cfg.horizon_checkpoints)
        log(f"# horizon: {res['horizon_without_net']}")
    t_f, t_c = pipe.seconds_per_unit_time()
    res.update({"s_per_unit_time_fine": t_f, "s_per_unit_time_learned": t_c,
                "speedup": t_f / t_c,
                "effective_speedup": 1.0 if res["fallback_to_fine"] else t_f / t_c,
                "train_losses": losses, "scales": scales,
                "pairs": len(cfg.train_seeds) * cfg.windows,
                "seconds_pairs": t_pairs, "seconds_train": t_train})
    pipe.close()
    return res
