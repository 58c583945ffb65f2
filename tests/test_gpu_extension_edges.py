"""Edge cases of the optional parts of the step on the GPU, against the oracle.

Members of one size class that differ in their optional parts (one with an
external potential, one without; self-interaction on one member only), vacuum
steps on an elongated box, static members with no or one particle, and a
complex128 ensemble mixing vacuum and periodic members.  Tolerances as in the
other stepping tests (relative L2 1e-5 complex64, 1e-11 complex128).
"""
import numpy as np
import pytest

from paper_2606_25026_amd import inputs
from test_gpu_parity import Run, check_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def stored(a, prec):
    return a.astype(np.complex64).astype(np.complex128) if prec == 0 else a


def run_plan(wdm, cfgs, states, steps, dt, prec, ext=None):
    """Step a multi-member plan; return each member's psi (complex128 numpy)."""
    plan = wdm.Plan(cfgs)
    cdt = torch.complex64 if prec == 0 else torch.complex128
    rdt = torch.float32 if prec == 0 else torch.float64
    keep = []
    for i, (psi, pos, vel) in enumerate(states):
        if ext is not None and ext[i] is not None:
            t = torch.from_numpy(ext[i]).to(rdt).cuda()
            keep.append(t)
            wdm.wdm_set_external_potential(plan.handle, i, t)
        args = [torch.from_numpy(psi).to(cdt).cuda()]
        if pos is not None:
            args += [torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()]
        keep.append(args)
        wdm.wdm_set_state(plan.handle, i, *args)
    wdm.wdm_step(plan.handle, steps, dt)
    out = []
    for i, (psi, _, _) in enumerate(states):
        o = torch.empty(psi.shape, dtype=cdt, device="cuda")
        wdm.wdm_get_psi(plan.handle, i, o)
        torch.cuda.synchronize()
        out.append(o.cpu().numpy().astype(np.complex128))
    plan.close()
    return out


def test_one_class_members_with_and_without_extensions(wdm, orc):
    n, steps = 32, 12
    wls = [inputs.plane_wave_box(n, seed=60 + i) for i in range(3)]
    x = np.arange(n) / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    trap = 30.0 * ((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2)
    extras = [dict(external_potential=1), dict(), dict(kappa=-1.5, absorb_alpha=40.0, absorb_nb=8.0)]
    cfgs = [wdm.make_config(n, **e) for e in extras]
    states = [(wl.psi, None, None) for wl in wls]
    got = run_plan(wdm, cfgs, states, steps, wls[0].dt, 0, ext=[trap, None, None])
    for i, (wl, e) in enumerate(zip(wls, extras)):
        ce = {k: v for k, v in e.items() if k != "external_potential"}
        cfg = orc.make_config((n,) * 3, **ce)
        phi_ext = orc.tidal_correct(cfg, trap.astype(np.float32).astype(np.float64)) if i == 0 else None
        ref, _, _ = orc.kdk(cfg, stored(wl.psi, 0), nsteps=steps, dt=wls[0].dt, phi_ext=phi_ext)
        check_l2(got[i], ref, 1e-5)


@pytest.mark.parametrize("prec", [0, 1])
def test_vacuum_steps_on_an_elongated_box(wdm, orc, prec):
    shape, L = (32, 16, 64), (1.0, 0.5, 2.0)
    rng = np.random.default_rng(61)
    x = [np.arange(m) * (l / m) for m, l in zip(shape, L)]
    X, Y, Z = np.meshgrid(*x, indexing="ij")
    r2 = (X - 0.5) ** 2 + (Y - 0.25) ** 2 + (Z - 1.0) ** 2
    psi = np.exp(-r2 / 0.02) * np.exp(2j * np.pi * rng.random(shape) * 0.1)
    r = Run(wdm, psi, L=L, prec=prec, four_pi_G=20.0, boundary=1)
    dt = 0.2 * (1 / 32) ** 2
    r.step(20, dt)
    cfg = orc.make_config(shape, L=L, four_pi_G=20.0, boundary=orc.BOUNDARY_VACUUM)
    ref, _, _ = orc.kdk(cfg, stored(psi, prec), nsteps=20, dt=dt)
    check_l2(r.get_psi(), ref, 1e-5 if prec == 0 else 1e-11)
    r.close()


@pytest.mark.parametrize("npart", [0, 1])
def test_static_members_with_no_or_one_particle(wdm, orc, npart):
    n = 32
    wl = inputs.coupled_halo(n=n, n_particles=max(npart, 1), seed=62, steps=0)
    pos = wl.pos[:npart] if npart else None
    vel = wl.vel[:npart] if npart else None
    mp = 0.05 if npart else 0.0
    r = Run(wdm, wl.psi, pos=pos, vel=vel, mp=mp, baryon_mode=1, nbody_substeps=3)
    r.step(10, wl.dt)
    cfg = orc.make_config((n,) * 3, n_particles=npart, particle_mass=mp, baryon_mode=1,
                          nbody_substeps=3)
    ref, _, _ = orc.kdk(cfg, stored(wl.psi, 0),
                        pos.astype(np.float64) if npart else None,
                        vel.astype(np.float64) if npart else None, nsteps=10, dt=wl.dt)
    check_l2(r.get_psi(), ref, 1e-5)
    if npart:
        p, v = r.get_particles()
        assert np.array_equal(p, pos.astype(np.float64))
    r.close()


def test_complex128_ensemble_vacuum_and_periodic(wdm, orc):
    sizes = (32, 32, 64, 32)
    bounds = (1, 0, 1, 1)
    wls = [inputs.coupled_halo(n=s, n_particles=300, seed=70 + i, steps=0)
           for i, s in enumerate(sizes)]
    cfgs = [wdm.make_config(s, n_particles=300, particle_mass=wl.particle_mass,
                            precision=wdm.WDM_C128, boundary=b)
            for s, b, wl in zip(sizes, bounds, wls)]
    dt = wls[0].dt
    states = [(wl.psi, wl.pos, wl.vel) for wl in wls]
    got = run_plan(wdm, cfgs, states, 8, dt, 1)
    for g, s, b, wl in zip(got, sizes, bounds, wls):
        cfg = orc.make_config((s,) * 3, n_particles=300, particle_mass=wl.particle_mass,
                              boundary=b)
        ref, _, _ = orc.kdk(cfg, wl.psi, wl.pos.astype(np.float64), wl.vel.astype(np.float64),
                            nsteps=8, dt=dt)
        check_l2(g, ref, 1e-11)
