"""GPU parity of the static baryon mode and the particle sub-steps (Sec. 3.2.2).

Through the C ABI against the FP64 oracle on the same seeded inputs: the wave
to the stepping tests' tolerances (relative L2 1e-5 complex64, 1e-11
complex128); particles, which are float32 on the GPU, to 1e-5 relative L2 in
velocity and in position to the rounding bound of float32 storage: every
drift rounds a coordinate in [0, 1) by at most half an ulp, 2^-25, and with a
near-constant increment per sub-step those roundings add up in one direction,
so after D drifts the bound is D * 2^-25 (a float32 emulation of the same
updates in the oracle's potentials reproduces the GPU's largest position
error, 2.36e-6 after 80 drifts, to all digits).

Inputs: the GRF + soliton halo with Plummer baryons.  Sub-steps are tested at
the workload's dt and at a step long enough (dt = 0.05, particles cross about
one cell) for the sub-steps to change the particle orbits far beyond the
tolerance.
"""
import numpy as np
import pytest

from paper_2606_25026_amd import inputs
from test_gpu_parity import Run, check_l2, periodic_diff, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def tol(prec):
    return 1e-5 if prec == 0 else 1e-11


def f64(a):
    return a.astype(np.float64)


def pos_tol(drifts):
    """float32 storage bound after `drifts` drifts of coordinates in [0, 1)."""
    return drifts * 2.0 ** -25 + 1e-7


@pytest.mark.parametrize("prec", [0, 1])
def test_static_baryons_match_oracle(wdm, orc, prec):
    n, npart, steps = 64, 5000, 20
    wl = inputs.coupled_halo(n=n, n_particles=npart, seed=21, steps=steps, mass_fraction=0.3)
    r = Run(wdm, wl.psi, pos=wl.pos, vel=wl.vel, mp=wl.particle_mass, prec=prec,
            baryon_mode=wdm.WDM_BARYON_STATIC)
    e0 = wdm.wdm_energy(r.plan.handle, 0)
    r.step(steps, wl.dt)
    cfg = orc.make_config((n,) * 3, n_particles=npart, particle_mass=wl.particle_mass,
                          baryon_mode=orc.BARYON_STATIC)
    psi_ref, _, _ = orc.kdk(cfg, wl.psi, f64(wl.pos), f64(wl.vel), nsteps=steps, dt=wl.dt)
    err = check_l2(r.get_psi(), psi_ref, tol(prec))
    p, v = r.get_particles()
    assert np.array_equal(p, f64(wl.pos)) and np.array_equal(v, f64(wl.vel))
    e = wdm.wdm_energy(r.plan.handle, 0)
    ref = orc.energy(cfg, psi_ref, f64(wl.pos), f64(wl.vel))
    for key in ("mass", "e_pot", "e_total"):
        assert e[key] == pytest.approx(ref[key], rel=2e-6), key
    # the static deposit is still in place after the steps: the potential
    # of the final state equals the oracle's
    check_l2(r.get_phi(), orc.potential(cfg, psi_ref, f64(wl.pos)), 1e-5 if prec == 0 else 1e-11)
    print(f"static baryons 64^3 + {npart}, prec={prec}: psi {err:.3e}, "
          f"e_total {e0['e_total']:.6e} -> {e['e_total']:.6e}")
    r.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_substeps_at_workload_dt_match_oracle(wdm, orc, prec):
    n, npart, steps, S = 64, 5000, 20, 4
    wl = inputs.coupled_halo(n=n, n_particles=npart, seed=22, steps=steps)
    r = Run(wdm, wl.psi, pos=wl.pos, vel=wl.vel, mp=wl.particle_mass, prec=prec,
            nbody_substeps=S)
    wdm.wdm_set_sort_interval(r.plan.handle, 8)
    r.step(steps, wl.dt)
    cfg = orc.make_config((n,) * 3, n_particles=npart, particle_mass=wl.particle_mass,
                          nbody_substeps=S)
    psi_ref, p_ref, v_ref = orc.kdk(cfg, wl.psi, f64(wl.pos), f64(wl.vel), nsteps=steps,
                                    dt=wl.dt)
    check_l2(r.get_psi(), psi_ref, tol(prec))
    p, v = r.get_particles()
    assert np.max(np.abs(periodic_diff(p, p_ref))) < pos_tol(steps * S)
    check_l2(v, v_ref, 1e-5)
    r.close()


@pytest.mark.parametrize("S", [1, 8])
def test_substeps_on_a_long_step_match_oracle(wdm, orc, S):
    n, npart, DT, steps = 32, 400, 0.05, 2
    wl = inputs.coupled_halo(n=n, n_particles=npart, seed=3, steps=0, mass_fraction=0.3)
    r = Run(wdm, wl.psi, pos=wl.pos, vel=wl.vel, mp=wl.particle_mass, prec=1,
            nbody_substeps=S)
    r.step(steps, DT)
    p, v = r.get_particles()
    refs = {}
    for s in {1, S}:
        cfg = orc.make_config((n,) * 3, n_particles=npart, particle_mass=wl.particle_mass,
                              nbody_substeps=s)
        refs[s] = orc.kdk(cfg, wl.psi, f64(wl.pos), f64(wl.vel), nsteps=steps, dt=DT)
    _, p_ref, v_ref = refs[S]
    dp = np.max(np.abs(periodic_diff(p, p_ref)))
    assert dp < pos_tol(steps * S)
    check_l2(v, v_ref, 2e-5)
    # the orbit change from the sub-steps is far above the tolerance
    gap = np.max(np.abs(periodic_diff(refs[1][1], p_ref)))
    print(f"long step, S={S}: position error {dp:.2e}; S=1 vs S={S} differ by {gap:.2e}")
    if S > 1:
        assert gap > 100 * pos_tol(steps * S)
    r.close()


def test_static_and_substepped_members_in_one_class(wdm, orc):
    # one size class, three members: static with the most particles, dynamic
    # with 3 sub-steps, dynamic plain; every member against its own oracle run
    n, steps = 32, 15
    specs = [(3000, dict(baryon_mode=1)), (1500, dict(nbody_substeps=3)), (800, dict())]
    wls = [inputs.coupled_halo(n=n, n_particles=npart, seed=30 + i, steps=steps,
                               mass_fraction=0.2)
           for i, (npart, _) in enumerate(specs)]
    cfgs = [wdm.make_config(n, n_particles=npart, particle_mass=wl.particle_mass, **extra)
            for (npart, extra), wl in zip(specs, wls)]
    plan = wdm.Plan(cfgs)
    keep = []
    for i, wl in enumerate(wls):
        t = [torch.from_numpy(a).cuda() for a in (wl.psi.astype(np.complex64), wl.pos, wl.vel)]
        keep.append(t)
        wdm.wdm_set_state(plan.handle, i, *t)
    wdm.wdm_step(plan.handle, steps, wls[0].dt)
    for i, ((npart, extra), wl) in enumerate(zip(specs, wls)):
        psi = torch.empty((n,) * 3, dtype=torch.complex64, device="cuda")
        pos = torch.empty((npart, 3), dtype=torch.float32, device="cuda")
        vel = torch.empty((npart, 3), dtype=torch.float32, device="cuda")
        wdm.wdm_get_psi(plan.handle, i, psi)
        wdm.wdm_particles(plan.handle, i, pos, vel)
        torch.cuda.synchronize()
        cfg = orc.make_config((n,) * 3, n_particles=npart, particle_mass=wl.particle_mass,
                              **extra)
        psi_ref, p_ref, v_ref = orc.kdk(cfg, wl.psi, f64(wl.pos), f64(wl.vel), nsteps=steps,
                                        dt=wls[0].dt)
        check_l2(psi.cpu().numpy(), psi_ref, 1e-5)
        p = pos.cpu().numpy().astype(np.float64)
        drifts = steps * extra.get("nbody_substeps", 1)
        assert np.max(np.abs(periodic_diff(p, p_ref))) < pos_tol(drifts), i
        check_l2(vel.cpu().numpy(), v_ref, 1e-5)
    plan.close()
