"""CPU pins of the oracle's particle sub-steps and static baryons (Sec. 3.2.2).

Sub-steps: one wave step of dt advances the particles by S leapfrog sub-steps
of h = dt/S in the grid potential of the step's start, the last half kick
taking the new potential.  Pinned against an independent high-order ODE
integration (scipy's DOP853) of the particles in that frozen CIC force field,
which the sub-steps must approach as h^2.

Static baryons: the particles source the potential from fixed positions and
are never kicked or moved.  The wave then moves in a time-independent external
potential, so the total energy (whose particle and baryon self-energy parts
are constants) is conserved to O(dt^2) -- which a wave that ignored the
baryons, or baryons that moved or vanished after the first step, would break.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2606_25026_amd import inputs


def halo(n, npart, seed, frac):
    wl = inputs.coupled_halo(n=n, n_particles=npart, seed=seed, steps=0, mass_fraction=frac)
    return wl, wl.pos.astype(np.float64), wl.vel.astype(np.float64)


def test_one_substep_is_the_plain_step(orc):
    wl, pos, vel = halo(32, 300, 1, 0.1)
    out = []
    for s in (0, 1):
        cfg = orc.make_config((32,) * 3, n_particles=300, particle_mass=wl.particle_mass,
                              nbody_substeps=s)
        out.append(orc.kdk(cfg, wl.psi, pos, vel, nsteps=5, dt=wl.dt))
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_substeps_approach_the_orbit_in_the_frozen_field(orc):
    n, npart, DT = 32, 40, 0.05        # particles move ~1.4 cells in the step
    wl, pos, vel = halo(n, npart, 3, 0.3)
    cfg = orc.make_config((n,) * 3, n_particles=npart, particle_mass=wl.particle_mass)
    phi0 = orc.potential(cfg, wl.psi, pos)

    def rhs(t, y):
        x = np.mod(y[:3 * npart].reshape(-1, 3), 1.0)
        return np.concatenate([y[3 * npart:], orc.cic_force(cfg, phi0, x).ravel()])

    sol = solve_ivp(rhs, (0.0, DT), np.concatenate([pos.ravel(), vel.ravel()]),
                    method="DOP853", rtol=1e-11, atol=1e-13)
    assert sol.status == 0
    x_ref = np.mod(sol.y[:3 * npart, -1].reshape(-1, 3), 1.0)
    v_ref = sol.y[3 * npart:, -1].reshape(-1, 3)
    errs = []
    for S in (8, 16, 32, 64):
        c = orc.make_config((n,) * 3, n_particles=npart, particle_mass=wl.particle_mass,
                            nbody_substeps=S)
        psi1, p, v = orc.kdk(c, wl.psi, pos, vel, nsteps=1, dt=DT)
        d = p - x_ref
        d -= np.round(d)
        errs.append(np.max(np.abs(d)))
        # the closing half kick used the new potential; swapping it for the
        # frozen one gives the frozen-field velocity
        h = DT / S
        phi1 = orc.potential(c, psi1, p)
        v_frozen = v - 0.5 * h * orc.cic_force(c, phi1, p) + 0.5 * h * orc.cic_force(c, phi0, p)
        assert np.max(np.abs(v_frozen - v_ref)) < 400 * errs[-1]
    ratios = [a / b for a, b in zip(errs, errs[1:])]
    assert all(3.5 < r < 4.5 for r in ratios), ratios
    assert errs[-1] < 1e-6


def test_substeps_change_the_result_only_at_order_h2(orc):
    # at the workload's dt the particles barely curve within a step: S = 1 and
    # S = 4 differ by the leapfrog error only, far below the motion itself
    wl, pos, vel = halo(32, 300, 2, 0.1)
    res = []
    for S in (1, 4):
        cfg = orc.make_config((32,) * 3, n_particles=300, particle_mass=wl.particle_mass,
                              nbody_substeps=S)
        res.append(orc.kdk(cfg, wl.psi, pos, vel, nsteps=10, dt=wl.dt))
    dp = res[0][1] - res[1][1]
    dp -= np.round(dp)
    moved = res[0][1] - pos
    moved -= np.round(moved)
    assert 0 < np.max(np.abs(dp)) < 1e-4 * np.max(np.abs(moved))
    assert np.linalg.norm(res[0][0] - res[1][0]) / np.linalg.norm(res[0][0]) < 1e-7


def test_static_baryons_stay_and_source_the_potential(orc):
    wl, pos, vel = halo(32, 1000, 4, 0.3)
    kw = dict(n_particles=1000, particle_mass=wl.particle_mass)
    st = orc.make_config((32,) * 3, baryon_mode=orc.BARYON_STATIC, **kw)
    psi_s, p_s, v_s = orc.kdk(st, wl.psi, pos, vel, nsteps=20, dt=wl.dt)
    assert np.array_equal(p_s, pos) and np.array_equal(v_s, vel)
    # sub-steps do not apply to particles that never move
    st4 = orc.make_config((32,) * 3, baryon_mode=orc.BARYON_STATIC, nbody_substeps=4, **kw)
    assert np.array_equal(orc.kdk(st4, wl.psi, pos, vel, nsteps=20, dt=wl.dt)[0], psi_s)
    dyn = orc.make_config((32,) * 3, **kw)
    psi_d, p_d, _ = orc.kdk(dyn, wl.psi, pos, vel, nsteps=20, dt=wl.dt)
    none = orc.make_config((32,) * 3)
    psi_0, _, _ = orc.kdk(none, wl.psi, nsteps=20, dt=wl.dt)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(psi_s, psi_0) > 1e-4          # the baryons pull on the wave
    assert rel(psi_s, psi_d) > 1e-8          # ... from where they were put
    assert np.max(np.abs(p_d - pos)) > 1e-4


def test_static_mode_energy_second_order(orc):
    wl, pos, vel = halo(32, 2000, 5, 0.5)
    cfg = orc.make_config((32,) * 3, n_particles=2000, particle_mass=wl.particle_mass,
                          baryon_mode=orc.BARYON_STATIC, four_pi_G=10.0)
    e0 = orc.energy(cfg, wl.psi, pos, vel)["e_total"]
    T, drifts = 0.004, []
    for k in (20, 40, 80):
        psi, p, v = orc.kdk(cfg, wl.psi, pos, vel, nsteps=k, dt=T / k)
        drifts.append(orc.energy(cfg, psi, p, v)["e_total"] - e0)
        assert np.array_equal(p, pos)
    e_pot_change = orc.energy(cfg, psi, pos, vel)["e_pot"] - orc.energy(cfg, wl.psi, pos, vel)["e_pot"]
    assert abs(e_pot_change) > 1000 * abs(drifts[-1])     # the wave moved a lot
    for a, b in zip(drifts, drifts[1:]):
        assert 3.8 < a / b < 4.2, drifts
