"""The step passes' other FFT plans -- the second radix plan (twice the lanes
per pencil, half the values per lane) and, for the strided passes, the
wide-row plan (twice the pencils per work-group, 256-byte row segments),
and the complex-exchange plan (whole complex values through LDS; strided
passes, and z passes whose default splits the exchange) -- and the autotuner that chooses among them: forced plans against the FP64
oracle, tuned plans against the oracle, and the choice table's validation and
cache.
"""
import json

import numpy as np
import pytest

from paper_2606_25026_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def periodic_diff(a, b, L=1.0):
    d = a - b
    return d - L * np.round(d / L)


def all_second(wdm, plan):
    """Choice table with the second plan on every pass that has one."""
    n = wdm.wdm_tuning_entries(plan.handle)
    table = [1] * n
    try:
        wdm.wdm_set_tuning(plan.handle, table)
    except wdm.WdmError:
        table = None
    return table


# tuning slots: P1, P2/P4, P3, P5, P6/P8, P7; the strided ones take the wide-row
# plan (2), every pass the complex-exchange plan (3) at these lengths
WIDE = [0, 2, 2, 0, 2, 2]
CX = [3, 3, 3, 3, 3, 3]
STRIDED_PLANS = {"wide-row": WIDE, "complex-exchange": CX}


def run_psi(wdm, plan, psi, steps, dt, prec, pos=None, vel=None):
    x = torch.from_numpy(psi).to(torch.complex64 if prec == 0 else torch.complex128).cuda()
    p = torch.from_numpy(pos).cuda() if pos is not None else None
    v = torch.from_numpy(vel).cuda() if vel is not None else None
    wdm.wdm_set_state(plan.handle, 0, x, p, v)
    wdm.wdm_step(plan.handle, steps, dt)
    out = torch.empty_like(x)
    wdm.wdm_get_psi(plan.handle, 0, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("prec", [0, 1])
def test_second_plans_plane_wave_box_vs_oracle(wdm, orc, prec):
    wl = inputs.plane_wave_box(32, seed=0)
    plan = wdm.Plan(wdm.make_config(32, precision=prec))
    table = all_second(wdm, plan)
    assert table is not None and all(v == 1 for v in table)
    got = run_psi(wdm, plan, wl.psi, 100, wl.dt, prec)
    ref, _, _ = orc.kdk(orc.make_config((32,) * 3), wl.psi, nsteps=100, dt=wl.dt)
    err = rel_l2(got, ref)
    print(f"second plans, 32^3 plane waves, 100 steps, prec={prec}: rel L2 {err:.3e}")
    assert err < (1e-5 if prec == 0 else 1e-11)
    plan.close()


def test_second_plans_halo_64_with_particles_vs_oracle(wdm, orc):
    n, npart, steps = 64, 10_000, 20
    wl = inputs.coupled_halo(n=n, n_particles=npart, seed=1, steps=steps)
    plan = wdm.Plan(wdm.make_config(n, n_particles=npart, particle_mass=wl.particle_mass))
    assert all_second(wdm, plan) is not None
    wdm.wdm_set_sort_interval(plan.handle, 8)
    got = run_psi(wdm, plan, wl.psi, steps, wl.dt, 0, wl.pos, wl.vel)
    cfg = orc.make_config((n,) * 3, n_particles=npart, particle_mass=wl.particle_mass)
    ref, p_ref, _ = orc.kdk(cfg, wl.psi, wl.pos.astype(np.float64), wl.vel.astype(np.float64),
                            nsteps=steps, dt=wl.dt)
    err = rel_l2(got, ref)
    p = torch.empty((npart, 3), dtype=torch.float32, device="cuda")
    v = torch.empty_like(p)
    wdm.wdm_particles(plan.handle, 0, p, v)
    torch.cuda.synchronize()
    print(f"second plans, halo 64^3 + 1e4, {steps} steps: rel L2 {err:.3e}")
    assert err < 1e-5
    assert np.max(np.abs(periodic_diff(p.cpu().numpy(), p_ref))) < 1e-6
    plan.close()


def test_autotuned_plan_matches_oracle(wdm, orc):
    wl = inputs.plane_wave_box(32, seed=3)
    cfg = wdm.make_config(32)
    plan = wdm.Plan(cfg)
    wdm.wdm_autotune(plan.handle, 3)
    table = wdm.wdm_get_tuning(plan.handle)
    assert len(table) == 6 and set(table) <= {0, 1, 2, 3}
    assert table[0] in (0, 1, 3) and table[3] in (0, 1, 3)  # z passes: no wide-row plan
    print(f"32^3 tuned plan variants: {table}")
    got = run_psi(wdm, plan, wl.psi, 100, wl.dt, 0)
    ref, _, _ = orc.kdk(orc.make_config((32,) * 3), wl.psi, nsteps=100, dt=wl.dt)
    assert rel_l2(got, ref) < 1e-5
    plan.close()


def test_autotune_overwrites_state_and_validates_tables(wdm):
    wl = inputs.plane_wave_box(32, seed=0)
    # two size classes: 96^3 has no second radix plan, 32^3 has
    cfgs = [wdm.make_config(96), wdm.make_config(32)]
    plan = wdm.Plan(cfgs)
    assert wdm.wdm_tuning_entries(plan.handle) == 12
    x = torch.from_numpy(wl.psi.astype(np.complex64)).cuda()
    wdm.wdm_set_state(plan.handle, 1, x)
    with pytest.raises(wdm.WdmError):
        wdm.wdm_set_tuning(plan.handle, [0] * 11)            # wrong length
    with pytest.raises(wdm.WdmError):
        wdm.wdm_set_tuning(plan.handle, [1] * 12)            # 96 has no second plan
    with pytest.raises(wdm.WdmError):
        wdm.wdm_set_tuning(plan.handle, [2] + [0] * 11)      # not 0 / 1
    assert wdm.wdm_get_tuning(plan.handle) == [0] * 12       # unchanged
    ok = [0] * 12
    ok[:6] = [1] * 6     # classes in ascending shape order: 32^3 first
    wdm.wdm_set_tuning(plan.handle, ok)
    assert wdm.wdm_get_tuning(plan.handle) == ok
    wdm.wdm_autotune(plan.handle, 2)
    t96 = wdm.wdm_get_tuning(plan.handle)[6:]
    # 96 has no second radix plan and its z passes exchange whole complex
    # values already: they stay on the default, its strided passes may take
    # the wide-row or the complex-exchange plan
    assert t96[0] == 0 and t96[3] == 0 and set(t96) <= {0, 2, 3}
    with pytest.raises(wdm.WdmError):
        wdm.wdm_step(plan.handle, 1, 1e-4)                  # states were overwritten
    plan.close()


def test_tuning_cache_round_trip(wdm, tmp_path):
    cfg = wdm.make_config(64)
    cache = tmp_path / "tune.json"
    plan = wdm.Plan(cfg)
    t1 = wdm.autotune(plan.handle, cfg, cache=str(cache), reps=2)
    store = json.loads(cache.read_text())
    assert store[wdm.tuning_key(cfg)] == t1
    plan.close()
    plan2 = wdm.Plan(cfg)
    # a different stored table is taken from the cache without re-timing
    forced = [1 if v == 0 else 0 for v in t1]
    store[wdm.tuning_key(cfg)] = forced
    cache.write_text(json.dumps(store))
    assert wdm.autotune(plan2.handle, cfg, cache=str(cache)) == forced
    assert wdm.wdm_get_tuning(plan2.handle) == forced
    plan2.close()


@pytest.mark.parametrize("kind", sorted(STRIDED_PLANS))
@pytest.mark.parametrize("prec", [0, 1])
def test_strided_plans_plane_wave_box_vs_oracle(wdm, orc, prec, kind):
    wl = inputs.plane_wave_box(32, seed=0)
    plan = wdm.Plan(wdm.make_config(32, precision=prec))
    table = STRIDED_PLANS[kind]
    wdm.wdm_set_tuning(plan.handle, table)
    assert wdm.wdm_get_tuning(plan.handle) == table
    got = run_psi(wdm, plan, wl.psi, 100, wl.dt, prec)
    ref, _, _ = orc.kdk(orc.make_config((32,) * 3), wl.psi, nsteps=100, dt=wl.dt)
    err = rel_l2(got, ref)
    print(f"{kind} plans, 32^3 plane waves, 100 steps, prec={prec}: rel L2 {err:.3e}")
    assert err < (1e-5 if prec == 0 else 1e-11)
    plan.close()


@pytest.mark.parametrize("kind", sorted(STRIDED_PLANS))
def test_strided_plans_halo_64_with_particles_vs_oracle(wdm, orc, kind):
    n, npart, steps = 64, 10_000, 20
    wl = inputs.coupled_halo(n=n, n_particles=npart, seed=1, steps=steps)
    plan = wdm.Plan(wdm.make_config(n, n_particles=npart, particle_mass=wl.particle_mass))
    wdm.wdm_set_tuning(plan.handle, STRIDED_PLANS[kind])
    wdm.wdm_set_sort_interval(plan.handle, 8)
    got = run_psi(wdm, plan, wl.psi, steps, wl.dt, 0, wl.pos, wl.vel)
    cfg = orc.make_config((n,) * 3, n_particles=npart, particle_mass=wl.particle_mass)
    ref, p_ref, _ = orc.kdk(cfg, wl.psi, wl.pos.astype(np.float64), wl.vel.astype(np.float64),
                            nsteps=steps, dt=wl.dt)
    err = rel_l2(got, ref)
    p = torch.empty((npart, 3), dtype=torch.float32, device="cuda")
    v = torch.empty_like(p)
    wdm.wdm_particles(plan.handle, 0, p, v)
    torch.cuda.synchronize()
    print(f"{kind} plans, halo 64^3 + 1e4, {steps} steps: rel L2 {err:.3e}")
    assert err < 1e-5
    assert np.max(np.abs(periodic_diff(p.cpu().numpy(), p_ref))) < 1e-6
    plan.close()


def test_strided_plan_validation(wdm):
    plan = wdm.Plan(wdm.make_config(32))
    # z passes have no wide-row plan; 4 and -1 are no plan
    for bad in ([2, 0, 0, 0, 0, 0], [0, 0, 0, 2, 0, 0], [0, 4, 0, 0, 0, 0], [0, -1, 0, 0, 0, 0]):
        with pytest.raises(wdm.WdmError):
            wdm.wdm_set_tuning(plan.handle, bad)
    assert wdm.wdm_get_tuning(plan.handle) == [0] * 6
    wdm.wdm_set_tuning(plan.handle, [3, 0, 0, 3, 0, 0])     # z passes at 32: complex exchange
    plan.close()
    plan = wdm.Plan(wdm.make_config((32, 32, 96)))       # z 96 exchanges whole values already
    for bad in ([3, 0, 0, 0, 0, 0], [0, 0, 0, 3, 0, 0]):
        with pytest.raises(wdm.WdmError):
            wdm.wdm_set_tuning(plan.handle, bad)
    plan.close()
    for table in (WIDE, [0, 3, 3, 0, 3, 3]):
        plan = wdm.Plan(wdm.make_config((32, 32, 384)))  # x and y 32, z 384
        wdm.wdm_set_tuning(plan.handle, table)
        plan.close()
        plan = wdm.Plan(wdm.make_config((384, 32, 32)))  # x 384: P3 and P7 have none
        with pytest.raises(wdm.WdmError):
            wdm.wdm_set_tuning(plan.handle, table)
        wdm.wdm_set_tuning(plan.handle, [0, table[1], 0, 0, table[4], 0])
        plan.close()
