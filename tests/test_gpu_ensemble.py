"""Batched ensembles: several independent boxes of mixed sizes advanced by one
wdm_step call (one launch per pass per size class), each member with its own
time step, checked member by member against the FP64 oracle."""
import numpy as np
import pytest

from paper_2606_25026_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def periodic_diff(a, b):
    d = a - b
    return d - np.round(d)


# FFT plan tables of the three size classes (ascending shapes: 32^3, 64^3,
# 96^3; slots P1, P2/P4, P3, P5, P6/P8, P7): the defaults, the wide-row plan on
# the strided passes, and the complex exchange wherever it exists (z passes at
# 96 exchange whole values by default)
PLANS = {"default": [0] * 18,
         "wide": [0, 2, 2, 0, 2, 2] * 3,
         "exchange": [3] * 12 + [0, 3, 3, 0, 3, 3]}


@pytest.mark.parametrize("plans", sorted(PLANS))
def test_mixed_size_ensemble_matches_oracle(wdm, orc, plans):
    sizes = [64, 32, 64, 96, 32]
    npart = 2000
    steps = 10
    members = [inputs.ensemble_member(seed=s, n=n, n_particles=npart) for s, n in enumerate(sizes)]
    cfgs = [wdm.make_config(m.n, n_particles=npart, particle_mass=m.particle_mass) for m in members]
    plan = wdm.Plan(cfgs)
    wdm.wdm_set_tuning(plan.handle, PLANS[plans])
    bufs = []
    for i, m in enumerate(members):
        psi = torch.from_numpy(m.psi.astype(np.complex64)).cuda()
        pos = torch.from_numpy(m.pos).cuda()
        vel = torch.from_numpy(m.vel).cuda()
        bufs.append((psi, pos, vel))
        wdm.wdm_set_state(plan.handle, i, psi, pos, vel)
        wdm.wdm_set_member_dt(plan.handle, i, m.dt)
    wdm.wdm_step(plan.handle, steps, 0.0)
    for i, m in enumerate(members):
        out = torch.empty_like(bufs[i][0])
        wdm.wdm_get_psi(plan.handle, i, out)
        p = torch.empty_like(bufs[i][1])
        v = torch.empty_like(bufs[i][2])
        wdm.wdm_particles(plan.handle, i, p, v)
        e = wdm.wdm_energy(plan.handle, i)
        torch.cuda.synchronize()
        cfg = orc.make_config((m.n,) * 3, n_particles=npart, particle_mass=m.particle_mass)
        ref, pr, vr = orc.kdk(cfg, m.psi, m.pos.astype(np.float64), m.vel.astype(np.float64),
                              nsteps=steps, dt=m.dt)
        err = rel_l2(out.cpu().numpy().astype(np.complex128), ref)
        print(f"[{plans}] member {i} ({m.n}^3): psi rel L2 {err:.2e}, t = {e['t']:.3e}")
        assert err < 1e-5
        assert e["t"] == pytest.approx(steps * m.dt, rel=1e-12)
        assert np.max(np.abs(periodic_diff(p.cpu().numpy().astype(np.float64), pr))) < 1e-6
    plan.close()


def test_ensemble_member_equals_single_plan(wdm):
    # a member advanced inside an ensemble equals the same box advanced alone
    a = inputs.ensemble_member(seed=3, n=64, n_particles=0)
    b = inputs.ensemble_member(seed=4, n=32, n_particles=0)
    cfg_a = wdm.make_config(64)
    cfg_b = wdm.make_config(32)
    ens = wdm.Plan([cfg_a, cfg_b])
    one = wdm.Plan(cfg_a)
    pa = torch.from_numpy(a.psi.astype(np.complex64)).cuda()
    pb = torch.from_numpy(b.psi.astype(np.complex64)).cuda()
    wdm.wdm_set_state(ens.handle, 0, pa)
    wdm.wdm_set_state(ens.handle, 1, pb)
    wdm.wdm_set_state(one.handle, 0, pa)
    wdm.wdm_step(ens.handle, 5, a.dt)
    wdm.wdm_step(one.handle, 5, a.dt)
    x = torch.empty_like(pa)
    y = torch.empty_like(pa)
    wdm.wdm_get_psi(ens.handle, 0, x)
    wdm.wdm_get_psi(one.handle, 0, y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    ens.close()
    one.close()
