"""Oracle pins for the local self-interaction (Sec. 2.2, 2.4: the kick
potential becomes Phi + kappa |psi|^2) and the absorbing boundary mask
(Sec. 3.1, Algorithm 1: psi <- psi * B after the second half kick), against
exact solutions, the mask's special values and symmetries, and invariants.
"""
import math

import numpy as np
import pytest

from paper_2606_25026_amd import inputs

TWO_PI = 2.0 * math.pi


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def coords(n, L):
    return np.arange(n) * (L / n)


@pytest.mark.parametrize("kappa,eta", [(0.7, 1.0), (-1.3, 0.6)])
def test_self_interaction_single_plane_wave_is_exact(orc, kappa, eta):
    # |psi|^2 = A^2 is uniform, so Phi = 0 (mean removed) and every step only
    # adds the phase -(eta |k|^2 / 2 + kappa A^2 / eta) dt: exact for any dt
    n, L, A = 16, 1.0, 0.8
    x = coords(n, L)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    k = TWO_PI * np.array([2.0, -1.0, 3.0]) / L
    psi0 = A * np.exp(1j * (k[0] * X + k[1] * Y + k[2] * Z))
    cfg = orc.make_config((n,) * 3, hbar_over_m=eta, four_pi_G=5.0, kappa=kappa)
    steps, dt = 40, 2.5e-4
    psi, _, _ = orc.kdk(cfg, psi0, nsteps=steps, dt=dt)
    t = steps * dt
    exact = psi0 * np.exp(-1j * (0.5 * eta * (k @ k) + kappa * A * A / eta) * t)
    assert rel_l2(psi, exact) < 1e-11


def test_self_interaction_is_unitary_and_reversible(orc):
    wl = inputs.plane_wave_box(16, seed=5)
    cfg = orc.make_config((16,) * 3, four_pi_G=3.0, kappa=0.9)
    m0 = orc.energy(cfg, wl.psi)["mass"]
    psi, _, _ = orc.kdk(cfg, wl.psi, nsteps=50, dt=1e-3)
    assert orc.energy(cfg, psi)["mass"] == pytest.approx(m0, rel=1e-12)
    back, _, _ = orc.kdk(cfg, psi, nsteps=50, dt=-1e-3)
    assert rel_l2(back, wl.psi) < 1e-10


def test_self_interaction_energy_is_conserved_to_second_order(orc):
    # the contact term kappa/2 int |psi|^4 completes the Hamiltonian, so the
    # KDK energy error stays O(dt^2); without it the "energy" would drift at O(1)
    wl = inputs.plane_wave_box(16, seed=3)
    cfg = orc.make_config((16,) * 3, four_pi_G=10.0, kappa=2.0)
    e0 = orc.energy(cfg, wl.psi)
    assert e0["e_self"] == pytest.approx(
        0.5 * 2.0 * np.sum(np.abs(wl.psi) ** 4) / 16 ** 3, rel=1e-13)
    drifts = []
    for n in (20, 40, 80):
        psi, _, _ = orc.kdk(cfg, wl.psi, nsteps=n, dt=0.005 / n)
        e1 = orc.energy(cfg, psi)
        drifts.append(abs(e1["e_total"] - e0["e_total"]))
    assert abs(drifts[0] / drifts[1] - 4) < 0.2 and abs(drifts[1] / drifts[2] - 4) < 0.2
    # the contact energy itself moves far more than the total's error
    assert abs(e1["e_self"] - e0["e_self"]) > 100 * drifts[2]


def test_absorbing_mask_special_values_and_symmetry(orc):
    n, L, alpha, nb, dt = 32, 1.0, 10.0, 50.0, 3e-3   # n_b = 50: the paper's default
    cfg = orc.make_config((n,) * 3, L=L, absorb_alpha=alpha, absorb_nb=nb)
    B = orc.absorb_mask(cfg, dt)
    c = n // 2
    # interior ~ 1 (every tanh saturated), a face exp(-alpha dt), a corner
    # exp(-3 alpha dt): each axis contributes 0 inside and 1 on its faces
    assert B[c, c, c] == pytest.approx(1.0, abs=1e-12)
    assert B[0, c, c] == pytest.approx(math.exp(-alpha * dt), rel=1e-9)
    assert B[c, 0, c] == pytest.approx(math.exp(-alpha * dt), rel=1e-9)
    assert B[c, c, 0] == pytest.approx(math.exp(-alpha * dt), rel=1e-9)
    assert B[0, 0, 0] == pytest.approx(math.exp(-3 * alpha * dt), rel=1e-9)
    # mirror symmetry about the box centre (node i <-> node n - i) per axis
    idx = (-np.arange(n)) % n
    assert np.allclose(B, B[idx, :, :], rtol=0, atol=1e-15)
    assert np.allclose(B, B[:, idx, :], rtol=0, atol=1e-15)
    assert np.allclose(B, B[:, :, idx], rtol=0, atol=1e-15)
    # separable and monotone: the factor falls from the centre to each face
    line = B[:, c, c]
    assert np.all(np.diff(line[c::-1]) <= 1e-15)
    assert B[3, 5, 7] == pytest.approx(B[3, c, c] * B[c, 5, c] * B[c, c, 7], rel=1e-12)
    # the layer scales with n_b: a wider layer absorbs more a quarter box in
    wide = orc.absorb_mask(orc.make_config((n,) * 3, absorb_alpha=alpha, absorb_nb=4.0), dt)
    assert wide[n // 4, c, c] < B[n // 4, c, c] < 1.0
    # a step of -dt gives the reciprocal factor
    inv = orc.absorb_mask(cfg, -dt)
    assert np.allclose(B * inv, 1.0, rtol=0, atol=1e-14)


def test_absorbing_mask_acts_once_per_step_after_the_kick(orc):
    # a uniform field has uniform density (Phi = 0) and only a k = 0 mode (the
    # drift leaves it alone), so one step is exactly the mask
    n, alpha, nb, dt = 16, 20.0, 6.0, 2e-3
    cfg = orc.make_config((n,) * 3, four_pi_G=4.0, absorb_alpha=alpha, absorb_nb=nb)
    psi0 = np.full((n,) * 3, 0.7 + 0.2j)
    psi1, _, _ = orc.kdk(cfg, psi0, nsteps=1, dt=dt)
    B = orc.absorb_mask(cfg, dt)
    assert np.max(np.abs(psi1 - B * psi0)) < 1e-14
    # the mass lost in the step is the masked mass
    e = orc.energy(cfg, psi1)
    assert e["mass"] == pytest.approx(np.sum(B ** 2) * abs(0.7 + 0.2j) ** 2 / n ** 3, rel=1e-13)
    # a field reaching the layer loses mass
    wl = inputs.plane_wave_box(n, seed=2)
    psi, _, _ = orc.kdk(cfg, wl.psi, nsteps=20, dt=dt)
    assert orc.energy(cfg, psi)["mass"] < orc.energy(cfg, wl.psi)["mass"]


def test_dt_auto_self_interaction_term(orc):
    n = 16
    cfg = orc.make_config((n,) * 3, kappa=-50.0)
    psi = np.full((n,) * 3, 2.0 + 0j)
    phi = np.zeros((n,) * 3)
    # kinetic limit 4/(3 pi) dx^2 = 1.66e-3; self-interaction 2 pi / (50 * 4)
    # = 3.1e-2: kinetic wins; with kappa = -5e4 the contact term wins
    kin = 4.0 / (3.0 * math.pi) / n ** 2
    assert orc.dt_auto(cfg, phi, psi) == pytest.approx(0.45 * kin, rel=1e-15)
    cfg = orc.make_config((n,) * 3, kappa=-5e4)
    assert orc.dt_auto(cfg, phi, psi) == pytest.approx(0.45 * TWO_PI / (5e4 * 4.0), rel=1e-14)
