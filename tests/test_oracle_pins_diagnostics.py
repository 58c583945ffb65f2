"""CPU pins of the oracle's diagnostics (Sec. 3.6, App. A.1): the paper's K, Q,
V and virial sum, the wave momentum, and the mass-fraction radii.

K, Q and the momentum use second-order central differences on the nodes, so
for smooth fields they converge to their continuum integrals as dx^2: pinned
against closed forms of a Gaussian density with a uniform phase gradient
(K = eta^2 k0^2 M / 2, P = eta k0 M, Q = 3 (2 pi)^(3/2) sigma A^2 / 4).  The
radii are pinned by exact cases (a point mass, single shells), by a brute
force over a random field, by translation covariance and by the quantiles of
the chi distribution with three degrees of freedom for a Gaussian.
"""
import math

import numpy as np
import pytest
from scipy.stats import chi

SIG = 0.08


def gaussian_state(n, k0=(0.0, 0.0, 0.0), eta=1.0, sig=SIG):
    x = np.arange(n) / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2
    amp = np.exp(-r2 / (4 * sig * sig))
    phase = 2 * math.pi * (k0[0] * X + k0[1] * Y + k0[2] * Z)
    return amp * np.exp(1j * phase)


def test_quantum_gradient_energy_converges_to_closed_form(orc):
    exact = 3 * (2 * math.pi) ** 1.5 * SIG / 4
    errs = []
    for n in (32, 64, 128):
        cfg = orc.make_config((n,) * 3)
        errs.append(orc.paper_energies(cfg, gaussian_state(n), np.zeros((n,) * 3))["Q"] - exact)
    assert abs(errs[-1]) < 3e-3 * exact
    for a, b in zip(errs, errs[1:]):
        assert 3.6 < a / b < 4.4, errs


@pytest.mark.parametrize("eta", [1.0, 0.5])
def test_flow_energy_and_momentum_of_a_moving_gaussian(orc, eta):
    m = (3, -2, 1)
    k0 = 2 * math.pi * np.array(m, dtype=float)
    errs_k, errs_p = [], []
    for n in (32, 64, 128):
        cfg = orc.make_config((n,) * 3, hbar_over_m=eta)
        psi = gaussian_state(n, m)
        mass = float(np.sum(np.abs(psi) ** 2)) / n ** 3
        d = orc.paper_energies(cfg, psi, np.zeros((n,) * 3))
        errs_k.append(d["K"] / (0.5 * eta ** 2 * (k0 @ k0) * mass) - 1)
        p = np.array([d["Px"], d["Py"], d["Pz"]])
        errs_p.append(np.max(np.abs(p / (eta * k0 * mass) - 1)))
        # the phase carries no density gradient: Q is that of the amplitude
        q0 = orc.paper_energies(cfg, np.abs(psi), np.zeros((n,) * 3))
        assert d["Q"] == pytest.approx(q0["Q"], rel=1e-12) and q0["K"] == 0.0
    assert abs(errs_k[-1]) < 1e-2 and errs_p[-1] < 1e-2
    for errs in (errs_k, errs_p):
        for a, b in zip(errs, errs[1:]):
            assert 3.6 < a / b < 4.4, errs


def test_potential_term_and_virial_sum(orc):
    n = 32
    cfg = orc.make_config((n,) * 3)
    psi = gaussian_state(n, (1, 0, 0))
    mass = float(np.sum(np.abs(psi) ** 2)) / n ** 3
    d = orc.paper_energies(cfg, psi, np.full((n,) * 3, -2.5))
    assert d["V"] == pytest.approx(-2.5 * mass, rel=1e-13)
    assert d["virial"] == pytest.approx(2 * d["K"] + 2 * d["Q"] + d["V"], rel=1e-14)


# ------------------------------------------------------------------ radii
def test_radii_of_point_mass_and_single_shell(orc):
    n = 16
    cfg = orc.make_config((n,) * 3)
    psi = np.zeros((n,) * 3, complex)
    psi[8, 8, 8] = 2.0
    assert np.all(orc.mass_fraction_radii(cfg, psi) == 0.0)
    # the 24 nodes at s = 5 (permutations of (+-1, +-2, 0)); other centre
    psi[:] = 0
    c = (3, 14, 7)
    for d in [(1, 2, 0), (2, 1, 0), (1, 0, 2), (2, 0, 1), (0, 1, 2), (0, 2, 1)]:
        for sx in (1, -1):
            for sy in (1, -1):
                idx = [c[0] + sx * d[0], c[1] + sy * d[1], c[2] + d[2]]
                idx2 = [c[0] + sx * d[0], c[1] + d[1], c[2] + sy * d[2]]
                for q in (idx, idx2):
                    psi[q[0] % n, q[1] % n, q[2] % n] = 1.0
    r = orc.mass_fraction_radii(cfg, psi, centre=c)
    assert np.allclose(r, math.sqrt(5) / n, rtol=0, atol=1e-15)


def test_radii_two_shells_split_by_fraction(orc):
    n = 16
    cfg = orc.make_config((n,) * 3)
    psi = np.zeros((n,) * 3, complex)
    psi[9, 8, 8] = math.sqrt(0.35)       # s = 1, mass 0.35
    psi[8, 8, 11] = math.sqrt(0.65)      # s = 9, mass 0.65
    r = orc.mass_fraction_radii(cfg, psi)
    expect = [1 / n if f <= 0.35 else 3 / n for f in orc.MASS_FRACTIONS]
    assert np.allclose(r, expect, rtol=0, atol=1e-15)


def brute_radii(psi, centre, fractions, dx):
    """Nodes sorted by distance; the first node whose running mass reaches f M."""
    n = np.array(psi.shape)
    idx = np.indices(psi.shape).reshape(3, -1).T
    d = (idx - np.array(centre)) % n
    d = np.minimum(d, n - d)
    s = (d * d).sum(axis=1)
    m = (np.abs(psi) ** 2).ravel()
    order = np.argsort(s, kind="stable")
    s_sorted, cum = s[order], np.cumsum(m[order])
    return np.array([dx * math.sqrt(s_sorted[np.nonzero(cum >= f * cum[-1])[0][0]])
                     for f in fractions])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_radii_brute_force_and_translation(orc, seed):
    rng = np.random.default_rng(seed)
    n = 12
    psi = rng.standard_normal((n,) * 3) + 1j * rng.standard_normal((n,) * 3)
    psi *= np.exp(-rng.uniform(0, 3, (n,) * 3))
    cfg = orc.make_config((n,) * 3, L=2.0)
    centre = tuple(int(v) for v in rng.integers(0, n, 3))
    fr = np.sort(rng.uniform(0.05, 0.95, 9))
    r = orc.mass_fraction_radii(cfg, psi, centre=centre, fractions=fr)
    assert np.array_equal(r, brute_radii(psi, centre, fr, 2.0 / n))
    shift = (5, -3, 7)
    moved = np.roll(psi, shift, axis=(0, 1, 2))
    c2 = tuple((c + s) % n for c, s in zip(centre, shift))
    assert np.array_equal(orc.mass_fraction_radii(cfg, moved, centre=c2, fractions=fr), r)


def test_radii_of_a_gaussian_follow_the_chi3_quantiles(orc):
    n = 64
    cfg = orc.make_config((n,) * 3)
    r = orc.mass_fraction_radii(cfg, gaussian_state(n))
    # |psi|^2 = exp(-r^2 / (2 sig^2)): the enclosed-mass radius is chi(3) * sig
    exact = chi(3).ppf(np.array(orc.MASS_FRACTIONS)) * SIG
    assert np.all(np.abs(r - exact) < 0.6 / n), (r - exact) * n


def test_radii_need_cubic_cells(orc):
    cfg = orc.make_config((16, 16, 32))
    with pytest.raises(ValueError):
        orc.mass_fraction_radii(cfg, np.ones((16, 16, 32), complex))
