"""Seeded synthetic initial conditions for the wave-DM split-step solver.

This module only *builds inputs*: it holds none of the method's arithmetic
(no kick, drift, Poisson solve, deposit or reduction).  The GPU library and the
FP64 CPU oracle both consume exactly the arrays produced here, so every parity
comparison starts from identical bits.

Everything is drawn from ``numpy.random.default_rng(seed)`` (PCG64) in a fixed
order that is documented per generator.  Grids are node-centred on
``x_i = i * dx`` with ``dx = L / n`` (the periodic reading of the paper's grid,
Sec. 3.1), arrays are C-ordered ``[nx][ny][nz]`` with z contiguous.

The synthetic workloads stand in for the paper's galaxy set-ups (Sec. 4), which
need observational mass models that are not available here:

* ``plane_waves``  -- sum of plane waves, the free/nonlinear Schroedinger test
  field (band limited, so the free evolution is known exactly).
* ``grf_soliton``  -- complex Gaussian random field with power ``exp(-k^2/k0^2)``
  plus a central soliton core ``rho_c / (1 + 0.091 (r/r_c)^2)^8``.
* ``plummer``      -- equal-mass baryon particles drawn from a Plummer sphere
  with isotropic velocities from its distribution function (Aarseth, Henon &
  Wielen 1974 rejection method).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------------------
# plane waves
# ---------------------------------------------------------------------------
@dataclass
class PlaneWaves:
    """A band-limited sum of unit plane waves, scaled to mean |psi|^2 = 1."""

    modes: np.ndarray      # int64 [n_waves][3], integer wave vectors m (k = 2 pi m / L)
    phases: np.ndarray     # float64 [n_waves], uniform in [0, 2 pi)
    scale: float           # amplitude factor applied to every wave
    n: tuple               # grid shape
    L: tuple               # box lengths

    def evaluate(self, t: float = 0.0, hbar_over_m: float = 1.0) -> np.ndarray:
        """psi(x, t) of the *free* equation: each wave carries exp(-i eta k^2 t / 2)."""
        nx, ny, nz = self.n
        lx, ly, lz = self.L
        x = np.arange(nx) * (lx / nx)
        y = np.arange(ny) * (ly / ny)
        z = np.arange(nz) * (lz / nz)
        psi = np.zeros((nx, ny, nz), dtype=np.complex128)
        for m, ph in zip(self.modes, self.phases):
            kx, ky, kz = TWO_PI * m[0] / lx, TWO_PI * m[1] / ly, TWO_PI * m[2] / lz
            omega = 0.5 * hbar_over_m * (kx * kx + ky * ky + kz * kz)
            ex = np.exp(1j * kx * x)
            ey = np.exp(1j * ky * y)
            ez = np.exp(1j * (kz * z + ph - omega * t))
            psi += ex[:, None, None] * ey[None, :, None] * ez[None, None, :]
        return psi * self.scale


def plane_waves(n: int = 32, L: float = 1.0, n_waves: int = 64, m_max: int = 6,
                seed: int = 0) -> PlaneWaves:
    """Draw ``n_waves`` integer wave vectors with Euclidean |m| <= m_max.

    Draw order: for each wave in turn, ``rng.integers(-m_max, m_max+1, 3)``
    repeated until |m| <= m_max (m = 0 and repeats allowed); then
    ``rng.uniform(0, 2 pi, n_waves)`` for the phases.
    """
    rng = np.random.default_rng(seed)
    modes = np.zeros((n_waves, 3), dtype=np.int64)
    for j in range(n_waves):
        while True:
            m = rng.integers(-m_max, m_max + 1, size=3)
            if int(m @ m) <= m_max * m_max:
                modes[j] = m
                break
    phases = rng.uniform(0.0, TWO_PI, size=n_waves)
    pw = PlaneWaves(modes=modes, phases=phases, scale=1.0, n=(n, n, n), L=(L, L, L))
    psi = pw.evaluate(0.0)
    pw.scale = 1.0 / math.sqrt(float(np.mean(np.abs(psi) ** 2)))
    return pw


# ---------------------------------------------------------------------------
# Gaussian random field + soliton
# ---------------------------------------------------------------------------
def _min_image(n: int, L: float) -> np.ndarray:
    """Signed minimum-image offset of node i from the box centre L/2."""
    x = np.arange(n) * (L / n) - 0.5 * L
    return x - L * np.round(x / L)


def grf_soliton(n: int, L: float = 1.0, k0: float = 16.0 * TWO_PI, rc: float = 0.05,
                rho_c: float = 50.0, seed: int = 0, rng: np.random.Generator | None = None
                ) -> np.ndarray:
    """Complex GRF with power spectrum exp(-k^2/k0^2), mean |psi|^2 = 1, plus a soliton.

    Each Fourier mode gets ``(a + i b) exp(-|k|^2 / (2 k0^2))`` with a, b iid N(0,1)
    (no Hermitian symmetry: psi is complex).  Draw order: all ``a`` (shape n^3,
    C order over FFT-ordered mode indices), then all ``b``.  The field is
    inverse transformed with numpy, scaled to mean |psi|^2 = 1, and then the real
    soliton amplitude sqrt(rho_c / (1 + 0.091 (r/rc)^2)^8) is added, r being the
    minimum-image distance to the box centre.  ``k0`` is absolute (2 pi / length).
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n, n))
    b = rng.standard_normal((n, n, n))
    m = np.fft.fftfreq(n, d=1.0 / n)
    k = TWO_PI * m / L
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    spec = (a + 1j * b) * np.exp(-k2 / (2.0 * k0 * k0))
    del a, b, k2
    psi = np.fft.ifftn(spec)
    del spec
    psi *= 1.0 / math.sqrt(float(np.mean(np.abs(psi) ** 2)))
    d = _min_image(n, L)
    r2 = d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2
    psi += np.sqrt(rho_c / (1.0 + 0.091 * r2 / (rc * rc)) ** 8)
    return psi


# ---------------------------------------------------------------------------
# Plummer sphere
# ---------------------------------------------------------------------------
def plummer(n_particles: int, a: float = 0.03, total_mass: float = 0.1,
            G: float = 1.0 / (4.0 * math.pi), L: float = 1.0, r_max: float = 0.4,
            seed: int = 0, rng: np.random.Generator | None = None):
    """Equal-mass particles from a Plummer sphere centred on the box centre.

    Radii from the inverse enclosed-mass fraction r = a / sqrt(u^(-2/3) - 1),
    resampled until r <= r_max; isotropic directions; speeds q * v_esc(r) with q
    drawn from q^2 (1 - q^2)^(7/2) by rejection (Aarseth, Henon & Wielen 1974),
    v_esc = sqrt(2 G M / sqrt(r^2 + a^2)); isotropic velocity directions.

    Draw order: radii in batches of ``n_particles`` uniforms (accepted draws kept
    in order), position cos(theta) then phi, speed pairs (q, y) in batches, then
    velocity cos(theta) then phi.  Returns float32 ``pos, vel`` of shape [Np][3]
    with positions wrapped into [0, L).
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    npart = int(n_particles)
    r = np.empty(0)
    while r.size < npart:
        u = rng.uniform(0.0, 1.0, size=npart)
        u = u[u > 0.0]
        rr = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        r = np.concatenate([r, rr[rr <= r_max]])
    r = r[:npart]
    ct = rng.uniform(-1.0, 1.0, size=npart)
    ph = rng.uniform(0.0, TWO_PI, size=npart)
    st = np.sqrt(1.0 - ct * ct)
    off = np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * ct], axis=1)
    q = np.empty(0)
    while q.size < npart:
        qq = rng.uniform(0.0, 1.0, size=npart)
        yy = rng.uniform(0.0, 0.1, size=npart)
        q = np.concatenate([q, qq[yy < qq * qq * (1.0 - qq * qq) ** 3.5]])
    q = q[:npart]
    vesc = np.sqrt(2.0 * G * total_mass / np.sqrt(r * r + a * a))
    vct = rng.uniform(-1.0, 1.0, size=npart)
    vph = rng.uniform(0.0, TWO_PI, size=npart)
    vst = np.sqrt(1.0 - vct * vct)
    speed = q * vesc
    vel = np.stack([speed * vst * np.cos(vph), speed * vst * np.sin(vph), speed * vct], axis=1)
    pos = (0.5 * L + off) % L
    pos = pos.astype(np.float32)
    pos[pos >= np.float32(L)] = 0.0
    return pos, vel.astype(np.float32)


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------
@dataclass
class Workload:
    """One synthetic run: grid, physics constants, initial state and time step."""

    name: str
    n: int
    L: float
    psi: np.ndarray                 # complex128 [n][n][n]
    pos: np.ndarray | None = None   # float32 [Np][3]
    vel: np.ndarray | None = None
    particle_mass: float = 0.0
    hbar_over_m: float = 1.0
    four_pi_G: float = 1.0
    dt: float = 0.0
    steps: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n_particles(self) -> int:
        return 0 if self.pos is None else int(self.pos.shape[0])


def wave_mass(psi: np.ndarray, L: float) -> float:
    """Total mass sum |psi|^2 dV of an initial field (used only to size particles)."""
    n = psi.shape[0]
    return float(np.sum(np.abs(psi) ** 2)) * (L / n) ** 3


def plane_wave_box(n: int = 32, seed: int = 0, steps: int = 100) -> Workload:
    """32^3 box, 64 plane waves |m| <= 6, no particles, dt = 0.2 dx^2."""
    pw = plane_waves(n=n, seed=seed)
    L = 1.0
    dx = L / n
    return Workload(name=f"plane-waves {n}^3", n=n, L=L, psi=pw.evaluate(0.0),
                    dt=0.2 * dx * dx, steps=steps, extra={"waves": pw})


def coupled_halo(n: int = 256, n_particles: int = 1_000_000, seed: int = 0, rc: float = 0.05,
                 rho_c: float = 50.0, L: float = 1.0, plummer_a: float = 0.03,
                 mass_fraction: float = 0.1, steps: int = 1000, k0_modes: float = 16.0) -> Workload:
    """GRF (k0 = k0_modes * 2 pi / L, 16 in the workloads) + soliton halo with a
    Plummer sphere of baryons.

    The particles' total mass is ``mass_fraction`` of the wave mass; one
    generator stream feeds the field first and the particles second.
    """
    rng = np.random.default_rng(seed)
    psi = grf_soliton(n, L=L, k0=k0_modes * TWO_PI / L, rc=rc, rho_c=rho_c, rng=rng)
    mw = wave_mass(psi, L)
    pos = vel = None
    mp = 0.0
    if n_particles > 0:
        mtot = mass_fraction * mw
        pos, vel = plummer(n_particles, a=plummer_a, total_mass=mtot, L=L, rng=rng)
        mp = mtot / n_particles
    dx = L / n
    return Workload(name=f"coupled halo {n}^3 + {n_particles} particles", n=n, L=L, psi=psi,
                    pos=pos, vel=vel, particle_mass=mp, dt=0.2 * dx * dx, steps=steps,
                    extra={"rc": rc, "rho_c": rho_c, "wave_mass": mw})


def ensemble_member(seed: int, n: int, n_particles: int = 10_000) -> Workload:
    """One member of the mixed-size ensemble: r_c ~ U[0.03, 0.08] drawn first."""
    rng = np.random.default_rng(seed)
    rc = float(rng.uniform(0.03, 0.08))
    L = 1.0
    psi = grf_soliton(n, L=L, k0=16.0 * TWO_PI / L, rc=rc, rho_c=50.0, rng=rng)
    mw = wave_mass(psi, L)
    mtot = 0.1 * mw
    pos = vel = None
    if n_particles > 0:
        pos, vel = plummer(n_particles, a=0.03, total_mass=mtot, L=L, rng=rng)
    dx = L / n
    return Workload(name=f"ensemble member seed {seed} {n}^3", n=n, L=L, psi=psi, pos=pos,
                    vel=vel, particle_mass=mtot / n_particles if n_particles else 0.0,
                    dt=0.2 * dx * dx, steps=100, extra={"rc": rc, "seed": seed})


ENSEMBLE_SIZES = (64,) * 16 + (96,) * 16 + (128,) * 16
