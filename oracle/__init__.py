"""FP64 CPU oracle of the Schroedinger-Poisson KDK split step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the slow, plain reference that the GPU library is
checked against.  Only ``tests/``, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product path never does.  It shares no code
with the GPU library.

Every function here marshals numpy arrays into ``liboracle.so`` (C++17, FP64,
built by :func:`build`).  Parity is unpinned nowhere except where a function's
docstring says so.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
# ORACLE_LIB selects another build of the same sources (the sanitized one)
LIB = Path(os.environ.get("ORACLE_LIB", HERE / "liboracle.so"))
SAN_LIB = HERE / "liboracle_san.so"
SOURCES = ["fft.cpp", "spe.cpp", "analysis.cpp"]


def build(verbose: bool = False, sanitize: bool = False) -> Path:
    """Compile the oracle with g++ -O2 (no fast-math) into oracle/liboracle.so;
    with ``sanitize``, an AddressSanitizer + UndefinedBehaviorSanitizer build
    (-O1, halting on the first report) into oracle/liboracle_san.so, which a
    process loads with libasan preloaded and ORACLE_LIB pointing at it."""
    out = SAN_LIB if sanitize else HERE / "liboracle.so"
    opt = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"])
    cmd = ["g++", *opt, "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall",
           "-o", str(out) + ".tmp"] + [str(HERE / s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(str(out) + ".tmp", out)
    return out


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("hbar_over_m", C.c_double), ("four_pi_G", C.c_double),
                ("n_particles", C.c_int64), ("particle_mass", C.c_double),
                ("kappa", C.c_double), ("absorb_alpha", C.c_double), ("absorb_nb", C.c_double),
                ("baryon_mode", C.c_int32), ("nbody_substeps", C.c_int32),
                ("boundary", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB.exists():
            build(sanitize=LIB == SAN_LIB)
        L = C.CDLL(str(LIB))
        dp, ip = C.POINTER(C.c_double), C.c_int
        L.orc_set_threads.argtypes = [ip]
        L.orc_set_threads.restype = ip
        L.orc_get_threads.restype = ip
        L.orc_fft1d.argtypes = [dp, ip, ip]
        L.orc_fft3d.argtypes = [dp, ip, ip, ip, ip]
        L.orc_dft3d_brute.argtypes = [dp, dp, ip, ip, ip, ip]
        cp = C.POINTER(Config)
        L.orc_poisson.argtypes = [cp, dp, dp]
        L.orc_cic_deposit.argtypes = [cp, dp, dp]
        L.orc_cic_force.argtypes = [cp, dp, dp, dp]
        L.orc_potential.argtypes = [cp, dp, dp, dp]
        L.orc_kdk.argtypes = [cp, dp, dp, dp, C.c_int64, C.c_double]
        L.orc_energy.argtypes = [cp, dp, dp, dp, dp]
        L.orc_paper_energies.argtypes = [cp, dp, dp, dp]
        L.orc_dt_auto.argtypes = [cp, dp, dp, C.c_double, C.c_double]
        L.orc_absorb_mask.argtypes = [cp, C.c_double, dp]
        L.orc_mass_fraction_radii.argtypes = [cp, dp, C.POINTER(C.c_int32), dp, ip, dp]
        L.orc_mass_fraction_radii.restype = ip
        L.orc_kdk_ext.argtypes = [cp, dp, dp, dp, C.c_int64, C.c_double, dp]
        L.orc_poisson_direct.argtypes = [cp, dp, dp]
        L.orc_poisson_direct_at.argtypes = [cp, dp, C.POINTER(C.c_int64), C.c_int64, dp]
        L.orc_cube_self_integral.restype = C.c_double
        L.orc_tidal_correct.argtypes = [cp, dp, dp]
        L.orc_energy_ext.argtypes = [cp, dp, dp, dp, dp, dp]
        L.orc_dt_auto.restype = C.c_double
        L.orc_power_spectrum.argtypes = [dp, ip, ip, dp, C.POINTER(C.c_int64)]
        L.orc_restrict.argtypes = [dp, ip, dp, ip]
        L.orc_conv3d_fwd.argtypes = [dp, dp, dp, dp, ip, ip, ip]
        L.orc_conv3d_bwd.argtypes = [dp, dp, dp, dp, dp, dp, ip, ip, ip]
        L.orc_round_bf16.argtypes = [dp, C.c_int64]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int = 0) -> int:
    return lib().orc_set_threads(int(n))


def get_threads() -> int:
    return lib().orc_get_threads()


BARYON_DYNAMIC, BARYON_STATIC = 0, 1
BOUNDARY_PERIODIC, BOUNDARY_VACUUM = 0, 1


def make_config(shape, L=1.0, hbar_over_m=1.0, four_pi_G=1.0, n_particles=0,
                particle_mass=0.0, kappa=0.0, absorb_alpha=0.0, absorb_nb=50.0,
                baryon_mode=BARYON_DYNAMIC, nbody_substeps=1,
                boundary=BOUNDARY_PERIODIC) -> Config:
    if isinstance(L, (int, float)):
        L = (float(L),) * 3
    nx, ny, nz = shape
    return Config(nx, ny, nz, L[0], L[1], L[2], hbar_over_m, four_pi_G, int(n_particles),
                  float(particle_mass), float(kappa), float(absorb_alpha), float(absorb_nb),
                  int(baryon_mode), int(nbody_substeps), int(boundary))


def fft1d(x, sign=-1):
    a = _c128(x).copy()
    if lib().orc_fft1d(_p(a.view(np.float64)), a.shape[0], sign) != 0:
        raise ValueError("unsupported length")
    return a


def fft3d(x, sign=-1):
    a = _c128(x).copy()
    if lib().orc_fft3d(_p(a.view(np.float64)), *a.shape, sign) != 0:
        raise ValueError("unsupported shape")
    return a


def dft3d_brute(x, sign=-1):
    a = _c128(x)
    out = np.empty_like(a)
    lib().orc_dft3d_brute(_p(a.view(np.float64)), _p(out.view(np.float64)), *a.shape, sign)
    return out


def poisson(cfg: Config, rho):
    r = _f64(rho)
    phi = np.empty_like(r)
    lib().orc_poisson(C.byref(cfg), _p(r), _p(phi))
    return phi


def cic_deposit(cfg: Config, pos):
    p = _f64(pos)
    out = np.empty((cfg.nx, cfg.ny, cfg.nz))
    lib().orc_cic_deposit(C.byref(cfg), _p(p), _p(out))
    return out


def cic_force(cfg: Config, phi, pos):
    p = _f64(pos)
    acc = np.empty_like(p)
    lib().orc_cic_force(C.byref(cfg), _p(_f64(phi)), _p(p), _p(acc))
    return acc


def potential(cfg: Config, psi, pos=None):
    a = _c128(psi)
    phi = np.empty(a.shape)
    lib().orc_potential(C.byref(cfg), _p(a.view(np.float64)),
                        _p(_f64(pos)) if pos is not None else None, _p(phi))
    return phi


def kdk(cfg: Config, psi, pos=None, vel=None, nsteps=1, dt=1e-4, phi_ext=None):
    """Run ``nsteps`` unmerged KDK steps; returns new (psi, pos, vel) arrays.
    ``phi_ext``: external potential already passed through tidal_correct."""
    a = _c128(psi).copy()
    p = _f64(pos).copy() if pos is not None else None
    v = _f64(vel).copy() if vel is not None else None
    ext = _f64(phi_ext) if phi_ext is not None else None
    lib().orc_kdk_ext(C.byref(cfg), _p(a.view(np.float64)), _p(p), _p(v), int(nsteps),
                      float(dt), _p(ext) if ext is not None else None)
    return a, p, v


def poisson_direct(cfg: Config, rho):
    """Isolated potential by direct summation (small grids only)."""
    r = _f64(rho)
    phi = np.empty_like(r)
    lib().orc_poisson_direct(C.byref(cfg), _p(r), _p(phi))
    return phi


def poisson_direct_at(cfg: Config, rho, nodes):
    """Isolated potential by direct summation at the listed (i, j, k) nodes."""
    r = _f64(rho)
    nd = np.ascontiguousarray(np.asarray(nodes, dtype=np.int64).reshape(-1, 3))
    phi = np.empty(nd.shape[0])
    lib().orc_poisson_direct_at(C.byref(cfg), _p(r), nd.ctypes.data_as(C.POINTER(C.c_int64)),
                                nd.shape[0], _p(phi))
    return phi


def cube_self_integral() -> float:
    return float(lib().orc_cube_self_integral())


def tidal_correct(cfg: Config, phi_ext):
    """External potential with its mean acceleration removed (Sec. 4.3)."""
    a = _f64(phi_ext)
    out = np.empty_like(a)
    lib().orc_tidal_correct(C.byref(cfg), _p(a), _p(out))
    return out


ENERGY_FIELDS = ("mass", "e_kin", "e_pot", "e_kin_particles", "e_total", "px", "py", "pz",
                 "max_abs_phi", "e_self", "max_rho", "e_ext")


def energy(cfg: Config, psi, pos=None, vel=None, phi_ext=None) -> dict:
    out = np.zeros(12)
    ext = _f64(phi_ext) if phi_ext is not None else None
    lib().orc_energy_ext(C.byref(cfg), _p(_c128(psi).view(np.float64)),
                         _p(_f64(pos)) if pos is not None else None,
                         _p(_f64(vel)) if vel is not None else None,
                         _p(ext) if ext is not None else None, _p(out))
    return dict(zip(ENERGY_FIELDS, out.tolist()))


def paper_energies(cfg: Config, psi, phi) -> dict:
    """The paper's K, Q, V, 2K + 2Q + V and the wave momentum (Sec. 3.6)."""
    out = np.zeros(7)
    lib().orc_paper_energies(C.byref(cfg), _p(_c128(psi).view(np.float64)), _p(_f64(phi)),
                             _p(out))
    return dict(zip(("K", "Q", "V", "virial", "Px", "Py", "Pz"), out.tolist()))


MASS_FRACTIONS = tuple(0.1 * f for f in range(1, 10))


def mass_fraction_radii(cfg: Config, psi, centre=None, fractions=MASS_FRACTIONS) -> np.ndarray:
    """Radii enclosing the given fractions of the wave mass (App. A.1.2)."""
    if centre is None:
        centre = (cfg.nx // 2, cfg.ny // 2, cfg.nz // 2)
    cen = (C.c_int32 * 3)(*centre)
    fr = np.ascontiguousarray(fractions, dtype=np.float64)
    out = np.zeros(len(fr))
    if lib().orc_mass_fraction_radii(C.byref(cfg), _p(_c128(psi).view(np.float64)), cen,
                                     _p(fr), len(fr), _p(out)) != 0:
        raise ValueError("mass-fraction radii need cubic cells")
    return out


def dt_auto(cfg: Config, phi, psi=None, zeta=0.9, c_kin=4.0 / (3.0 * np.pi)) -> float:
    """CFL step of Sec. 3.5: zeta * 0.5 * min{c_kin dx^2 / eta, 2 pi eta / max|Phi|,
    2 pi eta / (|kappa| max|psi|^2)}.  Each term is the step over which the grid's
    fastest drift mode, the kick at the deepest node, or the self-interaction kick
    turns the phase by pi (pinned through one oracle step each); the printed
    kinetic constant 4 / (3 pi) is itself a reading of the paper."""
    ps = _c128(psi).view(np.float64) if psi is not None else None
    return float(lib().orc_dt_auto(C.byref(cfg), _p(_f64(phi)), _p(ps), zeta, c_kin))


def absorb_mask(cfg: Config, dt) -> np.ndarray:
    """The absorbing boundary factor B of one step (Sec. 3.1, Algorithm 1)."""
    out = np.zeros((cfg.nx, cfg.ny, cfg.nz))
    lib().orc_absorb_mask(C.byref(cfg), float(dt), _p(out))
    return out


def power_spectrum(rho, nbins=None):
    r = _f64(rho)
    n = r.shape[0]
    nbins = nbins or (n // 2)
    pk = np.zeros(nbins)
    cnt = np.zeros(nbins, dtype=np.int64)
    lib().orc_power_spectrum(_p(r), n, nbins, _p(pk), cnt.ctypes.data_as(C.POINTER(C.c_int64)))
    return pk, cnt


def restrict(fine, nc):
    f = _c128(fine)
    out = np.empty((nc, nc, nc), dtype=np.complex128)
    lib().orc_restrict(_p(f.view(np.float64)), f.shape[0], _p(out.view(np.float64)), nc)
    return out


def conv3d_fwd(x, w, b):
    x = _f64(x)
    w = _f64(w)
    b = _f64(b)
    cin, n = x.shape[0], x.shape[1]
    cout = w.shape[0]
    y = np.empty((cout, n, n, n))
    lib().orc_conv3d_fwd(_p(x), _p(w), _p(b), _p(y), n, cin, cout)
    return y


def conv3d_bwd(x, w, dy, want_dx=True):
    x = _f64(x)
    w = _f64(w)
    dy = _f64(dy)
    cin, n = x.shape[0], x.shape[1]
    cout = w.shape[0]
    dx = np.empty_like(x) if want_dx else None
    dw = np.empty_like(w)
    db = np.empty(cout)
    lib().orc_conv3d_bwd(_p(x), _p(w), _p(dy), _p(dx) if want_dx else None, _p(dw), _p(db), n,
                         cin, cout)
    return dx, dw, db


def round_bf16(v):
    a = _f64(v).copy()
    lib().orc_round_bf16(_p(a), a.size)
    return a
