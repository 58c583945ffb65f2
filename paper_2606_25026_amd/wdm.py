"""ctypes binding of libwdm (include/wdm.h): argument marshalling only.

Every function has the name of the C entry point it wraps, takes torch
tensors (or raw integer device pointers) where the C call takes device
pointers, raises :class:`WdmError` with ``wdm_last_error()`` on a non-zero
status, and does no arithmetic of its own.  The shared library must have been
built in-tree (``__graft_entry__.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libwdm.so"

WDM_C64, WDM_C128 = 0, 1
WDM_BARYON_DYNAMIC, WDM_BARYON_STATIC = 0, 1
WDM_BOUNDARY_PERIODIC, WDM_BOUNDARY_VACUUM = 0, 1
WDM_DETERMINISTIC_DEPOSIT, WDM_STRICT_CFL = 0x1, 0x2
STATUS = {0: "WDM_OK", 1: "WDM_EINVAL", 2: "WDM_ENOMEM", 3: "WDM_EDEVICE", 4: "WDM_ESTATE",
          5: "WDM_EUNSTABLE", 6: "WDM_EUNSUPPORTED"}


class WdmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class wdm_config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("hbar_over_m", C.c_double), ("four_pi_G", C.c_double),
                ("n_particles", C.c_int64), ("particle_mass", C.c_double),
                ("precision", C.c_int32), ("flags", C.c_uint32),
                ("kappa", C.c_double), ("absorb_alpha", C.c_double), ("absorb_nb", C.c_double),
                ("baryon_mode", C.c_int32), ("nbody_substeps", C.c_int32),
                ("boundary", C.c_int32), ("external_potential", C.c_int32)]


class wdm_energy_t(C.Structure):
    _fields_ = [("mass", C.c_double), ("e_kin", C.c_double), ("e_pot", C.c_double),
                ("e_kin_particles", C.c_double), ("e_total", C.c_double),
                ("momentum", C.c_double * 3), ("max_abs_phi", C.c_double), ("t", C.c_double),
                ("dt", C.c_double), ("dt_auto", C.c_double), ("e_self", C.c_double),
                ("max_rho", C.c_double), ("e_ext", C.c_double), ("cfl_ratio", C.c_double)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "momentum"}
        d["momentum"] = list(self.momentum)
        return d


class wdm_diagnostics_t(C.Structure):
    _fields_ = [("K", C.c_double), ("Q", C.c_double), ("V", C.c_double), ("virial", C.c_double),
                ("momentum", C.c_double * 3), ("mass", C.c_double), ("radii", C.c_double * 9)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("momentum", "radii")}
        d["momentum"] = list(self.momentum)
        d["radii"] = list(self.radii)
        return d


class wdm_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int64), ("total_ms", C.c_double)]


_lib = None
_vp, _i32, _i64, _f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
_SIGS = {
    "wdm_workspace_bytes": (C.c_size_t, [C.POINTER(wdm_config), _i32]),
    "wdm_plan_create": (C.c_int, [C.POINTER(wdm_config), _i32, _vp, C.c_size_t, _vp,
                                  C.POINTER(_vp)]),
    "wdm_plan_destroy": (C.c_int, [_vp]),
    "wdm_set_state": (C.c_int, [_vp, _i32, _vp, _vp, _vp, _f64]),
    "wdm_set_member_dt": (C.c_int, [_vp, _i32, _f64]),
    "wdm_step": (C.c_int, [_vp, _i64, _f64]),
    "wdm_get_psi": (C.c_int, [_vp, _i32, _vp]),
    "wdm_density": (C.c_int, [_vp, _i32, _vp, _i32]),
    "wdm_potential": (C.c_int, [_vp, _i32, _vp]),
    "wdm_energy": (C.c_int, [_vp, _i32, C.POINTER(wdm_energy_t)]),
    "wdm_diagnostics": (C.c_int, [_vp, _i32, C.POINTER(C.c_int32), C.POINTER(wdm_diagnostics_t)]),
    "wdm_set_external_potential": (C.c_int, [_vp, _i32, _vp]),
    "wdm_particles": (C.c_int, [_vp, _i32, _vp, _vp]),
    "wdm_fft3d": (C.c_int, [_vp, _i32, _i32]),
    "wdm_fft3d_noalloc": (C.c_int, [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _vp]),
    "wdm_set_sort_interval": (C.c_int, [_vp, _i32]),
    "wdm_use_graphs": (C.c_int, [_vp, _i32]),
    "wdm_autotune": (C.c_int, [_vp, _i32]),
    "wdm_tuning_entries": (_i32, [_vp]),
    "wdm_get_tuning": (C.c_int, [_vp, C.POINTER(_i32), _i32]),
    "wdm_set_tuning": (C.c_int, [_vp, C.POINTER(_i32), _i32]),
    "wdm_profile": (C.c_int, [_vp, _i32]),
    "wdm_profile_read": (C.c_int, [_vp, C.POINTER(wdm_kernel_stat), _i32, C.POINTER(_i32)]),
    "wdm_copy_bandwidth": (C.c_int, [_vp, _vp, C.c_size_t, _i32, _vp, C.POINTER(_f64)]),
    "wdm_restrict": (C.c_int, [_vp, _i32, _vp, _i32, _vp]),
    "wdm_power_spectrum": (C.c_int, [_vp, _i32, _i32, C.POINTER(_f64), C.POINTER(_i64)]),
    "wdm_distance": (C.c_int, [_vp, _i32, _vp, C.POINTER(_f64)]),
    "wdm_net_param_count": (_i32, []),
    "wdm_net_workspace_bytes": (C.c_size_t, [_i32]),
    "wdm_net_create": (C.c_int, [_i32, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "wdm_net_destroy": (C.c_int, [_vp]),
    "wdm_net_set_params": (C.c_int, [_vp, C.POINTER(C.c_float)]),
    "wdm_net_get_params": (C.c_int, [_vp, C.POINTER(C.c_float)]),
    "wdm_net_get_grads": (C.c_int, [_vp, C.POINTER(C.c_float)]),
    "wdm_net_forward": (C.c_int, [_vp, _vp, _vp]),
    "wdm_net_backward": (C.c_int, [_vp, _vp]),
    "wdm_net_mse_backward": (C.c_int, [_vp, _vp, C.POINTER(_f64)]),
    "wdm_net_adam": (C.c_int, [_vp, _f64, _f64, _f64, _f64]),
    "wdm_net_apply": (C.c_int, [_vp, _vp, _i32]),
    "wdm_net_set_scales": (C.c_int, [_vp, _f64, _f64, _f64]),
    "wdm_net_get_scales": (C.c_int, [_vp, C.POINTER(_f64)]),
    "wdm_net_fit_scales": (C.c_int, [_vp, C.POINTER(_vp), C.POINTER(_vp), _i32]),
    "wdm_net_pair": (C.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "wdm_plan_attach_corrector": (C.c_int, [_vp, _vp, _i32, _i32]),
    "wdm_last_error": (C.c_char_p, []),
}


def load():
    """Load libwdm.so; raises if the HIP build is missing.

    torch is imported first: the library then binds to the HIP runtime torch
    has loaded, so the process holds one runtime (loaded the other way round,
    the library's runtime and torch's own copy would both be in the process
    and the library's would find no device)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        import torch  # noqa: F401  (see above)

        lib = C.CDLL(str(LIB_PATH))
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS)


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def _check(status: int):
    if status != 0:
        raise WdmError(status, load().wdm_last_error().decode())


def _cfg_array(configs):
    if isinstance(configs, wdm_config):
        configs = [configs]
    arr = (wdm_config * len(configs))(*configs)
    return arr, len(configs)


def make_config(n, L=1.0, hbar_over_m=1.0, four_pi_G=1.0, n_particles=0, particle_mass=0.0,
                precision=WDM_C64, kappa=0.0, absorb_alpha=0.0, absorb_nb=50.0,
                baryon_mode=0, nbody_substeps=1, boundary=0,
                external_potential=0, flags=0) -> wdm_config:
    nx, ny, nz = (n, n, n) if isinstance(n, int) else n
    lx, ly, lz = (L, L, L) if isinstance(L, (int, float)) else L
    return wdm_config(nx, ny, nz, lx, ly, lz, hbar_over_m, four_pi_G, int(n_particles),
                      float(particle_mass), precision, int(flags), float(kappa), float(absorb_alpha),
                      float(absorb_nb), int(baryon_mode), int(nbody_substeps), int(boundary),
                      int(external_potential))


# ---- entry points --------------------------------------------------------
def wdm_last_error() -> str:
    return load().wdm_last_error().decode()


def wdm_workspace_bytes(configs) -> int:
    arr, n = _cfg_array(configs)
    return int(load().wdm_workspace_bytes(arr, n))


def wdm_plan_create(configs, workspace, workspace_bytes=None, stream=None):
    arr, n = _cfg_array(configs)
    out = C.c_void_p()
    nbytes = workspace_bytes if workspace_bytes is not None else workspace.numel() * workspace.element_size()
    _check(load().wdm_plan_create(arr, n, _ptr(workspace), nbytes, _stream(stream), C.byref(out)))
    return out


def wdm_plan_destroy(plan):
    _check(load().wdm_plan_destroy(plan))


def wdm_set_state(plan, member, psi, pos=None, vel=None, t0=0.0):
    _check(load().wdm_set_state(plan, member, _ptr(psi), _ptr(pos), _ptr(vel), float(t0)))


def wdm_set_member_dt(plan, member, dt):
    _check(load().wdm_set_member_dt(plan, member, float(dt)))


def wdm_step(plan, n, dt=0.0):
    _check(load().wdm_step(plan, int(n), float(dt)))


def wdm_get_psi(plan, member, psi_out):
    _check(load().wdm_get_psi(plan, member, _ptr(psi_out)))


def wdm_density(plan, member, rho_out, include_baryons=True):
    _check(load().wdm_density(plan, member, _ptr(rho_out), 1 if include_baryons else 0))


def wdm_potential(plan, member, phi_out):
    _check(load().wdm_potential(plan, member, _ptr(phi_out)))


def wdm_energy(plan, member=0) -> dict:
    e = wdm_energy_t()
    _check(load().wdm_energy(plan, member, C.byref(e)))
    return e.as_dict()


def wdm_set_external_potential(plan, member, phi_ext):
    _check(load().wdm_set_external_potential(plan, member, _ptr(phi_ext)))


def wdm_diagnostics(plan, member=0, centre=None) -> dict:
    d = wdm_diagnostics_t()
    cen = (C.c_int32 * 3)(*centre) if centre is not None else None
    _check(load().wdm_diagnostics(plan, member, cen, C.byref(d)))
    return d.as_dict()


def wdm_particles(plan, member, pos_out=None, vel_out=None):
    _check(load().wdm_particles(plan, member, _ptr(pos_out), _ptr(vel_out)))


def wdm_fft3d(plan, member, inverse=False):
    _check(load().wdm_fft3d(plan, member, 1 if inverse else 0))


def wdm_fft3d_noalloc(psi_in, psi_out, shape, precision=WDM_C64, inverse=False, stream=None):
    nx, ny, nz = shape
    _check(load().wdm_fft3d_noalloc(_ptr(psi_in), _ptr(psi_out), int(nx), int(ny), int(nz),
                                    int(precision), 1 if inverse else 0, _stream(stream)))


def wdm_set_sort_interval(plan, interval):
    _check(load().wdm_set_sort_interval(plan, int(interval)))


def wdm_use_graphs(plan, enable=True):
    _check(load().wdm_use_graphs(plan, 1 if enable else 0))


def wdm_autotune(plan, reps=20):
    _check(load().wdm_autotune(plan, int(reps)))


def wdm_tuning_entries(plan):
    return int(load().wdm_tuning_entries(plan))


def wdm_get_tuning(plan):
    n = wdm_tuning_entries(plan)
    out = (_i32 * n)()
    _check(load().wdm_get_tuning(plan, out, n))
    return [int(v) for v in out]


def wdm_set_tuning(plan, table):
    n = len(table)
    arr = (_i32 * n)(*[int(v) for v in table])
    _check(load().wdm_set_tuning(plan, arr, n))


def tuning_key(configs) -> str:
    """Cache key of a plan's tuning table: its distinct grid shapes in the
    order of its size classes, and the precision."""
    configs = [configs] if isinstance(configs, wdm_config) else list(configs)
    shapes = sorted({(c.nx, c.ny, c.nz) for c in configs})
    return f"{'c128' if configs[0].precision else 'c64'}:" + ";".join(
        f"{a}x{b}x{c}" for a, b, c in shapes)


def autotune(plan, configs, cache=None, reps=20):
    """Choose the step passes' FFT plans: from the JSON file `cache` when it
    holds this plan's key, else by wdm_autotune (and store the result there).
    Overwrites the members' states (set them afterwards).  Returns the table."""
    import json
    from pathlib import Path

    key = tuning_key(configs)
    store = {}
    if cache is not None and Path(cache).exists():
        store = json.loads(Path(cache).read_text())
        if key in store and len(store[key]) == wdm_tuning_entries(plan):
            wdm_set_tuning(plan, store[key])
            return list(store[key])
    wdm_autotune(plan, reps)
    table = wdm_get_tuning(plan)
    if cache is not None:
        store[key] = table
        Path(cache).write_text(json.dumps(store, indent=1))
    return table


def wdm_profile(plan, enable=True):
    _check(load().wdm_profile(plan, 1 if enable else 0))


def wdm_profile_read(plan, cap=32) -> list:
    buf = (wdm_kernel_stat * cap)()
    cnt = C.c_int32()
    _check(load().wdm_profile_read(plan, buf, cap, C.byref(cnt)))
    return [{"name": buf[i].name.decode(), "launches": buf[i].launches,
             "total_ms": buf[i].total_ms} for i in range(min(cnt.value, cap))]


def wdm_copy_bandwidth(dst, src, nbytes, reps=20, stream=None) -> float:
    ms = C.c_double()
    _check(load().wdm_copy_bandwidth(_ptr(dst), _ptr(src), int(nbytes), int(reps),
                                     _stream(stream), C.byref(ms)))
    return ms.value


def wdm_restrict(fine, fine_member, coarse, coarse_member, psi_out):
    _check(load().wdm_restrict(fine, fine_member, coarse, coarse_member, _ptr(psi_out)))


def wdm_power_spectrum(plan, member, nbins):
    import numpy as np

    pk = np.zeros(nbins)
    cnt = np.zeros(nbins, dtype=np.int64)
    _check(load().wdm_power_spectrum(plan, member, int(nbins),
                                     pk.ctypes.data_as(C.POINTER(_f64)),
                                     cnt.ctypes.data_as(C.POINTER(_i64))))
    return pk, cnt


def wdm_distance(plan, member, other):
    """(sum |psi - other|^2, sum |other|^2) of a member's field."""
    out = (_f64 * 2)()
    _check(load().wdm_distance(plan, int(member), _ptr(other), out))
    return out[0], out[1]


def wdm_net_param_count() -> int:
    return int(load().wdm_net_param_count())


def wdm_net_workspace_bytes(n) -> int:
    return int(load().wdm_net_workspace_bytes(int(n)))


def wdm_net_create(n, workspace, workspace_bytes=None, stream=None):
    out = C.c_void_p()
    nbytes = workspace_bytes if workspace_bytes is not None else workspace.numel() * workspace.element_size()
    _check(load().wdm_net_create(int(n), _ptr(workspace), nbytes, _stream(stream), C.byref(out)))
    return out


def wdm_net_destroy(net):
    _check(load().wdm_net_destroy(net))


def _f32_host(a):
    import numpy as np

    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


def wdm_net_set_params(net, params):
    a, p = _f32_host(params)
    _check(load().wdm_net_set_params(net, p))


def wdm_net_get_params(net):
    import numpy as np

    a = np.zeros(wdm_net_param_count(), dtype=np.float32)
    _check(load().wdm_net_get_params(net, a.ctypes.data_as(C.POINTER(C.c_float))))
    return a


def wdm_net_get_grads(net):
    import numpy as np

    a = np.zeros(wdm_net_param_count(), dtype=np.float32)
    _check(load().wdm_net_get_grads(net, a.ctypes.data_as(C.POINTER(C.c_float))))
    return a


def wdm_net_forward(net, x, y=None):
    _check(load().wdm_net_forward(net, _ptr(x), _ptr(y)))


def wdm_net_backward(net, dy):
    _check(load().wdm_net_backward(net, _ptr(dy)))


def wdm_net_mse_backward(net, target) -> float:
    loss = C.c_double()
    _check(load().wdm_net_mse_backward(net, _ptr(target), C.byref(loss)))
    return loss.value


def wdm_net_adam(net, lr, b1=0.9, b2=0.999, eps=1e-8):
    _check(load().wdm_net_adam(net, float(lr), float(b1), float(b2), float(eps)))


def wdm_net_apply(net, plan, member=0):
    _check(load().wdm_net_apply(net, plan, int(member)))


def wdm_net_set_scales(net, s_psi, s_phi, s_out):
    _check(load().wdm_net_set_scales(net, float(s_psi), float(s_phi), float(s_out)))


def wdm_net_get_scales(net):
    out = (_f64 * 3)()
    _check(load().wdm_net_get_scales(net, out))
    return tuple(out)


def wdm_net_fit_scales(net, xs, ys):
    n = len(xs)
    xa = (_vp * n)(*[_ptr(x) for x in xs])
    ya = (_vp * n)(*[_ptr(y) for y in ys])
    _check(load().wdm_net_fit_scales(net, xa, ya, n))


def wdm_net_pair(plan, member, target, x_out, y_out):
    _check(load().wdm_net_pair(plan, int(member), _ptr(target), _ptr(x_out), _ptr(y_out)))


def wdm_plan_attach_corrector(plan, net, member=0, every=8):
    _check(load().wdm_plan_attach_corrector(plan, net, int(member), int(every)))


class Net:
    """Owns a torch workspace and a corrector-network handle."""

    def __init__(self, n, device="cuda"):
        import torch

        self.n = n
        nbytes = wdm_net_workspace_bytes(n)
        if nbytes == 0:
            raise WdmError(1, wdm_last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.handle = wdm_net_create(n, self.workspace, nbytes)

    def close(self):
        if self.handle is not None:
            wdm_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Owns a torch workspace and a plan handle (marshalling convenience)."""

    def __init__(self, configs, device="cuda"):
        import torch

        self.configs = [configs] if isinstance(configs, wdm_config) else list(configs)
        nbytes = wdm_workspace_bytes(self.configs)
        if nbytes == 0:
            raise WdmError(1, wdm_last_error())
        # 256-byte alignment is guaranteed by the caching allocator
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.handle = wdm_plan_create(self.configs, self.workspace, nbytes)

    def close(self):
        if self.handle is not None:
            wdm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
