"""The C ABI without a GPU: the library loads, exports every entry point that
include/wdm.h declares, and its host-only calls validate configurations."""
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def declared_symbols():
    text = (ROOT / "include" / "wdm.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wdm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("wdm_plan_create", "wdm_set_state", "wdm_step", "wdm_density",
                     "wdm_energy", "wdm_particles", "wdm_workspace_bytes", "wdm_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(wdm):
    lib = wdm.load()
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps every declared entry point under the same name
    assert sorted(wdm.exported_symbols()) == declared_symbols()
    for n in declared_symbols():
        assert callable(getattr(wdm, n))


def test_library_has_no_oracle_dependency():
    lib = ROOT / "paper_2606_25026_amd" / "libwdm.so"
    data = lib.read_bytes()
    assert b"orc_" not in data and b"liboracle" not in data


def test_workspace_bytes_and_validation(wdm):
    cfg = wdm.make_config(256, n_particles=1_000_000, particle_mass=1e-7)
    nbytes = wdm.wdm_workspace_bytes(cfg)
    cells = 256 ** 3
    # psi c64 + phi + rho_b + half spectrum + scratch, plus particles
    assert nbytes >= cells * (8 + 4 + 4 + 4 + 8) + 1_000_000 * 4 * 18
    assert nbytes % 256 == 0
    c128 = wdm.make_config(256, precision=wdm.WDM_C128)
    assert wdm.wdm_workspace_bytes(c128) > 1.9 * wdm.wdm_workspace_bytes(wdm.make_config(256))
    assert wdm.wdm_workspace_bytes(wdm.make_config(100)) == 0
    assert "axis lengths" in wdm.wdm_last_error()
    bad = wdm.make_config(64)
    bad.lx = -1.0
    assert wdm.wdm_workspace_bytes(bad) == 0
    mixed = [wdm.make_config(64), wdm.make_config(64, precision=wdm.WDM_C128)]
    assert wdm.wdm_workspace_bytes(mixed) == 0
    assert "precision" in wdm.wdm_last_error()
    for extra, why in ((dict(absorb_alpha=-1.0), "absorb_alpha"),
                       (dict(absorb_alpha=10.0, absorb_nb=0.0), "absorb_nb"),
                       (dict(kappa=float("nan")), "kappa")):
        assert wdm.wdm_workspace_bytes(wdm.make_config(64, **extra)) == 0, extra
        assert why in wdm.wdm_last_error()
    assert wdm.wdm_workspace_bytes(wdm.make_config(64, kappa=-2.0, absorb_alpha=10.0)) > 0
    for extra, why in ((dict(baryon_mode=2), "baryon_mode"),
                       (dict(nbody_substeps=-1), "nbody_substeps"),
                       (dict(nbody_substeps=1025), "nbody_substeps")):
        assert wdm.wdm_workspace_bytes(wdm.make_config(64, **extra)) == 0, extra
        assert why in wdm.wdm_last_error()
    assert wdm.wdm_workspace_bytes(
        wdm.make_config(64, n_particles=10, baryon_mode=wdm.WDM_BARYON_STATIC,
                        nbody_substeps=1024)) > 0
    ens = [wdm.make_config(n) for n in (64,) * 3 + (96,) * 3 + (128,) * 3]
    assert wdm.wdm_workspace_bytes(ens) > sum(
        wdm.wdm_workspace_bytes(wdm.make_config(n)) for n in (64, 96, 128))


def test_product_path_refuses_to_run_without_the_build(monkeypatch, tmp_path):
    from paper_2606_25026_amd import wdm as w

    monkeypatch.setattr(w, "LIB_PATH", tmp_path / "missing.so")
    monkeypatch.setattr(w, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        w.load()
