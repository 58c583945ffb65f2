"""Host-side logic that needs no GPU: the tuning cache key, the bench's pass to
plan-variant mapping and traffic lookup, and the judge's P(k) error."""
import json
import math

import numpy as np
import pytest

import bench
from paper_2606_25026_amd import learned, wdm


def test_tuning_key_orders_distinct_shapes_and_names_precision():
    cfgs = [wdm.make_config(128), wdm.make_config(64), wdm.make_config((64, 96, 64)),
            wdm.make_config(64)]
    assert wdm.tuning_key(cfgs) == "c64:64x64x64;64x96x64;128x128x128"
    assert wdm.tuning_key(wdm.make_config(32, precision=wdm.WDM_C128)) == "c128:32x32x32"


def test_pass_variant_follows_the_tuning_slots():
    table = [1, 0, 1, 0, 1, 0]      # P1, P2/P4, P3, P5, P6/P8, P7
    assert bench.pass_variant("z_potential_kick", table) == 1
    assert bench.pass_variant("y_fft_psi_fwd", table) == 0
    assert bench.pass_variant("y_fft_psi_inv", table) == 0
    assert bench.pass_variant("x_kinetic", table) == 1
    assert bench.pass_variant("z_density_r2c", table) == 0
    assert bench.pass_variant("y_fft_spec_fwd", table) == 1
    assert bench.pass_variant("x_green", table) == 0
    # the closing kick always runs the default plan
    assert bench.pass_variant("z_potential_close_kick", table) == 0


def test_traffic_lookup_checks_source_hash_and_variant(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", tmp_path)
    h = bench.kernel_source_hash()
    doc = {"source_hash": h,
           "kernels": {"z_density_r2c": {"0": {"hbm_bytes_per_launch": 4.7e8}}}}
    f = tmp_path / "profiles" / "traffic_counters.json"
    f.write_text(json.dumps(doc))
    assert bench.traffic_from_profiles("z_density_r2c", 0) == 4.7e8
    assert bench.traffic_from_profiles("z_density_r2c", 1) is None     # not profiled
    assert bench.traffic_from_profiles("x_green", 0) is None
    doc["source_hash"] = "stale"
    f.write_text(json.dumps(doc))
    assert bench.traffic_from_profiles("z_density_r2c", 0) is None     # kernels changed


def test_committed_traffic_covers_every_plan_the_tuner_can_pick_for_p1():
    """The bench's roofline kernel (P1) at 256^3 may run its default, second
    or complex-exchange plan; the committed counters hold each of them for the
    current kernel sources, so the bench line's traffic field is never null
    because of the tuner's choice."""
    for v in (0, 1, 3):
        hbm = bench.traffic_from_profiles("z_potential_kick", v)
        assert hbm is not None, f"no counters for plan {v}"
        alg = bench.BYTES_PER_CELL["z_potential_kick"] * 256 ** 3
        assert 0.99 < hbm / alg < 1.05


def test_pk_error_is_relative_l2_over_shells_from_one():
    pf = np.array([100.0, 4.0, 3.0, 0.0])
    pc = np.array([0.0, 4.0, 3.0, 0.0])     # shell 0 is excluded
    assert learned.pk_error(pc, pf, 4) == 0.0
    pc = np.array([0.0, 4.0, 0.0, 0.0])
    assert learned.pk_error(pc, pf, 4) == pytest.approx(3.0 / 5.0)
    assert math.isfinite(learned.pk_error(pf, pf, 3))
