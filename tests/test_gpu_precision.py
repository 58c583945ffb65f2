"""Precision study on the GPU: the 128^3 sub-box (L' = 0.25, the dx and dt of
the 512^3 run) after 2000 KDK steps against sampled FP64-oracle values written
by tests/golden/make_subbox_reference.py, for the complex64 path (FP64 phase
arguments, FP64-formed kinetic factors) and the complex128 path, plus the
conservation the oracle shows over the same run.

Bars: complex128 within 1e-10 of the oracle; complex64 within 3e-5 relative L2
(two thousand steps of single-precision FFT rounding, measured 1.1e-5) and a
mass drift below 2e-6 (measured -5.6e-7).
"""
import math
from pathlib import Path

import numpy as np
import pytest

from paper_2606_25026_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = Path(__file__).resolve().parent / "golden" / "subbox_128_steps2000.npz"


@pytest.mark.parametrize("prec", [0, 1])
def test_subbox_2000_steps_vs_oracle(wdm, prec):
    g = np.load(GOLDEN)
    n, L, steps = int(g["n"]), float(g["L"]), int(g["steps"])
    psi0 = inputs.grf_soliton(n, L=L, k0=16.0 * 2 * math.pi, rc=0.03, rho_c=50.0,
                              seed=int(g["seed"]))
    assert np.max(np.abs(psi0.ravel()[g["cells"]] - g["psi0"])) < 1e-12
    plan = wdm.Plan(wdm.make_config(n, L=L, precision=prec))
    x = torch.from_numpy(psi0).to(torch.complex64 if prec == 0 else torch.complex128).cuda()
    wdm.wdm_set_state(plan.handle, 0, x)
    e0 = wdm.wdm_energy(plan.handle, 0)
    wdm.wdm_step(plan.handle, steps, float(g["dt"]))
    out = torch.empty_like(x)
    wdm.wdm_get_psi(plan.handle, 0, out)
    e1 = wdm.wdm_energy(plan.handle, 0)
    torch.cuda.synchronize()
    got = out.cpu().numpy().ravel()[g["cells"]].astype(np.complex128)
    err = float(np.linalg.norm(got - g["psi"]) / np.linalg.norm(g["psi"]))
    drift = e1["mass"] / e0["mass"] - 1
    edrift = e1["e_total"] / e0["e_total"] - 1
    print(f"sub-box 128^3, {steps} steps, prec={prec}: rel L2 {err:.3e}, mass drift {drift:.2e}, "
          f"energy drift {edrift:.2e} (oracle {g['etot1'] / g['etot0'] - 1:.2e})")
    assert e0["mass"] == pytest.approx(float(g["mass0"]), rel=1e-6 if prec == 0 else 1e-12)
    if prec == 1:
        assert err < 1e-10
        assert abs(drift) < 1e-11
    else:
        assert err < 3e-5
        assert abs(drift) < 2e-6
    plan.close()
