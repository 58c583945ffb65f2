"""The allocation-free transform (wdm_fft3d_noalloc) against the plan-based
wdm_fft3d on the same inputs: two calls in a row, the second on a smaller grid,
complex64 and complex128, forward and inverse, through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {0: 1e-6, 1: 1e-13}   # the 3D transform's parity bars (complex64, complex128)


def plan_fft(wdm, torch, psi, prec, inverse):
    shape = psi.shape
    cfg = wdm.make_config(shape, precision=prec)
    plan = wdm.Plan(cfg, device="cuda")
    wdm.wdm_set_state(plan.handle, 0, psi)
    wdm.wdm_fft3d(plan.handle, 0, inverse)
    out = torch.empty_like(psi)
    wdm.wdm_get_psi(plan.handle, 0, out)
    torch.cuda.synchronize()
    plan.close()
    return out.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_fft_matches_plan_fft(wdm, prec):
    import torch

    cdt = torch.complex64 if prec == 0 else torch.complex128
    rng = np.random.default_rng(7)
    cases = [((64, 32, 96), False, False), ((32, 16, 32), True, True)]
    for shape, inverse, in_place in cases:
        print(f"noalloc fft: shape={shape} prec={prec} inverse={inverse} in_place={in_place}",
              flush=True)
        host = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        psi = torch.from_numpy(host).to(cdt).cuda()
        ref = plan_fft(wdm, torch, psi, prec, inverse)
        if in_place:
            out = psi.clone()
            wdm.wdm_fft3d_noalloc(out, out, shape, prec, inverse)
        else:
            out = torch.full_like(psi, float("nan"))
            wdm.wdm_fft3d_noalloc(psi, out, shape, prec, inverse)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"  rel L2 vs wdm_fft3d = {err:.3e}", flush=True)
        assert err <= TOL[prec], err
        # the input of an out-of-place call is left as it was
        if not in_place:
            assert np.array_equal(psi.cpu().numpy(), host.astype(got.dtype))


def test_noalloc_fft_rejects_bad_arguments(wdm):
    import torch

    psi = torch.zeros((32, 32, 32), dtype=torch.complex64, device="cuda")
    with pytest.raises(wdm.WdmError) as e:
        wdm.wdm_fft3d_noalloc(psi, psi, (32, 32, 1024), 0, False)
    assert e.value.status == 6
    with pytest.raises(wdm.WdmError) as e:
        wdm.wdm_fft3d_noalloc(None, psi, (32, 32, 32), 0, False)
    assert e.value.status == 1
    with pytest.raises(wdm.WdmError) as e:
        wdm.wdm_fft3d_noalloc(psi, psi, (32, 32, 32), 2, False)
    assert e.value.status == 1
