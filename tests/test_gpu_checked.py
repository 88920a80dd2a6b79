"""Checked mode of the C interface (settings.checked = 1): NaN and infinity
guards that report through a device status word, with every kernel running to
its end.  The guarded calls are the projection (Section 3.3, Eq. 3's splat
from the primitive parameters of Section 3.1) and the chain rule with the
fixed-rate optimiser step (Section 4.1)."""

import numpy as np
import pytest
import torch

import scenes
from tests.gpu_util import plan_for, require_gpu

pytestmark = pytest.mark.gpu

BAD = [(5, 0, np.nan), (17, 3, np.inf), (40, 10, np.nan), (77, 30, np.nan), (90, 7, -np.inf)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def test_nan_in_params_is_flagged_and_culled():
    from paper_2311_16728_amd import gs
    from paper_2311_16728_amd.mapper import Mapper

    p, tp, cam = scenes.tiny_scene(0)
    n = 2000
    bad = p.copy()
    clean = p.copy()
    for col, row, val in BAD:
        bad[row, col] = val
        clean[10, col] = -100.0     # the same columns, invisible
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    checked = gs.default_settings(checked=1, status=status)
    print("checked-mode case: tiny scene, non-finite values at", BAD, flush=True)

    plan = plan_for([cam], n_cap=p.shape[1], settings=checked)
    plan.render(_dev(bad), n)
    torch.cuda.synchronize()
    word = int(status.item())
    assert word & gs.STATUS_NUMERIC
    assert gs.gs_status_word(word) == 5
    with pytest.raises(gs.GsError, match="non-finite"):
        gs.check_status_word(word)
    img = plan.rgb.clone()
    assert torch.isfinite(img).all()

    # the guarded columns render as if they were not there
    ref = plan_for([cam], n_cap=p.shape[1])
    ref.render(_dev(clean), n)
    torch.cuda.synchronize()
    assert torch.equal(img, ref.rgb)

    # a clean map in checked mode: no report, bitwise the unchecked render
    status.zero_()
    plan.render(_dev(p), n)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    ref.render(_dev(p), n)
    torch.cuda.synchronize()
    assert torch.equal(plan.rgb, ref.rgb)

    # the fused backward + Adam step reports the non-finite parameters it updates
    target = ref.rgb.clone()
    status.zero_()
    mp = Mapper(_dev(bad), n)
    mp.step(plan, target, lam=0.2)
    mp.step(plan, target, lam=0.2)
    torch.cuda.synchronize()
    assert int(status.item()) & gs.STATUS_NUMERIC
    assert torch.isfinite(plan.rgb).all()
    good_cols = np.setdiff1d(np.arange(n), [c for c, _, _ in BAD])
    assert torch.isfinite(mp.params[:, torch.as_tensor(good_cols).cuda()]).all()


def test_checked_clean_step_matches_unchecked():
    """On finite inputs the guards change nothing: one fused step in checked mode
    equals the unchecked step bitwise on the parameters, and reports nothing."""
    from paper_2311_16728_amd import gs
    from paper_2311_16728_amd.mapper import Mapper

    p, tp, cam = scenes.tiny_scene(2)
    n = 2000
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    tplan = plan_for([cam], n_cap=p.shape[1])
    tplan.render(_dev(tp), n)
    target = tplan.rgb.clone()
    outs = []
    for settings in (gs.default_settings(checked=1, status=status), gs.default_settings()):
        plan = plan_for([cam], n_cap=p.shape[1], settings=settings)
        mp = Mapper(_dev(p), n)
        mp.step(plan, target, lam=0.2, fused=False)
        torch.cuda.synchronize()
        outs.append(plan.rgb.clone())
    assert int(status.item()) == 0
    assert torch.equal(outs[0], outs[1])
