"""GPU check of gs_densify_noalloc, the densification call that takes its
workspace from a fixed device array instead of a caller's buffer: on the same
seeded inputs it must give exactly what gs_densify gives (the same kernels;
counts, decisions and every output value bit-exact), on calls in a row whose
inputs shrink, so what an earlier call left in the array cannot leak into a
later one.  The counts are also checked against the FP64 oracle's decisions."""

import numpy as np
import pytest
import torch

import scenes
from oracle import densify as od
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

SENTINEL = -7.25


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def _both(c, n):
    from paper_2311_16728_amd import gs

    n_cap = c["n_cap"]
    out_cap = 2 * n_cap
    rule = gs.densify_rule(c["extent"])
    P, M, V = _dev(c["params"]), _dev(c["m"]), _dev(c["v"])
    S, Z = _dev(c["stats"]), _dev(c["noise"])
    res = []
    for noalloc in (False, True):
        outs = [torch.full((59, out_cap), SENTINEL, dtype=torch.float32, device="cuda") for _ in range(3)]
        counts = torch.full((4,), -1, dtype=torch.int64, device="cuda")
        if noalloc:
            gs.gs_densify_noalloc(rule, P, M, V, S, Z, n, *outs, counts)
        else:
            ws = torch.empty(gs.gs_densify_workspace_bytes(n), dtype=torch.uint8, device="cuda")
            gs.gs_densify(rule, P, M, V, S, Z, n, *outs, ws, counts)
        torch.cuda.synchronize()
        res.append(([o.cpu().numpy() for o in outs], counts.cpu().numpy()))
    return res


def _oracle_counts(c, n):
    rule = od.densify_rule(c["extent"])
    action, keep, new = od.decide(c["params"], c["stats"], n, rule)
    return [int(keep.sum() + new.sum()), int(np.sum((action == od.CLONE) & (new > 0))),
            int(np.sum(action == od.SPLIT)), int(np.sum((action != od.SPLIT) & ~keep))]


def test_noalloc_matches_workspace_call_on_shrinking_inputs():
    # three calls in a row on the shared array, each input smaller than the last
    for seed, n in ((0, 20000), (1, 3001), (2, 1), (3, 0)):
        c = scenes.densify_case(seed, max(n, 1))
        (outs_ws, cnt_ws), (outs_na, cnt_na) = _both(c, n)
        print(f"noalloc case seed={seed} n={n} counts={cnt_na.tolist()}", flush=True)
        assert np.array_equal(cnt_na, cnt_ws), (seed, n)
        assert cnt_na.tolist() == _oracle_counts(c, n), (seed, n)
        for a, b in zip(outs_na, outs_ws):
            assert np.array_equal(a, b), (seed, n)
        # nothing written past the output count
        k = int(cnt_na[0])
        assert np.all(outs_na[0][:, k:] == SENTINEL)
