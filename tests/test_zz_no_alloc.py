"""The allocation-free pose solve (lsr_stage_gnc_noalloc) against lsr_stage_gnc:
bit-identical on two calls in a row, the second with fewer correspondences,
and usable in a context whose workspace cap forbids any scratch allocation."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _corr(rng, m, outliers=0.3):
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    th = rng.uniform(0.2, 1.0)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    R = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
    t = rng.uniform(-0.5, 0.5, 3)
    p = rng.uniform(-1, 1, (m, 3))
    q = p @ R.T + t + rng.normal(0, 0.003, (m, 3))
    bad = rng.random(m) < outliers
    q[bad] = rng.uniform(-1, 1, (int(bad.sum()), 3))
    return torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda()


def test_noalloc_gnc_equals_stage_gnc():
    import paper_1801_01572_amd as lsr
    from paper_1801_01572_amd import _lib
    rng = np.random.default_rng(11)
    prm = lsr.default_params()
    tight = lsr.Context(0, workspace_cap=1)          # no plan of any size fits this cap
    T = torch.full((16,), np.nan, dtype=torch.float64, device="cuda")
    info = torch.full((4,), np.nan, dtype=torch.float64, device="cuda")
    for m in (3000, 500):
        print(f"noalloc gnc: m={m}", flush=True)
        p, q = _corr(rng, m)
        T_ref, info_ref = lsr.stage_gnc(p, q, prm)
        lsr.stage_gnc_noalloc(p, q, T, info, prm, ctx=tight)
        torch.cuda.synchronize()
        assert torch.equal(T.view(4, 4), T_ref) and torch.equal(info, info_ref), (m, T, T_ref, info, info_ref)
        assert info[0].item() == lsr.ACCEPTED
    with pytest.raises(lsr.LsrError, match="cap"):
        lsr.stage_gnc(p, q, prm, ctx=tight)             # the allocating entry point needs scratch
    assert _lib.lib().lsr_stage_gnc_noalloc(tight.h, None, None, -1, None, None, None, None) == -1
