"""The allocation-free loss entry point (gs_loss_l2_noalloc) against the
workspace form (gs_loss_l2) through the C ABI: two calls in a row on the
library's per-GPU partial-sum array, the second on a smaller input, each
bit-identical to the workspace call (same kernels, same reduction order) and
within 1e-6 of the FP64 oracle."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def test_loss_l2_noalloc_matches_workspace_call():
    import torch
    from paper_2606_11390_amd import binding as B
    rng = np.random.default_rng(21)
    # a large call (2048 partial sums) and then a small one (one partial sum)
    for n in (3 * 1920 * 1080 + 7, 3 * 37 * 21):
        img = rng.uniform(0, 1, n).astype(np.float32)
        tgt = rng.uniform(0, 1, n).astype(np.float32)
        ti = torch.from_numpy(img).cuda()
        tt = torch.from_numpy(tgt).cuda()
        loss_ws = torch.zeros(1, device="cuda")
        d_ws = torch.zeros(n, device="cuda")
        ws = torch.empty(B.loss_workspace_size(n), dtype=torch.uint8, device="cuda")
        B.loss_l2(ti, tt, loss_ws, d_ws, ws)
        loss_na = torch.full((1,), float("nan"), device="cuda")
        d_na = torch.full((n,), float("nan"), device="cuda")
        B.loss_l2_noalloc(ti, tt, loss_na, d_na)
        torch.cuda.synchronize()
        a, b = loss_ws.cpu().numpy(), loss_na.cpu().numpy()
        print(f"n={n}: loss workspace {a[0]:.9g}, allocation-free {b[0]:.9g}", flush=True)
        assert a.view(np.uint32)[0] == b.view(np.uint32)[0]
        assert np.array_equal(d_ws.cpu().numpy().view(np.uint32), d_na.cpu().numpy().view(np.uint32))
        L, (dref,) = oracle.l2_loss([img], [tgt])
        assert float(b[0]) == pytest.approx(L, rel=1e-6)
        assert np.max(np.abs(d_na.cpu().numpy() - dref)) <= 1e-6 * np.max(np.abs(dref))
