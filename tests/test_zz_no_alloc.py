"""GPU test of rt_trace_batch_noalloc, the entry point for callers that
cannot allocate device memory: through the C ABI, its outputs equal
rt_trace_batch's on the same rays, on two calls in a row (the second with
a smaller input, so that the fixed work table holds the first call's
contents when it starts)."""
import numpy as np
import pytest

from paper_1209_6038_amd import workloads as W
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _same(a, b):
    import torch
    if a.dtype.is_floating_point:
        return torch.equal(torch.nan_to_num(a, nan=-7.0), torch.nan_to_num(b, nan=-7.0))
    return torch.equal(a, b)


@pytest.mark.parametrize("axis,branch", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_noalloc_trace_equals_trace_batch(axis, branch):
    """Per-ray work does not depend on the table it runs in: every output
    (exit ray, optical path, status, drift, step count, Eq. (12) weight)
    equals rt_trace_batch's bit for bit."""
    import torch
    from paper_1209_6038_amd import rt
    cl = rt.Cloak(W.cloak(axis, height=W.HEIGHT))
    for k, n in enumerate((rt.NOALLOC_MAX_RAYS, 3001)):
        say(f"case noalloc axis={axis} branch={branch} call {k} n={n}")
        rays = torch.from_numpy(W.random_rays(n, seed=40 + k, z_range=(-1.0, 5.0))).cuda()
        ref = rt.trace_batch(cl, W.opts_dp45(), branch, rays, with_trans=True)
        got = rt.trace_batch(cl, W.opts_dp45(), branch, rays, with_trans=True, noalloc=True)
        torch.cuda.synchronize()
        for key in ref:
            assert _same(ref[key], got[key]), (key, n)
        say(f"  equal; statuses {np.bincount(got['status'].cpu().numpy(), minlength=8).tolist()}")
    cl.close()


def test_noalloc_rejects_more_than_its_table_holds():
    import torch
    from paper_1209_6038_amd import rt
    cl = rt.Cloak(W.cloak(0, height=W.HEIGHT))
    rays = torch.zeros((6, rt.NOALLOC_MAX_RAYS + 1), dtype=torch.float64, device="cuda")
    with pytest.raises(rt.RtError, match="at most"):
        rt.trace_batch(cl, W.opts_dp45(), 1, rays, noalloc=True)
    cl.close()
