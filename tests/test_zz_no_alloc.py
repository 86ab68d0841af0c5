"""The pressure-tensor entry point that allocates nothing
(mdpd_read_stress_noalloc) against mdpd_read_stress (needs an MI355X).

Two calls in a row on one GPU, the second on a smaller system, in host and
device output memory: the fixed scratch is shared, so the second call must
not see anything of the first.  A batch of replicas with a sub-range checks
the per-replica reduction.  Bar: FP64 sums in another order, within 1e-12 of
the diagonal scale.
"""
import numpy as np
import pytest

from paper_1903_10134_amd import workloads as W
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpd():
    import torch
    assert torch.cuda.is_available()
    import paper_1903_10134_amd as m
    m.lib()
    return m


def close(a, b):
    scale = max(np.abs(b[..., :3]).max(), 1e-300)
    return np.abs(a - b).max() / scale < 1e-12


@pytest.mark.parametrize("where", ["host", "device"])
def test_noalloc_matches_stress_two_calls(mdpd, where):
    import torch
    big = W.bulk(L=12.0, seed=3)
    small = W.bulk(L=7.0, seed=4, A=-30.0)
    say("noalloc stress", where, big.n, small.n)
    systems = [mdpd.System(big, precision=mdpd.FP32_FORCES), mdpd.System(small)]
    for s in systems:
        s.step(3)
    for s in systems:  # big first, then the smaller input
        ref = mdpd.mdpd_read_stress(s.h, 0, 1)
        if where == "host":
            got = mdpd.mdpd_read_stress_noalloc(s.h, 0, 1)
        else:
            dev = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
            mdpd.mdpd_read_stress_noalloc(s.h, 0, 1, out=dev)
            torch.cuda.synchronize()
            got = dev.cpu().numpy().reshape(1, 6)
        assert close(got, ref), (got, ref)
    for s in systems:
        s.close()


def test_noalloc_batch_subrange(mdpd):
    reps = W.replicas(count=5, lo=8.0, hi=10.0, seed=2)
    say("noalloc stress batch", sum(r.n for r in reps))
    b = mdpd.Batch(reps)
    b.step(2)
    ref = mdpd.mdpd_read_stress(b.h, 0, 5)
    for first, count in ((0, 5), (3, 2), (1, 1)):
        got = mdpd.mdpd_read_stress_noalloc(b.h, first, count)
        assert close(got, ref[first:first + count]), (first, count)
    with pytest.raises(mdpd.MdpdError):
        mdpd.mdpd_read_stress_noalloc(b.h, 4, 2)
    b.close()
