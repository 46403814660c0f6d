"""svgd_phi_noalloc (the allocation-free variant of svgd_phi, with the
library's fixed workspace array) against svgd_phi with a caller workspace,
through the C ABI: bitwise the same bandwidth and phi on two calls in a row,
the second with a smaller job, and a clear error for a batch above the
array."""
import numpy as np
import pytest
import torch

from paper_2109_08815_amd import lib as L
from paper_2109_08815_amd import synth
from tests.helpers import f32_problem, print_case, r32, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def _job(cfg, N, seed):
    pb = f32_problem(synth.make_problem(cfg, N=N, K=1, T=40, n_s=2))
    rng = np.random.default_rng(seed)
    theta = r32(pb.lo + rng.uniform(size=(N, pb.M)) * (pb.hi - pb.lo))
    G = rng.normal(scale=1e4, size=(N, pb.M))
    job = L.Job(pb, np.zeros((pb.K, pb.T, pb.d_x)), theta=theta)
    job.g_obs.copy_(torch.as_tensor(G, dtype=torch.float64))
    return job


def test_noalloc_phi_matches_workspace_phi():
    # calls in a row on the same array, each smaller than the one before:
    # the sampled-bracket median with the counting pass (2048 and 300
    # particles), then the all-pairs selection (70)
    for cfg, N, seed in (("c3", 2048, 1), ("c2", 300, 2), ("c2", 70, 3)):
        print_case("noalloc", cfg, N)
        a = _job(cfg, N, seed)
        b = _job(cfg, N, seed)
        L.svgd_phi(L.Batch([a]))
        L.svgd_phi_noalloc(L.Batch([b]))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(a.bandwidth.cpu().numpy(), b.bandwidth.cpu().numpy())
        np.testing.assert_array_equal(a.phi.cpu().numpy(), b.phi.cpu().numpy())


def test_noalloc_phi_rejects_batch_above_array():
    print_case("noalloc-too-large")
    job = _job("c2", 8000, 4)
    with pytest.raises(L.PdsError, match="svgd_phi_noalloc"):
        L.svgd_phi_noalloc(L.Batch([job]))
