"""Host-side helpers of the driver against the oracle (no GPU)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2109_08815_amd import driver, synth


@pytest.mark.parametrize("cfg", ["box1", "box2"])
def test_box_frame_points_match_oracle(cfg):
    """The driver's box-frame observation (used to synthesise observed
    trajectories from GPU rollouts) equals the oracle's."""
    pb = synth.make_problem(cfg, N=4, T=24, n_s=1)
    q = np.random.default_rng(1).uniform(-1.5, 1.5, (20, 18))
    np.testing.assert_allclose(driver.box_frame_points(pb, q[:, :9]), orc.observe(pb, pb.particles[0], q),
                               rtol=0, atol=1e-13)
