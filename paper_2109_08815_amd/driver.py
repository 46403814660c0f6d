"""CSVGD driver on the GPU library: problem set-up and the iteration loop.

Set-up uses the library's own rollout (sim_batch_forward) for the observed
trajectories (rollout at the generating parameters plus the problem's noise
draws) and for the default shooting states (each particle's own
single-shooting state at the start of every window).  One iteration is
Algorithm 1: sim_batch_adjoint -> svgd_phi -> svgd_step (optionally with the
bandwidth on a second stream, concurrent with the adjoint), optionally
captured once into a HIP graph and replayed.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import lib as L
from . import synth


def single_shooting(pb):
    """Same problem with one window (n_s = 1, h = T)."""
    return dataclasses.replace(pb, n_s=1, h=pb.T)


def gpu_rollout(pb, theta, device="cuda"):
    """Visited states [N, K, T, d_s] of every particle from every s0_k (a
    device tensor, ready in stream order on the current stream)."""
    ss = single_shooting(pb)
    obs = np.zeros((pb.K, pb.T, pb.d_x))
    job = L.Job(ss, obs, theta=theta, device=device, with_traj=True)
    b = L.Batch([job])
    L.sim_batch_forward(b)
    return job.traj


def gpu_observed_rollout(pb, theta, device="cuda"):
    """What the observation model sees of every particle's rollout from
    every s0_k: the library's f_obs of each visited state (traj_obs), a
    device tensor [N, K, T, d_x] in stream order on the current stream."""
    ss = single_shooting(pb)
    job = L.Job(ss, np.zeros((pb.K, pb.T, pb.d_x)), theta=theta, device=device, with_traj_obs=True)
    L.sim_batch_forward(L.Batch([job]))
    return job.traj_obs


def gpu_observed(pb, device="cuda"):
    """f_obs of trajectory k rolled out at theta_true[k] from s0[k], a device
    tensor [K, T, d_x] (gpu_observed_rollout's (k, k) entries)."""
    tro = gpu_observed_rollout(pb, pb.theta_true, device)
    k = torch.arange(pb.K, device=tro.device)
    return tro[k, k]


def gpu_observations(pb, device="cuda"):
    """Observed trajectories [K, T, d_x] (host array): gpu_observed plus the
    problem's noise draws."""
    return gpu_observed(pb, device).double().cpu().numpy() + pb.noise


def gpu_shooting_init_device(pb, theta, device="cuda"):
    """Shooting states [N, K, n_s-1, d_s] (device tensor) from each
    particle's own rollout: the state after step j h starts window j."""
    if pb.n_s == 1:
        return torch.zeros((theta.shape[0], pb.K, 0, pb.d_s), device=device)
    tr = gpu_rollout(pb, theta, device)
    idx = torch.arange(1, pb.n_s, device=tr.device) * pb.h - 1
    return tr[:, :, idx].contiguous()


def gpu_shooting_init(pb, theta, device="cuda"):
    """Shooting states [N, K, n_s-1, d_s] as a host array."""
    return gpu_shooting_init_device(pb, theta, device).double().cpu().numpy()


class CSVGD:
    """Runs CSVGD iterations on a batch of jobs (plain launches or a replayed graph)."""

    def __init__(self, jobs, optimizer=L.PDS_OPT_ADAM, overlap=False):
        for j in jobs:
            if j.iter_dev is None:
                j.iter_dev = torch.zeros(2, dtype=torch.int32, device=j.device)
        self.batch = L.Batch(jobs)
        self.optimizer = optimizer
        self.overlap = overlap
        self.graph = None
        self.stream = None

    def step(self):
        """One iteration with plain launches on the current stream."""
        L.csvgd_iteration(self.batch, 0, self.optimizer, overlap=self.overlap)

    def capture(self, iterations: int = 1):
        """Capture `iterations` consecutive iterations into one graph."""
        self.stream = torch.cuda.Stream()
        self.stream.wait_stream(torch.cuda.current_stream())
        self.graph = torch.cuda.CUDAGraph()
        self.graph_iterations = iterations
        with torch.cuda.graph(self.graph, stream=self.stream):
            for _ in range(iterations):
                L.csvgd_iteration(self.batch, 0, self.optimizer, stream=self.stream, overlap=self.overlap)
        torch.cuda.current_stream().wait_stream(self.stream)

    def replay(self):
        self.graph.replay()
