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


def box_frame_points(pb, q):
    """Box-frame observation of the universal-joint arm for joint angles q
    [n, 9]: the box origin and the points 1 m along its x, y, z axes in
    world coordinates [n, 12].  Per arm joint the modified-DH placement
    (Rot_x(alpha), Trans_x(a)) then Rot_z(q) Trans_z(d); then the flange
    offset along z, Rot_x(q_7) and Rot_y(q_8)."""
    a = pb.arm
    q = np.asarray(q, dtype=np.float64)
    n = q.shape[0]
    Rw = np.broadcast_to(np.eye(3), (n, 3, 3)).copy()
    o = np.zeros((n, 3))

    def rot(axis, t):
        c, s = np.cos(t), np.sin(t)
        R = np.zeros((len(t), 3, 3))
        i, j = [(1, 2), (2, 0), (0, 1)][axis]
        R[:, axis, axis] = 1.0
        R[:, i, i] = c
        R[:, j, j] = c
        R[:, i, j] = -s
        R[:, j, i] = s
        return R

    for i in range(7):
        al = np.full(n, a["dh_alpha"][i])
        Rw = Rw @ rot(0, al)
        o = o + Rw @ np.array([a["dh_a"][i], 0.0, 0.0])
        Rw = Rw @ rot(2, q[:, i])
        o = o + Rw @ np.array([0.0, 0.0, a["dh_d"][i]])
    o = o + Rw @ np.array([0.0, 0.0, a["flange_d"]])
    Rw = Rw @ rot(0, q[:, 7]) @ rot(1, q[:, 8])
    return np.concatenate([o, o + Rw[:, :, 0], o + Rw[:, :, 1], o + Rw[:, :, 2]], axis=1)


def gpu_observations(pb, device="cuda"):
    """Observed trajectories [K, T, d_x]: trajectory k rolled out at theta_true[k] from s0[k] plus noise."""
    tr = gpu_rollout(pb, pb.theta_true, device)
    k = torch.arange(pb.K, device=tr.device)
    if pb.kind in (synth.KIND_ARM_UJOINT, synth.KIND_ARM_UJOINT_WEIGHTS):
        q = tr[k, k][:, :, : pb.n_dof].double().cpu().numpy()
        x = np.stack([box_frame_points(pb, q[j]) for j in range(pb.K)])
        return x + pb.noise
    x = tr[k, k][:, :, torch.as_tensor(pb.obs_index, device=tr.device)]
    return x.double().cpu().numpy() + pb.noise


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
