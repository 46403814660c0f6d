"""Measured error of the HIP path against the FP64 oracle, per result and
workload (run on a GPU: ``python -m tests.parity_report [out.json]
[--workloads c1 ... box2] [--no-drift]``).

For every workload at its full size, from identical float32 inputs: the
window states, window log-likelihoods, log p, mixture weights, both theta
gradients, S_dot, the bandwidth, phi and one Adam step, each compared with
the oracle on a sample of particles (the bandwidth over all of them).  phi
and the step are compared from the GPU's own inputs to them (its g_obs,
phi, g_con, S_dot, g_def), so each row isolates one stage.  Then the
drift of the pendulum problem's particle set over 100 iterations run on
both sides.  Prints a Markdown table; writes the numbers as JSON.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np
import torch

from oracle import oracle as orc
from paper_2109_08815_amd import lib as L
from paper_2109_08815_amd import synth
from tests.helpers import f32_problem, r32
from tests.parity import (end_state_rel_err, grad_check, ll_tolerance, normwise, phi_scale, state_rel_err,
                          update_check)

WORKLOADS = ["c1", "c2", "c3", "c4", "rigid2", "box1", "box2"]
SAMPLE = 12


def np64(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measure(cfg):
    t0 = time.time()
    pb = f32_problem(synth.make_problem(cfg))
    obs = r32(orc.observations(pb))
    rng = np.random.default_rng(11)
    S = r32(synth.perturb(rng, orc.shooting_init(pb, pb.particles), 0.005))
    lam_def = r32(rng.uniform(0.0, 2.0, (pb.N, pb.K, pb.n_s - 1)))
    st = orc.State(pb, pb.particles, S, lam_def=lam_def)
    log("%s set up in %.1f s" % (cfg, time.time() - t0))
    job = L.Job(pb, obs, theta=pb.particles, S=S, with_traj=True)
    job.lam_def.copy_(torch.as_tensor(lam_def, dtype=torch.float32))
    b = L.Batch([job])
    L.sim_batch_forward(b)
    traj = job.traj
    L.sim_batch_adjoint(b)
    L.svgd_phi(b)
    pre = {k: np64(getattr(job, k)) for k in ("theta", "S", "lam_lim", "lam_def", "adam_m", "adam_v")}
    L.svgd_step(b, L.PDS_OPT_ADAM, 1)
    N = pb.N
    sel = np.unique(np.concatenate([[0, N - 1], rng.choice(N, size=min(N, SAMPLE) - 2, replace=False)])).astype(
        np.int32)
    tg = traj.detach()[torch.as_tensor(sel, device=traj.device, dtype=torch.long)].cpu().numpy().astype(np.float64)
    fwd = orc.forward(pb, obs, st, sel=sel, traj=True)
    ref = orc.gradient(pb, obs, st, sel=sel, per_unit=True)
    log("%s oracle sample done at %.1f s" % (cfg, time.time() - t0))
    out = {"workload": cfg, "N": N, "K": pb.K, "T": pb.T, "n_s": pb.n_s, "sample": int(len(sel))}
    out["states"] = float(state_rel_err(pb, tg, fwd["traj"]).max())
    out["end_states"] = float(end_state_rel_err(np64(job.end_states)[sel], fwd["end_states"]).max())
    llg = np64(job.ll_win)[sel]
    out["ll_win_rel"] = float((np.abs(llg - fwd["ll_win"]) / np.maximum(np.abs(fwd["ll_win"]), 1e-300)).max())
    if pb.kind not in (synth.KIND_ARM_UJOINT, synth.KIND_ARM_UJOINT_WEIGHTS):
        tol = ll_tolerance(pb, obs, fwd["traj"], fwd["ll_win"])
        out["ll_win_bar_ratio"] = float((np.abs(llg - fwd["ll_win"]) / tol).max())
    lp = np64(job.logp)[sel]
    out["logp_rel"] = float((np.abs(lp - fwd["logp"]) / np.abs(fwd["logp"])).max())
    out["wk_abs"] = float(np.abs(np64(job.wk)[sel] - fwd["wk"]).max())
    if pb.n_s > 1:
        gd = np64(job.gdef)[sel]
        out["gdef_rel"] = float((np.abs(gd - fwd["gdef"]) / np.maximum(np.abs(fwd["gdef"]), 1e-300)).max())
    go = grad_check(np64(job.g_obs)[sel], ref, "obs")
    out["g_obs_normwise"] = float(go["normwise"].max())
    out["g_obs_terms_over_norm"] = float(go["terms"].max())
    out["g_obs_bar_ratio"] = float(go["ratio"].max())
    if pb.n_s > 1:
        gc = grad_check(np64(job.g_con)[sel], ref, "con", pb, S[sel])
        out["g_con_normwise"] = float(gc["normwise"].max())
        out["g_con_bar_ratio"] = float(gc["ratio"].max())
        out["S_dot_normwise"] = float(normwise(np64(job.S_dot)[sel][:, :, : pb.n_s - 1], ref["S_dot"]).max())
    theta = pre["theta"]
    h_ref, _ = orc.bandwidth(theta, pb.rho)
    out["bandwidth_rel"] = float(abs(np64(job.bandwidth)[0] - h_ref) / h_ref)
    G = np64(job.g_obs)
    ph_ref = orc.phi(theta, G, pb.rho, h_ref, sel=sel)
    ph = np64(job.phi)[sel]
    out["phi_normwise"] = float(normwise(ph, ph_ref).max())
    out["phi_bar_ratio"] = float((np.abs(ph - ph_ref) / (1e-4 * phi_scale(theta, G, pb.rho, h_ref, sel) + 1e-300)).max())
    # one Adam step of the sampled particles from the GPU's inputs to it
    sub = orc.State(pb, pre["theta"][sel], pre["S"][sel], lam_lim=pre["lam_lim"][sel], lam_def=pre["lam_def"][sel],
                    adam_m=pre["adam_m"][sel], adam_v=pre["adam_v"][sel])
    gdef_in = np64(job.gdef)[sel][:, :, : pb.n_s - 1]
    orc.mdmm_step(pb, sub, np64(job.phi)[sel], np64(job.g_con)[sel], np64(job.S_dot)[sel][:, :, : pb.n_s - 1],
                  gdef_in, 1, 1)
    th_new = np64(job.theta)[sel]
    out["step_theta_normwise"] = float(normwise(th_new - pre["theta"][sel], sub.theta - pre["theta"][sel]).max())
    out["step_theta_bar_ratio"] = float(update_check(th_new, pre["theta"][sel], sub.theta).max())
    if pb.n_s > 1:
        S_new = np64(job.S)[sel]
        out["step_S_normwise"] = float(normwise(S_new - pre["S"][sel], sub.S - pre["S"][sel]).max())
        out["step_S_bar_ratio"] = float(update_check(S_new, pre["S"][sel], sub.S).max())
    out["seconds"] = time.time() - t0
    log(json.dumps(out))
    return out


def drift_c1(iters=100):
    """Particle-set mean and covariance of the pendulum problem after each
    of 100 Adam iterations on both sides, relative to the oracle's."""
    pb = f32_problem(synth.make_problem("c1"))
    obs = r32(orc.observations(pb))
    S = r32(orc.shooting_init(pb, pb.particles))
    st = orc.State(pb, pb.particles, S)
    job = L.Job(pb, obs, theta=pb.particles, S=S)
    b = L.Batch([job])
    curve = []
    for it in range(1, iters + 1):
        L.csvgd_iteration(b, it)
        orc.csvgd_iteration(pb, obs, st, it, optimizer=1)
        th = np64(job.theta)
        mu, mu_r = th.mean(0), st.theta.mean(0)
        cov, cov_r = np.cov(th.T), np.cov(st.theta.T)
        curve.append(dict(it=it, mean_rel=float((np.abs(mu - mu_r) / np.abs(mu_r)).max()),
                          cov_rel=float(np.linalg.norm(cov - cov_r) / np.linalg.norm(cov_r)),
                          particle_max=float(normwise(th, st.theta).max())))
    return curve


FIELDS = [("states", "states"), ("end_states", "end states"), ("ll_win_rel", "ℓ_win rel"),
          ("logp_rel", "log p rel"), ("wk_abs", "w abs"), ("gdef_rel", "g_def rel"),
          ("g_obs_normwise", "g_obs"), ("g_con_normwise", "g_con"), ("S_dot_normwise", "Ṡ"),
          ("bandwidth_rel", "h"), ("phi_normwise", "φ"), ("step_theta_normwise", "step θ"),
          ("step_S_normwise", "step S")]


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("out", nargs="?", help="JSON file for the rows and the drift curve")
    ap.add_argument("--workloads", nargs="*", default=WORKLOADS, choices=WORKLOADS)
    ap.add_argument("--no-drift", action="store_true", help="skip the pendulum's 100-iteration drift curve")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    L.lib()
    rows = [measure(c) for c in args.workloads]
    curve = [] if args.no_drift else drift_c1()
    print("| workload | " + " | ".join(n for _, n in FIELDS) + " |")
    print("|---" * (len(FIELDS) + 1) + "|")
    for r in rows:
        print("| %s | " % r["workload"] + " | ".join(
            ("%.1e" % r[k]) if k in r else "—" for k, _ in FIELDS) + " |")
    for c in curve:
        if c["it"] in (1, 2, 5, 10, 20, 50, 100):
            print("c1 drift it %3d: mean %.2e cov %.2e particle %.2e" % (c["it"], c["mean_rel"], c["cov_rel"],
                                                                       c["particle_max"]))
    if args.out:
        json.dump({"rows": rows, "c1_drift": curve}, open(args.out, "w"), indent=1)


if __name__ == "__main__":
    main()
