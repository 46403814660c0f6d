#!/usr/bin/env python3
"""Throughput of one CSVGD iteration (Algorithm 1) on one MI355X.

Workload (default): the largest single-GPU configuration -- the 7-joint arm
with a box on a passive hinge holding two 0.2 kg point masses at unknown
in-plane positions (M = 4), PD-tracking seeded sinusoids, the hinge angle
observed; N = 2048 particles, K = 1 trajectory of T = 1500 steps at
dt = 1/240 s, 30 shooting windows of 50 steps.  Synthetic data (seeded):
observations from the library's own rollout at the generating parameters
plus Gaussian noise.  --config selects the others (c1 pendulum, c2 double
pendulum, c3 5-link chain, rigid2, box1, box2).

A step is one full iteration over all particles: reverse-mode gradient of
the multiple-shooting likelihood and defects (sim_batch_adjoint), the SVGD
direction with the median-heuristic bandwidth (svgd_phi) and the MDMM/Adam
update (svgd_step).  Inputs are resident in HBM before the timed region.

Prints one JSON line: value = particle-sim-steps/s = N K T per iteration x
iterations / elapsed, plus the roofline of the dominant kernel (the window
forward+adjoint kernel) and the FP64 CPU oracle timed on a bounded sample
of the same workload on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32 (published)
# HBM traffic of the window-adjoint kernel per workload, from committed
# rocprofv3 counter summaries; valid while the kernel's source file hashes
# to the value recorded with the counters.
# Back-to-back launches of the window kernel per event pair when its
# duration is measured after the graph replays: an event pair adds the
# kernel's dispatch latency (a few microseconds) to what it brackets.
KERNEL_REPS = 8

ARM_SOURCES = ("arm.hip", "arm_math.h")
TRAFFIC_PROFILES = {
    "c2": ("planar_adjoint_c2_traffic.md", ("planar.hip",)),
    "c3": ("planar_adjoint_c3_traffic.md", ("planar.hip",)),
    "c4": ("arm_adjoint_c4_traffic.md", ARM_SOURCES),
    "rigid2": ("planar_adjoint_rigid2_traffic.md", ("planar.hip",)),
    "box1": ("arm_adjoint_box1_traffic.md", ARM_SOURCES),
    "box2": ("arm_adjoint_box2_traffic.md", ARM_SOURCES),
    "metrics_c3": ("metric_dist_c3_traffic.md", ("metrics.hip",)),
}


def source_hash(files):
    """sha256 of the kernel's source files, concatenated in order."""
    import hashlib

    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2109_08815_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(config):
    """HBM bytes per launch of the adjoint kernel from the committed PMC
    summary, or None when none covers this workload or the kernel source
    changed since the counters were taken."""
    if config not in TRAFFIC_PROFILES:
        return None
    prof, srcs = TRAFFIC_PROFILES[config]
    path = os.path.join(ROOT, "profiles", prof)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "source_sha256"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != source_hash(srcs) or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default=None, choices=["c1", "c2", "c3", "c4", "rigid2", "box1", "box2"],
                    help="workload (default c4; c3 with --metrics)")
    ap.add_argument("--metrics", action="store_true",
                    help="time the posterior-consistency metrics (KNN-KL both ways + MMD) between the particles' "
                         "rollouts and 10 held-out trajectories instead of the CSVGD iteration")
    ap.add_argument("--no-graph", action="store_true", help="plain launches instead of graph replay")
    ap.add_argument("--bandwidth", choices=["concurrent", "before", "after"], default="concurrent",
                    help="where the kernel bandwidth runs: on a second stream concurrently with the adjoint "
                         "(default), or on the iteration's stream before or after it")
    ap.add_argument("--no-overlap", action="store_true", help="same as --bandwidth after")
    ap.add_argument("--generic-dh", action="store_true",
                    help="arm configurations: a table off the Panda arm's kinematic structure (generic kernels)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB (20 times): the reference for HBM byte counters")
    return ap.parse_args()


def copy_calibration():
    """A plain copy of known size, for scaling FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    n = 64 * 1024 * 1024  # float32 elements = 256 MiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(20):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": 4 * n, "copies": 20}), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pb, obs, theta, S, target_s):
    """The FP64 oracle (forward-mode duals, OpenMP over window units) timed on
    a bounded sample: full CSVGD iterations over a subset of particles, on
    all host cores and, on a smaller sample, on one core."""
    from oracle import oracle as orc

    n_all = theta.shape[0]
    st = orc.State(pb, theta, S)
    lib = orc.lib()
    cores = int(lib.orc_threads())

    def timed(sel_n):
        sel = np.arange(sel_n, dtype=np.int32)
        t0 = time.perf_counter()
        orc.gradient(pb, obs, st, sel=sel)
        h, _ = orc.bandwidth(st.theta, pb.rho)
        orc.phi(st.theta, np.zeros((n_all, pb.M)), pb.rho, h, sel=sel)
        return time.perf_counter() - t0

    probe = max(1, min(n_all, 16))
    per_particle = timed(probe) / probe
    sel_n = int(max(1, min(n_all, target_s / max(per_particle, 1e-9))))
    # whole iterations over every particle, repeated to fill the time budget
    reps = max(1, int(target_s / max(per_particle * n_all, 1e-9))) if sel_n == n_all else 1
    el = sum(timed(sel_n) for _ in range(reps))
    out = {
        "value": reps * sel_n * pb.K * pb.T / el,
        "unit": "particle-sim-steps/s",
        "cores": cores,
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": "%d of %d particles, all %d trajectories x %d steps: forward-mode-dual gradient, bandwidth "
                  "and phi rows, %d iteration(s), %.1f s" % (sel_n, n_all, pb.K, pb.T, reps, el),
    }
    # fairer floor: the oracle's forward-only rollout (likelihood and
    # defects, no derivatives) on the same cores, a quarter of the budget
    probe_f = max(1, min(n_all, 16))
    selp = np.arange(probe_f, dtype=np.int32)
    t0 = time.perf_counter()
    orc.forward(pb, obs, st, sel=selp)
    per_f = (time.perf_counter() - t0) / probe_f
    nf = int(max(1, min(n_all, 0.25 * target_s / max(per_f, 1e-9))))
    repf = max(1, int(0.25 * target_s / max(per_f * n_all, 1e-9))) if nf == n_all else 1
    t0 = time.perf_counter()
    for _ in range(repf):
        orc.forward(pb, obs, st, sel=np.arange(nf, dtype=np.int32))
    elf = time.perf_counter() - t0
    out["forward_only_value"] = repf * nf * pb.K * pb.T / elf
    out["forward_only_sample"] = "%d of %d particles, forward rollout and likelihood only, %d pass(es), %.1f s" % (
        nf, n_all, repf, elf)
    # one core, on a quarter of the time budget
    lib.orc_set_threads(1)
    try:
        one = max(1, min(n_all, int(0.25 * target_s / max(per_particle * cores, 1e-9))))
        el1 = timed(one)
        out["value_1_core"] = one * pb.K * pb.T / el1
        out["sample_1_core"] = "%d particles, %.1f s" % (one, el1)
    finally:
        lib.orc_set_threads(cores)
    return out


METRIC_HELD_OUT = 10


def run_metrics(args):
    """Posterior-consistency metrics (Sec. III-F, App. A-D) between the N
    particles' rollouts from the first trajectory's start state and
    METRIC_HELD_OUT held-out trajectories (the generating parameters'
    rollout plus fresh observation noise), each row the observed joint
    angles of all T steps.  A step is one pds_traj_metrics call."""
    import torch

    from paper_2109_08815_amd import driver, synth
    from paper_2109_08815_amd import lib as L

    pb = synth.make_problem(args.config)
    dev = torch.device("cuda")
    tr = driver.gpu_observed_rollout(pb, pb.particles, dev)  # [N, K, T, d_x]
    P = tr[:, 0].reshape(pb.N, -1).float().contiguous()
    del tr
    tt = driver.gpu_observed_rollout(pb, pb.theta_true[:1], dev)[0, 0].reshape(1, -1).double()
    rng = np.random.Generator(np.random.PCG64(pb.seed + 77))
    noise = rng.normal(0.0, pb.sigma_obs, (METRIC_HELD_OUT, tt.shape[1]))
    Q = (tt + torch.as_tensor(noise, device=dev)).float().contiguous()
    n, d = P.shape
    m = Q.shape[0]
    R = n + m
    ws = torch.empty(L.traj_metrics_workspace(n, m, d), dtype=torch.uint8, device=dev)
    for _ in range(max(1, args.warmup)):
        out = L.traj_metrics(P, Q, ws=ws)
    torch.cuda.synchronize()
    L.timing_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        out = L.traj_metrics(P, Q, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    elapsed = max(e0.elapsed_time(e1) / 1e3, 1e-12)
    kt = L.timing_read()
    L.timing_enable(False)
    k_ms = float(np.mean(kt)) if len(kt) else float("nan")
    pairs = R * (R - 1) // 2
    flops = 3.0 * pairs * d  # difference, multiply, add per pair and coordinate
    res = out.cpu().numpy()
    line = {
        "metric": "trajectory-pair-coordinates/s (KNN-KL both ways + MMD)",
        "value": pairs * d * args.steps / elapsed,
        "unit": "pair-coordinates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 sums, logs, kernel values and median)",
        "data": "synthetic",
        "config": {"workload": "%s rollouts: %d particle rollouts vs %d held-out trajectories, d = T x d_x = %d x %d"
                               % (args.config, n, m, pb.T, pb.d_x), "k": 3, "l": 3},
        "outputs": {"kl_sim_real": float(res[0]), "kl_real_sim": float(res[1]), "mmd2": float(res[2]),
                    "sigma": float(res[3])},
        "wall_s": wall,
        "roofline": {
            "bound": "alu",
            "achieved": flops / (k_ms / 1e3) / 1e12,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": flops / (k_ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS,
            "traffic": measured_traffic("metrics_" + args.config),
            "kernel": "metric_dist_kernel (+ metric_dist_reduce_kernel of the coordinate splits)",
            "kernel_ms": k_ms,
            "flops_per_launch": flops,
        },
    }
    if not args.no_cpu_baseline:
        from oracle import metrics as om

        Ph, Qh = P.cpu().numpy().astype(np.float64), Q.cpu().numpy().astype(np.float64)
        ns, t = 32, 0.0
        while True:
            t0 = time.perf_counter()
            om.metrics(Ph[:ns], Qh)
            t = time.perf_counter() - t0
            if t > 0.25 * args.cpu_seconds or ns >= n:
                break
            ns = min(n, ns * 2)
        rs = ns + m
        line["cpu_baseline"] = {"value": rs * (rs - 1) // 2 * d / t, "unit": "pair-coordinates/s", "cores": 1,
                                "kind": "oracle",
                                "sample": "the oracle's metrics (explicit FP64 differences, numpy) on the first %d "
                                          "rollouts and the %d held-out trajectories, %.1f s" % (ns, m, t)}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the method's data-parallel path runs on a single device "
              "(see the sharding note in DESIGN.md); got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2109_08815_amd import driver, synth
    from paper_2109_08815_amd import lib as L

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    L.lib()
    if args.metrics:
        args.config = args.config or "c3"
        run_metrics(args)
        return
    args.config = args.config or "c4"
    pb = synth.make_problem(args.config, generic_dh=args.generic_dh)
    print("setup %s N=%d K=%d T=%d n_s=%d" % (args.config, pb.N, pb.K, pb.T, pb.n_s), file=sys.stderr, flush=True)
    obs = driver.gpu_observations(pb)
    S = driver.gpu_shooting_init(pb, pb.particles)
    job = L.Job(pb, obs, theta=pb.particles, S=S, device_iter=True)
    if args.no_overlap:
        args.bandwidth = "after"
    run = driver.CSVGD([job], overlap={"concurrent": True, "before": "before", "after": False}[args.bandwidth])
    for _ in range(max(1, args.warmup)):
        run.step()
    torch.cuda.synchronize()
    use_graph = not args.no_graph
    # iterations per captured graph: at least 20 replays for the percentiles
    per_graph = max(1, min(10, args.steps // 20))
    if args.steps % per_graph:
        per_graph = 1
    if use_graph:
        run.capture(per_graph)
        run.replay()
        torch.cuda.synchronize()

    # ---- timed region ----
    if not use_graph:
        L.timing_enable(True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    marks = []
    if use_graph:
        for _ in range(args.steps // per_graph):
            ev = torch.cuda.Event(enable_timing=True)
            ev.record()
            marks.append(ev)
            run.replay()
    else:
        for _ in range(args.steps):
            run.step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    # per-iteration time of each graph replay (events between replays)
    per_iter = [a.elapsed_time(b) / per_graph for a, b in zip(marks, marks[1:] + [e1])] if marks else []
    if use_graph:
        # kernel timing: the same iteration with plain launches right after,
        # each window-kernel launch repeated back to back inside its event
        # pair, with the bandwidth after the adjoint so that no concurrent
        # kernel takes compute units from the timed one
        timed = driver.CSVGD([job], overlap=False)
        L.timing_enable(True, reps=KERNEL_REPS)
        for _ in range(min(args.steps, 200)):
            timed.step()
        torch.cuda.synchronize()
    kt = L.timing_read()
    L.timing_enable(False)
    elapsed = max(ms / 1e3, wall) if ms > 0 else wall
    steps_per_iter = pb.N * pb.K * pb.T
    value = steps_per_iter * args.steps / elapsed

    k_ms = float(np.mean(kt)) if len(kt) else float("nan")
    model, raw = L.model_consts(pb)
    if model in (L.PDS_MODEL_ARM, L.PDS_MODEL_ARM_UJOINT, L.PDS_MODEL_ARM_UJOINT_WEIGHTS):
        # the step the kernels run for this table's kinematic structure
        fwd, rev, transc, panda = L.arm_algorithmic_flops(model, raw)
    else:
        fwd, rev, transc = L.algorithmic_flops(model, pb.n_dof)
        panda = None
    per_step = fwd + 2 * rev  # forward step + reverse step of each of the two adjoint channels
    achieved = steps_per_iter * per_step / (k_ms / 1e3) / 1e12
    finite = bool(torch.isfinite(job.theta).all().item())
    out = {
        "metric": "particle-sim-steps/s (fwd+adjoint)",
        "value": value,
        "unit": "particle-sim-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 accumulation and median)",
        "data": "synthetic",
        "config": {"workload": "%s: %s N=%d M=%d K=%d T=%d dt=%g n_s=%d" % (
            args.config, {"c1": "pendulum", "c2": "double pendulum", "c3": "5-link chain",
                          "c4": "7-joint arm with hinged box",
                          "rigid2": "rigid-link double pendulum",
                          "box1": "7-joint arm with the box on a universal joint",
                          "box2": "7-joint arm with two weights in the box on a universal joint"}[args.config],
            pb.N, pb.M, pb.K, pb.T, pb.dt, pb.n_s) + (", table off the Panda structure" if args.generic_dh else ""),
            "launch": ("graph of %d iterations" % per_graph) if use_graph else "plain",
            "bandwidth": {"concurrent": "concurrent with the adjoint", "before": "before the adjoint",
                          "after": "after the adjoint"}[args.bandwidth]},
        "iters_per_s": args.steps / elapsed,
        "iteration_ms": ({"p10": float(np.percentile(per_iter, 10)), "p50": float(np.percentile(per_iter, 50)),
                          "p90": float(np.percentile(per_iter, 90)), "replays": len(per_iter)} if per_iter else None),
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": measured_traffic(args.config),
            "kernel": ("arm_adjoint_kernel<%s>%s" % ({L.PDS_MODEL_ARM: "hinge", L.PDS_MODEL_ARM_UJOINT: "universal joint",
                                                      L.PDS_MODEL_ARM_UJOINT_WEIGHTS: "universal joint, weights"}[model],
                                                     ", Panda structure" if panda else ", generic structure"))
            if model in (L.PDS_MODEL_ARM, L.PDS_MODEL_ARM_UJOINT, L.PDS_MODEL_ARM_UJOINT_WEIGHTS) else "planar_adjoint_kernel<%d, %s links>" % (
                pb.n_dof, "rigid" if model == L.PDS_MODEL_PLANAR_RIGID else "point-mass"),
            "kernel_ms": k_ms,
            "kernel_timing": ("HIP events on the kernel's stream, %d back-to-back launches per pair, plain launches "
                              "with the bandwidth serialised, after the timed replays" % KERNEL_REPS) if use_graph else
                             "HIP events on the kernel's stream around each launch in the timed region",
            "flops_per_particle_step": per_step,
        },
        "finite": finite,
    }
    if not args.no_cpu_baseline:
        th = pb.particles
        out["cpu_baseline"] = cpu_baseline(pb, obs, th, S, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
