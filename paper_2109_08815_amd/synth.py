"""Seeded synthetic inputs for CSVGD inference problems.

This module only draws random numbers and lays out constants.  It contains
none of the method's arithmetic: observed trajectories are produced by the
caller as ``rollout(theta_true, s0) + noise`` with whichever simulator it is
checking (the FP64 oracle in the tests, the GPU library in the benchmark),
and initial shooting states likewise come from the caller's own rollout.

Problem families (shapes follow the paper's workloads; the data are
synthetic stand-ins for the recordings the paper used, Sec. IV):

* ``c1``  simple pendulum, theta = (m, l)                         (M = 2)
* ``c2``  unactuated double pendulum, theta = (m1, m2, l1, l2)     (M = 4);
  400 steps split into 10 shooting windows as in Sec. III-C / Fig. 2
* ``c3``  5-link planar chain with known joint damping, theta = masses and
  lengths                                                          (M = 10)
* ``c4``  7-joint arm (seeded synthetic modified-DH table) tracking a
  sinusoidal joint trajectory with PD control, carrying a box on a passive
  hinge that holds two 0.2 kg point masses at unknown in-plane positions
  theta = (x_a, y_a, x_b, y_b)                                     (M = 4);
  the synthetic analogue of the arm-and-box experiment of Sec. IV-C
* ``rigid2`` double pendulum with rigid links, the 11 parameters of the
  paper's physical double pendulum (Sec. IV-B): per link mass, inertia
  about the centre of mass, centre of mass (x, y) and joint friction, plus
  the length of link 2, inside that table's bounds; observes the whole
  state (q, qd) as that experiment does                             (M = 11)
* ``box1`` the 7-joint arm carrying the box on a passive universal joint
  (Sec. IV-C and its appendix, phase I): the box's inertia about its
  centre of mass (xx, yy, zz, xy, xz, yz), its centre of mass and the
  viscous friction of the two joint axes, inside the phase-I table's
  bounds; box mass 0.92 kg known; observes the box frame (origin and the
  points 1 m along its axes, 12 numbers)                           (M = 11)
* ``box2`` the same universal-joint mount with the box's phase-I values
  known and two 0.5 kg weights on the box floor (phase II): theta = their
  in-plane positions inside the phase-II table's bounds; observes the box
  frame                                                            (M = 4)
* ``toy`` one prismatic unit mass driven by force theta0 (+ theta1 * time),
  the linear-Gaussian check problem                                 (M = 1, 2)

Random streams: ``numpy.random.Generator(PCG64(seed))``.
Initial particles: unscrambled Sobol points (App. A-A) with the all-zero
first point skipped, scaled into the parameter limits.
"""
from __future__ import annotations

import math
import warnings
from dataclasses import dataclass, field

import numpy as np

KIND_PLANAR = 1
KIND_ARM = 2
KIND_TOY = 3
KIND_PLANAR_RIGID = 4
KIND_ARM_UJOINT = 5
KIND_ARM_UJOINT_WEIGHTS = 6

COMBINE_SUM = 0
COMBINE_PROD = 1
LIK_MDMM = 0    # defects as MDMM equality constraints (CSVGD)
LIK_DEFECT = 1  # defects as Gaussian factors inside the multiple-shooting likelihood
LIMITS_SOFT = 0     # parameter limits through MDMM only
LIMITS_PROJECT = 1  # ... and theta clamped into [lo, hi] after every step


@dataclass
class Problem:
    """Everything both simulators need for one inference job (host arrays)."""

    name: str
    kind: int
    n_dof: int
    M: int
    d_x: int
    obs_index: np.ndarray
    gravity: np.ndarray
    damping: np.ndarray           # [8]
    arm: dict | None              # arm constants (kind == KIND_ARM)
    N: int
    K: int
    T: int
    n_s: int
    h: int
    dt: float
    sigma_obs: float
    sigma_def: float
    c: float
    combine: int
    lo: np.ndarray
    hi: np.ndarray
    theta_true: np.ndarray        # [K, M] parameters that generated each trajectory
    s0: np.ndarray                # [K, d_s]
    noise: np.ndarray             # [K, T, d_x] observation noise draws
    particles: np.ndarray         # [N, M] initial particles
    w_x: np.ndarray               # [d_x]
    u: np.ndarray                 # [d_s]
    rho: np.ndarray               # [M]
    lr_theta: np.ndarray          # [M]
    lr_S: np.ndarray              # [d_s]
    eps_lam: float
    seed: int
    lik: int = 0                  # LIK_MDMM or LIK_DEFECT (how the defects enter)
    limits: int = 0               # LIMITS_SOFT or LIMITS_PROJECT
    extra: dict = field(default_factory=dict)

    @property
    def d_s(self) -> int:
        return 2 * self.n_dof


# Headline shapes: (family, N, K, T, n_s, dt, sigma_obs)
CONFIGS = {
    "c1": dict(family="pendulum", N=32, K=1, T=200, n_s=4, dt=0.01, sigma_obs=0.01),
    "c2": dict(family="double", N=256, K=4, T=400, n_s=10, dt=0.005, sigma_obs=0.01),
    "c3": dict(family="chain5", N=1024, K=8, T=1000, n_s=20, dt=0.002, sigma_obs=0.02),
    "rigid2": dict(family="rigid", N=256, K=4, T=400, n_s=10, dt=0.005, sigma_obs=0.01),
    "box1": dict(family="ujoint", N=2048, K=1, T=1500, n_s=30, dt=1.0 / 240.0, sigma_obs=0.01),
    "box2": dict(family="ujoint_weights", N=2048, K=1, T=1500, n_s=30, dt=1.0 / 240.0, sigma_obs=0.01),
    "c4": dict(family="arm", N=2048, K=1, T=1500, n_s=30, dt=1.0 / 240.0, sigma_obs=0.01),
}


def sobol_particles(N: int, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Unscrambled Sobol points 1..N (point 0 is the origin) scaled to [lo, hi]."""
    from scipy.stats import qmc

    M = len(lo)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        pts = qmc.Sobol(d=M, scramble=False).random(N + 1)[1:]
    return lo[None, :] + pts * (hi - lo)[None, :]


def _arm_constants(rng: np.random.Generator) -> dict:
    """Seeded synthetic 7-joint arm, box and hinge.  Not any real robot's table."""
    alpha = np.array([0.0, -np.pi / 2, np.pi / 2, np.pi / 2, -np.pi / 2, np.pi / 2, np.pi / 2])
    a = np.array([0.0, 0.0, 0.0, rng.uniform(0.05, 0.1), -rng.uniform(0.05, 0.1), 0.0, rng.uniform(0.05, 0.1)])
    d = np.array([rng.uniform(0.3, 0.35), 0.0, rng.uniform(0.3, 0.35), 0.0, rng.uniform(0.35, 0.4), 0.0, 0.0])
    m = np.concatenate([rng.uniform(2.5, 4.0, 3), rng.uniform(1.5, 2.5, 2), rng.uniform(0.5, 1.5, 2)])
    com = rng.uniform(-0.05, 0.05, (7, 3))
    r, L = 0.05, 0.3
    inertia = np.stack([np.array([mi * (3 * r * r + L * L) / 12.0, mi * (3 * r * r + L * L) / 12.0, 0.5 * mi * r * r]) for mi in m])
    # Fixed gain table: natural frequency 6 rad/s on nominal joint inertias.
    # Semi-implicit Euler at dt = 1/240 stays stable for every seed tried
    # with these gains (stiffer tables were not).
    I_nom = np.array([1.0, 3.0, 0.2, 1.0, 0.1, 0.15, 0.08])
    wn = 6.0
    kp = wn * wn * I_nom
    kd = 2.0 * wn * I_nom
    qc = rng.uniform(-0.5, 0.5, 7)
    amp = rng.uniform(0.05, 0.3, 7)
    omega = rng.uniform(1.0, 4.0, 7)
    phase = rng.uniform(0.0, 2 * np.pi, 7)
    return dict(
        dh_a=a, dh_alpha=alpha, dh_d=d, link_m=m, link_c=com, link_I=inertia,
        kp=kp, kd=kd, qc=qc, amp=amp, omega=omega, phase=phase,
        flange_d=0.1, box_m=0.92, box_c=np.array([0.0, 0.0, -0.25]),
        box_I=np.array([0.075, 0.075, 0.075]), pm_m=0.2, pm_z=-0.40, hinge_damping=0.05,
    )


def make_problem(config: str = "c2", seed: int | None = None, **over) -> Problem:
    """Build a seeded problem.  ``over`` overrides N, K, T, n_s, dt, sigma_obs,
    sigma_def, c, combine, lik, limits, n_dof (planar families), full_state (planar
    families: observe (q, qd) instead of q), damped, gravity_x (point-mass
    planar families: joint damping, a gravity component along x), M (toy),
    generic_dh (arm families: a table off the Panda arm's kinematic
    structure)."""
    base = dict(CONFIGS.get(config, {}))
    if config == "toy":
        base = dict(family="toy", N=256, K=1, T=50, n_s=1, dt=0.1, sigma_obs=0.5)
    base.update({k: v for k, v in over.items() if k in ("N", "K", "T", "n_s", "dt", "sigma_obs")})
    fam = base["family"]
    idx = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "rigid2": 5, "box1": 6, "box2": 8, "toy": 9}.get(config, 7)
    if seed is None:
        seed = 1000 * idx
    rng = np.random.Generator(np.random.PCG64(seed))
    N, K, T, n_s, dt = int(base["N"]), int(base["K"]), int(base["T"]), int(base["n_s"]), float(base["dt"])
    if T % n_s != 0:
        raise ValueError("T must be a multiple of n_s")
    h = T // n_s
    arm = None
    damping = np.zeros(8)
    if fam in ("pendulum", "double", "chain5"):
        kind = KIND_PLANAR
        n = int(over.get("n_dof", {"pendulum": 1, "double": 2, "chain5": 5}[fam]))
        M = 2 * n
        lo = np.array([0.5] * n + [0.5] * n)
        hi = np.array([2.0] * n + [1.5] * n)
        if fam == "chain5" or over.get("damped", False):
            damping[:n] = rng.uniform(0.0, 0.1, n)
        gravity = np.array([float(over.get("gravity_x", 0.0)), -9.81, 0.0])
        d_x = 2 * n if over.get("full_state", False) else n
        obs_index = np.arange(d_x)
        qmax = np.pi if fam == "double" else np.pi / 2
        s0 = np.zeros((K, 2 * n))
        s0[:, :n] = rng.uniform(-qmax, qmax, (K, n))
    elif fam == "rigid":
        kind = KIND_PLANAR_RIGID
        n = int(over.get("n_dof", 2))
        if n not in (1, 2):
            raise ValueError("the rigid planar family has 1 or 2 links")
        M = 6 * n - 1
        # Bounds of the Sec. IV-B table: mass, inertia, COM x, COM y, friction
        # per link, the length of link 2 ahead of its block.
        link_lo, link_hi = [0.05, 0.002, -0.2, -0.2, 0.0], [0.5, 1.0, 0.2, 0.2, 0.5]
        lo = np.array(link_lo + ([0.08] + link_lo) * (n - 1))
        hi = np.array(link_hi + ([0.3] + link_hi) * (n - 1))
        gravity = np.array([0.0, -9.81, 0.0])
        # the whole state is observed, as in the paper's pendulum experiment
        d_x = 2 * n if over.get("full_state", True) else n
        obs_index = np.arange(d_x)
        s0 = np.zeros((K, 2 * n))
        s0[:, :n] = rng.uniform(-np.pi / 2, np.pi / 2, (K, n))
    elif fam == "arm":
        kind = KIND_ARM
        n = 8
        M = 4
        lo = np.full(4, -0.1)
        hi = np.full(4, 0.1)
        arm = _arm_constants(rng)
        damping[7] = arm["hinge_damping"]
        gravity = np.array([0.0, 0.0, -9.81])
        d_x = 1
        obs_index = np.array([7])
        s0 = np.zeros((K, 16))
        s0[:, :7] = arm["qc"] + arm["amp"] * np.sin(arm["phase"])
        s0[:, 8:15] = arm["amp"] * arm["omega"] * np.cos(arm["phase"])
    elif fam == "ujoint":
        kind = KIND_ARM_UJOINT
        n = 9
        M = 11
        # phase-I table: inertia diagonal, products of inertia, COM, joint friction
        lo = np.array([0.05, 0.05, 0.05, -0.01, -0.01, -0.01, -0.005, -0.005, 0.1, 0.0, 0.0])
        hi = np.array([0.1, 0.1, 0.1, 0.01, 0.01, 0.01, 0.005, 0.005, 0.4, 0.15, 0.15])
        arm = _arm_constants(rng)
        arm["box_m"] = 0.92
        gravity = np.array([0.0, 0.0, -9.81])
        d_x = 12
        obs_index = np.arange(12)
        s0 = np.zeros((K, 18))
        s0[:, :7] = arm["qc"] + arm["amp"] * np.sin(arm["phase"])
        s0[:, 9:16] = arm["amp"] * arm["omega"] * np.cos(arm["phase"])
    elif fam == "ujoint_weights":
        kind = KIND_ARM_UJOINT_WEIGHTS
        n = 9
        M = 4
        lo = np.array([-0.14, -0.08, -0.14, -0.08])
        hi = np.array([0.14, 0.08, 0.14, 0.08])
        arm = _arm_constants(rng)
        # the empty box as phase I would have found it (seeded, inside that
        # table's bounds), two 0.5 kg weights on its floor
        arm["box_m"] = 0.92
        arm["box_c"] = np.array([rng.uniform(-0.005, 0.005), rng.uniform(-0.005, 0.005), rng.uniform(0.1, 0.4)])
        arm["box_I"] = rng.uniform(0.05, 0.1, 3)
        arm["box_Ioff"] = rng.uniform(-0.01, 0.01, 3)
        arm["ujoint_b"] = rng.uniform(0.0, 0.15, 2)
        arm["pm_m"] = 0.5
        arm["pm_z"] = 0.4
        gravity = np.array([0.0, 0.0, -9.81])
        d_x = 12
        obs_index = np.arange(12)
        s0 = np.zeros((K, 18))
        s0[:, :7] = arm["qc"] + arm["amp"] * np.sin(arm["phase"])
        s0[:, 9:16] = arm["amp"] * arm["omega"] * np.cos(arm["phase"])
    elif fam == "toy":
        kind = KIND_TOY
        n = 1
        M = int(over.get("M", 1))
        lo = np.full(M, -50.0)
        hi = np.full(M, 50.0)
        gravity = np.zeros(3)
        d_x = 1
        obs_index = np.array([0])
        s0 = np.zeros((K, 2))
    else:
        raise ValueError(fam)
    sigma_obs = float(base["sigma_obs"])
    theta_true = lo + rng.uniform(0.0, 1.0, (K, M)) * (hi - lo)
    if fam == "toy":
        theta_true = np.tile(np.array([1.5, -0.4][:M]), (K, 1))
    if over.get("same_theta", True) and fam != "toy":
        theta_true = np.tile(theta_true[:1], (K, 1))
    noise = rng.normal(0.0, sigma_obs, (K, T, d_x))
    # Adam moves every coordinate by about lr per iteration whatever the
    # gradient's size, and the limits act only softly (MDMM); the rigid
    # links' inertias sit near their lower bound (0.002 of a 1.0 range), so
    # that family takes smaller steps to keep them positive.
    lr_frac = 1e-3 if fam == "rigid" else 1e-2
    particles = sobol_particles(N, lo, hi)
    if arm is not None and over.get("generic_dh", False):
        # a table off the Panda arm's kinematic structure: one twist off its
        # right angle, two offsets that structure has as zeros
        arm["dh_alpha"] = arm["dh_alpha"] + np.array([0.0, 0.25, 0.0, 0.0, 0.0, 0.0, 0.0])
        arm["dh_a"] = arm["dh_a"] + np.array([0.0, 0.04, 0.0, 0.0, 0.0, 0.0, 0.0])
        arm["dh_d"] = arm["dh_d"] + np.array([0.0, 0.0, 0.0, 0.06, 0.0, 0.0, 0.0])
    d_s = 2 * n
    u = np.ones(d_s)
    lr_S = np.concatenate([np.full(n, 1e-3), np.full(n, 1e-2)])
    return Problem(
        name=config, kind=kind, n_dof=n, M=M, d_x=d_x, obs_index=obs_index, gravity=gravity,
        damping=damping, arm=arm, N=N, K=K, T=T, n_s=n_s, h=h, dt=dt, sigma_obs=sigma_obs,
        sigma_def=float(over.get("sigma_def", 0.1)), c=float(over.get("c", 1.0)),
        combine=int(over.get("combine", COMBINE_SUM)), lo=lo, hi=hi, theta_true=theta_true,
        s0=s0, noise=noise, particles=particles, w_x=np.full(d_x, 1.0 / sigma_obs), u=u,
        rho=hi - lo, lr_theta=lr_frac * (hi - lo), lr_S=lr_S, eps_lam=1e-2, seed=seed,
        lik=int(over.get("lik", LIK_MDMM)),
        # rigid links: masses and inertias must stay positive, and their
        # lower limits sit within one Adam step of zero; the box's inertia
        # must stay positive definite
        limits=int(over.get("limits", LIMITS_PROJECT if fam in ("rigid", "ujoint") else LIMITS_SOFT)),
    )


def random_states(rng: np.random.Generator, n_dof: int, count: int, qmax: float = math.pi,
                  vmax: float = 2.0) -> np.ndarray:
    """Random joint states [count, 2 n_dof] for dynamics spot checks."""
    q = rng.uniform(-qmax, qmax, (count, n_dof))
    v = rng.uniform(-vmax, vmax, (count, n_dof))
    return np.concatenate([q, v], axis=1)


def perturb(rng: np.random.Generator, x: np.ndarray, scale: float) -> np.ndarray:
    """Additive Gaussian perturbation of an array (e.g. shooting states)."""
    return x + rng.normal(0.0, scale, x.shape)


# ---------------------------------------------------------------------------
# Serving trace
# ---------------------------------------------------------------------------

@dataclass
class JobSpec:
    """One inference job of a serving trace: a seeded problem plus when it
    arrives (seconds from the start of the trace) and how many CSVGD
    iterations it runs."""

    job_id: int
    family: str
    N: int
    K: int
    T: int
    seed: int
    iterations: int
    arrival: float = 0.0
    limits: int | None = None  # LIMITS_SOFT / LIMITS_PROJECT, None: the family's default

    def problem(self) -> "Problem":
        over = {} if self.limits is None else {"limits": self.limits}
        return make_problem(self.family, seed=self.seed, N=self.N, K=self.K, T=self.T, n_s=self.T // SERVE_H,
                            **over)


SERVE_H = 50  # window length of every serving job
SERVE_T = (200, 400, 600, 800, 1000, 1200, 1500)


def serving_trace(n_jobs: int = 512, seed: int = 5000, iterations: int = 100, rate: float | None = None,
                  families=("c1", "c2", "c3"), max_log2_n: int = 5, limits: int | None = None,
                  shape: tuple | None = None) -> list[JobSpec]:
    """The mixed serving workload: family uniform over the planar problems,
    N = 64 * 2^u with u uniform on 0..max_log2_n, T uniform over SERVE_T
    (windows of SERVE_H steps), K uniform on 1..8.  With `rate` (jobs/s)
    the arrivals are a Poisson process, else every job arrives at 0.
    `limits` sets every job's limits mode (None: each family's default).
    `shape` = (family, N, K, T) gives every job that shape instead
    (homogeneous traffic; seeds and arrivals as in the mixed trace)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    t = 0.0
    for j in range(n_jobs):
        fam = families[int(rng.integers(len(families)))]
        N = 64 * 2 ** int(rng.integers(max_log2_n + 1))
        T = int(SERVE_T[int(rng.integers(len(SERVE_T)))])
        K = int(rng.integers(1, 9))
        if shape is not None:
            fam, N, K, T = shape
        if rate is not None:
            t += float(rng.exponential(1.0 / rate))
        out.append(JobSpec(j, fam, N, K, T, seed=seed * 1000 + j, iterations=iterations,
                           arrival=t if rate is not None else 0.0, limits=limits))
    return out


def metric_sets(seed: int, n: int, m: int, d: int, spread: float = 1.0, shift: float = 0.3):
    """Two seeded sets of trajectory-like rows for the consistency metrics
    (float32, [n, d] and [m, d]): a shared random-walk path, plus per-row
    random walks (step 0.05 * spread for P, 0.05 for Q) and, for Q, a
    constant offset `shift`.  Neighbouring rows are close, as rollouts of
    nearby particles are."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = np.cumsum(rng.normal(0.0, 0.1, (1, d)), axis=1)
    P = base + np.cumsum(rng.normal(0.0, 0.05 * spread, (n, d)), axis=1)
    Q = base + shift + np.cumsum(rng.normal(0.0, 0.05, (m, d)), axis=1)
    return P.astype(np.float32), Q.astype(np.float32)

