"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these compares the oracle with itself: each check uses a closed
form, an invariant, an independent textbook algorithm, a brute force, or a
hand-worked value from tests/golden/.  They are chosen so that a dropped
term, a wrong sign or index, or a transposed operand in the oracle fails at
least one of them.
"""
import itertools
import json
import math
import os
import statistics

import numpy as np
import pytest

from paper_2109_08815_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Dynamics (App. B-A: ABA forward dynamics + semi-implicit Euler)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("cfg", ["c1", "c2", "c3", "c4", "rigid2", "box1", "box2", "toy"])
def test_aba_equals_crba_rnea(orc, cfg):
    """ABA's q_dd equals H^{-1}(tau - C) from CRBA + RNEA (independent algorithms)."""
    pb = synth.make_problem(cfg, N=4, K=1, T=10, n_s=1)
    rng = np.random.default_rng(11)
    for _ in range(10):
        th = pb.lo + rng.uniform(size=pb.M) * (pb.hi - pb.lo)
        s = synth.random_states(rng, pb.n_dof, 1)[0]
        q, qd = s[: pb.n_dof], s[pb.n_dof:]
        tau = rng.normal(size=pb.n_dof)
        qdd = orc.aba(pb, th, q, qd, tau)
        H, Cb = orc.crba_rnea(pb, th, q, qd)
        ref = np.linalg.solve(H, tau - Cb)
        assert np.max(np.abs(qdd - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_pendulum_closed_form(orc):
    """Point-mass pendulum: q_dd = -(g/l) sin q - b q_d / (m l^2)."""
    pb = synth.make_problem("c1", damped=True)
    b = pb.damping[0]
    assert b > 0
    rng = np.random.default_rng(3)
    for _ in range(20):
        m, l = rng.uniform(0.5, 2.0), rng.uniform(0.5, 1.5)
        q, qd = rng.uniform(-3, 3), rng.uniform(-3, 3)
        tau = orc.tau(pb, [m, l], 0.0, [q], [qd])
        qdd = orc.aba(pb, [m, l], [q], [qd], tau)[0]
        ref = -(9.81 / l) * math.sin(q) - b * qd / (m * l * l)
        assert abs(qdd - ref) <= 1e-13 * max(1.0, abs(ref))


def test_double_pendulum_lagrangian(orc):
    """Textbook Lagrange equations of the point-mass double pendulum in
    absolute angles phi1 = q1, phi2 = q1 + q2 (measured from the downward
    vertical)."""
    pb = synth.make_problem("c2")
    g = 9.81
    rng = np.random.default_rng(5)
    for _ in range(20):
        m1, m2 = rng.uniform(0.5, 2, 2)
        l1, l2 = rng.uniform(0.5, 1.5, 2)
        q = rng.uniform(-3, 3, 2)
        qd = rng.uniform(-3, 3, 2)
        p1, p2 = q[0], q[0] + q[1]
        w1, w2 = qd[0], qd[0] + qd[1]
        dlt = p1 - p2
        A = np.array([[(m1 + m2) * l1, m2 * l2 * math.cos(dlt)], [l1 * math.cos(dlt), l2]])
        rhs = np.array([-m2 * l2 * w2 * w2 * math.sin(dlt) - (m1 + m2) * g * math.sin(p1),
                        l1 * w1 * w1 * math.sin(dlt) - g * math.sin(p2)])
        a1, a2 = np.linalg.solve(A, rhs)
        ref = np.array([a1, a2 - a1])
        qdd = orc.aba(pb, [m1, m2, l1, l2], q, qd, [0.0, 0.0])
        assert np.max(np.abs(qdd - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref)))


def test_rigid_link_compound_pendulum(orc):
    """One rigid link with its centre of mass at (cx, cy) in the link frame:
    (I + m |c|^2) q_dd = -m g (cx cos q - cy sin q) - b q_d (potential
    m g y_com with y_com = cx sin q + cy cos q)."""
    pb = synth.make_problem("rigid2", n_dof=1, N=4, K=1, T=10, n_s=1)
    assert pb.M == 5
    rng = np.random.default_rng(13)
    g = 9.81
    for _ in range(20):
        th = pb.lo + rng.uniform(size=5) * (pb.hi - pb.lo)
        m, I, cx, cy, b = th
        q, qd = rng.uniform(-3, 3), rng.uniform(-3, 3)
        tau = orc.tau(pb, th, 0.0, [q], [qd])
        qdd = orc.aba(pb, th, [q], [qd], tau)[0]
        ref = (-m * g * (cx * math.cos(q) - cy * math.sin(q)) - b * qd) / (I + m * (cx * cx + cy * cy))
        assert abs(qdd - ref) <= 1e-12 * max(1.0, abs(ref))


def _rigid_double_lagrange():
    """Euler-Lagrange equations of two rigid planar links, derived
    symbolically from their kinetic and potential energy: returns
    f(q, qd, theta) -> q_dd with joint friction as the generalised force."""
    sp = pytest.importorskip("sympy")
    q1, q2, w1, w2 = sp.symbols("q1 q2 w1 w2")
    m1, I1, cx1, cy1, b1, L2, m2, I2, cx2, cy2, b2 = sp.symbols("m1 I1 cx1 cy1 b1 L2 m2 I2 cx2 cy2 b2")
    g = sp.Rational(981, 100)

    def rot(a, v):
        return sp.Matrix([sp.cos(a) * v[0] - sp.sin(a) * v[1], sp.sin(a) * v[0] + sp.cos(a) * v[1]])

    q, w = sp.Matrix([q1, q2]), sp.Matrix([w1, w2])
    p1 = rot(q1, (cx1, cy1))
    p2 = rot(q1, (0, -L2)) + rot(q1 + q2, (cx2, cy2))
    v1, v2 = p1.jacobian(q) * w, p2.jacobian(q) * w
    Tk = (m1 * v1.dot(v1) + I1 * w1 ** 2 + m2 * v2.dot(v2) + I2 * (w1 + w2) ** 2) / 2
    V = g * (m1 * p1[1] + m2 * p2[1])
    Lg = Tk - V
    dL_dw = sp.Matrix([sp.diff(Lg, x) for x in (w1, w2)])
    H = dL_dw.jacobian(w)
    h = dL_dw.jacobian(q) * w - sp.Matrix([sp.diff(Lg, x) for x in (q1, q2)])
    fric = sp.Matrix([-b1 * w1, -b2 * w2])
    args = (q1, q2, w1, w2, m1, I1, cx1, cy1, b1, L2, m2, I2, cx2, cy2, b2)
    fH, fr = sp.lambdify(args, H.tolist(), "math"), sp.lambdify(args, (fric - h).tolist(), "math")

    def f(qv, qdv, th):
        a = tuple(qv) + tuple(qdv) + tuple(th)
        return np.linalg.solve(np.array(fH(*a), dtype=float), np.array(fr(*a), dtype=float).ravel())

    return f


def test_rigid_double_pendulum_lagrangian(orc):
    """Rigid-link double pendulum (11 parameters of Sec. IV-B): ABA with the
    friction torques equals the Euler-Lagrange equations derived
    symbolically from the links' energies."""
    f = _rigid_double_lagrange()
    pb = synth.make_problem("rigid2", N=4, K=1, T=10, n_s=1)
    assert pb.M == 11
    rng = np.random.default_rng(19)
    for _ in range(20):
        th = pb.lo + rng.uniform(size=11) * (pb.hi - pb.lo)
        q, qd = rng.uniform(-3, 3, 2), rng.uniform(-3, 3, 2)
        tau = orc.tau(pb, th, 0.0, q, qd)
        qdd = orc.aba(pb, th, q, qd, tau)
        ref = f(q, qd, th)
        assert np.max(np.abs(qdd - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))


def test_rigid_chain_reduces_to_point_masses(orc):
    """With zero inertia, the centre of mass at (0, -l_i) and joint 2 at
    the tip of link 1, the rigid chain is the point-mass chain."""
    rig = synth.make_problem("rigid2", N=4, K=1, T=10, n_s=1)
    pm = synth.make_problem("c2", damped=True, N=4, K=1, T=10, n_s=1)
    b = pm.damping[:2]
    rng = np.random.default_rng(23)
    for _ in range(10):
        m1, m2, l1, l2 = rng.uniform(0.5, 2.0, 4)
        th_pm = [m1, m2, l1, l2]
        th_rig = [m1, 0.0, 0.0, -l1, b[0], l1, m2, 0.0, 0.0, -l2, b[1]]
        q, qd = rng.uniform(-3, 3, 2), rng.uniform(-3, 3, 2)
        a = orc.aba(pm, th_pm, q, qd, orc.tau(pm, th_pm, 0.0, q, qd))
        r = orc.aba(rig, th_rig, q, qd, orc.tau(rig, th_rig, 0.0, q, qd))
        assert np.max(np.abs(a - r)) <= 1e-12 * max(1.0, np.max(np.abs(a)))


def _pendulum(orc, dt, l=1.0):
    pb = synth.make_problem("c1", dt=dt)
    pb.damping[:] = 0.0
    return pb, np.array([1.0, l])


def _energy(traj, w2):
    q, v = traj[:, 0], traj[:, 1]
    return 0.5 * v * v + w2 * (1 - np.cos(q))


def test_semi_implicit_euler_energy_orders(orc):
    """Semi-implicit (symplectic) Euler: energy error O(dt) without drift;
    the modified energy E - (dt/2) w^2 qd sin q has error O(dt^2)
    (modified-equation result for the symplectic Euler method)."""
    w2 = 9.81
    dev, mdev = [], []
    for dt in (0.004, 0.002):
        pb, th = _pendulum(orc, dt)
        n = int(round(20.0 / dt))
        tr = orc.rollout(pb, th, [1.0, 0.0], n)
        E = _energy(tr, w2)
        E0 = w2 * (1 - math.cos(1.0))
        dev.append(np.max(np.abs(E - E0)))
        # the state at step t: modified energy uses the same state
        Em = E - 0.5 * dt * w2 * tr[:, 1] * np.sin(tr[:, 0])
        mdev.append(np.max(np.abs(Em - Em[0])))
    assert 1.8 < dev[0] / dev[1] < 2.2
    assert 3.4 < mdev[0] / mdev[1] < 4.6
    # no secular drift over 1e5 steps
    pb, th = _pendulum(orc, 0.01)
    tr = orc.rollout(pb, th, [1.0, 0.0], 100000)
    E = _energy(tr, w2)
    first, last = E[:5000], E[-5000:]
    assert abs(first.mean() - last.mean()) < 0.05 * (first.max() - first.min())


def test_linearised_invariant_exact(orc):
    """For q_dd = -w^2 q the discrete map conserves Q = qd^2 + w^2 q^2 -
    w^2 dt q qd exactly; at small amplitude the nonlinear correction is
    O(theta0^2) relative, while plain energy varies at O(w dt)."""
    w2 = 9.81
    dt = 0.01
    pb, th = _pendulum(orc, dt)
    for a0, bound in ((1e-4, 1e-8), (1e-3, 1e-6)):
        tr = orc.rollout(pb, th, [a0, 0.0], 3000)
        q, v = tr[:, 0], tr[:, 1]
        Q = v * v + w2 * q * q - w2 * dt * q * v
        Q0 = w2 * a0 * a0
        assert np.max(np.abs(Q - Q0)) / Q0 <= bound
        E = v * v + w2 * q * q
        assert np.max(np.abs(E - Q0)) / Q0 > 1e-3


def _crossings(tr, dt):
    q = tr[:, 0]
    t = np.arange(1, len(q) + 1) * dt
    idx = np.where((q[:-1] > 0) & (q[1:] <= 0))[0]
    return t[idx] + dt * q[idx] / (q[idx] - q[idx + 1])


def test_small_angle_period(orc):
    """Discrete period 2 pi dt / arccos(1 - (w dt)^2 / 2); continuous 2 pi sqrt(l/g)."""
    dt, l, g = 0.01, 1.0, 9.81
    pb, th = _pendulum(orc, dt, l)
    tr = orc.rollout(pb, th, [1e-3, 0.0], 6000)
    z = _crossings(tr, dt)
    assert len(z) >= 21
    P = (z[-1] - z[0]) / (len(z) - 1)
    w = math.sqrt(g / l)
    P_disc = 2 * math.pi * dt / math.acos(1 - (w * dt) ** 2 / 2)
    assert abs(P - P_disc) / P_disc < 1e-6
    assert abs(P - 2 * math.pi * math.sqrt(l / g)) / P < 1e-4


def test_large_amplitude_period_second_order(orc):
    """Exact period 4 sqrt(l/g) K(sin^2(a/2)); the scheme's period error is O(dt^2)."""
    from scipy.special import ellipk

    a0, l, g = 2.0, 1.0, 9.81
    P_ex = 4 * math.sqrt(l / g) * ellipk(math.sin(a0 / 2) ** 2)
    errs = []
    for dt in (0.004, 0.002):
        pb, th = _pendulum(orc, dt, l)
        tr = orc.rollout(pb, th, [a0, 0.0], int(round(60.0 / dt)))
        z = _crossings(tr, dt)
        errs.append(abs((z[-1] - z[0]) / (len(z) - 1) - P_ex))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_hinge_inertia_parallel_axis(orc):
    """Arm + box: the joint-space inertia of the hinge (about the flange x
    axis through the hinge origin) is the box inertia plus parallel-axis
    terms of the box and the two point masses."""
    pb = synth.make_problem("c4", N=4, T=30, n_s=1)
    a = pb.arm
    rng = np.random.default_rng(2)
    for _ in range(5):
        th = rng.uniform(-0.1, 0.1, 4)
        s = synth.random_states(rng, 8, 1)[0]
        H, _ = orc.crba_rnea(pb, th, s[:8], s[8:])
        c = a["box_c"]
        Ih = a["box_I"][0] + a["box_m"] * (c[1] ** 2 + c[2] ** 2)
        Ih += a["pm_m"] * (th[1] ** 2 + a["pm_z"] ** 2) + a["pm_m"] * (th[3] ** 2 + a["pm_z"] ** 2)
        assert abs(H[7, 7] - Ih) <= 1e-13 * Ih


def _box_frame_by_homogeneous_matrices(a, q):
    """Box-frame points from 4x4 homogeneous matrices: per arm joint the
    modified-DH placement Rot_x(alpha) Trans_x(a) then Rot_z(q) Trans_z(d),
    then Trans_z(flange_d) Rot_x(q_7) Rot_y(q_8)."""
    def rx(t):
        c, s = math.cos(t), math.sin(t)
        return np.array([[1, 0, 0, 0], [0, c, -s, 0], [0, s, c, 0], [0, 0, 0, 1.0]])

    def ry(t):
        c, s = math.cos(t), math.sin(t)
        return np.array([[c, 0, s, 0], [0, 1, 0, 0], [-s, 0, c, 0], [0, 0, 0, 1.0]])

    def rz(t):
        c, s = math.cos(t), math.sin(t)
        return np.array([[c, -s, 0, 0], [s, c, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1.0]])

    def tr(x, y, z):
        T = np.eye(4)
        T[:3, 3] = (x, y, z)
        return T

    T = np.eye(4)
    for i in range(7):
        T = T @ rx(a["dh_alpha"][i]) @ tr(a["dh_a"][i], 0, 0) @ rz(q[i]) @ tr(0, 0, a["dh_d"][i])
    T = T @ tr(0, 0, a["flange_d"]) @ rx(q[7]) @ ry(q[8])
    pts = [T @ np.array(v) for v in ([0, 0, 0, 1.0], [1, 0, 0, 1.0], [0, 1, 0, 1.0], [0, 0, 1, 1.0])]
    return np.concatenate([p[:3] for p in pts])


@pytest.mark.parametrize("cfg", ["box1", "box2"])
def test_universal_joint_box_frame_points(orc, cfg):
    """The observed box frame equals forward kinematics written with
    homogeneous matrices from the DH table (an independent formulation)."""
    pb = synth.make_problem(cfg, N=4, T=24, n_s=1)
    rng = np.random.default_rng(21)
    for _ in range(10):
        th = pb.lo + rng.uniform(size=pb.M) * (pb.hi - pb.lo)
        s = rng.uniform(-1.5, 1.5, 18)
        got = orc.observe(pb, th, s[None])[0]
        ref = _box_frame_by_homogeneous_matrices(pb.arm, s[:9])
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_universal_joint_inertia_parallel_axis(orc):
    """With q_8 = 0 the joint-space inertia of the two passive axes is the
    box's inertia about the joint point (parallel axis): H_77 = I_xx +
    m (c_y^2 + c_z^2), H_88 = I_yy + m (c_x^2 + c_z^2), H_78 = I_xy -
    m c_x c_y (the ring is massless)."""
    pb = synth.make_problem("box1", N=4, T=24, n_s=1)
    m = pb.arm["box_m"]
    rng = np.random.default_rng(22)
    for _ in range(5):
        th = pb.lo + rng.uniform(size=pb.M) * (pb.hi - pb.lo)
        s = rng.uniform(-1.0, 1.0, 18)
        s[8] = 0.0
        H, _ = orc.crba_rnea(pb, th, s[:9], s[9:])
        cx, cy, cz = th[6:9]
        assert abs(H[7, 7] - (th[0] + m * (cy * cy + cz * cz))) <= 1e-14
        assert abs(H[8, 8] - (th[1] + m * (cx * cx + cz * cz))) <= 1e-14
        assert abs(H[7, 8] - (th[3] - m * cx * cy)) <= 1e-14


def test_universal_joint_weights_inertia_parallel_axis(orc):
    """Phase II: with q_8 = 0 the two passive axes see the box (parallel
    axis) plus the two point masses at (x_w, y_w, z_m): H_77 = I_xx +
    m (c_y^2 + c_z^2) + m_w sum (y_w^2 + z_m^2), H_88 = I_yy + m (c_x^2 +
    c_z^2) + m_w sum (x_w^2 + z_m^2)."""
    pb = synth.make_problem("box2", N=4, T=24, n_s=1)
    a = pb.arm
    m, c, I, mw, zm = a["box_m"], a["box_c"], a["box_I"], a["pm_m"], a["pm_z"]
    rng = np.random.default_rng(23)
    for _ in range(5):
        th = pb.lo + rng.uniform(size=4) * (pb.hi - pb.lo)
        s = rng.uniform(-1.0, 1.0, 18)
        s[8] = 0.0
        H, _ = orc.crba_rnea(pb, th, s[:9], s[9:])
        h77 = I[0] + m * (c[1] ** 2 + c[2] ** 2) + mw * (th[1] ** 2 + th[3] ** 2 + 2 * zm * zm)
        h88 = I[1] + m * (c[0] ** 2 + c[2] ** 2) + mw * (th[0] ** 2 + th[2] ** 2 + 2 * zm * zm)
        assert abs(H[7, 7] - h77) <= 1e-13 and abs(H[8, 8] - h88) <= 1e-13


# --------------------------------------------------------------------------
# Likelihood, multiple shooting, combination (Sec. III-B, III-C, App. A-B)
# --------------------------------------------------------------------------

def _setup(orc, cfg, **kw):
    pb = synth.make_problem(cfg, **kw)
    obs = orc.observations(pb)
    S = orc.shooting_init(pb, pb.particles)
    st = orc.State(pb, pb.particles, S)
    return pb, obs, st


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3", "c4", "rigid2", "box1", "box2"])
def test_multiple_shooting_on_trajectory_equals_single(orc, cfg):
    """Shooting states taken from the single-shooting rollout give zero
    defects, and the window log-likelihoods sum to the single-shooting one."""
    pb, obs, st = _setup(orc, cfg, N=5, K=2, T=120, n_s=4)
    f = orc.forward(pb, obs, st)
    assert np.all(f["gdef"] == 0.0)
    pb1 = synth.make_problem(cfg, N=5, K=2, T=120, n_s=1)
    st1 = orc.State(pb1, pb1.particles, np.zeros((5, 2, 0, pb1.d_s)))
    f1 = orc.forward(pb1, obs, st1)
    l_ms = f["ll_win"].sum(axis=2)
    l_ss = f1["ll_win"][:, :, 0]
    assert np.max(np.abs(l_ms - l_ss) / np.abs(l_ss)) < 1e-12


def test_gaussian_constant_and_single_step(orc):
    """Window log-likelihood = sum of log N(x_real | x_sim, sigma^2) with the
    normalising constant, checked against scipy.stats.norm on the oracle's
    own simulated states."""
    from scipy.stats import norm

    pb, obs, st = _setup(orc, "c2", N=3, K=2, T=40, n_s=2)
    f = orc.forward(pb, obs, st, traj=True)
    for i in range(3):
        for k in range(2):
            for j in range(2):
                xs = f["traj"][i, k, j * pb.h:(j + 1) * pb.h][:, pb.obs_index]
                xr = obs[k, j * pb.h:(j + 1) * pb.h]
                ref = norm.logpdf(xr, loc=xs, scale=pb.sigma_obs).sum()
                assert abs(f["ll_win"][i, k, j] - ref) <= 1e-9 * abs(ref)


def test_mixture_special_cases(orc):
    """K = 1 gives log p = l; K identical trajectories give log p = l under
    the equally weighted mixture and K l under the product."""
    pb, obs, st = _setup(orc, "c2", N=4, K=1, T=80, n_s=4)
    f = orc.forward(pb, obs, st)
    l = f["ll_win"].sum(axis=2)[:, 0]
    assert np.max(np.abs(f["logp"] - l) / np.abs(l)) < 1e-15
    K = 3
    for comb, factor in ((synth.COMBINE_SUM, 1.0), (synth.COMBINE_PROD, float(K))):
        pbK = synth.make_problem("c2", N=4, K=K, T=80, n_s=4, combine=comb)
        pbK.s0[:] = pb.s0[0]
        obsK = np.repeat(obs, K, axis=0)
        stK = orc.State(pbK, pb.particles, np.repeat(st.S, K, axis=1))
        fK = orc.forward(pbK, obsK, stK)
        assert np.max(np.abs(fK["logp"] - factor * l) / np.abs(l)) < 1e-14
        np.testing.assert_allclose(fK["wk"], 1.0 / K if comb == synth.COMBINE_SUM else 1.0, rtol=1e-14)


def test_mixture_weights_are_softmax(orc):
    """SUM combination: weights are exp(l_k - log p - log K) (they sum to one)."""
    pb, obs, st = _setup(orc, "c2", N=4, K=3, T=80, n_s=4)
    f = orc.forward(pb, obs, st)
    lk = f["ll_win"].sum(axis=2)
    w = np.exp(lk - f["logp"][:, None] - math.log(3))
    np.testing.assert_allclose(f["wk"], w, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(f["wk"].sum(axis=1), 1.0, rtol=1e-14)


# --------------------------------------------------------------------------
# Gradients (forward-mode duals) against central finite differences
# --------------------------------------------------------------------------

def _total_phi(pb, f, lam_def):
    g = f["gdef"]
    return np.sum(lam_def * g + 0.5 * pb.c * g * g, axis=(1, 2))


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3", "c4", "rigid2", "box1", "box2"])
def test_dual_gradients_match_finite_differences(orc, cfg):
    """g_obs = d log p / d theta, g_con = d Phi / d theta and S_dot =
    d (log p - Phi) / d S, with Phi = sum (lam g + c/2 g^2), by central
    differences through the whole forward pipeline."""
    rng = np.random.default_rng(17)
    pb, obs, st = _setup(orc, cfg, N=2, K=2, T=30, n_s=3)
    st.S = synth.perturb(rng, st.S, 0.02)
    st.lam_def = rng.uniform(0.0, 2.0, st.lam_def.shape)
    st.theta = pb.lo + rng.uniform(0.2, 0.8, st.theta.shape) * (pb.hi - pb.lo)
    g = orc.gradient(pb, obs, st)

    def F(theta=None, S=None):
        s2 = orc.State(pb, st.theta if theta is None else theta, st.S if S is None else S,
                       lam_def=st.lam_def)
        f = orc.forward(pb, obs, s2)
        return f["logp"], _total_phi(pb, f, st.lam_def)

    for i in range(2):
        go, gc = np.zeros(pb.M), np.zeros(pb.M)
        for m in range(pb.M):
            e = 1e-6 * max(1.0, abs(st.theta[i, m]))
            tp, tm = st.theta.copy(), st.theta.copy()
            tp[i, m] += e
            tm[i, m] -= e
            (lp, pp), (lm, pm) = F(theta=tp), F(theta=tm)
            go[m] = (lp[i] - lm[i]) / (2 * e)
            gc[m] = (pp[i] - pm[i]) / (2 * e)
        assert np.linalg.norm(g["g_obs"][i] - go) <= 1e-6 * np.linalg.norm(go)
        assert np.linalg.norm(g["g_con"][i] - gc) <= 1e-6 * max(np.linalg.norm(gc), 1e-3)
        sd = np.zeros_like(st.S[i])
        for idx in np.ndindex(*st.S[i].shape):
            e = 1e-6 * max(1.0, abs(st.S[i][idx]))
            Sp, Sm = st.S.copy(), st.S.copy()
            Sp[(i,) + idx] += e
            Sm[(i,) + idx] -= e
            (lp, pp), (lm, pm) = F(S=Sp), F(S=Sm)
            sd[idx] = ((lp[i] - pp[i]) - (lm[i] - pm[i])) / (2 * e)
        assert np.linalg.norm(g["S_dot"][i] - sd) <= 1e-6 * np.linalg.norm(sd)


@pytest.mark.parametrize("cfg", ["c2", "c4", "rigid2"])
def test_defect_density_in_likelihood_gradients_match_finite_differences(orc, cfg):
    """Defects inside p_ms (eq. ms_likelihood): g_obs = d log p_ms / d theta
    and S_dot = d log p_ms / d S by central differences through the whole
    forward pipeline, with no constraint part (g_con = 0)."""
    rng = np.random.default_rng(23)
    pb, obs, st = _setup(orc, cfg, N=2, K=2, T=30, n_s=3, lik=synth.LIK_DEFECT)
    st.S = synth.perturb(rng, st.S, 0.02)
    st.lam_def = rng.uniform(0.0, 2.0, st.lam_def.shape)  # must not matter
    st.theta = pb.lo + rng.uniform(0.2, 0.8, st.theta.shape) * (pb.hi - pb.lo)
    g = orc.gradient(pb, obs, st)
    assert np.all(g["g_con"] == 0.0)

    def F(theta=None, S=None):
        s2 = orc.State(pb, st.theta if theta is None else theta, st.S if S is None else S, lam_def=st.lam_def)
        return orc.forward(pb, obs, s2)["logp"]

    for i in range(2):
        go = np.zeros(pb.M)
        for m in range(pb.M):
            e = 1e-6 * max(1.0, abs(st.theta[i, m]))
            tp, tm = st.theta.copy(), st.theta.copy()
            tp[i, m] += e
            tm[i, m] -= e
            go[m] = (F(theta=tp)[i] - F(theta=tm)[i]) / (2 * e)
        assert np.linalg.norm(g["g_obs"][i] - go) <= 1e-6 * np.linalg.norm(go)
        sd = np.zeros_like(st.S[i])
        for idx in np.ndindex(*st.S[i].shape):
            e = 1e-6 * max(1.0, abs(st.S[i][idx]))
            Sp, Sm = st.S.copy(), st.S.copy()
            Sp[(i,) + idx] += e
            Sm[(i,) + idx] -= e
            sd[idx] = (F(S=Sp)[i] - F(S=Sm)[i]) / (2 * e)
        assert np.linalg.norm(g["S_dot"][i] - sd) <= 1e-6 * np.linalg.norm(sd)


@pytest.mark.parametrize("combine", [synth.COMBINE_SUM, synth.COMBINE_PROD])
def test_defect_density_constant_on_continuous_trajectories(orc, combine):
    """Shooting states taken from each particle's own rollout close every
    defect exactly (g_def = 0), so each density factor is its Gaussian
    normalising constant: log p_ms exceeds the observation-only log p by
    (n_s - 1) sum_d log(u_d / (sigma_def sqrt(2 pi))) per trajectory (times K
    for the product over trajectories)."""
    K, ns = 3, 4
    pb0, obs, st0 = _setup(orc, "c2", N=3, K=K, T=40, n_s=ns, combine=combine)
    pb1 = synth.make_problem("c2", N=3, K=K, T=40, n_s=ns, combine=combine, lik=synth.LIK_DEFECT)
    pb1.u = np.array([1.0, 2.0, 0.5, 0.25])
    pb0.u = pb1.u.copy()
    st0.S = orc.shooting_init(pb0, st0.theta)
    f0 = orc.forward(pb0, obs, st0)
    f1 = orc.forward(pb1, obs, orc.State(pb1, st0.theta, st0.S))
    assert np.all(f1["gdef"] == 0.0)
    per_traj = (ns - 1) * np.sum(np.log(pb1.u / (pb1.sigma_def * np.sqrt(2.0 * np.pi))))
    expect = per_traj * (K if combine == synth.COMBINE_PROD else 1)
    np.testing.assert_allclose(f1["logp"] - f0["logp"], expect, rtol=0, atol=1e-9 * np.abs(f0["logp"]).max())
    np.testing.assert_allclose(f1["wk"], f0["wk"], rtol=1e-12, atol=1e-15)


def test_mass_scale_invariance(orc):
    """Without damping the planar dynamics are degree-0 homogeneous in the
    masses: single pendulum d l / d m = 0, double pendulum sum m_i d l/d m_i
    = 0.  Joint damping breaks it (the 5-link chain must not satisfy it)."""
    for cfg, n in (("c1", 1), ("c2", 2)):
        pb, obs, st = _setup(orc, cfg, N=3, K=1, T=100, n_s=2)
        g = orc.gradient(pb, obs, st)["g_obs"]
        lhs = np.sum(st.theta[:, :n] * g[:, :n], axis=1)
        assert np.all(np.abs(lhs) <= 1e-10 * np.linalg.norm(g, axis=1))
    pb, obs, st = _setup(orc, "c3", N=3, K=1, T=100, n_s=2)
    g = orc.gradient(pb, obs, st)["g_obs"]
    lhs = np.sum(st.theta[:, :5] * g[:, :5], axis=1)
    assert np.all(np.abs(lhs) > 1e-6 * np.linalg.norm(g, axis=1))


@pytest.mark.parametrize("cfg", ["c4", "box2"])
def test_arm_weight_swap_symmetry(orc, cfg):
    """Equal point masses: swapping their positions leaves log p unchanged
    and permutes the gradient (the symmetry reported in Sec. IV-C)."""
    pb, obs, st = _setup(orc, cfg, N=3, K=1, T=100, n_s=2)
    sw = st.theta[:, [2, 3, 0, 1]]
    st2 = orc.State(pb, sw, st.S)
    g1 = orc.gradient(pb, obs, st)
    g2 = orc.gradient(pb, obs, st2)
    assert np.max(np.abs(g1["logp"] - g2["logp"]) / np.abs(g1["logp"])) < 1e-10
    np.testing.assert_allclose(g2["g_obs"], g1["g_obs"][:, [2, 3, 0, 1]], rtol=1e-7, atol=1e-9 * np.abs(g1["g_obs"]).max())


# --------------------------------------------------------------------------
# Kernel bandwidth, phi, MDMM step (Sec. III-A, III-E, Algorithm 1)
# --------------------------------------------------------------------------

def test_median_brute_force(orc):
    rng = np.random.default_rng(9)
    for N in (1, 2, 3, 4, 17, 64):
        th = rng.normal(size=(N, 3))
        rho = np.array([0.5, 2.0, 1.0])
        h, med = orc.bandwidth(th, rho)
        if N == 1:
            assert h == 1.0
            continue
        d = [math.sqrt(sum(((th[i, m] - th[j, m]) / rho[m]) ** 2 for m in range(3)))
             for i, j in itertools.combinations(range(N), 2)]
        ref = statistics.median(d)
        assert abs(med - ref) <= 1e-14 * ref
        assert abs(h - ref * ref / math.log(N)) <= 1e-14 * h


def test_phi_two_particles_hand_worked(orc):
    gd = json.load(open(os.path.join(GOLDEN, "phi_two_particles.json")))
    th = np.array(gd["theta"])
    h, med = orc.bandwidth(th, gd["rho"])
    assert abs(med - gd["median"]) < 1e-15 and abs(h - gd["h"]) < 1e-14
    np.testing.assert_allclose(orc.phi(th, np.zeros_like(th), gd["rho"], h), gd["phi_zero_grad"], rtol=1e-14)
    np.testing.assert_allclose(orc.phi(th, np.array(gd["grad"]), gd["rho"], h), gd["phi_with_grad"], rtol=1e-14)


def test_phi_invariances(orc):
    """phi is unchanged by a common translation, equivariant under particle
    permutation, equals the gradient for N = 1 and tends to the mean
    gradient as h grows (k -> 1, grad k -> 0)."""
    rng = np.random.default_rng(4)
    N, M = 12, 3
    th = rng.normal(size=(N, M))
    G = rng.normal(size=(N, M))
    rho = np.array([1.0, 0.3, 2.0])
    h, _ = orc.bandwidth(th, rho)
    p = orc.phi(th, G, rho, h)
    np.testing.assert_allclose(orc.phi(th + np.array([0.7, -1.1, 3.0]), G, rho, h), p, rtol=1e-12, atol=1e-14)
    perm = rng.permutation(N)
    np.testing.assert_allclose(orc.phi(th[perm], G[perm], rho, h), p[perm], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(orc.phi(th[:1], G[:1], rho, 1.0), G[:1], rtol=1e-15)
    np.testing.assert_allclose(orc.phi(th, G, rho, 1e12), np.tile(G.mean(axis=0), (N, 1)), rtol=1e-9, atol=1e-10)



# --------------------------------------------------------------------------
# Particles that leave the ensemble (failed simulations, Sec. III-D)
# --------------------------------------------------------------------------

def test_masked_median_brute_force(orc):
    """The median over the live particles is the brute-force median of the
    pairs among them, h uses the log of their number, and a non-finite
    row of a masked particle does not reach it."""
    rng = np.random.default_rng(21)
    rho = np.array([0.5, 2.0, 1.0])
    for N, dead in ((9, [0, 4]), (17, [16]), (6, [1, 2, 3, 4]), (5, [0, 1, 2, 3]), (4, [0, 1, 2, 3])):
        th = rng.normal(size=(N, 3))
        th[dead] = np.nan
        live = np.ones(N, dtype=bool)
        live[dead] = False
        h, med = orc.bandwidth(th, rho, live=live)
        idx = np.flatnonzero(live)
        if len(idx) <= 1:
            assert h == 1.0
            continue
        d = [math.sqrt(sum(((th[i, m] - th[j, m]) / rho[m]) ** 2 for m in range(3)))
             for i, j in itertools.combinations(idx, 2)]
        ref = statistics.median(d)
        assert abs(med - ref) <= 1e-14 * ref
        assert abs(h - ref * ref / math.log(len(idx))) <= 1e-14 * h


def test_masked_phi_is_the_live_ensembles(orc):
    """phi over the live particles equals phi of the ensemble made of them
    alone (pinned above by hand-worked values and invariances), rows of
    masked particles are zero, and NaN or infinite rows of masked
    particles do not leak into the others."""
    rng = np.random.default_rng(22)
    N, M = 15, 3
    th = rng.normal(size=(N, M))
    G = rng.normal(size=(N, M))
    rho = np.array([1.0, 0.3, 2.0])
    live = np.ones(N, dtype=bool)
    live[[0, 7, 14]] = False
    th[7] = np.nan
    G[0] = np.inf
    G[14] = np.nan
    h, _ = orc.bandwidth(th[live], rho)
    p = orc.phi(th, G, rho, h, live=live)
    np.testing.assert_allclose(p[live], orc.phi(th[live], G[live], rho, h), rtol=1e-15, atol=0)
    assert np.all(p[~live] == 0.0)
    sel = np.array([14, 3, 0], dtype=np.int32)
    np.testing.assert_array_equal(orc.phi(th, G, rho, h, sel=sel, live=live), p[sel])
    assert np.all(orc.phi(th, G, rho, h, live=np.zeros(N, dtype=bool)) == 0.0)


def test_frozen_particles_keep_their_state(orc):
    """An MDMM/Adam update with some particles frozen leaves every variable
    of those particles bitwise as it was and moves the others exactly as
    an update of the ensemble without them does."""
    pb = synth.make_problem("c2", N=6, K=2, T=40, n_s=4)
    rng = np.random.default_rng(23)
    N, M, K, ns, ds = 6, pb.M, pb.K, pb.n_s, pb.d_s
    th = pb.lo + rng.uniform(-0.1, 1.1, size=(N, M)) * (pb.hi - pb.lo)  # some outside the limits
    S = rng.normal(size=(N, K, ns - 1, ds))
    frozen = np.array([False, True, False, False, True, False])
    args = (rng.normal(size=(N, M)), rng.normal(size=(N, M)), rng.normal(size=(N, K, ns - 1, ds)),
            rng.uniform(size=(N, K, ns - 1)))
    lam = rng.normal(size=(N, M))
    for optimizer in (0, 1):
        a = orc.State(pb, th, S, lam_lim=lam, lam_def=rng.normal(size=(N, K, ns - 1)),
                      adam_m=rng.normal(size=(N, M + K * (ns - 1) * ds)),
                      adam_v=rng.uniform(size=(N, M + K * (ns - 1) * ds)))
        before = [x.copy() for x in (a.theta, a.S, a.lam_lim, a.lam_def, a.adam_m, a.adam_v)]
        keep = ~frozen
        b = orc.State(pb, th[keep], S[keep], lam_lim=lam[keep], lam_def=a.lam_def[keep], adam_m=a.adam_m[keep],
                      adam_v=a.adam_v[keep])
        orc.mdmm_step(pb, a, *args, optimizer, 2, frozen=frozen)
        orc.mdmm_step(pb, b, *(x[keep] for x in args), optimizer, 2)
        after = (a.theta, a.S, a.lam_lim, a.lam_def, a.adam_m, a.adam_v)
        for x0, x1, y in zip(before, after, (b.theta, b.S, b.lam_lim, b.lam_def, b.adam_m, b.adam_v)):
            np.testing.assert_array_equal(x1[frozen], x0[frozen])
            np.testing.assert_array_equal(x1[keep], y)


def test_failed_particle_leaves_the_ensemble(orc):
    """A particle whose shooting state is NaN is flagged (state and
    gradient), left out of phi at once and frozen; the median leaves it out
    from the next iteration on.  The other particles' phi equals phi of the
    ensemble without it, at the bandwidth of the ensemble with it."""
    pb = synth.make_problem("c2", N=12, K=1, T=40, n_s=4)
    obs = orc.observations(pb)
    S = orc.shooting_init(pb, pb.particles)
    S[5, 0, 1, 2] = np.nan
    st = orc.State(pb, pb.particles, S)
    th0 = st.theta.copy()
    live = np.arange(12) != 5
    g = orc.csvgd_iteration(pb, obs, st, 1)
    assert g["flags"][5] == orc.FLAG_STATE | orc.FLAG_GRAD | orc.FLAG_FROZEN
    assert np.all(g["flags"][live] == 0) and g["n_masked"] == 1
    assert g["bandwidth"] == orc.bandwidth(th0, pb.rho)[0]
    np.testing.assert_array_equal(g["phi"][live], orc.phi(th0[live], g["g_obs"][live], pb.rho, g["bandwidth"]))
    assert np.all(g["phi"][5] == 0.0) and np.all(np.isfinite(st.theta))
    np.testing.assert_array_equal(st.theta[5], th0[5])
    th1 = st.theta.copy()
    g2 = orc.csvgd_iteration(pb, obs, st, 2)
    assert g2["bandwidth"] == orc.bandwidth(th1[live], pb.rho)[0]
    np.testing.assert_array_equal(st.theta[5], th0[5])
    assert np.all(np.isfinite(st.theta)) and g2["n_masked"] == 1

def test_mdmm_limits_hand_worked(orc):
    gd = json.load(open(os.path.join(GOLDEN, "mdmm_limits.json")))
    pb = synth.make_problem("toy", N=1, M=1)
    pb.lo[:] = gd["lo"]
    pb.hi[:] = gd["hi"]
    pb.c = gd["c"]
    for th0, want_th, want_lam in ((gd["theta0"], gd["theta"], gd["lambda"]),
                                   (gd["inside_theta0"], [gd["inside_theta0"]] * 3, [0.0] * 3)):
        st = orc.State(pb, np.array([[th0]]), np.zeros((1, 1, 0, 2)))
        for it in range(3):
            orc.mdmm_step(pb, st, np.zeros((1, 1)), np.zeros((1, 1)), np.zeros((1, 1, 0, 2)), np.zeros((1, 1, 0)),
                          0, it + 1, lr_theta=np.array([gd["lr"]]), eps_lam=gd["eps_lambda"])
            assert abs(st.theta[0, 0] - want_th[it]) < 1e-12
            assert abs(st.lam_lim[0, 0] - want_lam[it]) < 1e-12


def test_single_particle_is_gradient_ascent(orc):
    """With N = 1 the kernel is 1 and its gradient 0, so a plain-SGD CSVGD
    step moves theta by lr * d (log p - Phi) / d theta and S by
    lr_S * d (log p - Phi) / d S; both checked against finite differences of
    the forward pipeline."""
    rng = np.random.default_rng(23)
    pb, obs, st = _setup(orc, "c2", N=1, K=2, T=40, n_s=2)
    st.S = synth.perturb(rng, st.S, 0.05)
    st.lam_def = rng.uniform(0, 1, st.lam_def.shape)
    th0, S0, lam0 = st.theta.copy(), st.S.copy(), st.lam_def.copy()
    g = orc.csvgd_iteration(pb, obs, st, it=1, optimizer=0)
    assert g["bandwidth"] == 1.0
    np.testing.assert_allclose(st.lam_def, lam0 + pb.eps_lam * g["gdef"], rtol=1e-15)

    def L(theta, S):
        s2 = orc.State(pb, theta, S, lam_def=lam0)
        f = orc.forward(pb, obs, s2)
        return f["logp"][0] - _total_phi(pb, f, lam0)[0]

    for m in range(pb.M):
        e = 1e-6
        tp, tm = th0.copy(), th0.copy()
        tp[0, m] += e
        tm[0, m] -= e
        fd = (L(tp, S0) - L(tm, S0)) / (2 * e)
        assert abs((st.theta[0, m] - th0[0, m]) - pb.lr_theta[m] * fd) <= 1e-6 * abs(pb.lr_theta[m] * fd) + 1e-12
    for idx in np.ndindex(*S0.shape):
        e = 1e-6
        Sp, Sm = S0.copy(), S0.copy()
        Sp[idx] += e
        Sm[idx] -= e
        fd = (L(th0, Sp) - L(th0, Sm)) / (2 * e)
        want = pb.lr_S[idx[-1]] * fd
        assert abs((st.S[idx] - S0[idx]) - want) <= 1e-6 * abs(want) + 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("M", [1])
def test_linear_gaussian_posterior(orc, M):
    """Linear toy (unit mass, force a0 + a1 t, semi-implicit Euler): the
    positions are linear in theta, q_t = c0_t a0 + c1_t a1 with c0_t =
    dt^2 t(t+1)/2 and c1_t = dt^3 (t+1) t (t-1) / 6, so under a flat prior the
    posterior is Gaussian with covariance sigma^2 (C^T C)^{-1}.  CSVGD with
    N particles must reproduce its mean and spread.  (The two-parameter
    variant is 98.5% correlated; plain SGD does not converge on it in a
    test-sized budget, so only the force-only case is pinned.)"""
    N = 128
    pb = synth.make_problem("toy", N=N, M=M)
    obs = orc.observations(pb)
    T, dt, sig = pb.T, pb.dt, pb.sigma_obs
    t = np.arange(1, T + 1, dtype=float)
    Cm = np.stack([dt * dt * t * (t + 1) / 2, dt ** 3 * (t + 1) * t * (t - 1) / 6], axis=1)[:, :M]
    cov = sig * sig * np.linalg.inv(Cm.T @ Cm)
    mu = np.linalg.solve(Cm.T @ Cm, Cm.T @ obs[0, :, 0])
    sd = np.sqrt(np.diag(cov))
    # start the particles near the posterior so plain SGD converges quickly
    rng = np.random.default_rng(1)
    th = mu + rng.normal(size=(N, M)) * sd * 3
    st = orc.State(pb, th, np.zeros((N, 1, 0, 2)))
    lr = 0.2 / np.max(np.linalg.eigvalsh(np.linalg.inv(cov)))
    for it in range(1, 1501):
        g = orc.gradient(pb, obs, st)
        h, _ = orc.bandwidth(st.theta, pb.rho)
        ph = orc.phi(st.theta, g["g_obs"], pb.rho, h)
        orc.mdmm_step(pb, st, ph, g["g_con"], g["S_dot"], g["gdef"], 0, it, lr_theta=np.full(M, lr))
    mean = st.theta.mean(axis=0)
    std = st.theta.std(axis=0)
    assert np.all(np.abs(mean - mu) <= 0.05 * sd)
    assert np.all(np.abs(std / sd - 1) <= 0.1)


def test_adam_hand_worked(orc):
    """Three Adam steps of theta, the shooting states and the defect
    multiplier against tests/golden/adam_three_steps.json (Kingma and Ba's
    rule with -x_dot as the gradient, bias corrections at t = 1, 2, 3)."""
    gd = json.load(open(os.path.join(GOLDEN, "adam_three_steps.json")))
    pb = synth.make_problem("toy", N=1, M=1, T=50, n_s=2)
    pb.lo[:] = gd["lo"]
    pb.hi[:] = gd["hi"]
    st = orc.State(pb, np.array([[gd["theta0"]]]), np.full((1, 1, 1, pb.d_s), gd["S0"]))
    nA = pb.M + pb.d_s
    for it in range(3):
        orc.mdmm_step(pb, st, np.array([[gd["phi"][it]]]), np.array([[gd["g_con"][it]]]),
                      np.full((1, 1, 1, pb.d_s), gd["S_dot"][it]), np.array([[[gd["g_def"][it]]]]), 1, it + 1,
                      lr_theta=np.array([gd["lr_theta"]]), lr_S=np.full(pb.d_s, gd["lr_S"]),
                      eps_lam=gd["eps_lambda"])
        assert abs(st.theta[0, 0] - float(gd["theta"][it])) <= 1e-15
        assert abs(st.adam_m[0, 0] - gd["adam_m_theta"][it]) <= 1e-16
        assert abs(st.adam_v[0, 0] - gd["adam_v_theta"][it]) <= 1e-17
        np.testing.assert_allclose(st.S.reshape(-1), float(gd["S"][it]), rtol=0, atol=1e-15)
        np.testing.assert_allclose(st.adam_m[0, 1:nA], gd["adam_m_S"][it], rtol=0, atol=1e-15)
        np.testing.assert_allclose(st.adam_v[0, 1:nA], gd["adam_v_S"][it], rtol=0, atol=1e-16)
        assert abs(st.lam_def[0, 0, 0] - gd["lam_def"][it]) <= 1e-15
        assert st.lam_lim[0, 0] == 0.0


def test_adam_matches_torch_adam(orc):
    """The oracle's Adam branch (theta and shooting states, per-coordinate
    step sizes, iterations 1..5) against torch.optim.Adam in float64 fed
    -x_dot as the gradient, every parameter inside its limits so that
    x_dot = phi - g_con for theta and S_dot for S."""
    import torch

    rng = np.random.default_rng(31)
    pb = synth.make_problem("c2", N=3, K=2, T=40, n_s=4)
    N, M, K, ns, ds = 3, pb.M, pb.K, pb.n_s, pb.d_s
    th0 = pb.lo + rng.uniform(0.3, 0.7, (N, M)) * (pb.hi - pb.lo)
    S0 = rng.normal(size=(N, K, ns - 1, ds))
    st = orc.State(pb, th0, S0)
    # one torch tensor per step-size group: theta column m, S component d
    tcols = [torch.tensor(th0[:, m].copy(), dtype=torch.float64, requires_grad=True) for m in range(M)]
    scols = [torch.tensor(S0[..., d].copy(), dtype=torch.float64, requires_grad=True) for d in range(ds)]
    groups = [{"params": [t], "lr": float(pb.lr_theta[m])} for m, t in enumerate(tcols)]
    groups += [{"params": [s], "lr": float(pb.lr_S[d])} for d, s in enumerate(scols)]
    opt = torch.optim.Adam(groups, betas=(0.9, 0.999), eps=1e-8, foreach=False)
    for it in range(1, 6):
        ph = rng.normal(size=(N, M)) * 1e3
        gc = rng.normal(size=(N, M)) * 1e3
        sd = rng.normal(size=(N, K, ns - 1, ds)) * 10.0
        gdef = rng.uniform(0, 1, (N, K, ns - 1))
        orc.mdmm_step(pb, st, ph, gc, sd, gdef, 1, it)
        for m, t in enumerate(tcols):
            t.grad = torch.tensor(-(ph[:, m] - gc[:, m]), dtype=torch.float64)
        for d, s in enumerate(scols):
            s.grad = torch.tensor(-sd[..., d], dtype=torch.float64)
        opt.step()
        for m, t in enumerate(tcols):
            np.testing.assert_allclose(st.theta[:, m], t.detach().numpy(), rtol=1e-14, atol=1e-15)
            np.testing.assert_allclose(st.adam_m[:, m], opt.state[t]["exp_avg"].numpy(), rtol=1e-13)
            np.testing.assert_allclose(st.adam_v[:, m], opt.state[t]["exp_avg_sq"].numpy(), rtol=1e-13)
        for d, s in enumerate(scols):
            np.testing.assert_allclose(st.S[..., d], s.detach().numpy(), rtol=1e-14, atol=1e-15)
        assert np.all(st.lam_lim == 0.0)


@pytest.mark.parametrize("cfg", ["c4", "box1", "box2"])
def test_arm_pd_torque(orc, cfg):
    """The arm's joint torques (the controls of App. B-A's f_step): PD
    tracking of the prescribed sinusoid q_d(t) = qc + A sin(omega t + phase)
    on the seven arm joints, viscous damping on the passive axes.  Pinned as
    an affine map of (q, qd): it vanishes at (q_d(t), dq_d/dt) -- the
    target's time derivative taken here by central differences of the
    sinusoid, not from any closed form -- and its Jacobian is -diag(kp) in
    q and -diag(kd) in qd (finite differences), -b on the passive axes."""
    pb = synth.make_problem(cfg, N=2, K=1, T=30, n_s=1)
    a = pb.arm
    th = pb.theta_true[0]
    n = pb.n_dof

    def qdes(t):
        return np.asarray(a["qc"]) + np.asarray(a["amp"]) * np.sin(np.asarray(a["omega"]) * t + np.asarray(a["phase"]))

    rng = np.random.default_rng(3)
    if cfg == "c4":
        b_passive = [pb.damping[7]]
    elif cfg == "box1":
        b_passive = [th[9], th[10]]
    else:
        b_passive = list(a["ujoint_b"])
    for t in (0.0, 1.37, 4.9):
        e = 1e-4
        qdot_des = (-qdes(t + 2 * e) + 8 * qdes(t + e) - 8 * qdes(t - e) + qdes(t - 2 * e)) / (12 * e)
        q = rng.normal(size=n)
        qd = rng.normal(size=n)
        q[:7], qd[:7] = qdes(t), qdot_des
        tau = orc.tau(pb, th, t, q, qd)
        np.testing.assert_allclose(tau[:7], 0.0, atol=1e-8 * max(np.max(a["kd"]), 1.0))
        # passive axes: -b qd whatever q is
        np.testing.assert_allclose(tau[7:], -np.asarray(b_passive) * qd[7:], rtol=1e-14)
        J_q = np.zeros((n, n))
        J_qd = np.zeros((n, n))
        for j in range(n):
            h = 1e-3
            qp, qm = q.copy(), q.copy()
            qp[j] += h
            qm[j] -= h
            J_q[:, j] = (orc.tau(pb, th, t, qp, qd) - orc.tau(pb, th, t, qm, qd)) / (2 * h)
            qp, qm = qd.copy(), qd.copy()
            qp[j] += h
            qm[j] -= h
            J_qd[:, j] = (orc.tau(pb, th, t, q, qp) - orc.tau(pb, th, t, q, qm)) / (2 * h)
        want_q = np.zeros((n, n))
        want_q[:7, :7] = -np.diag(a["kp"])
        want_qd = np.zeros((n, n))
        want_qd[:7, :7] = -np.diag(a["kd"])
        for p, b in enumerate(b_passive):
            want_qd[7 + p, 7 + p] = -b
        np.testing.assert_allclose(J_q, want_q, atol=1e-9 * np.max(a["kp"]))
        np.testing.assert_allclose(J_qd, want_qd, atol=1e-9 * max(np.max(a["kd"]), 1.0))
