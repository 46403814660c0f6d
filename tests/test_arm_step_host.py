"""The arm's step functions in FP64 on the host (the library's own spatial
algebra, compiled with g++): joint accelerations of its Articulated Body
Algorithm against the oracle's (an independent 6x6 implementation), the
box-frame observation against the oracle's kinematics, and the reverse
step of both adjoint channels and of the observation against central
differences of the same functions."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2109_08815_amd import lib as L
from paper_2109_08815_amd import synth
from tests.helpers import f32_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = tmp_path_factory.mktemp("armcheck") / "arm_step_check"
    subprocess.run([gxx, "-O2", "-std=c++17", "-Wno-unknown-pragmas", "-I", os.path.join(ROOT, "include"), "-I",
                    os.path.join(ROOT, "paper_2109_08815_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "arm_step_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True, timeout=600)
    return str(exe)


MOUNTS = {"c4": 0, "box1": 1, "box2": 2}


@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("cfg", ["c4", "box1", "box2"])
def test_arm_step_against_oracle(orc, checker, cfg, generic):
    """Both kinematic structures: the synthetic tables have the Panda arm's
    (its step functions take the twists as exact right angles, so the
    oracle gets exact multiples of pi/2 where the float table holds their
    rounding), and a table off that structure runs the generic ones."""
    pb = f32_problem(synth.make_problem(cfg, N=16, K=1, T=30, n_s=1, generic_dh=generic))
    _, raw = L.model_consts(pb)
    raw = np.asarray(raw, np.float32).astype(np.float64)
    if not generic:
        pb.arm["dh_alpha"] = np.round(pb.arm["dh_alpha"] / (np.pi / 2)) * (np.pi / 2)
    rng = np.random.default_rng(21)
    n = pb.n_dof
    cases = []
    for c in range(12):
        th = pb.particles[c]
        q = rng.uniform(-1.5, 1.5, n)
        qd = rng.uniform(-2.0, 2.0, n)
        t = float(rng.uniform(0, 6))
        cases.append((th, q, qd, t))
    lines = ["%d %d" % (MOUNTS[cfg], raw.size), " ".join("%.17g" % v for v in raw), str(len(cases))]
    for th, q, qd, t in cases:
        lines.append(" ".join("%.17g" % v for v in list(th) + list(q) + list(qd) + [t]))
    r = subprocess.run([checker], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = r.stdout.splitlines()
    assert out[0] == "structure %d" % (0 if generic else 1)
    qdd = [np.array(l.split()[1:], float) for l in out if l.startswith("qdd")]
    obs = [np.array(l.split()[1:], float) for l in out if l.startswith("frame ")]
    worst = 0.0
    for (th, q, qd, t), a in zip(cases, qdd):
        tau = orc.tau(pb, th, t, q, qd)
        ref = orc.aba(pb, th, q, qd, tau)
        worst = max(worst, np.abs(a - ref).max() / (1 + np.abs(ref).max()))
    print("ABA vs oracle: worst %.3e" % worst)
    # A general twist enters through its float cosine and sine (within 6e-8
    # of the oracle's FP64 ones); a right angle or a twist within float
    # rounding of one enters exactly.  A mistake in the algebra is O(1).
    assert worst < (1e-6 if generic else 1e-10)
    if obs:
        wo = 0.0
        for (th, q, qd, t), x in zip(cases, obs):
            ref = orc.observe(pb, th, np.concatenate([q, qd])[None])[0]
            wo = max(wo, np.abs(x - ref).max())
        print("box frame vs oracle: worst %.3e" % wo)
        assert wo < (1e-6 if generic else 1e-12)
    rev = float([l for l in out if l.startswith("reverse")][0].split()[1])
    ob = float([l for l in out if l.startswith("obs_adjoint")][0].split()[1])
    print("reverse vs central differences %.3e, observation adjoint %.3e" % (rev, ob))
    assert rev < 1e-8
    # the observation adjoint is the geometric Jacobian of a rigid chain; a
    # general twist's float cosine and sine are a rotation to within 6e-8
    assert ob < (1e-6 if generic else 1e-7)
