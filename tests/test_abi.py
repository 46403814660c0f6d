"""CPU-side checks of the C ABI: the library loads, exports every function
include/pds.h declares, the Python struct mirrors the C layout, and invalid
arguments are rejected on the host before anything is queued."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2109_08815_amd import lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions(headers=None):
    names = []
    for h in headers or HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**([a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_five_calls():
    names = declared_functions([os.path.join(ROOT, "include", "pds.h")])
    for n in ("sim_batch_forward", "loglik_multishoot", "sim_batch_adjoint", "svgd_phi", "svgd_step",
              "pds_workspace_size", "pds_last_error", "pds_version"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
    out = subprocess.check_output(["nm", "-D", "--defined-only", L.LIB_PATH]).decode()
    for n in declared_functions():
        assert re.search(r" T %s$" % n, out, flags=re.M), n
    assert lib.pds_version() >= 100


def test_struct_layout_matches_header():
    """Compile a tiny C program against pds.h that prints offsetof/sizeof and
    compare with the ctypes mirror."""
    fields = [f[0] for f in L.PdsJob._fields_]
    src = "#include <stdio.h>\n#include <stddef.h>\n#include \"pds.h\"\nint main(void){\n"
    src += 'printf("%zu\\n", sizeof(pds_job));\n'
    for f in fields:
        src += 'printf("%%zu\\n", offsetof(pds_job, %s));\n' % f
    src += "return 0;}\n"
    d = os.path.join("/tmp", "pds_layout_%d" % os.getpid())
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "t.c"), "w") as fh:
        fh.write(src)
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", os.path.join(d, "t"), os.path.join(d, "t.c")])
    vals = [int(x) for x in subprocess.check_output([os.path.join(d, "t")]).split()]
    assert vals[0] == C.sizeof(L.PdsJob)
    for f, off in zip(fields, vals[1:]):
        assert getattr(L.PdsJob, f).offset == off, f


def _job(**kw):
    j = L.PdsJob()
    j.model, j.n_dof, j.M, j.d_x = L.PDS_MODEL_PLANAR, 2, 4, 2
    j.N, j.K, j.T, j.n_s, j.h, j.combine = 8, 1, 20, 2, 10, 0
    j.dt, j.sigma_def, j.c = 0.01, 0.1, 1.0
    for k, v in kw.items():
        setattr(j, k, v)
    return j


@pytest.mark.parametrize("bad,code", [
    (dict(T=21), -1), (dict(N=0), -1), (dict(dt=0.0), -1), (dict(sigma_def=-1.0), -1),
    (dict(n_dof=6, M=12, d_x=6), -2), (dict(model=2), -1), (dict(model=7), -1), (dict(M=3), -1),
    (dict(combine=5), -1), (dict(N=32769), -2),
    (dict(model=3), -1), (dict(model=3, n_dof=3, M=17, d_x=3), -2), (dict(d_x=3), -1), (dict(limits=2), -1),
    (dict(model=4, n_dof=9, M=11, d_x=1), -1),
    (dict(N=32768, K=700, n_s=20, h=1, T=20), -2),  # states and multipliers past 32-bit flat indexing
])
def test_invalid_jobs_rejected_on_host(bad, code):
    lib = L.lib()
    arr = (L.PdsJob * 1)(_job(**bad))
    fake_dev = C.c_void_p(4096)  # never dereferenced: validation fails first
    for fn in (lib.sim_batch_forward, lib.loglik_multishoot, lib.sim_batch_adjoint):
        rc = fn(arr, fake_dev, 1, None, 0, None)
        assert rc == code
        assert len(lib.pds_last_error()) > 0


def test_null_buffers_and_batch_size_rejected():
    lib = L.lib()
    arr = (L.PdsJob * 1)(_job())
    fake_dev = C.c_void_p(4096)
    assert lib.sim_batch_forward(arr, fake_dev, 1, None, 0, None) == -1  # theta etc. NULL
    assert b"NULL" in lib.pds_last_error()
    assert lib.svgd_phi(arr, fake_dev, 0, None, 0, None) == -1
    assert lib.svgd_step(arr, fake_dev, 1, 7, 1, None) == -1
    assert lib.pds_workspace_size(arr, 0, 5) == 0


def test_exclusive_constraint_seeds_rejected():
    """seed_gdef and cot_gdef both set is rejected before anything is queued."""
    lib = L.lib()
    fake = C.c_void_p(4096)
    ptrs = {n: 4096 for n in ("consts", "theta", "s0", "end_states", "S", "obs", "w_x", "u", "ll_win", "logp", "wk",
                               "gdef", "g_obs", "g_con", "S_dot", "lam_def")}
    arr = (L.PdsJob * 1)(_job(seed_gdef=4096, cot_gdef=8192, **ptrs))
    assert lib.sim_batch_adjoint(arr, fake, 1, None, 0, None) == -1
    assert b"exclusive" in lib.pds_last_error()


def test_workspace_size_grows_with_problem():
    lib = L.lib()
    small = (L.PdsJob * 1)(_job())
    big = (L.PdsJob * 1)(_job(N=1024, K=8, T=1000, n_s=20, h=50))
    assert lib.pds_workspace_size(small, 1, L.PDS_CALL_FORWARD) == 0
    a = lib.pds_workspace_size(small, 1, L.PDS_CALL_ADJOINT)
    b = lib.pds_workspace_size(big, 1, L.PDS_CALL_ADJOINT)
    assert 0 < a < b
    assert b % 256 == 0


def test_algorithmic_flop_counts():
    """The counting scalar runs the library's own step functions: planar
    counts grow linearly with the links; the arm step evaluates sin and cos
    of its 8 joint angles and of the 7 desired-trajectory phases."""
    planar = [L.algorithmic_flops(L.PDS_MODEL_PLANAR, n) for n in range(1, 6)]
    fwd = np.array([p[0] for p in planar])
    rev = np.array([p[1] for p in planar])
    # the ABA's passes grow linearly with the links (1, 3, 4, 5); two links
    # run in closed form with less work than the ABA would need there
    assert fwd[3] - fwd[2] == fwd[4] - fwd[3] == (fwd[2] - fwd[0]) / 2
    assert rev[3] - rev[2] == rev[4] - rev[3] == (rev[2] - rev[0]) / 2
    assert fwd[1] < (fwd[0] + fwd[2]) / 2 and rev[1] < (rev[0] + rev[2]) / 2
    assert [p[2] for p in planar] == [2.0 * n for n in range(1, 6)]
    f, r, t = L.algorithmic_flops(L.PDS_MODEL_ARM, 8)
    assert t == 2 * 8 + 2 * 7
    assert f > 1000 and r > 1000
    assert L.algorithmic_flops(L.PDS_MODEL_ARM, 8) == (f, r, t)
    # universal joint: a ninth body, the box-frame kinematics and its adjoint
    uf, ur, ut = L.algorithmic_flops(L.PDS_MODEL_ARM_UJOINT, 9)
    assert uf > f and ur > r and ut > t
    wf, wr, wt = L.algorithmic_flops(L.PDS_MODEL_ARM_UJOINT_WEIGHTS, 9)
    assert wf > f and wr > r and wt == ut
    # rigid links: the same sin/cos per joint, more work per link than point masses
    for n in (1, 2):
        rf, rr, rt = L.algorithmic_flops(L.PDS_MODEL_PLANAR_RIGID, n)
        assert rt == 2.0 * n
        assert rf > planar[n - 1][0] and rr > planar[n - 1][1]


def test_arm_flop_counts_follow_the_tables_structure():
    """An arm table with the Panda arm's kinematic structure (the synthetic
    ones) is counted with that structure's step functions -- fewer FLOPs,
    the same sin/cos -- and one off it (a general twist, two more offsets)
    with the generic ones, which pds_algorithmic_flops also counts."""
    from paper_2109_08815_amd import synth
    for cfg, nb in (("c4", 8), ("box1", 9), ("box2", 9)):
        model, raw = L.model_consts(synth.make_problem(cfg, N=4, K=1, T=10, n_s=1))
        f, r, t, panda = L.arm_algorithmic_flops(model, raw)
        assert panda
        g = L.algorithmic_flops(model, nb)
        assert f < g[0] and r < g[1] and t == g[2]
        model, raw = L.model_consts(synth.make_problem(cfg, N=4, K=1, T=10, n_s=1, generic_dh=True))
        assert L.arm_algorithmic_flops(model, raw) == (*g, False)
    # within float rounding of the right angles still counts as the Panda structure
    model, raw = L.model_consts(synth.make_problem("c4", N=4, K=1, T=10, n_s=1))
    raw = np.asarray(raw, np.float32)
    raw[3 + 16 * 1 + 1] = np.nextafter(raw[3 + 16 * 1 + 1], np.float32(0))
    assert L.arm_algorithmic_flops(model, raw)[3]
    raw[3 + 16 * 1 + 1] -= np.float32(1e-5)
    assert not L.arm_algorithmic_flops(model, raw)[3]
    lib = L.lib()
    d = C.c_double()
    assert lib.pds_arm_algorithmic_flops(L.PDS_MODEL_PLANAR, raw.ctypes.data_as(C.c_void_p), C.byref(d), C.byref(d),
                                         C.byref(d), None) == -1
    assert lib.pds_arm_algorithmic_flops(model, None, C.byref(d), C.byref(d), C.byref(d), None) == -1


def test_metrics_arguments_rejected_on_host():
    """pds_traj_metrics validates before queueing anything (the fake device
    addresses are never dereferenced)."""
    lib = L.lib()
    dev = C.c_void_p(4096)
    ws = C.c_void_p(1 << 20)
    nb = lib.pds_traj_metrics_workspace(100, 20, 64)
    assert nb > 0 and nb % 256 == 0
    assert lib.pds_traj_metrics_workspace(1, 20, 64) == 0 and len(lib.pds_last_error()) > 0

    def call(n=100, m=20, d=64, k=3, l=3, sigma=0.0, P=dev, Q=dev, out=dev, w=None, ws_=ws, nbytes=nb):
        return lib.pds_traj_metrics(P, n, Q, m, d, w, k, l, sigma, out, None, ws_, nbytes, None)

    assert call(P=None) == -1
    assert call(k=9) == -2
    assert call(l=0) == -2
    assert call(n=3) == -1          # l + 1 = 4 rows needed
    assert call(m=3, k=4, l=2) == -1
    assert call(d=0) == -1
    assert call(n=16000, m=1000) == -2
    assert call(ws_=C.c_void_p((1 << 20) + 64)) == -1  # misaligned workspace
    assert call(nbytes=nb - 1) == -1
    assert call(sigma=float("nan")) == -1
    assert lib.pds_traj_metrics_workspace(1000, 40, 5000) > lib.pds_traj_metrics_workspace(100, 20, 64)


def test_timing_repeat_count_validated_on_host():
    """pds_timing_enable takes 0 (off) or 1..64 launches per timed call;
    anything else is rejected before any event is created."""
    lib = L.lib()
    assert lib.pds_timing_enable(-1) == -1 and b"64" in lib.pds_last_error()
    assert lib.pds_timing_enable(65) == -1
    assert lib.pds_timing_enable(0) == 0


def _shape(cfg, **over):
    from paper_2109_08815_amd import synth
    pb = synth.make_problem(cfg, **over)
    return L.adjoint_shape(L.shape_struct(pb))


def test_adjoint_launch_shape_boundaries():
    """The host's choice of adjoint storage at its boundaries.  A split job
    has fewer than 1024 waves of 64 units; the whole window ((h + 1) states
    of 2 n_dof floats per lane) stays in LDS when all of the job's waves fit
    on the 256 CUs at once (160 KiB each); the double pendulum's tape (7
    floats per step and unit, 32 units per wave) joins it on the same
    condition with the larger footprint."""
    full2 = lambda h: (h + 1) * 4 * 64 * 4
    tape2 = lambda h: full2(h) + h * 7 * 32 * 4
    # the benchmark's double pendulum: 320 waves, two 76 KiB waves per CU
    assert _shape("c2") == (True, True, True, tape2(40)) and tape2(40) == 77824
    # 512 waves still fit with the tape, 513 do not (K = 1, 16 windows)
    assert _shape("c2", N=1024, K=1, T=640, n_s=16) == (True, True, True, tape2(40))
    assert _shape("c2", N=1025, K=1, T=640, n_s=16) == (True, True, False, full2(40))
    # 750 waves: the window alone fits three per CU
    assert _shape("c2", N=600) == (True, True, False, full2(40))
    # one wave per CU with the tape up to h = 84, none at 85
    assert _shape("c2", N=40, K=1, T=168, n_s=2) == (True, True, True, tape2(84))
    assert _shape("c2", N=40, K=1, T=170, n_s=2) == (True, True, False, full2(85))
    # rigid links keep the re-evaluation
    assert _shape("rigid2")[:3] == (True, True, False)
    # the 5-link chain: 2560 waves, one lane per unit, sqrt(h) = 8-step segments
    # (7 checkpoints + 9 segment states of 10 floats per lane)
    assert _shape("c3") == (False, False, False, (7 + 8 + 1) * 10 * 64 * 4)


def test_adjoint_shape_rejects_other_models():
    from paper_2109_08815_amd import synth
    j = L.shape_struct(synth.make_problem("c4"))
    with pytest.raises(L.PdsError):
        L.adjoint_shape(j)
    j = L.shape_struct(synth.make_problem("c2"))
    j.h = 0
    with pytest.raises(L.PdsError):
        L.adjoint_shape(j)
