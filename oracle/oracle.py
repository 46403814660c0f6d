"""ctypes front end of the FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the GPU library or its
Python binding.  Every function takes a ``synth.Problem`` (or plain arrays)
and returns numpy float64 arrays.  Section / equation references for each
computation are in ``oracle.cpp``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRCS = [os.path.join(_HERE, f) for f in ("oracle.cpp", "dual.hpp", "spatial.hpp")]
_lock = threading.Lock()
_lib = None

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


class OrcModel(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("n_dof", C.c_int32), ("M", C.c_int32), ("d_x", C.c_int32),
        ("obs_index", C.c_int32 * 16), ("gravity", C.c_double * 3), ("damping", C.c_double * 8),
        ("dh_a", C.c_double * 7), ("dh_alpha", C.c_double * 7), ("dh_d", C.c_double * 7),
        ("link_m", C.c_double * 7), ("link_c", (C.c_double * 3) * 7), ("link_I", (C.c_double * 3) * 7),
        ("kp", C.c_double * 7), ("kd", C.c_double * 7), ("qc", C.c_double * 7), ("amp", C.c_double * 7),
        ("omega", C.c_double * 7), ("phase", C.c_double * 7), ("flange_d", C.c_double),
        ("box_m", C.c_double), ("box_c", C.c_double * 3), ("box_I", C.c_double * 3),
        ("pm_m", C.c_double), ("pm_z", C.c_double), ("box_Ioff", C.c_double * 3), ("ujoint_b", C.c_double * 2),
    ]


class OrcProblem(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("K", C.c_int32), ("T", C.c_int32), ("n_s", C.c_int32), ("h", C.c_int32),
        ("combine", C.c_int32), ("lik", C.c_int32), ("dt", C.c_double), ("sigma_def", C.c_double),
        ("c", C.c_double),
        ("w_x", _D), ("u", _D), ("s0", _D), ("obs", _D), ("theta", _D), ("S", _D), ("lam_def", _D),
    ]


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (OpenMP) if missing or stale."""
    stale = not os.path.exists(_SO) or any(os.path.getmtime(s) > os.path.getmtime(_SO) for s in _SRCS)
    if force or stale:
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                               os.path.join(_HERE, "oracle.cpp")])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_SO)
            L.orc_threads.restype = C.c_int
            L.orc_set_threads.argtypes = [C.c_int]
            L.orc_aba.argtypes = [C.POINTER(OrcModel), _D, _D, _D, _D, _D]
            L.orc_crba_rnea.argtypes = [C.POINTER(OrcModel), _D, _D, _D, _D, _D]
            L.orc_tau.argtypes = [C.POINTER(OrcModel), _D, C.c_double, _D, _D, _D]
            L.orc_rollout.argtypes = [C.POINTER(OrcModel), _D, _D, C.c_int, C.c_int, C.c_double, _D]
            L.orc_observe.argtypes = [C.POINTER(OrcModel), _D, _D, _D, _D]
            L.orc_forward.argtypes = [C.POINTER(OrcModel), C.POINTER(OrcProblem), C.c_int, _I, _D, _D, _D, _D, _D, _D]
            L.orc_gradient.argtypes = [C.POINTER(OrcModel), C.POINTER(OrcProblem), C.c_int, _I, _D, _D, _D, _D, _D,
                                       _D, _D, _D, _D, _D]
            L.orc_gradient.restype = C.c_int
            L.orc_bandwidth.argtypes = [C.c_int, C.c_int, _D, _D, _I, _D]
            L.orc_bandwidth.restype = C.c_double
            L.orc_phi.argtypes = [C.c_int, C.c_int, _D, _D, _D, C.c_double, _I, C.c_int, _I, _D]
            L.orc_mdmm_step.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, _D, _D, _D, _D,
                                        _D, _D, _D, _D, C.c_double, C.c_int, C.c_int, _D, _D, _D, _D, _D, _D, _I]
            _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _mask(a):
    """Boolean per-particle mask as a C int array (None stays None)."""
    return None if a is None else np.ascontiguousarray(np.asarray(a, dtype=bool), dtype=np.int32)


def _ip(a):
    return None if a is None else a.ctypes.data_as(_I)


# Particle status bits (the oracle's own bookkeeping of the ensemble):
# a non-finite state, a non-finite likelihood or gradient, and frozen
# (left out of the ensemble by an earlier update).
FLAG_STATE, FLAG_GRAD, FLAG_FROZEN = 1, 2, 8


def model_struct(pb) -> OrcModel:
    m = OrcModel()
    m.kind, m.n_dof, m.M, m.d_x = pb.kind, pb.n_dof, pb.M, pb.d_x
    for i, v in enumerate(pb.obs_index):
        m.obs_index[i] = int(v)
    for i in range(3):
        m.gravity[i] = float(pb.gravity[i])
    for i in range(8):
        m.damping[i] = float(pb.damping[i])
    if pb.arm is not None:
        a = pb.arm
        for i in range(7):
            m.dh_a[i], m.dh_alpha[i], m.dh_d[i] = a["dh_a"][i], a["dh_alpha"][i], a["dh_d"][i]
            m.link_m[i] = a["link_m"][i]
            for d in range(3):
                m.link_c[i][d] = a["link_c"][i][d]
                m.link_I[i][d] = a["link_I"][i][d]
            m.kp[i], m.kd[i], m.qc[i] = a["kp"][i], a["kd"][i], a["qc"][i]
            m.amp[i], m.omega[i], m.phase[i] = a["amp"][i], a["omega"][i], a["phase"][i]
        m.flange_d, m.box_m, m.pm_m, m.pm_z = a["flange_d"], a["box_m"], a["pm_m"], a["pm_z"]
        for d in range(3):
            m.box_c[d] = a["box_c"][d]
            m.box_I[d] = a["box_I"][d]
            m.box_Ioff[d] = a.get("box_Ioff", np.zeros(3))[d]
        for d in range(2):
            m.ujoint_b[d] = a.get("ujoint_b", np.zeros(2))[d]
    return m


class State:
    """Particle state of one job in FP64 (theta, S, multipliers, Adam moments)."""

    def __init__(self, pb, theta, S, lam_lim=None, lam_def=None, adam_m=None, adam_v=None):
        N, K, ns, ds, M = theta.shape[0], pb.K, pb.n_s, pb.d_s, pb.M
        self.theta = _f64(theta).copy()
        self.S = _f64(S).reshape(N, K, ns - 1, ds).copy()
        self.lam_lim = np.zeros((N, M)) if lam_lim is None else _f64(lam_lim).copy()
        self.lam_def = np.zeros((N, K, ns - 1)) if lam_def is None else _f64(lam_def).copy()
        nA = M + K * (ns - 1) * ds
        self.adam_m = np.zeros((N, nA)) if adam_m is None else _f64(adam_m).copy()
        self.adam_v = np.zeros((N, nA)) if adam_v is None else _f64(adam_v).copy()
        self.flags = np.zeros(N, dtype=np.int64)


def _problem(pb, obs, st: State, keep):
    keep.extend([_f64(pb.w_x), _f64(pb.u), _f64(pb.s0), _f64(obs), st.theta, st.S, st.lam_def])
    p = OrcProblem()
    p.N, p.K, p.T, p.n_s, p.h, p.combine = st.theta.shape[0], pb.K, pb.T, pb.n_s, pb.h, pb.combine
    p.lik = int(getattr(pb, "lik", 0))
    p.dt, p.sigma_def, p.c = pb.dt, pb.sigma_def, pb.c
    p.w_x, p.u, p.s0, p.obs, p.theta, p.S, p.lam_def = [_p(a) for a in keep[-7:]]
    return p


def aba(pb, theta, q, qd, tau):
    out = np.zeros(pb.n_dof)
    m = model_struct(pb)
    lib().orc_aba(C.byref(m), _p(_f64(theta)), _p(_f64(q)), _p(_f64(qd)), _p(_f64(tau)), _p(out))
    return out


def crba_rnea(pb, theta, q, qd):
    n = pb.n_dof
    H = np.zeros((n, n))
    Cb = np.zeros(n)
    m = model_struct(pb)
    lib().orc_crba_rnea(C.byref(m), _p(_f64(theta)), _p(_f64(q)), _p(_f64(qd)), _p(H), _p(Cb))
    return H, Cb


def tau(pb, theta, time, q, qd):
    out = np.zeros(pb.n_dof)
    m = model_struct(pb)
    lib().orc_tau(C.byref(m), _p(_f64(theta)), float(time), _p(_f64(q)), _p(_f64(qd)), _p(out))
    return out


def rollout(pb, theta, s0, n_steps, t0=0, dt=None):
    """States t0+1 .. t0+n_steps from s0 at step t0 (single shooting)."""
    out = np.zeros((n_steps, pb.d_s))
    m = model_struct(pb)
    lib().orc_rollout(C.byref(m), _p(_f64(theta)), _p(_f64(s0)), int(t0), int(n_steps),
                      float(pb.dt if dt is None else dt), _p(out))
    return out


def observations(pb, theta_true=None):
    """Observed trajectories [K, T, d_x]: oracle rollout from s0_k at theta_true_k plus the noise draws."""
    tt = pb.theta_true if theta_true is None else theta_true
    obs = np.zeros((pb.K, pb.T, pb.d_x))
    for k in range(pb.K):
        tr = rollout(pb, tt[k], pb.s0[k], pb.T)
        obs[k] = observe(pb, tt[k], tr) + pb.noise[k]
    return obs


def observe(pb, theta, states):
    """Observed quantities [n, d_x] of states [n, d_s] (the listed state
    components, or the box-frame points of the universal-joint arm)."""
    states = np.atleast_2d(states)
    if pb.kind not in (5, 6):
        return states[:, pb.obs_index]
    m = model_struct(pb)
    th = _f64(theta)
    n = pb.n_dof
    out = np.zeros((states.shape[0], pb.d_x))
    x = np.zeros(pb.d_x)
    for t in range(states.shape[0]):
        lib().orc_observe(C.byref(m), _p(th), _p(_f64(states[t, :n])), _p(_f64(states[t, n:])), _p(x))
        out[t] = x
    return out


def shooting_init(pb, theta, obs=None):
    """Default shooting states: each particle's own single-shooting state at
    step j*h (j >= 1), from one window over the whole trajectory per
    particle and trajectory (threads over them)."""
    import dataclasses

    N = theta.shape[0]
    if pb.n_s == 1:
        return np.zeros((N, pb.K, 0, pb.d_s))
    ss = dataclasses.replace(pb, n_s=1, h=pb.T, N=N)
    st = State(ss, theta, np.zeros((N, pb.K, 0, pb.d_s)))
    tr = forward(ss, np.zeros((pb.K, pb.T, pb.d_x)), st, traj=True)["traj"]
    return np.ascontiguousarray(tr[:, :, pb.h - 1 : pb.T - 1 : pb.h])


def forward(pb, obs, st: State, sel=None, traj=False):
    N = st.theta.shape[0]
    sel = np.arange(N, dtype=np.int32) if sel is None else np.ascontiguousarray(sel, dtype=np.int32)
    ns, K, ds = pb.n_s, pb.K, pb.d_s
    n = len(sel)
    keep = []
    p = _problem(pb, obs, st, keep)
    tr = np.zeros((n, K, pb.T, ds)) if traj else None
    es = np.zeros((n, K, ns, ds))
    ll = np.zeros((n, K, ns))
    gd = np.zeros((n, K, max(ns - 1, 1)))
    lp = np.zeros(n)
    wk = np.zeros((n, K))
    m = model_struct(pb)
    lib().orc_forward(C.byref(m), C.byref(p), n, sel.ctypes.data_as(_I), _p(tr), _p(es), _p(ll), _p(gd), _p(lp), _p(wk))
    out = dict(end_states=es, ll_win=ll, gdef=gd[:, :, : ns - 1], logp=lp, wk=wk)
    if traj:
        out["traj"] = tr
    return out


def gradient(pb, obs, st: State, sel=None, per_unit=False):
    N = st.theta.shape[0]
    sel = np.arange(N, dtype=np.int32) if sel is None else np.ascontiguousarray(sel, dtype=np.int32)
    ns, K, ds, M = pb.n_s, pb.K, pb.d_s, pb.M
    n = len(sel)
    keep = []
    p = _problem(pb, obs, st, keep)
    es = np.zeros((n, K, ns, ds))
    ll = np.zeros((n, K, ns))
    gd = np.zeros((n, K, max(ns - 1, 1)))
    lp = np.zeros(n)
    wk = np.zeros((n, K))
    go = np.zeros((n, M))
    gc = np.zeros((n, M))
    sd = np.zeros((n, K, max(ns - 1, 1), ds))
    pu = np.zeros((n, K, ns, M)) if per_unit else None
    pc = np.zeros((n, K, ns, M)) if per_unit else None
    m = model_struct(pb)
    rc = lib().orc_gradient(C.byref(m), C.byref(p), n, sel.ctypes.data_as(_I), _p(es), _p(ll), _p(gd), _p(lp),
                            _p(wk), _p(go), _p(gc), _p(sd), _p(pu), _p(pc))
    if rc != 0:
        raise ValueError("oracle: M + d_s exceeds the compiled dual width")
    out = dict(end_states=es, ll_win=ll, gdef=gd[:, :, : ns - 1], logp=lp, wk=wk, g_obs=go, g_con=gc,
               S_dot=sd[:, :, : ns - 1])
    if per_unit:
        out["dl_dtheta_unit"] = pu
        out["dcon_dtheta_unit"] = pc
    return out


def bandwidth(theta, rho, live=None):
    """Median-heuristic bandwidth over the particles with ``live`` true (all
    when None): pairs among them, log of their number."""
    th = _f64(theta)
    N, M = th.shape
    med = C.c_double(0.0)
    lv = _mask(live)
    h = lib().orc_bandwidth(N, M, _p(th), _p(_f64(rho)), _ip(lv), C.byref(med))
    return h, med.value


def phi(theta, grad, rho, h, sel=None, live=None):
    """SVGD direction of the rows ``sel`` over the ensemble of particles with
    ``live`` true (all when None); rows of other particles are zero."""
    th = _f64(theta)
    N, M = th.shape
    sel = np.arange(N, dtype=np.int32) if sel is None else np.ascontiguousarray(sel, dtype=np.int32)
    out = np.zeros((len(sel), M))
    lv = _mask(live)
    lib().orc_phi(N, M, _p(th), _p(_f64(grad)), _p(_f64(rho)), float(h), _ip(lv), len(sel), sel.ctypes.data_as(_I),
                  _p(out))
    return out


def nonfinite_flags(out):
    """Status bits of each particle from one gradient evaluation: FLAG_STATE
    for a non-finite window end state, FLAG_GRAD for a non-finite log
    likelihood or gradient."""
    n = out["logp"].shape[0]
    bad = lambda a: ~np.isfinite(a.reshape(n, -1)).all(axis=1)  # noqa: E731
    f = np.where(bad(out["end_states"]), FLAG_STATE, 0)
    g = bad(out["logp"]) | bad(out["g_obs"]) | bad(out["g_con"]) | bad(out["S_dot"])
    return f | np.where(g, FLAG_GRAD, 0)


def mdmm_step(pb, st: State, phi_, g_con, S_dot, gdef, optimizer, it, lr_theta=None, lr_S=None, eps_lam=None,
              frozen=None):
    """In-place MDMM / optimizer update of ``st`` (Algorithm 1); particles
    with ``frozen`` true keep every variable."""
    N = st.theta.shape[0]
    lrt = _f64(pb.lr_theta if lr_theta is None else lr_theta)
    lrs = _f64(pb.lr_S if lr_S is None else lr_S)
    el = pb.eps_lam if eps_lam is None else eps_lam
    Sd = _f64(S_dot).reshape(N, pb.K, pb.n_s - 1, pb.d_s) if pb.n_s > 1 else np.zeros((N, pb.K, 1, pb.d_s))
    # defects inside p_ms (lik = 1) are no constraints: lam_def stays put
    gd = _f64(gdef) if pb.n_s > 1 and getattr(pb, "lik", 0) == 0 else np.zeros((N, pb.K, max(pb.n_s - 1, 1)))
    lib().orc_mdmm_step(N, pb.M, pb.K, pb.n_s, pb.d_s, float(pb.c), _p(_f64(pb.lo)), _p(_f64(pb.hi)),
                        _p(_f64(phi_)), _p(_f64(g_con)), _p(np.ascontiguousarray(Sd)), _p(np.ascontiguousarray(gd)),
                        _p(lrt), _p(lrs), float(el), int(optimizer), int(it), _p(st.theta), _p(st.S), _p(st.lam_lim),
                        _p(st.lam_def), _p(st.adam_m), _p(st.adam_v), _ip(_mask(frozen)))
    if getattr(pb, "limits", 0) == 1:  # projected limits: clamp the updated theta into the box
        keep = np.ones(N, dtype=bool) if frozen is None else ~np.asarray(frozen, dtype=bool)
        st.theta[keep] = np.clip(st.theta[keep], pb.lo, pb.hi)


def csvgd_iteration(pb, obs, st: State, it, optimizer=1):
    """One CSVGD iteration (Algorithm 1) on FP64 state; returns intermediates.

    Particles whose simulation fails (a non-finite state, likelihood or
    gradient) leave the ensemble: they are left out of the phi sums at once
    and keep their variables; from the next iteration on (FLAG_FROZEN) they
    are left out of the bandwidth median as well.  The median is taken over
    the ensemble as the previous update left it, since it depends on the
    particles' positions alone."""
    h, med = bandwidth(st.theta, pb.rho, live=(st.flags & FLAG_FROZEN) == 0)
    g = gradient(pb, obs, st)
    st.flags |= nonfinite_flags(g)
    out = (st.flags & (FLAG_STATE | FLAG_GRAD | FLAG_FROZEN)) != 0
    ph = phi(st.theta, g["g_obs"], pb.rho, h, live=~out)
    mdmm_step(pb, st, ph, g["g_con"], g["S_dot"], g["gdef"], optimizer, it, frozen=out)
    st.flags |= np.where(out, FLAG_FROZEN, 0)
    g.update(bandwidth=h, median=med, phi=ph, flags=st.flags.copy(), n_masked=int(out.sum()))
    return g
