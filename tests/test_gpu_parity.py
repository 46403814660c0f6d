"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Both sides get identical inputs: every float the GPU sees is a float32
value, and the oracle receives exactly those values in float64.  The bars
(tests/parity.py) are computed from the oracle's values and the stated
tolerances only: states 1e-4 per window unit, gradients 1e-3 normwise
(term sums where the window terms cancel), S_dot 1e-3 normwise, window
log-likelihoods within what the state tolerance implies.
"""
import numpy as np
import pytest
import torch

from paper_2109_08815_amd import lib as L
from paper_2109_08815_amd import synth
from tests.helpers import f32_problem, print_case, r32, requires_gpu
from tests.parity import (end_state_rel_err, grad_bar, grad_check, ll_tolerance, normwise, observed_err_ratio,
                           state_rel_err, update_check)

pytestmark = [pytest.mark.gpu, requires_gpu]


def make_case(orc, cfg, seed=None, perturb_S=0.0, lam=False, with_traj=False, with_traj_obs=False, **over):
    print_case(cfg, seed, over)
    pb = f32_problem(synth.make_problem(cfg, seed=seed, **over))
    obs = r32(orc.observations(pb))
    S = r32(orc.shooting_init(pb, pb.particles))
    rng = np.random.default_rng(7 if seed is None else seed + 7)
    if perturb_S:
        S = r32(synth.perturb(rng, S, perturb_S))
    lam_def = r32(rng.uniform(0.0, 2.0, (pb.N, pb.K, pb.n_s - 1))) if lam else np.zeros((pb.N, pb.K, pb.n_s - 1))
    st = orc.State(pb, pb.particles, S, lam_def=lam_def)
    job = L.Job(pb, obs, theta=pb.particles, S=S, with_traj=with_traj, with_traj_obs=with_traj_obs)
    job.lam_def.copy_(torch.as_tensor(lam_def, dtype=torch.float32))
    b = L.Batch([job])
    return pb, obs, st, job, b


def np64(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def check_states(pb, traj_gpu, traj_ref):
    rel = state_rel_err(pb, traj_gpu, traj_ref)
    assert rel.max() <= 1e-4, "worst unit rel err %.3e" % rel.max()
    return rel.max()


def check_grads(pb, job, ref, S, sel=None, con=True):
    """g_obs, g_con and S_dot of the particles `sel` against the oracle's."""
    take = (lambda a: a) if sel is None else (lambda a: a[sel])
    Ssel = take(S)
    go = grad_check(take(np64(job.g_obs)), ref, "obs")
    print("g_obs normwise %.2e (terms/|g| up to %.1f), bar ratio %.3f" % (
        go["normwise"].max(), go["terms"].max(), go["ratio"].max()), flush=True)
    assert go["ratio"].max() <= 1.0
    if con and pb.n_s > 1:
        gc = grad_check(take(np64(job.g_con)), ref, "con", pb, Ssel)
        print("g_con normwise %.2e, bar ratio %.3f" % (gc["normwise"].max(), gc["ratio"].max()), flush=True)
        assert gc["ratio"].max() <= 1.0
        sd = normwise(take(np64(job.S_dot))[:, :, : pb.n_s - 1], ref["S_dot"])
        print("S_dot normwise %.2e" % sd.max(), flush=True)
        assert sd.max() <= 1e-3


CASES = [
    ("c1", {}),                                           # headline pendulum config
    ("c2", dict(N=70, K=3)),                              # ragged: 70 particles span 2 waves
    ("c3", dict(N=70, K=2, T=200, n_s=4)),                # 5-link chain, reduced
    ("c2", dict(N=5, K=1, T=40, n_s=1)),                  # single shooting, tiny N
    # launch-shape coverage of the adjoint: few units with windows too long
    # for LDS (two lanes per unit, checkpointed) and many units with short
    # windows (one lane per unit, whole window in LDS).  Windows stay short
    # in time for the chaotic chain (75 steps = 0.15 s): FP32 sensitivities
    # of a 5-link chain over 0.4 s windows drift past 1e-3.
    ("c3", dict(N=64, K=1, T=300, n_s=4)),
    ("c1", dict(N=64, K=1, T=800, n_s=2)),
    ("c1", dict(N=2048, K=8, T=40, n_s=4)),
    # product over trajectories (App. A-B) and defect densities inside p_ms
    # (eq. ms_likelihood), alone and together
    ("c2", dict(N=40, K=3, T=80, n_s=4, combine=synth.COMBINE_PROD)),
    ("c2", dict(N=70, K=3, T=80, n_s=4, lik=synth.LIK_DEFECT)),
    ("c3", dict(N=64, K=2, T=150, n_s=3, lik=synth.LIK_DEFECT, combine=synth.COMBINE_PROD)),
    # rigid links with the 11 parameters of the physical double pendulum
    # (Sec. IV-B), whole state observed, ragged; one rigid link with long
    # windows (two lanes per unit); defect densities inside p_ms
    ("rigid2", dict(N=70, K=3, T=80, n_s=4)),
    ("rigid2", dict(n_dof=1, N=64, K=1, T=800, n_s=2)),
    ("rigid2", dict(N=40, K=2, T=120, n_s=3, lik=synth.LIK_DEFECT)),
    # point masses observed in the whole state (q, qd); rigid links
    # observed in q only
    ("c2", dict(N=70, K=2, T=80, n_s=4, full_state=True)),
    # the double pendulum's closed-form dynamics with joint damping and a
    # gravity component along x
    ("c2", dict(N=70, K=2, T=80, n_s=4, damped=True, gravity_x=2.5)),
    ("rigid2", dict(N=33, K=2, T=80, n_s=2, full_state=False)),
    # one-step windows (a tape of one step).  The whole window without the
    # tape is covered at 40-step windows by the 600-particle comparison
    # below; at small N it needs windows of 85 steps or more, over which
    # FP32 rounding in this chaotic system alone drifts past 1e-3.
    ("c2", dict(N=40, K=2, T=12, n_s=12)),
]


@pytest.mark.parametrize("cfg,over", CASES)
def test_forward_states_and_loglik(orc, cfg, over):
    pb, obs, st, job, b = make_case(orc, cfg, perturb_S=0.01, lam=True, with_traj=True, **over)
    L.loglik_multishoot(b)
    L.sim_batch_forward(b)
    ref = orc.forward(pb, obs, st, traj=True)
    check_states(pb, np64(job.traj), ref["traj"])
    es = np64(job.end_states)
    np.testing.assert_array_equal(es, np64(job.traj).reshape(pb.N, pb.K, pb.n_s, pb.h, pb.d_s)[:, :, :, -1])
    tol = ll_tolerance(pb, obs, ref["traj"], ref["ll_win"])
    d = np.abs(np64(job.ll_win) - ref["ll_win"])
    assert np.all(d <= tol), "ll_win worst ratio %.3g" % (d / tol).max()
    if pb.n_s > 1:
        S = st.S
        e_ref = np.sqrt(ref["gdef"]) * pb.sigma_def
        e_gpu = np.sqrt(np64(job.gdef)[:, :, : pb.n_s - 1]) * pb.sigma_def
        es_scale = np.maximum(np.abs(ref["end_states"][:, :, :-1]).max(axis=3), 1e-6)
        assert np.all(np.abs(e_gpu - e_ref) <= 1e-4 * es_scale * np.sqrt(pb.d_s) + 1e-7), S.shape
    lp_tol = tol.sum(axis=2).max(axis=1)
    assert np.all(np.abs(np64(job.logp) - ref["logp"]) <= lp_tol)
    assert np.all(np.abs(np64(job.wk) - ref["wk"]) <= 2 * lp_tol[:, None] + 1e-12)


@pytest.mark.parametrize("cfg,over", CASES)
def test_adjoint_gradients(orc, cfg, over):
    pb, obs, st, job, b = make_case(orc, cfg, perturb_S=0.01, lam=True, **over)
    L.sim_batch_adjoint(b)
    ref = orc.gradient(pb, obs, st, per_unit=True)
    check_grads(pb, job, ref, st.S)
    assert np.all(np64(job.flags) == 0)


@pytest.mark.parametrize("cfg", ["c2", "rigid2"])
def test_adjoint_full_c2_sampled(orc, cfg):
    """Headline double-pendulum size (N=256, K=4, T=400, 10 windows), the
    launch the benchmark times (point-mass links), and the rigid-link model
    at the same size; every particle's forward quantities and a sample of
    particles' gradients against the oracle."""
    pb, obs, st, job, b = make_case(orc, cfg, perturb_S=0.01, lam=True)
    L.sim_batch_adjoint(b)
    sel = np.arange(0, pb.N, 17)
    ref = orc.gradient(pb, obs, st, sel=sel, per_unit=True)
    check_grads(pb, job, ref, st.S, sel)
    fwd = orc.forward(pb, obs, st, traj=True)
    tol = ll_tolerance(pb, obs, fwd["traj"], fwd["ll_win"])
    assert np.all(np.abs(np64(job.ll_win) - fwd["ll_win"]) <= tol)


def test_taped_and_reevaluated_double_pendulum_adjoints(orc):
    """The double pendulum's adjoint keeps each step's dynamics tape in LDS
    when all of the job's waves still fit on the chip with it (N = 256:
    320 waves of 76 KiB), and evaluates the dynamics again in the reverse
    sweep otherwise (N = 600: 750 waves, only 512 fit with the tape).  The
    first 256 particles of the larger job carry the smaller job's
    parameters, shooting states and multipliers; their outputs depend on
    their own windows alone.  The forward sweep is the same code on both
    paths (bitwise equal outputs).  The reverse sweep's re-evaluation may
    round differently from the forward sweep's evaluation (the compiler
    fuses multiply-adds per context), so the gradients agree to FP32
    rounding: 1e-4 of each particle's gradient norm, and both paths meet
    the oracle's bar."""
    import dataclasses

    pb, obs, st, big, b = make_case(orc, "c2", perturb_S=0.01, lam=True, N=600)
    n = 256
    pb_s = dataclasses.replace(pb, N=n, particles=pb.particles[:n].copy())
    small = L.Job(pb_s, obs, theta=pb_s.particles, S=st.S[:n])
    small.lam_def.copy_(torch.as_tensor(st.lam_def[:n], dtype=torch.float32))
    L.sim_batch_adjoint(b)
    L.sim_batch_adjoint(L.Batch([small]))
    for name in ("ll_win", "gdef", "logp", "wk"):
        np.testing.assert_array_equal(np64(getattr(big, name))[:n], np64(getattr(small, name)), err_msg=name)
    for name in ("g_obs", "g_con", "S_dot"):
        a = np64(getattr(big, name))[:n].reshape(n, -1)
        c = np64(getattr(small, name)).reshape(n, -1)
        assert np.all(np.linalg.norm(a - c, axis=1) <= 1e-4 * np.linalg.norm(c, axis=1)), name
    # both paths' sampled gradients against the oracle
    sel = np.arange(0, n, 37)
    ref = orc.gradient(pb, obs, st, sel=sel, per_unit=True)
    for job in (big, small):
        check_grads(pb, job, ref, st.S, sel)


def test_double_pendulum_checkpointed_adjoint_sampled(orc):
    """Split double-pendulum job whose whole windows do not all fit in LDS at
    once (N = 256, K = 8, 10 windows of 60 steps: 640 waves of 61 KiB, 512
    fit), so the adjoint keeps checkpoints and re-evaluates each segment:
    sampled particles against the oracle."""
    pb, obs, st, job, b = make_case(orc, "c2", perturb_S=0.01, lam=True, K=8, T=600, n_s=10)
    L.sim_batch_adjoint(b)
    sel = np.arange(0, pb.N, 51)
    ref = orc.gradient(pb, obs, st, sel=sel, per_unit=True)
    check_grads(pb, job, ref, st.S, sel)


@pytest.mark.slow
def test_full_c3_sampled(orc):
    """5-link chain at its full size (N=1024, K=8, T=1000, 20 windows): all
    window states of a particle sample and their gradients."""
    pb, obs, st, job, b = make_case(orc, "c3", perturb_S=0.005, lam=True)
    L.sim_batch_adjoint(b)
    sel = np.array([0, 1, 63, 64, 511, 1000, 1023])
    ref = orc.gradient(pb, obs, st, sel=sel, per_unit=True)
    check_grads(pb, job, ref, st.S, sel)
    rel = end_state_rel_err(np64(job.end_states)[sel], ref["end_states"])
    assert rel.max() <= 1e-4


@pytest.mark.slow
@pytest.mark.parametrize("cfg", ["c4", "box2"])
def test_full_arm_sampled(orc, cfg):
    """The 7-joint arm at its full size (N=2048, K=1, T=1500 at 240 Hz, 30
    windows of 50 steps), the launch the benchmark times: with the hinged
    box (c4) and with two weights in the box on a universal joint (box2).
    Every window state of a particle sample, their end states and window
    log-likelihoods, and their gradients against the oracle."""
    pb, obs, st, job, b = make_case(orc, cfg, perturb_S=0.005, lam=True, with_traj=True)
    L.sim_batch_forward(b)
    traj = np64(job.traj)
    L.sim_batch_adjoint(b)
    sel = np.array([0, 1, 63, 64, 511, 1024, 1500, 2047])
    ref = orc.gradient(pb, obs, st, sel=sel, per_unit=True)
    fwd = orc.forward(pb, obs, st, sel=sel, traj=True)
    rel = state_rel_err(pb, traj[sel], fwd["traj"])
    print("states %.2e" % rel.max(), flush=True)
    assert rel.max() <= 1e-4
    assert end_state_rel_err(np64(job.end_states)[sel], ref["end_states"]).max() <= 1e-4
    if cfg == "c4":
        tol = ll_tolerance(pb, obs, fwd["traj"], fwd["ll_win"])
        assert np.all(np.abs(np64(job.ll_win)[sel] - fwd["ll_win"]) <= tol)
    check_grads(pb, job, ref, st.S, sel)
    assert np.all(np64(job.flags) == 0)


def set_tensor(t, a):
    t.copy_(torch.as_tensor(np.asarray(a), dtype=t.dtype))


@pytest.mark.parametrize("N", [1, 2, 3, 64, 65, 200, 300, 512, 700])
def test_bandwidth_exact_and_phi(orc, N):
    print_case("phi", N)
    pb = f32_problem(synth.make_problem("c2", N=N, K=1, T=40, n_s=2))
    rng = np.random.default_rng(N)
    theta = r32(pb.lo + rng.uniform(size=(N, pb.M)) * (pb.hi - pb.lo))
    if N >= 3:
        theta[2] = theta[0]  # a tie at distance 0
    G = rng.normal(scale=1e4, size=(N, pb.M))
    obs = np.zeros((pb.K, pb.T, pb.d_x))
    job = L.Job(pb, obs, theta=theta)
    set_tensor(job.g_obs, G)
    b = L.Batch([job])
    L.svgd_phi(b)
    h_ref, _ = orc.bandwidth(theta, pb.rho)
    h = np64(job.bandwidth)[0]
    # Both sides scale the differences by 1/rho rounded in FP64 (a reading of
    # the median heuristic, not a property of the mathematics: the oracle's
    # form was chosen so that its keys round exactly as the kernel's do), so
    # the exact median agrees to the last bit; dividing by rho instead would
    # move h by a few ulps.
    assert abs(h - h_ref) <= 1e-15 * h_ref
    ph_ref = orc.phi(theta, r32(G), pb.rho, h_ref)
    ph = np64(job.phi)
    d2 = (((theta[:, None, :] - theta[None, :, :]) / pb.rho) ** 2).sum(-1)
    k = np.exp(-d2 / h_ref)
    gk = k[:, :, None] * 2.0 / h_ref * np.abs(theta[:, None, :] - theta[None, :, :]) / pb.rho ** 2
    scale = (k[:, :, None] * np.abs(G)[None, :, :] + gk).mean(axis=1)
    assert np.all(np.abs(ph - ph_ref) <= 1e-4 * scale + 1e-30)


@pytest.mark.parametrize("N,M", [(4500, 4), (4200, 10)])
def test_phi_partial_scheme_sampled_rows(orc, N, M):
    """Jobs above 4096 particles take the partial-sum phi and its reduction;
    sampled rows against the oracle's rows at the oracle's bandwidth."""
    print_case("phi-partial", N, M)
    pb = f32_problem(synth.make_problem("c2" if M == 4 else "c3", N=N, K=1, T=40, n_s=2))
    rng = np.random.default_rng(N + M)
    theta = r32(pb.lo + rng.uniform(size=(N, pb.M)) * (pb.hi - pb.lo))
    G = rng.normal(scale=1e4, size=(N, pb.M))
    job = L.Job(pb, np.zeros((pb.K, pb.T, pb.d_x)), theta=theta)
    set_tensor(job.g_obs, G)
    L.svgd_phi(L.Batch([job]))
    h_ref, _ = orc.bandwidth(theta, pb.rho)
    assert abs(np64(job.bandwidth)[0] - h_ref) <= 1e-15 * h_ref
    sel = np.sort(rng.choice(N, size=48, replace=False)).astype(np.int32)
    ph_ref = orc.phi(theta, r32(G), pb.rho, h_ref, sel=sel)
    ph = np64(job.phi)[sel]
    d = (theta[sel][:, None, :] - theta[None, :, :]) / pb.rho
    k = np.exp(-(d ** 2).sum(-1) / h_ref)
    gk = k[:, :, None] * 2.0 / h_ref * np.abs(d) / pb.rho
    scale = (k[:, :, None] * np.abs(G)[None, :, :] + gk).mean(axis=1)
    assert np.all(np.abs(ph - ph_ref) <= 1e-4 * scale + 1e-30)


def _bandwidth_gpu(pb, theta):
    obs = np.zeros((pb.K, pb.T, pb.d_x))
    job = L.Job(pb, obs, theta=theta)
    L.svgd_phi(L.Batch([job]))
    return np64(job.bandwidth)[0]


@pytest.mark.parametrize("config,N", [("c3", 1024), ("c2", 2048), ("c3", 181), ("c3", 182)])
def test_bandwidth_exact_at_full_size(orc, config, N):
    """Sampled bracket + counting pass (N > 181) and the all-in-LDS path
    (N = 181, 16290 pairs) against the oracle's full sort."""
    print_case("bandwidth", config, N)
    pb = f32_problem(synth.make_problem(config, N=N, K=1, T=40, n_s=2))
    theta = r32(pb.particles[:N]) if pb.particles.shape[0] >= N else r32(
        pb.lo + np.random.default_rng(N).uniform(size=(N, pb.M)) * (pb.hi - pb.lo))
    h_ref, _ = orc.bandwidth(theta, pb.rho)
    assert abs(_bandwidth_gpu(pb, theta) - h_ref) <= 1e-15 * h_ref


@pytest.mark.parametrize("shift", [400, -400, 20000, -20000])
def test_bandwidth_exact_when_bracket_misses(orc, shift):
    """A bracket moved off the middle ranks sends the count kernel's last
    block through its recovery pass; the median stays exact."""
    print_case("bandwidth-miss", shift)
    pb = f32_problem(synth.make_problem("c2", N=600, K=1, T=40, n_s=2))
    theta = r32(pb.lo + np.random.default_rng(7).uniform(size=(600, pb.M)) * (pb.hi - pb.lo))
    h_ref, _ = orc.bandwidth(theta, pb.rho)
    try:
        L.test_median_shift(shift)
        h = _bandwidth_gpu(pb, theta)
    finally:
        L.test_median_shift(0)
    assert abs(h - h_ref) <= 1e-15 * h_ref


@pytest.mark.parametrize("shift,n_frozen", [(0, 0), (0, 3), (400, 0), (-20000, 2)])
def test_narrow_bandwidth_beside_a_small_window_kernel(orc, shift, n_frozen):
    """svgd_bandwidth of a larger job whose window kernels leave SIMDs free
    (the 2048-particle arm job: 960 waves for 1024 SIMDs) runs the median
    in one-wave blocks; the bandwidth is the oracle's exact median, and
    bitwise svgd_phi's (the wide blocks), also with frozen particles and a
    bracket moved off the middle ranks (the final kernel's recovery pass)."""
    print_case("bandwidth-narrow", shift, n_frozen)
    pb = f32_problem(synth.make_problem("c4"))
    assert pb.N * pb.K * pb.n_s // 64 < 1024
    theta = r32(pb.particles)
    flags = np.zeros(pb.N, np.int32)
    flags[np.random.default_rng(11).choice(pb.N, n_frozen, replace=False)] = L.PDS_FLAG_FROZEN
    job = L.Job(pb, np.zeros((pb.K, pb.T, pb.d_x)), theta=theta)
    set_tensor(job.flags, flags)
    b = L.Batch([job])
    try:
        L.test_median_shift(shift)
        L.svgd_bandwidth(b)
        h_narrow = np64(job.bandwidth)[0]
        L.svgd_phi(b)
        h_wide = np64(job.bandwidth)[0]
    finally:
        L.test_median_shift(0)
    h_ref, _ = orc.bandwidth(theta, pb.rho, live=flags == 0)
    assert h_narrow == h_wide
    assert abs(h_narrow - h_ref) <= 1e-15 * h_ref


@pytest.mark.parametrize("groups", [(300, 300), (150, 200, 250), (599, 1), (100, 100), (150, 50), (199, 1),
                                    (64, 64, 72)])
def test_bandwidth_exact_with_heavy_ties(orc, groups):
    """Particles stacked on a few points: most pair distances are exactly
    equal, so candidate sets far exceed the LDS capacity (jobs of up to 200
    particles take the all-pairs selection, larger ones the sampled
    bracket)."""
    print_case("bandwidth-ties", groups)
    pb = f32_problem(synth.make_problem("c2", N=sum(groups), K=1, T=40, n_s=2))
    pts = r32(pb.lo + np.random.default_rng(3).uniform(size=(len(groups), pb.M)) * (pb.hi - pb.lo))
    theta = np.concatenate([np.repeat(pts[g:g + 1], n, axis=0) for g, n in enumerate(groups)])
    h_ref, _ = orc.bandwidth(theta, pb.rho)
    assert abs(_bandwidth_gpu(pb, theta) - h_ref) <= 1e-15 * h_ref


@pytest.mark.parametrize("optimizer,lik,limits,cfg,over", [
    (L.PDS_OPT_SGD, synth.LIK_MDMM, synth.LIMITS_SOFT, "c2", dict(N=70, K=2, T=80, n_s=4)),
    (L.PDS_OPT_ADAM, synth.LIK_MDMM, synth.LIMITS_SOFT, "c2", dict(N=70, K=2, T=80, n_s=4)),
    (L.PDS_OPT_ADAM, synth.LIK_DEFECT, synth.LIMITS_SOFT, "c2", dict(N=70, K=2, T=80, n_s=4)),
    (L.PDS_OPT_ADAM, synth.LIK_MDMM, synth.LIMITS_PROJECT, "c2", dict(N=70, K=2, T=80, n_s=4)),
    # the arm's full shape: 1.02 million elements, several per thread of 249 blocks
    (L.PDS_OPT_ADAM, synth.LIK_MDMM, synth.LIMITS_SOFT, "c4", {})])
def test_step_parity(orc, optimizer, lik, limits, cfg, over):
    print_case("step", optimizer, lik, limits, cfg)
    pb = f32_problem(synth.make_problem(cfg, lik=lik, limits=limits, **over))
    rng = np.random.default_rng(5)
    N, K, ns, ds, M = pb.N, pb.K, pb.n_s, pb.d_s, pb.M
    theta = r32(pb.lo - 0.2 + rng.uniform(size=(N, M)) * (pb.hi - pb.lo + 0.4))  # some outside the limits
    S = r32(rng.normal(size=(N, K, ns - 1, ds)))
    obs = np.zeros((K, pb.T, pb.d_x))
    job = L.Job(pb, obs, theta=theta, S=S, device_iter=True)
    job.iter_dev[0] = 2  # the step uses iteration iter_dev[0] + 1 = 3
    vals = dict(phi=r32(rng.normal(size=(N, M))), g_con=rng.normal(size=(N, M)),
                S_dot=r32(rng.normal(size=(N, K, ns - 1, ds))), gdef=rng.uniform(size=(N, K, ns - 1)),
                lam_lim=r32(rng.normal(size=(N, M))), lam_def=r32(rng.uniform(size=(N, K, ns - 1))),
                adam_m=r32(rng.normal(size=(N, M + K * (ns - 1) * ds)) * 0.1),
                adam_v=r32(rng.uniform(size=(N, M + K * (ns - 1) * ds)) * 0.1))
    for k_, v in vals.items():
        set_tensor(getattr(job, k_), v)
    b = L.Batch([job])
    L.svgd_step(b, optimizer, 3)
    st = orc.State(pb, theta, S, lam_lim=vals["lam_lim"], lam_def=vals["lam_def"], adam_m=vals["adam_m"],
                   adam_v=vals["adam_v"])
    orc.mdmm_step(pb, st, vals["phi"], r32(vals["g_con"]), vals["S_dot"], r32(vals["gdef"]), optimizer, 3)
    for name, ref, old in (("theta", st.theta, theta), ("S", st.S, S)):
        got = np64(getattr(job, name)).reshape(ref.shape)
        dref = ref - old
        assert np.all(np.abs((got - old) - dref) <= 1e-5 * np.abs(dref) + 1e-6 * np.abs(old) + 1e-7), name
    np.testing.assert_allclose(np64(job.lam_lim), st.lam_lim, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(np64(job.lam_def), st.lam_def, rtol=1e-6, atol=1e-7)
    # the blocks advanced the counter once and left their completion count at zero
    assert np64(job.iter_dev).astype(int).tolist() == [3, 0]
    fl = np64(job.flags).astype(int)
    outside = ((st.theta < pb.lo) | (st.theta > pb.hi)).any(axis=1)
    assert np.all(((fl & 4) != 0) == outside)
    if limits == synth.LIMITS_PROJECT:
        got = np64(job.theta).reshape(st.theta.shape)
        assert np.all((got >= pb.lo) & (got <= pb.hi)) and not outside.any()


@pytest.mark.parametrize("cfg,lik,over", [("c2", synth.LIK_MDMM, dict(K=3)), ("c2", synth.LIK_DEFECT, dict(K=3)),
                                          ("rigid2", synth.LIK_MDMM, dict(K=3)),
                                          ("c4", synth.LIK_MDMM, dict(K=1, T=300, n_s=6)),
                                          ("c4", synth.LIK_MDMM, dict(K=1, T=300, n_s=6, generic_dh=True)),
                                          ("box1", synth.LIK_MDMM, dict(K=1, T=192, n_s=4))])
def test_csvgd_iteration_sgd(orc, cfg, lik, over):
    """One full iteration (adjoint -> phi -> step) from identical inputs,
    with the defects as constraints (CSVGD) or inside p_ms; point-mass and
    rigid links (M = 11), the arm with the hinged box and with the box's
    own parameters on a universal joint (M = 11)."""
    pb, obs, st, job, b = make_case(orc, cfg, perturb_S=0.01 if cfg in ("c2", "rigid2") else 0.005, lam=True,
                                    N=70, lik=lik, **over)
    th0 = st.theta.copy()
    S0 = st.S.copy()
    L.csvgd_iteration(b, 1, L.PDS_OPT_SGD)
    g = orc.csvgd_iteration(pb, obs, st, 1, optimizer=0)
    assert abs(np64(job.bandwidth)[0] - g["bandwidth"]) <= 1e-15 * g["bandwidth"]
    assert update_check(np64(job.theta), th0, st.theta).max() <= 1.0
    sd = normwise(np64(job.S_dot)[:, :, : pb.n_s - 1], g["S_dot"])
    print("S_dot normwise %.2e" % sd.max(), flush=True)
    assert sd.max() <= 1e-3
    assert update_check(np64(job.S), S0, st.S, g["S_dot"], pb.lr_S).max() <= 1.0


def test_arm_two_trajectories_product(orc):
    """Two trajectories of the arm (N = 70, 6 windows of 50 steps) combined
    as a product (App. A-B), so every trajectory's terms enter with weight
    1: gradients at their bars.  (With the mixture, a particle whose two
    window log-likelihood sums nearly tie has non-saturated weights w =
    softmax(l) with dw/dl = w (1 - w); FP32 likelihoods within a thousandth
    of their bar then move w, and with it g_obs and S_dot, by up to a few
    tenths of a percent, so the mixture's weights are checked against the
    bar their likelihoods imply and the gradients here.)"""
    pb, obs, st, job, b = make_case(orc, "c4", perturb_S=0.005, lam=True, N=70, K=2, T=300, n_s=6,
                                    combine=synth.COMBINE_PROD)
    L.sim_batch_adjoint(b)
    ref = orc.gradient(pb, obs, st, per_unit=True)
    check_grads(pb, job, ref, st.S)
    assert np.all(np64(job.flags) == 0)


def test_batch_matches_single_jobs_bitwise(orc):
    """Two different problems in one batch give bitwise the results each
    gives alone (fixed-order per-job reductions)."""
    cases = [make_case(orc, "c2", perturb_S=0.01, lam=True, N=70, K=3),
             make_case(orc, "c1", perturb_S=0.01, lam=True, N=40),
             make_case(orc, "c3", perturb_S=0.01, lam=True, N=33, K=2, T=100, n_s=2),
             make_case(orc, "rigid2", perturb_S=0.01, lam=True, N=50, K=2, T=80, n_s=2)]
    solo = []
    for pb, obs, st, job, b in cases:
        L.csvgd_iteration(b, 1)
        solo.append([np64(t) for t in (job.theta, job.S, job.logp, job.g_obs, job.phi, job.bandwidth)])
    fresh = [L.Job(pb, obs, theta=pb.particles, S=st.S) for pb, obs, st, _, _ in cases]
    for (pb, obs, st, job, b), f in zip(cases, fresh):
        f.lam_def.copy_(torch.as_tensor(st.lam_def, dtype=torch.float32))
    bb = L.Batch(fresh)
    L.csvgd_iteration(bb, 1)
    for s, f in zip(solo, fresh):
        for a, t in zip(s, (f.theta, f.S, f.logp, f.g_obs, f.phi, f.bandwidth)):
            np.testing.assert_array_equal(a, np64(t))


def test_arm_structures_share_a_launch_bitwise(orc):
    """Arm jobs of one shape share their window-kernel launches; a table
    with the Panda structure and one off it in the same launch each take
    their own compiled variant (chosen per block) and give bitwise their
    solo results."""
    print_case("batch-structures")
    cases = [make_case(orc, "c4", perturb_S=0.01, lam=True, N=40, T=100, n_s=2),
             make_case(orc, "c4", perturb_S=0.01, lam=True, N=40, T=100, n_s=2, generic_dh=True),
             make_case(orc, "box2", perturb_S=0.01, lam=True, N=24, T=96, n_s=2, generic_dh=True)]
    solo = []
    for pb, obs, st, job, b in cases:
        L.csvgd_iteration(b, 1)
        solo.append([np64(t) for t in (job.theta, job.S, job.logp, job.g_obs, job.g_con, job.phi)])
    fresh = [L.Job(pb, obs, theta=pb.particles, S=st.S) for pb, obs, st, _, _ in cases]
    for (pb, obs, st, job, b), f in zip(cases, fresh):
        f.lam_def.copy_(torch.as_tensor(st.lam_def, dtype=torch.float32))
    bb = L.Batch(fresh)
    L.csvgd_iteration(bb, 1)
    for s, f in zip(solo, fresh):
        for a, t in zip(s, (f.theta, f.S, f.logp, f.g_obs, f.g_con, f.phi)):
            np.testing.assert_array_equal(a, np64(t))
    # (the second c4 table is the first moved off the Panda structure)
    assert not np.array_equal(solo[0][3], solo[1][3])


def test_batch_of_unlike_sizes_matches_single_jobs_bitwise(orc):
    """A job small enough for the two-lanes-per-unit adjoint shares a batch
    with one too large for it: each still takes its own launch shape and
    gives bitwise its solo results."""
    print_case("batch-sizes")
    cases = [make_case(orc, "c2", perturb_S=0.01, lam=True, N=1024, K=8),
             make_case(orc, "c2", perturb_S=0.01, lam=True, N=70, K=3),
             make_case(orc, "c3", perturb_S=0.01, lam=True, N=40, K=2, T=100, n_s=2)]
    solo = []
    for pb, obs, st, job, b in cases:
        L.csvgd_iteration(b, 1)
        solo.append([np64(t) for t in (job.theta, job.S, job.logp, job.g_obs, job.g_con, job.phi)])
    fresh = [L.Job(pb, obs, theta=pb.particles, S=st.S) for pb, obs, st, _, _ in cases]
    for (pb, obs, st, job, b), f in zip(cases, fresh):
        f.lam_def.copy_(torch.as_tensor(st.lam_def, dtype=torch.float32))
    bb = L.Batch(fresh)
    L.csvgd_iteration(bb, 1)
    for s, f in zip(solo, fresh):
        for a, t in zip(s, (f.theta, f.S, f.logp, f.g_obs, f.g_con, f.phi)):
            np.testing.assert_array_equal(a, np64(t))


def test_repeatable_bitwise(orc):
    outs = []
    for _ in range(2):
        pb, obs, st, job, b = make_case(orc, "c2", perturb_S=0.01, lam=True, N=70, K=3)
        for it in range(1, 4):
            L.csvgd_iteration(b, it)
        outs.append([np64(t) for t in (job.theta, job.S, job.lam_def, job.adam_v)])
    for a, c in zip(*outs):
        np.testing.assert_array_equal(a, c)


@pytest.mark.parametrize("cfg,over", [("c2", dict(N=70, K=3)), ("c4", dict(N=40, T=300, n_s=6))])
def test_timed_repeated_launches_leave_results_bitwise(orc, cfg, over):
    """With kernel timing on, each timed call launches its window kernels
    several times back to back; they rewrite the same outputs from the same
    inputs, so the iteration's results are bitwise those of an untimed
    run, and every recorded time is positive."""
    print_case("timing repeats", cfg, over)
    outs = []
    for reps in (0, 4):
        pb, obs, st, job, b = make_case(orc, cfg, perturb_S=0.01, lam=True, **over)
        if reps:
            L.timing_enable(True, reps=reps)
        try:
            for it in range(1, 3):
                L.loglik_multishoot(b)
                L.csvgd_iteration(b, it)
            torch.cuda.synchronize()
            if reps:
                kt = L.timing_read()
                assert len(kt) == 4 and np.all(kt > 0)
        finally:
            L.timing_enable(False)
        outs.append([np64(t) for t in (job.theta, job.S, job.logp, job.g_obs, job.g_con, job.lam_def)])
    for a, c in zip(*outs):
        np.testing.assert_array_equal(a, c)


def test_nonfinite_flags(orc):
    """A NaN parameter and an exploding time step are flagged, not errors."""
    pb, obs, st, job, b = make_case(orc, "c2", N=70, K=1, T=40, n_s=2)
    th = np64(job.theta)
    th[5, 0] = np.nan
    set_tensor(job.theta, th)
    L.sim_batch_adjoint(b)
    fl = np64(job.flags).astype(int)
    assert fl[5] & 3
    assert np.all(fl[np.arange(70) != 5] == 0)
    pb2 = f32_problem(synth.make_problem("c2", N=64, K=1, T=40, n_s=1, dt=50.0))
    job2 = L.Job(pb2, obs, theta=pb2.particles)
    b2 = L.Batch([job2])
    L.loglik_multishoot(b2)
    assert np.any(np64(job2.flags).astype(int) & 1)


def test_c1_hundred_iterations(orc):
    """Headline pendulum problem: 100 CSVGD iterations (Adam) on both sides;
    the particle set's mean and covariance agree within 1e-3 relative
    (componentwise for the mean, Frobenius for the covariance)."""
    pb, obs, st, job, b = make_case(orc, "c1")
    for it in range(1, 101):
        L.csvgd_iteration(b, it)
        orc.csvgd_iteration(pb, obs, st, it, optimizer=1)
    th = np64(job.theta)
    mu, mu_r = th.mean(0), st.theta.mean(0)
    assert np.all(np.abs(mu - mu_r) <= 1e-3 * np.abs(mu_r))
    cov, cov_r = np.cov(th.T), np.cov(st.theta.T)
    rel = np.linalg.norm(cov - cov_r) / np.linalg.norm(cov_r)
    print("mean %.2e covariance %.2e" % ((np.abs(mu - mu_r) / np.abs(mu_r)).max(), rel), flush=True)
    assert rel <= 1e-3


@pytest.mark.parametrize("cfg,over,iters", [("c2", dict(N=64, K=2, T=200, n_s=5), 100),
                                            ("rigid2", dict(N=64, K=2, T=200, n_s=5), 100),
                                            ("c4", dict(N=64, T=300, n_s=6), 100),
                                            ("c3", dict(N=64, K=2, T=200, n_s=4), 50)])
def test_posterior_after_many_iterations(orc, cfg, over, iters):
    """The other families' particle sets after many CSVGD iterations (Adam)
    on both sides, from identical inputs: mean (componentwise) and
    covariance (Frobenius) within 1e-3 relative of the oracle's.  The
    5-link chain under the paper's soft limits stops at 50 iterations: on
    this shape its particles then approach masses and lengths where the
    simulation fails, and which particle leaves the ensemble first is
    decided by rounding."""
    print_case("posterior", cfg, over, iters)
    pb, obs, st, job, b = make_case(orc, cfg, **over)
    for it in range(1, iters + 1):
        L.csvgd_iteration(b, it)
        orc.csvgd_iteration(pb, obs, st, it, optimizer=1)
    th = np64(job.theta)
    mu, mu_r = th.mean(0), st.theta.mean(0)
    cov, cov_r = np.cov(th.T), np.cov(st.theta.T)
    mrel = (np.abs(mu - mu_r) / np.abs(mu_r)).max()
    crel = np.linalg.norm(cov - cov_r) / np.linalg.norm(cov_r)
    print("mean %.2e covariance %.2e" % (mrel, crel), flush=True)
    assert mrel <= 1e-3 and crel <= 1e-3


def test_graph_replays_match_eager(orc):
    """An iteration captured once into a HIP graph and replayed several times
    (with eager work and synchronisation between replays) gives bitwise the
    state of the same number of eager iterations, after every replay."""
    from paper_2109_08815_amd import driver

    pb, obs, st, job_a, _ = make_case(orc, "c2", perturb_S=0.01, lam=True, N=70, K=3)
    job_b = L.Job(pb, obs, theta=pb.particles, S=st.S)
    for j in (job_a, job_b):
        j.lam_def.copy_(torch.as_tensor(st.lam_def, dtype=torch.float32))
    eager = driver.CSVGD([job_a])
    graph = driver.CSVGD([job_b])
    graph.capture(1)
    for rep in range(4):
        eager.step()
        graph.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        for name in ("theta", "S", "lam_def", "lam_lim", "adam_m", "adam_v", "phi", "g_obs", "bandwidth", "iter_dev"):
            np.testing.assert_array_equal(np64(getattr(job_a, name)), np64(getattr(job_b, name)), err_msg=name)
        assert np.isfinite(junk.item())
    assert int(np64(job_b.iter_dev)[0]) == 4


@pytest.mark.parametrize("cfg,over", [("c2", dict(N=70, K=3)), ("c3", dict(N=300, K=2, T=100, n_s=2)),
                                      ("c4", dict(N=300, T=300, n_s=6))])
def test_overlapped_bandwidth_matches_serial_iterations(orc, cfg, over):
    """The bandwidth on a second stream, concurrent with the adjoint, gives
    bitwise the serial iteration's state, with plain launches and in a
    replayed graph (the second case takes the large-problem median path,
    the third its narrow one-wave chain beside the arm's window kernel)."""
    from paper_2109_08815_amd import driver

    print_case("overlap", cfg, over)
    pb, obs, st, job_a, _ = make_case(orc, cfg, perturb_S=0.01, lam=True, **over)
    jobs = [job_a] + [L.Job(pb, obs, theta=pb.particles, S=st.S) for _ in range(2)]
    for j in jobs[1:]:
        j.lam_def.copy_(torch.as_tensor(st.lam_def, dtype=torch.float32))
    serial = driver.CSVGD([jobs[0]])
    over_plain = driver.CSVGD([jobs[1]], overlap=True)
    over_graph = driver.CSVGD([jobs[2]], overlap=True)
    over_graph.capture(2)
    for rep in range(3):
        for _ in range(2):
            serial.step()
            over_plain.step()
        over_graph.replay()
        torch.cuda.synchronize()
        for name in ("theta", "S", "lam_def", "adam_v", "phi", "g_obs", "bandwidth", "iter_dev"):
            ref = np64(getattr(jobs[0], name))
            np.testing.assert_array_equal(ref, np64(getattr(jobs[1], name)), err_msg=name)
            np.testing.assert_array_equal(ref, np64(getattr(jobs[2], name)), err_msg=name)


def test_autograd_function_matches_oracle(orc):
    """Backward of the autograd wrapper = oracle gradients of
    sum_i log p_i - sum b * g_def (b random, c = 0)."""
    from paper_2109_08815_amd.autograd import MultiShootingLikelihood

    pb, obs, st, job, b = make_case(orc, "c2", perturb_S=0.01, N=70, K=3, c=0.0)
    rng = np.random.default_rng(3)
    bw = r32(rng.uniform(0.5, 2.0, (pb.N, pb.K, pb.n_s - 1)))
    mod = MultiShootingLikelihood(pb, obs, pb.particles, st.S)
    th = torch.tensor(pb.particles, dtype=torch.float32, device="cuda", requires_grad=True)
    S = torch.tensor(st.S, dtype=torch.float32, device="cuda", requires_grad=True)
    logp, gdef = mod(th, S)
    loss = logp.sum() - (torch.as_tensor(bw, device="cuda") * gdef).sum()
    loss.backward()
    st_b = orc.State(pb, pb.particles, st.S, lam_def=bw)
    ref = orc.gradient(pb, obs, st_b, per_unit=True)
    np.testing.assert_allclose(np64(logp), ref["logp"], rtol=1e-4)
    # the combined gradient d(log p - sum b g_def)/d theta: each channel
    # within its own bar (tests/parity.py), so their difference within the sum
    bar = grad_bar(ref, "obs")[0] + grad_bar(ref, "con", pb, st.S)[0]
    gt = ref["g_obs"] - ref["g_con"]
    assert np.all(np.linalg.norm(np64(th.grad) - gt, axis=1) <= bar)
    assert normwise(np64(S.grad), ref["S_dot"]).max() <= 1e-3
    # g_theta is the library's own difference of its two channels
    np.testing.assert_array_equal(np64(mod.job.g_theta), np64(mod.job.g_obs) - np64(mod.job.g_con))


@pytest.mark.parametrize("cfg,over", [("c1", dict(N=20, K=2, T=60, n_s=3)), ("c2", dict(N=33, K=2, T=80, n_s=2)),
                                      ("rigid2", dict(N=20, K=2, T=60, n_s=3)), ("c3", dict(N=20, K=2, T=60, n_s=3)),
                                      ("c4", dict(N=20, K=1, T=60, n_s=2)), ("box1", dict(N=12, K=1, T=48, n_s=2)),
                                      ("box2", dict(N=12, K=2, T=48, n_s=2))])
def test_observed_quantities_match_oracle(orc, cfg, over):
    """traj_obs (f_obs of every visited state, which set-up uses to
    synthesise observed trajectories) against the oracle's observation model
    on its own rollout, within what the state tolerance permits."""
    pb, obs, st, job, b = make_case(orc, cfg, perturb_S=0.005, with_traj_obs=True, **over)
    L.sim_batch_forward(b)
    ref = orc.forward(pb, obs, st, traj=True)
    tr = ref["traj"]
    x_ref = np.stack([np.stack([orc.observe(pb, pb.particles[i], tr[i, k]) for k in range(pb.K)])
                      for i in range(pb.N)])
    ratio = observed_err_ratio(pb, np64(job.traj_obs), x_ref, tr)
    print("traj_obs worst ratio to its bar %.3g" % ratio.max(), flush=True)
    assert ratio.max() <= 1.0


ARM_CASES = [
    dict(N=70, K=1, T=100, n_s=2),      # two windows of 50 steps at dt = 1/240
    dict(N=33, K=2, T=60, n_s=3),       # two trajectories, short windows (whole window in LDS)
    dict(N=24, K=2, T=60, n_s=3, lik=synth.LIK_DEFECT),
    dict(N=20, K=2, T=60, n_s=2, combine=synth.COMBINE_PROD),
    dict(N=40, K=1, T=100, n_s=2, generic_dh=True),  # a table off the Panda structure: the generic kernels
]


@pytest.mark.parametrize("over", ARM_CASES)
def test_arm_forward_states_and_loglik(orc, over):
    pb, obs, st, job, b = make_case(orc, "c4", perturb_S=0.005, lam=True, with_traj=True, **over)
    L.loglik_multishoot(b)
    L.sim_batch_forward(b)
    ref = orc.forward(pb, obs, st, traj=True)
    check_states(pb, np64(job.traj), ref["traj"])
    tol = ll_tolerance(pb, obs, ref["traj"], ref["ll_win"])
    d = np.abs(np64(job.ll_win) - ref["ll_win"])
    assert np.all(d <= tol), "ll_win worst ratio %.3g" % (d / tol).max()


@pytest.mark.parametrize("over", ARM_CASES)
def test_arm_adjoint_gradients(orc, over):
    pb, obs, st, job, b = make_case(orc, "c4", perturb_S=0.005, lam=True, **over)
    L.sim_batch_adjoint(b)
    ref = orc.gradient(pb, obs, st, per_unit=True)
    check_grads(pb, job, ref, st.S)
    assert np.all(np64(job.flags) == 0)


BOX_CASES = [
    dict(N=70, K=1, T=96, n_s=2),       # two windows of 48 steps at dt = 1/240
    dict(N=33, K=2, T=60, n_s=3),
    dict(N=24, K=1, T=60, n_s=3, lik=synth.LIK_DEFECT),
    dict(N=20, K=1, T=96, n_s=2, generic_dh=True),
]


def box_ll_tolerance(orc, pb, obs, traj_ref, ll_ref):
    """The window log-likelihood error the state tolerance implies for the
    box-frame observation: each observed point moves by at most the sum
    over the 9 joints of |dq| times its distance from the joint (< 2.5 m),
    with |dq| <= 1e-4 max|x| of the window, plus FP32 rounding of the
    point itself."""
    N, K = traj_ref.shape[:2]
    tr = traj_ref.reshape(N, K, pb.n_s, pb.h, pb.d_s)
    scale = np.maximum(np.abs(tr).max(axis=(3, 4)), 1e-6)
    per = np.zeros((N, K, pb.n_s))
    for i in range(N):
        for k in range(K):
            x = orc.observe(pb, pb.particles[i], traj_ref[i, k])
            r = np.abs((obs[k] - x) * pb.w_x) * pb.w_x
            dx = 9 * 2.5 * 1e-4 * scale[i, k][:, None] + 1e-6 * np.abs(x).reshape(pb.n_s, pb.h, -1).max(axis=(1, 2))[:, None]
            per[i, k] = (r.reshape(pb.n_s, pb.h, -1).sum(axis=1) * dx).sum(axis=1)
    return per + 1e-9 * np.abs(ll_ref)


@pytest.mark.parametrize("cfg", ["box1", "box2"])
@pytest.mark.parametrize("over", BOX_CASES)
def test_box_universal_joint_forward_and_loglik(orc, cfg, over):
    """The arm with the box on a universal joint (phase I: the box's
    parameters; phase II: two weights in the box), box-frame observation:
    window states, log-likelihoods and defects."""
    pb, obs, st, job, b = make_case(orc, cfg, perturb_S=0.005, lam=True, with_traj=True, **over)
    L.loglik_multishoot(b)
    L.sim_batch_forward(b)
    ref = orc.forward(pb, obs, st, traj=True)
    check_states(pb, np64(job.traj), ref["traj"])
    tol = box_ll_tolerance(orc, pb, obs, ref["traj"], ref["ll_win"])
    d = np.abs(np64(job.ll_win) - ref["ll_win"])
    assert np.all(d <= tol), "ll_win worst ratio %.3g" % (d / tol).max()


@pytest.mark.parametrize("cfg", ["box1", "box2"])
@pytest.mark.parametrize("over", BOX_CASES)
def test_box_universal_joint_adjoint_gradients(orc, cfg, over):
    pb, obs, st, job, b = make_case(orc, cfg, perturb_S=0.005, lam=True, **over)
    L.sim_batch_adjoint(b)
    ref = orc.gradient(pb, obs, st, per_unit=True)
    check_grads(pb, job, ref, st.S)
    assert np.all(np64(job.flags) == 0)


@pytest.mark.parametrize("cfg,over", [("c2", dict(N=16, K=2, T=40, n_s=2)), ("c3", dict(N=16, K=1, T=60, n_s=3)),
                                      ("c4", dict(N=8, T=60, n_s=2)), ("c4", dict(N=8, T=60, n_s=2, generic_dh=True)),
                                      ("c2", dict(N=16, K=2, T=60, n_s=3, lik=synth.LIK_DEFECT)),
                                      ("c4", dict(N=8, K=2, T=60, n_s=2, lik=synth.LIK_DEFECT)),
                                      ("rigid2", dict(N=16, K=2, T=40, n_s=2)),
                                      ("box1", dict(N=8, T=48, n_s=2)), ("box2", dict(N=8, T=48, n_s=2))])
def test_adjoint_matches_central_differences_of_gpu_likelihood(orc, cfg, over):
    """The reverse-mode gradients against central differences of the GPU's
    own forward (FP32 states, FP64 sums), along a random direction in theta
    per particle: d log p / d theta (g_obs) and d Phi / d theta (g_con) with
    Phi = sum_j lam_j g_j + (c / 2) g_j^2.  FP32 rounding noise limits the
    differences from below and curvature (Phi is quartic in the defect) from
    above, so the best of five step sizes must agree to 5e-3 of |g| |v|."""
    print_case("fd", cfg, over)
    pb, obs, st, job, b = make_case(orc, cfg, perturb_S=0.01, lam=True, **over)
    L.sim_batch_adjoint(b)
    g_obs, g_con = np64(job.g_obs), np64(job.g_con)
    rng = np.random.default_rng(3)
    v = rng.normal(size=g_obs.shape) * (pb.hi - pb.lo)
    th0 = np64(job.theta)
    lam = np64(job.lam_def)

    def evaluate(theta):
        set_tensor(job.theta, theta)
        L.loglik_multishoot(b)
        gd = np64(job.gdef)
        phi_c = (lam * gd + 0.5 * pb.c * gd * gd).reshape(gd.shape[0], -1).sum(axis=1)
        if pb.lik == synth.LIK_DEFECT:  # no constraints: the defects are inside log p
            phi_c = np.zeros_like(phi_c)
        return np64(job.logp), phi_c

    best_o = np.full(pb.N, np.inf)
    best_c = np.full(pb.N, np.inf)
    want_o = (g_obs * v).sum(axis=1)
    want_c = (g_con * v).sum(axis=1)
    # error of the directional derivative relative to |g| |v| (independent of
    # how the random direction happens to align with the gradient)
    norm_o = np.maximum(np.linalg.norm(g_obs, axis=1) * np.linalg.norm(v, axis=1), 1e-12)
    norm_c = np.maximum(np.linalg.norm(g_con, axis=1) * np.linalg.norm(v, axis=1), 1e-12)
    for rel in (1e-2, 3e-3, 1e-3, 3e-4, 1e-4):
        lp_p, ph_p = evaluate(r32(th0 + rel * v))
        lp_m, ph_m = evaluate(r32(th0 - rel * v))
        step = (r32(th0 + rel * v) - r32(th0 - rel * v))  # the step actually taken in FP32
        scale = (step * v).sum(axis=1) / (v * v).sum(axis=1)  # = 2 rel up to rounding
        fd_o = (lp_p - lp_m) / scale
        fd_c = (ph_p - ph_m) / scale
        best_o = np.minimum(best_o, np.abs(fd_o - want_o) / norm_o)
        best_c = np.minimum(best_c, np.abs(fd_c - want_c) / norm_c)
    set_tensor(job.theta, th0)
    assert best_o.max() <= 5e-3, best_o
    assert best_c.max() <= 5e-3, best_c
