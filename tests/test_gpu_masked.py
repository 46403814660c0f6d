"""Particles whose simulation failed leave the ensemble (HIP path through the
C ABI against the FP64 oracle).

A particle with flag bit 0 or 1 (non-finite state, likelihood or gradient)
is left out of the phi sums, whose mean runs over the N' others, gets
phi = 0 and keeps its variables in the step, which sets bit 3; particles
with bit 3 are left out of the bandwidth median as well.  The oracle's
masked bandwidth and phi are pinned against brute force and the unmasked
functions on the live subset (tests/test_oracle_pins.py).
"""
import numpy as np
import pytest
import torch

from paper_2109_08815_amd import lib as L
from paper_2109_08815_amd import synth
from tests.helpers import f32_problem, print_case, r32, requires_gpu
from tests.parity import phi_scale, update_check

pytestmark = [pytest.mark.gpu, requires_gpu]

STATE, GRAD, FROZEN = L.PDS_FLAG_STATE, L.PDS_FLAG_GRAD, L.PDS_FLAG_FROZEN


def np64(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def set_tensor(t, a):
    t.copy_(torch.as_tensor(np.asarray(a), dtype=t.dtype))


def flagged_case(N, cfg, n_frozen, n_grad, n_state, seed):
    """Particles in the limits box with large scores; n_frozen particles
    carry bits 3 and 1 with NaN parameters and scores, n_grad bit 1 with a
    NaN score, n_state bit 0 with an infinite score."""
    pb = f32_problem(synth.make_problem(cfg, N=N, K=1, T=40, n_s=2))
    rng = np.random.default_rng(seed)
    theta = r32(pb.lo + rng.uniform(size=(N, pb.M)) * (pb.hi - pb.lo))
    G = rng.normal(scale=1e4, size=(N, pb.M))
    perm = rng.permutation(N)
    fz, gr, sv = np.split(perm[: n_frozen + n_grad + n_state], [n_frozen, n_frozen + n_grad])
    flags = np.zeros(N, dtype=np.int64)
    flags[fz] = FROZEN | GRAD
    flags[gr] = GRAD
    flags[sv] = STATE
    th_gpu = theta.copy()
    th_gpu[fz] = np.nan
    G[fz] = np.nan
    G[gr] = np.nan
    G[sv] = np.inf
    job = L.Job(pb, np.zeros((pb.K, pb.T, pb.d_x)), theta=th_gpu)
    set_tensor(job.g_obs, G)
    set_tensor(job.flags, flags)
    job.n_masked.fill_(-1)
    return pb, theta, th_gpu, G, flags, job


def check_phi(orc, pb, th, G, flags, job, sel=None):
    live_bw = (flags & FROZEN) == 0
    live = (flags & (STATE | GRAD | FROZEN)) == 0
    h_ref, _ = orc.bandwidth(th, pb.rho, live=live_bw)
    h = np64(job.bandwidth)[0]
    print("h %.17g oracle %.17g, ensemble %d of %d, phi over %d" % (h, h_ref, live_bw.sum(), len(th), live.sum()),
          flush=True)
    assert abs(h - h_ref) <= 1e-15 * h_ref
    ph = np64(job.phi)
    assert np.all(ph[~live] == 0.0)
    assert int(np64(job.n_masked)[0]) == int((~live).sum())
    idx = np.flatnonzero(live)
    if len(idx) == 0:
        return
    rows = idx if sel is None else idx[sel]
    ref = orc.phi(th, G, pb.rho, h_ref, sel=rows.astype(np.int32), live=live)
    scale = phi_scale(th[idx], r32(G[idx]), pb.rho, h_ref, sel=None if sel is None else sel)
    err = np.abs(ph[rows] - ref)
    print("phi worst err / scale %.2e" % (err / np.maximum(scale, 1e-300)).max(), flush=True)
    assert np.all(np.isfinite(ph))
    assert np.all(err <= 1e-4 * scale + 1e-30)


@pytest.mark.parametrize("N,nf,ng,ns", [(2, 1, 0, 0), (5, 0, 1, 1), (64, 3, 2, 1), (300, 7, 5, 4), (700, 0, 0, 9),
                                        (300, 298, 0, 0), (300, 0, 299, 0), (64, 64, 0, 0)])
def test_phi_leaves_out_flagged_particles(orc, N, nf, ng, ns):
    """All pairs enumerated (N(N-1)/2 <= 32768), one-kernel phi."""
    print_case("masked-phi", N, nf, ng, ns)
    pb, th, th_gpu, G, flags, job = flagged_case(N, "c2", nf, ng, ns, seed=N + nf)
    L.svgd_phi(L.Batch([job]))
    check_phi(orc, pb, th, G, flags, job)
    assert np.all(np64(job.flags).astype(np.int64) == flags)


@pytest.mark.parametrize("nf,ng,ns", [(200, 30, 10), (2046, 0, 0), (2047, 0, 0), (0, 2048, 0), (1900, 0, 0)])
def test_sampled_median_leaves_out_frozen_particles(orc, nf, ng, ns):
    """2048 particles: the sampled bracket, the count pass over all pairs
    and the final selection, with a small ensemble whose pairs the sample
    may miss altogether (2 particles: one pair in 2 million)."""
    print_case("masked-median", 2048, nf, ng, ns)
    pb, th, th_gpu, G, flags, job = flagged_case(2048, "c2", nf, ng, ns, seed=nf + 3 * ng + 7 * ns)
    L.svgd_phi(L.Batch([job]))
    check_phi(orc, pb, th, G, flags, job, sel=None)


@pytest.mark.parametrize("shift", [-20000, 20000])
def test_masked_median_when_bracket_misses(orc, shift):
    """The recovery pass (pairs recomputed from theta) skips frozen pairs."""
    print_case("masked-median-miss", shift)
    pb, th, th_gpu, G, flags, job = flagged_case(2048, "c2", 300, 0, 0, seed=11)
    L.lib().pds_test_median_shift(shift)
    try:
        L.svgd_phi(L.Batch([job]))
    finally:
        L.lib().pds_test_median_shift(0)
    check_phi(orc, pb, th, G, flags, job)


@pytest.mark.parametrize("N,M", [(4500, 4), (4200, 10)])
def test_partial_phi_leaves_out_flagged_particles(orc, N, M):
    """Above 4096 particles: partial sums per chunk of 32 rows and their
    reduction; whole chunks masked as well as single rows."""
    print_case("masked-phi-partial", N, M)
    pb, th, th_gpu, G, flags, job = flagged_case(N, "c2" if M == 4 else "c3", 50, 40, 30, seed=N)
    for j in range(64, 96):  # chunk 2 entirely
        flags[j] |= GRAD
        G[j] = np.nan
    set_tensor(job.flags, flags)
    set_tensor(job.g_obs, G)
    L.svgd_phi(L.Batch([job]))
    rng = np.random.default_rng(N + M)
    n_live = int(((flags & (STATE | GRAD | FROZEN)) == 0).sum())
    sel = np.sort(rng.choice(n_live, size=48, replace=False))
    check_phi(orc, pb, th, G, flags, job, sel=sel)


def failed_particle_case(orc, cfg, **over):
    """A problem whose particle 5 starts window 2 of trajectory 0 from a NaN
    shooting state; identical inputs on both sides."""
    pb = f32_problem(synth.make_problem(cfg, **over))
    obs = r32(orc.observations(pb))
    S = r32(orc.shooting_init(pb, pb.particles))
    rng = np.random.default_rng(3)
    S = r32(synth.perturb(rng, S, 0.01))
    S[5, 0, 1, 2] = np.nan
    lam_def = r32(rng.uniform(0.0, 2.0, (pb.N, pb.K, pb.n_s - 1)))
    st = orc.State(pb, pb.particles, S, lam_def=lam_def)
    job = L.Job(pb, obs, theta=pb.particles, S=S)
    job.lam_def.copy_(torch.as_tensor(lam_def, dtype=torch.float32))
    return pb, obs, st, job


@pytest.mark.parametrize("cfg,over", [("c2", dict(N=70, K=2, T=80, n_s=4)),
                                      ("c4", dict(N=40, K=1, T=120, n_s=4))])
def test_iterations_with_a_failed_particle(orc, cfg, over):
    """Two iterations (SGD) with one particle whose window diverges: it is
    flagged (state, gradient) and frozen on both sides, the bandwidth of
    the first iteration includes it and that of the second does not, and
    every other particle's update matches the oracle's."""
    print_case("failed-particle", cfg, over)
    pb, obs, st, job = failed_particle_case(orc, cfg, **over)
    b = L.Batch([job])
    live = np.arange(pb.N) != 5
    th0 = np64(job.theta)
    S0 = np64(job.S)
    for it in (1, 2):
        thp, Sp = st.theta.copy(), st.S.copy()
        # the bandwidth is exact for the particles it is given: the oracle's
        # median of the GPU's parameters over the particles not yet frozen
        h_ref, _ = orc.bandwidth(np64(job.theta), pb.rho, live=(st.flags & orc.FLAG_FROZEN) == 0)
        L.csvgd_iteration(b, it, L.PDS_OPT_SGD)
        g = orc.csvgd_iteration(pb, obs, st, it, optimizer=0)
        fl = np64(job.flags).astype(np.int64)
        print("iteration", it, "flags of particle 5:", fl[5], "oracle", g["flags"][5], flush=True)
        assert fl[5] == g["flags"][5] == STATE | GRAD | FROZEN
        assert np.all(fl[live] & (STATE | GRAD | FROZEN) == 0)
        assert int(np64(job.n_masked)[0]) == g["n_masked"] == 1
        assert abs(np64(job.bandwidth)[0] - h_ref) <= 1e-15 * h_ref
        if it == 1:
            assert h_ref == g["bandwidth"]
        th = np64(job.theta)
        np.testing.assert_array_equal(th[5], th0[5])
        np.testing.assert_array_equal(np64(job.S)[5], S0[5])
        assert np.all(np64(job.phi)[5] == 0.0)
        assert np.all(np.isfinite(th))
        assert update_check(th[live], thp[live], st.theta[live]).max() <= 1.0
        Sg = np64(job.S).reshape(st.S.shape)
        assert update_check(Sg[live], Sp[live], st.S[live], g["S_dot"][live], pb.lr_S).max() <= 1.0


def test_overlapped_bandwidth_with_a_failed_particle_matches_serial(orc):
    """The overlapped bandwidth reads flag bit 3 only, which the adjoint
    never writes: the same state bitwise as serial iterations, plain and
    in a replayed graph."""
    from paper_2109_08815_amd import driver

    print_case("failed-particle-overlap")
    pb, obs, st, _ = failed_particle_case(orc, "c2", N=300, K=2, T=80, n_s=4)
    jobs = [L.Job(pb, obs, theta=pb.particles, S=st.S) for _ in range(3)]
    for j in jobs:
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
        for name in ("theta", "S", "lam_def", "adam_v", "phi", "g_obs", "bandwidth", "flags", "n_masked"):
            ref = np64(getattr(jobs[0], name))
            np.testing.assert_array_equal(ref, np64(getattr(jobs[1], name)), err_msg=name)
            np.testing.assert_array_equal(ref, np64(getattr(jobs[2], name)), err_msg=name)
    assert np.all(np.isfinite(np64(jobs[0].theta)))
