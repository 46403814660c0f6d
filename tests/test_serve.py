"""Serving loop: host-side admission logic, the footprint closed form and
the trace (CPU), and bitwise equality of every job's results between the
batched loop and one-job-at-a-time runs (GPU)."""
import numpy as np
import pytest

from paper_2109_08815_amd import lib as L
from paper_2109_08815_amd import serve, synth

from helpers import print_case, requires_gpu

BUFFERS = ("consts", "lo", "hi", "rho", "w_x", "u", "lr_theta", "lr_S", "s0", "obs", "theta", "S", "lam_lim",
           "lam_def", "adam_m", "adam_v", "end_states", "traj", "ll_win", "gdef", "logp", "wk", "g_obs", "g_con",
           "S_dot", "phi", "bandwidth", "flags", "iter_dev", "n_masked", "seed_logp", "seed_gdef")


@pytest.mark.parametrize("config,over", [("c1", dict(K=2, T=1500, n_s=30)), ("c2", {}), ("c2", dict(n_s=1)),
                                         ("c3", dict(N=300, K=3, T=600, n_s=12)), ("c4", dict(N=40)),
                                         ("c3", dict(N=1024, K=2, T=200, n_s=4))])
def test_footprint_is_every_buffer_plus_workspace(config, over):
    pb = synth.make_problem(config, **over)
    job = L.Job(pb, np.zeros((pb.K, pb.T, pb.d_x)), device="cpu", device_iter=True)
    nbytes = sum(getattr(job, n).numel() * getattr(job, n).element_size() for n in BUFFERS
                 if getattr(job, n) is not None)
    ws = L.lib().pds_workspace_size((L.PdsJob * 1)(job.struct()), 1, L.PDS_CALL_ALL)
    assert L.job_footprint(job.struct()) == nbytes + ws
    assert L.job_footprint(L.shape_struct(pb)) == nbytes + ws
    with_traj = L.Job(pb, np.zeros((pb.K, pb.T, pb.d_x)), device="cpu", device_iter=True, with_traj=True)
    assert L.job_footprint(with_traj.struct()) == nbytes + ws + with_traj.traj.numel() * 4


def test_footprint_rejects_invalid_shapes():
    pb = synth.make_problem("c2")
    j = L.shape_struct(pb)
    j.T = pb.T + 1
    with pytest.raises(L.PdsError):
        L.job_footprint(j)


def _spec(i, size):
    return synth.JobSpec(i, "c2", N=size, K=1, T=200, seed=i, iterations=1)


def test_scheduler_fifo_slots_and_budget():
    fp = lambda s: s.N  # noqa: E731  footprint = N bytes
    sch = serve.Scheduler(budget_bytes=100, footprint=fp, max_slots=3)
    for i, n in enumerate([40, 30, 20, 10, 5]):
        sch.arrive(_spec(i, n))
    got = [s.job_id for s in sch.admit()]
    assert got == [0, 1, 2]                      # slot limit
    assert sch.used == 90
    assert sch.admit() == []
    sch.release(_spec(0, 40))
    assert [s.job_id for s in sch.admit()] == [3]  # job 3 fits (10), slots full again
    sch.release(_spec(1, 30))
    sch.release(_spec(2, 20))
    assert [s.job_id for s in sch.admit()] == [4]
    assert sch.used == 15 and not sch.queue


def test_scheduler_head_of_line_waits_and_oversize_is_rejected():
    fp = lambda s: s.N  # noqa: E731
    sch = serve.Scheduler(budget_bytes=100, footprint=fp, max_slots=8)
    for i, n in enumerate([60, 50, 10, 500, 5]):
        sch.arrive(_spec(i, n))
    assert [s.job_id for s in sch.admit()] == [0]  # 50 does not fit; 10 may not overtake it
    sch.release(_spec(0, 60))
    assert [s.job_id for s in sch.admit()] == [1, 2, 4]  # 500 can never fit: rejected, queue moves on
    assert [s.job_id for s in sch.rejected] == [3]


def test_scheduler_rejects_bad_slot_count():
    with pytest.raises(ValueError):
        serve.Scheduler(1, lambda s: 0, max_slots=65)


def test_serving_trace_is_seeded_and_in_range():
    a = synth.serving_trace(200, seed=11, rate=50.0)
    b = synth.serving_trace(200, seed=11, rate=50.0)
    assert a == b
    assert {s.family for s in a} == {"c1", "c2", "c3"}
    assert {s.N for s in a} <= {64, 128, 256, 512, 1024, 2048}
    assert all(1 <= s.K <= 8 and s.T in synth.SERVE_T and s.T % synth.SERVE_H == 0 for s in a)
    gaps = np.diff([0.0] + [s.arrival for s in a])
    assert np.all(gaps >= 0) and abs(gaps.mean() * 50.0 - 1.0) < 0.25
    closed = synth.serving_trace(10, seed=11)
    assert all(s.arrival == 0.0 for s in closed)


@pytest.mark.gpu
@requires_gpu
@pytest.mark.parametrize("graph", [0, 2])
def test_batched_serving_equals_jobs_run_alone(graph):
    """Each job's particles and log-likelihoods after its iterations are
    bitwise the same in the mixed batches as run alone."""
    print_case("serve", graph)
    trace = synth.serving_trace(8, seed=21, iterations=4, rate=400.0, max_log2_n=4)
    eng = serve.Engine(budget_bytes=8 << 30, graph_iters=graph, max_slots=4)
    bat = eng.run_batched(trace)
    seq = eng.run_sequential(trace)
    assert bat["jobs"] == seq["jobs"] == len(trace)
    n, bad = serve.same_results(bat, seq)
    assert n == len(trace) and bad == 0
    for r in bat["records"].values():
        assert np.isfinite(r.theta).all() and r.done >= r.spec.arrival


def test_shape_signature_and_rebind_guard():
    """Jobs of one shape share a signature whatever their buffers; a batch
    refuses to rebind to jobs of other shapes (host logic, CPU buffers)."""
    pb = synth.make_problem("c2", N=64, K=1, T=40, n_s=2)
    obs = np.zeros((pb.K, pb.T, pb.d_x))
    a, b = (L.Job(pb, obs, device="cpu", device_iter=True) for _ in range(2))
    assert L.shape_signature(a.struct()) == L.shape_signature(b.struct())
    pb2 = synth.make_problem("c2", N=65, K=1, T=40, n_s=2)
    c = L.Job(pb2, obs, device="cpu", device_iter=True)
    assert L.shape_signature(c.struct()) != L.shape_signature(a.struct())
    d = L.Job(pb, obs, device="cpu", device_iter=False)
    assert L.shape_signature(d.struct()) != L.shape_signature(a.struct())
    batch = L.Batch([a])
    with pytest.raises(L.PdsError):
        batch.rebind([c])
    with pytest.raises(L.PdsError):
        batch.rebind([a, b])


@pytest.mark.gpu
@requires_gpu
@pytest.mark.skip(reason=serve.GRAPH_CACHE_OFF)
def test_cached_graphs_rebound_to_new_jobs_equal_jobs_run_alone():
    """Jobs of one shape arriving two at a time through two slots: batches
    return to shapes seen before, so cached graphs are rebound to new jobs
    and replayed; every job's results stay bitwise those it gets alone."""
    print_case("serve-graph-cache")
    trace = [synth.JobSpec(i, "c2", N=64, K=1, T=200, seed=100 + i, iterations=6, arrival=0.0) for i in range(6)]
    eng = serve.Engine(budget_bytes=8 << 30, graph_iters=1, max_slots=2, capture_after=1, graph_cache=True)
    bat = eng.run_batched(trace)
    seq = eng.run_sequential(trace)
    assert bat["graph_reuses"] >= 1 and bat["graph_captures"] >= 1
    n, bad = serve.same_results(bat, seq)
    assert n == len(trace) and bad == 0


def test_graph_cache_is_switched_off():
    with pytest.raises(RuntimeError, match="switched off"):
        serve.Engine(graph_iters=1, graph_cache=True)
