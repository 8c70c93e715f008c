"""GPU tests of the served form: requests of different sizes arrive while
others run, are admitted as the device budget frees up, share window
launches, and each result is bit-identical to the same simulation run alone
(and, for the small ones, to the oracle)."""
import sys
import time

import numpy as np
import pytest

from paper_1610_02258_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rdx():
    from paper_1610_02258_amd import rdx as R
    R.lib()
    return R


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _requests(n, seed, t_lo=150, t_hi=15000, t_end=5e-3):
    reqs = I.request_stream(n_requests=n, rate_per_s=1e4, seed=seed, t_lo=t_lo, t_hi=t_hi, t_end=t_end)
    # uneven horizons as well as uneven sizes
    out = []
    for j, (arrival, w) in enumerate(reqs):
        w.t_end = t_end * (1.0 + 0.5 * (j % 3))
        out.append((arrival, w))
    return out


def _solo(rdx, w):
    s = rdx.Sim(w.mesh.as_dict(), w.model.as_dict(), w.seed)
    s.set_counts(w.counts)
    s.run(w.t_end)
    c, st = s.get_counts(), s.stats()
    s.close()
    return c, st


def test_results_equal_alone_and_in_the_mix(rdx, oracle_lib):
    reqs = _requests(14, seed=21)
    sizes = [w.mesh.n_tets for _, w in reqs]
    _say(f"case: server, 14 requests, T = {sizes}, 4 MiB budget")
    srv = rdx.Server(reqs[0][1].model.as_dict(), hbm_budget_bytes=4 << 20, tick_windows=4)
    tickets = []
    for arrival, w in reqs:
        tickets.append(srv.submit(w.mesh.as_dict(), w.model.as_dict(), w.seed, w.counts, w.t_end))
        time.sleep(0.0005)
    results = [srv.wait(tk, timeout_s=120.0) for tk in tickets]
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["queued"] == 0
    # the budget cannot hold every request at once: some waited for others
    assert sum(sizes) > st["capacity_tets"]
    admits = sorted(info["t_admit"] for _, info in results)
    dones = sorted(info["t_done"] for _, info in results)
    assert admits[-1] > dones[0]
    for (arrival, w), (counts, info) in zip(reqs, results):
        assert info["state"] == "done"
        ref_c, ref_st = _solo(rdx, w)
        np.testing.assert_array_equal(counts, ref_c)
        assert info["stats"] == ref_st
        assert info["t_submit"] <= info["t_admit"] <= info["t_done"]
    # the two smallest against the oracle too
    for j in np.argsort(sizes)[:2]:
        w = reqs[j][1]
        ref = oracle_lib.Instance(w.mesh.as_dict(), w.model.as_dict(), w.seed)
        ref.reset(w.counts)
        ref.run(w.t_end)
        np.testing.assert_array_equal(results[j][0], ref.counts)
        assert results[j][1]["stats"].ssa_events == ref.tallies.ssa_events
    assert st["latency_p50_s"] > 0 and st["latency_p99_s"] >= st["latency_p50_s"]
    # device time of the ticks and the worker's own time are both inside the uptime
    assert 0 < st["busy_s"] <= st["uptime_s"] and 0 < st["worker_s"] <= st["uptime_s"]
    assert st["ticks"] > 0
    srv.close()


def test_zero_length_and_back_to_back_requests(rdx):
    """A request with t_end = 0 returns its initial counts after no window;
    requests submitted while ticks are in flight, finishing on successive
    ticks, each equal the same simulation alone."""
    reqs = _requests(6, seed=13, t_lo=300, t_hi=600)
    model = reqs[0][1].model.as_dict()
    srv = rdx.Server(model, hbm_budget_bytes=64 << 20, tick_windows=3)
    w0 = reqs[0][1]
    tk0 = srv.submit(w0.mesh.as_dict(), model, w0.seed, w0.counts, 0.0)
    tks = []
    for j, (_, w) in enumerate(reqs[1:]):
        w.t_end = w.t_end * (1 + 0.37 * j)  # ends spread over several ticks
        tks.append(srv.submit(w.mesh.as_dict(), w.model.as_dict(), w.seed, w.counts, w.t_end))
    c0, info0 = srv.wait(tk0, timeout_s=60.0)
    np.testing.assert_array_equal(c0, w0.counts)
    assert info0["stats"].windows == 0 and info0["state"] == "done"
    for tk, (_, w) in zip(tks, reqs[1:]):
        c, info = srv.wait(tk, timeout_s=60.0)
        ref_c, ref_st = _solo(rdx, w)
        np.testing.assert_array_equal(c, ref_c)
        assert info["stats"] == ref_st
    srv.close()


def test_budget_errors_and_cancel(rdx):
    reqs = _requests(3, seed=5, t_lo=2000, t_hi=3000)
    model = reqs[0][1].model.as_dict()
    srv = rdx.Server(model, hbm_budget_bytes=2 << 20, tick_windows=2)
    big = I.box_mesh(5, 5, 600, 0.5e-6)  # 90,000 tets: more than 2 MiB can ever hold
    with pytest.raises(rdx.RdxError) as e:
        srv.submit(big.as_dict(), model, 1, np.zeros((10, big.n_tets), np.int32), 1e-3)
    assert e.value.status == -7
    with pytest.raises(rdx.RdxError) as e:
        srv.submit(reqs[0][1].mesh.as_dict(), I.model_abc().as_dict(), 1,
                   np.zeros((3, reqs[0][1].mesh.n_tets), np.int32), 1e-3)
    assert e.value.status == -1
    # a long request, cancelled while it runs or waits
    w = reqs[1][1]
    tk = srv.submit(w.mesh.as_dict(), w.model.as_dict(), w.seed, w.counts, 50.0)
    time.sleep(0.05)
    srv.cancel(tk)
    with pytest.raises(rdx.RdxError) as e:
        srv.wait(tk, timeout_s=60.0)
    assert e.value.status == -8
    # the server still serves after the cancellation
    w2 = reqs[2][1]
    tk2 = srv.submit(w2.mesh.as_dict(), w2.model.as_dict(), w2.seed, w2.counts, w2.t_end)
    c2, info2 = srv.wait(tk2, timeout_s=60.0)
    ref_c, _ = _solo(rdx, w2)
    np.testing.assert_array_equal(c2, ref_c)
    st = srv.stats()
    assert st["cancelled"] == 1 and st["completed"] == 1
    srv.close()


def test_destroy_with_work_in_flight(rdx):
    reqs = _requests(4, seed=8, t_lo=500, t_hi=2000)
    srv = rdx.Server(reqs[0][1].model.as_dict(), hbm_budget_bytes=4 << 20)
    for _, w in reqs:
        w.t_end = 5.0
        srv.submit(w.mesh.as_dict(), w.model.as_dict(), w.seed, w.counts, w.t_end)
    time.sleep(0.05)
    t0 = time.time()
    srv.close()  # cancels the queued and running requests and joins the worker
    assert time.time() - t0 < 30.0


def test_random_structure_requests_with_regions(rdx, oracle_lib):
    """Requests sharing a random reaction structure (two regions, homodimers,
    sources, immobile species) with per-request rates, diffusion
    coefficients and meshes, more than the budget holds at once: each result
    equals the oracle run alone."""
    from tests.randmodels import random_counts, random_model
    rng = np.random.default_rng(909)
    S, R = 12, 12
    base = random_model(rng, S, R, 2)
    reqs = []
    for j in range(8):
        dims = tuple(int(v) for v in rng.integers(4, 11, 3))
        mesh = I.box_mesh(*dims, 0.5e-6, jitter=0.1, seed=60 + j)
        mesh.region = rng.integers(0, 2, mesh.n_tets).astype(np.uint8)
        md = dict(base)
        md["kcst"] = base["kcst"] * rng.uniform(0.5, 1.5, base["kcst"].shape)
        md["D"] = base["D"] * rng.uniform(0.5, 1.5, S)
        counts = random_counts(rng, S, mesh.n_tets, mean=4.0)
        reqs.append((mesh, md, 500 + j, counts))
    sizes = [m.n_tets for m, _, _, _ in reqs]
    _say(f"case: server, random S={S} R={R} structure, T = {sizes}, 1 MiB budget")
    srv = rdx.Server(base, hbm_budget_bytes=1 << 20, tick_windows=2)
    t_end = []
    tickets = []
    for mesh, md, seed, counts in reqs:
        ref = oracle_lib.Instance(mesh.as_dict(), md, seed)
        t_end.append(4.5 * ref.tau)
        tickets.append(srv.submit(mesh.as_dict(), md, seed, counts, t_end[-1]))
    st = srv.stats()
    assert sum(sizes) > st["capacity_tets"]
    for (mesh, md, seed, counts), tk, te in zip(reqs, tickets, t_end):
        got, info = srv.wait(tk, timeout_s=120.0)
        ref = oracle_lib.Instance(mesh.as_dict(), md, seed)
        ref.reset(counts)
        ref.run(te)
        np.testing.assert_array_equal(got, ref.counts)
        assert info["stats"].ssa_events == ref.tallies.ssa_events
        assert info["stats"].moves == ref.tallies.moves
        assert info["stats"].face_moves == ref.tallies.face_moves
    srv.close()


def test_benchmarked_request_stream_sampled(rdx, oracle_lib):
    """The head of the served leg's request stream (48 Poisson requests,
    T ~ logU(1296, 2e5), 10-species model, 100 ms each) through a server set
    up as the benchmark's (16 GiB budget, 8 windows per tick); 8 requests
    spread over the size range against the oracle run alone."""
    reqs = I.request_stream(n_requests=48)
    T = np.array([w.mesh.n_tets for _, w in reqs])
    idx = [int(i) for i in np.argsort(T, kind="stable")[::6]][:8]
    _say(f"case: served stream of {len(reqs)} requests, {int(T.sum())} tets, sampled {idx}")
    model = reqs[0][1].model.as_dict()
    srv = rdx.Server(model, hbm_budget_bytes=16 << 30, tick_windows=8)
    tickets = [srv.submit(w.mesh.as_dict(), model, w.seed, w.counts, w.t_end) for _, w in reqs]
    results = [srv.wait(tk, timeout_s=120.0) for tk in tickets]
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    srv.close()
    for i in idx:
        w = reqs[i][1]
        ref = oracle_lib.Instance(w.mesh.as_dict(), model, w.seed)
        ref.reset(w.counts)
        ref.run(w.t_end)
        got, info = results[i]
        assert info["state"] == "done"
        np.testing.assert_array_equal(got, ref.counts, err_msg=f"request {i}")
        assert (info["stats"].ssa_events, info["stats"].moves) == (ref.tallies.ssa_events, ref.tallies.moves)
