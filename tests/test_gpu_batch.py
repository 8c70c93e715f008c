"""GPU parity of the batched form: many independent runs of uneven sizes and
per-run parameters advanced by the same window launches.  Every run must
equal the oracle run alone, bit for bit, whatever the launch shape (plain
launches, captured HIP graphs replayed several times, other grid sizes, the
online tuner)."""
import sys

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


def _small_ensemble(n=7, seed=31, t_lo=150, t_hi=4000, t_end=0.25):
    return I.ensemble_runs(n_runs=n, seed=seed, t_lo=t_lo, t_hi=t_hi, t_end=t_end)


def _refs(O, runs):
    refs = []
    for w in runs:
        r = O.Instance(w.mesh.as_dict(), w.model.as_dict(), w.seed)
        r.reset(w.counts)
        refs.append(r)
    return refs


def _batch(rdx, runs):
    b = rdx.Batch([(w.mesh.as_dict(), w.model.as_dict(), w.seed) for w in runs])
    for i, w in enumerate(runs):
        b.set_counts(i, w.counts)
    return b


def _assert_run(b, i, ref, what):
    got = b.get_counts(i)
    if not np.array_equal(got, ref.counts):
        bad = np.argwhere(got != ref.counts)
        s, t = bad[0]
        raise AssertionError(f"{what} run {i}: {len(bad)} mismatches, first species {s} tet {t}: "
                             f"gpu {got[s, t]} oracle {ref.counts[s, t]}")
    st = b.stats(i)
    assert st.ssa_events == ref.tallies.ssa_events, (what, i)
    assert st.moves == ref.tallies.moves, (what, i)
    assert st.face_moves == ref.tallies.face_moves, (what, i)
    assert st.voxel_steps == ref.tallies.voxel_steps, (what, i)
    assert st.window_index == ref.window and st.t == ref.t, (what, i)


@pytest.mark.parametrize("shape", [dict(fast_grid_div=1, graph_windows=1, event_group=1),
                                   dict(fast_grid_div=2, graph_windows=4),
                                   dict(fast_grid_div=4, graph_windows=8, event_group=8),
                                   # tiles claimed at run time, event blocks joining the claims
                                   dict(fast_grid_div=1, graph_windows=4, event_group=4, tile_claim=1),
                                   dict(autotune=True)])
def test_batch_matches_oracle_runs(rdx, oracle_lib, shape):
    runs = _small_ensemble()
    _say(f"case: batch of {len(runs)} runs, T = {[w.mesh.n_tets for w in runs]}, shape {shape}")
    refs = _refs(oracle_lib, runs)
    b = _batch(rdx, runs)
    b.set_exec_options(**shape)
    # uneven horizons: every run has its own t_end, so runs drop out of the
    # launches at different windows, and the last window of each is truncated
    t_end = [0.05 + 0.03 * i for i in range(len(runs))]
    b.run(t_end)
    for r, t in zip(refs, t_end):
        r.run(t)
    for i, r in enumerate(refs):
        _assert_run(b, i, r, "run(t_end_i)")
    # full windows on top, in several calls (graphs are replayed across calls)
    for k in range(3):
        b.step(5)
        for r in refs:
            r.step(5)
        for i, r in enumerate(refs):
            _assert_run(b, i, r, f"step(5) #{k}")


def test_batch_equals_solo_runs_and_restart(rdx, oracle_lib):
    """A run gives the same counts alone (rdx_create) and in a batch; a run
    restarted mid-way does not disturb the others."""
    runs = _small_ensemble(n=5, seed=77)
    _say("case: batch of 5 vs solo simulations, restart of run 2")
    b = _batch(rdx, runs)
    b.set_exec_options(graph_windows=4)
    solos = []
    for w in runs:
        s = rdx.Sim(w.mesh.as_dict(), w.model.as_dict(), w.seed)
        s.set_counts(w.counts)
        solos.append(s)
    b.run(0.2)
    for s in solos:
        s.run(0.2)
    for i, s in enumerate(solos):
        np.testing.assert_array_equal(b.get_counts(i), s.get_counts())
        assert b.stats(i) == s.stats()
    # restart run 2 from new counts at t = 0 and take every run to 0.3 s
    w2 = runs[2]
    new2 = I.place_uniform(w2.mesh, [300, 200, 0, 100, 0, 0], 5)
    b.set_counts(2, new2)
    solos[2].set_counts(new2)
    b.run(0.3)
    for s in solos:
        s.run(0.3)
    # the oracle: run 2 from its new counts at t = 0; the others through the
    # same two calls (the 0.2 s call ends in a truncated window)
    refs = _refs(oracle_lib, runs)
    refs[2].reset(new2)
    for i, r in enumerate(refs):
        if i != 2:
            r.run(0.2)
        r.run(0.3)
    for i, s in enumerate(solos):
        np.testing.assert_array_equal(b.get_counts(i), s.get_counts())
    _assert_run(b, 2, refs[2], "restarted run")
    for i in (0, 1, 3, 4):
        _assert_run(b, i, refs[i], "untouched run")
    for s in solos:
        s.close()
    b.close()


def test_graph_replays_interleaved_with_eager_work(rdx, oracle_lib):
    """Captured graphs replayed many times, with other device work and
    synchronisations between the replays; every replay's result is checked."""
    import torch
    runs = _small_ensemble(n=3, seed=5, t_lo=200, t_hi=1500)
    _say("case: graph replays with eager torch work between them")
    refs = _refs(oracle_lib, runs)
    b = _batch(rdx, runs)
    b.set_exec_options(graph_windows=2)
    x = torch.ones(1 << 20, device="cuda")
    for k in range(6):
        b.step(4)
        y = (x * float(k)).sum()
        torch.cuda.synchronize()
        assert float(y) == float(k) * (1 << 20)
        for r in refs:
            r.step(4)
        for i, r in enumerate(refs):
            _assert_run(b, i, r, f"replay set {k}")


def test_single_sim_with_graphs(rdx, oracle_lib):
    w = I.config_small()
    _say("case: 6x6x6 box single simulation with 8-window graphs")
    s = rdx.Sim(w.mesh.as_dict(), w.model.as_dict(), w.seed)
    s.set_exec_options(graph_windows=8)
    s.set_counts(w.counts)
    ref = oracle_lib.Instance(w.mesh.as_dict(), w.model.as_dict(), w.seed)
    ref.reset(w.counts)
    for n in (1, 8, 17, 3):
        s.step(n)
        ref.step(n)
        got = s.get_counts()
        assert np.array_equal(got, ref.counts), n
        st = s.stats()
        assert st.ssa_events == ref.tallies.ssa_events and st.moves == ref.tallies.moves
        assert st.face_moves == ref.tallies.face_moves


def test_set_counts_all_in_one_launch(rdx, oracle_lib):
    """Resetting every run from device tensors in one launch gives the same
    results as the oracle, also when it restarts runs that already ran (the
    count buffers then swap roles)."""
    import torch
    runs = _small_ensemble(n=5, seed=17)
    _say(f"case: batched reset of {len(runs)} runs, T = {[w.mesh.n_tets for w in runs]}")
    dev = [torch.from_numpy(np.ascontiguousarray(w.counts)).cuda() for w in runs]
    b = _batch(rdx, runs)
    b.set_exec_options(graph_windows=4)
    t_end = [0.05 + 0.02 * i for i in range(len(runs))]
    for rep in range(2):
        refs = _refs(oracle_lib, runs)
        b.set_counts_all(dev)
        b.run(t_end)
        for r, t in zip(refs, t_end):
            r.run(t)
        for i, r in enumerate(refs):
            _assert_run(b, i, r, f"pass {rep}")
        b.step(3)  # leave the runs at an odd window before the next reset


def test_batch_structure_mismatch_is_rejected(rdx):
    a = I.ensemble_runs(n_runs=1, seed=1, t_lo=200, t_hi=300)[0]
    other = I.model_abc().as_dict()
    with pytest.raises(rdx.RdxError) as e:
        rdx.Batch([(a.mesh.as_dict(), a.model.as_dict(), 1), (a.mesh.as_dict(), other, 2)])
    assert e.value.status == -1


def test_batch_options_validation(rdx):
    runs = _small_ensemble(n=2, seed=9, t_lo=200, t_hi=300)
    b = _batch(rdx, runs)
    assert b.exec_options()["autotune"] == 1
    with pytest.raises(rdx.RdxError):
        b.set_exec_options(fast_grid_div=3)
    with pytest.raises(rdx.RdxError):
        b.set_exec_options(graph_windows=0)
    with pytest.raises(rdx.RdxError):
        b.set_exec_options(event_group=65)
    with pytest.raises(rdx.RdxError):
        b.set_exec_options(event_bins=2)
    b.set_exec_options(fast_grid_div=2, graph_windows=16)
    assert b.exec_options() == dict(autotune=0, fast_grid_div=2, graph_windows=16, event_group=4,
                                    event_bins=1, tile_claim=0)
    with pytest.raises(rdx.RdxError):
        b.set_exec_options(tile_claim=2)
    b.set_exec_options(event_group=2, event_bins=0)
    assert b.exec_options()["event_group"] == 2 and b.exec_options()["event_bins"] == 0
    # the tuner's choice is one of its candidates and is kept once tuning ends
    b.set_exec_options(autotune=True)
    b.step(600)  # enough windows for every candidate, three passes
    o = b.exec_options()
    assert o["autotune"] == 0 and o["event_group"] in (4, 8, 16, 64) and o["fast_grid_div"] in (1, 2, 4)


@pytest.mark.parametrize("S,R", [(16, 30), (12, 12)])
def test_batch_random_models_with_regions(rdx, oracle_lib, S, R):
    """Runs that share one random reaction structure (homodimers, sources,
    immobile species) but differ in mesh, regions, rate constants, diffusion
    coefficients and seed, with enough molecules that most tets list events:
    the event chunks mix nothing across runs and every run equals the oracle
    alone."""
    from tests.randmodels import random_counts, random_model
    rng = np.random.default_rng(700 + S + R)
    base = random_model(rng, S, R, 2)
    runs = []
    for j, dims in enumerate([(3, 2, 2), (5, 4, 3), (2, 2, 7)]):
        mesh = I.box_mesh(*dims, 0.5e-6, jitter=0.1, seed=40 + j)
        mesh.region = rng.integers(0, 2, mesh.n_tets).astype(np.uint8)
        md = dict(base)
        md["kcst"] = base["kcst"] * rng.uniform(0.5, 1.5, base["kcst"].shape)
        md["D"] = base["D"] * rng.uniform(0.5, 1.5, S)
        counts = random_counts(rng, S, mesh.n_tets, mean=6.0)
        runs.append((mesh, md, 300 + j, counts))
    _say(f"case: batch of random S={S} R={R} models, T = {[m.n_tets for m, _, _, _ in runs]}")
    b = rdx.Batch([(m.as_dict(), md, seed) for m, md, seed, _ in runs])
    b.set_exec_options(graph_windows=2)
    refs = []
    for i, (m, md, seed, c) in enumerate(runs):
        b.set_counts(i, c)
        r = oracle_lib.Instance(m.as_dict(), md, seed)
        r.reset(c)
        refs.append(r)
    for k in range(4):
        b.step(1)
        for r in refs:
            r.step(1)
        for i, r in enumerate(refs):
            _assert_run(b, i, r, f"window {k}")


def test_ensemble_as_benchmarked_sampled(rdx, oracle_lib):
    """The batched leg at its benchmarked size: 1024 uneven runs (T ~ logU(1e3,
    5e4), 1 s each), every run reset from device counts in one launch and run
    to t_end on graphs once the launch shape is tuned; every 64th run plus the
    smallest and the largest against the oracle run alone."""
    import torch
    runs = I.ensemble_runs()
    T = np.array([w.mesh.n_tets for w in runs])
    idx = sorted(set(list(range(0, len(runs), 64)) + [int(T.argmin()), int(T.argmax())]))
    _say(f"case: ensemble of {len(runs)} runs, {int(T.sum())} tets, sampled runs {idx}")
    b = rdx.Batch([(w.mesh.as_dict(), w.model.as_dict(), w.seed) for w in runs])
    c0 = [torch.from_numpy(np.ascontiguousarray(w.counts)).to("cuda:0") for w in runs]
    stream = torch.cuda.current_stream()
    t_end = [w.t_end for w in runs]
    for _ in range(20):  # as the benchmark's warm-up: until the tuner has settled
        b.set_counts_all(c0, stream=stream)
        b.run(t_end, stream=stream)
        torch.cuda.synchronize()
        if not b.exec_options()["autotune"]:
            break
    assert b.exec_options()["autotune"] == 0
    b.set_counts_all(c0, stream=stream)
    b.run(t_end, stream=stream)
    for i in idx:
        w = runs[i]
        ref = oracle_lib.Instance(w.mesh.as_dict(), w.model.as_dict(), w.seed)
        ref.reset(w.counts)
        ref.run(w.t_end)
        assert np.array_equal(b.get_counts(i), ref.counts), f"run {i}"
        st = b.stats(i)
        assert (st.ssa_events, st.moves, st.window_index) == (ref.tallies.ssa_events, ref.tallies.moves,
                                                              ref.window), f"run {i}"
    b.close()
