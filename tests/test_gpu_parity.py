"""GPU parity: the HIP path through the C ABI against the oracle, element by
element on the same seeded inputs.  Integer counts and tallies must match bit
for bit after every window (the oracle and the kernels compute the same
sequence of IEEE-754 binary64 operations with fp contraction off)."""
import math
import sys

import numpy as np
import pytest

from paper_1610_02258_amd import inputs as I
from tests.meshes import mirror_pair, model, single_tet, stars
from tests.randmodels import random_counts, random_model

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rdx():
    from paper_1610_02258_amd import rdx as R
    R.lib()
    return R


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(rdx, O, mesh, model_, seed, counts, tau=0.0):
    sim = rdx.Sim(mesh, model_, seed, tau_override=tau)
    ref = O.Instance(mesh, model_, seed, tau_override=tau)
    assert sim.tau == ref.tau
    sim.set_counts(counts)
    ref.reset(counts)
    return sim, ref


def _assert_same(sim, ref, what=""):
    got = sim.get_counts()
    if not np.array_equal(got, ref.counts):
        bad = np.argwhere(got != ref.counts)
        s, t = bad[0]
        raise AssertionError(f"{what}: {len(bad)} mismatches, first species {s} tet {t}: "
                             f"gpu {got[s, t]} oracle {ref.counts[s, t]}")
    st = sim.stats()
    assert st.ssa_events == ref.tallies.ssa_events, (what, st.ssa_events, ref.tallies.ssa_events)
    assert st.moves == ref.tallies.moves, (what, st.moves, ref.tallies.moves)
    assert st.face_moves == ref.tallies.face_moves, (what, st.face_moves, ref.tallies.face_moves)
    assert st.voxel_steps == ref.tallies.voxel_steps
    assert st.window_index == ref.window and st.t == ref.t


# ------------------------------------------------------- random layer ----

def test_device_philox_matches(rdx, oracle_lib):
    rows = [[0] * 6, [0xffffffff] * 6,
            [0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344, 0xa4093822, 0x299f31d0]]
    rng = np.random.default_rng(1)
    rnd = rng.integers(0, 2**32, size=(5000, 6), dtype=np.uint64).astype(np.uint32)
    inp = np.concatenate([np.array(rows, np.uint32), rnd])
    out = rdx.selftest_philox(inp)
    for j in range(inp.shape[0]):
        np.testing.assert_array_equal(out[j], oracle_lib.philox4x32_10(inp[j, :4], inp[j, 4:]))


def test_device_ln_bitwise(rdx, oracle_lib):
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.uniform(2.0**-53, 1.0, 100000),
                        np.exp(rng.uniform(math.log(2.0**-53), 0.0, 100000)),
                        [1.0, 0.5, 2.0**-53, 0.7071067811865476, 0.7071067811865475]])
    y = rdx.selftest_ln(x)
    ref = np.array([oracle_lib.ln(v) for v in x])
    assert np.array_equal(y.view(np.int64), ref.view(np.int64))


@pytest.mark.parametrize("m,p", [(7, 0.3), (40, 0.8), (1500, 0.2), (3, 1.0), (0, 0.4),
                                 (1000, 1.0 - 2.0**-53), (25, 0.5)])
def test_device_binomial_bitwise(rdx, oracle_lib, m, p):
    got = rdx.selftest_binom(42, m, p, 20000, stream_id=3, window=9)
    ref = oracle_lib.sample_binom(42, m, p, 20000, stream_id=3, window=9)
    np.testing.assert_array_equal(got, ref)


# -------------------------------------------------------- window parity ----

def test_small_workload_parity(rdx, oracle_lib):
    w = I.config_small()
    _say("case: 6x6x6 box, A+B<->C, 10 ms (one truncated window), then 40 windows")
    sim, ref = _pair(rdx, oracle_lib, w.mesh.as_dict(), w.model.as_dict(), w.seed, w.counts)
    sim.run(w.t_end)
    ref.run(w.t_end)
    _assert_same(sim, ref, "run(10 ms)")
    for k in range(40):
        sim.step(1)
        ref.step(1)
        _assert_same(sim, ref, f"window {k}")


def test_small_workload_fast_reactions(rdx, oracle_lib):
    """Same mesh with reactions 1000x faster: many SSA events per window."""
    w = I.config_small()
    m = I.model_abc(kf=1e9, kb=1e3).as_dict()
    counts = I.place_uniform(w.mesh, [20000, 15000, 3000], 11)
    sim, ref = _pair(rdx, oracle_lib, w.mesh.as_dict(), m, 123, counts)
    for k in range(6):
        sim.step(1)
        ref.step(1)
        _assert_same(sim, ref, f"window {k}")
    assert ref.tallies.ssa_events > 100000


@pytest.mark.parametrize("case", range(14))
def test_random_models_parity(rdx, oracle_lib, case):
    rng = np.random.default_rng(1000 + case)
    S = int(rng.integers(1, 17))
    R = int(rng.integers(0, 33))
    n_regions = int(rng.integers(1, 4))
    if case == 0:
        S, R = 16, 32          # the largest tables
    if case == 1:
        S, R = 1, 0            # pure diffusion of one species
    nx, ny, nz = (int(v) for v in rng.integers(1, 8, 3))
    mesh = I.box_mesh(nx, ny, nz, 0.5e-6, jitter=0.1, seed=case)
    mesh.region = rng.integers(0, n_regions, mesh.n_tets).astype(np.uint8)
    md = random_model(rng, S, R, n_regions)
    counts = random_counts(rng, S, mesh.n_tets, mean=float(rng.uniform(0.5, 30)))
    _say(f"case {case}: T={mesh.n_tets} S={S} R={R} regions={n_regions}")
    sim, ref = _pair(rdx, oracle_lib, mesh.as_dict(), md, 77 + case, counts)
    t_end = 5.5 * ref.tau
    sim.run(t_end)
    ref.run(t_end)
    _assert_same(sim, ref, "run 5.5 tau")
    sim.step(3)
    ref.step(3)
    _assert_same(sim, ref, "3 more windows")


@pytest.mark.parametrize("S,R", [(16, 20), (16, 30), (12, 12)])
def test_dense_events_every_tet_listed(rdx, oracle_lib, S, R):
    """Random models with a dozen molecules per species and tet: nearly every
    tet has SSA events in every window, so tiles list up to 64 tets, which the
    event blocks take in chunks of 64, 32 or 16 lanes by reaction-table size;
    2 regions, ragged last tile."""
    rng = np.random.default_rng(50 + S + R)
    mesh = I.box_mesh(6, 5, 4, 0.5e-6, jitter=0.1, seed=S + R)  # 720 tets: 11 full tiles + 16
    mesh.region = rng.integers(0, 2, mesh.n_tets).astype(np.uint8)
    md = random_model(rng, S, R, 2)
    counts = random_counts(rng, S, mesh.n_tets, mean=12.0)
    _say(f"case: dense events T={mesh.n_tets} S={S} R={R}")
    sim, ref = _pair(rdx, oracle_lib, mesh.as_dict(), md, 900 + R, counts)
    for k in range(3):
        sim.step(1)
        ref.step(1)
        _assert_same(sim, ref, f"window {k}")
    # most tets had events (each listed tet is one lane of an event chunk)
    assert ref.tallies.ssa_events > 3 * mesh.n_tets


def test_edge_cases(rdx, oracle_lib):
    # all counts zero
    w = I.config_small()
    zero = np.zeros_like(w.counts)
    sim, ref = _pair(rdx, oracle_lib, w.mesh.as_dict(), w.model.as_dict(), 5, zero)
    sim.step(3)
    ref.step(3)
    _assert_same(sim, ref, "zero counts")
    assert sim.get_counts().sum() == 0
    # a single tet: no neighbours, tau given
    md = model([0, 0], [(["A"], ["B"], 5.0), (["B"], ["A"], 1.0)], ["A", "B"])
    sim, ref = _pair(rdx, oracle_lib, single_tet(), md, 9, np.array([[50], [3]], np.int32), tau=0.01)
    sim.step(20)
    ref.step(20)
    _assert_same(sim, ref, "single tet")
    # mirror pair: p = 1 swaps every window
    c0 = np.array([[37, 5]], np.int32)
    sim, ref = _pair(rdx, oracle_lib, mirror_pair(), model([1e-12], [], ["A"]), 3, c0)
    sim.step(3)
    ref.step(3)
    _assert_same(sim, ref, "mirror pair")
    np.testing.assert_array_equal(sim.get_counts(), c0[:, ::-1])
    # run to a time already reached is a no-op
    sim.run(sim.stats().t)
    assert sim.stats().windows == 3


@pytest.mark.parametrize("p_centre", [0.9, 1.0])
def test_binomial_items_where_the_cap_binds(rdx, oracle_lib, p_centre):
    """Listed centres whose binomial items would lose more molecules than the
    reactions left (A -> 0 in the centre at k tau = 0.2, 60 molecules, p = 0.9
    or 1): the branch that splits the post-reaction count afresh, bit for bit
    against the oracle, then two more windows with every tet in play."""
    n_st, N0, D = 2000, 60, 1e-12
    G = oracle_lib.Instance(stars(1), model([D], [(["A"], [], 1.0)], ["A"]), 1).geometry()["G"][0]
    tau = (p_centre if p_centre < 1.0 else 1.5) / (D * G)
    md = model([D], [(["A"], [], 0.2 / tau)], ["A"])
    c = np.zeros((1, 5 * n_st), np.int32)
    c[0, 0::5] = N0
    _say(f"capped binomial items, p {p_centre}, {5 * n_st} tets")
    sim, ref = _pair(rdx, oracle_lib, stars(n_st), md, 31, c, tau=tau)
    sim.step(1)
    ref.step(1)
    _assert_same(sim, ref, f"p {p_centre}, window 1")
    # the centres the cap emptied (all of them at p = 1)
    assert (ref.counts[0, 0::5] == 0).mean() > 0.2
    sim.step(2)
    ref.step(2)
    _assert_same(sim, ref, f"p {p_centre}, windows 2-3")


def test_checkpoint_resume_is_bit_identical(rdx, oracle_lib):
    w = I.config_small()
    m = I.model_abc(kf=1e8, kb=50.0).as_dict()
    a = rdx.Sim(w.mesh.as_dict(), m, 31)
    a.set_counts(w.counts)
    a.step(12)
    straight = a.get_counts()
    b = rdx.Sim(w.mesh.as_dict(), m, 31)
    b.set_counts(w.counts)
    b.step(5)
    blob = b.save()
    c = rdx.Sim(w.mesh.as_dict(), m, 31)
    c.load(blob)
    c.step(7)
    np.testing.assert_array_equal(c.get_counts(), straight)
    assert c.stats().ssa_events == a.stats().ssa_events


def test_device_pointer_io(rdx, oracle_lib):
    torch = pytest.importorskip("torch")
    w = I.config_small()
    sim, ref = _pair(rdx, oracle_lib, w.mesh.as_dict(), w.model.as_dict(), 2, w.counts)
    dev = torch.from_numpy(w.counts.copy()).cuda()
    stream = torch.cuda.current_stream()
    sim.set_counts(dev, stream=stream)
    sim.step(4, stream=stream)
    out = torch.zeros_like(dev)
    sim.get_counts(out, stream=stream)
    torch.cuda.synchronize()
    ref.step(4)
    np.testing.assert_array_equal(out.cpu().numpy(), ref.counts)


# ------------------------------------------------- full-size workloads ----

def test_simple_model_full_size_prefix(rdx, oracle_lib):
    """480,000-tet jittered box, 10 species / 12 reactions: the first windows
    of the benchmarked run, compared on every count."""
    w = I.config_simple()
    _say(f"case: simple model, T={w.mesh.n_tets}")
    sim, ref = _pair(rdx, oracle_lib, w.mesh.as_dict(), w.model.as_dict(), w.seed, w.counts)
    for k in range(3):
        sim.step(1)
        ref.step(1)
        _assert_same(sim, ref, f"window {k}")


@pytest.mark.parametrize("claim", [0, 1])
def test_dendrite_full_size_prefix(rdx, oracle_lib, claim):
    """The dendrite's first windows, diffusion tiles in static ranges and
    claimed at run time, in graphs of one window."""
    w = I.config_dendrite()
    _say(f"case: dendrite, T={w.mesh.n_tets}, tile claim {claim}")
    sim, ref = _pair(rdx, oracle_lib, w.mesh.as_dict(), w.model.as_dict(), w.seed, w.counts)
    sim.set_exec_options(autotune=False, fast_grid_div=1, graph_windows=1, event_group=16, tile_claim=claim)
    for k in range(2):
        sim.step(1)
        ref.step(1)
        _assert_same(sim, ref, f"window {k}")


@pytest.mark.parametrize("density,h,extent", [(10.0, 0.5, (3.0, 3.0, 4.0)), (0.1, 0.5, (3.0, 3.0, 4.0)),
                                              (1.0, 0.25, (2.0, 2.0, 3.0)), (1.0, 1.0, (4.0, 4.0, 6.0))])
def test_density_and_refinement_series(rdx, oracle_lib, density, h, extent):
    """The simple-model recipe at 0.1x and 10x molecule density and at 0.25 and
    1 um cubes, on boxes small enough for the oracle: every window compared."""
    w = I.config_simple_variant(density, h, extent_um=extent)
    _say(f"case: {w.name}, T={w.mesh.n_tets}, {int(w.counts.sum())} molecules")
    sim, ref = _pair(rdx, oracle_lib, w.mesh.as_dict(), w.model.as_dict(), w.seed, w.counts)
    for k in range(30):
        sim.step(1)
        ref.step(1)
        _assert_same(sim, ref, f"window {k}")


@pytest.mark.parametrize("density,h,bins,claim", [(10.0, 0.5, 1, 0), (10.0, 0.5, 0, 0), (10.0, 0.5, 1, 1),
                                                  (1.0, 0.25, 1, 1)])
def test_series_full_size_prefix(rdx, oracle_lib, density, h, bins, claim):
    """The series at full size: 480,000 tets with 1e7 molecules (10x the
    benchmarked density, with the listed tets binned by expected events and
    in one queue, diffusion tiles in static ranges and claimed at run time)
    and the refined 3,840,000-tet box (0.25 um cubes): the first windows
    compared on every count."""
    w = I.config_simple_variant(density, h)
    _say(f"case: {w.name}, T={w.mesh.n_tets}, event bins {bins}, tile claim {claim}")
    sim, ref = _pair(rdx, oracle_lib, w.mesh.as_dict(), w.model.as_dict(), w.seed, w.counts)
    sim.set_exec_options(autotune=False, fast_grid_div=1, graph_windows=1, event_group=8,
                         event_bins=bins, tile_claim=claim)
    for k in range(2):
        sim.step(1)
        ref.step(1)
        _assert_same(sim, ref, f"window {k}")


def test_simple_model_whole_benchmarked_run(rdx, oracle_lib):
    """The benchmarked step itself at full size: 480,000 tets, 10 species,
    1e6 molecules, 100 ms = 220 windows, reset from device counts and run to
    t_end on the graph path once the launch shape is tuned (as the timed
    steps do), against the oracle's whole run: every count and tally."""
    import torch
    w = I.config_simple()
    _say(f"case: whole benchmarked run, T={w.mesh.n_tets}, t_end={w.t_end}")
    sim = rdx.Sim(w.mesh.as_dict(), w.model.as_dict(), w.seed)
    c0 = torch.from_numpy(np.ascontiguousarray(w.counts)).to("cuda:0")
    stream = torch.cuda.current_stream()
    for k in range(6):  # the first runs also tune the launch shape
        sim.set_counts(c0, stream=stream)
        sim.run(w.t_end, stream=stream)
        if k >= 1 and not sim.exec_options()["autotune"]:
            break
    assert sim.exec_options()["autotune"] == 0
    ref = oracle_lib.Instance(w.mesh.as_dict(), w.model.as_dict(), w.seed)
    ref.reset(w.counts)
    ref.run(w.t_end)
    _assert_same(sim, ref, "whole run")
    assert ref.window == 220
    sim.close()
