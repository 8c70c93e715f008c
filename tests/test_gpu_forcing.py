"""GPU parity of time-varying forcing (rate constants replaced between
windows) and recording (per-region counts, also into a device ring buffer)
against the oracle, through the C ABI (section 3.2: influx updated every
1 ms, per-region counts recorded every 0.02 ms)."""
import sys

import numpy as np
import pytest

from paper_1610_02258_amd import inputs as I
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


def _same(sim, ref, what):
    got = sim.get_counts()
    assert np.array_equal(got, ref.counts), f"{what}: {(got != ref.counts).sum()} count mismatches"
    st = sim.stats()
    assert (st.ssa_events, st.moves, st.window_index) == (ref.tallies.ssa_events, ref.tallies.moves,
                                                          ref.window), what
    assert np.array_equal(sim.region_counts(), ref.region_counts()), what


def test_switched_rates_match_oracle(rdx, oracle_lib):
    """Random structure (sources, homodimers, two regions), rates redrawn six
    times; segments of several windows run as captured graphs, one switch
    falls inside a window (the window is cut there)."""
    rng = np.random.default_rng(71)
    S, R = 10, 14
    mesh = I.box_mesh(6, 5, 4, 0.5e-6, jitter=0.1, seed=7)  # 720 tets, ragged last tile
    mesh.region = rng.integers(0, 2, mesh.n_tets).astype(np.uint8)
    md = random_model(rng, S, R, 2)
    counts = random_counts(rng, S, mesh.n_tets, mean=5.0)
    _say(f"case: forcing, T={mesh.n_tets} S={S} R={R}, 6 switches")
    sim = rdx.Sim(mesh.as_dict(), md, 41)
    ref = oracle_lib.Instance(mesh.as_dict(), md, 41)
    sim.set_counts(counts)
    ref.reset(counts)
    t = 0.0
    for seg in range(6):
        k = md["kcst"] * rng.uniform(0.2, 2.0, md["kcst"].shape)
        if seg == 3:
            k[:, 0] = 0.0  # a reaction switched off everywhere
        sim.set_rate_constants(k)
        ref.set_rates(k)
        t += (8.5 if seg == 2 else 8.0) * sim.tau
        sim.run(t)
        ref.run(t)
        _same(sim, ref, f"segment {seg}")
    sim.close()


def test_device_ring_recording(rdx, oracle_lib):
    """One record per window into a device int64 ring [K, n_regions, S],
    no host synchronisation between windows, influx switched half way."""
    import torch
    rng = np.random.default_rng(72)
    S, R, K = 8, 10, 24
    mesh = I.box_mesh(5, 5, 6, 0.5e-6, jitter=0.1, seed=8)
    mesh.region = (np.arange(mesh.n_tets) % 3).astype(np.uint8)
    md = random_model(rng, S, R, 3)
    counts = random_counts(rng, S, mesh.n_tets, mean=4.0)
    _say(f"case: ring recording, T={mesh.n_tets} S={S} R={R} regions=3, K={K}")
    sim = rdx.Sim(mesh.as_dict(), md, 42)
    ref = oracle_lib.Instance(mesh.as_dict(), md, 42)
    sim.set_counts(counts)
    ref.reset(counts)
    ring = torch.full((K, 3, S), -1, dtype=torch.int64, device="cuda:0")
    want = np.zeros((K, 3, S), np.int64)
    k2 = md["kcst"] * 3.0
    for k in range(K):
        if k == K // 2:
            sim.set_rate_constants(k2)
            ref.set_rates(k2)
        sim.step(1)
        sim.region_counts(out=ring[k])
        ref.step(1)
        want[k] = ref.region_counts()
    got = ring.cpu().numpy()
    assert np.array_equal(got, want)
    assert np.array_equal(sim.get_counts(), ref.counts)
    sim.close()


def test_forcing_errors_keep_the_old_table(rdx, oracle_lib):
    rng = np.random.default_rng(73)
    mesh = I.box_mesh(4, 4, 4, 0.5e-6, seed=9)
    md = random_model(rng, 6, 6, 1)
    counts = random_counts(rng, 6, mesh.n_tets, mean=5.0)
    _say(f"case: forcing errors, T={mesh.n_tets}")
    sim = rdx.Sim(mesh.as_dict(), md, 43)
    ref = oracle_lib.Instance(mesh.as_dict(), md, 43)
    sim.set_counts(counts)
    ref.reset(counts)
    bad = md["kcst"].copy()
    bad[0, 1] = -1.0
    for k in (bad, np.full_like(md["kcst"], np.nan), md["kcst"][:, :-1]):
        with pytest.raises(rdx.RdxError):
            sim.set_rate_constants(k)
    sim.step(5)
    ref.step(5)
    _same(sim, ref, "after rejected tables")
    sim.close()


def test_batch_per_run_forcing_and_recording(rdx, oracle_lib):
    """Three runs in one batch; only run 1's rates change: each run equals
    its oracle run alone, with per-run region sums."""
    rng = np.random.default_rng(74)
    S, R = 8, 10
    base = random_model(rng, S, R, 2)
    runs = []
    for j, dims in enumerate([(4, 4, 5), (6, 3, 4), (3, 3, 3)]):
        mesh = I.box_mesh(*dims, 0.5e-6, jitter=0.1, seed=20 + j)
        mesh.region = rng.integers(0, 2, mesh.n_tets).astype(np.uint8)
        runs.append((mesh, dict(base), 300 + j, random_counts(rng, S, mesh.n_tets, mean=4.0)))
    _say(f"case: batch forcing, T = {[m.n_tets for m, _, _, _ in runs]}")
    b = rdx.Batch([(m.as_dict(), md, seed) for m, md, seed, _ in runs])
    refs = []
    for i, (m, md, seed, c) in enumerate(runs):
        b.set_counts(i, c)
        r = oracle_lib.Instance(m.as_dict(), md, seed)
        r.reset(c)
        refs.append(r)
    b.step(6)
    for r in refs:
        r.step(6)
    k1 = base["kcst"] * rng.uniform(0.1, 3.0, base["kcst"].shape)
    b.set_rate_constants(1, k1)
    refs[1].set_rates(k1)
    b.step(6)
    for r in refs:
        r.step(6)
    for i, r in enumerate(refs):
        assert np.array_equal(b.get_counts(i), r.counts), f"run {i}"
        assert np.array_equal(b.region_counts(i), r.region_counts()), f"run {i}"
        assert b.stats(i).ssa_events == r.tallies.ssa_events
    b.close()


def test_dendrite_influx_switch_full_size(rdx, oracle_lib):
    """The ~1e6-tet dendrite: calcium influx (region 1) tripled after the
    first window, then switched off; counts and per-region sums compared."""
    w = I.config_dendrite()
    md = w.model.as_dict()
    _say(f"case: dendrite influx switch, T={w.mesh.n_tets}")
    sim = rdx.Sim(w.mesh.as_dict(), md, w.seed)
    ref = oracle_lib.Instance(w.mesh.as_dict(), md, w.seed)
    sim.set_counts(w.counts)
    ref.reset(w.counts)
    sim.step(1)
    ref.step(1)
    influx = np.flatnonzero(np.asarray(md["lhs"]).sum(axis=1) == 0)  # zero-order reactions
    assert md["kcst"][1, influx].max() > 0
    for scale in (3.0, 0.0):
        k = md["kcst"].copy()
        k[1, influx] *= scale
        sim.set_rate_constants(k)
        ref.set_rates(k)
        sim.step(1)
        ref.step(1)
        _same(sim, ref, f"influx x{scale}")
    sim.close()


@pytest.mark.parametrize("dims,n_regions", [((10, 9, 7), 8), ((7, 6, 5), 5), ((1, 1, 1), 2), ((9, 9, 9), 1)])
def test_region_counts_sizes_and_wide_sums(rdx, oracle_lib, dims, n_regions):
    """Region sums straight after set_counts with counts up to 2^30 - 1, so
    sums pass 2^32: 8 and 5 regions (the widest accumulator variant), a
    6-tet mesh smaller than one block, one region; host and device output."""
    import torch
    rng = np.random.default_rng(sum(dims) + n_regions)
    S = 16 if n_regions == 8 else 3
    mesh = I.box_mesh(*dims, 0.5e-6, seed=5)
    mesh.region = rng.integers(0, n_regions, mesh.n_tets).astype(np.uint8)
    mesh.region[:n_regions] = np.arange(min(n_regions, mesh.n_tets))
    md = random_model(rng, S, 4, n_regions)
    counts = rng.integers(0, 2**30, (S, mesh.n_tets)).astype(np.int32)
    _say(f"case: region sums, T={mesh.n_tets} S={S} regions={n_regions}")
    sim = rdx.Sim(mesh.as_dict(), md, 1)
    ref = oracle_lib.Instance(mesh.as_dict(), md, 1)
    sim.set_counts(counts)
    ref.set_counts(counts)
    want = ref.region_counts()
    if mesh.n_tets > 100:
        assert want.max() > 2**32
    assert np.array_equal(sim.region_counts(), want)
    dev = torch.full((n_regions, S), -7, dtype=torch.int64, device="cuda:0")
    sim.region_counts(out=dev)
    assert np.array_equal(dev.cpu().numpy(), want)
    sim.close()


def test_step_recorded_ring_wraps(rdx, oracle_lib):
    """rdx_step_recorded: 26 windows, a record every 3 into a 5-slot ring
    (8 records, so slots 0-2 hold records 5-7 and slots 3-4 records 3-4; the
    last 2 windows are not recorded), against the oracle; then every 1 window
    across graph-sized groups."""
    import torch
    rng = np.random.default_rng(75)
    S, R = 9, 11
    mesh = I.box_mesh(7, 5, 4, 0.5e-6, jitter=0.1, seed=10)
    mesh.region = rng.integers(0, 3, mesh.n_tets).astype(np.uint8)
    md = random_model(rng, S, R, 3)
    counts = random_counts(rng, S, mesh.n_tets, mean=4.0)
    _say(f"case: step_recorded, T={mesh.n_tets} S={S} R={R} regions=3")
    sim = rdx.Sim(mesh.as_dict(), md, 44)
    ref = oracle_lib.Instance(mesh.as_dict(), md, 44)
    sim.set_counts(counts)
    ref.reset(counts)
    ring = torch.full((5, 3, S), -1, dtype=torch.int64, device="cuda:0")
    assert sim.step_recorded(26, 3, ring) == 8
    recs = []
    for j in range(8):
        ref.step(3)
        recs.append(ref.region_counts())
    ref.step(2)
    got = ring.cpu().numpy()
    for slot, j in enumerate([5, 6, 7, 3, 4]):
        assert np.array_equal(got[slot], recs[j]), f"slot {slot}"
    assert np.array_equal(sim.get_counts(), ref.counts)
    ring2 = torch.full((20, 3, S), -1, dtype=torch.int64, device="cuda:0")
    assert sim.step_recorded(20, 1, ring2) == 20
    want = []
    for j in range(20):
        ref.step(1)
        want.append(ref.region_counts())
    assert np.array_equal(ring2.cpu().numpy(), np.stack(want))
    st = sim.stats()
    assert (st.ssa_events, st.moves, st.window_index) == (ref.tallies.ssa_events, ref.tallies.moves, ref.window)
    with pytest.raises(rdx.RdxError):
        sim.step_recorded(4, 0, ring2)
    sim.close()
