"""The dendrite workload (about 1e6 tets, 15 species / 20 reactions, calcium
influx in 5% of the tets) deep into its run, in the launch configuration the
benchmark times: 2.5 ms segments of one run (Algorithm 1 to each segment
end), launch shape tuned online, windows replayed from captured graphs, the
influx tripled at the start of the third segment (section 3.2's
time-varying influx).  The oracle is a pure function of (counts, window
index, seed, rates), so at several depths it starts from the GPU's counts and
runs the next three windows; the GPU does the same from a checkpoint and is
then restored, so the benchmarked sequence continues untouched."""
import sys

import numpy as np
import pytest

from paper_1610_02258_amd import inputs as I

pytestmark = pytest.mark.gpu

SEGMENT = 2.5e-3


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_dendrite_deep_checkpoints(oracle_lib):
    import torch
    from paper_1610_02258_amd import rdx

    w = I.config_dendrite()
    md = w.model.as_dict()
    _say(f"case: dendrite deep checkpoints, T={w.mesh.n_tets}")
    sim = rdx.Sim(w.mesh.as_dict(), md, w.seed)
    ref = oracle_lib.Instance(w.mesh.as_dict(), md, w.seed)
    assert sim.tau == ref.tau
    stream = torch.cuda.current_stream()
    c0 = torch.from_numpy(np.ascontiguousarray(w.counts)).to("cuda:0")
    sim.set_counts(c0, stream=stream)
    influx = np.flatnonzero(np.asarray(md["lhs"]).sum(axis=1) == 0)
    k3 = np.array(md["kcst"], np.float64)
    k3[:, influx] *= 3.0
    rates = md["kcst"]
    checked = []
    for seg in range(3):
        if seg == 2:  # the influx switch
            sim.set_rate_constants(k3, stream=stream)
            rates = k3
        # checkpoint at the segment start: three windows on both sides
        st0 = sim.stats(stream)
        counts = sim.get_counts()
        blob = sim.save(stream)
        ref.set_rates(rates)
        ref.counts = counts.copy()
        ref.window = st0.window_index
        ref.tallies = oracle_lib.Tallies()
        _say(f"checkpoint at window {st0.window_index} (t = {st0.t:.6f} s)")
        sim.step(3, stream=stream)
        ref.step(3)
        got = sim.get_counts()
        assert np.array_equal(got, ref.counts), (st0.window_index, int((got != ref.counts).sum()))
        st1 = sim.stats(stream)
        assert st1.ssa_events - st0.ssa_events == ref.tallies.ssa_events
        assert st1.moves - st0.moves == ref.tallies.moves
        assert st1.face_moves - st0.face_moves == ref.tallies.face_moves
        checked.append(st0.window_index)
        sim.load(blob, stream)
        # the benchmarked segment
        sim.run((seg + 1) * SEGMENT, stream=stream)
        torch.cuda.synchronize()
    _say(f"checked windows {checked}, tuned shape {sim.exec_options()}")
    assert checked[0] == 0 and checked[-1] > 600
    sim.close()
