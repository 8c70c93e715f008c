"""Library calls on one thread while another thread holds a stream in HIP
graph capture (thread-local mode, as the library's own captures use): a
server's worker captures window graphs whenever a new launch shape appears,
so a simulation created, run and destroyed beside it must not depend on a
device-wide synchronisation, which the runtime refuses during any capture."""
import sys
import threading

import numpy as np
import pytest

from paper_1610_02258_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_sim_and_batch_beside_an_open_capture(oracle_lib):
    import torch
    from paper_1610_02258_amd import rdx

    w = I.config_simple_variant(1.0, 0.5, extent_um=(3.0, 3.0, 4.0))
    md, mesh = w.model.as_dict(), w.mesh.as_dict()
    ref = oracle_lib.Instance(mesh, md, w.seed)
    ref.reset(w.counts)
    ref.step(12)

    x = torch.zeros(64, device="cuda:0")
    torch.cuda.synchronize()
    started, release = threading.Event(), threading.Event()
    cap_err = []

    def capture():
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        try:
            with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
                x.add_(1.0)
                started.set()
                release.wait(120.0)
        except Exception as e:  # the runtime's verdict on the capture, not the library's
            cap_err.append(repr(e))
        finally:
            started.set()

    th = threading.Thread(target=capture)
    th.start()
    try:
        assert started.wait(120.0)
        _say(f"case: simulation beside an open capture, T={w.mesh.n_tets}")
        sim = rdx.Sim(mesh, md, w.seed)
        sim.set_counts(w.counts)
        sim.step(12)
        got = sim.get_counts()
        st = sim.stats()
        sim.close()
        np.testing.assert_array_equal(got, ref.counts)
        assert st.ssa_events == ref.tallies.ssa_events
        _say("case: batch beside an open capture")
        b = rdx.Batch([(mesh, md, w.seed), (mesh, md, w.seed + 1)])
        b.set_counts(0, w.counts)
        b.set_counts(1, w.counts)
        b.step(12)
        np.testing.assert_array_equal(b.get_counts(0), ref.counts)
        b.close()
    finally:
        release.set()
        th.join(180.0)
    _say(f"capture thread: {cap_err or 'captured'}")
    torch.cuda.synchronize()
