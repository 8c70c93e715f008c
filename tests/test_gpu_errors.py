"""Device-side limits through the C ABI on the GPU: the overflow flag a
window kernel raises when a count passes 2^30 (reported by rdx_sync as
RDX_EOVERFLOW, counts equal to the oracle's at the failing window), and the
large-count path of the diffusion sampler (counts of 2^22 and more are not
packed into the item word and are read again from the count buffer),
compared with the oracle for one window."""
import sys
import time

import numpy as np
import pytest

from paper_1610_02258_amd import inputs as I
from tests.meshes import model, single_tet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rdx():
    from paper_1610_02258_amd import rdx as R
    R.lib()
    return R


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_count_overflow_flag(rdx, oracle_lib):
    """A zero-order source into a count just below 2^30 (single tet, about
    50 events per window): the window's SSA stops at the first count above
    2^30 and flags it; rdx_sync reports RDX_EOVERFLOW."""
    tet = single_tet()
    probe = oracle_lib.Instance(tet, model([0.0], [([], ["A"], 1.0)], ["A"]), 0, tau_override=1e-3)
    md = model([0.0], [([], ["A"], 5e4 / probe.geometry()["nav"][0])], ["A"])
    start = np.array([[(1 << 30) - 10]], np.int32)
    _say("case: overflow flag, single tet, start 2^30 - 10")
    sim = rdx.Sim(tet, md, 4, tau_override=1e-3)
    ref = oracle_lib.Instance(tet, md, 4, tau_override=1e-3)
    sim.set_counts(start)
    ref.reset(start)
    sim.run(1e-3)
    with pytest.raises(rdx.RdxError) as e:
        sim.sync()
    assert e.value.status == -5
    with pytest.raises(oracle_lib.OracleError) as eo:
        ref.run(1e-3)
    assert eo.value.code == -5
    assert np.array_equal(sim.get_counts(), ref.counts)
    assert int(sim.get_counts()[0, 0]) == (1 << 30) + 1
    sim.close()


def test_large_counts_unpacked_path(rdx, oracle_lib):
    """Pure diffusion on a 48-tet box with one count just above 2^22 and one
    near 2^24 (binomial over thousands of chunks, millions of leavers): one
    window equals the oracle's, counts and moved molecules."""
    mesh = I.box_mesh(2, 2, 2, 1e-6, jitter=0.1, seed=3)
    md = model([1e-12, 0.3e-12], [], ["A", "B"])
    counts = np.zeros((2, mesh.n_tets), np.int32)
    counts[0, 0] = (1 << 22) + 5
    counts[0, 17] = (1 << 24) - 3
    counts[1, 5] = (1 << 22) + 1
    counts[1, 1:] += 7
    _say(f"case: large counts, T={mesh.n_tets}, counts 2^22+5, 2^24-3, 2^22+1")
    sim = rdx.Sim(mesh.as_dict(), md, 8)
    ref = oracle_lib.Instance(mesh.as_dict(), md, 8)
    sim.set_counts(counts)
    ref.reset(counts)
    t0 = time.perf_counter()
    sim.step(1)
    sim.sync()
    el = time.perf_counter() - t0
    ref.step(1)
    got = sim.get_counts()
    assert np.array_equal(got, ref.counts), (got != ref.counts).sum()
    st = sim.stats()
    assert st.moves == ref.tallies.moves and st.face_moves == ref.tallies.face_moves
    _say(f"large counts: one window {el * 1e3:.1f} ms, {st.moves} molecules moved")
    sim.close()
