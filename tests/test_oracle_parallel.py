"""The all-core build of the oracle (the benchmark's all-core CPU baseline)
equals the serial oracle bit for bit: counts and tallies after every window,
on a random model with regions, homodimers, sources and immobile species and
on the dense-event 10x-density simple-model recipe, at several thread
counts.  Under the snapshot reading of Algorithm 1 each tet's draws depend
only on its own streams and the moves are integer sums, so the tet order of
a parallel loop cannot change a result."""
import numpy as np
import pytest

from paper_1610_02258_amd import inputs as I
from tests.randmodels import random_counts, random_model


def _compare(O, mesh, md, seed, counts, windows, threads):
    a = O.Instance(mesh, md, seed)
    b = O.Instance(mesh, md, seed, parallel=True)
    a.reset(counts)
    b.reset(counts)
    for k in range(windows):
        a.step(1)
        b.step_parallel(1, threads)
        assert np.array_equal(a.counts, b.counts), (k, int((a.counts != b.counts).sum()))
    assert (a.tallies.ssa_events, a.tallies.moves, a.tallies.face_moves, a.tallies.voxel_steps) == \
        (b.tallies.ssa_events, b.tallies.moves, b.tallies.face_moves, b.tallies.voxel_steps)
    assert a.window == b.window
    return a.tallies


@pytest.mark.parametrize("threads", [2, 4, 8])
def test_parallel_oracle_random_model(oracle_lib, threads):
    rng = np.random.default_rng(5)
    mesh = I.box_mesh(10, 8, 6, 0.5e-6, jitter=0.1, seed=5)
    mesh.region = rng.integers(0, 3, mesh.n_tets).astype(np.uint8)
    md = random_model(rng, 9, 14, 3)
    counts = random_counts(rng, 9, mesh.n_tets, mean=12.0)
    tal = _compare(oracle_lib, mesh.as_dict(), md, 17, counts, 6, threads)
    assert tal.ssa_events > 1000 and tal.moves > 10_000


def test_parallel_oracle_dense_events(oracle_lib):
    w = I.config_simple_variant(10.0, 0.5, extent_um=(3.0, 3.0, 4.0))
    tal = _compare(oracle_lib, w.mesh.as_dict(), w.model.as_dict(), w.seed, w.counts, 5, 8)
    assert tal.ssa_events > 500
