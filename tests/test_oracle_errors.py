"""Error paths of the oracle's window (Algorithm 1 with the caps the scheme
states): more than 2^22 SSA events of one tet in one window ends the run
with the events error, a count passing 2^30 with the overflow error.  Both
stop the run at the window where they happen."""
import numpy as np
import pytest

from tests.meshes import model, single_tet

OS_EOVERFLOW, OS_EEVENTS = -5, -9


def test_event_cap_raises(oracle_lib):
    """A <-> B at 2e7 events/s over a 0.5 s window: the cap of 2^22 events
    per tet and window is reached, the run stops with the events error."""
    md = model([0.0, 0.0], [(["A"], ["B"], 1e4), (["B"], ["A"], 1e4)], ["A", "B"])
    inst = oracle_lib.Instance(single_tet(), md, 3, tau_override=0.5)
    inst.reset(np.array([[1000], [1000]], np.int32))
    with pytest.raises(oracle_lib.OracleError) as e:
        inst.run(1.0)
    assert e.value.code == OS_EEVENTS
    assert inst.window == 1 and inst.tallies.ssa_events == 1 << 22
    assert inst.counts.sum() == 2000


def test_count_cap_raises(oracle_lib):
    """A zero-order source into a count just below 2^30: the window that
    passes 2^30 ends with the overflow error (about 50 events per window
    would be due; the SSA stops at the first count above the cap)."""
    tet = single_tet()
    md = model([0.0], [([], ["A"], 1.0)], ["A"])
    probe = oracle_lib.Instance(tet, md, 0, tau_override=1e-3)
    k = 5e4 / probe.geometry()["nav"][0]  # a0 = 5e4 /s, a0 tau = 50
    md = model([0.0], [([], ["A"], k)], ["A"])
    inst = oracle_lib.Instance(tet, md, 4, tau_override=1e-3)
    start = (1 << 30) - 10
    inst.reset(np.array([[start]], np.int32))
    with pytest.raises(oracle_lib.OracleError) as e:
        inst.run(5e-3)
    assert e.value.code == OS_EOVERFLOW
    assert inst.window == 1
    assert inst.counts[0, 0] == (1 << 30) + 1
