"""Pins of the oracle's time-varying forcing (rate constants replaced between
windows) and recording (per-region counts), against closed forms and hand
values (section 3.2: influx updated every 1 ms, per-region recording)."""
import numpy as np
import pytest
from scipy import stats

from tests.meshes import mirror_pair, model, single_tet
from tests.test_oracle_scheme import _chi2_sf


def _source_inst(oracle_lib, k, tau):
    # zero-order influx 0 -> A and nothing else, one tet: exact Poisson counts
    return oracle_lib.Instance(single_tet(), model([0], [([], ["A"], k)], ["A"]), 0, tau_override=tau)


def test_piecewise_constant_influx_is_poisson(oracle_lib):
    """Influx k1 for 4 windows, then k2 for 6: A(t) ~ Poisson(N_A V (k1 t1 +
    k2 (t2 - t1))).  Ignoring the switch gives a mean of 25 instead of 50."""
    tau, k1, k2, runs = 0.1, 2.5e-7, 6.67e-7, 3000
    inst = _source_inst(oracle_lib, k1, tau)
    nav = inst.geometry()["nav"][0]  # N_A V in molecules per molar
    mean = nav * (k1 * 0.4 + k2 * 0.6)
    assert 45 < mean < 55
    out = np.zeros(runs, int)
    for r in range(runs):
        inst.set_rates(np.array([[k1]]))
        inst.reset(np.zeros((1, 1), np.int32), seed=r)
        inst.run(0.4)
        assert inst.window == 4
        inst.set_rates(np.array([[k2]]))
        inst.run(1.0)
        out[r] = inst.counts[0, 0]
    top = int(mean * 3)
    obs = np.bincount(np.minimum(out, top), minlength=top + 1)
    exp = runs * stats.poisson.pmf(np.arange(top + 1), mean)
    exp[-1] = runs * stats.poisson.sf(top - 1, mean)
    assert _chi2_sf(obs, exp) > 1e-3


def test_switch_takes_effect_at_the_next_window(oracle_lib):
    """Rate 0 for two windows, then k: nothing before, events after; rate k
    then 0: the count freezes at the switch."""
    tau, k = 0.1, 3e-7
    inst = _source_inst(oracle_lib, 0.0, tau)
    inst.reset(np.zeros((1, 1), np.int32), seed=3)
    inst.step(2)
    assert inst.counts[0, 0] == 0 and inst.tallies.ssa_events == 0
    inst.set_rates(np.array([[k]]))
    inst.step(3)
    assert inst.counts[0, 0] == inst.tallies.ssa_events > 0
    frozen = int(inst.counts[0, 0])
    inst.set_rates(np.array([[0.0]]))
    inst.step(5)
    assert inst.counts[0, 0] == frozen


def test_same_rates_change_nothing(oracle_lib):
    """Setting the rates a run already has between windows leaves its
    trajectory bit-identical (the window's random draws do not depend on it)."""
    tau, k = 0.1, 3e-7
    a = _source_inst(oracle_lib, k, tau)
    b = _source_inst(oracle_lib, k, tau)
    for inst in (a, b):
        inst.reset(np.zeros((1, 1), np.int32), seed=11)
    a.step(7)
    b.step(3)
    b.set_rates(np.array([[k]]))
    b.step(4)
    assert np.array_equal(a.counts, b.counts)


def test_bad_rates_rejected(oracle_lib):
    inst = _source_inst(oracle_lib, 1e-7, 0.1)
    for bad in (-1.0, np.nan, np.inf):
        with pytest.raises(oracle_lib.OracleError):
            inst.set_rates(np.array([[bad]]))
    assert inst.kcst[0, 0] == 1e-7


def test_region_counts_hand_values(oracle_lib):
    """Two tets in regions 1 and 0, two species: the sums written out by hand."""
    mesh = mirror_pair()
    mesh["region"] = np.array([1, 0], np.uint8)
    md = model([1e-12, 1e-12], [(["A"], ["B"], 1.0)], ["A", "B"], n_regions=2)
    inst = oracle_lib.Instance(mesh, md, 0)
    inst.set_counts(np.array([[3, 5], [0, 7]], np.int32))
    assert inst.region_counts().tolist() == [[5, 7], [3, 0]]


def test_region_counts_partition_the_totals(oracle_lib):
    """Three regions on a 2 x 2 x 3 box: the regions' sums add up to each
    species' total, and region 0's sum equals a tet-by-tet loop."""
    from paper_1610_02258_amd import inputs as I
    rng = np.random.default_rng(5)
    mesh = I.box_mesh(2, 2, 3, 1e-6)
    mesh.region = rng.integers(0, 3, mesh.n_tets).astype(np.uint8)
    md = model([1e-12] * 4, [(["A"], ["B"], 1.0)], ["A", "B", "C", "D"], n_regions=3)
    inst = oracle_lib.Instance(mesh.as_dict(), md, 0)
    c = rng.integers(0, 1000, (4, mesh.n_tets)).astype(np.int32)
    inst.set_counts(c)
    rc = inst.region_counts()
    assert rc.shape == (3, 4)
    assert np.array_equal(rc.sum(axis=0), c.sum(axis=1))
    assert np.array_equal(rc[0], sum(c[:, i] for i in range(mesh.n_tets) if mesh.region[i] == 0))
